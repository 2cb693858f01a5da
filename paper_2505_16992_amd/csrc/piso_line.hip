// Line smoothing on the fine level of the multigrid preconditioner (single-block grids
// stretched along one axis, the wall-normal axis of a channel).
//
// The pressure operator M (a weighted graph Laplacian) is strongly anisotropic where the
// grid is stretched: the faces normal to the stretched axis carry weights 100x those of
// the other faces next to a wall, and point Jacobi then smooths the error poorly.  The
// smoother here is omega T^-1 with T the tridiagonal part of M along the line axis (the
// full diagonal D and the couplings to the two line neighbours; couplings across a
// periodic wrap of the line axis are left out, which keeps T symmetric positive
// definite).  Pre- and post-smoothing use the same symmetric operator, so the V-cycle
// stays a symmetric positive definite preconditioner.
//
// GPU layout.  A work-group owns 32 lines (consecutive lines, x fastest, so that the 32
// lanes of a half-wave load 128 contiguous bytes of a row) and cuts each line into S = 8
// segments of L cells, one per half-wave (288 groups at 96^3; 16 lines of 16 shorter
// segments per group spread better over the CUs but ran slower).  A thread eliminates its
// segment with the Thomas algorithm for three right-hand sides (the line's right-hand
// side and the two couplings to the neighbouring segments), so that
// w = U + V w_prev_last + G w_next_first on the segment; the first and last values of
// the segments go through LDS, one thread per line solves the two-term recurrence for
// the segment interface values, and every thread reconstructs its cells.
//
// Kernels: k_line_pre (the PCG update fused with the pre-smoothing), k_line_restrict (the
// restriction of r' - M y to level 1, which needs y of other groups' lines) and
// k_line_post (prolongation fused with the post-smoothing and the partial sums of r.z).
#include <string>

#include "piso_impl.h"
#include "piso_quad.h"

namespace piso {

namespace {

constexpr int kLineLanes = 32;
constexpr int kLineSegs = 8;
constexpr int kLineThreads = kLineLanes * kLineSegs;
constexpr int kLineWaves = kLineThreads / 64;

struct LineGeo {
  int nx, ny, nz;
  int n;        // cells per line
  int stride;   // cell stride along the line
  int nlines;
};

__device__ __forceinline__ LineGeo line_geo(const Grid& g, int la) {
  LineGeo q;
  q.nx = g.tab[1];
  q.ny = g.tab[2];
  q.nz = g.tab[3];
  q.n = la == 1 ? q.ny : q.nz;
  q.stride = la == 1 ? q.nx : q.nx * q.ny;
  q.nlines = g.N / q.n;
  return q;
}

// first cell of line l: lines run x fastest, then over the remaining transverse axis
__device__ __forceinline__ int line_base(const LineGeo& q, int la, int l) {
  return la == 1 ? (l % q.nx) + q.nx * q.ny * (l / q.nx) : l;
}

// Sum over the work-group of one double (fixed order), in every thread.
__device__ __forceinline__ double line_wg_sum(double v, double* lds /* [kLineWaves] */) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kLineWaves; ++w) t += lds[w];
  __syncthreads();
  return t;
}

// Load from a uniform base at a 32-bit byte offset (the host keeps line smoothing to
// grids whose fields are below 4 GiB): the base stays in scalar registers and loads at
// the same cell share one offset register across arrays.
template <typename R>
__device__ __forceinline__ R ldo(const R* __restrict__ base, uint32_t off) {
  return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base) + off);
}

// Reciprocal of a pivot: the hardware reciprocal (1 ulp) in FP32, exact in FP64.
template <typename R>
__device__ __forceinline__ R line_rcp(R x) {
  if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);
  else return R(1) / x;
}

// Solve T w = d on the lines of this work-group.  Each thread holds its segment's
// coefficients a (lower), b (diagonal), c (upper) and right-hand side d for k <= L cells
// (k = 0: no cells); on return d holds w.  Cells t >= k must carry a = 0, finite b > 0,
// c and d: they are then decoupled from the segment and the recursions run over all L
// cells without branches.  All threads of the work-group call it.
template <typename R, int L>
__device__ __forceinline__ void line_solve(const R (&a)[L], const R (&b)[L], const R (&c)[L], R (&d)[L], int k,
                                           int nseg, R* sh /* [kLineLanes][kLineSegs][6] */,
                                           R* sif /* [kLineLanes][kLineSegs][2] */) {
  const int lane = threadIdx.x % kLineLanes, m = threadIdx.x / kLineLanes;
  R cp[L], V[L], G[L];
  // forward elimination; the segment's first lower coupling a[0] and last upper coupling
  // c[k-1] are the right-hand sides of V and G (G is zero above cell k-1 until then)
  R pc = R(0), pu = R(0), pv = R(1);
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const R inv = line_rcp(b[t] - a[t] * pc);
    const bool last = t == k - 1;
    cp[t] = last ? R(0) : c[t] * inv;
    d[t] = (d[t] - a[t] * pu) * inv;
    V[t] = -a[t] * pv * inv;
    G[t] = last ? -c[t] * inv : R(0);
    pc = cp[t];
    pu = d[t];
    pv = V[t];
  }
  // back substitution (cp[k-1] = 0 cuts the cells above the segment off)
#pragma unroll
  for (int t = L - 2; t >= 0; --t) {
    d[t] -= cp[t] * d[t + 1];
    V[t] -= cp[t] * V[t + 1];
    G[t] -= cp[t] * G[t + 1];
  }
  // segment end values through LDS
  R ul = d[0], vl = V[0], gl = G[0];
#pragma unroll
  for (int t = 1; t < L; ++t) {
    const bool last = t == k - 1;
    ul = last ? d[t] : ul;
    vl = last ? V[t] : vl;
    gl = last ? G[t] : gl;
  }
  R* e = sh + ((size_t)lane * kLineSegs + m) * 6;
  e[0] = d[0]; e[1] = V[0]; e[2] = G[0]; e[3] = ul; e[4] = vl; e[5] = gl;
  __syncthreads();
  // interface recurrence, one thread per line: l_{m-1} = al + be f_m, f_m = A_m + B_m f_{m+1}
  if (m == 0) {
    const R* sl = sh + (size_t)lane * kLineSegs * 6;
    R* il = sif + (size_t)lane * kLineSegs * 2;
    R A[kLineSegs], B[kLineSegs], al[kLineSegs], be[kLineSegs];
    R alp = R(0), bep = R(0);
#pragma unroll
    for (int s = 0; s < kLineSegs; ++s) {
      if (s < nseg) {
        const R* q = sl + s * 6;
        const R den = R(1) / (R(1) - q[1] * bep);
        A[s] = (q[0] + q[1] * alp) * den;
        B[s] = q[2] * den;
        al[s] = q[3] + q[4] * alp + q[4] * bep * A[s];
        be[s] = q[4] * bep * B[s] + q[5];
        alp = al[s];
        bep = be[s];
      }
    }
    R f[kLineSegs];
    R fn = R(0);
#pragma unroll
    for (int s = kLineSegs - 1; s >= 0; --s) {
      if (s < nseg) {
        f[s] = A[s] + B[s] * fn;
        fn = f[s];
      } else {
        f[s] = R(0);
      }
    }
#pragma unroll
    for (int s = 0; s < kLineSegs; ++s) {
      if (s < nseg) {
        const R next = s + 1 < nseg ? f[s + 1] : R(0);
        const R last_prev = s > 0 ? al[s - 1] + be[s - 1] * f[s] : R(0);
        il[s * 2 + 0] = last_prev;
        il[s * 2 + 1] = next;
      }
    }
  }
  __syncthreads();
  // segments past the line's end read values never written: only their cells use them
  const R* ii = sif + ((size_t)lane * kLineSegs + m) * 2;
  const R lp = ii[0], fn = ii[1];
#pragma unroll
  for (int t = 0; t < L; ++t) d[t] += V[t] * lp + G[t] * fn;
}

}  // namespace

// Where a thread's cells lie.  Cells past the line's end (a ragged or empty last
// segment, a lane past the last line) are clamped to the line's last cell, a line past
// the last one to line 0: every load stays in bounds and needs no condition; such cells
// are masked in the arithmetic and never stored.
struct LineCells {
  int k;       // cells of the segment (0..L)
  int lp0;     // position of the segment's first cell along the line
  int pl0;     // first cell of the line
  int ci, co;  // the line's x and other transverse coordinate
  int nseg;    // segments of a line
};

template <int L>
__device__ __forceinline__ LineCells line_cells(const LineGeo& geo, int la) {
  LineCells q;
  const int lane = threadIdx.x % kLineLanes, m = threadIdx.x / kLineLanes;
  const int l = xcd_logical_group() * kLineLanes + lane;
  const bool lv = l < geo.nlines;
  const int li = lv ? l : 0;
  q.nseg = (geo.n + L - 1) / L;
  q.lp0 = m * L;
  int k = geo.n - q.lp0;
  q.k = lv ? (k < 0 ? 0 : (k > L ? L : k)) : 0;
  q.pl0 = line_base(geo, la, li);
  q.ci = li % geo.nx;
  q.co = li / geo.nx;
  return q;
}

// cell t of the segment (clamped into the line)
template <int L>
__device__ __forceinline__ int line_cell(const LineGeo& geo, const LineCells& q, int t) {
  const int lp = q.lp0 + t;
  return q.pl0 + (lp < geo.n ? lp : geo.n - 1) * geo.stride;
}

// Pre-smoothing from zero on the fine level, y = omega T^-1 r', with the PCG update in
// front of it when UPD (alpha from the Gp partials of d.q, x += alpha d, r' = rin -
// alpha q stored in rout); without UPD r' = rin (the first V-cycle of a solve).
template <typename R, int L, bool UPD>
__global__ void __launch_bounds__(kLineThreads)
k_line_pre(Grid g, int la, const R* __restrict__ Pf, const R* __restrict__ Dinv, R* __restrict__ x,
           const R* __restrict__ rin, R* __restrict__ rout, const R* __restrict__ dnew, const R* __restrict__ q,
           R* __restrict__ y, R omega, CgState* st, const double* __restrict__ partA, int Gp, int par) {
  __shared__ R sh[kLineLanes * kLineSegs * 6];
  __shared__ R sif[kLineLanes * kLineSegs * 2];
  __shared__ double red[kLineWaves];
  const int done = st->done;
  const double rzp = UPD ? st->rz[par] : 0.0;
  const LineGeo geo = line_geo(g, la);
  const LineCells lc = line_cells<L>(geo, la);
  const int k = lc.k;
  const R* Pa = Pf + (size_t)la * g.N;
  constexpr uint32_t es = sizeof(R);
  R a[L], b[L], c[L], d[L];
  R xv[L], dv[L], qv[L];
  uint32_t off[L];
  // loads first, then the partials
#pragma unroll
  for (int t = 0; t < L; ++t) {
    off[t] = (uint32_t)line_cell<L>(geo, lc, t) * es;
    b[t] = ldo(Dinv, off[t]);
    d[t] = ldo(rin, off[t]);
    c[t] = ldo(Pa, off[t]);
    if constexpr (UPD) {
      xv[t] = ldo(x, off[t]);
      dv[t] = ldo(dnew, off[t]);
      qv[t] = ldo(q, off[t]);
    }
  }
  // the face below the segment (its weight is stored at the cell below)
  const int lpb = lc.lp0 > 0 ? (lc.lp0 < geo.n ? lc.lp0 : geo.n) - 1 : 0;
  const R wlo = ldo(Pa, (uint32_t)(lc.pl0 + lpb * geo.stride) * es);
  R alpha = R(0);
  if constexpr (UPD) {
    double v = 0.0;
    for (int w0 = 0; w0 < Gp; w0 += 4 * kLineThreads) {
      double u4[4];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int w = w0 + (int)threadIdx.x + cc * kLineThreads;
        u4[cc] = w < Gp ? partA[w] : 0.0;
      }
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) v += u4[cc];
    }
    const double dq = line_wg_sum(v, red);
    if (done) return;
    if (!(dq > 0.0) || !std::isfinite(dq)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->status = std::isfinite(dq) ? PISO_BREAKDOWN : PISO_E_NAN;
        st->iters = st->k;
        st->done = 1;
      }
      return;
    }
    alpha = (R)(rzp / dq);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->k = st->k + 1;   // no other group reads it here
  } else {
    if (done) return;
  }
  // T along the line: the lower coupling of cell t is the upper one of cell t-1; no
  // coupling across the line's ends (walls, or a wrap left out of T)
  R cl = wlo;
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const int lp = lc.lp0 + t;
    if constexpr (UPD) d[t] = d[t] - alpha * qv[t];
    const R up = c[t];
    a[t] = (t < k && lp > 0) ? -cl : R(0);
    c[t] = lp + 1 < geo.n ? -up : R(0);
    b[t] = line_rcp(b[t]);
    cl = up;
  }
  if constexpr (UPD) {
#pragma unroll
    for (int t = 0; t < L; ++t) {
      if (t < k) {
        *reinterpret_cast<R*>(reinterpret_cast<char*>(x) + off[t]) = xv[t] + alpha * dv[t];
        *reinterpret_cast<R*>(reinterpret_cast<char*>(rout) + off[t]) = d[t];
      }
    }
  }
  line_solve<R, L>(a, b, c, d, k, lc.nseg, sh, sif);
#pragma unroll
  for (int t = 0; t < L; ++t)
    if (t < k) *reinterpret_cast<R*>(reinterpret_cast<char*>(y) + off[t]) = omega * d[t];
}

// Fine-level prolongation and post-smoothing with the line smoother:
// z1 = y + e1[parent], z = z1 + omega T^-1 (r - M z1); partial sums of r.z and r.r.
// A face that does not exist (a wall) is given the cell itself as neighbour: its term
// of M z1 is then exactly zero.  The block's sides are walls or wrap onto the block (the
// host checks this before choosing lines).
template <typename R, int L>
__global__ void __launch_bounds__(kLineThreads)
k_line_post(Grid g, Grid g1, int la, const R* __restrict__ Pf, const R* __restrict__ Dinv, const R* __restrict__ r,
            const R* __restrict__ y, const R* __restrict__ ec, R omega, R* __restrict__ z,
            double* __restrict__ partB, const CgState* st) {
  __shared__ R sh[kLineLanes * kLineSegs * 6];
  __shared__ R sif[kLineLanes * kLineSegs * 2];
  __shared__ double red[kLineWaves];
  if (st->done) return;
  const LineGeo geo = line_geo(g, la);
  const LineCells lc = line_cells<L>(geo, la);
  const int k = lc.k, n = geo.n, nx = geo.nx, ci = lc.ci, co = lc.co;
  const int wrap = g.tab[kTabWrap];
  const int ot = la == 1 ? 2 : 1;                      // the other transverse axis
  const int no = ot == 1 ? geo.ny : geo.nz;
  const int so = ot == 1 ? nx : nx * geo.ny;
  const bool has_ot = g.dim == 3;
  // neighbour offsets (cells) of the thread's line, 0 where the face does not exist
  const bool xl_in = ci > 0, xr_in = ci + 1 < nx;
  const bool xl_on = xl_in || (wrap & 1), xr_on = xr_in || ((wrap >> 1) & 1);
  const int dxl = xl_in ? -1 : (xl_on ? nx - 1 : 0);
  const int dxr = xr_in ? 1 : (xr_on ? 1 - nx : 0);
  const bool om_in = co > 0, op_in = co + 1 < no;
  const bool om_on = has_ot && (om_in || ((wrap >> (2 * ot)) & 1));
  const bool op_on = has_ot && (op_in || ((wrap >> (2 * ot + 1)) & 1));
  const int dom = om_on ? (om_in ? -so : (no - 1) * so) : 0;
  const int dop = op_on ? (op_in ? so : -(no - 1) * so) : 0;
  // aggregate (coarse cell) of fine cell (i, line position lp, other o): the coarse grid
  // halves every axis of the block
  const int* t1 = g1.tab;
  const int cs = la == 1 ? t1[1] : t1[1] * t1[2];     // coarse stride along the line
  const int cso = la == 1 ? t1[1] * t1[2] : t1[1];    // along the other transverse axis
  const int cil = xl_on ? (xl_in ? ci - 1 : nx - 1) : ci, cir = xr_on ? (xr_in ? ci + 1 : 0) : ci;
  const int com = om_on ? (om_in ? co - 1 : no - 1) : co, cop = op_on ? (op_in ? co + 1 : 0) : co;
  const int cb = t1[0] + (ci >> 1) + (co >> 1) * cso;
  const int cbl = t1[0] + (cil >> 1) + (co >> 1) * cso, cbr = t1[0] + (cir >> 1) + (co >> 1) * cso;
  const int cbm = t1[0] + (ci >> 1) + (com >> 1) * cso, cbp = t1[0] + (ci >> 1) + (cop >> 1) * cso;
  const R* Pa = Pf + (size_t)la * g.N;
  const R* Px = Pf;
  const R* Po = Pf + (size_t)(has_ot ? ot : 0) * g.N;
  constexpr uint32_t es = sizeof(R);
  R b[L], d[L], z1[L], rv[L], pa[L], px[L];
  R yxl[L], yxr[L], wxl[L], yom[L], yop[L], wom[L], wop[L];
  R eo[L / 2], exl[L / 2], exr[L / 2], eom[L / 2], eop[L / 2];
  uint32_t off[L];
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const int P = line_cell<L>(geo, lc, t);
    off[t] = (uint32_t)P * es;
    rv[t] = ldo(r, off[t]);
    b[t] = ldo(Dinv, off[t]);
    pa[t] = ldo(Pa, off[t]);
    px[t] = ldo(Px, off[t]);
    z1[t] = ldo(y, off[t]);
    yxl[t] = ldo(y, (uint32_t)(P + dxl) * es);
    wxl[t] = ldo(Px, (uint32_t)(P + dxl) * es);
    yxr[t] = ldo(y, (uint32_t)(P + dxr) * es);
    yom[t] = ldo(y, (uint32_t)(P + dom) * es);
    wom[t] = ldo(Po, (uint32_t)(P + dom) * es);
    yop[t] = ldo(y, (uint32_t)(P + dop) * es);
    wop[t] = ldo(Po, off[t]);
  }
  // the coarse correction is shared by the two cells of a pair (L and lp0 are even)
#pragma unroll
  for (int h = 0; h < L / 2; ++h) {
    const int lp = lc.lp0 + 2 * h;
    const int cc = ((lp < n ? lp : n - 1) >> 1) * cs;
    eo[h] = ldo(ec, (uint32_t)(cb + cc) * es);
    exl[h] = ldo(ec, (uint32_t)(cbl + cc) * es);
    exr[h] = ldo(ec, (uint32_t)(cbr + cc) * es);
    eom[h] = ldo(ec, (uint32_t)(cbm + cc) * es);
    eop[h] = ldo(ec, (uint32_t)(cbp + cc) * es);
  }
  // along the line beyond the segment's ends (the cell itself where that face does not
  // exist, or for a segment without cells)
  const int lpk = lc.lp0 + (k > 0 ? k - 1 : 0);
  const int lpo = lc.lp0 > 0 ? (lc.lp0 < n ? lc.lp0 : n) - 1 : (((wrap >> (2 * la)) & 1) ? n - 1 : 0);
  const int lph = k == 0 ? 0 : (lpk + 1 < n ? lpk + 1 : (((wrap >> (2 * la + 1)) & 1) ? 0 : lpk));
  const int Plo = lc.pl0 + lpo * geo.stride, Phi = lc.pl0 + lph * geo.stride;
  const R zlo = ldo(y, (uint32_t)Plo * es) + ldo(ec, (uint32_t)(cb + (lpo >> 1) * cs) * es);
  const R zhi = ldo(y, (uint32_t)Phi * es) + ldo(ec, (uint32_t)(cb + (lph >> 1) * cs) * es);
  const R wlo = ldo(Pa, (uint32_t)Plo * es);
  R a[L], c[L];
#pragma unroll
  for (int t = 0; t < L; ++t) z1[t] += eo[t / 2];
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const int lp = lc.lp0 + t;
    const int h = t / 2;
    const R z = z1[t];
    R mz = wxl[t] * (z - (yxl[t] + exl[h]));
    mz += px[t] * (z - (yxr[t] + exr[h]));
    mz += wom[t] * (z - (yom[t] + eom[h]));
    mz += wop[t] * (z - (yop[t] + eop[h]));
    // along the line: the lower face's weight is stored at the lower cell
    const R wl = t > 0 ? pa[t - 1] : wlo;
    mz += wl * (z - (t > 0 ? z1[t - 1] : zlo));
    mz += pa[t] * (z - (t + 1 < k ? z1[t + 1] : zhi));
    d[t] = rv[t] - mz;
    // T: tridiagonal part along the line (couplings across a wrap left out)
    b[t] = line_rcp(b[t]);
    a[t] = (t < k && lp > 0) ? -wl : R(0);
    c[t] = lp + 1 < n ? -pa[t] : R(0);
  }
  line_solve<R, L>(a, b, c, d, k, lc.nseg, sh, sif);
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const R zo = z1[t] + omega * d[t];
    acc0 += t < k ? (double)rv[t] * (double)zo : 0.0;
    acc1 += t < k ? (double)rv[t] * (double)rv[t] : 0.0;
    if (t < k) *reinterpret_cast<R*>(reinterpret_cast<char*>(z) + off[t]) = zo;
  }
  const double s0 = line_wg_sum(acc0, red);
  const double s1 = line_wg_sum(acc1, red);
  if (threadIdx.x == 0) {
    partB[blockIdx.x] = s0;
    partB[gridDim.x + blockIdx.x] = s1;
  }
}

// Fine-grid restriction with line smoothing (y from the line solve, stored by
// k_line_pre): rc[I] = sum over the children P of aggregate I of r'_P - (M y)_P.  Faces
// between two children of I cancel in the sum; a face that leaves the aggregate
// through a wall takes the cell itself as neighbour, which makes its term exactly zero.
// Single block with nx % 4 == 0 whose sides are walls or wrap onto it (checked by the
// host).  Unit: one x-quad (two aggregates along x) of one coarse row and plane, one
// thread per fine row and plane parity of the unit (2^(d-1)); the aggregate sums are
// added across those threads by shuffles.  All loads are unconditional (rows past an
// odd extent are clamped to the last row and masked).
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_line_restrict(Grid g, Grid g1, int units, const R* __restrict__ Pf, const R* __restrict__ y,
                const R* __restrict__ r, R* __restrict__ rc, const CgState* st) {
  if (st->done) return;
  constexpr int NP = 1 << (D - 1);
  const int* tf = g.tab;
  const int* tc = g1.tab;
  const int N = g.N;
  const int nx = tf[1], ny = tf[2], nz = tf[3], wrap = tf[kTabWrap];
  const int cx = tc[1], cy = tc[2];
  const int nxq = nx >> 2;
  const int p = (int)threadIdx.x & (NP - 1);
  const int u0 = xcd_logical_group() * (kWG / NP) + (int)threadIdx.x / NP;
  const bool uv = u0 < units;
  const int u = uv ? u0 : 0;
  const int xq = u % nxq, rest = u / nxq;
  const int cj = rest % cy, ck = rest / cy;
  const int jj = 2 * cj + (p & 1), kk = D == 3 ? 2 * ck + (p >> 1) : 0;
  const bool valid = uv && jj < ny && kk < nz;
  const int j = jj < ny ? jj : ny - 1, k = kk < nz ? kk : nz - 1;
  const int i0 = 4 * xq;
  const int P0 = tf[0] + i0 + nx * (j + ny * k);
  const Q4<R> yq = ldq(y, P0), rq = ldq(r, P0), px = ldq(Pf, P0);
  // x faces that leave the quad's aggregates: left of cell 0 (weight stored at the left
  // cell) and right of cell 3; the face between cells 1 and 2 separates the two
  const int dl = i0 > 0 ? -1 : ((wrap & 1) ? nx - 1 : 0);
  const int dr = i0 + 4 < nx ? 4 : ((wrap & 2) ? 4 - nx : 3);
  const R yl = y[P0 + dl], pl = Pf[P0 + dl], yr = y[P0 + dr];
  R res[4];
  res[0] = rq.v[0] - pl * (yq.v[0] - yl);
  res[1] = rq.v[1] - px.v[1] * (yq.v[1] - yq.v[2]);
  res[2] = rq.v[2] - px.v[1] * (yq.v[2] - yq.v[1]);
  res[3] = rq.v[3] - px.v[3] * (yq.v[3] - yr);
  // y (and z) faces: the one on the side away from the aggregate's other row, and for
  // the last row of an odd extent (an aggregate one row thick) the upper one as well
#pragma unroll
  for (int a = 1; a < D; ++a) {
    const int pos = a == 1 ? j : k;
    const int n = a == 1 ? ny : nz;
    const int stride = a == 1 ? nx : nx * ny;
    const int bit = pos & 1;
    const R* Pa = Pf + (size_t)a * N;
    const int dlo = pos > 0 ? -stride : (((wrap >> (2 * a)) & 1) ? (n - 1) * stride : 0);
    const int dhi = pos + 1 < n ? stride : (((wrap >> (2 * a + 1)) & 1) ? -(n - 1) * stride : 0);
    const int dm = bit ? dhi : dlo;
    const Q4<R> yn = ldq(y, P0 + dm), wn = ldq(Pa, bit ? P0 : P0 + dm);
#pragma unroll
    for (int e = 0; e < 4; ++e) res[e] -= wn.v[e] * (yq.v[e] - yn.v[e]);
    if (n & 1) {   // the same for every thread
      const int dx = (bit == 0 && pos + 1 == n) ? dhi : 0;
      const Q4<R> yx = ldq(y, P0 + dx), wx = ldq(Pa, P0);
#pragma unroll
      for (int e = 0; e < 4; ++e) res[e] -= wx.v[e] * (yq.v[e] - yx.v[e]);
    }
  }
  R sa = valid ? res[0] + res[1] : R(0);
  R sb = valid ? res[2] + res[3] : R(0);
#pragma unroll
  for (int o = 1; o < NP; o <<= 1) {
    sa += __shfl_xor(sa, o, 64);
    sb += __shfl_xor(sb, o, 64);
  }
  if (p == 0 && uv) {
    const int I = tc[0] + 2 * xq + cx * (cj + cy * ck);
    rc[I] = sa;
    rc[I + 1] = sb;
  }
}

// ------------------------------------------------------------------ host

int line_groups(const piso_ctx* c) {
  if (!c->mg_line_axis) return 0;
  const int n = c->h_tab[1 + c->mg_line_axis];
  const int nlines = c->N / n;
  return (nlines + kLineLanes - 1) / kLineLanes;
}

int line_choose(piso_ctx* c, const piso_domain_desc* desc) {
  c->mg_line_axis = 0;
  c->mg_line_L = 0;
  if (c->nblocks != 1) return PISO_OK;
  const int D = c->dim, N = c->N;
  // mean ratio of the metric weight alpha_aa = J |T_a|^2 to the largest other one
  double best = 0.0;
  int axis = 0;
  for (int a = 1; a < D; ++a) {
    double sum = 0.0;
    for (int P = 0; P < N; ++P) {
      double al[3] = {0, 0, 0};
      for (int j = 0; j < D; ++j) {
        double s = 0.0;
        for (int i = 0; i < D; ++i) {
          const double v = desc->T[(size_t)(j * D + i) * N + P];
          s += v * v;
        }
        al[j] = desc->J[P] * s;
      }
      double other = 0.0;
      for (int j = 0; j < D; ++j)
        if (j != a) other = std::max(other, al[j]);
      if (other > 0.0) sum += al[a] / other;
    }
    const double mean = sum / N;
    if (mean > best) {
      best = mean;
      axis = a;
    }
  }
  const int n = c->h_tab[1 + axis];
  int L = 0;
  // lines of at most 128 cells: longer segments than 16 cells no longer fit the
  // registers (FP64 spills from 24 on)
  for (int cand : {4, 8, 12, 16})
    if (cand * kLineSegs >= n) {
      L = cand;
      break;
    }
  const int groups = (N / n + kLineLanes - 1) / kLineLanes;   // their partial sums must fit
  // the post-smoothing kernel handles walls and sides that wrap onto the block only
  bool plain_sides = true;
  for (int side = 0; side < 2 * D; ++side) {
    if ((c->h_tab[kTabWrap] >> side) & 1) continue;
    const int ax = side / 2;
    const int faces = ax == 0 ? c->h_tab[2] * c->h_tab[3] : (ax == 1 ? c->h_tab[1] * c->h_tab[3]
                                                                      : c->h_tab[1] * c->h_tab[2]);
    for (int f = 0; f < faces; ++f)
      if (c->h_fmap[(size_t)c->h_tab[4 + side] + f] >= 0) plain_sides = false;
  }
  // the kernels address fields with 32-bit byte offsets
  const bool small = (size_t)N * sizeof(double) < (size_t(1) << 32);
  const bool fits = axis > 0 && L > 0 && groups <= kRedGrid && plain_sides && small;
  bool on = fits && best > 3.0;
  // PISO_MG_LINE=0: point Jacobi; =1: lines wherever the grid allows them
  if (const char* e = std::getenv("PISO_MG_LINE")) on = e[0] == '0' ? false : (e[0] == '1' ? fits : on);
  if (on) {
    c->mg_line_axis = axis;
    c->mg_line_L = L;
  }
  return PISO_OK;
}

template <typename R, bool UPD>
static void launch_pre_L(piso_ctx* c, hipStream_t s, int G, const R* Pf, const R* Dinv, R* x, const R* rin, R* rout,
                         const R* dnew, const R* q, R* y, CgState* st, const double* partA, int Gp, int par) {
  const R om = (R)kMgOmega;
  const int la = c->mg_line_axis, kind = UPD ? kTimeCgUpdateMg : kTimeMgSmooth0;
#define PRE(LL)                                                                                                  \
  launch_timed_wg(c, s, kind, k_line_pre<R, LL, UPD>, G, kLineThreads, c->grid, la, Pf, Dinv, x, rin, rout, dnew, \
                  q, y, om, st, partA, Gp, par)
  switch (c->mg_line_L) {
    case 4: PRE(4); break;
    case 8: PRE(8); break;
    case 12: PRE(12); break;
    default: PRE(16); break;
  }
#undef PRE
}

template <typename R>
int line_pre(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, R* x, const R* rin, R* rout, const R* dnew,
             const R* q, R* y, CgState* st, const double* partA, int Gp, int par, bool update) {
  const int G = line_groups(c);
  if (update) launch_pre_L<R, true>(c, s, G, Pf, Dinv, x, rin, rout, dnew, q, y, st, partA, Gp, par);
  else launch_pre_L<R, false>(c, s, G, Pf, Dinv, x, rin, rout, dnew, q, y, st, partA, Gp, par);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string("k_line_pre: ") + hipGetErrorString(e));
  return PISO_OK;
}

template <typename R>
int line_post(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* r, const R* y, const R* e1, R* z,
              double* partB, CgState* st) {
  const int G = line_groups(c);
  const R om = (R)kMgOmega;
  const int la = c->mg_line_axis;
#define POST(LL)                                                                                                   \
  launch_timed_wg(c, s, kTimeMgUp0, k_line_post<R, LL>, G, kLineThreads, c->grid, c->mg_g1, la, Pf, Dinv, r, y, e1, \
                  om, z, partB, (const CgState*)st)
  switch (c->mg_line_L) {
    case 4: POST(4); break;
    case 8: POST(8); break;
    case 12: POST(12); break;
    default: POST(16); break;
  }
#undef POST
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string("k_line_post: ") + hipGetErrorString(e));
  return PISO_OK;
}

// The restriction for line smoothing in the quad layout; 1 (nothing launched) where
// the grid or the operands do not allow it (the caller then uses the tile kernel).
template <typename R>
int line_restrict(piso_ctx* c, hipStream_t s, const R* Pf, const R* r, const R* y, CgState* st) {
  if (!c->mg_line_axis || !c->quad || c->nblocks != 1) return 1;
  if ((((uintptr_t)Pf) | ((uintptr_t)r) | ((uintptr_t)y)) & 15u) return 1;
  const int groups = c->mg_qtiles.off[1];
  const int units = c->mg_qtiles.units[0];
  R* rc = (R*)c->mg[0].r;
  if (c->dim == 2)
    launch_timed_wg(c, s, kTimeMgDown0, k_line_restrict<R, 2>, groups, kWG, c->grid, c->mg_g1, units, Pf, y, r, rc,
                    (const CgState*)st);
  else
    launch_timed_wg(c, s, kTimeMgDown0, k_line_restrict<R, 3>, groups, kWG, c->grid, c->mg_g1, units, Pf, y, r, rc,
                    (const CgState*)st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string("k_line_restrict: ") + hipGetErrorString(e));
  return PISO_OK;
}

template int line_pre<float>(piso_ctx*, hipStream_t, const float*, const float*, float*, const float*, float*,
                             const float*, const float*, float*, CgState*, const double*, int, int, bool);
template int line_pre<double>(piso_ctx*, hipStream_t, const double*, const double*, double*, const double*, double*,
                              const double*, const double*, double*, CgState*, const double*, int, int, bool);
template int line_post<float>(piso_ctx*, hipStream_t, const float*, const float*, const float*, const float*,
                              const float*, float*, double*, CgState*);
template int line_post<double>(piso_ctx*, hipStream_t, const double*, const double*, const double*, const double*,
                               const double*, double*, double*, CgState*);

template int line_restrict<float>(piso_ctx*, hipStream_t, const float*, const float*, const float*, CgState*);
template int line_restrict<double>(piso_ctx*, hipStream_t, const double*, const double*, const double*, CgState*);

}  // namespace piso
