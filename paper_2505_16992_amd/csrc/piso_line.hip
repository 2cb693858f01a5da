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
// segments of L cells, one per half-wave (32 lines per group keeps more than one group
// per CU at 96^3).  A thread eliminates its segment with the Thomas algorithm for three right-hand
// sides (the line's right-hand side and the two couplings to the neighbouring segments),
// so that w = U + V w_prev_last + G w_next_first on the segment; the first and last
// values of the segments go through LDS, one thread per line solves the two-term
// recurrence for the segment interface values, and every thread reconstructs its cells.
#include <string>

#include "piso_impl.h"

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

// Solve T w = d on the lines of this work-group.  Each thread holds its segment's
// coefficients a (lower), b (diagonal), c (upper) and right-hand side d for k <= L cells
// (k = 0: no cells); on return d holds w.  All threads of the work-group call it.
template <typename R, int L>
__device__ __forceinline__ void line_solve(const R (&a)[L], const R (&b)[L], const R (&c)[L], R (&d)[L], int k,
                                           int nseg, R* sh /* [kLineLanes][kLineSegs][6] */,
                                           R* sif /* [kLineLanes][kLineSegs][2] */) {
  const int lane = threadIdx.x % kLineLanes, m = threadIdx.x / kLineLanes;
  R cp[L], V[L], G[L];
  // forward elimination (the segment's first lower and last upper couplings are the
  // right-hand sides of V and G)
  R prev_cp = R(0), prev_u = R(0), prev_v = R(0), prev_g = R(0);
#pragma unroll
  for (int t = 0; t < L; ++t) {
    if (t < k) {
      const R at = t > 0 ? a[t] : R(0);
      const R inv = R(1) / (b[t] - at * prev_cp);
      cp[t] = t < k - 1 ? c[t] * inv : R(0);
      d[t] = (d[t] - at * prev_u) * inv;
      V[t] = (t == 0 ? -a[0] : -at * prev_v) * inv;
      G[t] = (t == k - 1 ? -c[t] : -at * prev_g) * inv;
      prev_cp = cp[t];
      prev_u = d[t];
      prev_v = V[t];
      prev_g = G[t];
    } else {
      cp[t] = V[t] = G[t] = R(0);
    }
  }
  // back substitution
#pragma unroll
  for (int t = L - 2; t >= 0; --t) {
    if (t < k - 1) {
      d[t] -= cp[t] * d[t + 1];
      V[t] -= cp[t] * V[t + 1];
      G[t] -= cp[t] * G[t + 1];
    }
  }
  // segment end values through LDS
  R* e = sh + ((size_t)lane * kLineSegs + m) * 6;
  if (k > 0) {
    R uf = d[0], vf = V[0], gf = G[0], ul = d[0], vl = V[0], gl = G[0];
#pragma unroll
    for (int t = 1; t < L; ++t)
      if (t == k - 1) {
        ul = d[t];
        vl = V[t];
        gl = G[t];
      }
    e[0] = uf; e[1] = vf; e[2] = gf; e[3] = ul; e[4] = vl; e[5] = gl;
  }
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
  const R* ii = sif + ((size_t)lane * kLineSegs + m) * 2;
  const R lp = k > 0 ? ii[0] : R(0), fn = k > 0 ? ii[1] : R(0);
#pragma unroll
  for (int t = 0; t < L; ++t)
    if (t < k) d[t] += V[t] * lp + G[t] * fn;
}

}  // namespace

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
  const int lane = threadIdx.x % kLineLanes, m = threadIdx.x / kLineLanes;
  const int l = xcd_logical_group() * kLineLanes + lane;
  const int nseg = (geo.n + L - 1) / L;
  int k = geo.n - m * L;
  k = l < geo.nlines ? (k < 0 ? 0 : (k > L ? L : k)) : 0;
  const int P0 = l < geo.nlines ? line_base(geo, la, l) + m * L * geo.stride : 0;
  const R* Pa = Pf + (size_t)la * g.N;
  R a[L], b[L], c[L], d[L];
  R xv[L], dv[L], qv[L];
  // loads first (clamped to cell 0 where there is no cell), then the partials
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const bool on = t < k;
    const int P = on ? P0 + t * geo.stride : 0;
    const int j = m * L + t;
    b[t] = Dinv[P];
    d[t] = rin[P];
    a[t] = Pa[on && j > 0 ? P - geo.stride : 0];
    c[t] = Pa[P];
    if constexpr (UPD) {
      xv[t] = x[P];
      dv[t] = dnew[P];
      qv[t] = q[P];
    }
  }
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
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const int j = m * L + t;
    if (t < k) {
      const int P = P0 + t * geo.stride;
      if constexpr (UPD) {
        d[t] = d[t] - alpha * qv[t];
        x[P] = xv[t] + alpha * dv[t];
        rout[P] = d[t];
      }
      b[t] = R(1) / b[t];
      a[t] = j > 0 ? -a[t] : R(0);
      c[t] = j < geo.n - 1 ? -c[t] : R(0);
    } else {
      a[t] = c[t] = d[t] = R(0);
      b[t] = R(1);
    }
  }
  line_solve<R, L>(a, b, c, d, k, nseg, sh, sif);
#pragma unroll
  for (int t = 0; t < L; ++t)
    if (t < k) y[P0 + t * geo.stride] = omega * d[t];
}

// Fine-level prolongation and post-smoothing with the line smoother:
// z1 = y + e1[parent], z = z1 + omega T^-1 (r - M z1); partial sums of r.z and r.r.
// M z1 on the segment: along the line from the thread's own cells (memory at the segment
// ends), across x from the neighbouring lanes (memory at the group's edges), across the
// other transverse axis from memory.  The block's sides are walls or wrap onto the
// block (the host checks this before choosing lines).
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
  const int lane = threadIdx.x % kLineLanes, m = threadIdx.x / kLineLanes;
  const int l = xcd_logical_group() * kLineLanes + lane;
  const int nseg = (geo.n + L - 1) / L;
  int k = geo.n - m * L;
  k = l < geo.nlines ? (k < 0 ? 0 : (k > L ? L : k)) : 0;
  const int P0 = l < geo.nlines ? line_base(geo, la, l) + m * L * geo.stride : 0;
  const int N = g.N;
  const int* t1 = g1.tab;
  const int wrap = g.tab[kTabWrap];
  const int nx = geo.nx;
  // the line's fixed coordinates: x = ci, the other transverse one = co along axis ot
  const int li = l < geo.nlines ? l : 0;
  const int ci = li % nx, co = li / nx;
  const int ot = la == 1 ? 2 : 1;
  const int no = ot == 1 ? geo.ny : geo.nz;
  const int so = ot == 1 ? nx : nx * geo.ny;
  const bool has_ot = g.dim == 3 || ot == 1;
  auto par_of = [&](int i, int lp, int op) {   // aggregate of the cell (x, line, other)
    const int j = la == 1 ? lp : op, kk = la == 1 ? op : lp;
    return t1[0] + (i >> 1) + t1[1] * ((j >> 1) + t1[2] * (kk >> 1));
  };
  const R* Pa = Pf + (size_t)la * N;
  const R* Px = Pf;
  const R* Po = Pf + (size_t)ot * N;
  // every load is issued before the stencil (indices clamped: a face that does not exist
  // reads the cell itself and is masked afterwards), so that nothing waits in a branch
  const bool xl_in = ci > 0, xr_in = ci + 1 < nx;
  const bool xl_on = xl_in || (wrap & 1), xr_on = xr_in || (wrap & 2);
  const int cil = xl_in ? ci - 1 : nx - 1, cir = xr_in ? ci + 1 : 0;
  const bool om_in = co > 0, op_in = co + 1 < no;
  const bool om_on = has_ot && (om_in || ((wrap >> (2 * ot)) & 1));
  const bool op_on = has_ot && (op_in || ((wrap >> (2 * ot + 1)) & 1));
  const int com = om_in ? co - 1 : no - 1, cop = op_in ? co + 1 : 0;
  R b[L], d[L], z1[L], rv[L], pa[L], px[L];
  R zxl[L], zxr[L], wxl[L], zom[L], zop[L], wom[L], wop[L];
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const bool on = t < k;
    const int P = on ? P0 + t * geo.stride : 0;
    const int lp = on ? m * L + t : 0;
    rv[t] = r[P];
    b[t] = Dinv[P];
    pa[t] = Pa[P];
    px[t] = Px[P];
    z1[t] = y[P] + ec[on ? par_of(ci, lp, co) : 0];
    const int FL = on && xl_on ? (xl_in ? P - 1 : P + nx - 1) : P;
    const int FR = on && xr_on ? (xr_in ? P + 1 : P + 1 - nx) : P;
    zxl[t] = y[FL] + ec[on ? par_of(cil, lp, co) : 0];
    zxr[t] = y[FR] + ec[on ? par_of(cir, lp, co) : 0];
    wxl[t] = Px[FL];
    const int FM = on && om_on ? (om_in ? P - so : P + (no - 1) * so) : P;
    const int FP = on && op_on ? (op_in ? P + so : P - (no - 1) * so) : P;
    zom[t] = y[FM] + ec[on && has_ot ? par_of(ci, lp, com) : 0];
    zop[t] = y[FP] + ec[on && has_ot ? par_of(ci, lp, cop) : 0];
    wom[t] = Po[FM];
    wop[t] = Po[P];
  }
  // along the line at the segment's two ends (the rest comes from the thread's own cells)
  const int lp0 = m * L, lpk = m * L + (k > 0 ? k - 1 : 0);
  const bool lo_in = lp0 > 0, hi_in = lpk + 1 < geo.n;
  const bool lo_on = k > 0 && (lo_in || ((wrap >> (2 * la)) & 1));
  const bool hi_on = k > 0 && (hi_in || ((wrap >> (2 * la + 1)) & 1));
  // (a segment past the line's end has no cells and P0 beyond it: it reads cell 0)
  const int Pb = k > 0 ? P0 : 0;
  const int Pk = Pb + (k > 0 ? k - 1 : 0) * geo.stride;
  const int FLo = lo_on ? (lo_in ? P0 - geo.stride : P0 + (geo.n - 1) * geo.stride) : Pb;
  const int FHi = hi_on ? (hi_in ? Pk + geo.stride : Pk - (geo.n - 1) * geo.stride) : Pk;
  const R zlo = y[FLo] + ec[k > 0 ? par_of(ci, lo_in ? lp0 - 1 : geo.n - 1, co) : 0];
  const R zhi = y[FHi] + ec[k > 0 ? par_of(ci, hi_in ? lpk + 1 : 0, co) : 0];
  const R wlo0 = Pa[FLo];
  // x neighbours held by the adjacent lanes of the same segment (width-32 shuffles)
  const bool left_lane = lane > 0 && xl_in, right_lane = lane + 1 < kLineLanes && xr_in;
  R a[L], c[L];
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const R zl = __shfl(z1[t], lane > 0 ? lane - 1 : lane, kLineLanes);
    const R pl = __shfl(px[t], lane > 0 ? lane - 1 : lane, kLineLanes);
    const R zr = __shfl(z1[t], lane + 1 < kLineLanes ? lane + 1 : lane, kLineLanes);
    if (t < k) {
      const int lp = m * L + t;
      R mz = R(0);
      if (xl_on) mz += (left_lane ? pl : wxl[t]) * (z1[t] - (left_lane ? zl : zxl[t]));
      if (xr_on) mz += px[t] * (z1[t] - (right_lane ? zr : zxr[t]));
      if (om_on) mz += wom[t] * (z1[t] - zom[t]);
      if (op_on) mz += wop[t] * (z1[t] - zop[t]);
      // along the line (the lower face's weight is stored at the lower cell)
      const R wlo = t > 0 ? pa[t - 1] : wlo0;
      if (t > 0 || lo_on) mz += wlo * (z1[t] - (t > 0 ? z1[t - 1] : zlo));
      if (t + 1 < k || hi_on) mz += pa[t] * (z1[t] - (t + 1 < k ? z1[t + 1] : zhi));
      d[t] = rv[t] - mz;
      // T: tridiagonal part along the line (couplings across a wrap left out)
      b[t] = R(1) / b[t];
      a[t] = lp > 0 ? -wlo : R(0);
      c[t] = lp + 1 < geo.n ? -pa[t] : R(0);
    } else {
      a[t] = c[t] = d[t] = R(0);
      b[t] = R(1);
    }
  }
  line_solve<R, L>(a, b, c, d, k, nseg, sh, sif);
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
  for (int t = 0; t < L; ++t) {
    if (t < k) {
      const R zo = z1[t] + omega * d[t];
      z[P0 + t * geo.stride] = zo;
      acc0 += (double)rv[t] * (double)zo;
      acc1 += (double)rv[t] * (double)rv[t];
    }
  }
  const double s0 = line_wg_sum(acc0, red);
  const double s1 = line_wg_sum(acc1, red);
  if (threadIdx.x == 0) {
    partB[blockIdx.x] = s0;
    partB[gridDim.x + blockIdx.x] = s1;
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
  for (int cand : {4, 8, 12, 16, 24, 32})
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
  bool on = best > 3.0 && L > 0 && groups <= kRedGrid && plain_sides;
  if (const char* e = std::getenv("PISO_MG_LINE")) on = on && e[0] != '0';
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
    case 16: PRE(16); break;
    case 24: PRE(24); break;
    default: PRE(32); break;
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
    case 16: POST(16); break;
    case 24: POST(24); break;
    default: POST(32); break;
  }
#undef POST
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string("k_line_post: ") + hipGetErrorString(e));
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

}  // namespace piso
