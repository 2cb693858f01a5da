// Aggregation multigrid preconditioner for the pressure PCG.
//
// The paper solves the pressure system with CG (App. A.6) and names multigrid for the
// pressure as the next step for speed (Sec. 6, App. A.6).  This is that step, kept
// inside the same CG so that the solution is the one the paper's solver converges to:
// only the preconditioner changes.
//
// Operator: M = -P, (M x)_P = sum_f P_f (x_P - x_F) (eq. pMatDiscrete), symmetric
// positive semi-definite with the constant vectors as null space.
//
// Hierarchy (built once per context on the host): level l+1 aggregates the cells of
// level l in 2x2(x2) boxes inside each block; prolongation is piecewise constant (Q),
// restriction its transpose, and the coarse operator the Galerkin product Q^T M Q,
// which for a graph Laplacian is again a graph Laplacian whose face weight between
// two aggregates is the sum of the finer face weights between them.  The weights are
// refreshed from Pf before every solve (P depends on A, eq. pMatDiscrete).
//
// One application z = B r is a V-cycle from a zero guess: on each level one damped
// Jacobi sweep before and one after the coarse correction (omega = 0.8 on the fine
// level, 0.9 on the coarse ones; on stretched single-block grids the fine level smooths
// along lines instead, in piso_line.hip), and on the coarsest level (<= 2048 cells, one
// work-group) a fixed Chebyshev iteration.  Every step is a fixed linear map and the
// pre- and post-smoothers are the same symmetric operator, so B is symmetric positive
// definite on the range of M and the outer CG keeps its theory.  On the coarse levels
// the pre-smoothing result omega D^-1 r is never stored: the kernels that need it at a
// neighbour recompute it from r and D^-1.
#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "piso_impl.h"
#include "piso_quad.h"

namespace piso {

// ------------------------------------------------------------------ kernels

// Work-group index for launches pinned to one XCD: small coarse-level kernels are
// launched with 8x the work-groups and only every eighth one (all on the XCD that
// receives work-group 0) works, so that consecutive small kernels share that XCD's L2.
// Returns -1 for the idle groups.  Unpinned launches use the XCD-aware group order.
__device__ __forceinline__ int mg_group(int pin) {
  if (!pin) return xcd_logical_group();   // contiguous index ranges per XCD, as on the fine grid
  return (blockIdx.x & 7) ? -1 : (int)(blockIdx.x >> 3);
}

// W[s][I] = sum of the finer face weights listed for (s, I); Dinv[I] = 1 / sum_s W.
template <typename R>
__global__ void __launch_bounds__(kWG)
k_mg_coef(int n, int K, const int* __restrict__ ptr, const int* __restrict__ idx, const R* __restrict__ Wsrc,
          R* __restrict__ W, R* __restrict__ Dinv) {
  const int I = blockIdx.x * kWG + threadIdx.x;
  if (I >= n) return;
  R diag = R(0);
  for (int s = 0; s < K; ++s) {
    const int q = s * n + I;
    R w = R(0);
    for (int t = ptr[q]; t < ptr[q + 1]; ++t) w += Wsrc[idx[t]];
    W[q] = w;
    diag += w;
  }
  Dinv[I] = diag > R(0) ? R(1) / diag : R(0);
}

// Restriction from the fine grid: rc[I] = sum over the children P of aggregate I of the
// residual r_P - (M y)_P of the pre-smoothed y = omega D^-1 r (stored by the PCG update).
// Faces between two children of I cancel in the sum and are skipped.  A work-group is a
// tile of 32 aggregates along x of one coarse row: wave (row parity, plane parity) holds
// 64 consecutive fine cells of one fine row, so every load is coalesced; lane pairs sum
// the x children with a shuffle and the waves' pair sums are added in LDS in a fixed
// order.  Tiles run seg-fastest, then coarse rows, then coarse planes (XCD-aware order).
template <typename R, int D>
__global__ void __launch_bounds__(64 << (D - 1))
k_mg_down0(Grid g, Grid g1, MgTiles tl, const R* __restrict__ Pf, const R* __restrict__ y,
           const R* __restrict__ r, R* __restrict__ rc, const CgState* st) {
  if (st->done) return;
  constexpr int NW = 1 << (D - 1);
  __shared__ R part[NW][32];
  const int tile = xcd_logical_group();
  int b = 0;
  for (int q = 1; q < tl.nb; ++q) b += tile >= tl.off[q] ? 1 : 0;
  int lt = tile - tl.off[b];
  const int* tf = g.tab + b * kTabStride;
  const int* tc = g1.tab + b * kTabStride;
  const int n[3] = {tf[1], tf[2], tf[3]};
  const int cx = tc[1], cy = tc[2];
  const int nseg = tl.nseg[b];
  const int seg = lt % nseg;
  lt /= nseg;
  const int cj = lt % cy, ck = lt / cy;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bit[3] = {lane & 1, w & 1, (w >> 1) & 1};
  Cell c;
  c.b = b;
  c.i = seg * 64 + lane;
  c.j = 2 * cj + bit[1];
  c.k = 2 * ck + bit[2];
  R v = R(0);
  if (c.i < n[0] && c.j < n[1] && c.k < n[2]) {
    const int N = g.N;
    const int pos[3] = {c.i, c.j, c.k};
    const int P = tf[0] + c.i + n[0] * (c.j + n[1] * c.k);
    const R yP = y[P];
    R res = r[P];
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const bool internal = sd ? (bit[j] == 0 && pos[j] + 1 < n[j]) : (bit[j] == 1);
        if (internal) continue;
        const int F = neighbour(g, c, P, j, sd);
        if (F >= 0) {
          const R wf = sd ? Pf[(size_t)j * N + P] : Pf[(size_t)j * N + F];
          res -= wf * (yP - y[F]);
        }
      }
    }
    v = res;
  }
  v += __shfl_xor(v, 1, 64);
  if (!(lane & 1)) part[w][lane >> 1] = v;
  __syncthreads();
  if (threadIdx.x < 32) {
    const int ci = seg * 32 + threadIdx.x;
    if (ci < cx) {
      R sum = part[0][threadIdx.x];
#pragma unroll
      for (int q = 1; q < NW; ++q) sum += part[q][threadIdx.x];
      rc[tc[0] + ci + cx * (cj + cy * ck)] = sum;
    }
  }
}

// The PCG update fused with the fine-grid restriction (multigrid PCG iterations):
//   alpha = (r.z) / (d.q),  x += alpha d,  r' = r - alpha q,  y = omega D^-1 r',
// then rc[I] = sum over the children P of aggregate I of r'_P - (M y)_P as in k_mg_down0.
// y on the far side of a face leaving the aggregate is recomputed from r, q and D^-1
// there (the same expressions as at P).  The residual is double-buffered (rin -> rout)
// so that no work-group reads a value that another one has already overwritten; x is
// updated in place (only at P).  Every work-group re-reduces the stencil kernel's
// partials of d.q; the lead thread advances the iteration index (no other work-group
// reads it in this kernel) and records a breakdown.  Same tiles as k_mg_down0.
template <typename R, int D>
__global__ void __launch_bounds__(64 << (D - 1))
k_mg_down0u(Grid g, Grid g1, MgTiles tl, const R* __restrict__ Pf, const R* __restrict__ Dinv,
            R* __restrict__ x, const R* __restrict__ rin, R* __restrict__ rout, const R* __restrict__ dnew,
            const R* __restrict__ q, R* __restrict__ y, R omega, R* __restrict__ rc, CgState* st,
            const double* __restrict__ partA, int Gp, int par) {
  constexpr int NW = 1 << (D - 1);
  const int done = st->done;
  const double rzp = st->rz[par];
  double t[1];
  {
    // reduce_partials for a work-group of NW waves
    constexpr int WGS = 64 * NW;
    __shared__ double red[NW];
    double v = 0.0;
    for (int w0 = 0; w0 < Gp; w0 += 4 * WGS) {
      double u[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int w = w0 + (int)threadIdx.x + c * WGS;
        u[c] = w < Gp ? partA[w] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) v += u[c];
    }
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double tt = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tt += red[w];
    t[0] = tt;
  }
  if (done) return;
  const double dq = t[0];
  if (!(dq > 0.0) || !std::isfinite(dq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->status = std::isfinite(dq) ? PISO_BREAKDOWN : PISO_E_NAN;
      st->iters = st->k;
      st->done = 1;
    }
    return;
  }
  const R alpha = (R)(rzp / dq);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->k = st->k + 1;
  __shared__ R part[NW][32];
  const int tile = xcd_logical_group();
  int b = 0;
  for (int qq = 1; qq < tl.nb; ++qq) b += tile >= tl.off[qq] ? 1 : 0;
  int lt = tile - tl.off[b];
  const int* tf = g.tab + b * kTabStride;
  const int* tc = g1.tab + b * kTabStride;
  const int n[3] = {tf[1], tf[2], tf[3]};
  const int cx = tc[1], cy = tc[2];
  const int nseg = tl.nseg[b];
  const int seg = lt % nseg;
  lt /= nseg;
  const int cj = lt % cy, ck = lt / cy;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bit[3] = {lane & 1, w & 1, (w >> 1) & 1};
  Cell c;
  c.b = b;
  c.i = seg * 64 + lane;
  c.j = 2 * cj + bit[1];
  c.k = 2 * ck + bit[2];
  R v = R(0);
  if (c.i < n[0] && c.j < n[1] && c.k < n[2]) {
    const int N = g.N;
    const int pos[3] = {c.i, c.j, c.k};
    const int P = tf[0] + c.i + n[0] * (c.j + n[1] * c.k);
    const R rn = rin[P] - alpha * q[P];
    const R yP = omega * Dinv[P] * rn;
    x[P] += alpha * dnew[P];
    rout[P] = rn;
    y[P] = yP;
    R res = rn;
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const bool internal = sd ? (bit[j] == 0 && pos[j] + 1 < n[j]) : (bit[j] == 1);
        if (internal) continue;
        const int F = neighbour(g, c, P, j, sd);
        if (F >= 0) {
          const R wf = sd ? Pf[(size_t)j * N + P] : Pf[(size_t)j * N + F];
          const R yF = omega * Dinv[F] * (rin[F] - alpha * q[F]);
          res -= wf * (yP - yF);
        }
      }
    }
    v = res;
  }
  v += __shfl_xor(v, 1, 64);
  if (!(lane & 1)) part[w][lane >> 1] = v;
  __syncthreads();
  if (threadIdx.x < 32) {
    const int ci = seg * 32 + threadIdx.x;
    if (ci < cx) {
      R sum = part[0][threadIdx.x];
#pragma unroll
      for (int qq = 1; qq < NW; ++qq) sum += part[qq][threadIdx.x];
      rc[tc[0] + ci + cx * (cj + cy * ck)] = sum;
    }
  }
}

// Quad-vectorised form of k_mg_down0u (every block has nx % 4 == 0).  Thread layout:
// lane = p + NP u with NP = 2^(d-1) parities p = (row parity) + 2 (plane parity) and u a
// unit, an x-quad of 4 fine cells (two aggregates in x) of one aggregate row and plane;
// units run x-quad fastest, then aggregate rows, then planes, per block.  All streams at
// the thread's own cells move as 16-byte (float) vectors.  Faces leaving an aggregate:
// in x, the faces of cells 0 and 3 of the quad to the neighbouring quads (their y comes
// from the neighbouring lane when it holds that quad, else it is recomputed from memory)
// and the face between cells 1 and 2 (two aggregates of the same quad); in y and z the
// face to the next row or plane away from the aggregate's other fine row or plane (both
// faces when the aggregate is one fine cell thick).  The NP parity lanes of a unit add
// their aggregate sums with shuffles, and the lane of parity 0 writes the two aggregates.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_mg_down0uq(Grid g, Grid g1, MgQuadTiles tl, const R* __restrict__ Pf, const R* __restrict__ Dinv,
             R* __restrict__ x, const R* __restrict__ rin, R* __restrict__ rout, const R* __restrict__ dnew,
             const R* __restrict__ q, R* __restrict__ y, R omega, R* __restrict__ rc, CgState* st,
             const double* __restrict__ partA, int Gp, int par) {
  constexpr int NP = 1 << (D - 1);
  const int done = st->done;
  const double rzp = st->rz[par];
  const int N = g.N;
  const int grp = xcd_logical_group();
  int b = 0;
  for (int qq = 1; qq < tl.nb; ++qq) b += grp >= tl.off[qq] ? 1 : 0;
  const int* tf = g.tab + b * kTabStride;
  const int* tc = g1.tab + b * kTabStride;
  const int nx = tf[1], ny = tf[2], nz = tf[3], wrap = tf[kTabWrap];
  const int cx = tc[1], cy = tc[2];
  const int nxq = nx >> 2;
  const int lane = threadIdx.x & 63, p = lane & (NP - 1);
  const int u = (grp - tl.off[b]) * (kWG / NP) + ((int)threadIdx.x / NP);
  const int xq = u % nxq, rest = u / nxq;
  // 3D: the aggregate rows are taken in tiles of kRowTile rows, each tile through every
  // plane pair in turn, so that a row pair's neighbours in z are a few work-groups away
  // (still in the XCD's L2) instead of a whole plane of rows
  int cj, ck;
  if (D == 3) {
    constexpr int kRowTile = 8;
    const int cz = tc[3];
    const int full = (cy / kRowTile) * kRowTile;
    if (rest >= cy * cz) {
      cj = ck = 0;   // past the block's units: not valid below
    } else if (rest < full * cz) {
      const int tile = rest / (kRowTile * cz), w = rest - tile * kRowTile * cz;
      ck = w / kRowTile;
      cj = tile * kRowTile + (w - ck * kRowTile);
    } else {
      const int tr = cy - full, w = rest - full * cz;
      ck = w / tr;
      cj = full + (w - ck * tr);
    }
  } else {
    cj = rest % cy;
    ck = rest / cy;
  }
  const int j = 2 * cj + (p & 1), k = D == 3 ? 2 * ck + (p >> 1) : 0;
  const bool valid = u < tl.units[b] && j < ny && k < nz;
  const int i0 = 4 * xq;
  const int P0 = valid ? tf[0] + i0 + nx * (j + ny * k) : 0;
  // own-cell streams are loaded (unconditionally, P0 = 0 when not valid) before the
  // partials of d.q, so that the prologue's latency overlaps them
  Q4<R> xv = ldq(x, P0);
  const Q4<R> dv = ldq(dnew, P0), rv = ldq(rin, P0), qv = ldq(q, P0), Dv = ldq(Dinv, P0);
  Q4<R> px = ldq(Pf, P0);
  double t[1];
  reduce_partials<1>(partA, Gp, t);
  if (done) return;
  const double dq = t[0];
  if (!(dq > 0.0) || !std::isfinite(dq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->status = std::isfinite(dq) ? PISO_BREAKDOWN : PISO_E_NAN;
      st->iters = st->k;
      st->done = 1;
    }
    return;
  }
  const R alpha = (R)(rzp / dq);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->k = st->k + 1;   // no other group reads it here
  // own cells: update, y, store
  Q4<R> yq, res;
  if (valid) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xv.v[e] += alpha * dv.v[e];
      res.v[e] = rv.v[e] - alpha * qv.v[e];
      yq.v[e] = omega * Dv.v[e] * res.v[e];
    }
    stq(x, P0, xv);
    stq(rout, P0, res);
    stq(y, P0, yq);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) yq.v[e] = res.v[e] = px.v[e] = R(0);
  }
  // y of one cell recomputed from memory (neighbours this thread's lanes do not hold)
  auto y1 = [&](int F) { return omega * Dinv[F] * (rin[F] - alpha * q[F]); };
  // x faces: cell 0 to the left quad, cells 1 | 2 inside, cell 3 to the right quad
  const R yl_lane = __shfl_up(yq.v[3], NP, 64), pl_lane = __shfl_up(px.v[3], NP, 64);
  const R yr_lane = __shfl_down(yq.v[0], NP, 64);
  if (valid) {
    // left: face coefficient stored at the left cell
    int F = -1;
    R yl = R(0), pl = R(0);
    if (i0 > 0) {
      if (lane >= NP && xq > 0) {
        yl = yl_lane;
        pl = pl_lane;
        F = P0 - 1;
      } else {
        F = P0 - 1;
        yl = y1(F);
        pl = Pf[F];
      }
    } else {
      F = (wrap & 1) ? P0 + nx - 1 : g.fmap[tf[4] + j + ny * k];
      if (F >= 0) {
        yl = y1(F);
        pl = Pf[F];
      }
    }
    if (F >= 0) res.v[0] -= pl * (yq.v[0] - yl);
    // between the quad's two aggregates
    res.v[1] -= px.v[1] * (yq.v[1] - yq.v[2]);
    res.v[2] -= px.v[1] * (yq.v[2] - yq.v[1]);
    // right: own face coefficient
    int Fr = -1;
    R yr = R(0);
    if (i0 + 4 < nx) {
      Fr = P0 + 4;
      yr = (lane + NP < 64 && xq + 1 < nxq) ? yr_lane : y1(Fr);
    } else {
      Fr = (wrap & 2) ? P0 + 4 - nx : g.fmap[tf[5] + j + ny * k];
      if (Fr >= 0) yr = y1(Fr);
    }
    if (Fr >= 0) res.v[3] -= px.v[3] * (yq.v[3] - yr);
    // y and z faces
#pragma unroll
    for (int a = 1; a < D; ++a) {
      const int pos = a == 1 ? j : k;
      const int n = a == 1 ? ny : nz;
      const int bit = pos & 1;
      const int stride = a == 1 ? nx : nx * ny;
      const R* Pa = Pf + (size_t)a * N;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const bool internal = sd ? (bit == 0 && pos + 1 < n) : (bit == 1);
        if (internal) continue;
        const bool in = sd ? pos + 1 < n : pos > 0;
        const bool wr = ((wrap >> (2 * a + sd)) & 1) != 0;
        if (in || wr) {
          const int Pn = sd ? (in ? P0 + stride : P0 - (n - 1) * stride) : (in ? P0 - stride : P0 + (n - 1) * stride);
          const Q4<R> rn = ldq(rin, Pn), qn = ldq(q, Pn), Dn = ldq(Dinv, Pn);
          const Q4<R> wf = ldq(Pa, sd ? P0 : Pn);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const R yn = omega * Dn.v[e] * (rn.v[e] - alpha * qn.v[e]);
            res.v[e] -= wf.v[e] * (yq.v[e] - yn);
          }
        } else {
          const int base = tf[4 + 2 * a + sd] + (a == 1 ? i0 + nx * k : i0 + nx * j);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int F2 = g.fmap[base + e];
            if (F2 >= 0) {
              const R wf = sd ? Pa[P0 + e] : Pa[F2];
              res.v[e] -= wf * (yq.v[e] - y1(F2));
            }
          }
        }
      }
    }
  }
  // aggregates A (cells 0, 1) and B (cells 2, 3): sum over the NP parity lanes
  R sa = valid ? res.v[0] + res.v[1] : R(0);
  R sb = valid ? res.v[2] + res.v[3] : R(0);
#pragma unroll
  for (int o = 1; o < NP; o <<= 1) {
    sa += __shfl_xor(sa, o, 64);
    sb += __shfl_xor(sb, o, 64);
  }
  if (p == 0 && u < tl.units[b]) {
    const int I = tc[0] + 2 * xq + cx * (cj + cy * ck);
    rc[I] = sa;
    rc[I + 1] = sb;
  }
}

// y = omega D^-1 r (pre-smoothing from zero) after the PCG initialisation.
template <typename R>
__global__ void __launch_bounds__(kWG)
k_mg_prescale(int N, const R* __restrict__ Dinv, const R* __restrict__ r, R omega, R* __restrict__ y) {
  const int P = blockIdx.x * kWG + threadIdx.x;
  if (P < N) y[P] = omega * Dinv[P] * r[P];
}

constexpr int kMgRowMax = 8;   // graph-row slots held in registers

// Graph row of cell P (0 <= P < n): neighbours q[s] (-1 where absent) and weights w[s]
// of the first KR <= kMgRowMax slots (0 beyond the row; a slot inside the row with q < 0 keeps
// its weight, callers use it with a zero difference).  The loads are unconditional
// (slot index clamped into the row) and nothing waits for them here, so that all of
// them are in flight together.
template <typename R, int KR>
__device__ __forceinline__ void mg_row(int n, int K, const int* __restrict__ nbr, const R* __restrict__ W, int P,
                                       int (&q)[KR], R (&w)[KR]) {
  const int Kc = K < KR ? K : KR;   // K >= 1: every level has a slot
#pragma unroll
  for (int s = 0; s < KR; ++s) {
    const int sc = s < Kc ? s : Kc - 1;
    const int qv = nbr[sc * n + P];
    const R wv = W[sc * n + P];
    q[s] = s < Kc ? qv : -1;
    w[s] = s < Kc ? wv : R(0);
  }
}

// r_P - (M x)_P for the pre-smoothed x = omega D^-1 r (absent slots add w (xP - xP) = 0).
template <typename R, int KR>
__device__ __forceinline__ R mg_row_residual(int n, int K, const int* __restrict__ nbr, const R* __restrict__ W,
                                             const R* __restrict__ Dinv, const R* __restrict__ r, int P, R omega) {
  int q[KR];
  R w[KR];
  mg_row<R, KR>(n, K, nbr, W, P, q, w);
  const R rP = r[P];
  const R xP = omega * Dinv[P] * rP;
  R res = rP;
#pragma unroll
  for (int s = 0; s < KR; ++s) {
    const int Q = q[s] >= 0 ? q[s] : P;
    res -= w[s] * (xP - omega * Dinv[Q] * r[Q]);
  }
  for (int s = KR; s < K; ++s) {
    const int Q = nbr[s * n + P];
    if (Q >= 0) res -= W[s * n + P] * (xP - omega * Dinv[Q] * r[Q]);
  }
  return res;
}

// Restriction between coarse levels (graph form).  One thread per (aggregate, child)
// so that the loads of different children are in flight together, and the NCH lanes
// of an aggregate are summed with a fixed butterfly of shuffles (deterministic).  The
// solver state is tested once the first loads are in flight.
template <typename R, int NCH, int KR>
__global__ void __launch_bounds__(kWG)
k_mg_down(int nf, int Kf, const int* __restrict__ nbr, const R* __restrict__ W, const R* __restrict__ Dinv,
          const R* __restrict__ r, const int* __restrict__ child, int nc, R omega, R* __restrict__ rc,
          const CgState* st, int pin) {
  const int done = st->done;
  const int wg = mg_group(pin);
  if (wg < 0) return;
  const int t = wg * kWG + threadIdx.x;
  const int I = t / NCH, q = t % NCH;
  const int P = I < nc ? child[q * nc + I] : -1;
  if (done) return;
  R v = mg_row_residual<R, KR>(nf, Kf, nbr, W, Dinv, r, P >= 0 ? P : 0, omega);
  if (P < 0) v = R(0);
#pragma unroll
  for (int o = 1; o < NCH; o <<= 1) v += __shfl_xor(v, o, 64);
  if (I < nc && q == 0) rc[I] = v;
}

// Single-block levels: the cell at (i, j, k) of extents n, its neighbour in direction
// (axis a, side) as a cell index and its coordinate along a (the cell itself where no
// face leaves that way: its weight is 0 there).
struct MgBox {
  int n[3];
  int wrap;
};

__device__ __forceinline__ void mg_box_nb(const MgBox& bx, const int (&pos)[3], int P, int a, int side, int& Q,
                                          int& qa) {
  const int st = a == 0 ? 1 : (a == 1 ? bx.n[0] : bx.n[0] * bx.n[1]);
  const int p = pos[a], n = bx.n[a];
  if (side) qa = p + 1 < n ? p + 1 : (((bx.wrap >> (2 * a + 1)) & 1) ? 0 : p);
  else qa = p > 0 ? p - 1 : (((bx.wrap >> (2 * a)) & 1) ? n - 1 : p);
  Q = P + (qa - p) * st;
}

__device__ __forceinline__ void mg_box_pos(const MgBox& bx, int P, uint64_t mx, int sx, uint64_t mxy, int sxy, int D,
                                           int (&pos)[3]) {
  const uint32_t jk = fast_div((uint32_t)P, mx, sx);
  pos[0] = P - (int)jk * bx.n[0];
  if (D == 3) {
    pos[2] = (int)fast_div((uint32_t)P, mxy, sxy);
    pos[1] = (int)jk - pos[2] * bx.n[1];
  } else {
    pos[1] = (int)jk;
    pos[2] = 0;
  }
}

// k_mg_down on a single block: children, neighbours and their positions by arithmetic,
// so that all loads of a thread are independent (one memory latency instead of a chain
// of child, neighbour and value loads).  Same sums, in the same slot order.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_mg_down_s(MgBox fb, const R* __restrict__ W, const R* __restrict__ Dinv, const R* __restrict__ r, MgBox cb,
            uint64_t cmx, int csx, uint64_t cmxy, int csxy, int nc, R omega, R* __restrict__ rc, const CgState* st,
            int pin) {
  constexpr int NCH = 1 << D, K = 2 * D;
  const int done = st->done;
  const int wg = mg_group(pin);
  if (wg < 0) return;
  const int t = wg * kWG + threadIdx.x;
  const int I0 = t / NCH, q = t % NCH;
  const int I = I0 < nc ? I0 : 0;
  int cpos[3];
  mg_box_pos(cb, I, cmx, csx, cmxy, csxy, D, cpos);
  const int ch[3] = {2 * cpos[0] + (q & 1), 2 * cpos[1] + ((q >> 1) & 1), D == 3 ? 2 * cpos[2] + (q >> 2) : 0};
  const bool ok = I0 < nc && ch[0] < fb.n[0] && ch[1] < fb.n[1] && ch[2] < fb.n[2];
  // a child past an odd extent is replaced by the aggregate's first child and masked
  const int pos[3] = {ok ? ch[0] : 2 * cpos[0], ok ? ch[1] : 2 * cpos[1], ok ? ch[2] : 2 * cpos[2]};
  const int nf = fb.n[0] * fb.n[1] * fb.n[2];
  const int P = pos[0] + fb.n[0] * (pos[1] + fb.n[1] * pos[2]);
  R w[K], rq[K], dq[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
    int Q, qa;
    mg_box_nb(fb, pos, P, s / 2, s & 1, Q, qa);
    w[s] = W[s * nf + P];
    rq[s] = r[Q];
    dq[s] = Dinv[Q];
  }
  const R rP = r[P], xP = omega * Dinv[P] * rP;
  if (done) return;
  R res = rP;
#pragma unroll
  for (int s = 0; s < K; ++s) res -= w[s] * (xP - omega * dq[s] * rq[s]);
  R v = ok ? res : R(0);
#pragma unroll
  for (int o = 1; o < NCH; o <<= 1) v += __shfl_xor(v, o, 64);
  if (I0 < nc && q == 0) rc[I0] = v;
}

// k_mg_up on a single block, parents and neighbours by arithmetic.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_mg_up_s(MgBox fb, uint64_t mx, int sx, uint64_t mxy, int sxy, const R* __restrict__ W, const R* __restrict__ Dinv,
          const R* __restrict__ r, MgBox cb, const R* __restrict__ ec, R omega, R* __restrict__ e, const CgState* st,
          int pin) {
  constexpr int K = 2 * D;
  const int done = st->done;
  const int wg = mg_group(pin);
  if (wg < 0) return;
  const int n = fb.n[0] * fb.n[1] * fb.n[2];
  const int P = wg * kWG + threadIdx.x;
  if (P >= n) return;
  int pos[3];
  mg_box_pos(fb, P, mx, sx, mxy, sxy, D, pos);
  const int cst[3] = {1, cb.n[0], cb.n[0] * cb.n[1]};
  const int pP = (pos[0] >> 1) + cb.n[0] * ((pos[1] >> 1) + cb.n[1] * (pos[2] >> 1));
  R w[K], rq[K], dq[K], eq[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const int a = s / 2;
    int Q, qa;
    mg_box_nb(fb, pos, P, a, s & 1, Q, qa);
    w[s] = W[s * n + P];
    rq[s] = r[Q];
    dq[s] = Dinv[Q];
    eq[s] = ec[pP + ((qa >> 1) - (pos[a] >> 1)) * cst[a]];
  }
  const R rP = r[P], dP = Dinv[P], eP = ec[pP];
  if (done) return;
  const R zP = omega * dP * rP + eP;
  R mz = R(0);
#pragma unroll
  for (int s = 0; s < K; ++s) mz += w[s] * (zP - (omega * dq[s] * rq[s] + eq[s]));
  e[P] = zP + omega * dP * (rP - mz);
}

// Coarsest level (n <= kMgCoarse cells, one work-group of kMgCoarseThreads): e = B r with
// B the Chebyshev iteration of `steps` steps from zero, preconditioned by D^-1, for the
// interval [lo, hi] of the spectrum of D^-1 M.  M is a weighted graph Laplacian, so that
// spectrum lies in [0, 2]: with hi = 2 the error polynomial p (p(0) = 1) has |p| < 1 on
// (0, 2], hence B is a fixed symmetric positive definite map on the range of M and the
// outer CG stays a plain PCG; eigenvalues below lo are damped less, not amplified.
// Recurrence (theta = (hi + lo) / 2, delta = (hi - lo) / 2, sigma = theta / delta):
//   x = 0, s = r, d = D^-1 r / theta, rho = 1 / sigma;  per step
//   x += d, s -= M d, rho' = 1 / (2 sigma - rho), d = rho' rho d + (2 rho' / delta) D^-1 s,
// with the step coefficients a = rho' rho and b = 2 rho' / delta computed on the host.
// Thread t owns cells t + c kMgCoarseThreads with their graph rows in registers (KR
// slots; longer rows read the rest from global memory); d is exchanged through a double
// buffer in LDS, one barrier per step.  One work-group does all the arithmetic, so a
// step is bound by its VALU work: the LDS addresses are fixed before the steps, the
// buffer roles at compile time, and (M d)_I = d_I sum_s w_s - sum_s w_s d_q(s) takes one
// fused multiply-add per slot.
// Constants span the null space of M (the pressure operator is pure Neumann and the
// grid connected).  The restricted right-hand side has a rounding-size constant part
// which p(0) = 1 leaves in the residual and the iteration amplifies into x (by
// q(0) = -p'(0), about 60 at 12 steps and 160 at 32); in FP32 the iterates of the outer CG then carry a large constant and
// lose their precision (and the form of M d above turns a large constant in d into
// noise).  The coarse solve is therefore Pi B Pi with Pi the projection onto zero mean,
// applied to r and to x (fixed order sums in double): still symmetric and positive
// semi-definite, and unchanged on zero-mean input in exact arithmetic.
template <typename R>
struct MgCheb {
  R inv_theta;
  R a[kMgCoarseStepsMax], b[kMgCoarseStepsMax];
};

template <typename R, int KR>
__device__ __forceinline__ void mg_cheb_step(int n, int K, const int* __restrict__ nbr, const R* __restrict__ W,
                                             const R* dold, R* dnew, R a, R b, const int (&q)[2][KR],
                                             const R (&w)[2][KR], const R (&wsum)[2], const R (&di)[2], R (&x)[2],
                                             R (&res)[2], R (&dv)[2]) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int I = (int)threadIdx.x + c * kMgCoarseThreads;
    if (I < n) {
      R md = dv[c] * wsum[c];
#pragma unroll
      for (int s = 0; s < KR; ++s) md -= w[c][s] * dold[q[c][s]];
      for (int s = KR; s < K; ++s) {   // rows longer than the register block
        const int Q = nbr[s * n + I];
        if (Q >= 0) md += W[s * n + I] * (dv[c] - dold[Q]);
      }
      x[c] += dv[c];
      res[c] -= md;
      dv[c] = a * dv[c] + b * di[c] * res[c];
      dnew[I] = dv[c];   // the other buffer: nobody reads it during this step
    }
  }
}

// Sum over the coarse work-group of two values per thread (fixed order), in every thread.
__device__ __forceinline__ double mg_coarse_sum(double v, double* lds /* [kMgCoarseThreads / 64] */) {
  constexpr int NW = kMgCoarseThreads / 64;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += lds[w];
  __syncthreads();   // lds is reused by the next call
  return t;
}

template <typename R, int KR>
__global__ void __launch_bounds__(kMgCoarseThreads)
k_mg_coarse(int n, int K, const int* __restrict__ nbr, const R* __restrict__ W, const R* __restrict__ Dinv,
            const R* __restrict__ r, MgCheb<R> cc, int steps, R* __restrict__ e, const CgState* st) {
  static_assert(kMgCoarse == 2 * kMgCoarseThreads, "two cells per thread");
  const int done = st->done;   // tested once the row loads are in flight
  __shared__ R ds[2][kMgCoarse];
  int q[2][KR];
  R w[2][KR];
  R x[2], res[2], dv[2], di[2], wsum[2];
  // every load is unconditional (indices clamped into the arrays, results masked after),
  // so that all of them are in flight together
  const int Kc = K < KR ? K : KR;   // K >= 1: every level has a slot
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int I = (int)threadIdx.x + c * kMgCoarseThreads;
    const int Ic = I < n ? I : 0;
#pragma unroll
    for (int s = 0; s < KR; ++s) {
      const int sc = s < Kc ? s : Kc - 1;
      q[c][s] = nbr[sc * n + Ic];
      w[c][s] = W[sc * n + Ic];
    }
    res[c] = r[Ic];
    di[c] = Dinv[Ic];
  }
  if (done) return;
  __shared__ double red[kMgCoarseThreads / 64];
  {
    const int I1 = (int)threadIdx.x + kMgCoarseThreads;
    if ((int)threadIdx.x >= n) res[0] = R(0);
    if (I1 >= n) res[1] = R(0);
    const R mean = (R)(mg_coarse_sum((double)res[0] + (double)res[1], red) / n);
    if ((int)threadIdx.x < n) res[0] -= mean;
    if (I1 < n) res[1] -= mean;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int I = (int)threadIdx.x + c * kMgCoarseThreads;
    const bool on = I < n;
    if (!on) res[c] = di[c] = R(0);
    wsum[c] = R(0);
#pragma unroll
    for (int s = 0; s < KR; ++s) {
      if (!on || s >= Kc || q[c][s] < 0) {   // absent slot: weight 0 on the cell itself
        q[c][s] = on ? I : 0;
        w[c][s] = R(0);
      }
      wsum[c] += w[c][s];   // register slots only: longer rows use the difference form
    }
    x[c] = R(0);
    dv[c] = di[c] * res[c] * cc.inv_theta;
    if (on) ds[0][I] = dv[c];
  }
  __syncthreads();
  int it = 0;
  for (; it + 1 < steps; it += 2) {   // buffer roles fixed at compile time
    mg_cheb_step<R, KR>(n, K, nbr, W, ds[0], ds[1], cc.a[it], cc.b[it], q, w, wsum, di, x, res, dv);
    __syncthreads();
    mg_cheb_step<R, KR>(n, K, nbr, W, ds[1], ds[0], cc.a[it + 1], cc.b[it + 1], q, w, wsum, di, x, res, dv);
    __syncthreads();
  }
  if (it < steps) mg_cheb_step<R, KR>(n, K, nbr, W, ds[0], ds[1], cc.a[it], cc.b[it], q, w, wsum, di, x, res, dv);
  const R mean = (R)(mg_coarse_sum((double)x[0] + (double)x[1], red) / n);   // x is 0 off the level
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int I = (int)threadIdx.x + c * kMgCoarseThreads;
    if (I < n) e[I] = x[c] - mean;
  }
}

// Prolongation and post-smoothing on a coarse level: with z = omega D^-1 r + ec[parent],
// e = z + omega D^-1 (r - M z).  The row's loads are issued together (unrolled slots).
template <typename R, int KR>
__global__ void __launch_bounds__(kWG)
k_mg_up(int n, int K, const int* __restrict__ nbr, const R* __restrict__ W, const R* __restrict__ Dinv,
        const R* __restrict__ r, const int* __restrict__ parent, const R* __restrict__ ec, R omega,
        R* __restrict__ e, const CgState* st, int pin) {
  const int done = st->done;   // tested once the first loads are in flight
  const int wg = mg_group(pin);
  if (wg < 0) return;
  const int P = wg * kWG + threadIdx.x;
  if (P >= n) return;
  int q[KR];
  R w[KR];
  mg_row<R, KR>(n, K, nbr, W, P, q, w);
  const R rP = r[P], dP = Dinv[P];
  const int pP = parent[P];
  if (done) return;
  const R zP = omega * dP * rP + ec[pP];
  R mz = R(0);
#pragma unroll
  for (int s = 0; s < KR; ++s) {
    const int Q = q[s] >= 0 ? q[s] : P;   // absent slots add w (zP - zP) = 0
    mz += w[s] * (zP - (omega * Dinv[Q] * r[Q] + ec[parent[Q]]));
  }
  for (int s = KR; s < K; ++s) {
    const int Q = nbr[s * n + P];
    if (Q >= 0) mz += W[s * n + P] * (zP - (omega * Dinv[Q] * r[Q] + ec[parent[Q]]));
  }
  e[P] = zP + omega * dP * (rP - mz);
}

// Aggregate (level-1 cell) of the fine cell at (b, i, j, k).
__device__ __forceinline__ int mg_parent(const Grid& g1, int b, int i, int j, int k) {
  const int* t = g1.tab + b * kTabStride;
  return t[0] + (i >> 1) + t[1] * ((j >> 1) + t[2] * (k >> 1));
}

// The same on the fine grid (with y = omega D^-1 r as stored by the PCG update), writing
// z and the partial sums of r.z and r.r.  Parents of
// neighbours inside the block follow from the coordinates; across a block side they
// come from the parent table.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_mg_up0(Grid g, Grid g1, const R* __restrict__ Pf, const R* __restrict__ Dinv, const R* __restrict__ r,
         const R* __restrict__ y, const int* __restrict__ parent, const R* __restrict__ ec, R omega, R* __restrict__ z,
         double* __restrict__ partB, const CgState* st) {
  if (st->done) return;
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2] = {0.0, 0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    const Cell c = locate(g, P);
    const int* t = g.tab + c.b * kTabStride;
    const R rP = r[P], dP = Dinv[P];
    const R zP = y[P] + ec[mg_parent(g1, c.b, c.i, c.j, c.k)];
    R mz = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int pos = j == 0 ? c.i : (j == 1 ? c.j : c.k);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int F = neighbour(g, c, P, j, sd);
        if (F >= 0) {
          const bool inside = sd ? pos < t[1 + j] - 1 : pos > 0;
          const int dd = sd ? 1 : -1;
          const int pF = inside ? mg_parent(g1, c.b, c.i + (j == 0 ? dd : 0), c.j + (j == 1 ? dd : 0),
                                            c.k + (j == 2 ? dd : 0))
                                : parent[F];
          const R w = sd ? Pf[(size_t)j * N + P] : Pf[(size_t)j * N + F];
          mz += w * (zP - (y[F] + ec[pF]));
        }
      }
    }
    const R zo = zP + omega * dP * (rP - mz);
    z[P] = zo;
    acc[0] += (double)rP * (double)zo;
    acc[1] += (double)rP * (double)rP;
  }
  write_partials<2>(acc, partB);
}

// Quad form (every block has nx % 4 == 0): cells i0 .. i0+3 of a row share the
// aggregates i0/2 and i0/2 + 1.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_mg_up0_q(Grid g, Grid g1, const R* __restrict__ Pf, const R* __restrict__ Dinv, const R* __restrict__ r,
           const R* __restrict__ y, const int* __restrict__ parent, const R* __restrict__ ec, R omega, R* __restrict__ z,
           double* __restrict__ partB, const CgState* st) {
  if (st->done) return;
  int first, end, stride;
  quad_sweep(g.N >> 2, first, end, stride);
  double acc[2] = {0.0, 0.0};
  for (int qd = first; qd < end; qd += stride) {
    const int P0 = qd << 2;
    const Cell c = locate(g, P0);
    const int* t1 = g1.tab + c.b * kTabStride;
    // operand z = y + e[parent] over the quad at P (row jj, plane kk of this block)
    auto dq = [&](int P, int jj, int kk) {
      const int base = t1[0] + (c.i >> 1) + t1[1] * ((jj >> 1) + t1[2] * (kk >> 1));
      const R e0 = ec[base], e1 = ec[base + 1];
      const Q4<R> a = ldq(y, P);
      Q4<R> o;
      o.v[0] = a.v[0] + e0;
      o.v[1] = a.v[1] + e0;
      o.v[2] = a.v[2] + e1;
      o.v[3] = a.v[3] + e1;
      return o;
    };
    auto d1 = [&](int P, bool known, int ii, int jj, int kk) {
      return y[P] + ec[known ? mg_parent(g1, c.b, ii, jj, kk) : parent[P]];
    };
    const Q4<R> zq = dq(P0, c.j, c.k);
    const Q4<R> M = quad_stencil<R, D>(g, c, P0, Pf, zq, dq, d1);
    const Q4<R> rq = ldq(r, P0), Dq = ldq(Dinv, P0);
    Q4<R> o;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      o.v[e] = zq.v[e] + omega * Dq.v[e] * (rq.v[e] - M.v[e]);
      acc[0] += (double)rq.v[e] * (double)o.v[e];
      acc[1] += (double)rq.v[e] * (double)rq.v[e];
    }
    stq(z, P0, o);
  }
  write_partials<2>(acc, partB);
}

// ------------------------------------------------------------------ host

namespace {

struct HostLevel {
  int n = 0, K = 0;
  std::vector<std::array<int, 3>> dims;   // per block
  std::vector<int> off;                   // per block (+1)
};

int host_neighbour(const piso_ctx* c, int P, int axis, int side) {
  int b = 0;
  while (b + 1 < c->nblocks && P >= c->h_tab[(size_t)(b + 1) * kTabStride]) ++b;
  const int* t = &c->h_tab[(size_t)b * kTabStride];
  const int L = P - t[0];
  const int nx = t[1], ny = t[2];
  const int pos[3] = {L % nx, (L / nx) % ny, L / (nx * ny)};
  const int stride[3] = {1, nx, nx * ny};
  const int n = t[1 + axis];
  if (side && pos[axis] < n - 1) return P + stride[axis];
  if (!side && pos[axis] > 0) return P - stride[axis];
  int tg;
  if (axis == 0) tg = pos[1] + ny * pos[2];
  else if (axis == 1) tg = pos[0] + nx * pos[2];
  else tg = pos[0] + nx * pos[1];
  return c->h_fmap[(size_t)t[4 + 2 * axis + side] + tg];
}

}  // namespace

int mg_build(piso_ctx* c) {
  const int D = c->dim, B = c->nblocks, NCH = 1 << D;
  HostLevel fine;
  fine.n = c->N;
  fine.K = 2 * D;
  fine.dims.resize(B);
  fine.off.resize(B + 1);
  for (int b = 0; b < B; ++b) {
    const int* t = &c->h_tab[(size_t)b * kTabStride];
    fine.dims[b] = {t[1], t[2], t[3]};
    fine.off[b] = t[0];
  }
  fine.off[B] = c->N;
  // finer-level adjacency, slot-major; on the fine grid slot 2*axis + side
  std::vector<int> nbr_f((size_t)fine.K * fine.n);
  for (int P = 0; P < fine.n; ++P)
    for (int a = 0; a < D; ++a)
      for (int sd = 0; sd < 2; ++sd) {
        const int F = host_neighbour(c, P, a, sd);
        nbr_f[(size_t)(2 * a + sd) * fine.n + P] = F >= 0 ? F : -1;
      }
  c->mg.clear();
  HostLevel cur = fine;
  for (int level = 1; level <= kMgMaxLevels; ++level) {
    if (level > 1 && cur.n <= kMgCoarse) break;
    HostLevel nx;
    nx.dims.resize(B);
    nx.off.assign(B + 1, 0);
    for (int b = 0; b < B; ++b) {
      for (int a = 0; a < 3; ++a) nx.dims[b][a] = a < D ? (cur.dims[b][a] + 1) / 2 : 1;
      nx.off[b + 1] = nx.off[b] + nx.dims[b][0] * nx.dims[b][1] * nx.dims[b][2];
    }
    nx.n = nx.off[B];
    if (nx.n >= cur.n) break;
    // parent of each finer cell, children of each aggregate
    std::vector<int> parent(cur.n), child((size_t)NCH * nx.n, -1);
    for (int b = 0; b < B; ++b) {
      const auto& d = cur.dims[b];
      const auto& e = nx.dims[b];
      for (int k = 0; k < d[2]; ++k)
        for (int j = 0; j < d[1]; ++j)
          for (int i = 0; i < d[0]; ++i) {
            const int P = cur.off[b] + i + d[0] * (j + d[1] * k);
            const int I = nx.off[b] + i / 2 + e[0] * (j / 2 + e[1] * (k / 2));
            const int q = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
            parent[P] = I;
            child[(size_t)q * nx.n + I] = P;
          }
    }
    // coarse adjacency and contribution lists (fixed traversal order).  On a single
    // block a finer face in direction (axis, side) leaves an aggregate towards the
    // aggregate next to it in the same direction, so there the slots are the directions
    // 2 * axis + side on every level, as on the fine grid (-1 and weight 0 where no face
    // leaves that way); with several blocks they are numbered as neighbours are found.
    const bool by_dir = B == 1;
    std::vector<int> nb_off(nx.n + 1, 0), nb_list;
    std::vector<int> pr_off(nx.n + 1, 0), pr_slot, pr_face;
    nb_list.reserve((size_t)nx.n * 2 * D);
    int K = 0;
    for (int I = 0; I < nx.n; ++I) {
      const size_t nb0 = nb_list.size(), pr0 = pr_slot.size();
      if (by_dir) nb_list.resize(nb0 + 2 * D, -1);
      for (int q = 0; q < NCH; ++q) {
        const int P = child[(size_t)q * nx.n + I];
        if (P < 0) continue;
        for (int s = 0; s < cur.K; ++s) {
          const int Q = nbr_f[(size_t)s * cur.n + P];
          if (Q < 0) continue;
          const int J = parent[Q];
          if (J == I) continue;
          int slot = -1;
          if (by_dir) {
            slot = s;
            if (nb_list[nb0 + s] >= 0 && nb_list[nb0 + s] != J)
              return fail(c, PISO_E_ARG, "multigrid: aggregate with two neighbours in one direction");
            nb_list[nb0 + s] = J;
          } else {
            for (size_t u = nb0; u < nb_list.size(); ++u)
              if (nb_list[u] == J) slot = (int)(u - nb0);
            if (slot < 0) {
              slot = (int)(nb_list.size() - nb0);
              nb_list.push_back(J);
            }
          }
          long long face;
          if (level == 1) {
            const int a = s / 2;
            face = (long long)a * c->N + ((s & 1) ? P : Q);
          } else {
            face = (long long)s * cur.n + P;
          }
          if (face > INT32_MAX) return fail(c, PISO_E_ARG, "multigrid: face index overflow");
          pr_slot.push_back(slot);
          pr_face.push_back((int)face);
        }
      }
      nb_off[I + 1] = (int)nb_list.size();
      pr_off[I + 1] = (int)pr_slot.size();
      K = std::max(K, (int)(nb_list.size() - nb0));
      (void)pr0;
    }
    if (K == 0) K = 1;
    std::vector<int> nbr((size_t)K * nx.n, -1), ptr((size_t)K * nx.n + 1, 0), idx;
    idx.reserve(pr_face.size());
    for (int I = 0; I < nx.n; ++I)
      for (int u = nb_off[I]; u < nb_off[I + 1]; ++u) nbr[(size_t)(u - nb_off[I]) * nx.n + I] = nb_list[u];
    size_t q = 0;
    for (int s = 0; s < K; ++s)
      for (int I = 0; I < nx.n; ++I) {
        for (int u = pr_off[I]; u < pr_off[I + 1]; ++u)
          if (pr_slot[u] == s) idx.push_back(pr_face[u]);
        ptr[++q] = (int)idx.size();
      }
    nx.K = K;
    MgLevel L;
    L.n = nx.n;
    L.K = K;
    if (by_dir) {
      for (int a = 0; a < 3; ++a) L.dims[a] = nx.dims[0][a];
      div_magic((uint32_t)L.dims[0], L.mx_lo, L.mx_hi, L.mx_sh);
      div_magic((uint32_t)(L.dims[0] * L.dims[1]), L.mxy_lo, L.mxy_hi, L.mxy_sh);
    }
    if (int rc = upload(c, (void**)&L.nbr, nbr)) return rc;
    if (int rc = upload(c, (void**)&L.child, child)) return rc;
    if (int rc = upload(c, (void**)&L.parent, parent)) return rc;
    if (int rc = upload(c, (void**)&L.ptr, ptr)) return rc;
    if (int rc = upload(c, (void**)&L.idx, idx)) return rc;
    if (int rc = dev_alloc(c, &L.W, (size_t)K * nx.n * c->esz)) return rc;
    if (int rc = dev_alloc(c, &L.Dinv, (size_t)nx.n * c->esz)) return rc;
    if (int rc = dev_alloc(c, &L.r, (size_t)nx.n * c->esz)) return rc;
    if (int rc = dev_alloc(c, &L.e, (size_t)nx.n * c->esz)) return rc;
    if (level == 1) {
      // level 1 as a block table for the structured fine-level kernels
      std::vector<int> tab1((size_t)B * kTabStride, 0);
      for (int b = 0; b < B; ++b) {
        int* t = &tab1[(size_t)b * kTabStride];
        t[0] = nx.off[b];
        t[1] = nx.dims[b][0];
        t[2] = nx.dims[b][1];
        t[3] = nx.dims[b][2];
        uint32_t lo, hi;
        int sh;
        div_magic((uint32_t)t[1], lo, hi, sh);
        t[10] = (int)lo; t[11] = (int)hi; t[12] = sh;
        div_magic((uint32_t)(t[1] * t[2]), lo, hi, sh);
        t[13] = (int)lo; t[14] = (int)hi; t[15] = sh;
      }
      int* d_tab1 = nullptr;
      if (int rc = upload(c, (void**)&d_tab1, tab1)) return rc;
      c->mg_g1.dim = D;
      c->mg_g1.nblocks = B;
      c->mg_g1.N = nx.n;
      c->mg_g1.NB = 0;
      c->mg_g1.tab = d_tab1;
      c->mg_g1.fmap = nullptr;
      // fine-grid restriction tiles: 64 fine x-cells (32 aggregates) of one coarse row
      c->mg_tiles.nb = B;
      c->mg_tiles.off[0] = 0;
      for (int b = 0; b < B; ++b) {
        const int nseg = (cur.dims[b][0] + 63) / 64;
        c->mg_tiles.nseg[b] = nseg;
        c->mg_tiles.off[b + 1] = c->mg_tiles.off[b] + nseg * nx.dims[b][1] * nx.dims[b][2];
      }
      // quad tiles: units of one x-quad per aggregate row and plane, kWG / 2^(d-1) per group
      const int upw = kWG >> (D - 1);
      c->mg_qtiles.nb = B;
      c->mg_qtiles.off[0] = 0;
      for (int b = 0; b < B; ++b) {
        const long long units = (long long)(cur.dims[b][0] / 4) * nx.dims[b][1] * nx.dims[b][2];
        if (units > INT32_MAX / 2) return fail(c, PISO_E_ARG, "multigrid: block too large");
        c->mg_qtiles.units[b] = (int)units;
        c->mg_qtiles.off[b + 1] = c->mg_qtiles.off[b] + (int)((units + upw - 1) / upw);
      }
    }
    c->mg.push_back(L);
    nbr_f.swap(nbr);
    cur = nx;
  }
  if (!c->mg.empty() && c->mg.back().n > kMgCoarse) c->mg.clear();   // cannot happen: blocks <= 16
  // PISO_MG_GRAPH=1 keeps the table-driven kernels on single-block grids
  c->mg_struct = B == 1 && !c->mg.empty();
  if (const char* e = std::getenv("PISO_MG_GRAPH")) c->mg_struct = c->mg_struct && e[0] != '1';
  if (!c->mg.empty()) {
    if (int rc = dev_alloc(c, &c->k_z, (size_t)c->N * c->esz)) return rc;
    if (int rc = dev_alloc(c, &c->k_y, (size_t)c->N * c->esz)) return rc;
  }
  return PISO_OK;
}

static int mg_check(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

template <typename R>
int mg_setup(piso_ctx* c, hipStream_t s, const R* Pf) {
  const R* src = Pf;
  for (const MgLevel& L : c->mg) {
    k_mg_coef<R><<<grid_cells(L.n), kWG, 0, s>>>(L.n, L.K, L.ptr, L.idx, src, (R*)L.W, (R*)L.Dinv);
    src = (const R*)L.W;
  }
  return mg_check(c, "k_mg_coef");
}

template <typename R>
int mg_prescale(piso_ctx* c, hipStream_t s, const R* Dinv, const R* r, R* y) {
  k_mg_prescale<R><<<grid_cells(c->N), kWG, 0, s>>>(c->N, Dinv, r, (R)kMgOmega, y);
  return mg_check(c, "k_mg_prescale");
}

// Chebyshev step coefficients of the coarsest solve (see k_mg_coarse), in double.
template <typename R>
static MgCheb<R> mg_cheb_coef(int steps) {
  const double lo = 2.0 / kMgChebRatio, hi = 2.0;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  MgCheb<R> cc{};
  cc.inv_theta = (R)(1.0 / theta);
  double rho = 1.0 / sigma;
  for (int i = 0; i < steps && i < kMgCoarseStepsMax; ++i) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    cc.a[i] = (R)(rn * rho);
    cc.b[i] = (R)(2.0 * rn / delta);
    rho = rn;
  }
  return cc;
}

// The V-cycle after the fine-grid restriction (level-1 residual in mg[0].r): coarse
// levels, coarsest solve, prolongations, and the fine-grid prolongation and smoothing
// into z with the partial sums of r.z and r.r.
template <typename R>
static int mg_tail(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* r, const R* y, R* z,
                   CgState* st, double* partB, int G) {
  const int nl = (int)c->mg.size();
  const R om = (R)kMgOmega, omc = (R)kMgOmegaCoarse;
  const Grid& g1 = c->mg_g1;
  // launches of at most kMgPinGroups work-groups run on one XCD (see mg_group)
  auto pinned = [](int groups) { return groups <= kMgPinGroups ? 1 : 0; };
  auto grid_of = [](int groups, int pin) { return pin ? 8 * groups : groups; };
  const int wrap = c->h_tab[kTabWrap];
  auto box = [&](const MgLevel& L) { return MgBox{{L.dims[0], L.dims[1], L.dims[2]}, wrap}; };
  auto m64 = [](uint32_t lo, uint32_t hi) { return (uint64_t)lo | ((uint64_t)hi << 32); };
  for (int l = 1; l < nl; ++l) {
    const MgLevel& F = c->mg[l - 1];
    const MgLevel& C = c->mg[l];
    const int gw = grid_cells((1 << c->dim) * C.n), pin = pinned(gw);
    if (c->mg_struct) {
      auto ks = c->dim == 2 ? k_mg_down_s<R, 2> : k_mg_down_s<R, 3>;
      launch_timed(c, s, kTimeMgCoarse, ks, grid_of(gw, pin), box(F), (const R*)F.W, (const R*)F.Dinv,
                   (const R*)F.r, box(C), m64(C.mx_lo, C.mx_hi), C.mx_sh, m64(C.mxy_lo, C.mxy_hi), C.mxy_sh, C.n, omc,
                   (R*)C.r, (const CgState*)st, pin);
      continue;
    }
    auto kern = c->dim == 2 ? (F.K <= 4 ? k_mg_down<R, 4, 4> : (F.K <= 6 ? k_mg_down<R, 4, 6> : k_mg_down<R, 4, 8>))
                            : (F.K <= 4 ? k_mg_down<R, 8, 4> : (F.K <= 6 ? k_mg_down<R, 8, 6> : k_mg_down<R, 8, 8>));
    launch_timed(c, s, kTimeMgCoarse, kern, grid_of(gw, pin), F.n, F.K, (const int*)F.nbr, (const R*)F.W,
                 (const R*)F.Dinv, (const R*)F.r, (const int*)C.child, C.n, omc, (R*)C.r, (const CgState*)st, pin);
  }
  {
    const MgLevel& L = c->mg[nl - 1];
    const int steps = c->dim == 3 ? kMgCoarseSteps3 : kMgCoarseSteps2;
    const MgCheb<R> cc = mg_cheb_coef<R>(steps);
    auto kern = L.K <= 4 ? k_mg_coarse<R, 4> : (L.K <= 6 ? k_mg_coarse<R, 6> : k_mg_coarse<R, 8>);
    launch_timed_wg(c, s, kTimeMgCoarse, kern, 1, kMgCoarseThreads, L.n, L.K, (const int*)L.nbr, (const R*)L.W,
                    (const R*)L.Dinv, (const R*)L.r, cc, steps, (R*)L.e, (const CgState*)st);
  }
  for (int l = nl - 2; l >= 0; --l) {
    const MgLevel& F = c->mg[l];
    const MgLevel& C = c->mg[l + 1];
    const int gw = grid_cells(F.n), pin = pinned(gw);
    if (c->mg_struct) {
      auto ks = c->dim == 2 ? k_mg_up_s<R, 2> : k_mg_up_s<R, 3>;
      launch_timed(c, s, kTimeMgCoarse, ks, grid_of(gw, pin), box(F), m64(F.mx_lo, F.mx_hi), F.mx_sh,
                   m64(F.mxy_lo, F.mxy_hi), F.mxy_sh, (const R*)F.W, (const R*)F.Dinv, (const R*)F.r, box(C),
                   (const R*)C.e, omc, (R*)F.e, (const CgState*)st, pin);
      continue;
    }
    auto kern = F.K <= 4 ? k_mg_up<R, 4> : (F.K <= 6 ? k_mg_up<R, 6> : k_mg_up<R, 8>);
    launch_timed(c, s, kTimeMgCoarse, kern, grid_of(gw, pin), F.n, F.K, (const int*)F.nbr, (const R*)F.W,
                 (const R*)F.Dinv, (const R*)F.r, (const int*)C.parent, (const R*)C.e, omc, (R*)F.e,
                 (const CgState*)st, pin);
  }
  if (c->mg_line_axis) return line_post<R>(c, s, Pf, Dinv, r, y, (const R*)c->mg[0].e, z, partB, st);
  {
    const MgLevel& L1 = c->mg[0];
    const bool quad = c->quad && ((((uintptr_t)Pf) | ((uintptr_t)Dinv) | ((uintptr_t)r) | ((uintptr_t)y) |
                                   ((uintptr_t)z)) & 15u) == 0;
    const R* e1 = (const R*)L1.e;
    if (quad && zm_use(c, sizeof(R))) {
      zm_launch_up<R>(c, s, Pf, Dinv, r, y, (const int*)L1.parent, e1, z, partB, (const CgState*)st);
    } else if (quad) {
      if (c->dim == 2)
        launch_timed(c, s, kTimeMgUp0, k_mg_up0_q<R, 2>, G, c->grid, g1, Pf, Dinv, r, y, (const int*)L1.parent, e1,
                     om, z, partB, (const CgState*)st);
      else
        launch_timed(c, s, kTimeMgUp0, k_mg_up0_q<R, 3>, G, c->grid, g1, Pf, Dinv, r, y, (const int*)L1.parent, e1,
                     om, z, partB, (const CgState*)st);
    } else {
      if (c->dim == 2)
        launch_timed(c, s, kTimeMgUp0, k_mg_up0<R, 2>, G, c->grid, g1, Pf, Dinv, r, y, (const int*)L1.parent, e1, om,
                     z, partB, (const CgState*)st);
      else
        launch_timed(c, s, kTimeMgUp0, k_mg_up0<R, 3>, G, c->grid, g1, Pf, Dinv, r, y, (const int*)L1.parent, e1, om,
                     z, partB, (const CgState*)st);
    }
  }
  return mg_check(c, "multigrid V-cycle");
}

template <typename R>
int mg_apply(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* r, const R* y, R* z, CgState* st,
             double* partB, int G) {
  const int lr = line_restrict<R>(c, s, Pf, r, y, st);
  if (lr < 0) return lr;
  if (lr == 0) return mg_tail<R>(c, s, Pf, Dinv, r, y, z, st, partB, G);
  const int tiles = c->mg_tiles.off[c->nblocks];
  if (c->dim == 2)
    launch_timed_wg(c, s, kTimeMgDown0, k_mg_down0<R, 2>, tiles, 128, c->grid, c->mg_g1, c->mg_tiles, Pf, y, r,
                    (R*)c->mg[0].r, (const CgState*)st);
  else
    launch_timed_wg(c, s, kTimeMgDown0, k_mg_down0<R, 3>, tiles, 256, c->grid, c->mg_g1, c->mg_tiles, Pf, y, r,
                    (R*)c->mg[0].r, (const CgState*)st);
  return mg_tail<R>(c, s, Pf, Dinv, r, y, z, st, partB, G);
}

template <typename R>
int mg_update_apply(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, R* x, const R* rin, R* rout,
                    const R* dnew, const R* q, R* y, R* z, CgState* st, const double* partA, int Gp, int par,
                    double* partB, int G) {
  const R om = (R)kMgOmega;
  const bool quad = c->quad && ((((uintptr_t)Pf) | ((uintptr_t)Dinv) | ((uintptr_t)x) | ((uintptr_t)rin) |
                                 ((uintptr_t)rout) | ((uintptr_t)dnew) | ((uintptr_t)q) | ((uintptr_t)y)) & 15u) == 0;
  if (quad && zm_use(c, sizeof(R))) {
    zm_launch_down<R>(c, s, Pf, Dinv, x, rin, rout, dnew, q, y, (R*)c->mg[0].r, st, partA, Gp, par);
  } else if (quad) {
    const int groups = c->mg_qtiles.off[c->nblocks];
    if (c->dim == 2)
      launch_timed(c, s, kTimeCgUpdateMg, k_mg_down0uq<R, 2>, groups, c->grid, c->mg_g1, c->mg_qtiles, Pf, Dinv, x,
                   rin, rout, dnew, q, y, om, (R*)c->mg[0].r, st, partA, Gp, par);
    else
      launch_timed(c, s, kTimeCgUpdateMg, k_mg_down0uq<R, 3>, groups, c->grid, c->mg_g1, c->mg_qtiles, Pf, Dinv, x,
                   rin, rout, dnew, q, y, om, (R*)c->mg[0].r, st, partA, Gp, par);
  } else {
    const int tiles = c->mg_tiles.off[c->nblocks];
    if (c->dim == 2)
      launch_timed_wg(c, s, kTimeCgUpdateMg, k_mg_down0u<R, 2>, tiles, 128, c->grid, c->mg_g1, c->mg_tiles, Pf,
                      Dinv, x, rin, rout, dnew, q, y, om, (R*)c->mg[0].r, st, partA, Gp, par);
    else
      launch_timed_wg(c, s, kTimeCgUpdateMg, k_mg_down0u<R, 3>, tiles, 256, c->grid, c->mg_g1, c->mg_tiles, Pf,
                      Dinv, x, rin, rout, dnew, q, y, om, (R*)c->mg[0].r, st, partA, Gp, par);
  }
  return mg_tail<R>(c, s, Pf, Dinv, (const R*)rout, (const R*)y, z, st, partB, G);
}

template int mg_setup<float>(piso_ctx*, hipStream_t, const float*);
template int mg_setup<double>(piso_ctx*, hipStream_t, const double*);
template int mg_prescale<float>(piso_ctx*, hipStream_t, const float*, const float*, float*);
template int mg_prescale<double>(piso_ctx*, hipStream_t, const double*, const double*, double*);
template int mg_apply<float>(piso_ctx*, hipStream_t, const float*, const float*, const float*, const float*, float*,
                             CgState*, double*, int);
template int mg_apply<double>(piso_ctx*, hipStream_t, const double*, const double*, const double*, const double*,
                              double*, CgState*, double*, int);
template int mg_update_apply<float>(piso_ctx*, hipStream_t, const float*, const float*, float*, const float*, float*,
                                    const float*, const float*, float*, float*, CgState*, const double*, int, int,
                                    double*, int);
template int mg_update_apply<double>(piso_ctx*, hipStream_t, const double*, const double*, double*, const double*,
                                     double*, const double*, const double*, double*, double*, CgState*,
                                     const double*, int, int, double*, int);

}  // namespace piso
