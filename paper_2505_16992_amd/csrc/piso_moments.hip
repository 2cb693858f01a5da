// Arbitrary-order online (co)moments over homogeneous planes, their gradient, cell-centred
// field gradients and the turbulent energy-budget terms (Sec. 2.5 of arXiv 2505.16992).
//
// Comoments.  m variables per sample (fields x [m][N]); per plane the state record is
// [n, mu_0 .. mu_{m-1}, S_alpha for every multi-index alpha of total order 2 .. K], where
// S_alpha = sum over the plane's samples of prod_i (x_i - mu_i)^alpha_i, a multi-index
// written as its sorted tuple of variable indices, stored by order and then
// lexicographically (order 2: (0,0), (0,1), .., the covariance pairs).  One work-group
// owns one plane: it takes the batch mean of the new step in a first pass, the batch
// central sums of every alpha in a second, and merges them with the state by the
// binomial expansion of the deviations from the combined mean,
//   S_alpha = sum_{beta <= alpha} C(alpha, beta) [S^A_beta c_A^(alpha - beta)
//                                                  + S^B_beta c_B^(alpha - beta)],
//   c_A = -delta n_B / n,  c_B = delta n_A / n,  delta = mu_B - mu_A,
// with S_0 = n_X and S of order 1 zero (the online merging of arbitrary-order moments the
// paper builds on).  Moments M_alpha = S_alpha / n; their gradient with respect to one
// accumulated sample x_t is (alpha_k / n)(dev_t^(alpha - e_k) - M_(alpha - e_k)).
//
// Budget terms (planes normal to axis a, the other axes homogeneous), R the covariance of
// u, G^(k) the covariance of du/dx_k, X_ij = cov(u_i, dp/dx_j):
//   P_ij = -(R_ia dU_j/dx_a + R_ja dU_i/dx_a),  eps_ij = 2 sum_k G^(k)_ij,
//   T_ij = -d<u_i' u_j' u_a'>/dx_a,  D_ij = d^2 R_ij / dx_a^2,  Pi_ij = -(X_ij + X_ji).
// Profile derivatives across the planes use the plane's metric: T_aa (f_+ - f_-) / 2 and
// (1/J)[alpha_+ (f_+ - f) + alpha_- (f_- - f)] with alpha = J T_aa^2 and face weights
// lerp(alpha) (the step's diffusion discretisation); across a wall the ghost 2 f_w - f
// and the face weight 2 alpha, f_w = the wall's mean velocity for U and zero for every
// fluctuation statistic.  Field gradients: d phi/dx_i = sum_j T_ji (phi_+j - phi_-j) / 2,
// a Dirichlet face giving the ghost 2 phi_b - phi_P (or phi_P when no face values are
// given: the step's pressure gradient).
#include <string>

#include "piso_impl.h"

namespace piso {

namespace {

constexpr int kMomMaxAlpha = 32;   // multi-indices of order 2..K for m <= 6 (K = 2) or m <= 3 (K = 4)
constexpr int kMomMaxVars = 6;

// Multi-index table passed by value: tuple of variable indices (padded with -1) and
// exponents per variable.
struct MomTab {
  int n;                                   // number of multi-indices
  signed char tup[kMomMaxAlpha][4];
  signed char e[kMomMaxAlpha][kMomMaxVars];
};

int momtab(int m, int K, MomTab& t) {
  t.n = 0;
  int idx[4];
  for (int o = 2; o <= K; ++o) {
    // sorted tuples (i_1 <= .. <= i_o) in lexicographic order
    for (int q = 0; q < o; ++q) idx[q] = 0;
    for (;;) {
      if (t.n >= kMomMaxAlpha) return -1;
      for (int q = 0; q < 4; ++q) t.tup[t.n][q] = q < o ? (signed char)idx[q] : (signed char)-1;
      for (int v = 0; v < kMomMaxVars; ++v) t.e[t.n][v] = 0;
      for (int q = 0; q < o; ++q) t.e[t.n][idx[q]]++;
      ++t.n;
      int q = o - 1;
      while (q >= 0 && idx[q] == m - 1) --q;
      if (q < 0) break;
      ++idx[q];
      for (int r = q + 1; r < o; ++r) idx[r] = idx[q];
    }
  }
  return t.n;
}

__device__ __forceinline__ int plane_cell_m(int axis, int p, int t, int nx, int ny) {
  if (axis == 1) {
    const int i = t % nx, k = t / nx;
    return i + nx * (p + ny * k);
  }
  if (axis == 0) {
    const int j = t % ny, k = t / ny;
    return p + nx * (j + ny * k);
  }
  const int i = t % nx, j = t / nx;
  return i + nx * (j + ny * p);
}

__device__ __forceinline__ double ipow(double x, int k) {
  double r = 1.0;
  for (int q = 0; q < k; ++q) r *= x;
  return r;
}

__device__ __forceinline__ int binom(int n, int k) {
  int r = 1;
  for (int q = 1; q <= k; ++q) r = r * (n - k + q) / q;
  return r;
}

// Index of the multi-index with exponents e in the table (-1 if its order is below 2).
__device__ __forceinline__ int mom_find(const MomTab& t, int M, const int* e) {
  for (int q = 0; q < t.n; ++q) {
    bool same = true;
    for (int v = 0; v < M; ++v) same &= t.e[q][v] == e[v];
    if (same) return q;
  }
  return -1;
}

}  // namespace

template <typename R, int M>
__global__ void __launch_bounds__(kWG)
k_mom_acc(const R* __restrict__ x, int N, int nx, int ny, int ms, int axis, MomTab tab,
          double* __restrict__ state) {
  const int p = blockIdx.x;
  const int NA = tab.n;
  const int REC = 1 + M + NA;
  double s1[M];
#pragma unroll
  for (int i = 0; i < M; ++i) s1[i] = 0.0;
  for (int t = threadIdx.x; t < ms; t += kWG) {
    const int P = plane_cell_m(axis, p, t, nx, ny);
#pragma unroll
    for (int i = 0; i < M; ++i) s1[i] += (double)x[(size_t)i * N + P];
  }
  wg_sum_all<M>(s1);
  double mu_b[M];
#pragma unroll
  for (int i = 0; i < M; ++i) mu_b[i] = s1[i] / ms;
  double s2[kMomMaxAlpha];
#pragma unroll
  for (int q = 0; q < kMomMaxAlpha; ++q) s2[q] = 0.0;
  for (int t = threadIdx.x; t < ms; t += kWG) {
    const int P = plane_cell_m(axis, p, t, nx, ny);
    double dv[M];
#pragma unroll
    for (int i = 0; i < M; ++i) dv[i] = (double)x[(size_t)i * N + P] - mu_b[i];
#pragma unroll
    for (int q = 0; q < kMomMaxAlpha; ++q) {
      if (q < NA) {
        double pr = 1.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int v = tab.tup[q][r];
          if (v >= 0) pr *= dv[v];
        }
        s2[q] += pr;
      }
    }
  }
  __shared__ double lds[kMomMaxAlpha * kWaves];
  wg_sum<kMomMaxAlpha>(s2, lds);
  if (threadIdx.x != 0) return;
  double* rec = state + (size_t)p * REC;
  const double nA = rec[0], nB = (double)ms, n = nA + nB;
  double delta[M], cA[M], cB[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    delta[i] = mu_b[i] - rec[1 + i];
    cA[i] = -delta[i] * (nB / n);
    cB[i] = delta[i] * (nA / n);
  }
  double out[kMomMaxAlpha];
  for (int q = 0; q < NA; ++q) {
    // sum over beta <= alpha: beta = 0, then every table entry (order >= 2) below alpha;
    // order-1 betas contribute nothing (central sums of order 1 vanish)
    double acc = nA * 1.0, accB = nB * 1.0;
    {
      double pa = 1.0, pb = 1.0;
      for (int v = 0; v < M; ++v) {
        pa *= ipow(cA[v], tab.e[q][v]);
        pb *= ipow(cB[v], tab.e[q][v]);
      }
      acc *= pa;
      accB *= pb;
    }
    double sum = acc + accB;
    for (int b = 0; b < NA; ++b) {
      bool le = true;
      for (int v = 0; v < M; ++v) le &= tab.e[b][v] <= tab.e[q][v];
      if (!le) continue;
      double c = 1.0, pa = 1.0, pb = 1.0;
      for (int v = 0; v < M; ++v) {
        const int a = tab.e[q][v], bb = tab.e[b][v];
        c *= binom(a, bb);
        pa *= ipow(cA[v], a - bb);
        pb *= ipow(cB[v], a - bb);
      }
      sum += c * (rec[1 + M + b] * pa + s2[b] * pb);
    }
    out[q] = sum;
  }
  for (int q = 0; q < NA; ++q) rec[1 + M + q] = out[q];
#pragma unroll
  for (int i = 0; i < M; ++i) rec[1 + i] += delta[i] * (nB / n);
  rec[0] = n;
}

__global__ void __launch_bounds__(kWG)
k_mom_final(int n_planes, int M, int NA, const double* __restrict__ state, double* __restrict__ mean,
            double* __restrict__ mom) {
  const int p = blockIdx.x * kWG + threadIdx.x;
  if (p >= n_planes) return;
  const int REC = 1 + M + NA;
  const double* rec = state + (size_t)p * REC;
  const double n = rec[0];
  for (int i = 0; i < M; ++i) mean[p * M + i] = rec[1 + i];
  for (int q = 0; q < NA; ++q) mom[(size_t)p * NA + q] = n > 0 ? rec[1 + M + q] / n : 0.0;
}

template <typename R, int M>
__global__ void __launch_bounds__(kWG)
k_mom_bwd(const R* __restrict__ x, int N, int nx, int ny, int axis, MomTab tab, const double* __restrict__ state,
          const double* __restrict__ mbar, const double* __restrict__ obar, R* __restrict__ dx) {
  const int P = cell_of_thread(N);
  if (P < 0) return;
  const int NA = tab.n;
  const int REC = 1 + M + NA;
  const int i0 = P % nx, j0 = (P / nx) % ny, k0 = P / (nx * ny);
  const int p = axis == 0 ? i0 : (axis == 1 ? j0 : k0);
  const double* rec = state + (size_t)p * REC;
  const double inv_n = 1.0 / rec[0];
  double dv[M], g[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    dv[i] = (double)x[(size_t)i * N + P] - rec[1 + i];
    g[i] = mbar[p * M + i];
  }
  for (int q = 0; q < NA; ++q) {
    const double ob = obar[(size_t)p * NA + q];
    if (ob == 0.0) continue;
    for (int k = 0; k < M; ++k) {
      const int ak = tab.e[q][k];
      if (ak == 0) continue;
      int r[kMomMaxVars];
      int ord = 0;
      double pr = 1.0;
      for (int v = 0; v < M; ++v) {
        r[v] = tab.e[q][v] - (v == k ? 1 : 0);
        ord += r[v];
        pr *= ipow(dv[v], r[v]);
      }
      if (ord >= 2) pr -= rec[1 + M + mom_find(tab, M, r)] * inv_n;
      g[k] += ob * ak * pr;
    }
  }
#pragma unroll
  for (int i = 0; i < M; ++i) dx[(size_t)i * N + P] += (R)(g[i] * inv_n);
}

// d phi_c / d x_i for the nc components of phi: out[i][c][P].  JT is J T (diagonal-only
// [d][N] when diag), invJ = 1/J.  phi_b [nc][NB] or null (then the face value is phi_P).
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_field_grad(Grid g, const R* __restrict__ JT, const R* __restrict__ invJ, const R* __restrict__ phi, int nc,
             const R* __restrict__ phib, R* __restrict__ out) {
  const int N = g.N, NB = g.NB;
  const int P = cell_of_thread(N);
  if (P < 0) return;
  const Cell c = locate(g, P);
  int Fp[D], Fm[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    Fp[j] = neighbour(g, c, P, j, 1);
    Fm[j] = neighbour(g, c, P, j, 0);
  }
  const R iJ = invJ[P];
  for (int q = 0; q < nc; ++q) {
    const R* f = phi + (size_t)q * N;
    const R fP = f[P];
    R dxi[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R vp, vm;
      if (Fp[j] >= 0) vp = f[Fp[j]];
      else vp = phib ? R(2) * phib[(size_t)q * NB + (-1 - Fp[j])] - fP : fP;
      if (Fm[j] >= 0) vm = f[Fm[j]];
      else vm = phib ? R(2) * phib[(size_t)q * NB + (-1 - Fm[j])] - fP : fP;
      dxi[j] = R(0.5) * (vp - vm);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      R s = R(0);
      if constexpr (DIAG) {
        s = JT[(size_t)i * N + P] * iJ * dxi[i];
      } else {
#pragma unroll
        for (int j = 0; j < D; ++j) s += JT[(size_t)(j * D + i) * N + P] * iJ * dxi[j];
      }
      out[((size_t)i * nc + q) * N + P] = s;
    }
  }
}

// Budget terms per plane (one thread per plane) from the accumulated states: su (m = d,
// order >= 3, table tu), sg[k] (m = d, order 2; k = 0 .. d-1, each REC_g long per plane),
// sup (m = 2d, order 2, table tp).  Planes normal to axis a; tmet[p] = T_aa and jm[p] = J
// of the plane.  out[term][p][pair], terms P, eps, T, D, Pi.
template <int D>
__global__ void __launch_bounds__(kWG)
k_budget(int np, int a, int periodic, MomTab tu, MomTab tg, MomTab tp, const double* __restrict__ su,
         const double* __restrict__ sg, const double* __restrict__ sup, const double* __restrict__ tmet,
         const double* __restrict__ jm, double wl0, double wl1, double wl2, double wh0, double wh1, double wh2,
         double* __restrict__ out) {
  const int p = blockIdx.x * kWG + threadIdx.x;
  if (p >= np) return;
  constexpr int NP = D * (D + 1) / 2;
  const int RU = 1 + D + tu.n, RG = 1 + D + tg.n, RP = 1 + 2 * D + tp.n;
  const double wl[3] = {wl0, wl1, wl2}, wh[3] = {wh0, wh1, wh2};
  // moment of u for the exponent vector e (order 2 or 3) at plane q
  auto Mu = [&](int q, const int* e) { const double* r = su + (size_t)q * RU; return r[1 + D + mom_find(tu, D, e)] / r[0]; };
  auto Um = [&](int q, int i) { return su[(size_t)q * RU + 1 + i]; };
  const int pp = p + 1 < np ? p + 1 : (periodic ? 0 : -1);
  const int pm = p > 0 ? p - 1 : (periodic ? np - 1 : -1);
  const double T = tmet[p], J = jm[p], al = J * T * T;
  auto d1 = [&](auto f, double fwl, double fwh) {
    const double fp = pp >= 0 ? f(pp) : 2.0 * fwh - f(p);
    const double fm = pm >= 0 ? f(pm) : 2.0 * fwl - f(p);
    return T * 0.5 * (fp - fm);
  };
  auto d2 = [&](auto f) {
    const double fP = f(p);
    double s = 0.0;
    if (pp >= 0) s += 0.5 * (al + jm[pp] * tmet[pp] * tmet[pp]) * (f(pp) - fP);
    else s += 2.0 * al * (0.0 - fP);
    if (pm >= 0) s += 0.5 * (al + jm[pm] * tmet[pm] * tmet[pm]) * (f(pm) - fP);
    else s += 2.0 * al * (0.0 - fP);
    return s / J;
  };
  double dU[D];
#pragma unroll
  for (int i = 0; i < D; ++i) dU[i] = d1([&](int q) { return Um(q, i); }, wl[i], wh[i]);
  int q = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j, ++q) {
      int eia[D] = {}, eja[D] = {}, eij[D] = {}, eija[D] = {};
      eia[i]++; eia[a]++;
      eja[j]++; eja[a]++;
      eij[i]++; eij[j]++;
      eija[i]++; eija[j]++; eija[a]++;
      const double P_ = -(Mu(p, eia) * dU[j] + Mu(p, eja) * dU[i]);
      double eps = 0.0;
      for (int k = 0; k < D; ++k) {
        const double* r = sg + ((size_t)k * np + p) * RG;
        eps += r[1 + D + mom_find(tg, D, eij)] / r[0];
      }
      eps *= 2.0;
      const double Tt = -d1([&](int qq) { return Mu(qq, eija); }, 0.0, 0.0);
      const double Dd = d2([&](int qq) { return Mu(qq, eij); });
      int xij[2 * D] = {}, xji[2 * D] = {};
      xij[i]++; xij[D + j]++;
      xji[j]++; xji[D + i]++;
      const double* r = sup + (size_t)p * RP;
      const double Pi = -(r[1 + 2 * D + mom_find(tp, 2 * D, xij)] + r[1 + 2 * D + mom_find(tp, 2 * D, xji)]) / r[0];
      out[((size_t)0 * np + p) * NP + q] = P_;
      out[((size_t)1 * np + p) * NP + q] = eps;
      out[((size_t)2 * np + p) * NP + q] = Tt;
      out[((size_t)3 * np + p) * NP + q] = Dd;
      out[((size_t)4 * np + p) * NP + q] = Pi;
    }
}

// Plane metric: T_aa and J of the first cell of each plane (computed from J T and 1/J).
template <typename R, bool DIAG, int D>
__global__ void __launch_bounds__(kWG)
k_plane_metric(int np, int a, int nx, int ny, const R* __restrict__ JT, const R* __restrict__ invJ, int N,
               double* __restrict__ tmet, double* __restrict__ jm) {
  const int p = blockIdx.x * kWG + threadIdx.x;
  if (p >= np) return;
  const int P = a == 0 ? p : (a == 1 ? nx * p : nx * ny * p);
  const double iJ = (double)invJ[P];
  const double jt = DIAG ? (double)JT[(size_t)a * N + P] : (double)JT[(size_t)(a * D + a) * N + P];
  tmet[p] = jt * iJ;
  jm[p] = 1.0 / iJ;
}

// ------------------------------------------------------------------ host

static int mom_check(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

int moments_layout(const piso_ctx* c, int axis, int m, int order, int* n_planes, int* samples, int* n_alpha) {
  if (c->nblocks != 1 || axis < 0 || axis >= c->dim) return PISO_E_ARG;
  if (m < 1 || order < 2 || order > 4) return PISO_E_ARG;
  if (!(m == 2 || m == 3 || m == 4 || m == 6)) return PISO_E_ARG;
  MomTab t;
  if (momtab(m, order, t) < 0) return PISO_E_ARG;
  const int* tb = &c->h_tab[0];
  const int nn[3] = {tb[1], tb[2], tb[3]};
  *n_planes = nn[axis];
  *samples = c->N / nn[axis];
  *n_alpha = t.n;
  return PISO_OK;
}

template <typename R>
int moments_accumulate(piso_ctx* c, hipStream_t s, const R* x, int m, int order, int axis, double* state) {
  int np, ms, na;
  if (moments_layout(c, axis, m, order, &np, &ms, &na))
    return fail(c, PISO_E_ARG, "moments: single-block grid, axis < d, m in {2, 3, 4, 6}, order 2..4 with at most 32 "
                               "multi-indices");
  MomTab t;
  momtab(m, order, t);
  const int nx = c->h_tab[1], ny = c->h_tab[2];
  switch (m) {
    case 2: k_mom_acc<R, 2><<<np, kWG, 0, s>>>(x, c->N, nx, ny, ms, axis, t, state); break;
    case 3: k_mom_acc<R, 3><<<np, kWG, 0, s>>>(x, c->N, nx, ny, ms, axis, t, state); break;
    case 4: k_mom_acc<R, 4><<<np, kWG, 0, s>>>(x, c->N, nx, ny, ms, axis, t, state); break;
    default: k_mom_acc<R, 6><<<np, kWG, 0, s>>>(x, c->N, nx, ny, ms, axis, t, state); break;
  }
  return mom_check(c, "k_mom_acc");
}

int moments_finalize(piso_ctx* c, hipStream_t s, int m, int order, int axis, const double* state, double* mean,
                     double* mom) {
  int np, ms, na;
  if (moments_layout(c, axis, m, order, &np, &ms, &na)) return fail(c, PISO_E_ARG, "moments: bad layout");
  k_mom_final<<<grid_cells(np), kWG, 0, s>>>(np, m, na, state, mean, mom);
  return mom_check(c, "k_mom_final");
}

template <typename R>
int moments_backward(piso_ctx* c, hipStream_t s, const R* x, int m, int order, int axis, const double* state,
                     const double* mbar, const double* obar, R* dx) {
  int np, ms, na;
  if (moments_layout(c, axis, m, order, &np, &ms, &na)) return fail(c, PISO_E_ARG, "moments: bad layout");
  MomTab t;
  momtab(m, order, t);
  const int nx = c->h_tab[1], ny = c->h_tab[2], G = grid_cells(c->N);
  switch (m) {
    case 2: k_mom_bwd<R, 2><<<G, kWG, 0, s>>>(x, c->N, nx, ny, axis, t, state, mbar, obar, dx); break;
    case 3: k_mom_bwd<R, 3><<<G, kWG, 0, s>>>(x, c->N, nx, ny, axis, t, state, mbar, obar, dx); break;
    case 4: k_mom_bwd<R, 4><<<G, kWG, 0, s>>>(x, c->N, nx, ny, axis, t, state, mbar, obar, dx); break;
    default: k_mom_bwd<R, 6><<<G, kWG, 0, s>>>(x, c->N, nx, ny, axis, t, state, mbar, obar, dx); break;
  }
  return mom_check(c, "k_mom_bwd");
}

template <typename R>
int field_gradient(piso_ctx* c, hipStream_t s, const R* phi, int nc, const R* phib, R* out) {
  if (nc < 1) return fail(c, PISO_E_ARG, "field gradient: no components");
  const int G = grid_cells(c->N);
  const R* JT = (const R*)c->JT;
  const R* iJ = (const R*)c->invJ;
  if (c->dim == 2) {
    if (c->diagT) k_field_grad<R, 2, true><<<G, kWG, 0, s>>>(c->grid, JT, iJ, phi, nc, phib, out);
    else k_field_grad<R, 2, false><<<G, kWG, 0, s>>>(c->grid, JT, iJ, phi, nc, phib, out);
  } else {
    if (c->diagT) k_field_grad<R, 3, true><<<G, kWG, 0, s>>>(c->grid, JT, iJ, phi, nc, phib, out);
    else k_field_grad<R, 3, false><<<G, kWG, 0, s>>>(c->grid, JT, iJ, phi, nc, phib, out);
  }
  return mom_check(c, "k_field_grad");
}

template <typename R>
int budget(piso_ctx* c, hipStream_t s, int axis, int order_u, const double* su, const double* sg, const double* sup,
           const double* wall_mean, double* out) {
  const int D = c->dim;
  int np, ms, nu, ng, npp;
  if (moments_layout(c, axis, D, order_u, &np, &ms, &nu) || order_u < 3 ||
      moments_layout(c, axis, D, 2, &np, &ms, &ng) || moments_layout(c, axis, 2 * D, 2, &np, &ms, &npp))
    return fail(c, PISO_E_ARG, "budget: single-block grid, axis < d, u moments of order >= 3");
  MomTab tu, tg, tp;
  momtab(D, order_u, tu);
  momtab(D, 2, tg);
  momtab(2 * D, 2, tp);
  const int* tb = &c->h_tab[0];
  const int periodic = (tb[kTabWrap] >> (2 * axis)) & 1;
  const int nx = tb[1], ny = tb[2];
  double* tmet = c->plane_work;
  double* jm = c->plane_work + np;
  const int G = grid_cells(np);
  const R* JT = (const R*)c->JT;
  const R* iJ = (const R*)c->invJ;
  if (c->diagT) {
    if (D == 2) k_plane_metric<R, true, 2><<<G, kWG, 0, s>>>(np, axis, nx, ny, JT, iJ, c->N, tmet, jm);
    else k_plane_metric<R, true, 3><<<G, kWG, 0, s>>>(np, axis, nx, ny, JT, iJ, c->N, tmet, jm);
  } else {
    if (D == 2) k_plane_metric<R, false, 2><<<G, kWG, 0, s>>>(np, axis, nx, ny, JT, iJ, c->N, tmet, jm);
    else k_plane_metric<R, false, 3><<<G, kWG, 0, s>>>(np, axis, nx, ny, JT, iJ, c->N, tmet, jm);
  }
  const double* w = wall_mean;
  const double wl[3] = {w[0], w[1], D == 3 ? w[2] : 0.0};
  const double wh[3] = {w[D], w[D + 1], D == 3 ? w[D + 2] : 0.0};
  if (D == 2)
    k_budget<2><<<G, kWG, 0, s>>>(np, axis, periodic, tu, tg, tp, su, sg, sup, tmet, jm, wl[0], wl[1], wl[2], wh[0],
                                  wh[1], wh[2], out);
  else
    k_budget<3><<<G, kWG, 0, s>>>(np, axis, periodic, tu, tg, tp, su, sg, sup, tmet, jm, wl[0], wl[1], wl[2], wh[0],
                                  wh[1], wh[2], out);
  return mom_check(c, "k_budget");
}

template int moments_accumulate<float>(piso_ctx*, hipStream_t, const float*, int, int, int, double*);
template int moments_accumulate<double>(piso_ctx*, hipStream_t, const double*, int, int, int, double*);
template int moments_backward<float>(piso_ctx*, hipStream_t, const float*, int, int, int, const double*,
                                     const double*, const double*, float*);
template int moments_backward<double>(piso_ctx*, hipStream_t, const double*, int, int, int, const double*,
                                      const double*, const double*, double*);
template int field_gradient<float>(piso_ctx*, hipStream_t, const float*, int, const float*, float*);
template int field_gradient<double>(piso_ctx*, hipStream_t, const double*, int, const double*, double*);
template int budget<float>(piso_ctx*, hipStream_t, int, int, const double*, const double*, const double*,
                           const double*, double*);
template int budget<double>(piso_ctx*, hipStream_t, int, int, const double*, const double*, const double*,
                            const double*, double*);

}  // namespace piso
