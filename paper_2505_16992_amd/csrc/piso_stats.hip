// Online turbulence statistics over homogeneous planes (Sec. 2.5 of arXiv 2505.16992)
// and their gradient.
//
// The planes normal to an axis of a single-block grid each collect the d velocity
// components of their cells at every accumulated step.  The state of a plane is the
// record [n, mu_0 .. mu_{d-1}, C_00, C_01, .., C_{d-1,d-1}] (doubles; C over i <= j):
// sample count, mean and central comoment sums.  One work-group owns one plane: it
// takes the batch mean of the new step in a first pass over the plane, the batch
// central sums in a second, and merges them with the pairwise update for central
// comoments (delta = mu_B - mu_A, mu += delta m / n, C += C_B + delta_i delta_j n_A m / n),
// so no raw second moment is formed.  Deterministic: fixed-order work-group sums.
//
// Gradient of the final mean and covariance (C / n) with respect to an accumulated
// sample u(P) of plane p: d mu_i / d u_k = delta_ik / n and
// d cov_ij / d u_k = (delta_ik (u_j - mu_j) + delta_jk (u_i - mu_i)) / n.
#include <string>

#include "piso_impl.h"

namespace piso {

namespace {

__device__ __forceinline__ int plane_cell(int axis, int p, int t, int nx, int ny) {
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

}  // namespace

template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_stats_acc(const R* __restrict__ u, int N, int nx, int ny, int m, int axis, double* __restrict__ state) {
  constexpr int NP = D * (D + 1) / 2;
  constexpr int REC = 1 + D + NP;
  const int p = blockIdx.x;
  double s1[D];
#pragma unroll
  for (int i = 0; i < D; ++i) s1[i] = 0.0;
  for (int t = threadIdx.x; t < m; t += kWG) {
    const int P = plane_cell(axis, p, t, nx, ny);
#pragma unroll
    for (int i = 0; i < D; ++i) s1[i] += (double)u[(size_t)i * N + P];
  }
  wg_sum_all<D>(s1);
  double mu_b[D];
#pragma unroll
  for (int i = 0; i < D; ++i) mu_b[i] = s1[i] / m;
  double s2[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) s2[q] = 0.0;
  for (int t = threadIdx.x; t < m; t += kWG) {
    const int P = plane_cell(axis, p, t, nx, ny);
    double dv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) dv[i] = (double)u[(size_t)i * N + P] - mu_b[i];
    int q = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j) s2[q++] += dv[i] * dv[j];
  }
  __shared__ double lds[NP * kWaves];
  wg_sum<NP>(s2, lds);
  if (threadIdx.x == 0) {
    double* rec = state + (size_t)p * REC;
    const double nA = rec[0], n = nA + m;
    double delta[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      delta[i] = mu_b[i] - rec[1 + i];
      rec[1 + i] += delta[i] * ((double)m / n);
    }
    const double f = nA * (double)m / n;
    int q = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j, ++q) rec[1 + D + q] += s2[q] + delta[i] * delta[j] * f;
    rec[0] = n;
  }
}

template <int D>
__global__ void __launch_bounds__(kWG)
k_stats_final(int n_planes, const double* __restrict__ state, double* __restrict__ mean, double* __restrict__ cov) {
  constexpr int NP = D * (D + 1) / 2;
  constexpr int REC = 1 + D + NP;
  const int p = blockIdx.x * kWG + threadIdx.x;
  if (p >= n_planes) return;
  const double* rec = state + (size_t)p * REC;
  const double n = rec[0];
#pragma unroll
  for (int i = 0; i < D; ++i) mean[p * D + i] = rec[1 + i];
#pragma unroll
  for (int q = 0; q < NP; ++q) cov[p * NP + q] = n > 0 ? rec[1 + D + q] / n : 0.0;
}

template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_stats_bwd(const R* __restrict__ u, int N, int nx, int ny, int axis, const double* __restrict__ state,
            const double* __restrict__ mbar, const double* __restrict__ cbar, R* __restrict__ du) {
  constexpr int NP = D * (D + 1) / 2;
  constexpr int REC = 1 + D + NP;
  const int P = cell_of_thread(N);
  if (P < 0) return;
  const int i0 = P % nx, j0 = (P / nx) % ny, k0 = P / (nx * ny);
  const int p = axis == 0 ? i0 : (axis == 1 ? j0 : k0);
  const double* rec = state + (size_t)p * REC;
  const double inv_n = 1.0 / rec[0];
  double dv[D], g[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    dv[i] = (double)u[(size_t)i * N + P] - rec[1 + i];
    g[i] = mbar[p * D + i];
  }
  int q = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j, ++q) {
      const double cb = cbar[p * NP + q];
      g[i] += cb * dv[j];
      g[j] += cb * dv[i];
    }
#pragma unroll
  for (int i = 0; i < D; ++i) du[(size_t)i * N + P] += (R)(g[i] * inv_n);
}

// ------------------------------------------------------------------ host

static int stats_check(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

int stats_planes(const piso_ctx* c, int axis, int* n_planes, int* m) {
  if (c->nblocks != 1 || axis < 0 || axis >= c->dim) return PISO_E_ARG;
  const int* t = &c->h_tab[0];
  const int n[3] = {t[1], t[2], t[3]};
  *n_planes = n[axis];
  *m = c->N / n[axis];
  return PISO_OK;
}

template <typename R>
int stats_accumulate(piso_ctx* c, hipStream_t s, const R* u, int axis, double* state) {
  int np, m;
  if (stats_planes(c, axis, &np, &m)) return fail(c, PISO_E_ARG, "statistics: single-block grid and axis < d");
  const int nx = c->h_tab[1], ny = c->h_tab[2];
  if (c->dim == 2) k_stats_acc<R, 2><<<np, kWG, 0, s>>>(u, c->N, nx, ny, m, axis, state);
  else k_stats_acc<R, 3><<<np, kWG, 0, s>>>(u, c->N, nx, ny, m, axis, state);
  return stats_check(c, "k_stats_acc");
}

int stats_finalize(piso_ctx* c, hipStream_t s, int axis, const double* state, double* mean, double* cov) {
  int np, m;
  if (stats_planes(c, axis, &np, &m)) return fail(c, PISO_E_ARG, "statistics: single-block grid and axis < d");
  if (c->dim == 2) k_stats_final<2><<<grid_cells(np), kWG, 0, s>>>(np, state, mean, cov);
  else k_stats_final<3><<<grid_cells(np), kWG, 0, s>>>(np, state, mean, cov);
  return stats_check(c, "k_stats_final");
}

template <typename R>
int stats_backward(piso_ctx* c, hipStream_t s, const R* u, int axis, const double* state, const double* mbar,
                   const double* cbar, R* du) {
  int np, m;
  if (stats_planes(c, axis, &np, &m)) return fail(c, PISO_E_ARG, "statistics: single-block grid and axis < d");
  const int nx = c->h_tab[1], ny = c->h_tab[2];
  if (c->dim == 2) k_stats_bwd<R, 2><<<grid_cells(c->N), kWG, 0, s>>>(u, c->N, nx, ny, axis, state, mbar, cbar, du);
  else k_stats_bwd<R, 3><<<grid_cells(c->N), kWG, 0, s>>>(u, c->N, nx, ny, axis, state, mbar, cbar, du);
  return stats_check(c, "k_stats_bwd");
}

template int stats_accumulate<float>(piso_ctx*, hipStream_t, const float*, int, double*);
template int stats_accumulate<double>(piso_ctx*, hipStream_t, const double*, int, double*);
template int stats_backward<float>(piso_ctx*, hipStream_t, const float*, int, const double*, const double*,
                                   const double*, float*);
template int stats_backward<double>(piso_ctx*, hipStream_t, const double*, int, const double*, const double*,
                                    const double*, double*);

}  // namespace piso
