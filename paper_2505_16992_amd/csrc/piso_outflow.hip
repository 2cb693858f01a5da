// Advective outflow boundary (App. A.4, eq. advOut) and its adjoint.
//
// Between two steps the Dirichlet values of the faces marked as outflow are advanced
// implicitly and upwind from their boundary cell P over the half cell between the
// face and the cell centre,
//     u_b* = (u_b + c u_P) / (1 + c),   c = 2 dt |T_j(P) . u_m|,
// with u_m the prescribed characteristic velocity and j the face's axis.  The printed
// update factor has the opposite sign inside the fraction, which would make the
// scheme anti-upwind for an outflow; this is the stable (upwind) reading.  The
// outflow values are then scaled by s = -Q_rest / Q_out so that the net flux
// sum_b N_b J_P T_j(P) . u_b through the boundary vanishes (Q_out: the updated outflow
// faces, Q_rest: every other Dirichlet face; s = 1 when Q_out = 0).  The face flux is
// the one the step adds to the pressure right-hand side.
#include <algorithm>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "piso_impl.h"

namespace piso {

// J T_j(P) . v for a face of axis j: the metrics are [d*d][N] (or [d][N] when T is
// diagonal) and hold J T_ji.
template <typename R, int D, bool DIAG>
__device__ __forceinline__ R jt_dot(const R* __restrict__ JT, int N, int P, int j, const R (&v)[D]) {
  if (DIAG) return JT[(size_t)j * N + P] * v[j];
  R s = R(0);
#pragma unroll
  for (int i = 0; i < D; ++i) s += JT[(size_t)(j * D + i) * N + P] * v[i];
  return s;
}

// (J T_j)_f . v with the metrics of Dirichlet face f (bjt [d][NB]): the face's flux of v,
// the Dirichlet flux the step adds to the pressure right-hand side.
template <typename R, int D>
__device__ __forceinline__ R bjt_dot(const R* __restrict__ bjt, int NB, int f, const R (&v)[D]) {
  R s = R(0);
#pragma unroll
  for (int i = 0; i < D; ++i) s += bjt[(size_t)i * NB + f] * v[i];
  return s;
}

// Per face: the advanced value u_b* (outflow faces) or u_b (others), written to
// star, and the partial sums of Q_out and Q_rest.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_out_star(int N, int NB, const int* __restrict__ bcell, const int* __restrict__ bside,
           const R* __restrict__ JT, const R* __restrict__ bjt, const R* __restrict__ invJ, const R* __restrict__ u,
           const R* __restrict__ ub, const int* __restrict__ outflow, OutflowUm um, R dt2,
           R* __restrict__ star, double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (int f = blockIdx.x * kWG + threadIdx.x; f < NB; f += gridDim.x * kWG) {
    const int P = bcell[f], j = bside[f] >> 1;
    const R sgn = (bside[f] & 1) ? R(1) : R(-1);
    R v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = ub[(size_t)i * NB + f];
    const bool out = outflow[f] != 0;
    if (out) {
      R m[D];
#pragma unroll
      for (int i = 0; i < D; ++i) m[i] = (R)um.v[i];
      const R cf = dt2 * std::fabs(jt_dot<R, D, DIAG>(JT, N, P, j, m) * invJ[P]);
#pragma unroll
      for (int i = 0; i < D; ++i) v[i] = (v[i] + cf * u[(size_t)i * N + P]) / (R(1) + cf);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) star[(size_t)i * NB + f] = v[i];
    const double q = (double)(sgn * bjt_dot<R, D>(bjt, NB, f, v));
    if (out) acc[0] += q;
    else acc[1] += q;
  }
  write_partials<2>(acc, partials);
}

// out = s * star on outflow faces, star elsewhere; s from the re-reduced partials.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_out_scale(int NB, const int* __restrict__ outflow, const R* __restrict__ star,
            const double* __restrict__ partials, int Gp, R* __restrict__ out) {
  double t[2];
  reduce_partials<2>(partials, Gp, t);
  const R s = t[0] != 0.0 ? (R)(-t[1] / t[0]) : R(1);
  for (int f = blockIdx.x * kWG + threadIdx.x; f < NB; f += gridDim.x * kWG) {
    const bool o = outflow[f] != 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const R v = star[(size_t)i * NB + f];
      out[(size_t)i * NB + f] = o ? s * v : v;
    }
  }
}

// Adjoint, first pass: star again, with the partial sums of Q_out, Q_rest and
// sigma = sum over outflow faces of gbar . star.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_outb_1(int N, int NB, const int* __restrict__ bcell, const int* __restrict__ bside,
         const R* __restrict__ JT, const R* __restrict__ bjt, const R* __restrict__ invJ, const R* __restrict__ u,
         const R* __restrict__ ub, const int* __restrict__ outflow, OutflowUm um, R dt2,
         const R* __restrict__ gbar, R* __restrict__ star, double* __restrict__ partials) {
  double acc[3] = {0.0, 0.0, 0.0};
  for (int f = blockIdx.x * kWG + threadIdx.x; f < NB; f += gridDim.x * kWG) {
    const int P = bcell[f], j = bside[f] >> 1;
    const R sgn = (bside[f] & 1) ? R(1) : R(-1);
    R v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = ub[(size_t)i * NB + f];
    const bool out = outflow[f] != 0;
    if (out) {
      R m[D];
#pragma unroll
      for (int i = 0; i < D; ++i) m[i] = (R)um.v[i];
      const R cf = dt2 * std::fabs(jt_dot<R, D, DIAG>(JT, N, P, j, m) * invJ[P]);
#pragma unroll
      for (int i = 0; i < D; ++i) v[i] = (v[i] + cf * u[(size_t)i * N + P]) / (R(1) + cf);
      double sg = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) sg += (double)gbar[(size_t)i * NB + f] * (double)v[i];
      acc[2] += sg;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) star[(size_t)i * NB + f] = v[i];
    const double q = (double)(sgn * bjt_dot<R, D>(bjt, NB, f, v));
    if (out) acc[0] += q;
    else acc[1] += q;
  }
  write_partials<3>(acc, partials);
}

// Adjoint, second pass: star_bar per face, du_b = star_bar / (1 + c) on outflow faces
// (star_bar elsewhere), and the cell contribution c / (1 + c) star_bar of each outflow
// face into contrib [d][NB] (0 elsewhere).
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_outb_2(int N, int NB, const int* __restrict__ bcell, const int* __restrict__ bside,
         const R* __restrict__ JT, const R* __restrict__ bjt, const R* __restrict__ invJ,
         const int* __restrict__ outflow, OutflowUm um,
         R dt2, const R* __restrict__ gbar, const double* __restrict__ partials, int Gp, R* __restrict__ dub,
         R* __restrict__ contrib) {
  double t[3];
  reduce_partials<3>(partials, Gp, t);
  const double q_out = t[0], q_rest = t[1], sigma = t[2];
  const bool scaled = q_out != 0.0;
  const R s = scaled ? (R)(-q_rest / q_out) : R(1);
  const R k_out = scaled ? (R)(sigma * (double)s / q_out) : R(0);   // sigma s / Q_out
  const R k_rest = scaled ? (R)(sigma / q_out) : R(0);              // sigma / Q_out
  for (int f = blockIdx.x * kWG + threadIdx.x; f < NB; f += gridDim.x * kWG) {
    const int P = bcell[f], j = bside[f] >> 1;
    const R sgn = (bside[f] & 1) ? R(1) : R(-1);
    const bool out = outflow[f] != 0;
    R cf = R(0);
    if (out) {
      R m[D];
#pragma unroll
      for (int i = 0; i < D; ++i) m[i] = (R)um.v[i];
      cf = dt2 * std::fabs(jt_dot<R, D, DIAG>(JT, N, P, j, m) * invJ[P]);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      // flux weight w_i = N_b (J T_ji)_f of the face
      const R w = sgn * bjt[(size_t)i * NB + f];
      const R g = gbar[(size_t)i * NB + f];
      const R sb = out ? s * g - k_out * w : g - k_rest * w;
      dub[(size_t)i * NB + f] = out ? sb / (R(1) + cf) : sb;
      contrib[(size_t)i * NB + f] = out ? sb * cf / (R(1) + cf) : R(0);
    }
  }
}

// du_n[i][P] += sum of the contributions of P's boundary faces, in face order.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_outb_3(int N, int NB, int nbc, const int* __restrict__ bc_cell, const int* __restrict__ bc_ptr,
         const int* __restrict__ bc_face, const R* __restrict__ contrib, R* __restrict__ du) {
  const int q = blockIdx.x * kWG + threadIdx.x;
  if (q >= nbc) return;
  const int P = bc_cell[q];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    R s = R(0);
    for (int t = bc_ptr[q]; t < bc_ptr[q + 1]; ++t) s += contrib[(size_t)i * NB + bc_face[t]];
    du[(size_t)i * N + P] += s;
  }
}

// ------------------------------------------------------------------ host

int bface_cells(piso_ctx* c, std::vector<int>& bcell, std::vector<int>& bside) {
  const int NB = c->NB, B = c->nblocks, D = c->dim;
  bcell.assign(NB, -1);
  bside.assign(NB, -1);
  for (int b = 0; b < B; ++b) {
    const int* t = &c->h_tab[(size_t)b * kTabStride];
    const int n[3] = {t[1], t[2], t[3]};
    for (int side = 0; side < 2 * D; ++side) {
      const int a = side / 2, sd = side % 2;
      int tn[2] = {1, 1}, q = 0;
      for (int x = 0; x < D; ++x)
        if (x != a) tn[q++] = n[x];
      for (int t1 = 0; t1 < tn[1]; ++t1)
        for (int t0 = 0; t0 < tn[0]; ++t0) {
          const int v = c->h_fmap[(size_t)t[4 + side] + t0 + tn[0] * t1];
          if (v >= 0) continue;
          const int f = -1 - v;
          int pos[3] = {0, 0, 0}, r = 0;
          for (int x = 0; x < 3; ++x) {
            if (x == a) pos[x] = sd ? n[x] - 1 : 0;
            else pos[x] = r++ == 0 ? t0 : t1;
          }
          if (f < 0 || f >= NB) return fail(c, PISO_E_TOPOLOGY, "boundary face index out of range");
          bcell[f] = t[0] + pos[0] + n[0] * (pos[1] + n[1] * pos[2]);
          bside[f] = side;
        }
    }
  }
  for (int f = 0; f < NB; ++f)
    if (bcell[f] < 0) return fail(c, PISO_E_TOPOLOGY, "Dirichlet face without a cell");
  return PISO_OK;
}

int outflow_build(piso_ctx* c) {
  const int NB = c->NB, D = c->dim;
  if (NB == 0) return PISO_OK;
  std::vector<int> bcell, bside;
  if (int rc = bface_cells(c, bcell, bside)) return rc;
  // boundary cells and their faces, cells ascending, faces ascending
  std::vector<std::pair<int, int>> cf(NB);
  for (int f = 0; f < NB; ++f) cf[f] = {bcell[f], f};
  std::sort(cf.begin(), cf.end());
  std::vector<int> cells, ptr{0}, faces;
  for (int q = 0; q < NB; ++q) {
    if (q == 0 || cf[q].first != cf[q - 1].first) {
      if (q) ptr.push_back(q);
      cells.push_back(cf[q].first);
    }
    faces.push_back(cf[q].second);
  }
  ptr.push_back(NB);
  c->out_nbc = (int)cells.size();
  if (int rc = upload(c, (void**)&c->out_bcell, bcell)) return rc;
  if (int rc = upload(c, (void**)&c->out_bside, bside)) return rc;
  if (int rc = upload(c, (void**)&c->out_bc_cell, cells)) return rc;
  if (int rc = upload(c, (void**)&c->out_bc_ptr, ptr)) return rc;
  if (int rc = upload(c, (void**)&c->out_bc_face, faces)) return rc;
  if (int rc = dev_alloc(c, &c->out_star, (size_t)D * NB * c->esz)) return rc;
  if (int rc = dev_alloc(c, &c->out_contrib, (size_t)D * NB * c->esz)) return rc;
  return PISO_OK;
}

static int out_check(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

#define PISO_OUT_DISPATCH(ctx, CALL)                                                   \
  do {                                                                                 \
    if ((ctx)->dim == 2) {                                                             \
      if ((ctx)->diagT) { constexpr int D = 2; constexpr bool DG = true; CALL; }       \
      else { constexpr int D = 2; constexpr bool DG = false; CALL; }                   \
    } else {                                                                           \
      if ((ctx)->diagT) { constexpr int D = 3; constexpr bool DG = true; CALL; }       \
      else { constexpr int D = 3; constexpr bool DG = false; CALL; }                   \
    }                                                                                  \
  } while (0)

template <typename R>
int outflow_update(piso_ctx* c, hipStream_t s, const R* u, const R* ub, const int* outflow, OutflowUm um,
                   double dt, R* ub_out) {
  const int NB = c->NB, N = c->N;
  if (NB == 0) return PISO_OK;
  const int G = std::min(grid_cells(NB), 256);
  double* pS = part(c, kPartS);
  R* star = (R*)c->out_star;
  const R dt2 = (R)(2.0 * dt);
  PISO_OUT_DISPATCH(c, (k_out_star<R, D, DG><<<G, kWG, 0, s>>>(N, NB, c->out_bcell, c->out_bside,
                                                                (const R*)c->JT, (const R*)c->bjt,
                                                                (const R*)c->invJ, u, ub,
                                                                outflow, um, dt2, star, pS)));
  if (c->dim == 2) k_out_scale<R, 2><<<G, kWG, 0, s>>>(NB, outflow, star, pS, G, ub_out);
  else k_out_scale<R, 3><<<G, kWG, 0, s>>>(NB, outflow, star, pS, G, ub_out);
  return out_check(c, "outflow update");
}

template <typename R>
int outflow_update_bwd(piso_ctx* c, hipStream_t s, const R* u, const R* ub, const int* outflow, OutflowUm um,
                       double dt, const R* gbar, R* du, R* dub) {
  const int NB = c->NB, N = c->N;
  if (NB == 0) return PISO_OK;
  const int G = std::min(grid_cells(NB), 256);
  double* pS = part(c, kPartS);
  R* star = (R*)c->out_star;
  R* contrib = (R*)c->out_contrib;
  const R dt2 = (R)(2.0 * dt);
  PISO_OUT_DISPATCH(c, (k_outb_1<R, D, DG><<<G, kWG, 0, s>>>(N, NB, c->out_bcell, c->out_bside, (const R*)c->JT,
                                                              (const R*)c->bjt, (const R*)c->invJ, u, ub, outflow,
                                                              um, dt2, gbar,
                                                              star, pS)));
  PISO_OUT_DISPATCH(c, (k_outb_2<R, D, DG><<<G, kWG, 0, s>>>(N, NB, c->out_bcell, c->out_bside, (const R*)c->JT,
                                                              (const R*)c->bjt, (const R*)c->invJ, outflow, um,
                                                              dt2, gbar, pS, G,
                                                              dub, contrib)));
  if (du) {
    const int Gc = grid_cells(c->out_nbc);
    if (c->dim == 2)
      k_outb_3<R, 2><<<Gc, kWG, 0, s>>>(N, NB, c->out_nbc, c->out_bc_cell, c->out_bc_ptr, c->out_bc_face, contrib,
                                         du);
    else
      k_outb_3<R, 3><<<Gc, kWG, 0, s>>>(N, NB, c->out_nbc, c->out_bc_cell, c->out_bc_ptr, c->out_bc_face, contrib,
                                         du);
  }
  return out_check(c, "outflow update adjoint");
}

template int outflow_update<float>(piso_ctx*, hipStream_t, const float*, const float*, const int*, OutflowUm,
                                   double, float*);
template int outflow_update<double>(piso_ctx*, hipStream_t, const double*, const double*, const int*, OutflowUm,
                                    double, double*);
template int outflow_update_bwd<float>(piso_ctx*, hipStream_t, const float*, const float*, const int*, OutflowUm,
                                       double, const float*, float*, float*);
template int outflow_update_bwd<double>(piso_ctx*, hipStream_t, const double*, const double*, const int*,
                                        OutflowUm, double, const double*, double*, double*);

}  // namespace piso
