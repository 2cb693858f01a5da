// Krylov solvers of the PISO step (arXiv 2505.16992, App. A.6: CG for the pressure,
// BiCGStab for advection-diffusion; the adjoint reuses them with the transposed
// operator, Sec. 2.3).  Matrix-free stencil operators over the multi-block grid; all
// dot products accumulate in double with deterministic two-stage reductions; the
// scalars alpha, beta, omega stay on the device and the host only reads the
// convergence state every check_every iterations.
#include <algorithm>
#include <cmath>

#include "piso_impl.h"

namespace piso {

// ------------------------------------------------------------------------ PCG
// Solves M x = b with M = -P (symmetric positive semi-definite: (M x)_P =
// sum_f P_f (x_P - x_F)), Jacobi preconditioner Dinv.  b = sign * (bsrc - mean).

template <typename R, int D>
__device__ __forceinline__ void faces_of(const Grid& g, int P, int (&Fp)[D], int (&Fm)[D]) {
  const Cell c = locate(g, P);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    Fp[j] = neighbour(g, c, P, j, 1);
    Fm[j] = neighbour(g, c, P, j, 0);
  }
}

template <typename R, typename BT, int D>
__global__ void __launch_bounds__(kWG)
k_cg_init(Grid g, const R* __restrict__ Pf, const R* __restrict__ Dinv, const BT* __restrict__ bsrc,
          const double* __restrict__ mean, double sign, const R* __restrict__ x, R* __restrict__ r,
          R* __restrict__ dold, CgState* st, double* partials, double tol2) {
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  const double mu = mean ? mean[0] : 0.0;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<R, D>(g, P, Fp, Fm);
    const R b = (R)(sign * ((double)bsrc[P] - mu));
    const R xP = x[P];
    R Mx = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (Fp[j] >= 0) Mx += Pf[(size_t)j * N + P] * (xP - x[Fp[j]]);
      if (Fm[j] >= 0) Mx += Pf[(size_t)j * N + Fm[j]] * (xP - x[Fm[j]]);
    }
    const R rv = b - Mx;
    r[P] = rv;
    dold[P] = R(0);
    acc[0] += (double)rv * (double)(Dinv[P] * rv);
    acc[1] += (double)rv * (double)rv;
    acc[2] += (double)b * (double)b;
  }
  double t[3];
  if (grid_sum<3>(acc, partials, &st->counter, t) && threadIdx.x == 0) {
    st->rz = t[0];
    st->rr = t[1];
    st->bb = t[2];
    st->beta = 0.0;
    st->alpha = 0.0;
    st->tol2 = tol2;
    st->iters = 0;
    st->zero_rhs = (t[2] == 0.0) ? 1 : 0;
    if (!std::isfinite(t[0]) || !std::isfinite(t[1]) || !std::isfinite(t[2])) {
      st->status = PISO_E_NAN;
      st->done = 1;
    } else {
      st->status = 0;
      st->done = (t[2] == 0.0 || t[1] <= tol2 * t[2]) ? 1 : 0;
    }
  }
}

// d_new = Dinv r + beta d_old (evaluated at the cell and its neighbours), q = M d_new,
// partial d_new . q; the last work-group sets alpha = (r.z) / (d.q).
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_cg_spmv(Grid g, const R* __restrict__ Pf, const R* __restrict__ Dinv, const R* __restrict__ r,
          const R* __restrict__ dold, R* __restrict__ dnew, R* __restrict__ q, CgState* st,
          double* partials) {
  if (st->done) return;
  const int N = g.N;
  const R beta = (R)st->beta;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[1] = {0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<R, D>(g, P, Fp, Fm);
    const R dP = Dinv[P] * r[P] + beta * dold[P];
    R Md = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (Fp[j] >= 0) {
        const int F = Fp[j];
        Md += Pf[(size_t)j * N + P] * (dP - (Dinv[F] * r[F] + beta * dold[F]));
      }
      if (Fm[j] >= 0) {
        const int F = Fm[j];
        Md += Pf[(size_t)j * N + F] * (dP - (Dinv[F] * r[F] + beta * dold[F]));
      }
    }
    dnew[P] = dP;
    q[P] = Md;
    acc[0] += (double)dP * (double)Md;
  }
  double t[1];
  if (grid_sum<1>(acc, partials, &st->counter, t) && threadIdx.x == 0) {
    st->dq = t[0];
    if (t[0] > 0.0 && std::isfinite(t[0])) {
      st->alpha = st->rz / t[0];
    } else {
      st->alpha = 0.0;
      st->status = std::isfinite(t[0]) ? PISO_BREAKDOWN : PISO_E_NAN;
      st->done = 1;
    }
  }
}

// x += alpha d; r -= alpha q; partial r.z and r.r; the last work-group sets beta and
// the convergence flag.
template <typename R>
__global__ void __launch_bounds__(kWG)
k_cg_update(int N, const R* __restrict__ Dinv, R* __restrict__ x, R* __restrict__ r,
            const R* __restrict__ dnew, const R* __restrict__ q, CgState* st, double* partials) {
  if (st->done) return;
  const R alpha = (R)st->alpha;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2] = {0.0, 0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    x[P] += alpha * dnew[P];
    const R rn = r[P] - alpha * q[P];
    r[P] = rn;
    acc[0] += (double)rn * (double)(Dinv[P] * rn);
    acc[1] += (double)rn * (double)rn;
  }
  double t[2];
  if (grid_sum<2>(acc, partials, &st->counter, t) && threadIdx.x == 0) {
    st->beta = t[0] / st->rz;
    st->rz = t[0];
    st->rr = t[1];
    st->iters += 1;
    if (!std::isfinite(t[1])) {
      st->status = PISO_E_NAN;
      st->done = 1;
    } else if (t[1] <= st->tol2 * st->bb) {
      st->done = 1;
    }
  }
}

// MIXED form: r64 = b64 - M x64 in double with b64 = -(rhs64 - mean) and the float face
// coefficients, r32 = (float) r64; partial r.r and b.b.
template <int D>
__global__ void __launch_bounds__(kWG)
k_mix_resid(Grid g, const float* __restrict__ Pf, const double* __restrict__ rhs64,
            const double* __restrict__ mean, const double* __restrict__ x64, float* __restrict__ r32,
            double* partials, unsigned* counter, double* out /* [2]: rr, bb */) {
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  const double mu = mean[0];
  double acc[2] = {0.0, 0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<float, D>(g, P, Fp, Fm);
    const double b = -(rhs64[P] - mu);
    const double xP = x64[P];
    double Mx = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (Fp[j] >= 0) Mx += (double)Pf[(size_t)j * N + P] * (xP - x64[Fp[j]]);
      if (Fm[j] >= 0) Mx += (double)Pf[(size_t)j * N + Fm[j]] * (xP - x64[Fm[j]]);
    }
    const double rv = b - Mx;
    r32[P] = (float)rv;
    acc[0] += rv * rv;
    acc[1] += b * b;
  }
  double t[2];
  if (grid_sum<2>(acc, partials, counter, t) && threadIdx.x == 0) {
    out[0] = t[0];
    out[1] = t[1];
  }
}

__global__ void __launch_bounds__(kWG) k_mix_add(int N, double* __restrict__ x64, const float* __restrict__ e) {
  const int P = cell_of_thread(N);
  if (P < 0) return;
  x64[P] += (double)e[P];
}

// ------------------------------------------------------------------- BiCGStab
// d right-hand sides sharing every coefficient read; right Jacobi preconditioning
// K = diag(A).  TRANS applies C^T instead of C (adjoint solve).

template <typename R, int D, bool TRANS>
__device__ __forceinline__ R coef_p(const R* __restrict__ C, int j, int P, int Fp, int N) {
  return TRANS ? C[(size_t)(D + j) * N + P] : C[(size_t)j * N + P];
  (void)Fp;
}
template <typename R, int D, bool TRANS>
__device__ __forceinline__ R coef_m(const R* __restrict__ C, int j, int Fm, int N) {
  return TRANS ? C[(size_t)j * N + Fm] : C[(size_t)(D + j) * N + Fm];
}

template <typename R, int D, bool TRANS>
__global__ void __launch_bounds__(kWG)
k_bi_init(Grid g, const R* __restrict__ A, const R* __restrict__ C, const R* __restrict__ b,
          const R* __restrict__ x, R* __restrict__ r, R* __restrict__ rh, R* __restrict__ p0,
          R* __restrict__ v0, BiState* st, double* partials, double tol2) {
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<R, D>(g, P, Fp, Fm);
    R cp[D], cm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      cp[j] = Fp[j] >= 0 ? coef_p<R, D, TRANS>(C, j, P, Fp[j], N) : R(0);
      cm[j] = Fm[j] >= 0 ? coef_m<R, D, TRANS>(C, j, Fm[j], N) : R(0);
    }
    const R AP = A[P];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const R* xc = x + (size_t)c * N;
      R Cx = AP * xc[P];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (Fp[j] >= 0) Cx += cp[j] * xc[Fp[j]];
        if (Fm[j] >= 0) Cx += cm[j] * xc[Fm[j]];
      }
      const R bv = b[(size_t)c * N + P];
      const R rv = bv - Cx;
      r[(size_t)c * N + P] = rv;
      rh[(size_t)c * N + P] = rv;
      p0[(size_t)c * N + P] = R(0);
      v0[(size_t)c * N + P] = R(0);
      acc[c] += (double)rv * (double)rv;
      acc[D + c] += (double)bv * (double)bv;
    }
  }
  double t[2 * D];
  if (grid_sum<2 * D>(acc, partials, &st->counter, t) && threadIdx.x == 0) {
    int all = 1;
    st->tol2 = tol2;
    for (int c = 0; c < D; ++c) {
      st->rho[c] = t[c];
      st->rr[c] = t[c];
      st->bb[c] = t[D + c];
      st->rho_prev[c] = 1.0;
      st->alpha[c] = 1.0;
      st->omega[c] = 1.0;
      st->iters[c] = 0;
      if (!std::isfinite(t[c]) || !std::isfinite(t[D + c])) {
        st->status[c] = PISO_E_NAN;
        st->done[c] = 1;
      } else {
        st->status[c] = 0;
        st->done[c] = (t[D + c] == 0.0 || t[c] <= tol2 * t[D + c]) ? 1 : 0;
      }
      all &= st->done[c];
    }
    for (int c = D; c < 3; ++c) st->done[c] = 1;
    st->all_done = all;
  }
}

// p = r + beta (p_old - omega v_old); v = C K^-1 p; partial rh . v; alpha = rho / (rh . v).
template <typename R, int D, bool TRANS>
__global__ void __launch_bounds__(kWG)
k_bi_1(Grid g, const R* __restrict__ A, const R* __restrict__ C, const R* __restrict__ r,
       const R* __restrict__ rh, const R* __restrict__ p_old, const R* __restrict__ v_old,
       R* __restrict__ p_new, R* __restrict__ v_new, BiState* st, double* partials) {
  if (st->all_done) return;
  const int N = g.N;
  R beta[D], omega[D];
  bool act[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    beta[c] = (R)((st->rho[c] / st->rho_prev[c]) * (st->alpha[c] / st->omega[c]));
    omega[c] = (R)st->omega[c];
  }
  int beg, end;
  chunk_range(N, beg, end);
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<R, D>(g, P, Fp, Fm);
    R cp[D], cm[D], iAp[D], iAm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      cp[j] = Fp[j] >= 0 ? coef_p<R, D, TRANS>(C, j, P, Fp[j], N) : R(0);
      cm[j] = Fm[j] >= 0 ? coef_m<R, D, TRANS>(C, j, Fm[j], N) : R(0);
      iAp[j] = Fp[j] >= 0 ? R(1) / A[Fp[j]] : R(0);
      iAm[j] = Fm[j] >= 0 ? R(1) / A[Fm[j]] : R(0);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (!act[c]) continue;
      const size_t o = (size_t)c * N;
      auto pn = [&](int X) { return r[o + X] + beta[c] * (p_old[o + X] - omega[c] * v_old[o + X]); };
      const R pP = pn(P);
      R v = pP;   // A_P * (p_P / A_P)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (Fp[j] >= 0) v += cp[j] * pn(Fp[j]) * iAp[j];
        if (Fm[j] >= 0) v += cm[j] * pn(Fm[j]) * iAm[j];
      }
      p_new[o + P] = pP;
      v_new[o + P] = v;
      acc[c] += (double)rh[o + P] * (double)v;
    }
  }
  double t[D];
  if (grid_sum<D>(acc, partials, &st->counter, t) && threadIdx.x == 0) {
    for (int c = 0; c < D; ++c) {
      if (st->done[c]) continue;
      if (t[c] != 0.0 && std::isfinite(t[c])) {
        st->alpha[c] = st->rho[c] / t[c];
      } else {
        st->alpha[c] = 0.0;
        st->status[c] = std::isfinite(t[c]) ? PISO_BREAKDOWN : PISO_E_NAN;
        st->done[c] = 1;
      }
    }
    int all = 1;
    for (int c = 0; c < D; ++c) all &= st->done[c];
    st->all_done = all;
  }
}

// s = r - alpha v; t = C K^-1 s; partial t.s and t.t; omega = (t.s)/(t.t).
template <typename R, int D, bool TRANS>
__global__ void __launch_bounds__(kWG)
k_bi_2(Grid g, const R* __restrict__ A, const R* __restrict__ C, const R* __restrict__ r,
       const R* __restrict__ v, R* __restrict__ s, R* __restrict__ t, BiState* st, double* partials) {
  if (st->all_done) return;
  const int N = g.N;
  R alpha[D];
  bool act[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    alpha[c] = (R)st->alpha[c];
  }
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<R, D>(g, P, Fp, Fm);
    R cp[D], cm[D], iAp[D], iAm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      cp[j] = Fp[j] >= 0 ? coef_p<R, D, TRANS>(C, j, P, Fp[j], N) : R(0);
      cm[j] = Fm[j] >= 0 ? coef_m<R, D, TRANS>(C, j, Fm[j], N) : R(0);
      iAp[j] = Fp[j] >= 0 ? R(1) / A[Fp[j]] : R(0);
      iAm[j] = Fm[j] >= 0 ? R(1) / A[Fm[j]] : R(0);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (!act[c]) continue;
      const size_t o = (size_t)c * N;
      auto sv = [&](int X) { return r[o + X] - alpha[c] * v[o + X]; };
      const R sP = sv(P);
      R tv = sP;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (Fp[j] >= 0) tv += cp[j] * sv(Fp[j]) * iAp[j];
        if (Fm[j] >= 0) tv += cm[j] * sv(Fm[j]) * iAm[j];
      }
      s[o + P] = sP;
      t[o + P] = tv;
      acc[c] += (double)tv * (double)sP;
      acc[D + c] += (double)tv * (double)tv;
    }
  }
  double tt[2 * D];
  if (grid_sum<2 * D>(acc, partials, &st->counter, tt) && threadIdx.x == 0) {
    for (int c = 0; c < D; ++c) {
      if (st->done[c]) continue;
      st->omega[c] = tt[D + c] > 0.0 ? tt[c] / tt[D + c] : 0.0;
    }
  }
}

// x += K^-1 (alpha p + omega s); r = s - omega t; partial rh.r and r.r; convergence.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_bi_3(int N, const R* __restrict__ A, R* __restrict__ x, R* __restrict__ r, const R* __restrict__ rh,
       const R* __restrict__ p, const R* __restrict__ s, const R* __restrict__ t, BiState* st,
       double* partials) {
  if (st->all_done) return;
  R alpha[D], omega[D];
  bool act[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    alpha[c] = (R)st->alpha[c];
    omega[c] = (R)st->omega[c];
  }
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    const R iA = R(1) / A[P];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (!act[c]) continue;
      const size_t o = (size_t)c * N + P;
      const R sv = s[o];
      x[o] += (alpha[c] * p[o] + omega[c] * sv) * iA;
      const R rn = sv - omega[c] * t[o];
      r[o] = rn;
      acc[c] += (double)rh[o] * (double)rn;
      acc[D + c] += (double)rn * (double)rn;
    }
  }
  double tt[2 * D];
  if (grid_sum<2 * D>(acc, partials, &st->counter, tt) && threadIdx.x == 0) {
    int all = 1;
    for (int c = 0; c < D; ++c) {
      if (!st->done[c]) {
        st->rho_prev[c] = st->rho[c];
        st->rho[c] = tt[c];
        st->rr[c] = tt[D + c];
        st->iters[c] += 1;
        if (!std::isfinite(tt[D + c])) {
          st->status[c] = PISO_E_NAN;
          st->done[c] = 1;
        } else if (tt[D + c] <= st->tol2 * st->bb[c]) {
          st->done[c] = 1;
        } else if (tt[c] == 0.0 || st->omega[c] == 0.0) {
          st->status[c] = PISO_BREAKDOWN;
          st->done[c] = 1;
        }
      }
      all &= st->done[c];
    }
    st->all_done = all;
  }
}

// ------------------------------------------------------------------ host drivers

static int check(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

// Timed launch: when timing is enabled, brackets the launch with an event pair.
struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
};

static EvPair timing_begin(piso_ctx* c, hipStream_t s) {
  EvPair p;
  Timing& t = c->timing;
  if (!t.enabled) return p;
  if (t.used + 2 > t.ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return p;
      t.ev.push_back(e);
    }
  }
  p.a = t.ev[t.used++];
  p.b = t.ev[t.used++];
  (void)hipEventRecord(p.a, s);
  return p;
}

static void timing_end(piso_ctx* c, hipStream_t s, const EvPair& p) {
  if (p.b) (void)hipEventRecord(p.b, s);
}

// After a stream sync: fold the elapsed times of the recorded pairs (spmv, update
// alternate in the pool) into the totals.
static void timing_collect(piso_ctx* c, const std::vector<int>& kinds) {
  Timing& t = c->timing;
  if (!t.enabled) return;
  size_t k = 0;
  for (size_t q = 0; q + 1 < t.used && k < kinds.size(); q += 2, ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev[q], t.ev[q + 1]) != hipSuccess) continue;
    if (kinds[k] == 0) {
      t.spmv_ms += ms;
      t.spmv_calls += 1;
    } else {
      t.update_ms += ms;
      t.update_calls += 1;
    }
  }
  t.used = 0;
}

template <typename R, typename BT>
static int pcg_run(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const BT* b,
                   const double* mean, double sign, R* x, double rtol, int max_iter, int check_every,
                   int* iters_out, double* rel_out, int* status_out) {
  const int N = c->N, G = grid_red(N);
  R* r = (R*)c->k_r;
  R* q = (R*)c->k_q;
  R* d[2] = {(R*)c->k_d0, (R*)c->k_d1};
  CgState* st = c->cg;
  const double tol2 = rtol * rtol;
  if (c->dim == 2)
    k_cg_init<R, BT, 2><<<G, kWG, 0, s>>>(c->grid, Pf, Dinv, b, mean, sign, x, r, d[0], st, c->partials, tol2);
  else
    k_cg_init<R, BT, 3><<<G, kWG, 0, s>>>(c->grid, Pf, Dinv, b, mean, sign, x, r, d[0], st, c->partials, tol2);
  if (int rc = check(c, "k_cg_init")) return rc;
  PISO_HIP(c, hipMemcpyAsync(c->h_cg, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
  PISO_HIP(c, hipStreamSynchronize(s));
  if (c->h_cg->zero_rhs) {
    PISO_HIP(c, hipMemsetAsync(x, 0, sizeof(R) * (size_t)N, s));
  }
  int it = 0;
  if (check_every < 1) check_every = 8;
  std::vector<int> kinds;
  while (!c->h_cg->done && it < max_iter) {
    const int n = std::min(check_every, max_iter - it);
    kinds.clear();
    for (int k = 0; k < n; ++k, ++it) {
      R* dold = d[it & 1];
      R* dnew = d[(it + 1) & 1];
      EvPair e1 = timing_begin(c, s);
      if (c->dim == 2)
        k_cg_spmv<R, 2><<<G, kWG, 0, s>>>(c->grid, Pf, Dinv, r, dold, dnew, q, st, c->partials);
      else
        k_cg_spmv<R, 3><<<G, kWG, 0, s>>>(c->grid, Pf, Dinv, r, dold, dnew, q, st, c->partials);
      timing_end(c, s, e1);
      if (e1.a) kinds.push_back(0);
      EvPair e2 = timing_begin(c, s);
      k_cg_update<R><<<G, kWG, 0, s>>>(N, Dinv, x, r, dnew, q, st, c->partials);
      timing_end(c, s, e2);
      if (e2.a) kinds.push_back(1);
    }
    if (int rc = check(c, "k_cg iteration")) return rc;
    PISO_HIP(c, hipMemcpyAsync(c->h_cg, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    PISO_HIP(c, hipStreamSynchronize(s));
    timing_collect(c, kinds);
  }
  const CgState& h = *c->h_cg;
  *iters_out += h.iters;
  *rel_out = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
  if (h.status < 0) *status_out = h.status;
  else if (h.status > 0) *status_out = std::max(*status_out, h.status);
  else if (!h.done) *status_out = std::max(*status_out, (int)PISO_NOT_CONVERGED);
  return PISO_OK;
}

template <typename R, typename BT>
int pressure_solve(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const BT* rhs,
                   const double* mean, R* x, const piso_solve_opts* o, piso_solve_info* info) {
  int iters = 0, status = 0;
  double rel = 0.0;
  int rc = pcg_run<R, BT>(c, s, Pf, Dinv, rhs, mean, -1.0, x, o->rtol, o->max_iter, o->check_every,
                          &iters, &rel, &status);
  if (rc) return rc;
  // zero-mean gauge
  rc = launch_sum<R, double>(c, s, x, c->N, 1.0 / c->N, c->mean + 1);
  if (rc) return rc;
  rc = launch_sub_mean<R, R>(c, s, x, c->mean + 1, x, c->N);
  if (rc) return rc;
  if (info) {
    info->status = status;
    info->iters = iters;
    info->refinements = 0;
    info->rel_residual = rel;
  }
  return status < 0 ? status : PISO_OK;
}

int pressure_solve_mixed(piso_ctx* c, hipStream_t s, const float* Pf, const float* Dinv,
                         const double* rhs64, const double* mean, double* x64, const piso_solve_opts* o,
                         piso_solve_info* info) {
  const int N = c->N, G = grid_red(N);
  float* r32 = (float*)c->m_r32;
  float* e32 = (float*)c->m_e32;
  int iters = 0, status = 0, sweeps = 0;
  double rel = 0.0;
  for (;;) {
    if (c->dim == 2)
      k_mix_resid<2><<<G, kWG, 0, s>>>(c->grid, Pf, rhs64, mean, x64, r32, c->partials, c->counter, c->mean + 2);
    else
      k_mix_resid<3><<<G, kWG, 0, s>>>(c->grid, Pf, rhs64, mean, x64, r32, c->partials, c->counter, c->mean + 2);
    if (int rc = check(c, "k_mix_resid")) return rc;
    PISO_HIP(c, hipMemcpyAsync(c->h_scal, c->mean + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    PISO_HIP(c, hipStreamSynchronize(s));
    const double rr = c->h_scal[0], bb = c->h_scal[1];
    if (!std::isfinite(rr)) {
      status = PISO_E_NAN;
      break;
    }
    rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    if (bb == 0.0) {
      PISO_HIP(c, hipMemsetAsync(x64, 0, sizeof(double) * (size_t)N, s));
      rel = 0.0;
      break;
    }
    if (rel <= o->rtol) break;
    if (sweeps >= o->max_refine) {
      status = PISO_NOT_CONVERGED;
      break;
    }
    PISO_HIP(c, hipMemsetAsync(e32, 0, sizeof(float) * (size_t)N, s));
    int st_in = 0;
    double rel_in = 0.0;
    int rc = pcg_run<float, float>(c, s, Pf, Dinv, r32, nullptr, 1.0, e32, o->inner_rtol, o->max_iter,
                                   o->check_every, &iters, &rel_in, &st_in);
    if (rc) return rc;
    if (st_in < 0) {
      status = st_in;
      break;
    }
    k_mix_add<<<grid_cells(N), kWG, 0, s>>>(N, x64, e32);
    if (int rc2 = check(c, "k_mix_add")) return rc2;
    ++sweeps;
  }
  int rc = launch_sum<double, double>(c, s, x64, N, 1.0 / N, c->mean + 1);
  if (rc) return rc;
  rc = launch_sub_mean<double, double>(c, s, x64, c->mean + 1, x64, N);
  if (rc) return rc;
  if (info) {
    info->status = status;
    info->iters = iters;
    info->refinements = sweeps;
    info->rel_residual = rel;
  }
  return status < 0 ? status : PISO_OK;
}

template <typename R>
int velocity_solve(piso_ctx* c, hipStream_t s, bool trans, const R* A, const R* C, const R* b, R* x,
                   const piso_solve_opts* o, piso_solve_info* info) {
  const int N = c->N, G = grid_red(N), D = c->dim;
  R* r = (R*)c->b_r;
  R* rh = (R*)c->b_rh;
  R* pb[2] = {(R*)c->b_p0, (R*)c->b_p1};
  R* vb[2] = {(R*)c->b_v0, (R*)c->b_v1};
  R* sb = (R*)c->b_s;
  R* tb = (R*)c->b_t;
  BiState* st = c->bi;
  const double tol2 = o->rtol * o->rtol;
#define BI_LAUNCH(KERNEL, ...)                                                    \
  do {                                                                            \
    if (D == 2) {                                                                 \
      if (trans) KERNEL<R, 2, true><<<G, kWG, 0, s>>>(__VA_ARGS__);               \
      else KERNEL<R, 2, false><<<G, kWG, 0, s>>>(__VA_ARGS__);                    \
    } else {                                                                      \
      if (trans) KERNEL<R, 3, true><<<G, kWG, 0, s>>>(__VA_ARGS__);               \
      else KERNEL<R, 3, false><<<G, kWG, 0, s>>>(__VA_ARGS__);                    \
    }                                                                             \
  } while (0)
  BI_LAUNCH(k_bi_init, c->grid, A, C, b, x, r, rh, pb[0], vb[0], st, c->partials, tol2);
  if (int rc = check(c, "k_bi_init")) return rc;
  PISO_HIP(c, hipMemcpyAsync(c->h_bi, st, sizeof(BiState), hipMemcpyDeviceToHost, s));
  PISO_HIP(c, hipStreamSynchronize(s));
  for (int q = 0; q < D; ++q)
    if (c->h_bi->bb[q] == 0.0) PISO_HIP(c, hipMemsetAsync(x + (size_t)q * N, 0, sizeof(R) * (size_t)N, s));
  int it = 0;
  const int ce = o->check_every < 1 ? 4 : o->check_every;
  while (!c->h_bi->all_done && it < o->max_iter) {
    const int n = std::min(ce, o->max_iter - it);
    for (int k = 0; k < n; ++k, ++it) {
      R* po = pb[it & 1];
      R* pn = pb[(it + 1) & 1];
      R* vo = vb[it & 1];
      R* vn = vb[(it + 1) & 1];
      BI_LAUNCH(k_bi_1, c->grid, A, C, r, rh, po, vo, pn, vn, st, c->partials);
      BI_LAUNCH(k_bi_2, c->grid, A, C, r, vn, sb, tb, st, c->partials);
      if (D == 2) k_bi_3<R, 2><<<G, kWG, 0, s>>>(N, A, x, r, rh, pn, sb, tb, st, c->partials);
      else k_bi_3<R, 3><<<G, kWG, 0, s>>>(N, A, x, r, rh, pn, sb, tb, st, c->partials);
    }
    if (int rc = check(c, "k_bi iteration")) return rc;
    PISO_HIP(c, hipMemcpyAsync(c->h_bi, st, sizeof(BiState), hipMemcpyDeviceToHost, s));
    PISO_HIP(c, hipStreamSynchronize(s));
  }
#undef BI_LAUNCH
  const BiState& h = *c->h_bi;
  int status = 0, iters = 0;
  double rel = 0.0;
  for (int q = 0; q < D; ++q) {
    iters = std::max(iters, h.iters[q]);
    if (h.bb[q] > 0) rel = std::max(rel, std::sqrt(h.rr[q] / h.bb[q]));
    if (h.status[q] < 0) status = h.status[q];
    else if (status >= 0) status = std::max(status, h.status[q]);
    if (!h.done[q] && status >= 0) status = std::max(status, (int)PISO_NOT_CONVERGED);
  }
  if (info) {
    info->status = status;
    info->iters = iters;
    info->refinements = 0;
    info->rel_residual = rel;
  }
  return status < 0 ? status : PISO_OK;
}

template int pressure_solve<float, float>(piso_ctx*, hipStream_t, const float*, const float*, const float*,
                                          const double*, float*, const piso_solve_opts*, piso_solve_info*);
template int pressure_solve<double, double>(piso_ctx*, hipStream_t, const double*, const double*,
                                            const double*, const double*, double*, const piso_solve_opts*,
                                            piso_solve_info*);
template int velocity_solve<float>(piso_ctx*, hipStream_t, bool, const float*, const float*, const float*,
                                   float*, const piso_solve_opts*, piso_solve_info*);
template int velocity_solve<double>(piso_ctx*, hipStream_t, bool, const double*, const double*,
                                    const double*, double*, const piso_solve_opts*, piso_solve_info*);

}  // namespace piso
