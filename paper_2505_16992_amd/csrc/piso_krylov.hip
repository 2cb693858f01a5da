// Krylov solvers of the PISO step (arXiv 2505.16992, App. A.6: CG for the pressure,
// BiCGStab for advection-diffusion; the adjoint reuses them with the transposed
// operator, Sec. 2.3).  Matrix-free stencil operators over the multi-block grid.
//
// Reductions: each kernel writes per-work-group partial sums; the next kernel of the
// iteration re-reduces them (same order in every work-group: deterministic and
// identical everywhere) and derives its scalar (alpha, beta, omega) on the device.  No
// device-scope fences or atomics are used.  The host reads the convergence state only
// every check_every iterations, through a one-work-group check kernel.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "piso_impl.h"
#include "piso_quad.h"

namespace piso {

template <int D>
__device__ __forceinline__ void faces_of(const Grid& g, int P, int (&Fp)[D], int (&Fm)[D]) {
  const Cell c = locate(g, P);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    Fp[j] = neighbour(g, c, P, j, 1);
    Fm[j] = neighbour(g, c, P, j, 0);
  }
}

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

// ------------------------------------------------------------------------ PCG
// Solves M x = b with M = -P (symmetric positive semi-definite, (M x)_P =
// sum_f P_f (x_P - x_F)) and the Jacobi preconditioner Dinv; b = sign (bsrc - mean).
// Iteration k: spmv_k reduces the r.z, r.r partials of update_{k-1} (or of init),
// tests convergence, forms beta_k = rz_k / rz_{k-1}, d_k = z + beta_k d_{k-1},
// q = M d_k and the d.q partials; update_k forms alpha_k = rz_k / (d.q), updates x, r
// and writes the new r.z, r.r partials.

template <typename R, typename BT, int D>
__global__ void __launch_bounds__(kWG)
k_cg_init(Grid g, const R* __restrict__ Pf, const R* __restrict__ Dinv, const BT* __restrict__ bsrc,
          const double* __restrict__ mean, double sign, const R* __restrict__ x, R* __restrict__ r,
          R* __restrict__ dold, double* __restrict__ partB) {
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  const double mu = mean ? mean[0] : 0.0;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    const R b = (R)(sign * ((double)bsrc[P] - mu));
    const R xP = x[P];
    R Mx = R(0);
    // a face without a neighbour cell reads the cell itself: its term is exactly zero
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int Fpj = Fp[j] >= 0 ? Fp[j] : P, Fmj = Fm[j] >= 0 ? Fm[j] : P;
      Mx += Pf[(size_t)j * N + P] * (xP - x[Fpj]);
      Mx += Pf[(size_t)j * N + Fmj] * (xP - x[Fmj]);
    }
    const R rv = b - Mx;
    r[P] = rv;
    dold[P] = R(0);
    acc[0] += (double)rv * (double)(Dinv[P] * rv);
    acc[1] += (double)rv * (double)rv;
    acc[2] += (double)b * (double)b;
  }
  write_partials<3>(acc, partB);
}

// One work-group: publishes the state after init (first: also resets the iteration
// index and sets its limit) or after a chunk of iterations (convergence of the latest
// residual).
__global__ void __launch_bounds__(kWG)
k_cg_check(const double* __restrict__ partB, int G, int first, int max_k, double tol2, CgState* st) {
  double t[3];
  reduce_partials<3>(partB, G, t);
  if (threadIdx.x != 0) return;
  if (first) {
    st->bb = t[2];
    st->tol2 = tol2;
    st->status = 0;
    st->done = 0;
    st->iters = 0;
    st->k = 0;
    st->max_k = max_k;
    st->zero_rhs = t[2] == 0.0 ? 1 : 0;
  }
  if (st->done) return;
  st->rr = t[1];
  st->iters = st->k;
  if (!std::isfinite(t[0]) || !std::isfinite(t[1]) || !std::isfinite(st->bb)) {
    st->status = PISO_E_NAN;
    st->done = 1;
  } else if (st->bb == 0.0 || t[1] <= st->tol2 * st->bb) {
    st->done = 1;
  }
}

template <typename R, int D, bool ZOP = false>
__global__ void __launch_bounds__(kWG)
k_cg_spmv(Grid g, const R* __restrict__ Pf, const R* __restrict__ Dinv, const R* __restrict__ r,
          const R* __restrict__ dold, R* __restrict__ dnew, R* __restrict__ q, CgState* st,
          const double* __restrict__ partB, double* __restrict__ partA, int Gp, int par) {
  // the state and the partials are loaded together, before the first wait
  const int done = st->done, kd = st->k, max_k = st->max_k;
  const double tol2bb = st->tol2 * st->bb, rz_old = st->rz[par ^ 1];
  double t[2];
  reduce_partials<2>(partB, Gp, t);
  if (done) return;
  const double rz = t[0], rr = t[1];
  if (!std::isfinite(rz) || !std::isfinite(rr) || rr <= tol2bb || kd >= max_k) {
    if (lead()) {
      st->rr = rr;
      st->iters = kd;
      if (!std::isfinite(rz) || !std::isfinite(rr)) st->status = PISO_E_NAN;
      else if (!(rr <= tol2bb)) st->status = PISO_NOT_CONVERGED;
      st->done = 1;
    }
    return;
  }
  const R beta = kd == 0 ? R(0) : (R)(rz / rz_old);
  if (lead()) {
    st->rz[par] = rz;
    st->rr = rr;
  }
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[1] = {0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    auto op = [&](int Q) { return (ZOP ? r[Q] : Dinv[Q] * r[Q]) + beta * dold[Q]; };
    const R dP = op(P);
    R Md = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (Fp[j] >= 0) Md += Pf[(size_t)j * N + P] * (dP - op(Fp[j]));
      if (Fm[j] >= 0) Md += Pf[(size_t)j * N + Fm[j]] * (dP - op(Fm[j]));
    }
    dnew[P] = dP;
    q[P] = Md;
    acc[0] += (double)dP * (double)Md;
  }
  write_partials<1>(acc, partA);
}

// Jacobi PCG update: x += alpha d, r -= alpha q, partials of r.D^-1 r and r.r (the
// multigrid PCG fuses its update with the fine-grid restriction instead).
template <typename R>
__global__ void __launch_bounds__(kWG)
k_cg_update(int N, const R* __restrict__ Dinv, R* __restrict__ x, R* __restrict__ r,
            const R* __restrict__ dnew, const R* __restrict__ q, CgState* st, const double* __restrict__ partA,
            double* __restrict__ partB, int Gp, int par) {
  const int done = st->done;
  const double rzp = st->rz[par];
  double t[1];
  reduce_partials<1>(partA, Gp, t);
  if (done) return;
  const double dq = t[0];
  if (!(dq > 0.0) || !std::isfinite(dq)) {
    if (lead()) {
      st->status = std::isfinite(dq) ? PISO_BREAKDOWN : PISO_E_NAN;
      st->iters = st->k;
      st->done = 1;
    }
    return;
  }
  const R alpha = (R)(rzp / dq);
  if (lead()) st->k = st->k + 1;   // no other work-group reads the index in this kernel
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
  write_partials<2>(acc, partB);
}


template <typename R, int D, bool ZOP = false>
__global__ void __launch_bounds__(kWG)
k_cg_spmv_q(Grid g, const R* __restrict__ Pf, const R* __restrict__ Dinv, const R* __restrict__ r,
            const R* __restrict__ dold, R* __restrict__ dnew, R* __restrict__ q, CgState* st,
            const double* __restrict__ partB, double* __restrict__ partA, int Gp, int par) {
  // the state, the partials and this thread's first quad of the operand streams are
  // loaded together, before the first wait (at one trip per thread the prologue's
  // latency then overlaps the main loads)
  const int done = st->done, kd = st->k, max_k = st->max_k;
  const double tol2bb = st->tol2 * st->bb, rz_old = st->rz[par ^ 1];
  int qd0, end, stride;
  quad_sweep(g.N >> 2, qd0, end, stride);
  const int P00 = qd0 < end ? qd0 << 2 : 0;   // unconditional (clamped) loads: no branch to wait at
  const Q4<R> b0 = ldq(r, P00), c0 = ldq(dold, P00);
  Q4<R> a0{};
  if constexpr (!ZOP) a0 = ldq(Dinv, P00);
  double t[2];
  reduce_partials<2>(partB, Gp, t);
  if (done) return;
  const double rz = t[0], rr = t[1];
  if (!std::isfinite(rz) || !std::isfinite(rr) || rr <= tol2bb || kd >= max_k) {
    if (lead()) {
      st->rr = rr;
      st->iters = kd;
      if (!std::isfinite(rz) || !std::isfinite(rr)) st->status = PISO_E_NAN;
      else if (!(rr <= tol2bb)) st->status = PISO_NOT_CONVERGED;
      st->done = 1;
    }
    return;
  }
  const R beta = kd == 0 ? R(0) : (R)(rz / rz_old);
  if (lead()) {
    st->rz[par] = rz;
    st->rr = rr;
  }
  auto dq = [&](int P, int, int) {
    const Q4<R> b = ldq(r, P), c = ldq(dold, P);
    Q4<R> o;
    if constexpr (ZOP) {
#pragma unroll
      for (int e = 0; e < 4; ++e) o.v[e] = b.v[e] + beta * c.v[e];
    } else {
      const Q4<R> a = ldq(Dinv, P);
#pragma unroll
      for (int e = 0; e < 4; ++e) o.v[e] = a.v[e] * b.v[e] + beta * c.v[e];
    }
    return o;
  };
  auto d1 = [&](int P, bool, int, int, int) { return (ZOP ? r[P] : Dinv[P] * r[P]) + beta * dold[P]; };
  double acc[1] = {0.0};
  for (int qd = qd0; qd < end; qd += stride) {
    const int P0 = qd << 2;
    const Cell c = locate(g, P0);
    Q4<R> dP;
    if (qd == qd0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) dP.v[e] = (ZOP ? b0.v[e] : a0.v[e] * b0.v[e]) + beta * c0.v[e];
    } else {
      dP = dq(P0, c.j, c.k);
    }
    const Q4<R> M = quad_stencil<R, D>(g, c, P0, Pf, dP, dq, d1);
    stq(dnew, P0, dP);
    stq(q, P0, M);
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[0] += (double)dP.v[e] * (double)M.v[e];
  }
  write_partials<1>(acc, partA);
}

template <typename R>
__global__ void __launch_bounds__(kWG)
k_cg_update_q(int N, const R* __restrict__ Dinv, R* __restrict__ x, R* __restrict__ r,
              const R* __restrict__ dnew, const R* __restrict__ q, CgState* st, const double* __restrict__ partA,
              double* __restrict__ partB, int Gp, int par) {
  const int done = st->done;
  const double rzp = st->rz[par];
  double t[1];
  reduce_partials<1>(partA, Gp, t);
  if (done) return;
  const double dq = t[0];
  if (!(dq > 0.0) || !std::isfinite(dq)) {
    if (lead()) {
      st->status = std::isfinite(dq) ? PISO_BREAKDOWN : PISO_E_NAN;
      st->iters = st->k;
      st->done = 1;
    }
    return;
  }
  const R alpha = (R)(rzp / dq);
  if (lead()) st->k = st->k + 1;   // no other work-group reads the index in this kernel
  int beg, end;
  quad_range(N >> 2, beg, end);
  double acc[2] = {0.0, 0.0};
  for (int qd = beg + (int)threadIdx.x; qd < end; qd += kWG) {
    const int P = qd << 2;
    Q4<R> xv = ldq(x, P), rv = ldq(r, P);
    const Q4<R> dv = ldq(dnew, P), qv = ldq(q, P);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xv.v[e] += alpha * dv.v[e];
      rv.v[e] -= alpha * qv.v[e];
    }
    const Q4<R> Dv = ldq(Dinv, P);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[0] += (double)rv.v[e] * (double)(Dv.v[e] * rv.v[e]);
      acc[1] += (double)rv.v[e] * (double)rv.v[e];
    }
    stq(x, P, xv);
    stq(r, P, rv);
  }
  write_partials<2>(acc, partB);
}

// MIXED form: r64 = b64 - M x64 in double, with b64 = -(rhs64 - mean) and the double
// face coefficients (the operator of the step), r32 = (float) r64; partials of r.r and
// b.b.
template <int D>
__global__ void __launch_bounds__(kWG)
k_mix_resid(Grid g, const double* __restrict__ Pf, const double* __restrict__ rhs64,
            const double* __restrict__ mean, const double* __restrict__ x64, float* __restrict__ r32,
            double* __restrict__ partials) {
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  const double mu = mean ? mean[0] : 0.0;
  double acc[2] = {0.0, 0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    const double b = -(rhs64[P] - mu);
    const double xP = x64[P];
    double Mx = 0.0;
    // a face without a neighbour cell reads the cell itself: its term is exactly zero
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int Fpj = Fp[j] >= 0 ? Fp[j] : P, Fmj = Fm[j] >= 0 ? Fm[j] : P;
      Mx += Pf[(size_t)j * N + P] * (xP - x64[Fpj]);
      Mx += Pf[(size_t)j * N + Fmj] * (xP - x64[Fmj]);
    }
    const double rv = b - Mx;
    r32[P] = (float)rv;
    acc[0] += rv * rv;
    acc[1] += b * b;
  }
  write_partials<2>(acc, partials);
}

template <int NV>
__global__ void __launch_bounds__(kWG)
k_finalize(const double* __restrict__ partials, int G, double* __restrict__ out) {
  double t[NV];
  reduce_partials<NV>(partials, G, t);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = t[q];
  }
}

// x = 0 when the right-hand side is zero (set by k_cg_check), decided on the device so
// that the host need not wait for the initial state.
template <typename R>
__global__ void __launch_bounds__(kWG) k_cg_zero_if(int N, const CgState* st, R* __restrict__ x) {
  if (!st->zero_rhs) return;
  const int P = cell_of_thread(N);
  if (P >= 0) x[P] = R(0);
}

// x_c = 0 for the components whose right-hand side is zero (set by k_bi_check).
template <typename R, int D>
__global__ void __launch_bounds__(kWG) k_bi_zero_if(int N, const BiState* st, R* __restrict__ x) {
  const int P = cell_of_thread(N);
  if (P < 0) return;
#pragma unroll
  for (int c = 0; c < D; ++c)
    if (st->bb[c] == 0.0) x[(size_t)c * N + P] = R(0);
}

// x64 += e over n elements (the refinement update of both MIXED solves).
__global__ void __launch_bounds__(kWG) k_mix_add(int n, double* __restrict__ x64, const float* __restrict__ e) {
  const int P = cell_of_thread(n);
  if (P < 0) return;
  x64[P] += (double)e[P];
}

// ------------------------------------------------------------------- BiCGStab
// d right-hand sides sharing every coefficient read; right Jacobi preconditioning
// K = diag(A); TRANS applies C^T instead of C (adjoint solve).  Iteration k:
//   bi1_k: rho_k = rh.r, convergence, beta_k, p = r + beta (p - omega v), v = C K^-1 p
//   bi2_k: alpha_k = rho_k / rh.v, s = r - alpha v, t = C K^-1 s
//   bi3_k: omega_k = t.s / t.t, x += K^-1 (alpha p + omega s), r = s - omega t

template <typename R, int D, bool TRANS>
__device__ __forceinline__ R coef_p(const R* __restrict__ C, int j, int P, int N) {
  return TRANS ? C[(size_t)(D + j) * N + P] : C[(size_t)j * N + P];
}
template <typename R, int D, bool TRANS>
__device__ __forceinline__ R coef_m(const R* __restrict__ C, int j, int Fm, int N) {
  return TRANS ? C[(size_t)j * N + Fm] : C[(size_t)(D + j) * N + Fm];
}

// 1 / A once per solve (the same correctly rounded quotient the iterations would form
// per neighbour).
template <typename R>
__global__ void __launch_bounds__(kWG) k_bi_recip(int N, const R* __restrict__ A, R* __restrict__ iA) {
  const int P = cell_of_thread(N);
  if (P >= 0) iA[P] = R(1) / A[P];
}

template <typename R, int D, bool TRANS>
__global__ void __launch_bounds__(kWG)
k_bi_init(Grid g, const R* __restrict__ A, const R* __restrict__ C, const R* __restrict__ b,
          const R* __restrict__ x, R* __restrict__ r, R* __restrict__ rh, R* __restrict__ p0,
          R* __restrict__ v0, double* __restrict__ part3) {
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[3 * D];
#pragma unroll
  for (int q = 0; q < 3 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    // a face without a neighbour cell reads the cell itself with coefficient 0
    R cp[D], cm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const bool hp = Fp[j] >= 0, hm = Fm[j] >= 0;
      Fp[j] = hp ? Fp[j] : P;
      Fm[j] = hm ? Fm[j] : P;
      const R cpv = coef_p<R, D, TRANS>(C, j, P, N), cmv = coef_m<R, D, TRANS>(C, j, Fm[j], N);
      cp[j] = hp ? cpv : R(0);
      cm[j] = hm ? cmv : R(0);
    }
    const R AP = A[P];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const R* xc = x + (size_t)c * N;
      R Cx = AP * xc[P];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        Cx += cp[j] * xc[Fp[j]];
        Cx += cm[j] * xc[Fm[j]];
      }
      const R bv = b[(size_t)c * N + P];
      const R rv = bv - Cx;
      r[(size_t)c * N + P] = rv;
      rh[(size_t)c * N + P] = rv;
      p0[(size_t)c * N + P] = R(0);
      v0[(size_t)c * N + P] = R(0);
      acc[c] += (double)rv * (double)rv;
      acc[D + c] += (double)rv * (double)rv;
      acc[2 * D + c] += (double)bv * (double)bv;
    }
  }
  write_partials<3 * D>(acc, part3);
}

// MIXED form: r32 = (float)(b - C x) (C^T x with TRANS), formed in double with the
// double coefficients of the step; partials of r_c.r_c and b_c.b_c per component.
template <int D, bool TRANS>
__global__ void __launch_bounds__(kWG)
k_bi_mix_resid(Grid g, const double* __restrict__ A, const double* __restrict__ C, const double* __restrict__ b,
               const double* __restrict__ x, float* __restrict__ r32, double* __restrict__ part) {
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    double cp[D], cm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const bool hp = Fp[j] >= 0, hm = Fm[j] >= 0;
      Fp[j] = hp ? Fp[j] : P;
      Fm[j] = hm ? Fm[j] : P;
      const double cpv = coef_p<double, D, TRANS>(C, j, P, N), cmv = coef_m<double, D, TRANS>(C, j, Fm[j], N);
      cp[j] = hp ? cpv : 0.0;
      cm[j] = hm ? cmv : 0.0;
    }
    const double AP = A[P];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double* xc = x + (size_t)c * N;
      double Cx = AP * xc[P];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        Cx += cp[j] * xc[Fp[j]];
        Cx += cm[j] * xc[Fm[j]];
      }
      const double bv = b[(size_t)c * N + P];
      const double rv = bv - Cx;
      r32[(size_t)c * N + P] = (float)rv;
      acc[c] += rv * rv;
      acc[D + c] += bv * bv;
    }
  }
  write_partials<2 * D>(acc, part);
}

template <int D>
__global__ void __launch_bounds__(kWG)
k_bi_check(const double* __restrict__ part3, int G, int first, int k_total, double tol2, BiState* st) {
  double t[3 * D];
  if (first) {
    reduce_partials<3 * D>(part3, G, t);
  } else {
    double t2[2 * D];
    reduce_partials<2 * D>(part3, G, t2);
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) t[q] = t2[q];
#pragma unroll
    for (int q = 2 * D; q < 3 * D; ++q) t[q] = 0.0;
  }
  if (threadIdx.x != 0) return;
  if (first) {
    st->tol2 = tol2;
    for (int c = 0; c < 3; ++c) {
      st->rho[1][c] = st->alpha[1][c] = st->omega[1][c] = 1.0;
      st->iters[c] = 0;
      st->status[c] = 0;
      st->done[c] = c < D ? 0 : 1;
    }
    for (int c = 0; c < D; ++c) st->bb[c] = t[2 * D + c];
  }
  int all = 1;
  for (int c = 0; c < D; ++c) {
    if (!st->done[c]) {
      st->rr[c] = t[D + c];
      st->iters[c] = k_total;
      if (!std::isfinite(t[c]) || !std::isfinite(t[D + c]) || !std::isfinite(st->bb[c])) {
        st->status[c] = PISO_E_NAN;
        st->done[c] = 1;
      } else if (st->bb[c] == 0.0 || t[D + c] <= tol2 * st->bb[c]) {
        st->done[c] = 1;
      }
    }
    all &= st->done[c];
  }
  st->all_done = all;
}

template <typename R, int D, bool TRANS>
__global__ void __launch_bounds__(kWG)
k_bi_1(Grid g, const R* __restrict__ iA, const R* __restrict__ C, const R* __restrict__ r,
       const R* __restrict__ rh, const R* __restrict__ p_old, const R* __restrict__ v_old,
       R* __restrict__ p_new, R* __restrict__ v_new, BiState* st, const double* __restrict__ part3,
       double* __restrict__ part1, int Gp, int k) {
  if (st->all_done) return;
  double t[2 * D];
  reduce_partials<2 * D>(part3, Gp, t);
  const int ko = k & 1, kp = (k + 1) & 1;
  R beta[D], omega[D];
  bool act[D];
  int nact = 0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    beta[c] = R(0);
    omega[c] = R(0);
    if (!act[c]) continue;
    const double rho = t[c], rr = t[D + c];
    const bool conv = rr <= st->tol2 * st->bb[c];
    const bool bad = !std::isfinite(rho) || !std::isfinite(rr);
    const bool brk = !conv && !bad && (rho == 0.0 || st->omega[kp][c] == 0.0);
    if (conv || bad || brk) {
      if (lead()) {
        st->rr[c] = rr;
        st->iters[c] = k;
        st->status[c] = bad ? PISO_E_NAN : (brk ? PISO_BREAKDOWN : 0);
        st->done[c] = 1;
      }
      act[c] = false;
      continue;
    }
    beta[c] = (R)((rho / st->rho[kp][c]) * (st->alpha[kp][c] / st->omega[kp][c]));
    omega[c] = (R)st->omega[kp][c];
    ++nact;
    if (lead()) {
      st->rho[ko][c] = rho;
      st->rr[c] = rr;
    }
  }
  if (nact == 0) {
    if (lead()) st->all_done = 1;
    return;
  }
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    // a face without a neighbour cell (a Dirichlet side) reads the cell itself with
    // coefficient 0: every load is unconditional and its term adds exactly nothing
    R cp[D], cm[D], iAp[D], iAm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const bool hp = Fp[j] >= 0, hm = Fm[j] >= 0;
      Fp[j] = hp ? Fp[j] : P;
      Fm[j] = hm ? Fm[j] : P;
      const R cpv = coef_p<R, D, TRANS>(C, j, P, N), cmv = coef_m<R, D, TRANS>(C, j, Fm[j], N);
      const R ipv = iA[Fp[j]], imv = iA[Fm[j]];
      cp[j] = hp ? cpv : R(0);
      cm[j] = hm ? cmv : R(0);
      iAp[j] = hp ? ipv : R(0);
      iAm[j] = hm ? imv : R(0);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (!act[c]) continue;
      const size_t o = (size_t)c * N;
      auto pn = [&](int X) { return r[o + X] + beta[c] * (p_old[o + X] - omega[c] * v_old[o + X]); };
      const R pP = pn(P);
      R v = pP;   // A_P (p_P / A_P)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        v += cp[j] * pn(Fp[j]) * iAp[j];
        v += cm[j] * pn(Fm[j]) * iAm[j];
      }
      p_new[o + P] = pP;
      v_new[o + P] = v;
      acc[c] += (double)rh[o + P] * (double)v;
    }
  }
  write_partials<D>(acc, part1);
}

template <typename R, int D, bool TRANS>
__global__ void __launch_bounds__(kWG)
k_bi_2(Grid g, const R* __restrict__ iA, const R* __restrict__ C, const R* __restrict__ r,
       const R* __restrict__ v, R* __restrict__ s, R* __restrict__ t, BiState* st,
       const double* __restrict__ part1, double* __restrict__ part2, int Gp, int k) {
  if (st->all_done) return;
  double rv[D];
  reduce_partials<D>(part1, Gp, rv);
  const int ko = k & 1;
  R alpha[D];
  bool act[D];
  int nact = 0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    alpha[c] = R(0);
    if (!act[c]) continue;
    if (rv[c] == 0.0 || !std::isfinite(rv[c])) {
      if (lead()) {
        st->status[c] = std::isfinite(rv[c]) ? PISO_BREAKDOWN : PISO_E_NAN;
        st->iters[c] = k;
        st->done[c] = 1;
      }
      act[c] = false;
      continue;
    }
    const double a = st->rho[ko][c] / rv[c];
    alpha[c] = (R)a;
    ++nact;
    if (lead()) st->alpha[ko][c] = a;
  }
  if (nact == 0) return;
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    // a face without a neighbour cell (a Dirichlet side) reads the cell itself with
    // coefficient 0: every load is unconditional and its term adds exactly nothing
    R cp[D], cm[D], iAp[D], iAm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const bool hp = Fp[j] >= 0, hm = Fm[j] >= 0;
      Fp[j] = hp ? Fp[j] : P;
      Fm[j] = hm ? Fm[j] : P;
      const R cpv = coef_p<R, D, TRANS>(C, j, P, N), cmv = coef_m<R, D, TRANS>(C, j, Fm[j], N);
      const R ipv = iA[Fp[j]], imv = iA[Fm[j]];
      cp[j] = hp ? cpv : R(0);
      cm[j] = hm ? cmv : R(0);
      iAp[j] = hp ? ipv : R(0);
      iAm[j] = hm ? imv : R(0);
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
        tv += cp[j] * sv(Fp[j]) * iAp[j];
        tv += cm[j] * sv(Fm[j]) * iAm[j];
      }
      s[o + P] = sP;
      t[o + P] = tv;
      acc[c] += (double)tv * (double)sP;
      acc[D + c] += (double)tv * (double)tv;
    }
  }
  write_partials<2 * D>(acc, part2);
}

template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_bi_3(int N, const R* __restrict__ iAv, R* __restrict__ x, R* __restrict__ r, const R* __restrict__ rh,
       const R* __restrict__ p, const R* __restrict__ s, const R* __restrict__ t, BiState* st,
       const double* __restrict__ part2, double* __restrict__ part3, int Gp, int k) {
  if (st->all_done) return;
  double ts[2 * D];
  reduce_partials<2 * D>(part2, Gp, ts);
  const int ko = k & 1;
  R alpha[D], omega[D];
  bool act[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    const double w = ts[D + c] > 0.0 ? ts[c] / ts[D + c] : 0.0;
    omega[c] = (R)w;
    alpha[c] = (R)st->alpha[ko][c];
    if (act[c] && lead()) st->omega[ko][c] = w;
  }
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    const R iA = iAv[P];
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
  write_partials<2 * D>(acc, part3);
}

// ------------------------------------------------- BiCGStab with ILU(0) (App. A.6)
// Right preconditioning with the ILU(0) factorisation of C in red-black order: a cell's
// colour is (i + j + k + parity of its block) & 1, and every face joins two colours, so
// with the first colour ordered first C = [D_1 B; E D_2] with diagonal D_1, D_2 and
//   L = [I 0; E D_1^-1 I],   U = [D_1 B; 0 S],   S = D_2 - diag(E D_1^-1 B)
// (ILU(0) keeps the sparsity of C, whose second-colour block is diagonal: only the
// diagonal of the fill-in E D_1^-1 B survives).  For a second-colour cell P
//   S_P = A_P - sum_F C_PF C_FP / A_F.
// z = M^-1 r = U^-1 L^-1 r is one sweep per colour:
//   second colour:  z_P = (r_P - sum_F C_PF r_F / A_F) / S_P
//   first colour:   z_P = (r_P - sum_F C_PF z_F) / A_P.
// The transposed operator (the adjoint solve) uses the ILU(0) of C^T: the same S, the
// couplings swapped.  The iteration is the Jacobi one's with K^-1 = M^-1 applied to p
// and s as separate passes (the sweeps need neighbours' values of a finished pass).

template <int D>
__device__ __forceinline__ int cell_colour(const Grid& g, const Cell& c) {
  return (c.i + c.j + (D == 3 ? c.k : 0) + g.tab[c.b * kTabStride + kTabColour]) & 1;
}

// 1 / S on second-colour cells, 1 / A on first-colour cells.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_ilu_setup(Grid g, const R* __restrict__ A, const R* __restrict__ C, R* __restrict__ sinv) {
  const int N = g.N;
  const int P = cell_of_thread(N);
  if (P < 0) return;
  const Cell c = locate(g, P);
  R piv = A[P];
  if (cell_colour<D>(g, c)) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int Fp = neighbour(g, c, P, j, 1), Fm = neighbour(g, c, P, j, 0);
      // C_PF C_FP is the same product for C and C^T
      if (Fp >= 0) piv -= C[(size_t)j * N + P] * C[(size_t)(D + j) * N + P] / A[Fp];
      if (Fm >= 0) piv -= C[(size_t)(D + j) * N + Fm] * C[(size_t)j * N + Fm] / A[Fm];
    }
  }
  sinv[P] = R(1) / piv;
}

// One colour sweep of z = M^-1 r for the d components: SECOND = 1 forms the
// second-colour values from r, SECOND = 0 the first-colour ones from r and the finished
// second-colour z.
template <typename R, int D, bool TRANS, bool SECOND>
__global__ void __launch_bounds__(kWG)
k_ilu_sweep(Grid g, const R* __restrict__ A, const R* __restrict__ C, const R* __restrict__ sinv,
            const R* __restrict__ r, R* __restrict__ z, const BiState* st) {
  if (st->all_done) return;
  const int N = g.N;
  const int P = cell_of_thread(N);
  if (P < 0) return;
  const Cell c = locate(g, P);
  if (cell_colour<D>(g, c) != (SECOND ? 1 : 0)) return;
  int Fp[D], Fm[D];
  bool hp[D], hm[D];
  R cp[D], cm[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    Fp[j] = neighbour(g, c, P, j, 1);
    Fm[j] = neighbour(g, c, P, j, 0);
    hp[j] = Fp[j] >= 0;
    hm[j] = Fm[j] >= 0;
    Fp[j] = hp[j] ? Fp[j] : P;
    Fm[j] = hm[j] ? Fm[j] : P;
    const R cpv = coef_p<R, D, TRANS>(C, j, P, N), cmv = coef_m<R, D, TRANS>(C, j, Fm[j], N);
    // second colour: the neighbours' 1/A folded into the coupling
    cp[j] = SECOND ? cpv / A[Fp[j]] : cpv;
    cm[j] = SECOND ? cmv / A[Fm[j]] : cmv;
  }
  const R sp = sinv[P];
  const R* src = SECOND ? r : z;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const size_t o = (size_t)q * N;
    R v = r[o + P];
    // a face without a neighbour reads the cell itself and drops the term by selection:
    // in the first-colour sweep that value is this sweep's own, not yet written output
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const R vp = src[o + Fp[j]], vm = src[o + Fm[j]];
      v -= (hp[j] ? cp[j] * vp : R(0)) + (hm[j] ? cm[j] * vm : R(0));
    }
    z[o + P] = v * sp;
  }
}

// rho_k = rh.r, convergence and breakdown, beta_k; p = r + beta (p - omega v).
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_bii_p(int N, const R* __restrict__ r, const R* __restrict__ p_old, const R* __restrict__ v_old,
        R* __restrict__ p_new, BiState* st, const double* __restrict__ part3, int Gp, int k) {
  if (st->all_done) return;
  double t[2 * D];
  reduce_partials<2 * D>(part3, Gp, t);
  const int ko = k & 1, kp = (k + 1) & 1;
  R beta[D], omega[D];
  bool act[D];
  int nact = 0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    beta[c] = omega[c] = R(0);
    if (!act[c]) continue;
    const double rho = t[c], rr = t[D + c];
    const bool conv = rr <= st->tol2 * st->bb[c];
    const bool bad = !std::isfinite(rho) || !std::isfinite(rr);
    const bool brk = !conv && !bad && (rho == 0.0 || st->omega[kp][c] == 0.0);
    if (conv || bad || brk) {
      if (lead()) {
        st->rr[c] = rr;
        st->iters[c] = k;
        st->status[c] = bad ? PISO_E_NAN : (brk ? PISO_BREAKDOWN : 0);
        st->done[c] = 1;
      }
      act[c] = false;
      continue;
    }
    beta[c] = (R)((rho / st->rho[kp][c]) * (st->alpha[kp][c] / st->omega[kp][c]));
    omega[c] = (R)st->omega[kp][c];
    ++nact;
    if (lead()) {
      st->rho[ko][c] = rho;
      st->rr[c] = rr;
    }
  }
  if (nact == 0) {
    if (lead()) st->all_done = 1;
    return;
  }
  int beg, end;
  chunk_range(N, beg, end);
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (!act[c]) continue;
      const size_t o = (size_t)c * N + P;
      p_new[o] = r[o] + beta[c] * (p_old[o] - omega[c] * v_old[o]);
    }
  }
}

// y = C x (C^T x with TRANS) for the d components; partials of h1.y (NV = D: h1 = r-hat)
// or of h1.y and y.y (NV = 2 D: h1 = s).
template <typename R, int D, bool TRANS, int NV>
__global__ void __launch_bounds__(kWG)
k_bii_spmv(Grid g, const R* __restrict__ A, const R* __restrict__ C, const R* __restrict__ x,
           const R* __restrict__ h1, R* __restrict__ y, const BiState* st, double* __restrict__ part) {
  if (st->all_done) return;
  const int N = g.N;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    int Fp[D], Fm[D];
    faces_of<D>(g, P, Fp, Fm);
    R cp[D], cm[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const bool hp = Fp[j] >= 0, hm = Fm[j] >= 0;
      Fp[j] = hp ? Fp[j] : P;
      Fm[j] = hm ? Fm[j] : P;
      const R cpv = coef_p<R, D, TRANS>(C, j, P, N), cmv = coef_m<R, D, TRANS>(C, j, Fm[j], N);
      cp[j] = hp ? cpv : R(0);
      cm[j] = hm ? cmv : R(0);
    }
    const R AP = A[P];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const size_t o = (size_t)c * N;
      R v = AP * x[o + P];
#pragma unroll
      for (int j = 0; j < D; ++j) v += cp[j] * x[o + Fp[j]] + cm[j] * x[o + Fm[j]];
      y[o + P] = v;
      acc[c] += (double)h1[o + P] * (double)v;
      if constexpr (NV == 2 * D) acc[D + c] += (double)v * (double)v;
    }
  }
  write_partials<NV>(acc, part);
}

// alpha_k = rho_k / rh.v (breakdown checks); s = r - alpha v.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_bii_s(int N, const R* __restrict__ r, const R* __restrict__ v, R* __restrict__ s, BiState* st,
        const double* __restrict__ part1, int Gp, int k) {
  if (st->all_done) return;
  double rv[D];
  reduce_partials<D>(part1, Gp, rv);
  const int ko = k & 1;
  R alpha[D];
  bool act[D];
  int nact = 0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    alpha[c] = R(0);
    if (!act[c]) continue;
    if (rv[c] == 0.0 || !std::isfinite(rv[c])) {
      if (lead()) {
        st->status[c] = std::isfinite(rv[c]) ? PISO_BREAKDOWN : PISO_E_NAN;
        st->iters[c] = k;
        st->done[c] = 1;
      }
      act[c] = false;
      continue;
    }
    const double a = st->rho[ko][c] / rv[c];
    alpha[c] = (R)a;
    ++nact;
    if (lead()) st->alpha[ko][c] = a;
  }
  if (nact == 0) return;
  int beg, end;
  chunk_range(N, beg, end);
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (!act[c]) continue;
      const size_t o = (size_t)c * N + P;
      s[o] = r[o] - alpha[c] * v[o];
    }
  }
}

// omega_k = t.s / t.t; x += alpha M^-1 p + omega M^-1 s; r = s - omega t.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_bii_x(int N, R* __restrict__ x, R* __restrict__ r, const R* __restrict__ rh, const R* __restrict__ ph,
        const R* __restrict__ sh, const R* __restrict__ s, const R* __restrict__ t, BiState* st,
        const double* __restrict__ part2, double* __restrict__ part3, int Gp, int k) {
  if (st->all_done) return;
  double ts[2 * D];
  reduce_partials<2 * D>(part2, Gp, ts);
  const int ko = k & 1;
  R alpha[D], omega[D];
  bool act[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    act[c] = !st->done[c];
    const double w = ts[D + c] > 0.0 ? ts[c] / ts[D + c] : 0.0;
    omega[c] = (R)w;
    alpha[c] = (R)st->alpha[ko][c];
    if (act[c] && lead()) st->omega[ko][c] = w;
  }
  int beg, end;
  chunk_range(N, beg, end);
  double acc[2 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) acc[q] = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (!act[c]) continue;
      const size_t o = (size_t)c * N + P;
      x[o] += alpha[c] * ph[o] + omega[c] * sh[o];
      const R rn = s[o] - omega[c] * t[o];
      r[o] = rn;
      acc[c] += (double)rh[o] * (double)rn;
      acc[D + c] += (double)rn * (double)rn;
    }
  }
  write_partials<2 * D>(acc, part3);
}

// ------------------------------------------------------------------ host drivers

static int check(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

// Operands of the PCG iterations.  The solver copies the caller's coefficients and
// iterate into context-owned buffers, so that every pointer an iteration uses belongs
// to the context and a recorded iteration stays valid for the context's lifetime.
template <typename R>
struct PcgOps {
  const R* Pf;
  const R* Dinv;
  R* x;
  R *r, *r2, *q, *d0, *d1, *z, *y;   // r2: second residual buffer (multigrid: r alternates by parity)
  double *pA, *pB;
  int G;
  int Gz;          // work-groups whose partial sums of r.z, r.r the V-cycle leaves (G, or the line kernels')
  bool mg, quad, line;
};

// One PCG iteration with slot parity par (the direction buffers alternate with it).
template <typename R>
static int pcg_iteration(piso_ctx* c, hipStream_t s, const PcgOps<R>& o, int par) {
  const int N = c->N, G = o.G;
  CgState* st = c->cg;
  R* dold = par ? o.d1 : o.d0;
  R* dnew = par ? o.d0 : o.d1;
  const R* opnd = o.mg ? (const R*)o.z : (const R*)o.r;
  const double* pBc = o.pB;
  // 3D multigrid with point smoothing: the plane-marching kernels (their own grid)
  const bool zm = o.quad && o.mg && !o.line && zm_use(c, sizeof(R));
  const int Gs = zm ? zm_groups(c) : G;   // groups of the stencil kernel's d.q partials
  if (zm) {
    zm_launch_spmv<R>(c, s, o.Pf, (const R*)o.z, (const R*)dold, dnew, o.q, st, pBc, o.pA, o.Gz, par);
  } else if (o.quad) {
    if (c->dim == 2) {
      if (o.mg)
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv_q<R, 2, true>, G, c->grid, o.Pf, o.Dinv, opnd,
                     (const R*)dold, dnew, o.q, st, pBc, o.pA, o.Gz, par);
      else
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv_q<R, 2>, G, c->grid, o.Pf, o.Dinv, opnd, (const R*)dold,
                     dnew, o.q, st, pBc, o.pA, G, par);
    } else {
      if (o.mg)
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv_q<R, 3, true>, G, c->grid, o.Pf, o.Dinv, opnd,
                     (const R*)dold, dnew, o.q, st, pBc, o.pA, o.Gz, par);
      else
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv_q<R, 3>, G, c->grid, o.Pf, o.Dinv, opnd, (const R*)dold,
                     dnew, o.q, st, pBc, o.pA, G, par);
    }
    if (!o.mg)
      launch_timed(c, s, kTimeCgUpdate, k_cg_update_q<R>, G, N, o.Dinv, o.x, o.r, (const R*)dnew, (const R*)o.q,
                   st, (const double*)o.pA, o.pB, G, par);
  } else {
    if (c->dim == 2) {
      if (o.mg)
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv<R, 2, true>, G, c->grid, o.Pf, o.Dinv, opnd, (const R*)dold,
                     dnew, o.q, st, pBc, o.pA, o.Gz, par);
      else
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv<R, 2>, G, c->grid, o.Pf, o.Dinv, opnd, (const R*)dold, dnew,
                     o.q, st, pBc, o.pA, G, par);
    } else {
      if (o.mg)
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv<R, 3, true>, G, c->grid, o.Pf, o.Dinv, opnd, (const R*)dold,
                     dnew, o.q, st, pBc, o.pA, o.Gz, par);
      else
        launch_timed(c, s, kTimeCgStencil, k_cg_spmv<R, 3>, G, c->grid, o.Pf, o.Dinv, opnd, (const R*)dold, dnew,
                     o.q, st, pBc, o.pA, G, par);
    }
    if (!o.mg)
      launch_timed(c, s, kTimeCgUpdate, k_cg_update<R>, G, N, o.Dinv, o.x, o.r, (const R*)dnew, (const R*)o.q, st,
                   (const double*)o.pA, o.pB, G, par);
  }
  // multigrid: the update is fused with the fine-grid restriction; the residual moves
  // between r (even iterations read it) and r2 (odd ones)
  if (o.mg && o.line) {
    // line smoothing: the update with the line pre-smoothing, then the V-cycle on r'
    const R* rin = par ? (const R*)o.r2 : (const R*)o.r;
    R* rout = par ? o.r : o.r2;
    if (int rc = line_pre<R>(c, s, o.Pf, o.Dinv, o.x, rin, rout, (const R*)dnew, (const R*)o.q, o.y, st,
                             (const double*)o.pA, G, par, true))
      return rc;
    return mg_apply<R>(c, s, o.Pf, o.Dinv, (const R*)rout, (const R*)o.y, o.z, st, o.pB, G);
  }
  if (o.mg)
    return mg_update_apply<R>(c, s, o.Pf, o.Dinv, o.x, par ? (const R*)o.r2 : (const R*)o.r, par ? o.r : o.r2,
                              (const R*)dnew, (const R*)o.q, o.y, o.z, st, (const double*)o.pA, Gs, par, o.pB, G);
  return check(c, "PCG iteration");
}

// Two iterations (parity 0 then 1) recorded once per preconditioner and replayed.
template <typename R>
static int pcg_graph(piso_ctx* c, const PcgOps<R>& o, hipGraphExec_t* out) {
  if (!c->cap_stream) PISO_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = c->cap_stream;
  PISO_HIP(c, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  int rc = pcg_iteration<R>(c, cs, o, 0);
  if (!rc) rc = pcg_iteration<R>(c, cs, o, 1);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc ? rc : fail(c, PISO_E_HIP, std::string("PCG graph capture: ") + hipGetErrorString(e));
  }
  const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return fail(c, PISO_E_HIP, std::string("PCG graph instantiate: ") + hipGetErrorString(ei));
  return PISO_OK;
}

static int pcg_groups(const piso_ctx* c) {
  if (c->cg_grid > 0) return c->cg_grid;
  return solver_groups(c->quad ? (long)c->N / 4 : (long)c->N);
}

template <typename R, typename BT>
static int pcg_run(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const BT* b,
                   const double* mean, double sign, R* x, double rtol, int max_iter, int check_every,
                   int precond, int* iters_out, double* rel_out, int* status_out, int hint_slot = 0) {
  const int N = c->N, G = pcg_groups(c);
  CgState* st = c->cg;
  PcgOps<R> o;
  o.Pf = (const R*)c->g_Pf;
  o.Dinv = (const R*)c->g_Dinv;
  o.x = (R*)c->g_x;
  o.r = (R*)c->k_r;
  o.r2 = (R*)c->k_r2;
  o.q = (R*)c->k_q;
  o.d0 = (R*)c->k_d0;
  o.d1 = (R*)c->k_d1;
  o.z = (R*)c->k_z;
  o.y = (R*)c->k_y;
  o.pA = part(c, kPartA);
  o.pB = part(c, kPartB);
  o.G = G;
  // multigrid: z = B r is stored by the V-cycle (which also writes the r.z, r.r
  // partials); the stencil kernel then forms d from z instead of Dinv r
  o.mg = precond == PISO_PRECOND_MG && !c->mg.empty();
  o.quad = c->quad;   // the context's buffers are 256-byte aligned
  o.line = o.mg && c->mg_line_axis != 0;
  o.Gz = o.line ? line_groups(c) : (o.mg && o.quad && zm_use(c, sizeof(R)) ? zm_groups(c) : G);
  const size_t es = sizeof(R);
  const bool reuse = c->pcg_same_op && c->pcg_op_src == (const void*)Pf && c->pcg_op_es == (int)es &&
                     (c->pcg_op_mg || !o.mg);
  if (!reuse) {
    c->pcg_op_src = nullptr;   // invalid until the setup below is enqueued
    PISO_HIP(c, hipMemcpyAsync((void*)o.Pf, Pf, es * (size_t)c->dim * N, hipMemcpyDeviceToDevice, s));
    PISO_HIP(c, hipMemcpyAsync((void*)o.Dinv, Dinv, es * (size_t)N, hipMemcpyDeviceToDevice, s));
    if (o.mg) {
      if (int rc = mg_setup<R>(c, s, o.Pf)) return rc;
    }
    c->pcg_op_src = Pf;
    c->pcg_op_es = (int)es;
    c->pcg_op_mg = o.mg;
  }
  PISO_HIP(c, hipMemcpyAsync(o.x, x, es * (size_t)N, hipMemcpyDeviceToDevice, s));
  const double tol2 = rtol * rtol;
  if (c->dim == 2)
    k_cg_init<R, BT, 2><<<G, kWG, 0, s>>>(c->grid, o.Pf, o.Dinv, b, mean, sign, o.x, o.r, o.d0, o.pB);
  else
    k_cg_init<R, BT, 3><<<G, kWG, 0, s>>>(c->grid, o.Pf, o.Dinv, b, mean, sign, o.x, o.r, o.d0, o.pB);
  k_cg_check<<<1, kWG, 0, s>>>(o.pB, G, 1, max_iter, tol2, st);
  if (int rc = check(c, "k_cg_init")) return rc;
  if (o.mg) {
    if (o.line) {
      if (int rc = line_pre<R>(c, s, o.Pf, o.Dinv, o.x, (const R*)o.r, o.r, nullptr, nullptr, o.y, st, nullptr, 0, 0,
                               false))
        return rc;
    } else {
      if (int rc = mg_prescale<R>(c, s, o.Dinv, (const R*)o.r, o.y)) return rc;
    }
    if (int rc = mg_apply<R>(c, s, o.Pf, o.Dinv, (const R*)o.r, (const R*)o.y, o.z, st, o.pB, G)) return rc;
  }
  // no read-back here: a zero right-hand side is handled on the device, and iterations
  // launched after convergence return at once
  k_cg_zero_if<R><<<grid_cells(N), kWG, 0, s>>>(N, st, o.x);
  c->h_cg->done = 0;
  // chunks of an even number of iterations: the recorded pair keeps the slot parity
  if (check_every < 2) check_every = 2;
  check_every += check_every & 1;
  // replay the recorded pair unless the kernels are being timed one by one
  hipGraphExec_t* gx = &c->cg_graph[o.mg ? 1 : 0];
  const bool use_graph = !c->timing.enabled && c->use_graphs;
  if (use_graph && !*gx) {
    if (int rc = pcg_graph<R>(c, o, gx)) return rc;
  }
  // the first chunk covers the iterations of the previous solve of the same kind less two
  // (solves of one kind in consecutive steps take similar counts, different kinds do
  // not; an iteration launched after convergence costs about as much as a read-back),
  // later chunks check_every
  const int kind = c->pcg_kind >= 0 && c->pcg_kind <= kPcgOther ? c->pcg_kind : kPcgOther;
  int& hint = c->pcg_hint[o.mg ? 1 : 0][kind][hint_slot];
  int chunk = std::max(check_every, (hint - 2) & ~1);
  int launched = 0;
  while (!c->h_cg->done && launched < max_iter) {
    const int n = std::min(chunk, max_iter - launched + 1);
    chunk = check_every;
    for (int k = 0; k < n; k += 2) {
      if (use_graph) {
        PISO_HIP(c, hipGraphLaunch(*gx, s));
      } else {
        if (int rc = pcg_iteration<R>(c, s, o, 0)) return rc;
        if (int rc = pcg_iteration<R>(c, s, o, 1)) return rc;
      }
    }
    launched += n + (n & 1);
    k_cg_check<<<1, kWG, 0, s>>>(o.pB, o.Gz, 0, max_iter, tol2, st);
    if (int rc = check(c, "k_cg iteration")) return rc;
    PISO_HIP(c, hipMemcpyAsync(c->h_cg, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    PISO_HIP(c, hipStreamSynchronize(s));
    timing_collect(c);
  }
  PISO_HIP(c, hipMemcpyAsync(x, o.x, es * (size_t)N, hipMemcpyDeviceToDevice, s));
  const CgState& h = *c->h_cg;
  if (h.status == 0) hint = h.iters;
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
  if constexpr (std::is_same<R, double>::value && std::is_same<BT, double>::value) {
    if (c->prec == PISO_MIXED) return pressure_solve_mixed(c, s, Pf, Dinv, rhs, mean, x, o, info);
  }
  if (o->precond != PISO_PRECOND_JACOBI && o->precond != PISO_PRECOND_MG)
    return fail(c, PISO_E_ARG, "pressure solve: unknown preconditioner");
  int iters = 0, status = 0;
  double rel = 0.0;
  int rc = pcg_run<R, BT>(c, s, Pf, Dinv, rhs, mean, -1.0, x, o->rtol, o->max_iter, o->check_every,
                          o->precond, &iters, &rel, &status);
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

// MIXED form (pressure): the residual of the double system rhs64 - P x64 (the step's
// double face coefficients) in double, an inner float PCG on the float-rounded operator
// for the correction, x64 += e; repeated until the double relative residual is <= rtol.
int pressure_solve_mixed(piso_ctx* c, hipStream_t s, const double* Pf, const double* Dinv,
                         const double* rhs64, const double* mean, double* x64, const piso_solve_opts* o,
                         piso_solve_info* info) {
  if (o->precond != PISO_PRECOND_JACOBI && o->precond != PISO_PRECOND_MG)
    return fail(c, PISO_E_ARG, "pressure solve: unknown preconditioner");
  const int N = c->N, G = grid_red(N);
  float* r32 = (float*)c->m_r32;
  float* e32 = (float*)c->m_e32;
  float* Pf32 = (float*)c->x_Pf32;
  float* Dinv32 = (float*)c->x_Dinv32;
  double* pS = part(c, kPartS);
  // the float operator of the inner solves, rounded once per operator
  const bool same = c->pcg_same_op && c->mix_op_src == (const void*)Pf;
  if (!same) {
    c->mix_op_src = nullptr;
    if (int rc = launch_copy<double, float>(c, s, Pf, Pf32, c->dim * N)) return rc;
    if (int rc = launch_copy<double, float>(c, s, Dinv, Dinv32, N)) return rc;
    c->mix_op_src = Pf;
  }
  int iters = 0, status = 0, sweeps = 0;
  double rel = 0.0;
  for (;;) {
    if (c->dim == 2)
      k_mix_resid<2><<<G, kWG, 0, s>>>(c->grid, Pf, rhs64, mean, x64, r32, pS);
    else
      k_mix_resid<3><<<G, kWG, 0, s>>>(c->grid, Pf, rhs64, mean, x64, r32, pS);
    k_finalize<2><<<1, kWG, 0, s>>>(pS, G, c->mean + 2);
    if (int rc = check(c, "k_mix_resid")) return rc;
    PISO_HIP(c, hipMemcpyAsync(c->h_scal, c->mean + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    PISO_HIP(c, hipStreamSynchronize(s));
    const double rr = c->h_scal[0], bb = c->h_scal[1];
    if (!std::isfinite(rr) || !std::isfinite(bb)) {
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
    // ask the inner solve only for the reduction still missing, rtol / rel (the check of
    // the double residual above decides whether another sweep follows), but never for more
    // than inner_rtol, the floor the float iteration reliably reaches
    const double tol_in = std::min(0.5, std::max(o->inner_rtol, o->rtol / rel));
    const bool same_in = c->pcg_same_op;
    c->pcg_same_op = same || sweeps > 0;   // later sweeps and correctors: same operator
    int rc = pcg_run<float, float>(c, s, Pf32, Dinv32, r32, nullptr, 1.0, e32, tol_in, o->max_iter,
                                   o->check_every, o->precond, &iters, &rel_in, &st_in,
                                   1 + std::min(sweeps, 2));
    c->pcg_same_op = same_in;
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

static int velocity_solve_mixed(piso_ctx* c, hipStream_t s, bool trans, const double* A, const double* C,
                                const double* b, double* x, const piso_solve_opts* o, piso_solve_info* info);

template <typename R>
int velocity_solve(piso_ctx* c, hipStream_t s, bool trans, const R* A, const R* C, const R* b, R* x,
                   const piso_solve_opts* o, piso_solve_info* info) {
  if constexpr (std::is_same<R, double>::value) {
    if (c->prec == PISO_MIXED) return velocity_solve_mixed(c, s, trans, A, C, b, x, o, info);
  }
  return velocity_solve_ws<R>(c, s, trans, A, C, b, x, o, info, bi_work_ctx(c));
}

BiWork bi_work_ctx(piso_ctx* c) {
  BiWork w;
  w.r = c->b_r;
  w.rh = c->b_rh;
  w.p0 = c->b_p0;
  w.p1 = c->b_p1;
  w.v0 = c->b_v0;
  w.v1 = c->b_v1;
  w.s = c->b_s;
  w.t = c->b_t;
  w.iA = c->b_iA;
  w.ph = c->b_ph;
  w.sh = c->b_sh;
  w.sinv = c->b_sinv;
  w.part1 = part(c, kPart1);
  w.part2 = part(c, kPart2);
  w.part3 = part(c, kPart3);
  w.st = c->bi;
  return w;
}

// One BiCGStab solve from x (Jacobi or, with ilu, red-black ILU(0) right
// preconditioning).  Returns < 0 only for a failed HIP call; the solve's own outcome is
// info->status.
template <typename R>
static int bicgstab_run(piso_ctx* c, hipStream_t s, bool trans, const R* A, const R* C, const R* b, R* x,
                        const piso_solve_opts* o, piso_solve_info* info, const BiWork& w, bool ilu) {
  const int N = c->N, G = solver_groups(N), D = c->dim;   // cell-per-thread kernels
  R* r = (R*)w.r;
  R* rh = (R*)w.rh;
  R* pb[2] = {(R*)w.p0, (R*)w.p1};
  R* vb[2] = {(R*)w.v0, (R*)w.v1};
  R* sb = (R*)w.s;
  R* tb = (R*)w.t;
  BiState* st = w.st;
  double* p1 = w.part1;
  double* p2 = w.part2;
  double* p3 = w.part3;
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
#define BI_CHECK(FIRST, KT)                                                       \
  do {                                                                            \
    if (D == 2) k_bi_check<2><<<1, kWG, 0, s>>>(p3, G, FIRST, KT, tol2, st);      \
    else k_bi_check<3><<<1, kWG, 0, s>>>(p3, G, FIRST, KT, tol2, st);             \
  } while (0)
  R* iA = (R*)w.iA;
  R* ph = (R*)w.ph;
  R* sh = (R*)w.sh;
  R* sinv = (R*)w.sinv;
#define ILU_SWEEPS(SRC, DST)                                                                               \
  do {                                                                                                     \
    if (D == 2) {                                                                                          \
      if (trans) {                                                                                         \
        k_ilu_sweep<R, 2, true, true><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);    \
        k_ilu_sweep<R, 2, true, false><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);   \
      } else {                                                                                             \
        k_ilu_sweep<R, 2, false, true><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);   \
        k_ilu_sweep<R, 2, false, false><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);  \
      }                                                                                                    \
    } else {                                                                                               \
      if (trans) {                                                                                         \
        k_ilu_sweep<R, 3, true, true><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);    \
        k_ilu_sweep<R, 3, true, false><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);   \
      } else {                                                                                             \
        k_ilu_sweep<R, 3, false, true><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);   \
        k_ilu_sweep<R, 3, false, false><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv, SRC, DST, st);  \
      }                                                                                                    \
    }                                                                                                      \
  } while (0)
#define BII_SPMV(NVM, X, H1, Y, PART)                                                                      \
  do {                                                                                                     \
    if (D == 2) {                                                                                          \
      if (trans) k_bii_spmv<R, 2, true, 2 * NVM><<<G, kWG, 0, s>>>(c->grid, A, C, X, H1, Y, st, PART);     \
      else k_bii_spmv<R, 2, false, 2 * NVM><<<G, kWG, 0, s>>>(c->grid, A, C, X, H1, Y, st, PART);          \
    } else {                                                                                               \
      if (trans) k_bii_spmv<R, 3, true, 3 * NVM><<<G, kWG, 0, s>>>(c->grid, A, C, X, H1, Y, st, PART);     \
      else k_bii_spmv<R, 3, false, 3 * NVM><<<G, kWG, 0, s>>>(c->grid, A, C, X, H1, Y, st, PART);          \
    }                                                                                                      \
  } while (0)
  if (ilu) {
    if (D == 2) k_ilu_setup<R, 2><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv);
    else k_ilu_setup<R, 3><<<grid_cells(N), kWG, 0, s>>>(c->grid, A, C, sinv);
  } else {
    k_bi_recip<R><<<grid_cells(N), kWG, 0, s>>>(N, A, iA);
  }
  BI_LAUNCH(k_bi_init, c->grid, A, C, b, x, r, rh, pb[0], vb[0], p3);
  BI_CHECK(1, 0);
  // zero right-hand sides are handled on the device (no read-back before the iterations)
  if (D == 2) k_bi_zero_if<R, 2><<<grid_cells(N), kWG, 0, s>>>(N, st, x);
  else k_bi_zero_if<R, 3><<<grid_cells(N), kWG, 0, s>>>(N, st, x);
  if (int rc = check(c, "k_bi_init")) return rc;
  c->h_bi->all_done = 0;
  int it = 0;
  const int ce = o->check_every < 1 ? 4 : o->check_every;
  while (!c->h_bi->all_done && it < o->max_iter) {
    const int n = std::min(ce, o->max_iter - it);
    for (int k = 0; k < n; ++k, ++it) {
      R* po = pb[it & 1];
      R* pn = pb[(it + 1) & 1];
      R* vo = vb[it & 1];
      R* vn = vb[(it + 1) & 1];
      if (ilu) {
        // p, M^-1 p, v = C M^-1 p; s, M^-1 s, t = C M^-1 s; x, r
        if (D == 2) k_bii_p<R, 2><<<G, kWG, 0, s>>>(N, r, po, vo, pn, st, p3, G, it);
        else k_bii_p<R, 3><<<G, kWG, 0, s>>>(N, r, po, vo, pn, st, p3, G, it);
        ILU_SWEEPS(pn, ph);
        BII_SPMV(1, ph, rh, vn, p1);
        if (D == 2) k_bii_s<R, 2><<<G, kWG, 0, s>>>(N, r, vn, sb, st, p1, G, it);
        else k_bii_s<R, 3><<<G, kWG, 0, s>>>(N, r, vn, sb, st, p1, G, it);
        ILU_SWEEPS(sb, sh);
        BII_SPMV(2, sh, sb, tb, p2);
        if (D == 2) k_bii_x<R, 2><<<G, kWG, 0, s>>>(N, x, r, rh, ph, sh, sb, tb, st, p2, p3, G, it);
        else k_bii_x<R, 3><<<G, kWG, 0, s>>>(N, x, r, rh, ph, sh, sb, tb, st, p2, p3, G, it);
        continue;
      }
      BI_LAUNCH(k_bi_1, c->grid, iA, C, r, rh, po, vo, pn, vn, st, p3, p1, G, it);
      BI_LAUNCH(k_bi_2, c->grid, iA, C, r, vn, sb, tb, st, p1, p2, G, it);
      if (D == 2) k_bi_3<R, 2><<<G, kWG, 0, s>>>(N, iA, x, r, rh, pn, sb, tb, st, p2, p3, G, it);
      else k_bi_3<R, 3><<<G, kWG, 0, s>>>(N, iA, x, r, rh, pn, sb, tb, st, p2, p3, G, it);
    }
    BI_CHECK(0, it);
    if (int rc = check(c, "k_bi iteration")) return rc;
    PISO_HIP(c, hipMemcpyAsync(c->h_bi, st, sizeof(BiState), hipMemcpyDeviceToHost, s));
    PISO_HIP(c, hipStreamSynchronize(s));
  }
#undef BI_LAUNCH
#undef BI_CHECK
#undef ILU_SWEEPS
#undef BII_SPMV
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
  *info = piso_solve_info{};
  info->status = status;
  info->iters = iters;
  info->rel_residual = rel;
  return PISO_OK;
}

template <typename R>
int velocity_solve_ws(piso_ctx* c, hipStream_t s, bool trans, const R* A, const R* C, const R* b, R* x,
                      const piso_solve_opts* o, piso_solve_info* info, const BiWork& w) {
  const int pc = o->precond;
  if (pc != PISO_PRECOND_JACOBI && pc != PISO_PRECOND_ILU0 && pc != PISO_PRECOND_JACOBI_ILU0)
    return fail(c, PISO_E_ARG, "velocity solve: preconditioner must be Jacobi, ILU(0) or Jacobi with ILU(0) restart");
  if (pc == PISO_PRECOND_ILU0 && !c->ilu_ok)
    return fail(c, PISO_E_ARG, "velocity solve: ILU(0) needs a grid two colours tile (even periodic extents)");
  piso_solve_info tmp{};
  piso_solve_info* inf = info ? info : &tmp;
  int rc = bicgstab_run<R>(c, s, trans, A, C, b, x, o, inf, w, pc == PISO_PRECOND_ILU0);
  if (rc < 0) return rc;
  if (pc == PISO_PRECOND_JACOBI_ILU0 && inf->status != PISO_OK && c->ilu_ok) {
    // the Jacobi solve failed: restart with ILU(0) from its last iterate, or from zero
    // after a non-finite residual (the iterate may then hold non-finite values)
    if (inf->status == PISO_E_NAN)
      PISO_HIP(c, hipMemsetAsync(x, 0, sizeof(R) * (size_t)c->dim * c->N, s));
    const int first = inf->iters;
    rc = bicgstab_run<R>(c, s, trans, A, C, b, x, o, inf, w, true);
    if (rc < 0) return rc;
    inf->iters += first;
    inf->fallback = 1;
  }
  return inf->status < 0 ? inf->status : PISO_OK;
}

// MIXED form (velocity): the residuals b_c - C x_c (C^T with trans) of the double system
// in double, an inner float BiCGStab on the float-rounded operator for the corrections,
// x += e; repeated until every component's double relative residual is <= rtol.
static int velocity_solve_mixed(piso_ctx* c, hipStream_t s, bool trans, const double* A, const double* C,
                                const double* b, double* x, const piso_solve_opts* o, piso_solve_info* info) {
  const int pc = o->precond;
  if (pc != PISO_PRECOND_JACOBI && pc != PISO_PRECOND_ILU0 && pc != PISO_PRECOND_JACOBI_ILU0)
    return fail(c, PISO_E_ARG, "velocity solve: preconditioner must be Jacobi, ILU(0) or Jacobi with ILU(0) restart");
  const int N = c->N, D = c->dim, G = solver_groups(N);
  float* A32 = (float*)c->x_A32;
  float* C32 = (float*)c->x_C32;
  float* r32 = (float*)c->m_r32;
  float* e32 = (float*)c->m_e32;
  double* p3 = part(c, kPart3);
  if (int rc = launch_copy<double, float>(c, s, A, A32, N)) return rc;
  if (int rc = launch_copy<double, float>(c, s, C, C32, 2 * D * N)) return rc;
  int iters = 0, status = 0, sweeps = 0, fallback = 0;
  double rel = 0.0;
  bool zero_done = false;
  for (;;) {
    if (D == 2) {
      if (trans) k_bi_mix_resid<2, true><<<G, kWG, 0, s>>>(c->grid, A, C, b, x, r32, p3);
      else k_bi_mix_resid<2, false><<<G, kWG, 0, s>>>(c->grid, A, C, b, x, r32, p3);
      k_finalize<4><<<1, kWG, 0, s>>>(p3, G, c->mix_scal);
    } else {
      if (trans) k_bi_mix_resid<3, true><<<G, kWG, 0, s>>>(c->grid, A, C, b, x, r32, p3);
      else k_bi_mix_resid<3, false><<<G, kWG, 0, s>>>(c->grid, A, C, b, x, r32, p3);
      k_finalize<6><<<1, kWG, 0, s>>>(p3, G, c->mix_scal);
    }
    if (int rc = check(c, "k_bi_mix_resid")) return rc;
    PISO_HIP(c, hipMemcpyAsync(c->h_scal, c->mix_scal, 2 * D * sizeof(double), hipMemcpyDeviceToHost, s));
    PISO_HIP(c, hipStreamSynchronize(s));
    rel = 0.0;
    bool bad = false;
    for (int q = 0; q < D; ++q) {
      const double rr = c->h_scal[q], bb = c->h_scal[D + q];
      if (!std::isfinite(rr) || !std::isfinite(bb)) bad = true;
      else if (bb > 0.0) rel = std::max(rel, std::sqrt(rr / bb));
      else if (!zero_done) {
        // a zero right-hand side: the solution component is zero, and so its residual
        PISO_HIP(c, hipMemsetAsync(x + (size_t)q * N, 0, sizeof(double) * (size_t)N, s));
        PISO_HIP(c, hipMemsetAsync(r32 + (size_t)q * N, 0, sizeof(float) * (size_t)N, s));
      }
    }
    zero_done = true;
    if (bad) {
      status = PISO_E_NAN;
      break;
    }
    if (rel <= o->rtol) break;
    if (sweeps >= o->max_refine) {
      status = PISO_NOT_CONVERGED;
      break;
    }
    PISO_HIP(c, hipMemsetAsync(e32, 0, sizeof(float) * (size_t)D * N, s));
    piso_solve_opts in = *o;
    in.rtol = std::min(0.5, std::max(o->inner_rtol, 0.5 * o->rtol / rel));
    piso_solve_info ii{};
    int rc = velocity_solve<float>(c, s, trans, A32, C32, r32, e32, &in, &ii);
    if (rc < 0) {
      status = rc;
      break;
    }
    iters += ii.iters;
    if (ii.fallback) fallback = 1;
    k_mix_add<<<grid_cells(D * N), kWG, 0, s>>>(D * N, x, e32);
    if (int rc2 = check(c, "k_mix_add")) return rc2;
    ++sweeps;
  }
  if (info) {
    info->status = status;
    info->iters = iters;
    info->refinements = sweeps;
    info->fallback = fallback;
    info->rel_residual = rel;
  }
  return status < 0 ? status : PISO_OK;
}

template int pressure_solve<float, float>(piso_ctx*, hipStream_t, const float*, const float*, const float*,
                                          const double*, float*, const piso_solve_opts*, piso_solve_info*);
template int pressure_solve<double, double>(piso_ctx*, hipStream_t, const double*, const double*,
                                            const double*, const double*, double*, const piso_solve_opts*,
                                            piso_solve_info*);
template int velocity_solve_ws<float>(piso_ctx*, hipStream_t, bool, const float*, const float*, const float*,
                                      float*, const piso_solve_opts*, piso_solve_info*, const BiWork&);
template int velocity_solve_ws<double>(piso_ctx*, hipStream_t, bool, const double*, const double*,
                                       const double*, double*, const piso_solve_opts*, piso_solve_info*,
                                       const BiWork&);
template int velocity_solve<float>(piso_ctx*, hipStream_t, bool, const float*, const float*, const float*,
                                   float*, const piso_solve_opts*, piso_solve_info*);
template int velocity_solve<double>(piso_ctx*, hipStream_t, bool, const double*, const double*,
                                    const double*, double*, const piso_solve_opts*, piso_solve_info*);

}  // namespace piso
