// Forward kernels of the PISO step (arXiv 2505.16992, App. A.3): per-cell stencils over
// multi-block structured grids, one thread per cell, XCD-aware cell ranges.
//
// Conventions (see include/piso.h): SoA fields [comp][N]; face arrays [j][N] belong to
// the +j face of each cell; C is stored as A [N] plus C[0][j][P] = C(P, P+j) and
// C[1][j][P] = C(P+j, P); rows of C are per unit volume.
#include "piso_impl.h"

namespace piso {

// J T_ji at cell P (J T is stored diagonal-only when T is diagonal everywhere).
template <typename R, int D, bool DIAG>
__device__ __forceinline__ R jt(const R* __restrict__ JT, int j, int i, int P, int N) {
  if (DIAG) return j == i ? JT[(size_t)j * N + P] : R(0);
  return JT[(size_t)(j * D + i) * N + P];
}

// Contravariant flux U^j = J T_j . v of the cell vector v (components in v[i*N + P]).
template <typename R, int D, bool DIAG>
__device__ __forceinline__ R contra(const R* __restrict__ JT, const R* __restrict__ v, int j, int P, int N) {
  if (DIAG) return JT[(size_t)j * N + P] * v[(size_t)j * N + P];
  R s = R(0);
#pragma unroll
  for (int i = 0; i < D; ++i) s += JT[(size_t)(j * D + i) * N + P] * v[(size_t)i * N + P];
  return s;
}

__device__ __forceinline__ int ax_index(int j, int k) { return (j < k ? j : k) + (j < k ? k : j) - 1; }

// Tangential computational difference along axis k of a scalar field with one-sided
// differences next to a non-connected side (App. A.3.4, non-orthogonal treatment).
template <typename R>
__device__ __forceinline__ R tdiff(const Grid& g, const Cell& c, int P, int k, const R* __restrict__ f) {
  const int Fp = neighbour(g, c, P, k, 1), Fm = neighbour(g, c, P, k, 0);
  if (Fp >= 0 && Fm >= 0) return R(0.5) * (f[Fp] - f[Fm]);
  if (Fp >= 0) return f[Fp] - f[P];
  if (Fm >= 0) return f[P] - f[Fm];
  return R(0);
}

template <typename R, int D>
__global__ void __launch_bounds__(kWG) k_tgrad(Grid g, const R* __restrict__ phi, int ncomp, R* __restrict__ out) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const Cell c = locate(g, P);
  const int N = g.N;
  for (int q = 0; q < ncomp; ++q) {
#pragma unroll
    for (int k = 0; k < D; ++k) out[(size_t)(q * D + k) * N + P] = tdiff<R>(g, c, P, k, phi + (size_t)q * N);
  }
}

// Tangential difference along k of the Dirichlet values of side (j, s) around the face of
// cell P, through the same-side faces of P's k-neighbours (one-sided at segment ends).
template <typename R>
__device__ __forceinline__ R bdiff(const Grid& g, const Cell& c, int P, int j, int s, int k, int fown,
                                   const R* __restrict__ ubc) {
  int fp = -1, fm = -1;
  const int Qp = neighbour(g, c, P, k, 1), Qm = neighbour(g, c, P, k, 0);
  if (Qp >= 0) {
    int e = neighbour_of(g, Qp, j, s);
    if (e < 0) fp = -1 - e;
  }
  if (Qm >= 0) {
    int e = neighbour_of(g, Qm, j, s);
    if (e < 0) fm = -1 - e;
  }
  if (fp >= 0 && fm >= 0) return R(0.5) * (ubc[fp] - ubc[fm]);
  if (fp >= 0) return ubc[fp] - ubc[fown];
  if (fm >= 0) return ubc[fown] - ubc[fm];
  return R(0);
}

// Predictor assembly (App. A.3.3): face flux U_f = (U_P + U_F)/2, advective entries
// 0.5 N U_f (eq. advMatDiscrete), diffusive entries -lerp(alpha_jj nu) and 2 alpha_jj nu
// at Dirichlet faces (eq. difMatDiscrete), temporal term 1/dt; right-hand side
// u/dt + S + (1/J) sum_b u_b (2 alpha nu - N U_b) (eq. velRHSdiscrete) plus the deferred
// non-orthogonal diffusion of u^n and u_b (eq. velRHSnonOrtho); b = b_u - grad p^n.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_assemble(Grid g, const R* __restrict__ JT, const R* __restrict__ invJ, const R* __restrict__ alpha,
           const R* __restrict__ alphax, const R* __restrict__ bjt, const R* __restrict__ balpha,
           const R* __restrict__ u, const R* __restrict__ p,
           const R* __restrict__ nu, int nu_field, const R* __restrict__ S, const R* __restrict__ ub,
           R dt_inv, int gradp, const R* __restrict__ tgu, int nonorth, R* __restrict__ A,
           R* __restrict__ C, R* __restrict__ bu, R* __restrict__ b) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N, NB = g.NB;
  const Cell c = locate(g, P);
  const R iJ = invJ[P];
  const R nuP = nu_field ? nu[P] : nu[0];
  R Ad = dt_inv;
  R r[D];
#pragma unroll
  for (int i = 0; i < D; ++i) r[i] = u[(size_t)i * N + P] * dt_inv + S[(size_t)i * N + P];
  R gp[D];
#pragma unroll
  for (int i = 0; i < D; ++i) gp[i] = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const R UP = contra<R, D, DIAG>(JT, u, j, P, N);
    const R aP = alpha[(size_t)j * N + P];
    R pnb[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const R Nf = s ? R(1) : R(-1);
      const int F = neighbour(g, c, P, j, s);
      if (F >= 0) {
        const R phi = R(0.5) * (UP + contra<R, D, DIAG>(JT, u, j, F, N));
        const R nuF = nu_field ? nu[F] : nuP;
        const R knu = R(0.5) * (aP * nuP + alpha[(size_t)j * N + F] * nuF);
        Ad += (R(0.5) * Nf * phi + knu) * iJ;
        if (s) {
          C[(size_t)j * N + P] = (R(0.5) * phi - knu) * iJ;
          C[(size_t)(D + j) * N + P] = (R(-0.5) * phi - knu) * invJ[F];
        }
        if (nonorth) {
#pragma unroll
          for (int k = 0; k < D; ++k) {
            if (k == j) continue;
            const int ai = ax_index(j, k);
            const R w = R(0.5) * (alphax[(size_t)ai * N + P] * nuP + alphax[(size_t)ai * N + F] * nuF);
#pragma unroll
            for (int i = 0; i < D; ++i) {
              const R t = R(0.5) * (tgu[(size_t)(i * D + k) * N + P] + tgu[(size_t)(i * D + k) * N + F]);
              r[i] += Nf * w * t * iJ;
            }
          }
        }
        pnb[s] = p[F];
      } else {
        const int f = -1 - F;
        if (s) {
          C[(size_t)j * N + P] = R(0);
          C[(size_t)(D + j) * N + P] = R(0);
        }
        // the face's own metrics (App. A.4; the boundary cell's unless given)
        const R ab = balpha[(size_t)j * NB + f];
        Ad += R(2) * ab * nuP * iJ;
        R Ub = R(0);
#pragma unroll
        for (int i = 0; i < D; ++i) Ub += bjt[(size_t)i * NB + f] * ub[(size_t)i * NB + f];
        const R coef = (R(2) * ab * nuP - Nf * Ub) * iJ;
#pragma unroll
        for (int i = 0; i < D; ++i) r[i] += ub[(size_t)i * NB + f] * coef;
        if (nonorth) {
#pragma unroll
          for (int k = 0; k < D; ++k) {
            if (k == j) continue;
            const R w = balpha[(size_t)k * NB + f] * nuP;
#pragma unroll
            for (int i = 0; i < D; ++i) r[i] += Nf * w * bdiff<R>(g, c, P, j, s, k, f, ub + (size_t)i * NB) * iJ;
          }
        }
        pnb[s] = p[P];
      }
    }
    if (gradp) {
      const R dpj = R(0.5) * (pnb[1] - pnb[0]);
#pragma unroll
      for (int i = 0; i < D; ++i) gp[i] += jt<R, D, DIAG>(JT, j, i, P, N) * iJ * dpj;
    }
  }
  A[P] = Ad;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    bu[(size_t)i * N + P] = r[i];
    b[(size_t)i * N + P] = r[i] - gp[i];
  }
}

// Pressure matrix faces P_f = lerp(alpha_jj / A) (eq. pMatDiscrete) and the inverse of
// the diagonal of -P (Jacobi).
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_pcoef(Grid g, const R* __restrict__ alpha, const R* __restrict__ A, R* __restrict__ Pf, R* __restrict__ Dinv) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N;
  const Cell c = locate(g, P);
  const R iA = R(1) / A[P];
  R sum = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const R aP = alpha[(size_t)j * N + P] * iA;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int F = neighbour(g, c, P, j, s);
      R pf = R(0);
      if (F >= 0) {
        pf = R(0.5) * (aP + alpha[(size_t)j * N + F] / A[F]);
        sum += pf;
      }
      if (s) Pf[(size_t)j * N + P] = pf;
    }
  }
  Dinv[P] = sum > R(0) ? R(1) / sum : R(0);
}

// h = A^-1 (b_u - H u) (eq. pressureRHS) and W^j = J T_j . h.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_h(Grid g, const R* __restrict__ JT, const R* __restrict__ A, const R* __restrict__ C,
    const R* __restrict__ bu, const R* __restrict__ u, R* __restrict__ h, R* __restrict__ W) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N;
  const Cell c = locate(g, P);
  R acc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = bu[(size_t)i * N + P];
  // a face without a neighbour cell (a Dirichlet side, whose value is in bu) reads the
  // cell itself with coefficient 0: every load is unconditional, the term is zero
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int F0 = neighbour(g, c, P, j, 1), F1 = neighbour(g, c, P, j, 0);
    const int Fp = F0 >= 0 ? F0 : P, Fm = F1 >= 0 ? F1 : P;
    const R cpv = C[(size_t)j * N + P], cmv = C[(size_t)(D + j) * N + Fm];
    const R cp = F0 >= 0 ? cpv : R(0), cm = F1 >= 0 ? cmv : R(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      acc[i] -= cp * u[(size_t)i * N + Fp];
      acc[i] -= cm * u[(size_t)i * N + Fm];
    }
  }
  const R iA = R(1) / A[P];
  R hv[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    hv[i] = acc[i] * iA;
    h[(size_t)i * N + P] = hv[i];
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    R w = R(0);
#pragma unroll
    for (int i = 0; i < D; ++i) w += jt<R, D, DIAG>(JT, j, i, P, N) * hv[i];
    W[(size_t)j * N + P] = w;
  }
}

// rhs = sum_f N_f lerp(W^j)_f + sum_b N_b J T_j . u_b (eqs. pressureRHSdivDiscrete and the
// Dirichlet flux) - deferred cross flux of p_lag with kappa = 1/A (eq. pressureRHSnonOrtho);
// mean_out[0] receives mean(rhs).  OT is the output type (double in the MIXED form).
template <typename R, typename OT, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_div(Grid g, const R* __restrict__ bjt, const R* __restrict__ W, const R* __restrict__ ub,
      const R* __restrict__ A, const R* __restrict__ alphax, const R* __restrict__ tgp, int nonorth,
      OT* __restrict__ rhs, double* __restrict__ partials) {
  const int N = g.N, NB = g.NB;
  int beg, end;
  chunk_range(N, beg, end);
  double acc[1] = {0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    const Cell c = locate(g, P);
    OT r = OT(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const OT WP = (OT)W[(size_t)j * N + P];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const OT Nf = s ? OT(1) : OT(-1);
        const int F = neighbour(g, c, P, j, s);
        if (F >= 0) {
          r += Nf * OT(0.5) * (WP + (OT)W[(size_t)j * N + F]);
          if (nonorth) {
            const R iAP = R(1) / A[P], iAF = R(1) / A[F];
#pragma unroll
            for (int k = 0; k < D; ++k) {
              if (k == j) continue;
              const int ai = ax_index(j, k);
              const R w = R(0.5) * (alphax[(size_t)ai * N + P] * iAP + alphax[(size_t)ai * N + F] * iAF);
              const R t = R(0.5) * (tgp[(size_t)k * N + P] + tgp[(size_t)k * N + F]);
              r -= Nf * (OT)(w * t);
            }
          }
        } else {
          const int f = -1 - F;
          OT Ub = OT(0);
#pragma unroll
          for (int i = 0; i < D; ++i) Ub += (OT)bjt[(size_t)i * NB + f] * (OT)ub[(size_t)i * NB + f];
          r += Nf * Ub;
        }
      }
    }
    rhs[P] = r;
    acc[0] += (double)r;
  }
  write_partials<1>(acc, partials);
}

// Face-flux divergence of a corrected flux F ([d][N], the +j face of every cell as
// k_correct writes it) with the Dirichlet boundary fluxes (J T_j)_f . u_b (eq. divtheorem,
// N_f = +1 on high sides): the largest |sum_f N_f F_f| of the work-group's cells into
// partials.  A face across the -j side is the +j face of the neighbour.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_flux_div(Grid g, const R* __restrict__ bjt, const R* __restrict__ F, const R* __restrict__ ub,
           double* __restrict__ partials) {
  const int N = g.N, NB = g.NB;
  int beg, end;
  chunk_range(N, beg, end);
  double m = 0.0;
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) {
    const Cell c = locate(g, P);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const double Nf = sd ? 1.0 : -1.0;
        const int Fn = neighbour(g, c, P, j, sd);
        if (Fn >= 0) {
          s += Nf * (double)F[(size_t)j * N + (sd ? P : Fn)];
        } else {
          const int f = -1 - Fn;
          double Ub = 0.0;
#pragma unroll
          for (int i = 0; i < D; ++i) Ub += (double)bjt[(size_t)i * NB + f] * (double)ub[(size_t)i * NB + f];
          s += Nf * Ub;
        }
      }
    }
    m = fmax(m, fabs(s));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  __shared__ double wm[kWaves];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t = fmax(t, wm[w]);
    partials[blockIdx.x] = t;
  }
}

// One work-group: *out = the largest of G partials.
__global__ void __launch_bounds__(kWG) k_max_partials(const double* __restrict__ partials, int G, double* out) {
  double m = 0.0;
  for (int w = (int)threadIdx.x; w < G; w += kWG) m = fmax(m, partials[w]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  __shared__ double wm[kWaves];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t = fmax(t, wm[w]);
    *out = t;
  }
}

// One work-group: out[q] = scale * sum of the G partials of value q (q < nv <= 2).
__global__ void __launch_bounds__(kWG)
k_finalize(const double* __restrict__ partials, int G, int nv, double scale, double* __restrict__ out) {
  double t[2];
  if (nv == 1) {
    double t1[1];
    reduce_partials<1>(partials, G, t1);
    t[0] = t1[0];
    t[1] = 0.0;
  } else {
    reduce_partials<2>(partials, G, t);
  }
  if (threadIdx.x == 0) {
    out[0] = t[0] * scale;
    if (nv > 1) out[1] = t[1] * scale;
  }
}

// u = h - A^-1 grad p with (grad p)_i = sum_j T_ji (p_+ - p_-)/2, p_b = p_P (eq.
// velCorrDiscrete); optional corrected face flux of every +j face,
// lerp(J T_j . h) - P_f (p_F - p_P) - deferred cross flux of p_lag.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_correct(Grid g, const R* __restrict__ JT, const R* __restrict__ invJ, const R* __restrict__ A,
          const R* __restrict__ h, const R* __restrict__ p, const R* __restrict__ Pf,
          const R* __restrict__ alphax, const R* __restrict__ tgp, int nonorth, R* __restrict__ u,
          R* __restrict__ F_out) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N;
  const Cell c = locate(g, P);
  const R pP = p[P];
  const R iJ = invJ[P];
  R gp[D];
#pragma unroll
  for (int i = 0; i < D; ++i) gp[i] = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int Fp = neighbour(g, c, P, j, 1), Fm = neighbour(g, c, P, j, 0);
    const R pp = Fp >= 0 ? p[Fp] : pP;
    const R pm = Fm >= 0 ? p[Fm] : pP;
    const R dj = R(0.5) * (pp - pm) * iJ;
#pragma unroll
    for (int i = 0; i < D; ++i) gp[i] += jt<R, D, DIAG>(JT, j, i, P, N) * dj;
    if (F_out) {
      R fl = R(0);
      if (Fp >= 0) {
        const R WP = contra<R, D, DIAG>(JT, h, j, P, N);
        const R WF = contra<R, D, DIAG>(JT, h, j, Fp, N);
        fl = R(0.5) * (WP + WF) - Pf[(size_t)j * N + P] * (pp - pP);
        if (nonorth) {
          const R iAP = R(1) / A[P], iAF = R(1) / A[Fp];
#pragma unroll
          for (int k = 0; k < D; ++k) {
            if (k == j) continue;
            const int ai = ax_index(j, k);
            const R w = R(0.5) * (alphax[(size_t)ai * N + P] * iAP + alphax[(size_t)ai * N + Fp] * iAF);
            fl -= w * R(0.5) * (tgp[(size_t)k * N + P] + tgp[(size_t)k * N + Fp]);
          }
        }
      }
      F_out[(size_t)j * N + P] = fl;
    }
  }
  const R iA = R(1) / A[P];
#pragma unroll
  for (int i = 0; i < D; ++i) u[(size_t)i * N + P] = h[(size_t)i * N + P] - gp[i] * iA;
}

template <typename R>
__global__ void __launch_bounds__(kWG)
k_scale_invJ(int N, int ncomp, const R* __restrict__ invJ, const R* __restrict__ x, R* __restrict__ y) {
  const int P = cell_of_thread(N);
  if (P < 0) return;
  for (int q = 0; q < ncomp; ++q) y[(size_t)q * N + P] = x[(size_t)q * N + P] * invJ[P];
}

template <typename R>
__global__ void k_add_scalar(const double* __restrict__ v, R* __restrict__ y) {
  if (threadIdx.x == 0 && blockIdx.x == 0) y[0] += (R)v[0];
}

// y = 2 p - q (a linear extrapolation in time of the pressure initial guess)
template <typename R>
__global__ void __launch_bounds__(kWG) k_extrapolate(int n, const R* __restrict__ p, const R* __restrict__ q,
                                                    R* __restrict__ y) {
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = R(2) * p[i] - q[i];
}

// y = a + b - c
template <typename R>
__global__ void __launch_bounds__(kWG) k_add_diff(int n, const R* __restrict__ a, const R* __restrict__ b,
                                                 const R* __restrict__ q, R* __restrict__ y) {
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = a[i] + (b[i] - q[i]);
}

template <typename R>
__global__ void __launch_bounds__(kWG) k_fill(int n, R v, R* __restrict__ y) {
  const int i = blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = v;
}

// W^j = J T_j . S for a cell vector field S (the contravariant flux of eq. pressureRHS
// without the A^-1 (b_u - H u) part).
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_jt_field(int N, const R* __restrict__ JT, const R* __restrict__ S, R* __restrict__ W) {
  const int P = cell_of_thread(N);
  if (P < 0) return;
  R v[D];
#pragma unroll
  for (int i = 0; i < D; ++i) v[i] = S[(size_t)i * N + P];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    R w = R(0);
#pragma unroll
    for (int i = 0; i < D; ++i) w += jt<R, D, DIAG>(JT, j, i, P, N) * v[i];
    W[(size_t)j * N + P] = w;
  }
}

template <typename TI>
__global__ void __launch_bounds__(kWG)
k_sum(const TI* __restrict__ x, int n, double* __restrict__ partials) {
  int beg, end;
  chunk_range(n, beg, end);
  double acc[1] = {0.0};
  for (int P = beg + (int)threadIdx.x; P < end; P += kWG) acc[0] += (double)x[P];
  write_partials<1>(acc, partials);
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kWG)
k_sub_mean(const TI* __restrict__ x, const double* __restrict__ mean, TO* __restrict__ y, int n) {
  const int P = cell_of_thread(n);
  if (P < 0) return;
  y[P] = (TO)((double)x[P] - mean[0]);
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kWG) k_copy(const TI* __restrict__ x, TO* __restrict__ y, int n) {
  const int P = cell_of_thread(n);
  if (P < 0) return;
  y[P] = (TO)x[P];
}

// ------------------------------------------------------------------ host wrappers

#define PISO_DISPATCH_D_DIAG(ctx, KERNEL_CALL)           \
  do {                                                   \
    if ((ctx)->dim == 2) {                               \
      if ((ctx)->diagT) { constexpr int D = 2; constexpr bool DG = true; KERNEL_CALL; } \
      else { constexpr int D = 2; constexpr bool DG = false; KERNEL_CALL; }            \
    } else {                                             \
      if ((ctx)->diagT) { constexpr int D = 3; constexpr bool DG = true; KERNEL_CALL; } \
      else { constexpr int D = 3; constexpr bool DG = false; KERNEL_CALL; }            \
    }                                                    \
  } while (0)

static inline int check_launch(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

template <typename R>
int launch_tgrad(piso_ctx* c, hipStream_t s, const R* phi, int ncomp, R* out) {
  const int G = grid_cells(c->N);
  if (c->dim == 2) k_tgrad<R, 2><<<G, kWG, 0, s>>>(c->grid, phi, ncomp, out);
  else k_tgrad<R, 3><<<G, kWG, 0, s>>>(c->grid, phi, ncomp, out);
  return check_launch(c, "k_tgrad");
}

template <typename R>
int launch_assemble(piso_ctx* c, hipStream_t s, const R* u, const R* p, const R* nu, int nu_field,
                    const R* S, const R* ub, double dt, int gradp, R* A, R* C, R* bu, R* b) {
  const int G = grid_cells(c->N);
  const R* tgu = nullptr;
  if (c->nonorth) {
    int rc = launch_tgrad<R>(c, s, u, c->dim, (R*)c->w_tg);
    if (rc) return rc;
    tgu = (const R*)c->w_tg;
  }
  PISO_DISPATCH_D_DIAG(c, (k_assemble<R, D, DG><<<G, kWG, 0, s>>>(
                              c->grid, (const R*)c->JT, (const R*)c->invJ, (const R*)c->alpha,
                              (const R*)c->alphax, (const R*)c->bjt, (const R*)c->balpha, u, p, nu, nu_field, S,
                              ub, R(1.0 / dt), gradp, tgu,
                              c->nonorth ? 1 : 0, A, C, bu, b)));
  return check_launch(c, "k_assemble");
}

template <typename R>
int launch_pcoef(piso_ctx* c, hipStream_t s, const R* A, R* Pf, R* Dinv) {
  const int G = grid_cells(c->N);
  if (c->dim == 2) k_pcoef<R, 2><<<G, kWG, 0, s>>>(c->grid, (const R*)c->alpha, A, Pf, Dinv);
  else k_pcoef<R, 3><<<G, kWG, 0, s>>>(c->grid, (const R*)c->alpha, A, Pf, Dinv);
  return check_launch(c, "k_pcoef");
}

template <typename R>
int launch_h(piso_ctx* c, hipStream_t s, const R* A, const R* C, const R* bu, const R* u, R* h, R* W) {
  const int G = grid_cells(c->N);
  PISO_DISPATCH_D_DIAG(c, (k_h<R, D, DG><<<G, kWG, 0, s>>>(c->grid, (const R*)c->JT, A, C, bu, u, h, W)));
  return check_launch(c, "k_h");
}

template <typename R, typename OT>
int launch_div(piso_ctx* c, hipStream_t s, const R* W, const R* ub, const R* A, const R* p_lag,
               OT* rhs, double* mean_out) {
  const R* tgp = nullptr;
  if (c->nonorth) {
    int rc = launch_tgrad<R>(c, s, p_lag, 1, (R*)c->w_tgp);
    if (rc) return rc;
    tgp = (const R*)c->w_tgp;
  }
  const int G = grid_red(c->N);
  double* pt = part(c, kPartS);
  PISO_DISPATCH_D_DIAG(c, (k_div<R, OT, D, DG><<<G, kWG, 0, s>>>(
                              c->grid, (const R*)c->bjt, W, ub, A, (const R*)c->alphax, tgp,
                              c->nonorth ? 1 : 0, rhs, pt)));
  if (int rc = check_launch(c, "k_div")) return rc;
  k_finalize<<<1, kWG, 0, s>>>(pt, G, 1, 1.0 / c->N, mean_out);
  return check_launch(c, "k_finalize");
}

template <typename R>
int launch_correct(piso_ctx* c, hipStream_t s, const R* A, const R* h, const R* p, const R* Pf,
                   const R* p_lag, R* u_out, R* F_out) {
  const R* tgp = nullptr;
  if (c->nonorth && F_out) {
    int rc = launch_tgrad<R>(c, s, p_lag, 1, (R*)c->w_tgp);
    if (rc) return rc;
    tgp = (const R*)c->w_tgp;
  }
  const int G = grid_cells(c->N);
  PISO_DISPATCH_D_DIAG(c, (k_correct<R, D, DG><<<G, kWG, 0, s>>>(
                              c->grid, (const R*)c->JT, (const R*)c->invJ, A, h, p, Pf,
                              (const R*)c->alphax, tgp, (c->nonorth && F_out) ? 1 : 0, u_out, F_out)));
  return check_launch(c, "k_correct");
}

template <typename R>
int launch_flux_div(piso_ctx* c, hipStream_t s, const R* F, const R* ub, double* out) {
  const int G = grid_red(c->N);
  double* pt = part(c, kPartS);
  PISO_DISPATCH_D_DIAG(c, (k_flux_div<R, D, DG><<<G, kWG, 0, s>>>(c->grid, (const R*)c->bjt, F, ub, pt)));
  if (int rc = check_launch(c, "k_flux_div")) return rc;
  k_max_partials<<<1, kWG, 0, s>>>(pt, G, out);
  return check_launch(c, "k_max_partials");
}

template <typename R>
int launch_extrapolate(piso_ctx* c, hipStream_t s, const R* p, const R* q, R* y, int ncomp) {
  const int n = ncomp * c->N;
  k_extrapolate<R><<<grid_cells(n), kWG, 0, s>>>(n, p, q, y);
  return check_launch(c, "k_extrapolate");
}

template <typename R>
int launch_add_diff(piso_ctx* c, hipStream_t s, const R* a, const R* b, const R* q, R* y) {
  k_add_diff<R><<<grid_cells(c->N), kWG, 0, s>>>(c->N, a, b, q, y);
  return check_launch(c, "k_add_diff");
}

template <typename R>
int launch_scale_invJ(piso_ctx* c, hipStream_t s, const R* x, int ncomp, R* y) {
  k_scale_invJ<R><<<grid_cells(c->N), kWG, 0, s>>>(c->N, ncomp, (const R*)c->invJ, x, y);
  return check_launch(c, "k_scale_invJ");
}

template <typename R>
int launch_add_scalar(piso_ctx* c, hipStream_t s, const double* v, R* y) {
  k_add_scalar<R><<<1, 64, 0, s>>>(v, y);
  return check_launch(c, "k_add_scalar");
}

template <typename R>
int launch_fill(piso_ctx* c, hipStream_t s, int n, R v, R* y) {
  k_fill<R><<<grid_cells(n), kWG, 0, s>>>(n, v, y);
  return check_launch(c, "k_fill");
}

template <typename R>
int launch_jt_field(piso_ctx* c, hipStream_t s, const R* S, R* W) {
  const int G = grid_cells(c->N);
  PISO_DISPATCH_D_DIAG(c, (k_jt_field<R, D, DG><<<G, kWG, 0, s>>>(c->N, (const R*)c->JT, S, W)));
  return check_launch(c, "k_jt_field");
}

template <typename TI, typename TO>
int launch_sum(piso_ctx* c, hipStream_t s, const TI* x, int n, double scale, double* out) {
  const int G = grid_red(n);
  double* pt = part(c, kPartS);
  k_sum<TI><<<G, kWG, 0, s>>>(x, n, pt);
  if (int rc = check_launch(c, "k_sum")) return rc;
  k_finalize<<<1, kWG, 0, s>>>(pt, G, 1, scale, out);
  return check_launch(c, "k_finalize");
}

template <typename TI, typename TO>
int launch_sub_mean(piso_ctx* c, hipStream_t s, const TI* x, const double* mean, TO* y, int n) {
  k_sub_mean<TI, TO><<<grid_cells(n), kWG, 0, s>>>(x, mean, y, n);
  return check_launch(c, "k_sub_mean");
}

template <typename TI, typename TO>
int launch_copy(piso_ctx* c, hipStream_t s, const TI* x, TO* y, int n) {
  k_copy<TI, TO><<<grid_cells(n), kWG, 0, s>>>(x, y, n);
  return check_launch(c, "k_copy");
}

#define PISO_INST_FWD(R)                                                                              \
  template int launch_tgrad<R>(piso_ctx*, hipStream_t, const R*, int, R*);                           \
  template int launch_assemble<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, int, const R*, \
                                  const R*, double, int, R*, R*, R*, R*);                            \
  template int launch_pcoef<R>(piso_ctx*, hipStream_t, const R*, R*, R*);                            \
  template int launch_h<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, const R*, R*, R*);  \
  template int launch_correct<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, const R*,     \
                                 const R*, R*, R*);                                                  \
  template int launch_scale_invJ<R>(piso_ctx*, hipStream_t, const R*, int, R*);                      \
  template int launch_flux_div<R>(piso_ctx*, hipStream_t, const R*, const R*, double*);                      \
  template int launch_extrapolate<R>(piso_ctx*, hipStream_t, const R*, const R*, R*, int);                 \
  template int launch_add_diff<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, R*);               \
  template int launch_add_scalar<R>(piso_ctx*, hipStream_t, const double*, R*);                       \
  template int launch_fill<R>(piso_ctx*, hipStream_t, int, R, R*);                                    \
  template int launch_jt_field<R>(piso_ctx*, hipStream_t, const R*, R*);

PISO_INST_FWD(float)
PISO_INST_FWD(double)
template int launch_div<float, float>(piso_ctx*, hipStream_t, const float*, const float*, const float*,
                                      const float*, float*, double*);
template int launch_div<float, double>(piso_ctx*, hipStream_t, const float*, const float*, const float*,
                                       const float*, double*, double*);
template int launch_div<double, double>(piso_ctx*, hipStream_t, const double*, const double*,
                                        const double*, const double*, double*, double*);
template int launch_sum<float, double>(piso_ctx*, hipStream_t, const float*, int, double, double*);
template int launch_sum<double, double>(piso_ctx*, hipStream_t, const double*, int, double, double*);
template int launch_sub_mean<float, float>(piso_ctx*, hipStream_t, const float*, const double*, float*, int);
template int launch_sub_mean<double, double>(piso_ctx*, hipStream_t, const double*, const double*, double*, int);
template int launch_sub_mean<double, float>(piso_ctx*, hipStream_t, const double*, const double*, float*, int);
template int launch_copy<float, double>(piso_ctx*, hipStream_t, const float*, double*, int);
template int launch_copy<double, float>(piso_ctx*, hipStream_t, const double*, float*, int);
template int launch_copy<float, float>(piso_ctx*, hipStream_t, const float*, float*, int);
template int launch_copy<double, double>(piso_ctx*, hipStream_t, const double*, double*, int);

}  // namespace piso
