// Adjoint kernels of the PISO step (arXiv 2505.16992, App. A.5, Sec. 2.3).  Each
// kernel is the exact transpose of its forward counterpart in piso_fwd.hip, written as
// a per-cell gather (no float atomics, deterministic).  Gradients accumulate (+=).
#include "piso_impl.h"

namespace piso {

template <typename R, int D, bool DIAG>
__device__ __forceinline__ R jtb(const R* __restrict__ JT, int j, int i, int P, int N) {
  if (DIAG) return j == i ? JT[(size_t)j * N + P] : R(0);
  return JT[(size_t)(j * D + i) * N + P];
}

__device__ __forceinline__ int ax_idx(int j, int k) { return (j < k ? j : k) + (j < k ? k : j) - 1; }

// s_j(X) = sum_i T_ji(X) g_i(X) [/ A(X)]: the computational-gradient adjoint at a cell.
template <typename R, int D, bool DIAG>
__device__ __forceinline__ R sgrad(const R* __restrict__ JT, const R* __restrict__ invJ,
                                   const R* __restrict__ A, const R* __restrict__ gv, int j, int X, int N) {
  R s = R(0);
#pragma unroll
  for (int i = 0; i < D; ++i) s += jtb<R, D, DIAG>(JT, j, i, X, N) * gv[(size_t)i * N + X];
  s *= invJ[X];
  if (A) s /= A[X];
  return s;
}

// dp += scale * G^T (g [/ A]) with G the central gradient of the correction (boundary
// value p_b = p_P): the adjoint of eq. velCorrDiscrete's gradient (App. A.5.1).
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_gradT(Grid g, const R* __restrict__ JT, const R* __restrict__ invJ, const R* __restrict__ gv,
        const R* __restrict__ A, R scale, R* __restrict__ dp) {
  const int Q = cell_of_thread(g.N);
  if (Q < 0) return;
  const int N = g.N;
  const Cell c = locate(g, Q);
  R acc = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int Fp = neighbour(g, c, Q, j, 1), Fm = neighbour(g, c, Q, j, 0);
    if (Fm >= 0) acc += R(0.5) * sgrad<R, D, DIAG>(JT, invJ, A, gv, j, Fm, N);
    else acc -= R(0.5) * sgrad<R, D, DIAG>(JT, invJ, A, gv, j, Q, N);
    if (Fp >= 0) acc -= R(0.5) * sgrad<R, D, DIAG>(JT, invJ, A, gv, j, Fp, N);
    else acc += R(0.5) * sgrad<R, D, DIAG>(JT, invJ, A, gv, j, Q, N);
  }
  dp[Q] += scale * acc;
}

// dA += (grad p) . du / A^2 (eq. diff:velcorr_grad_advdiag).
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_correct_bwd(Grid g, const R* __restrict__ JT, const R* __restrict__ invJ, const R* __restrict__ A,
              const R* __restrict__ p, const R* __restrict__ du, R* __restrict__ dA) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N;
  const Cell c = locate(g, P);
  const R pP = p[P], iJ = invJ[P];
  R acc = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int Fp = neighbour(g, c, P, j, 1), Fm = neighbour(g, c, P, j, 0);
    const R dj = R(0.5) * ((Fp >= 0 ? p[Fp] : pP) - (Fm >= 0 ? p[Fm] : pP)) * iJ;
#pragma unroll
    for (int i = 0; i < D; ++i) acc += jtb<R, D, DIAG>(JT, j, i, P, N) * dj * du[(size_t)i * N + P];
  }
  const R iA = R(1) / A[P];
  dA[P] += acc * iA * iA;
}

// dA_P += sum_f (lam_P - lam_F)(p_P - p_F) (-alpha_jj,P / (2 A_P^2)): the pressure-solve
// matrix gradient dP = -lam (x) p mapped through P_f = lerp(alpha_jj / A).
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_pface_bwd(Grid g, const R* __restrict__ alpha, const R* __restrict__ A, const R* __restrict__ lam,
            const R* __restrict__ p, R* __restrict__ dA) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N;
  const Cell c = locate(g, P);
  const R iA = R(1) / A[P];
  R acc = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    R sj = R(0);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int F = neighbour(g, c, P, j, s);
      if (F >= 0) sj += (lam[P] - lam[F]) * (p[P] - p[F]);
    }
    acc += sj * alpha[(size_t)j * N + P];
  }
  dA[P] += R(-0.5) * acc * iA * iA;
}

// Adjoint of h = A^-1 (b_u - H u) and rhs = div(lerp J T h) + Dirichlet flux
// (eqs. diff:divpressurerhs_grad_pressurerhs, diff:pressurerhs_grad_*): with lam the
// gradient of rhs, hbar = dh + (J T)^T Wbar, g = hbar / A; db_u += g;
// dA += -hbar . h / A; du_b += N J T_j . lam at Dirichlet faces.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_h_bwd(Grid g, const R* __restrict__ JT, const R* __restrict__ bjt, const R* __restrict__ A,
        const R* __restrict__ h, const R* __restrict__ dh, const R* __restrict__ lam, R* __restrict__ gout,
        R* __restrict__ dbu, R* __restrict__ dA, R* __restrict__ dub) {
  const int X = cell_of_thread(g.N);
  if (X < 0) return;
  const int N = g.N, NB = g.NB;
  const Cell c = locate(g, X);
  R Wb[D];
#pragma unroll
  for (int j = 0; j < D; ++j) Wb[j] = R(0);
  if (lam) {
    const R lX = lam[X];
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int F = neighbour(g, c, X, j, s);
        if (F >= 0) {
          Wb[j] += s ? R(0.5) * (lX - lam[F]) : R(0.5) * (lam[F] - lX);
        } else if (dub) {
          const int f = -1 - F;
          const R Nf = s ? R(1) : R(-1);
#pragma unroll
          for (int i = 0; i < D; ++i) dub[(size_t)i * NB + f] += Nf * bjt[(size_t)i * NB + f] * lX;
        }
      }
    }
  }
  const R iA = R(1) / A[X];
  R dAx = R(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    R hb = dh ? dh[(size_t)i * N + X] : R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) hb += jtb<R, D, DIAG>(JT, j, i, X, N) * Wb[j];
    const R gi = hb * iA;
    gout[(size_t)i * N + X] = gi;
    dbu[(size_t)i * N + X] += gi;
    dAx -= hb * h[(size_t)i * N + X];
  }
  dA[X] += dAx * iA;
}

// du_in += -H^T g (eq. diff:pressurerhs_grad_velguess); dC += -g (x) u on the off-diagonal
// stencil (eq. diff:pressurerhs_grad_advndiag, and dA = -db (x) x of a solve); if dAdiag,
// also dA += -g . u (the diagonal of a solve's matrix gradient).
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_outer_bwd(Grid g, const R* __restrict__ C, const R* __restrict__ gv, const R* __restrict__ u,
            R* __restrict__ du_in, R* __restrict__ dC, R* __restrict__ dAdiag) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N;
  const Cell c = locate(g, P);
  R acc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int Fp = neighbour(g, c, P, j, 1), Fm = neighbour(g, c, P, j, 0);
    if (Fp >= 0) {
      const R cf = C[(size_t)(D + j) * N + P];   // C(P+j, P)
      R s0 = R(0), s1 = R(0);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const R gF = gv[(size_t)i * N + Fp];
        acc[i] += cf * gF;
        s0 += gv[(size_t)i * N + P] * u[(size_t)i * N + Fp];
        s1 += gF * u[(size_t)i * N + P];
      }
      dC[(size_t)j * N + P] -= s0;
      dC[(size_t)(D + j) * N + P] -= s1;
    }
    if (Fm >= 0) {
      const R cp = C[(size_t)j * N + Fm];         // C(P-j, P)
#pragma unroll
      for (int i = 0; i < D; ++i) acc[i] += cp * gv[(size_t)i * N + Fm];
    }
  }
  if (du_in) {
#pragma unroll
    for (int i = 0; i < D; ++i) du_in[(size_t)i * N + P] -= acc[i];
  }
  if (dAdiag) {
    R s = R(0);
#pragma unroll
    for (int i = 0; i < D; ++i) s += gv[(size_t)i * N + P] * u[(size_t)i * N + P];
    dAdiag[P] -= s;
  }
}

// Adjoint of the deferred cross operator y = K(kappa) phi (App. A.3.5), pass 1: for each
// cell X and axis k, cbar_k(X) = sum over X's faces along j != k of
// (1/2) w_f (ybar_low - ybar_high) with w_f = lerp(alpha_jk kappa); and
// kbar_X += sum_f sum_k (1/2) alpha_jk,X t_k,f (ybar_low - ybar_high), t from the
// forward tangential gradients of phi.  kappa = 1/A if kappa_inverse.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_cross_bwd_a(Grid g, const R* __restrict__ alphax, const R* __restrict__ kap, int kap_field, int kap_inv,
              const R* __restrict__ ybar, int ncomp, const R* __restrict__ phi_tg, R scale,
              R* __restrict__ cbar, R* __restrict__ kbar) {
  const int X = cell_of_thread(g.N);
  if (X < 0) return;
  const int N = g.N;
  const Cell c = locate(g, X);
  auto kv = [&](int Y) {
    const R v = kap_field ? kap[Y] : kap[0];
    return kap_inv ? R(1) / v : v;
  };
  const R kX = kv(X);
  R kb = R(0);
  for (int q = 0; q < ncomp; ++q) {
    const R* yq = ybar + (size_t)q * N;
    R cb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) cb[k] = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int F = neighbour(g, c, X, j, s);
        if (F < 0) continue;
        const R dy = s ? (yq[X] - yq[F]) : (yq[F] - yq[X]);
        const R kF = kv(F);
#pragma unroll
        for (int k = 0; k < D; ++k) {
          if (k == j) continue;
          const int ai = ax_idx(j, k);
          const R aX = alphax[(size_t)ai * N + X];
          const R w = R(0.5) * (aX * kX + alphax[(size_t)ai * N + F] * kF);
          cb[k] += R(0.5) * w * dy;
          if (kbar && phi_tg) {
            const R t = R(0.5) * (phi_tg[(size_t)(q * D + k) * N + X] + phi_tg[(size_t)(q * D + k) * N + F]);
            kb += R(0.5) * aX * t * dy;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) cbar[(size_t)(q * D + k) * N + X] = cb[k];
  }
  if (kbar) {
    if (kap_inv) kbar[X] += scale * kb * (-kX * kX);   // d(1/A)/dA = -1/A^2
    else kbar[X] += scale * kb;
  }
}

// Pass 2: phibar += Gt^T cbar, the transpose of the one-sided-aware tangential difference.
template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_cross_bwd_b(Grid g, const R* __restrict__ cbar, int ncomp, R scale, R* __restrict__ phibar) {
  const int Q = cell_of_thread(g.N);
  if (Q < 0) return;
  const int N = g.N;
  const Cell c = locate(g, Q);
  for (int q = 0; q < ncomp; ++q) {
    R acc = R(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const R* cb = cbar + (size_t)(q * D + k) * N;
      const int Fp = neighbour(g, c, Q, k, 1), Fm = neighbour(g, c, Q, k, 0);
      if (Fp < 0 && Fm >= 0) acc += cb[Q];
      if (Fm < 0 && Fp >= 0) acc -= cb[Q];
      if (Fm >= 0) {   // Q is the +k neighbour of Fm
        const bool both = neighbour_of(g, Fm, k, 0) >= 0;
        acc += (both ? R(0.5) : R(1)) * cb[Fm];
      }
      if (Fp >= 0) {   // Q is the -k neighbour of Fp
        const bool both = neighbour_of(g, Fp, k, 1) >= 0;
        acc -= (both ? R(0.5) : R(1)) * cb[Fp];
      }
    }
    phibar[(size_t)q * N + Q] += scale * acc;
  }
}

// Boundary part of the deferred velocity cross terms: v = N alpha_jk nu_P bdiff_k(u_b) / J
// at each Dirichlet face.  Accumulates dnu_cell (per cell) and, as a gather over the
// faces whose tangential differences involve a given face, du_b.
template <typename R, int D>
__device__ __forceinline__ R bcoef(const Grid& g, int P, int j, int s, int k, int f_target) {
  // coefficient of u_b[f_target] in bdiff_k of the (j, s) face of cell P
  const Cell c = locate(g, P);
  const int own = -1 - neighbour(g, c, P, j, s);
  int fp = -1, fm = -1;
  const int Qp = neighbour(g, c, P, k, 1), Qm = neighbour(g, c, P, k, 0);
  if (Qp >= 0) {
    const int e = neighbour_of(g, Qp, j, s);
    if (e < 0) fp = -1 - e;
  }
  if (Qm >= 0) {
    const int e = neighbour_of(g, Qm, j, s);
    if (e < 0) fm = -1 - e;
  }
  R cf = R(0);
  if (fp >= 0 && fm >= 0) {
    if (f_target == fp) cf += R(0.5);
    if (f_target == fm) cf -= R(0.5);
  } else if (fp >= 0) {
    if (f_target == fp) cf += R(1);
    if (f_target == own) cf -= R(1);
  } else if (fm >= 0) {
    if (f_target == own) cf += R(1);
    if (f_target == fm) cf -= R(1);
  }
  return cf;
}

template <typename R, int D>
__global__ void __launch_bounds__(kWG)
k_bcross_bwd(Grid g, const R* __restrict__ balpha, const R* __restrict__ invJ, const R* __restrict__ nu,
             int nu_field, const R* __restrict__ ub, const R* __restrict__ dbu, R* __restrict__ dnu_cell,
             R* __restrict__ dub) {
  const int P = cell_of_thread(g.N);
  if (P < 0) return;
  const int N = g.N, NB = g.NB;
  const Cell c = locate(g, P);
  const R nuP = nu_field ? nu[P] : nu[0];
#pragma unroll
  for (int j = 0; j < D; ++j) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int e = neighbour(g, c, P, j, s);
      if (e >= 0) continue;
      const int f = -1 - e;
      const R Nf = s ? R(1) : R(-1);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if (k == j) continue;
        // nu gradient: sum_i N alpha bdiff_k(u_b,i) dbu_i(P) / J_P (alpha of the face)
        if (dnu_cell) {
          R acc = R(0);
#pragma unroll
          for (int i = 0; i < D; ++i) {
            // bdiff via coefficients of the faces it touches
            const int Qp = neighbour(g, c, P, k, 1), Qm = neighbour(g, c, P, k, 0);
            R bd = R(0);
            int fp = -1, fm = -1;
            if (Qp >= 0) { const int ee = neighbour_of(g, Qp, j, s); if (ee < 0) fp = -1 - ee; }
            if (Qm >= 0) { const int ee = neighbour_of(g, Qm, j, s); if (ee < 0) fm = -1 - ee; }
            const R* uc = ub + (size_t)i * NB;
            if (fp >= 0 && fm >= 0) bd = R(0.5) * (uc[fp] - uc[fm]);
            else if (fp >= 0) bd = uc[fp] - uc[f];
            else if (fm >= 0) bd = uc[f] - uc[fm];
            acc += bd * dbu[(size_t)i * N + P];
          }
          dnu_cell[P] += Nf * balpha[(size_t)k * NB + f] * acc * invJ[P];
        }
        // u_b gradient of the faces entering this face's difference: gather for face f
        if (dub) {
          // contributions to u_b[f] from the differences taken at f itself and at the
          // same-side faces of P's k-neighbours
          int cells[3] = {P, neighbour(g, c, P, k, 1), neighbour(g, c, P, k, 0)};
          if (cells[1] == P) cells[1] = -1;
          if (cells[2] == P || cells[2] == cells[1]) cells[2] = -1;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const int Y = cells[q];
            if (Y < 0) continue;
            const int ey = neighbour_of(g, Y, j, s);
            if (ey >= 0) continue;
            const R cf = bcoef<R, D>(g, Y, j, s, k, f);
            if (cf == R(0)) continue;
            const R nuY = nu_field ? nu[Y] : nu[0];
            const R w = Nf * balpha[(size_t)k * NB + (-1 - ey)] * nuY * invJ[Y] * cf;
#pragma unroll
            for (int i = 0; i < D; ++i) dub[(size_t)i * NB + f] += w * dbu[(size_t)i * N + Y];
          }
        }
      }
    }
  }
  (void)nuP;
}

// Adjoint of the predictor assembly (eqs. diff:advmat_grad_vel, diff:advmat_grad_visc,
// diff:advrhs_grad_*): from dA, dC (face arrays), db_u: du += db_u/dt + (J T)^T Ubar,
// dS += db_u, dnu_cell += face and boundary terms, du_b += boundary terms.
template <typename R, int D, bool DIAG>
__global__ void __launch_bounds__(kWG)
k_assemble_bwd(Grid g, const R* __restrict__ JT, const R* __restrict__ invJ, const R* __restrict__ alpha,
               const R* __restrict__ bjt, const R* __restrict__ balpha, const R* __restrict__ nu, int nu_field,
               const R* __restrict__ ub, R dt_inv,
               const R* __restrict__ dA, const R* __restrict__ dC, const R* __restrict__ dbu,
               R* __restrict__ du, R* __restrict__ dS, R* __restrict__ dnu_cell, R* __restrict__ dub) {
  const int X = cell_of_thread(g.N);
  if (X < 0) return;
  const int N = g.N, NB = g.NB;
  const Cell c = locate(g, X);
  const R iJX = invJ[X];
  const R nuX = nu_field ? nu[X] : nu[0];
  R Ub[D];
  R dnu = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    Ub[j] = R(0);
    const R aX = alpha[(size_t)j * N + X];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int F = neighbour(g, c, X, j, s);
      if (F >= 0) {
        const int P = s ? X : F;       // low cell of the face
        const int H = s ? F : X;       // high cell
        const R dcP = dC[(size_t)j * N + P], dcF = dC[(size_t)(D + j) * N + P];
        const R iJP = invJ[P], iJH = invJ[H];
        const R phib = R(0.5) * (dcP * iJP - dcF * iJH + dA[P] * iJP - dA[H] * iJH);
        const R kb = -dcP * iJP - dcF * iJH + dA[P] * iJP + dA[H] * iJH;
        Ub[j] += R(0.5) * phib;
        dnu += R(0.5) * aX * kb;
      } else {
        const int f = -1 - F;
        const R Nf = s ? R(1) : R(-1);
        const R ab = balpha[(size_t)j * NB + f];   // the face's own metrics
        dnu += R(2) * ab * dA[X] * iJX;
        R ubv[D], Ubd = R(0), dot = R(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
          ubv[i] = ub[(size_t)i * NB + f];
          Ubd += bjt[(size_t)i * NB + f] * ubv[i];
          dot += dbu[(size_t)i * N + X] * ubv[i];
        }
        dnu += dot * R(2) * ab * iJX;
        if (dub) {
          const R coef = (R(2) * ab * nuX - Nf * Ubd) * iJX;
#pragma unroll
          for (int i = 0; i < D; ++i)
            dub[(size_t)i * NB + f] += dbu[(size_t)i * N + X] * coef - Nf * bjt[(size_t)i * NB + f] * iJX * dot;
        }
      }
    }
  }
  if (du) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      R v = dbu[(size_t)i * N + X] * dt_inv;
#pragma unroll
      for (int j = 0; j < D; ++j) v += jtb<R, D, DIAG>(JT, j, i, X, N) * Ub[j];
      du[(size_t)i * N + X] += v;
    }
  }
  if (dS) {
#pragma unroll
    for (int i = 0; i < D; ++i) dS[(size_t)i * N + X] += dbu[(size_t)i * N + X];
  }
  if (dnu_cell) dnu_cell[X] += dnu;
}

template <typename R>
__global__ void __launch_bounds__(kWG) k_axpy(int n, R a, const R* __restrict__ x, R* __restrict__ y) {
  const int P = cell_of_thread(n);
  if (P < 0) return;
  y[P] += a * x[P];
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

static inline int check_b(piso_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PISO_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return PISO_OK;
}

template <typename R>
int launch_correct_bwd(piso_ctx* c, hipStream_t s, const R* A, const R* p, const R* du, R* dp, R* dA) {
  const int G = grid_cells(c->N);
  if (dA) {
    PISO_DISPATCH_D_DIAG(c, (k_correct_bwd<R, D, DG><<<G, kWG, 0, s>>>(c->grid, (const R*)c->JT,
                                                                          (const R*)c->invJ, A, p, du, dA)));
    if (int rc = check_b(c, "k_correct_bwd")) return rc;
  }
  if (dp) {
    PISO_DISPATCH_D_DIAG(c, (k_gradT<R, D, DG><<<G, kWG, 0, s>>>(c->grid, (const R*)c->JT, (const R*)c->invJ,
                                                                    du, A, R(-1), dp)));
    if (int rc = check_b(c, "k_gradT")) return rc;
  }
  return PISO_OK;
}

template <typename R>
int launch_gradT(piso_ctx* c, hipStream_t s, const R* gv, const R* A, R scale, R* dp) {
  const int G = grid_cells(c->N);
  PISO_DISPATCH_D_DIAG(c, (k_gradT<R, D, DG><<<G, kWG, 0, s>>>(c->grid, (const R*)c->JT, (const R*)c->invJ,
                                                                  gv, A, scale, dp)));
  return check_b(c, "k_gradT");
}

template <typename R>
int launch_pface_bwd(piso_ctx* c, hipStream_t s, const R* A, const R* lam, const R* p, R* dA) {
  const int G = grid_cells(c->N);
  if (c->dim == 2) k_pface_bwd<R, 2><<<G, kWG, 0, s>>>(c->grid, (const R*)c->alpha, A, lam, p, dA);
  else k_pface_bwd<R, 3><<<G, kWG, 0, s>>>(c->grid, (const R*)c->alpha, A, lam, p, dA);
  return check_b(c, "k_pface_bwd");
}

template <typename R>
int launch_h_bwd(piso_ctx* c, hipStream_t s, const R* A, const R* h, const R* du_h, const R* lam,
                 R* gout, R* dbu, R* dA, R* dub) {
  const int G = grid_cells(c->N);
  PISO_DISPATCH_D_DIAG(c, (k_h_bwd<R, D, DG><<<G, kWG, 0, s>>>(c->grid, (const R*)c->JT, (const R*)c->bjt, A, h,
                                                                  du_h, lam, gout, dbu, dA, dub)));
  return check_b(c, "k_h_bwd");
}

template <typename R>
int launch_outer_bwd(piso_ctx* c, hipStream_t s, const R* C, const R* gv, const R* u, R* du_in, R* dC,
                     R* dAdiag) {
  const int G = grid_cells(c->N);
  if (c->dim == 2) k_outer_bwd<R, 2><<<G, kWG, 0, s>>>(c->grid, C, gv, u, du_in, dC, dAdiag);
  else k_outer_bwd<R, 3><<<G, kWG, 0, s>>>(c->grid, C, gv, u, du_in, dC, dAdiag);
  return check_b(c, "k_outer_bwd");
}

// phibar += scale K(kappa)^T ybar and kbar += d<ybar, K phi>/d kappa (phi_tg: forward
// tangential gradients of phi, [ncomp][d][N], or NULL to skip kbar).
template <typename R>
int launch_cross_bwd(piso_ctx* c, hipStream_t s, const R* kap, int kap_field, int kap_inv, const R* ybar,
                     int ncomp, const R* phi_tg, R scale, R* phibar, R* kbar) {
  const int G = grid_cells(c->N);
  R* cbar = (R*)c->a_cbar;
  if (c->dim == 2)
    k_cross_bwd_a<R, 2><<<G, kWG, 0, s>>>(c->grid, (const R*)c->alphax, kap, kap_field, kap_inv, ybar, ncomp,
                                          phi_tg, scale, cbar, kbar);
  else
    k_cross_bwd_a<R, 3><<<G, kWG, 0, s>>>(c->grid, (const R*)c->alphax, kap, kap_field, kap_inv, ybar, ncomp,
                                          phi_tg, scale, cbar, kbar);
  if (int rc = check_b(c, "k_cross_bwd_a")) return rc;
  if (phibar) {
    if (c->dim == 2) k_cross_bwd_b<R, 2><<<G, kWG, 0, s>>>(c->grid, cbar, ncomp, scale, phibar);
    else k_cross_bwd_b<R, 3><<<G, kWG, 0, s>>>(c->grid, cbar, ncomp, scale, phibar);
    if (int rc = check_b(c, "k_cross_bwd_b")) return rc;
  }
  return PISO_OK;
}

template <typename R>
int launch_bcross_bwd(piso_ctx* c, hipStream_t s, const R* nu, int nu_field, const R* ub, const R* dbu,
                      R* dnu_cell, R* dub) {
  const int G = grid_cells(c->N);
  if (c->dim == 2)
    k_bcross_bwd<R, 2><<<G, kWG, 0, s>>>(c->grid, (const R*)c->balpha, (const R*)c->invJ, nu, nu_field, ub, dbu,
                                         dnu_cell, dub);
  else
    k_bcross_bwd<R, 3><<<G, kWG, 0, s>>>(c->grid, (const R*)c->balpha, (const R*)c->invJ, nu, nu_field, ub, dbu,
                                         dnu_cell, dub);
  return check_b(c, "k_bcross_bwd");
}

template <typename R>
int launch_assemble_bwd(piso_ctx* c, hipStream_t s, const R* u, const R* nu, int nu_field, const R* ub,
                        double dt, const R* dA, const R* dC, const R* dbu, R* du, R* dS, R* dnu_cell, R* dub) {
  const int G = grid_cells(c->N);
  PISO_DISPATCH_D_DIAG(c, (k_assemble_bwd<R, D, DG><<<G, kWG, 0, s>>>(
                              c->grid, (const R*)c->JT, (const R*)c->invJ, (const R*)c->alpha, (const R*)c->bjt,
                              (const R*)c->balpha, nu, nu_field, ub, R(1.0 / dt), dA, dC, dbu, du, dS, dnu_cell,
                              dub)));
  (void)u;
  return check_b(c, "k_assemble_bwd");
}

template <typename R>
int launch_axpy(piso_ctx* c, hipStream_t s, int n, R a, const R* x, R* y) {
  k_axpy<R><<<grid_cells(n), kWG, 0, s>>>(n, a, x, y);
  return check_b(c, "k_axpy");
}

#define PISO_INST_BWD(R)                                                                                   \
  template int launch_correct_bwd<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, R*, R*);         \
  template int launch_gradT<R>(piso_ctx*, hipStream_t, const R*, const R*, R, R*);                          \
  template int launch_pface_bwd<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, R*);               \
  template int launch_h_bwd<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, const R*, R*, R*, R*,   \
                               R*);                                                                         \
  template int launch_outer_bwd<R>(piso_ctx*, hipStream_t, const R*, const R*, const R*, R*, R*, R*);        \
  template int launch_cross_bwd<R>(piso_ctx*, hipStream_t, const R*, int, int, const R*, int, const R*, R,  \
                                   R*, R*);                                                                 \
  template int launch_bcross_bwd<R>(piso_ctx*, hipStream_t, const R*, int, const R*, const R*, R*, R*);     \
  template int launch_assemble_bwd<R>(piso_ctx*, hipStream_t, const R*, const R*, int, const R*, double,    \
                                      const R*, const R*, const R*, R*, R*, R*, R*);                        \
  template int launch_axpy<R>(piso_ctx*, hipStream_t, int, R, const R*, R*);

PISO_INST_BWD(float)
PISO_INST_BWD(double)

}  // namespace piso
