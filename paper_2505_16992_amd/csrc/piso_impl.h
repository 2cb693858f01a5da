// Host-side internals of the PISO library: the context and the launch wrappers that
// the C-ABI layer (piso_api.hip) composes.  Kernels live in piso_fwd.hip,
// piso_krylov.hip and piso_bwd.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/piso.h"
#include "piso_common.h"

namespace piso {

// Solver scalars live on the device.  Values produced at iteration k go to slot k & 1
// so that a kernel never overwrites a slot that other work-groups of the same launch
// still read.
struct CgState {
  double rz[2];
  double rr, bb, tol2, pad0;
  int done, iters, status, zero_rhs;
};

struct BiState {
  double rho[2][3], alpha[2][3], omega[2][3];
  double rr[3], bb[3], tol2, pad0;
  int done[3], iters[3], status[3], all_done;
};

// Partial-sum regions inside piso_ctx::partials, each [NV][kRedGrid] doubles.
constexpr int kPartA = 0;        // CG: d.q                        (1)
constexpr int kPartB = 1;        // CG: r.z, r.r (+ b.b at init)  (3)
constexpr int kPart1 = 4;        // BiCGStab: rh.v                 (3)
constexpr int kPart2 = 7;        // BiCGStab: t.s, t.t             (6)
constexpr int kPart3 = 13;       // BiCGStab: rh.r, r.r (+ b.b)    (9)
constexpr int kPartS = 22;       // one-shot sums                  (2)
constexpr int kPartRegions = 24;

struct Timing {
  bool enabled = false;
  double spmv_ms = 0.0, update_ms = 0.0;
  long long spmv_calls = 0, update_calls = 0;
  std::vector<hipEvent_t> ev;   // pool: pairs around each timed launch
  size_t used = 0;
};

}  // namespace piso

struct piso_ctx {
  int dim = 0, nblocks = 0, N = 0, NB = 0, prec = 0, device = 0;
  size_t esz = 8;                 // element bytes of the working precision
  bool diagT = false, nonorth = false;
  bool quad = false;              // every block has nx % 4 == 0: vectorised CG kernels
  piso::Grid grid{};
  int* d_tab = nullptr;
  int* d_fmap = nullptr;
  std::vector<int> h_tab, h_fmap;
  // metrics in working precision
  void* JT = nullptr;     // [d*d][N], or [d][N] (J T_jj) when T is diagonal
  void* invJ = nullptr;   // [N]
  void* alpha = nullptr;  // [d][N] alpha_jj
  void* alphax = nullptr; // [d(d-1)/2][N] alpha_jk (j < k), non-orthogonal grids only
  // workspaces, working precision unless noted
  void *w_A = nullptr, *w_C = nullptr, *w_bu = nullptr, *w_b = nullptr, *w_Pf = nullptr,
       *w_Dinv = nullptr, *w_h = nullptr, *w_W = nullptr, *w_rhs = nullptr, *w_us = nullptr,
       *w_u1 = nullptr, *w_p1 = nullptr, *w_h1 = nullptr;
  void* w_tg = nullptr;           // [d*d][N] tangential gradients (non-orthogonal)
  void* w_tgp = nullptr;          // [d][N]
  double* w_rhs64 = nullptr;      // [N] (MIXED)
  double* w_p64 = nullptr;        // [N] (MIXED)
  void *m_r32 = nullptr, *m_e32 = nullptr;   // float [N] (MIXED refinement)
  void *k_r = nullptr, *k_q = nullptr, *k_d0 = nullptr, *k_d1 = nullptr;   // PCG [N]
  void *b_r = nullptr, *b_rh = nullptr, *b_p0 = nullptr, *b_p1 = nullptr, *b_v0 = nullptr,
       *b_v1 = nullptr, *b_s = nullptr, *b_t = nullptr;                    // BiCGStab [d][N]
  // adjoint workspaces
  void *a_g = nullptr, *a_uin = nullptr, *a_lam = nullptr, *a_pbar = nullptr, *a_mu = nullptr,
       *a_dh = nullptr, *a_dA = nullptr, *a_dC = nullptr, *a_dbu = nullptr, *a_db = nullptr,
       *a_dp1 = nullptr, *a_dnu = nullptr, *a_ybar = nullptr, *a_cbar = nullptr;
  // reductions and solver state
  double* partials = nullptr;      // [kPartRegions * kRedGrid]
  double* mean = nullptr;          // [4] device scalars
  piso::CgState* cg = nullptr;
  piso::BiState* bi = nullptr;
  piso::CgState* h_cg = nullptr;   // pinned mirrors
  piso::BiState* h_bi = nullptr;
  double* h_scal = nullptr;        // pinned [8]
  int red_grid = 512;              // work-groups of the reduction kernels
  std::vector<void*> allocs;
  piso::Timing timing;
  std::string err;
};

namespace piso {

inline int fail(piso_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define PISO_HIP(ctx, expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::piso::fail((ctx), PISO_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

inline int grid_cells(int N) { return (N + kWG - 1) / kWG; }
inline int grid_red(int N, int cap = 512) {
  int g = (N + kWG - 1) / kWG;
  if (cap > kRedGrid) cap = kRedGrid;
  return g < cap ? (g < 1 ? 1 : g) : cap;
}
inline double* part(piso_ctx* c, int region) { return c->partials + (size_t)region * kRedGrid; }

// ---- forward launch wrappers (piso_fwd.hip) ----
template <typename R>
int launch_tgrad(piso_ctx* c, hipStream_t s, const R* phi, int ncomp, R* out);
template <typename R>
int launch_assemble(piso_ctx* c, hipStream_t s, const R* u, const R* p, const R* nu, int nu_field,
                    const R* S, const R* ub, double dt, int gradp, R* A, R* C, R* bu, R* b);
template <typename R>
int launch_pcoef(piso_ctx* c, hipStream_t s, const R* A, R* Pf, R* Dinv);
template <typename R>
int launch_h(piso_ctx* c, hipStream_t s, const R* A, const R* C, const R* bu, const R* u, R* h, R* W);
template <typename R, typename OT>
int launch_div(piso_ctx* c, hipStream_t s, const R* W, const R* ub, const R* A, const R* p_lag,
               OT* rhs, double* mean_out);
template <typename R>
int launch_correct(piso_ctx* c, hipStream_t s, const R* A, const R* h, const R* p, const R* Pf,
                   const R* p_lag, R* u_out, R* F_out);
template <typename R>
int launch_scale_invJ(piso_ctx* c, hipStream_t s, const R* x, int ncomp, R* y);
template <typename R>
int launch_add_scalar(piso_ctx* c, hipStream_t s, const double* v, R* y);
template <typename TI, typename TO>
int launch_sum(piso_ctx* c, hipStream_t s, const TI* x, int n, double scale, double* out);
template <typename TI, typename TO>
int launch_sub_mean(piso_ctx* c, hipStream_t s, const TI* x, const double* mean, TO* y, int n);
template <typename TI, typename TO>
int launch_copy(piso_ctx* c, hipStream_t s, const TI* x, TO* y, int n);

// ---- Krylov solvers (piso_krylov.hip) ----
// Zero-mean solution of P x = rhs - mean: rhs of type BT, mean a device scalar or null.
template <typename R, typename BT>
int pressure_solve(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const BT* rhs,
                   const double* mean, R* x, const piso_solve_opts* o, piso_solve_info* info);
// MIXED form: double residual of (Pf float) with rhs64, refinement of the double x64.
int pressure_solve_mixed(piso_ctx* c, hipStream_t s, const float* Pf, const float* Dinv,
                         const double* rhs64, const double* mean, double* x64,
                         const piso_solve_opts* o, piso_solve_info* info);
template <typename R>
int velocity_solve(piso_ctx* c, hipStream_t s, bool trans, const R* A, const R* C, const R* b, R* x,
                   const piso_solve_opts* o, piso_solve_info* info);

// ---- adjoint launch wrappers (piso_bwd.hip) ----
template <typename R>
int launch_correct_bwd(piso_ctx* c, hipStream_t s, const R* A, const R* p, const R* du, R* dp, R* dA);
template <typename R>
int launch_pface_bwd(piso_ctx* c, hipStream_t s, const R* A, const R* lam, const R* p, R* dA);
template <typename R>
int launch_h_bwd(piso_ctx* c, hipStream_t s, const R* A, const R* h, const R* du_h, const R* lam,
                 R* g, R* dbu, R* dA, R* dub);
template <typename R>
int launch_outer_bwd(piso_ctx* c, hipStream_t s, const R* C, const R* g, const R* u, R* du_in, R* dC,
                     R* dAdiag);
template <typename R>
int launch_gradT(piso_ctx* c, hipStream_t s, const R* g, const R* A, R scale, R* dp);
template <typename R>
int launch_cross_bwd(piso_ctx* c, hipStream_t s, const R* kappa, int kappa_field, int kappa_inverse,
                     const R* ybar, int ncomp, const R* phi_tg, R scale, R* phibar, R* kbar);
template <typename R>
int launch_bcross_bwd(piso_ctx* c, hipStream_t s, const R* nu, int nu_field, const R* ub, const R* dbu,
                      R* dnu_cell, R* dub);
template <typename R>
int launch_assemble_bwd(piso_ctx* c, hipStream_t s, const R* u, const R* nu, int nu_field,
                        const R* ub, double dt, const R* dA, const R* dC, const R* dbu, R* du,
                        R* dS, R* dnu_cell, R* dub);
template <typename R>
int launch_axpy(piso_ctx* c, hipStream_t s, int n, R a, const R* x, R* y);

}  // namespace piso
