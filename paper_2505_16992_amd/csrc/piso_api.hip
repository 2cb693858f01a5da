// C-ABI of the PISO library (include/piso.h): context creation with topology
// validation (Sec. 2.2, App. A.4 of arXiv 2505.16992), the fine-grained forward and
// backward calls, and the orchestration of one step (App. A.2) and of its adjoint
// (Sec. 2.3, App. A.5).
#include <algorithm>
#include <array>
#include <climits>
#include <type_traits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "piso_impl.h"

using namespace piso;

static std::string g_create_error;

namespace {

template <typename R>
std::vector<R> convert(const std::vector<double>& v) {
  return std::vector<R>(v.begin(), v.end());
}

template <typename R>
int upload_metrics(piso_ctx* c, const piso_domain_desc* d) {
  const int D = c->dim, N = c->N;
  const double* T = d->T;
  const double* J = d->J;
  bool diag = true;
  for (int j = 0; j < D && diag; ++j)
    for (int i = 0; i < D && diag; ++i)
      if (i != j)
        for (int P = 0; P < N; ++P)
          if (T[(size_t)(j * D + i) * N + P] != 0.0) { diag = false; break; }
  c->diagT = diag;
  std::vector<double> jt((size_t)(diag ? D : D * D) * N), invJ(N), al((size_t)D * N);
  std::vector<double> alx((size_t)(D == 3 ? 3 : 1) * N, 0.0);
  double nonorth = 0.0;
  for (int P = 0; P < N; ++P) {
    if (!(J[P] > 0.0) || !std::isfinite(J[P]))
      return fail(c, PISO_E_TOPOLOGY, "non-positive or non-finite Jacobian at cell " + std::to_string(P));
    invJ[P] = 1.0 / J[P];
    for (int j = 0; j < D; ++j) {
      for (int i = 0; i < D; ++i) {
        const double v = J[P] * T[(size_t)(j * D + i) * N + P];
        if (diag) { if (i == j) jt[(size_t)j * N + P] = v; }
        else jt[(size_t)(j * D + i) * N + P] = v;
      }
    }
    double a[3][3];
    for (int j = 0; j < D; ++j)
      for (int k = 0; k < D; ++k) {
        double s = 0.0;
        for (int i = 0; i < D; ++i) s += T[(size_t)(j * D + i) * N + P] * T[(size_t)(k * D + i) * N + P];
        a[j][k] = J[P] * s;
      }
    double mind = a[0][0];
    for (int j = 0; j < D; ++j) {
      al[(size_t)j * N + P] = a[j][j];
      mind = std::min(mind, std::fabs(a[j][j]));
    }
    for (int j = 0; j < D; ++j)
      for (int k = j + 1; k < D; ++k) {
        alx[(size_t)(j + k - 1) * N + P] = a[j][k];
        nonorth = std::max(nonorth, std::fabs(a[j][k]) / mind);
      }
  }
  // metrics of the Dirichlet faces: given on the faces, or the boundary cell's (then the
  // same numbers as the cell arrays above, so results do not change)
  const int NB = c->NB;
  std::vector<double> bjt((size_t)D * std::max(NB, 1), 0.0), bal((size_t)D * std::max(NB, 1), 0.0);
  if (NB > 0) {
    std::vector<int> bcell, bside;
    if (int rc = bface_cells(c, bcell, bside)) return rc;
    for (int f = 0; f < NB; ++f) {
      const int P = bcell[f], j = bside[f] / 2;
      const double* Tf = d->Tb ? d->Tb + f : T + P;
      const size_t st = d->Tb ? (size_t)NB : (size_t)N;
      const double Jf = d->Tb ? d->Jb[f] : J[P];
      for (int i = 0; i < D; ++i) bjt[(size_t)i * NB + f] = Jf * Tf[(size_t)(j * D + i) * st];
      double mind = 0.0, mx = 0.0;
      for (int k = 0; k < D; ++k) {
        double sm = 0.0;
        for (int i = 0; i < D; ++i) sm += Tf[(size_t)(j * D + i) * st] * Tf[(size_t)(k * D + i) * st];
        bal[(size_t)k * NB + f] = Jf * sm;
        if (k == j) mind = std::fabs(Jf * sm);
        else mx = std::max(mx, std::fabs(Jf * sm));
      }
      if (d->Tb && !(Jf > 0.0 && std::isfinite(Jf)))
        return fail(c, PISO_E_ARG, "face metrics: Jb of Dirichlet face " + std::to_string(f) + " not positive");
      if (!(mind > 0.0) || !std::isfinite(mind) || !std::isfinite(mx))
        return fail(c, PISO_E_ARG, "face metrics: alpha_jj of Dirichlet face " + std::to_string(f) + " not positive");
      nonorth = std::max(nonorth, mx / mind);   // cross terms of the face metrics count too
    }
  }
  c->nonorth = nonorth > 1e-12;
  if (int rc = upload(c, &c->bjt, convert<R>(bjt))) return rc;
  if (int rc = upload(c, &c->balpha, convert<R>(bal))) return rc;
  if (int rc = upload(c, &c->JT, convert<R>(jt))) return rc;
  if (int rc = upload(c, &c->invJ, convert<R>(invJ))) return rc;
  if (int rc = upload(c, &c->alpha, convert<R>(al))) return rc;
  if (c->nonorth) {
    if (int rc = upload(c, &c->alphax, convert<R>(alx))) return rc;
  } else {
    if (int rc = dev_alloc(c, &c->alphax, sizeof(R))) return rc;
  }
  return PISO_OK;
}

int alloc_workspaces(piso_ctx* c) {
  const size_t N = c->N, D = c->dim, e = c->esz;
  const size_t mx = c->prec == PISO_MIXED ? 1 : 0;   // the MIXED refinement buffers
  struct { void** p; size_t bytes; } L[] = {
      {&c->w_A, N * e}, {&c->w_C, 2 * D * N * e}, {&c->w_bu, D * N * e}, {&c->w_b, D * N * e},
      {&c->w_Pf, D * N * e}, {&c->w_Dinv, N * e}, {&c->w_h, D * N * e}, {&c->w_W, D * N * e},
      {&c->w_rhs, N * 8}, {&c->w_us, D * N * e}, {&c->w_u1, D * N * e}, {&c->w_p1, N * e},
      {&c->w_h1, D * N * e}, {&c->w_tg, D * D * N * e}, {&c->w_tgp, D * N * e},
      {&c->m_r32, mx * D * N * 4}, {&c->m_e32, mx * D * N * 4}, {&c->x_Pf32, mx * D * N * 4},
      {&c->x_Dinv32, mx * N * 4}, {&c->x_A32, mx * N * 4}, {&c->x_C32, mx * 2 * D * N * 4},
      {(void**)&c->mix_scal, 8 * sizeof(double)},
      {(void**)&c->plane_work, 2 * (size_t)std::max({c->h_tab[1], c->h_tab[2], c->h_tab[3]}) * sizeof(double)},
      {&c->k_r, N * e}, {&c->k_r2, N * e}, {&c->k_q, N * e}, {&c->k_d0, N * e}, {&c->k_d1, N * e},
      {&c->g_Pf, D * N * e}, {&c->g_Dinv, N * e}, {&c->g_x, N * e},
      {&c->b_r, D * N * e}, {&c->b_rh, D * N * e}, {&c->b_p0, D * N * e}, {&c->b_p1, D * N * e},
      {&c->b_v0, D * N * e}, {&c->b_v1, D * N * e}, {&c->b_s, D * N * e}, {&c->b_t, D * N * e},
      {&c->b_iA, N * e}, {&c->b_ph, D * N * e}, {&c->b_sh, D * N * e}, {&c->b_sinv, N * e},
      {&c->a_g, D * N * e}, {&c->a_uin, D * N * e}, {&c->a_lam, N * e}, {&c->a_pbar, N * e},
      {&c->a_mu, D * N * e}, {&c->a_dh, D * N * e}, {&c->a_dA, N * e}, {&c->a_dC, 2 * D * N * e},
      {&c->a_dbu, D * N * e}, {&c->a_db, D * N * e}, {&c->a_dp1, N * e}, {&c->a_dnu, N * e},
      {&c->a_ybar, D * N * e}, {&c->a_cbar, D * D * N * e}, {&c->a_lam_hist[0], N * 8}, {&c->a_lam_hist[1], N * 8},
      {&c->a_lam_hist2[0], N * 8}, {&c->a_lam_hist2[1], N * 8}, {&c->w_zb, D * (size_t)std::max(c->NB, 1) * e},
      {(void**)&c->partials, (size_t)kPartRegions * kRedGrid * sizeof(double)},
      {(void**)&c->mean, 8 * sizeof(double)}, {(void**)&c->cg, sizeof(CgState)}, {(void**)&c->bi, sizeof(BiState)},
  };
  for (auto& l : L)
    if (int rc = dev_alloc(c, l.p, l.bytes)) return rc;
  PISO_HIP(c, hipMemset(c->w_zb, 0, D * (size_t)std::max(c->NB, 1) * e));
  PISO_HIP(c, hipMemset(c->cg, 0, sizeof(CgState)));
  PISO_HIP(c, hipMemset(c->bi, 0, sizeof(BiState)));
  PISO_HIP(c, hipMemset(c->partials, 0, (size_t)kPartRegions * kRedGrid * sizeof(double)));
  PISO_HIP(c, hipHostMalloc((void**)&c->h_cg, sizeof(CgState), hipHostMallocDefault));
  PISO_HIP(c, hipHostMalloc((void**)&c->h_bi, sizeof(BiState), hipHostMallocDefault));
  PISO_HIP(c, hipHostMalloc((void**)&c->h_scal, 8 * sizeof(double), hipHostMallocDefault));
  return PISO_OK;
}

size_t tape_elems(const piso_ctx* c) { return (size_t)(4 + 7 * c->dim) * c->N; }

template <typename R>
struct Tape {
  R *A, *C, *Pf, *Dinv, *us, *h1, *p1, *u1, *h2, *p2;
  Tape(void* base, int N, int D) {
    R* t = (R*)base;
    const size_t n = N;
    A = t;
    C = A + n;
    Pf = C + 2 * D * n;
    Dinv = Pf + D * n;
    us = Dinv + n;
    h1 = us + D * n;
    p1 = h1 + D * n;
    u1 = p1 + n;
    h2 = u1 + D * n;
    p2 = h2 + D * n;
  }
};

int check_ctx(piso_ctx* c) {
  if (!c) return PISO_E_ARG;
  return PISO_OK;
}

#define REQUIRE(cond, msg) \
  do { if (!(cond)) return fail(c, PISO_E_ARG, msg); } while (0)

// ---------------------------------------------------------------- forward pieces

template <typename R>
int do_assemble(piso_ctx* c, hipStream_t s, const R* u, const R* p, const R* nu, int nu_field, const R* S,
                const R* ub, double dt, int gradp, R* A, R* C, R* bu, R* b, R* Pf, R* Dinv) {
  if (int rc = launch_assemble<R>(c, s, u, p, nu, nu_field, S, ub, dt, gradp, A, C, bu, b)) return rc;
  return launch_pcoef<R>(c, s, A, Pf, Dinv);
}

// h, rhs and the pressure solve of one corrector.  p holds x0 on entry.
template <typename R>
int do_pressure(piso_ctx* c, hipStream_t s, const R* A, const R* C, const R* bu, const R* Pf, const R* Dinv,
                const R* u_in, const R* ub, const R* p_lag, R* h, R* rhs_out, R* p, const piso_solve_opts* o,
                piso_solve_info* info) {
  R* W = (R*)c->w_W;
  if (int rc = launch_h<R>(c, s, A, C, bu, u_in, h, W)) return rc;
  R* rhs = rhs_out ? rhs_out : (R*)c->w_rhs;
  if (int rc = launch_div<R, R>(c, s, W, ub, A, p_lag, rhs, c->mean)) return rc;
  return pressure_solve<R, R>(c, s, Pf, Dinv, rhs, c->mean, p, o, info);
}

// Zero-mean lambda of P lambda = g - mean(g) (pressure adjoint).  x0 = 0, or with
// hist = 0 / 1 the kept solution of that corrector's previous adjoint solve when there is
// one, or 2 lambda_prev - lambda_prev2 when the two previous ones are kept; a solve that
// ends with status >= 0 is kept for the next calls.
template <typename R>
int do_pressure_adjoint(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* g, R* lam,
                        const piso_solve_opts* o, piso_solve_info* info, int hist = -1) {
  const int N = c->N;
  const bool warm = hist >= 0 && c->lam_hist_valid[hist];
  piso_solve_info tmp{};
  piso_solve_info* inf = info ? info : &tmp;
  if (int rc = launch_sum<R, double>(c, s, g, N, 1.0 / N, c->mean)) return rc;
  if (warm && c->lam_hist_valid2[hist]) {
    // two earlier solutions of this corrector's adjoint: start from their linear
    // extrapolation (consecutive backward steps walk back through time)
    if (int e = launch_extrapolate<R>(c, s, (const R*)c->a_lam_hist[hist], (const R*)c->a_lam_hist2[hist], lam))
      return e;
  } else if (warm) {
    PISO_HIP(c, hipMemcpyAsync(lam, c->a_lam_hist[hist], sizeof(R) * N, hipMemcpyDeviceToDevice, s));
  } else {
    PISO_HIP(c, hipMemsetAsync(lam, 0, sizeof(R) * N, s));
  }
  const int rc = pressure_solve<R, R>(c, s, Pf, Dinv, g, c->mean, lam, o, inf);
  if (rc < 0) return rc;
  if (hist >= 0 && inf->status >= 0) {
    if (c->lam_hist_valid[hist]) {
      PISO_HIP(c, hipMemcpyAsync(c->a_lam_hist2[hist], c->a_lam_hist[hist], sizeof(R) * N, hipMemcpyDeviceToDevice, s));
      c->lam_hist_valid2[hist] = true;
    }
    PISO_HIP(c, hipMemcpyAsync(c->a_lam_hist[hist], lam, sizeof(R) * N, hipMemcpyDeviceToDevice, s));
    c->lam_hist_valid[hist] = true;
  }
  return rc;
}

// Divergence-free gradient modification (eq. SgradPsgrad): p_S from P(A = 1) p_S =
// div lerp(J T . S) (no Dirichlet flux, zero lagged pressure, x0 = 0), then
// g_out = gS + lambda grad p_S, computed as the correction h - A^-1 grad p with h = gS
// and A = -1 / lambda.
template <typename R>
int do_divfree(piso_ctx* c, hipStream_t s, const R* S, const R* gS, double lam, const piso_solve_opts* o,
               R* g_out, R* p_out, piso_solve_info* info) {
  const int N = c->N;
  R* A = (R*)c->w_A;
  R* Pf = (R*)c->w_Pf;
  R* Dinv = (R*)c->w_Dinv;
  R* W = (R*)c->w_W;
  R* p = p_out ? p_out : (R*)c->a_lam;
  R* plag = (R*)c->w_p1;
  const R* zb = (const R*)c->w_zb;
  if (int rc = launch_fill<R>(c, s, N, R(1), A)) return rc;
  if (int rc = launch_pcoef<R>(c, s, A, Pf, Dinv)) return rc;
  if (int rc = launch_jt_field<R>(c, s, S, W)) return rc;
  PISO_HIP(c, hipMemsetAsync(plag, 0, sizeof(R) * N, s));
  PISO_HIP(c, hipMemsetAsync(p, 0, sizeof(R) * N, s));
  if (int rc = launch_div<R, R>(c, s, W, zb, A, plag, (R*)c->w_rhs, c->mean)) return rc;
  if (int rc = pressure_solve<R, R>(c, s, Pf, Dinv, (const R*)c->w_rhs, c->mean, p, o, info)) return rc;
  if (lam == 0.0) return launch_copy<R, R>(c, s, gS, g_out, c->dim * N);
  if (int rc = launch_fill<R>(c, s, N, (R)(-1.0 / lam), A)) return rc;
  return launch_correct<R>(c, s, A, gS, p, Pf, nullptr, g_out, nullptr);
}

template <typename R>
int do_step(piso_ctx* c, hipStream_t s, const R* u_n, const R* p_n, const R* nu, int nu_field, const R* S,
            const R* ub, double dt, R* u_np1, R* p_np1, void* tape, const piso_step_opts* o, piso_step_info* info) {
  const int N = c->N, D = c->dim;
  R *A, *C, *Pf, *Dinv, *us, *h1, *p1, *u1, *h2, *p2;
  if (tape) {
    Tape<R> t(tape, N, D);
    A = t.A; C = t.C; Pf = t.Pf; Dinv = t.Dinv; us = t.us; h1 = t.h1; p1 = t.p1; u1 = t.u1; h2 = t.h2; p2 = t.p2;
  } else {
    A = (R*)c->w_A; C = (R*)c->w_C; Pf = (R*)c->w_Pf; Dinv = (R*)c->w_Dinv; us = (R*)c->w_us;
    h1 = (R*)c->w_h1; p1 = (R*)c->w_p1; u1 = (R*)c->w_u1; h2 = (R*)c->w_h; p2 = p_np1;
  }
  R* bu = (R*)c->w_bu;
  R* b = (R*)c->w_b;
  if (int rc = do_assemble<R>(c, s, u_n, p_n, nu, nu_field, S, ub, dt, o->grad_p_in_predictor, A, C, bu, b, Pf, Dinv))
    return rc;
  if (o->u_prev) {
    // the velocity solve starts from u extrapolated in time, 2 u_n - u_{n-1}
    if (int e = launch_extrapolate<R>(c, s, u_n, (const R*)o->u_prev, us, D)) return e;
  } else {
    PISO_HIP(c, hipMemcpyAsync(us, u_n, sizeof(R) * D * N, hipMemcpyDeviceToDevice, s));
  }
  piso_solve_info vi{}, pi[2]{};
  int rc = velocity_solve<R>(c, s, false, A, C, b, us, &o->vel, &vi);
  if (rc < 0) return rc;
  const int ncorr = o->n_correctors;
  const R* u_in = us;
  const R* p_lag = p_n;
  // the face flux of a corrector for its divergence goes to the predictor's right-hand side
  // buffer, which nothing reads after the velocity solve
  const bool fdiv = info && o->report_flux_div;
  R* Fbuf = fdiv ? (R*)c->w_b : nullptr;
  for (int k = 0; k < ncorr; ++k) {
    // the last corrector writes the outputs; earlier ones use the u**, h*, p* slots, and
    // correctors between the first and the last alternate their pressure between a spare
    // buffer (the adjoint's, unused here) and p1, so that p_lag is never overwritten
    // before the right-hand side has read it
    const bool last = (k == ncorr - 1);
    R* h = last ? h2 : h1;
    R* pk = last ? p2 : (k == 0 ? p1 : ((k & 1) ? (R*)c->a_pbar : p1));
    R* uk = last ? u_np1 : u1;
    // starts of the solves from the earlier steps of the rollout: corrector 1 from the
    // previous p* advanced by the last change of p, or from p extrapolated in time;
    // corrector 2 from p* advanced by the previous step's corrector-2 increment
    const R* pv = (const R*)o->p_prev;
    const R* pvs = (const R*)o->p_prev_star;
    if (k == 0 && pv && pvs) {
      if (int e = launch_add_diff<R>(c, s, pvs, p_n, pv, pk)) return e;
    } else if (k == 0 && pv) {
      if (int e = launch_extrapolate<R>(c, s, p_n, pv, pk)) return e;
    } else if (k == 1 && pvs) {
      if (int e = launch_add_diff<R>(c, s, p_lag, p_n, pvs, pk)) return e;
    } else if (pk != p_lag) {
      PISO_HIP(c, hipMemcpyAsync(pk, p_lag, sizeof(R) * N, hipMemcpyDeviceToDevice, s));
    }
    c->pcg_kind = kPcgFwd1 + std::min(k, 1);
    c->pcg_same_op = k > 0;   // the correctors of a step share P_f and D^-1
    rc = do_pressure<R>(c, s, A, C, bu, Pf, Dinv, u_in, ub, p_lag, h, nullptr, pk, &o->pres, &pi[std::min(k, 1)]);
    c->pcg_kind = kPcgOther;
    c->pcg_same_op = false;
    if (rc < 0) return rc;
    rc = launch_correct<R>(c, s, A, h, pk, Pf, p_lag, uk, Fbuf);
    if (rc) return rc;
    if (fdiv && (k == 0 || last)) {
      rc = launch_flux_div<R>(c, s, Fbuf, ub, c->mix_scal + 6 + (last ? 1 : 0));
      if (rc) return rc;
    }
    if (k == 0 && o->p_star_out && o->p_star_out != (void*)pk)   // p* for the next step's start
      PISO_HIP(c, hipMemcpyAsync(o->p_star_out, pk, sizeof(R) * N, hipMemcpyDeviceToDevice, s));
    u_in = uk;
    p_lag = pk;
  }
  if (p2 != p_np1) PISO_HIP(c, hipMemcpyAsync(p_np1, p2, sizeof(R) * N, hipMemcpyDeviceToDevice, s));
  if (info) {
    info->vel = vi;
    info->pres[0] = pi[0];
    info->pres[1] = pi[1];
    info->flux_div_linf[0] = info->flux_div_linf[1] = 0.0;
    if (fdiv) {
      PISO_HIP(c, hipMemcpyAsync(c->h_scal + 6, c->mix_scal + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      PISO_HIP(c, hipStreamSynchronize(s));
      info->flux_div_linf[0] = c->h_scal[6];
      info->flux_div_linf[1] = c->h_scal[7];
    }
  }
  int st = vi.status;
  for (int k = 0; k < 2; ++k) st = (pi[k].status < 0 || st < 0) ? std::min(st, pi[k].status) : std::max(st, pi[k].status);
  return st;
}

// ---------------------------------------------------------------- adjoint pieces

// Adjoint of one corrector (correct after h/rhs/solve).  du_c: gradient of the
// corrector output u; pbar: gradient of its p (modified in place: receives -G^T du/A).
// Accumulates dA, dC, dbu, dub; writes du_in_out (+= -H^T g) and p_lag_bar (+=).
template <typename R>
int do_corrector_bwd(piso_ctx* c, hipStream_t s, const R* A, const R* C, const R* Pf, const R* Dinv,
                     const R* h, const R* u_in, const R* p_lag, const R* p, const R* du_c, R* pbar,
                     R* du_in_out, R* p_lag_bar, R* dA, R* dC, R* dbu, R* dub, bool skip_solve,
                     const piso_solve_opts* o, piso_solve_info* info, int hist) {
  if (int rc = launch_correct_bwd<R>(c, s, A, p, du_c, pbar, dA)) return rc;
  R* lam = nullptr;
  if (!skip_solve) {
    lam = (R*)c->a_lam;
    int rc = do_pressure_adjoint<R>(c, s, Pf, Dinv, pbar, lam, o, info, hist);
    if (rc < 0) return rc;
    if ((rc = launch_pface_bwd<R>(c, s, A, lam, p, dA))) return rc;
  } else if (info) {
    *info = piso_solve_info{};
  }
  R* gv = (R*)c->a_g;
  if (int rc = launch_h_bwd<R>(c, s, A, h, du_c, lam, gv, dbu, dA, dub)) return rc;
  if (c->nonorth && lam && p_lag_bar) {
    if (int rc = launch_tgrad<R>(c, s, p_lag, 1, (R*)c->w_tgp)) return rc;
    if (int rc = launch_cross_bwd<R>(c, s, A, 1, 1, lam, 1, (const R*)c->w_tgp, R(-1), p_lag_bar, dA)) return rc;
  }
  return launch_outer_bwd<R>(c, s, C, gv, u_in, du_in_out, dC, nullptr);
}

// Adjoint of the predictor right-hand side and assembly, given dA, dC, dbu (which
// already holds db = mu and the h contributions) and the p^n gradient of -grad p^n.
template <typename R>
int do_assemble_bwd(piso_ctx* c, hipStream_t s, const R* u_n, const R* nu, int nu_field, const R* ub, double dt,
                    const R* dA, const R* dC, const R* dbu, R* du_n, R* dS, R* dnu, R* dub) {
  const int N = c->N, D = c->dim;
  R* dnu_cell = dnu ? (R*)c->a_dnu : nullptr;
  if (dnu_cell) PISO_HIP(c, hipMemsetAsync(dnu_cell, 0, sizeof(R) * N, s));
  if (int rc = launch_assemble_bwd<R>(c, s, u_n, nu, nu_field, ub, dt, dA, dC, dbu, du_n, dS, dnu_cell, dub)) return rc;
  if (c->nonorth) {
    R* ybar = (R*)c->a_ybar;
    if (int rc = launch_scale_invJ<R>(c, s, dbu, D, ybar)) return rc;
    if (int rc = launch_tgrad<R>(c, s, u_n, D, (R*)c->w_tg)) return rc;
    if (int rc = launch_cross_bwd<R>(c, s, nu, nu_field, 0, ybar, D, (const R*)c->w_tg, R(1), du_n, dnu_cell)) return rc;
    if (c->NB && (dnu_cell || dub))
      if (int rc = launch_bcross_bwd<R>(c, s, nu, nu_field, ub, dbu, dnu_cell, dub)) return rc;
  }
  if (dnu) {
    if (nu_field) return launch_axpy<R>(c, s, N, R(1), dnu_cell, dnu);
    if (int rc = launch_sum<R, double>(c, s, dnu_cell, N, 1.0, c->mean + 3)) return rc;
    return launch_add_scalar<R>(c, s, c->mean + 3, dnu);
  }
  return PISO_OK;
}

template <typename R>
int do_step_backward(piso_ctx* c, hipStream_t s, const void* tape, const R* u_n, const R* p_n, const R* nu,
                     int nu_field, const R* ub, double dt, const R* du_np1, const R* dp_np1, R* du_n, R* dp_n,
                     R* dS, R* dnu, R* dub, const piso_step_opts* o, piso_step_info* info) {
  const int N = c->N, D = c->dim;
  if (o->n_correctors != 2) return fail(c, PISO_E_ARG, "backward supports n_correctors = 2");
  Tape<R> t(const_cast<void*>(tape), N, D);
  R* dA = (R*)c->a_dA;
  R* dC = (R*)c->a_dC;
  R* dbu = (R*)c->a_dbu;
  R* pbar = (R*)c->a_pbar;
  R* dp1 = (R*)c->a_dp1;
  R* uin = (R*)c->a_uin;
  R* duc = (R*)c->a_dh;
  PISO_HIP(c, hipMemsetAsync(dA, 0, sizeof(R) * N, s));
  PISO_HIP(c, hipMemsetAsync(dC, 0, sizeof(R) * 2 * D * N, s));
  PISO_HIP(c, hipMemsetAsync(dbu, 0, sizeof(R) * D * N, s));
  PISO_HIP(c, hipMemsetAsync(dp1, 0, sizeof(R) * N, s));
  if (du_np1) PISO_HIP(c, hipMemcpyAsync(duc, du_np1, sizeof(R) * D * N, hipMemcpyDeviceToDevice, s));
  else PISO_HIP(c, hipMemsetAsync(duc, 0, sizeof(R) * D * N, s));
  if (dp_np1) PISO_HIP(c, hipMemcpyAsync(pbar, dp_np1, sizeof(R) * N, hipMemcpyDeviceToDevice, s));
  else PISO_HIP(c, hipMemsetAsync(pbar, 0, sizeof(R) * N, s));
  const bool skipP = (o->grad_path_flags & 2) != 0, skipV = (o->grad_path_flags & 1) != 0;
  piso_solve_info pi[2]{}, vi{};
  // corrector 2: output u***, p**; inputs u**, lag p*
  PISO_HIP(c, hipMemsetAsync(uin, 0, sizeof(R) * D * N, s));
  const int warm = o->adjoint_warm_start ? 1 : 0;
  c->pcg_kind = kPcgAdj1 + 1;
  int rc = do_corrector_bwd<R>(c, s, t.A, t.C, t.Pf, t.Dinv, t.h2, t.u1, t.p1, t.p2, duc, pbar, uin, dp1, dA, dC, dbu,
                               dub, skipP, &o->pres, &pi[1], warm ? 1 : -1);
  c->pcg_kind = kPcgOther;
  if (rc < 0) return rc;
  // corrector 1: output u**, p*; inputs u*, lag p^n
  PISO_HIP(c, hipMemcpyAsync(duc, uin, sizeof(R) * D * N, hipMemcpyDeviceToDevice, s));
  PISO_HIP(c, hipMemcpyAsync(pbar, dp1, sizeof(R) * N, hipMemcpyDeviceToDevice, s));
  PISO_HIP(c, hipMemsetAsync(uin, 0, sizeof(R) * D * N, s));
  c->pcg_kind = kPcgAdj1;
  c->pcg_same_op = !skipP;   // the second adjoint solve of the step: the same tape P_f
  rc = do_corrector_bwd<R>(c, s, t.A, t.C, t.Pf, t.Dinv, t.h1, t.us, p_n, t.p1, duc, pbar, uin, dp_n, dA, dC, dbu, dub,
                           skipP, &o->pres, &pi[0], warm ? 0 : -1);
  c->pcg_kind = kPcgOther;
  c->pcg_same_op = false;
  if (rc < 0) return rc;
  // velocity solve: mu = C^-T du*, db = mu, dC -= mu (x) u*
  if (!skipV) {
    R* mu = (R*)c->a_mu;
    PISO_HIP(c, hipMemsetAsync(mu, 0, sizeof(R) * D * N, s));
    rc = velocity_solve<R>(c, s, true, t.A, t.C, uin, mu, &o->vel, &vi);
    if (rc < 0) return rc;
    if ((rc = launch_outer_bwd<R>(c, s, t.C, mu, t.us, nullptr, dC, dA))) return rc;
    if ((rc = launch_axpy<R>(c, s, D * N, R(1), mu, dbu))) return rc;
    if (dp_n && o->grad_p_in_predictor)
      if ((rc = launch_gradT<R>(c, s, mu, nullptr, R(-1), dp_n))) return rc;
  }
  rc = do_assemble_bwd<R>(c, s, u_n, nu, nu_field, ub, dt, dA, dC, dbu, du_n, dS, dnu, dub);
  if (rc) return rc;
  if (info) {
    info->vel = vi;
    info->pres[0] = pi[0];
    info->pres[1] = pi[1];
  }
  int st = vi.status;
  for (int k = 0; k < 2; ++k) st = (pi[k].status < 0 || st < 0) ? std::min(st, pi[k].status) : std::max(st, pi[k].status);
  return st;
}

}  // namespace

// ====================================================================== C-ABI

extern "C" {

const char* piso_create_error(void) { return g_create_error.c_str(); }

int piso_create(const piso_domain_desc* desc, int32_t precision, piso_ctx** out) {
  if (!out) return PISO_E_ARG;
  *out = nullptr;
  g_create_error.clear();
  // argument and topology validation first: host only, no device touched
  if (int rc = validate_desc(desc, precision, &g_create_error)) return rc;
  Topology topo;
  if (int rc = build_topology(desc, &topo, &g_create_error)) return rc;
  piso_ctx* c = new piso_ctx();
  c->N = topo.N;
  c->NB = topo.NB;
  c->h_tab.swap(topo.tab);
  c->h_fmap.swap(topo.fmap);
  c->ilu_ok = topo.ilu_ok;
  c->dim = desc->dim;
  c->nblocks = desc->n_blocks;
  c->prec = precision;
  c->esz = precision == PISO_F32 ? 4 : 8;   // MIXED stores its fields in double
  int rc = hipGetDevice(&c->device) == hipSuccess ? PISO_OK : fail(c, PISO_E_HIP, "hipGetDevice failed");
  if (!rc) rc = noalloc_bind(c);
  if (!rc) rc = upload(c, (void**)&c->d_tab, c->h_tab);
  if (!rc) rc = upload(c, (void**)&c->d_fmap, c->h_fmap);
  if (!rc) rc = c->esz == 8 ? upload_metrics<double>(c, desc) : upload_metrics<float>(c, desc);
  if (!rc) rc = alloc_workspaces(c);
  if (!rc) rc = mg_build(c);
  if (!rc && !c->mg.empty()) rc = line_choose(c, desc);
  if (!rc) rc = outflow_build(c);
  if (rc) {
    g_create_error = c->err;
    piso_destroy(c);
    return rc;
  }
  c->grid.dim = c->dim;
  c->grid.nblocks = c->nblocks;
  c->grid.N = c->N;
  c->grid.NB = c->NB;
  c->grid.tab = c->d_tab;
  c->grid.fmap = c->d_fmap;
  c->quad = true;
  for (int b = 0; b < c->nblocks; ++b)
    if (desc->block_cells[3 * b] % 4 != 0) c->quad = false;
  if (const char* e = std::getenv("PISO_NO_QUAD")) c->quad = c->quad && e[0] == '0';   // can only turn it off
  zm_setup(c);   // host only: tiles of the plane-marching kernels (needs quad and the hierarchy)
  if (const char* e = std::getenv("PISO_NO_GRAPH")) c->use_graphs = (e[0] == '0');
  if (const char* e = std::getenv("PISO_CG_GROUPS")) {
    const int v = std::atoi(e);
    c->cg_grid = v < 0 ? 0 : (v > kRedGrid ? kRedGrid : v);
  }
  *out = c;
  return PISO_OK;
}

void piso_destroy(piso_ctx* c) {
  if (!c) return;
  DevGuard g(c->device);
  (void)hipDeviceSynchronize();
  for (hipGraphExec_t& g : c->cg_graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->h_cg) (void)hipHostFree(c->h_cg);
  if (c->h_bi) (void)hipHostFree(c->h_bi);
  if (c->h_scal) (void)hipHostFree(c->h_scal);
  for (hipEvent_t e : c->timing.ev) (void)hipEventDestroy(e);
  delete c;
}

const char* piso_last_error(const piso_ctx* c) { return c ? c->err.c_str() : "null context"; }

int piso_sizes(const piso_ctx* c, int64_t* n_cells, int64_t* n_bfaces, int64_t* tape_bytes, int64_t* elem_bytes,
               int32_t* non_orthogonal) {
  if (!c) return PISO_E_ARG;
  if (n_cells) *n_cells = c->N;
  if (n_bfaces) *n_bfaces = c->NB;
  if (tape_bytes) *tape_bytes = (int64_t)(tape_elems(c) * c->esz);
  if (elem_bytes) *elem_bytes = (int64_t)c->esz;
  if (non_orthogonal) *non_orthogonal = c->nonorth ? 1 : 0;
  return PISO_OK;
}

int piso_mg_info(const piso_ctx* c, int32_t* n_levels, int64_t* cells, int32_t* slots) {
  if (!c) return PISO_E_ARG;
  if (n_levels) *n_levels = (int32_t)c->mg.size();
  for (size_t l = 0; l < c->mg.size(); ++l) {
    if (cells) cells[l] = c->mg[l].n;
    if (slots) slots[l] = c->mg[l].K;
  }
  return PISO_OK;
}

int piso_mg_marching(const piso_ctx* c, int32_t* groups) {
  if (!c || !groups) return PISO_E_ARG;
  // the pressure Krylov vectors are float in the F32 and MIXED forms
  *groups = zm_use(c, c->prec == PISO_F64 ? 8 : 4) ? zm_groups(c) : 0;
  return PISO_OK;
}

int piso_mg_smoother(const piso_ctx* c, int32_t* line_axis) {
  if (!c || !line_axis) return PISO_E_ARG;
  *line_axis = c->mg_line_axis;
  return PISO_OK;
}

void piso_default_step_opts(int32_t precision, piso_step_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->vel.rtol = precision == PISO_F32 ? 1e-7 : 1e-10;
  o->vel.max_iter = 500;
  o->vel.check_every = 4;
  o->pres.rtol = precision == PISO_F64 ? 1e-10 : (precision == PISO_MIXED ? 1e-8 : 1e-6);
  o->pres.max_iter = 20000;
  o->pres.check_every = 4;
  o->pres.precond = PISO_PRECOND_MG;
  o->vel.precond = PISO_PRECOND_JACOBI_ILU0;
  o->pres.inner_rtol = 1e-5;
  o->pres.max_refine = 20;
  o->vel.inner_rtol = 1e-5;
  o->vel.max_refine = 10;
  o->n_correctors = 2;
  o->grad_p_in_predictor = 1;
  o->grad_path_flags = 0;
  o->adjoint_warm_start = 1;
}

#define CTX_ENTER()                                  \
  if (!c) return PISO_E_ARG;                         \
  DevGuard dg_(c->device);                           \
  hipStream_t s = (hipStream_t)stream

#define DISPATCH_R(CALL_F64, CALL_F32) (c->esz == 8 ? (CALL_F64) : (CALL_F32))

int piso_assemble(piso_ctx* c, void* stream, const void* u_n, const void* p_n, const void* nu, int32_t nu_is_field,
                  const void* S, const void* u_b, double dt, int32_t gradp, const piso_system* sys) {
  CTX_ENTER();
  REQUIRE(u_n && p_n && nu && S && sys && sys->A && sys->C && sys->b_u && sys->b && sys->Pf && sys->Dinv,
          "piso_assemble: null pointer");
  REQUIRE(c->NB == 0 || u_b, "piso_assemble: u_b required");
  REQUIRE(dt > 0 && std::isfinite(dt), "piso_assemble: dt must be positive");
#define ARGS(R)                                                                                                    \
  c, s, (const R*)u_n, (const R*)p_n, (const R*)nu, nu_is_field, (const R*)S, (const R*)u_b, dt, gradp, (R*)sys->A, \
      (R*)sys->C, (R*)sys->b_u, (R*)sys->b, (R*)sys->Pf, (R*)sys->Dinv
  return DISPATCH_R(do_assemble<double>(ARGS(double)), do_assemble<float>(ARGS(float)));
#undef ARGS
}

int piso_solve_velocity(piso_ctx* c, void* stream, const piso_system* sys, void* u_star, const piso_solve_opts* o,
                        piso_solve_info* info) {
  CTX_ENTER();
  REQUIRE(sys && sys->A && sys->C && sys->b && u_star && o, "piso_solve_velocity: null pointer");
  REQUIRE(o->rtol > 0 && o->max_iter > 0, "piso_solve_velocity: bad options");
  piso_solve_info tmp{};
  int rc = DISPATCH_R(velocity_solve<double>(c, s, false, (const double*)sys->A, (const double*)sys->C,
                                             (const double*)sys->b, (double*)u_star, o, &tmp),
                      velocity_solve<float>(c, s, false, (const float*)sys->A, (const float*)sys->C,
                                            (const float*)sys->b, (float*)u_star, o, &tmp));
  if (info) *info = tmp;
  return rc < 0 ? rc : tmp.status;
}

int piso_solve_pressure(piso_ctx* c, void* stream, const piso_system* sys, const void* u_in, const void* u_b,
                        const void* p_lag, void* p, const piso_solve_opts* o, piso_solve_info* info) {
  CTX_ENTER();
  REQUIRE(sys && sys->A && sys->C && sys->b_u && sys->Pf && sys->Dinv && sys->h && u_in && p_lag && p && o,
          "piso_solve_pressure: null pointer");
  REQUIRE(c->NB == 0 || u_b, "piso_solve_pressure: u_b required");
  REQUIRE(o->rtol > 0 && o->max_iter > 0, "piso_solve_pressure: bad options");
  piso_solve_info tmp{};
#define ARGS(R)                                                                                                 \
  c, s, (const R*)sys->A, (const R*)sys->C, (const R*)sys->b_u, (const R*)sys->Pf, (const R*)sys->Dinv,          \
      (const R*)u_in, (const R*)u_b, (const R*)p_lag, (R*)sys->h, (R*)sys->rhs, (R*)p, o, &tmp
  int rc = DISPATCH_R(do_pressure<double>(ARGS(double)), do_pressure<float>(ARGS(float)));
#undef ARGS
  if (info) *info = tmp;
  return rc < 0 ? rc : tmp.status;
}

int piso_correct(piso_ctx* c, void* stream, const piso_system* sys, const void* p, const void* p_lag,
                 const void* u_b, void* u_out, void* F_out) {
  CTX_ENTER();
  REQUIRE(sys && sys->A && sys->h && p && u_out, "piso_correct: null pointer");
  REQUIRE(!F_out || (sys->Pf && p_lag), "piso_correct: F_out needs sys->Pf and p_lag");
  (void)u_b;
  return DISPATCH_R(launch_correct<double>(c, s, (const double*)sys->A, (const double*)sys->h, (const double*)p,
                                           (const double*)sys->Pf, (const double*)p_lag, (double*)u_out,
                                           (double*)F_out),
                    launch_correct<float>(c, s, (const float*)sys->A, (const float*)sys->h, (const float*)p,
                                          (const float*)sys->Pf, (const float*)p_lag, (float*)u_out,
                                          (float*)F_out));
}

int piso_step(piso_ctx* c, void* stream, const void* u_n, const void* p_n, const void* nu, int32_t nu_is_field,
              const void* S, const void* u_b, double dt, void* u_np1, void* p_np1, void* tape,
              const piso_step_opts* o, piso_step_info* info) {
  CTX_ENTER();
  REQUIRE(u_n && p_n && nu && S && u_np1 && p_np1 && o, "piso_step: null pointer");
  REQUIRE(c->NB == 0 || u_b, "piso_step: u_b required");
  REQUIRE(dt > 0 && std::isfinite(dt), "piso_step: dt must be positive");
  REQUIRE(o->n_correctors >= 1 && o->n_correctors <= 8, "piso_step: n_correctors must be 1..8");
  REQUIRE(!tape || o->n_correctors == 2, "piso_step: a tape requires n_correctors = 2");
  REQUIRE(u_np1 != u_n && p_np1 != p_n, "piso_step: outputs must not alias inputs");
  REQUIRE(!o->p_star_out || (o->p_star_out != p_n && o->p_star_out != p_np1 && o->p_star_out != o->p_prev &&
                             o->p_star_out != o->p_prev_star),
          "piso_step: p_star_out must not alias p_n, p_np1, p_prev or p_prev_star");
#define ARGS(R)                                                                                              \
  c, s, (const R*)u_n, (const R*)p_n, (const R*)nu, nu_is_field, (const R*)S, (const R*)u_b, dt, (R*)u_np1, \
      (R*)p_np1, tape, o, info
  return DISPATCH_R(do_step<double>(ARGS(double)), do_step<float>(ARGS(float)));
#undef ARGS
}

int piso_correct_backward(piso_ctx* c, void* stream, const piso_system* sys, const void* p, const void* du_out,
                          void* dh, void* dp, void* dA) {
  CTX_ENTER();
  REQUIRE(sys && sys->A && p && du_out, "piso_correct_backward: null pointer");
  const int n = c->dim * c->N;
  if (c->esz == 8) {
    if (dh)
      if (int rc = launch_axpy<double>(c, s, n, 1.0, (const double*)du_out, (double*)dh)) return rc;
    return launch_correct_bwd<double>(c, s, (const double*)sys->A, (const double*)p, (const double*)du_out,
                                      (double*)dp, (double*)dA);
  }
  if (dh)
    if (int rc = launch_axpy<float>(c, s, n, 1.0f, (const float*)du_out, (float*)dh)) return rc;
  return launch_correct_bwd<float>(c, s, (const float*)sys->A, (const float*)p, (const float*)du_out, (float*)dp,
                                   (float*)dA);
}

int piso_solve_pressure_backward(piso_ctx* c, void* stream, const piso_system* sys, const void* u_in,
                                 const void* p_lag, const void* p, const void* dh, const void* dp, void* du_in,
                                 void* dp_lag, void* du_b, const piso_system_grad* g, int32_t skip_solve,
                                 const piso_solve_opts* o, piso_solve_info* info) {
  CTX_ENTER();
  REQUIRE(sys && sys->A && sys->C && sys->Pf && sys->Dinv && sys->h && u_in && p_lag && p && o,
          "piso_solve_pressure_backward: null pointer");
  REQUIRE(g && g->dA && g->dC && g->db_u && du_in, "piso_solve_pressure_backward: null gradient pointer");
  const int N = c->N;
  piso_solve_info tmp{};
  // pbar = dp (copied so the call does not modify the caller's buffer); the correct
  // adjoint has already been applied by piso_correct_backward.
#define BODY(R)                                                                                                    \
  do {                                                                                                             \
    R* pbar = (R*)c->a_pbar;                                                                                        \
    if (dp) PISO_HIP(c, hipMemcpyAsync(pbar, dp, sizeof(R) * N, hipMemcpyDeviceToDevice, s));                      \
    else PISO_HIP(c, hipMemsetAsync(pbar, 0, sizeof(R) * N, s));                                                    \
    R* lam = nullptr;                                                                                               \
    if (!skip_solve) {                                                                                              \
      lam = (R*)c->a_lam;                                                                                           \
      int rc = do_pressure_adjoint<R>(c, s, (const R*)sys->Pf, (const R*)sys->Dinv, pbar, lam, o, &tmp);           \
      if (rc < 0) return rc;                                                                                        \
      if ((rc = launch_pface_bwd<R>(c, s, (const R*)sys->A, lam, (const R*)p, (R*)g->dA))) return rc;              \
    }                                                                                                               \
    R* gv = (R*)c->a_g;                                                                                             \
    if (int rc = launch_h_bwd<R>(c, s, (const R*)sys->A, (const R*)sys->h, (const R*)dh, lam, gv, (R*)g->db_u,     \
                                 (R*)g->dA, (R*)du_b))                                                              \
      return rc;                                                                                                    \
    if (c->nonorth && lam && dp_lag) {                                                                              \
      if (int rc = launch_tgrad<R>(c, s, (const R*)p_lag, 1, (R*)c->w_tgp)) return rc;                             \
      if (int rc = launch_cross_bwd<R>(c, s, (const R*)sys->A, 1, 1, lam, 1, (const R*)c->w_tgp, R(-1), (R*)dp_lag, \
                                       (R*)g->dA))                                                                  \
        return rc;                                                                                                  \
    }                                                                                                               \
    if (int rc = launch_outer_bwd<R>(c, s, (const R*)sys->C, gv, (const R*)u_in, (R*)du_in, (R*)g->dC, nullptr))   \
      return rc;                                                                                                    \
  } while (0)
  if (c->esz == 8) BODY(double);
  else BODY(float);
#undef BODY
  if (info) *info = tmp;
  return tmp.status;
}

int piso_solve_velocity_backward(piso_ctx* c, void* stream, const piso_system* sys, const void* u_star,
                                 const void* du_star, const piso_system_grad* g, int32_t skip_solve,
                                 const piso_solve_opts* o, piso_solve_info* info) {
  CTX_ENTER();
  REQUIRE(sys && sys->A && sys->C && u_star && du_star && o, "piso_solve_velocity_backward: null pointer");
  REQUIRE(g && g->dA && g->dC && g->db, "piso_solve_velocity_backward: null gradient pointer");
  piso_solve_info tmp{};
  if (skip_solve) {
    if (info) *info = tmp;
    return PISO_OK;
  }
  const int N = c->N, D = c->dim;
#define BODY(R)                                                                                                   \
  do {                                                                                                            \
    R* mu = (R*)c->a_mu;                                                                                           \
    PISO_HIP(c, hipMemsetAsync(mu, 0, sizeof(R) * D * N, s));                                                      \
    int rc = velocity_solve<R>(c, s, true, (const R*)sys->A, (const R*)sys->C, (const R*)du_star, mu, o, &tmp);   \
    if (rc < 0) return rc;                                                                                         \
    if ((rc = launch_outer_bwd<R>(c, s, (const R*)sys->C, mu, (const R*)u_star, nullptr, (R*)g->dC, (R*)g->dA)))   \
      return rc;                                                                                                   \
    if ((rc = launch_axpy<R>(c, s, D * N, R(1), mu, (R*)g->db))) return rc;                                        \
  } while (0)
  if (c->esz == 8) BODY(double);
  else BODY(float);
#undef BODY
  if (info) *info = tmp;
  return tmp.status;
}

int piso_assemble_backward(piso_ctx* c, void* stream, const void* u_n, const void* nu, int32_t nu_is_field,
                           const void* u_b, double dt, int32_t gradp, const piso_system_grad* g, void* du_n,
                           void* dp_n, void* dS, void* dnu, void* du_b) {
  CTX_ENTER();
  REQUIRE(u_n && nu && g && g->dA && g->dC && g->db_u && g->db, "piso_assemble_backward: null pointer");
  REQUIRE(c->NB == 0 || u_b, "piso_assemble_backward: u_b required");
  const int N = c->N, D = c->dim;
#define BODY(R)                                                                                                   \
  do {                                                                                                            \
    R* dbu = (R*)c->a_dbu;                                                                                         \
    PISO_HIP(c, hipMemcpyAsync(dbu, g->db_u, sizeof(R) * D * N, hipMemcpyDeviceToDevice, s));                      \
    if (int rc = launch_axpy<R>(c, s, D * N, R(1), (const R*)g->db, dbu)) return rc;                               \
    if (dp_n && gradp)                                                                                             \
      if (int rc = launch_gradT<R>(c, s, (const R*)g->db, nullptr, R(-1), (R*)dp_n)) return rc;                   \
    return do_assemble_bwd<R>(c, s, (const R*)u_n, (const R*)nu, nu_is_field, (const R*)u_b, dt, (const R*)g->dA,  \
                              (const R*)g->dC, dbu, (R*)du_n, (R*)dS, (R*)dnu, (R*)du_b);                         \
  } while (0)
  if (c->esz == 8) BODY(double);
  else BODY(float);
#undef BODY
}

int piso_step_backward(piso_ctx* c, void* stream, const void* tape, const void* u_n, const void* p_n, const void* nu,
                       int32_t nu_is_field, const void* u_b, double dt, const void* du_np1, const void* dp_np1,
                       void* du_n, void* dp_n, void* dS, void* dnu, void* du_b, const piso_step_opts* o,
                       piso_step_info* info) {
  CTX_ENTER();
  REQUIRE(tape && u_n && p_n && nu && o, "piso_step_backward: null pointer");
  REQUIRE(c->NB == 0 || u_b, "piso_step_backward: u_b required");
#define ARGS(R)                                                                                                     \
  c, s, tape, (const R*)u_n, (const R*)p_n, (const R*)nu, nu_is_field, (const R*)u_b, dt, (const R*)du_np1,          \
      (const R*)dp_np1, (R*)du_n, (R*)dp_n, (R*)dS, (R*)dnu, (R*)du_b, o, info
  return DISPATCH_R(do_step_backward<double>(ARGS(double)), do_step_backward<float>(ARGS(float)));
#undef ARGS
}

int piso_adjoint_reset(piso_ctx* c) {
  if (!c) return PISO_E_ARG;
  c->lam_hist_valid[0] = c->lam_hist_valid[1] = false;
  c->lam_hist_valid2[0] = c->lam_hist_valid2[1] = false;
  return PISO_OK;
}

int piso_outflow_update(piso_ctx* c, void* stream, const void* u_n, const void* u_b, const int32_t* outflow,
                        const double* u_m, double dt, void* u_b_out) {
  CTX_ENTER();
  REQUIRE(u_n && outflow && u_m, "piso_outflow_update: null pointer");
  REQUIRE(c->NB == 0 || (u_b && u_b_out), "piso_outflow_update: u_b and u_b_out required");
  REQUIRE(dt > 0 && std::isfinite(dt), "piso_outflow_update: dt must be positive");
  OutflowUm um{};
  for (int i = 0; i < c->dim; ++i) {
    REQUIRE(std::isfinite(u_m[i]), "piso_outflow_update: u_m must be finite");
    um.v[i] = u_m[i];
  }
  return DISPATCH_R(outflow_update<double>(c, s, (const double*)u_n, (const double*)u_b, outflow, um, dt,
                                           (double*)u_b_out),
                    outflow_update<float>(c, s, (const float*)u_n, (const float*)u_b, outflow, um, dt,
                                          (float*)u_b_out));
}

int piso_outflow_update_backward(piso_ctx* c, void* stream, const void* u_n, const void* u_b,
                                 const int32_t* outflow, const double* u_m, double dt, const void* du_b_out,
                                 void* du_n, void* du_b) {
  CTX_ENTER();
  REQUIRE(u_n && outflow && u_m, "piso_outflow_update_backward: null pointer");
  REQUIRE(c->NB == 0 || (u_b && du_b_out && du_b), "piso_outflow_update_backward: boundary arrays required");
  REQUIRE(du_b != du_b_out || c->NB == 0, "piso_outflow_update_backward: du_b must not alias du_b_out");
  REQUIRE(dt > 0 && std::isfinite(dt), "piso_outflow_update_backward: dt must be positive");
  OutflowUm um{};
  for (int i = 0; i < c->dim; ++i) {
    REQUIRE(std::isfinite(u_m[i]), "piso_outflow_update_backward: u_m must be finite");
    um.v[i] = u_m[i];
  }
  return DISPATCH_R(outflow_update_bwd<double>(c, s, (const double*)u_n, (const double*)u_b, outflow, um, dt,
                                               (const double*)du_b_out, (double*)du_n, (double*)du_b),
                    outflow_update_bwd<float>(c, s, (const float*)u_n, (const float*)u_b, outflow, um, dt,
                                              (const float*)du_b_out, (float*)du_n, (float*)du_b));
}

int piso_divfree_gradient(piso_ctx* c, void* stream, const void* S, const void* dS, double lambda,
                          const piso_solve_opts* o, void* dS_out, void* p_S, piso_solve_info* info) {
  CTX_ENTER();
  REQUIRE(S && dS && dS_out && o, "piso_divfree_gradient: null pointer");
  REQUIRE(std::isfinite(lambda), "piso_divfree_gradient: lambda must be finite");
  REQUIRE(o->rtol > 0 && o->max_iter > 0, "piso_divfree_gradient: bad options");
  REQUIRE(dS_out != S, "piso_divfree_gradient: dS_out must not alias S");
  piso_solve_info tmp{};
  int rc = DISPATCH_R(do_divfree<double>(c, s, (const double*)S, (const double*)dS, lambda, o, (double*)dS_out,
                                         (double*)p_S, &tmp),
                      do_divfree<float>(c, s, (const float*)S, (const float*)dS, lambda, o, (float*)dS_out,
                                        (float*)p_S, &tmp));
  if (info) *info = tmp;
  return rc < 0 ? rc : tmp.status;
}

int piso_stats_size(const piso_ctx* c, int32_t axis, int64_t* n_planes, int64_t* record_len) {
  if (!c) return PISO_E_ARG;
  int np, m;
  if (stats_planes(c, axis, &np, &m)) return PISO_E_ARG;
  if (n_planes) *n_planes = np;
  if (record_len) *record_len = 1 + c->dim + c->dim * (c->dim + 1) / 2;
  return PISO_OK;
}

int piso_stats_accumulate(piso_ctx* c, void* stream, const void* u, int32_t axis, double* state) {
  CTX_ENTER();
  REQUIRE(u && state, "piso_stats_accumulate: null pointer");
  return DISPATCH_R(stats_accumulate<double>(c, s, (const double*)u, axis, state),
                    stats_accumulate<float>(c, s, (const float*)u, axis, state));
}

int piso_stats_finalize(piso_ctx* c, void* stream, int32_t axis, const double* state, double* mean, double* cov) {
  CTX_ENTER();
  REQUIRE(state && mean && cov, "piso_stats_finalize: null pointer");
  return stats_finalize(c, s, axis, state, mean, cov);
}

int piso_stats_backward(piso_ctx* c, void* stream, const void* u, int32_t axis, const double* state,
                        const double* mean_bar, const double* cov_bar, void* du) {
  CTX_ENTER();
  REQUIRE(u && state && mean_bar && cov_bar && du, "piso_stats_backward: null pointer");
  return DISPATCH_R(stats_backward<double>(c, s, (const double*)u, axis, state, mean_bar, cov_bar, (double*)du),
                    stats_backward<float>(c, s, (const float*)u, axis, state, mean_bar, cov_bar, (float*)du));
}

int piso_moments_size(const piso_ctx* c, int32_t axis, int32_t m, int32_t order, int64_t* n_planes,
                      int64_t* record_len) {
  if (!c) return PISO_E_ARG;
  int np, ms, na;
  if (moments_layout(c, axis, m, order, &np, &ms, &na)) return PISO_E_ARG;
  if (n_planes) *n_planes = np;
  if (record_len) *record_len = 1 + m + na;
  return PISO_OK;
}

int piso_moments_accumulate(piso_ctx* c, void* stream, const void* x, int32_t m, int32_t order, int32_t axis,
                            double* state) {
  CTX_ENTER();
  REQUIRE(x && state, "piso_moments_accumulate: null pointer");
  return DISPATCH_R(moments_accumulate<double>(c, s, (const double*)x, m, order, axis, state),
                    moments_accumulate<float>(c, s, (const float*)x, m, order, axis, state));
}

int piso_moments_finalize(piso_ctx* c, void* stream, int32_t m, int32_t order, int32_t axis, const double* state,
                          double* mean, double* moments) {
  CTX_ENTER();
  REQUIRE(state && mean && moments, "piso_moments_finalize: null pointer");
  return moments_finalize(c, s, m, order, axis, state, mean, moments);
}

int piso_moments_backward(piso_ctx* c, void* stream, const void* x, int32_t m, int32_t order, int32_t axis,
                          const double* state, const double* mean_bar, const double* moments_bar, void* dx) {
  CTX_ENTER();
  REQUIRE(x && state && mean_bar && moments_bar && dx, "piso_moments_backward: null pointer");
  return DISPATCH_R(moments_backward<double>(c, s, (const double*)x, m, order, axis, state, mean_bar, moments_bar,
                                             (double*)dx),
                    moments_backward<float>(c, s, (const float*)x, m, order, axis, state, mean_bar, moments_bar,
                                            (float*)dx));
}

int piso_field_gradient(piso_ctx* c, void* stream, const void* phi, int32_t ncomp, const void* phi_b, void* out) {
  CTX_ENTER();
  REQUIRE(phi && out && ncomp >= 1, "piso_field_gradient: null pointer or no components");
  return DISPATCH_R(field_gradient<double>(c, s, (const double*)phi, ncomp, (const double*)phi_b, (double*)out),
                    field_gradient<float>(c, s, (const float*)phi, ncomp, (const float*)phi_b, (float*)out));
}

int piso_budget(piso_ctx* c, void* stream, int32_t axis, int32_t order_u, const double* state_u,
                const double* state_grad, const double* state_up, const double* wall_mean, double* out) {
  CTX_ENTER();
  REQUIRE(state_u && state_grad && state_up && wall_mean && out, "piso_budget: null pointer");
  return DISPATCH_R(budget<double>(c, s, axis, order_u, state_u, state_grad, state_up, wall_mean, out),
                    budget<float>(c, s, axis, order_u, state_u, state_grad, state_up, wall_mean, out));
}

int piso_set_timing(piso_ctx* c, int32_t enable) {
  if (!c) return PISO_E_ARG;
  c->timing.enabled = enable != 0;
  for (int k = 0; k < kTimeKinds; ++k) {
    c->timing.ms[k] = 0.0;
    c->timing.calls[k] = 0;
  }
  c->timing.used = 0;
  c->timing.kinds.clear();
  return PISO_OK;
}

int piso_get_timing(piso_ctx* c, int32_t kind, double* ms, int64_t* calls) {
  if (!c || kind < 0 || kind >= kTimeKinds) return PISO_E_ARG;
  if (ms) *ms = c->timing.ms[kind];
  if (calls) *calls = c->timing.calls[kind];
  return PISO_OK;
}

}  // extern "C"
