// Host-side internals of the PISO library: the context and the launch wrappers that
// the C-ABI layer (piso_api.hip) composes.  Kernels live in piso_fwd.hip,
// piso_krylov.hip and piso_bwd.hip.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/piso.h"
#include "piso_common.h"

namespace piso {

// Solver scalars live on the device.  Values produced at iteration k go to slot k & 1
// so that a kernel never overwrites a slot that other work-groups of the same launch
// still read.
// The iteration index k lives here too: the update kernel's lead thread advances it,
// and kernels take only its parity (slot) as an argument, so that a recorded sequence
// of two iterations can be replayed as a graph.
struct CgState {
  double rz[2];
  double rr, bb, tol2, pad0;
  int done, iters, status, zero_rhs;
  int k, max_k, pad1, pad2;
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

// Kernel classes of the solver timing (piso_get_timing).
// Kinds of pressure solve, for the iteration-count estimates of the host read-backs:
// forward correctors 1 and 2, adjoint correctors 1 and 2, everything else.
constexpr int kPcgFwd1 = 0, kPcgAdj1 = 2, kPcgOther = 4;

constexpr int kTimeCgStencil = 0;   // PCG stencil kernel (direction update and M d)
constexpr int kTimeCgUpdate = 1;    // PCG x, r update
constexpr int kTimeMgDown0 = 2;     // multigrid restriction from the fine grid
constexpr int kTimeMgUp0 = 3;       // multigrid prolongation and smoothing on the fine grid
constexpr int kTimeMgCoarse = 4;    // multigrid kernels on the coarse levels
constexpr int kTimeCgUpdateMg = 5;  // PCG update fused with the fine-grid pre-smoothing
constexpr int kTimeMgSmooth0 = 6;   // first fine-grid pre-smoothing of a solve (line smoother)
constexpr int kTimeKinds = 7;

struct Timing {
  bool enabled = false;
  double ms[kTimeKinds] = {};
  long long calls[kTimeKinds] = {};
  std::vector<hipEvent_t> ev;   // pool: pairs around each timed launch
  std::vector<int> kinds;       // kind of each recorded pair
  size_t used = 0;
};

// One coarse level of the aggregation multigrid preconditioner of the pressure
// solve.  Level 0 is the fine grid itself (face coefficients Pf, Jacobi scale Dinv);
// level l >= 1 aggregates 2^d cells of level l-1 (2 per axis inside each block) and
// carries its operator as a graph: slot s of cell I joins I to nbr[s][I] with face
// weight W[s][I] (both directions stored), the Galerkin sum of the finer level's face
// weights between the two aggregates.
struct MgLevel {
  int n = 0, K = 0;
  int* nbr = nullptr;     // [K][n] neighbour on this level, or -1
  int* child = nullptr;   // [2^d][n] finer-level cells of each aggregate, or -1
  int* parent = nullptr;  // [n_finer] aggregate of each finer-level cell
  int* ptr = nullptr;     // [K*n + 1] contribution range of (slot s, cell I) at s*n + I
  int* idx = nullptr;     // finer-level face-weight positions summed into each slot
  void* W = nullptr;      // [K][n] working precision
  void* Dinv = nullptr;   // [n] inverse of the diagonal sum_s W[s][I] (0 if isolated)
  void* r = nullptr;      // [n] restricted residual
  void* e = nullptr;      // [n] correction
  // single-block grids: the level's extents and the division magic for nx and nx * ny
  // (slots are the directions 2 * axis + side there)
  int dims[3] = {0, 0, 0};
  uint32_t mx_lo = 0, mx_hi = 0, mxy_lo = 0, mxy_hi = 0;
  int mx_sh = 0, mxy_sh = 0;
};

// Tiles of the fine-grid restriction: per block, the first tile and the number of
// 64-cell segments per fine row.
struct MgTiles {
  int nb;
  int off[kMaxBlocks + 1];
  int nseg[kMaxBlocks];
};

// Work-groups of the quad-vectorised fused update and restriction: per block, the first
// group and the number of units (an x-quad of 4 fine cells in one aggregate row and
// plane, handled by 2^(d-1) threads: one per fine row and plane parity).
struct MgQuadTiles {
  int nb;
  int off[kMaxBlocks + 1];
  int units[kMaxBlocks];
};

// Work-groups of the plane-marching fine-grid kernels (piso_zmarch.hip): per block, the
// first group, quads per tile row, rows per tile, planes per run, tiles in x and in y.
struct ZmTiles {
  int nb;
  int off[kMaxBlocks + 1];
  int xq[kMaxBlocks], rt[kMaxBlocks], ks[kMaxBlocks];
  int ntx[kMaxBlocks], nty[kMaxBlocks];
  bool plain;   // the kernels' form without sides connected to other blocks (see zm_setup)
};
constexpr int kZmWG = 512;         // threads of a plane-marching work-group
constexpr int kZmTarget = 256;     // work-groups the run length aims at (one per CU; measured
                                   // against 384-1024 at 256^3 and 192x128x192: best or equal)
constexpr int kZmMinPlanes = 4;    // shortest run of planes (each run re-reads two planes)
// Measured per PCG iteration against the one-quad-per-thread kernels: 256^3 505 -> 412 us
// (FP32) and 1020 -> 785 us (FP64); 192x128x192 145 -> 130 us (FP32) and 298 -> 265 us
// (FP64); 128^3 FP32 (8 MiB per field) 95 -> 81 us.  On smaller grids they lose (96^3: FP32
// 61 -> 58 us, FP64 80 -> 85 us; 64^3 FP32 47 -> 55 us): fewer, longer work-groups cost
// more than the re-reads, which the Infinity Cache then holds.
constexpr size_t kZmMinStreamBytes = size_t(8) << 20;

constexpr int kMgCoarse = 2048;     // stop coarsening at this many cells (one work-group solves it)
constexpr int kMgCoarseThreads = 1024;   // that work-group: kMgCoarse / kMgCoarseThreads cells per thread
constexpr int kMgMaxLevels = 16;
constexpr int kMgCoarseSteps3 = 12;   // Chebyshev steps on the coarsest level, 3D
constexpr int kMgCoarseSteps2 = 32;   // and 2D (cheaper steps, slower Jacobi-type convergence)
constexpr int kMgCoarseStepsMax = 32;
constexpr double kMgChebRatio = 100.0;   // their interval [2 / ratio, 2] of the spectrum of D^-1 M
constexpr double kMgOmega = 0.8;        // damping of the fine-level smoother
constexpr double kMgOmegaCoarse = 0.9;  // damping of the Jacobi sweeps on the coarse levels (< 1:
                                        // the V-cycle stays symmetric positive definite)
constexpr int kMgPinGroups = 64;    // coarse-level launches up to this many work-groups run on one XCD

}  // namespace piso

struct piso_ctx {
  int dim = 0, nblocks = 0, N = 0, NB = 0, prec = 0, device = 0;
  size_t esz = 8;                 // element bytes of the stored fields: 4 for F32, else 8
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
  // metrics of the Dirichlet faces (the boundary cell's unless given at piso_create), with
  // j_f the axis of face f: bjt[i][f] = (J T)_{j_f i}, balpha[k][f] = alpha_{j_f k}
  void* bjt = nullptr;    // [d][NB]
  void* balpha = nullptr; // [d][NB]
  // workspaces, working precision unless noted
  void *w_A = nullptr, *w_C = nullptr, *w_bu = nullptr, *w_b = nullptr, *w_Pf = nullptr,
       *w_Dinv = nullptr, *w_h = nullptr, *w_W = nullptr, *w_rhs = nullptr, *w_us = nullptr,
       *w_u1 = nullptr, *w_p1 = nullptr, *w_h1 = nullptr;
  void* w_tg = nullptr;           // [d*d][N] tangential gradients (non-orthogonal)
  void* w_tgp = nullptr;          // [d][N]
  void* w_zb = nullptr;           // [d][max(NB,1)] zeros (boundary values of a source field)
  // MIXED: float copies of the step's operators for the inner solves, and the float
  // residual and correction of the refinement (velocity: [d][N], pressure: [N])
  void *x_Pf32 = nullptr, *x_Dinv32 = nullptr, *x_A32 = nullptr, *x_C32 = nullptr;
  void *m_r32 = nullptr, *m_e32 = nullptr;
  const void* mix_op_src = nullptr;   // double P_f the float pressure operator was rounded from
  double* mix_scal = nullptr;         // [8] device scalars of the refinement residuals
  void *k_r = nullptr, *k_q = nullptr, *k_d0 = nullptr, *k_d1 = nullptr;   // PCG [N]
  void* k_r2 = nullptr;           // second residual buffer of the multigrid PCG [N]
  // adjoint pressure solutions of the last piso_step_backward per corrector (8 bytes per
  // cell), the warm start of the next call
  void* a_lam_hist[2] = {nullptr, nullptr};
  bool lam_hist_valid[2] = {false, false};
  void* a_lam_hist2[2] = {nullptr, nullptr};
  bool lam_hist_valid2[2] = {false, false};
  void* k_z = nullptr;            // PCG preconditioned residual [N] (multigrid)
  void* k_y = nullptr;            // omega D^-1 r, the multigrid pre-smoothing [N]
  // PCG operands copied into context-owned buffers (graph-stable pointers)
  void *g_Pf = nullptr, *g_Dinv = nullptr, *g_x = nullptr;
  hipGraphExec_t cg_graph[2] = {nullptr, nullptr};   // recorded iteration pair: Jacobi, multigrid
  hipStream_t cap_stream = nullptr;                 // stream used only for recording
  bool use_graphs = true;
  // iterations of the last solve per preconditioner (Jacobi, multigrid) and kind: plain
  // solves, then the first, second and later MIXED refinement sweeps
  // [kind][slot]: kind = the solve's place in a step (kPcgKinds below), slot = plain
  // solve, then the first, second and later MIXED refinement sweeps
  int pcg_hint[2][5][4] = {};
  int pcg_kind = 4;               // kind of the next pressure solves (set around them)
  // The PCG copies P_f and D^-1 into g_Pf / g_Dinv and builds the coarse operators from
  // them.  A caller that knows the operator has not changed since the last solve (the
  // second corrector of a step, the second adjoint solve, later MIXED sweeps) sets
  // pcg_same_op around the solve; the setup is then skipped when it was made from the
  // same buffer, element size and preconditioner.
  bool pcg_same_op = false;
  const void* pcg_op_src = nullptr;
  int pcg_op_es = 0;
  bool pcg_op_mg = false;
  std::vector<piso::MgLevel> mg;  // coarse levels 1..L of the pressure preconditioner
  piso::Grid mg_g1{};             // level 1 as a block table (offsets, dims, division magic)
  piso::MgTiles mg_tiles{};       // work-group tiles of the fine-grid restriction
  piso::MgQuadTiles mg_qtiles{};  // the same for the quad-vectorised fused update (nx % 4 == 0)
  piso::ZmTiles zm_tiles{};       // tiles of the plane-marching fine-grid kernels
  bool zm_on = false;             // 3D quad grid with a hierarchy: those kernels may run
  bool zm_force = false;          // PISO_ZMARCH=1: at every size
  bool mg_struct = false;         // single block: coarse levels indexed by position
  int mg_line_axis = 0;           // fine-level line smoothing along this axis (0: point Jacobi)
  int mg_line_L = 0;              // cells per line segment (8 segments per line)
  // Dirichlet faces: owning cell and side (2 * axis + high), and the boundary cells
  // with their faces (ascending) for deterministic gathers
  int *out_bcell = nullptr, *out_bside = nullptr, *out_bc_cell = nullptr, *out_bc_ptr = nullptr,
      *out_bc_face = nullptr;
  int out_nbc = 0;
  void *out_star = nullptr, *out_contrib = nullptr;   // [d][NB] working precision
  void *b_r = nullptr, *b_rh = nullptr, *b_p0 = nullptr, *b_p1 = nullptr, *b_v0 = nullptr,
       *b_v1 = nullptr, *b_s = nullptr, *b_t = nullptr;                    // BiCGStab [d][N]
  void* b_iA = nullptr;   // BiCGStab: 1 / A, formed once per solve [N]
  void *b_ph = nullptr, *b_sh = nullptr;   // BiCGStab with ILU(0): M^-1 p, M^-1 s [d][N]
  void* b_sinv = nullptr;                  // ILU(0): 1 / S (second colour), 1 / A (first) [N]
  bool ilu_ok = false;    // two colours tile the grid (tab[kTabColour] holds each block's parity)
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
  int cg_grid = 0;                 // work-groups of the PCG kernels (0: chosen from the size)
  std::vector<void*> allocs;
  void* noalloc_scratch = nullptr;   // device address of the allocation-free entry's array
  double* plane_work = nullptr;      // [2 * largest extent] plane metrics of the budget terms
  piso::Timing timing;
  std::string err;
};

namespace piso {

// Makes the context's device current for the duration of a call.
struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

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

// Device allocation owned by the context (freed by piso_destroy).
inline int dev_alloc(piso_ctx* c, void** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(c, PISO_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocs.push_back(*p);
  return PISO_OK;
}

template <typename T>
int upload(piso_ctx* c, void** dst, const std::vector<T>& v) {
  if (int rc = dev_alloc(c, dst, v.size() * sizeof(T))) return rc;
  PISO_HIP(c, hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return PISO_OK;
}

// Kernel timing for the benchmark: when enabled, solver kernels are launched with
// start/stop events attached to the dispatch itself (hipExtLaunchKernelGGL), so the
// elapsed time is the kernel's execution, as a kernel trace reports it.
inline bool timing_pair(piso_ctx* c, hipEvent_t& a, hipEvent_t& b) {
  Timing& t = c->timing;
  if (!t.enabled) return false;
  if (t.used + 2 > t.ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      t.ev.push_back(e);
    }
  }
  a = t.ev[t.used++];
  b = t.ev[t.used++];
  return true;
}

// After a stream sync: fold the elapsed times of the recorded pairs into the totals.
inline void timing_collect(piso_ctx* c) {
  Timing& t = c->timing;
  if (!t.enabled) return;
  for (size_t q = 0, k = 0; q + 1 < t.used && k < t.kinds.size(); q += 2, ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev[q], t.ev[q + 1]) != hipSuccess) continue;
    t.ms[t.kinds[k]] += ms;
    t.calls[t.kinds[k]] += 1;
  }
  t.used = 0;
  t.kinds.clear();
}

// Launch with optional dispatch-attached timing events.
template <typename K, typename... Args>
void launch_timed_wg(piso_ctx* c, hipStream_t s, int kind, K kernel, int G, int wg, Args... args) {
  hipEvent_t a, b;
  if (timing_pair(c, a, b)) {
    hipExtLaunchKernelGGL(kernel, dim3(G), dim3(wg), 0, s, a, b, 0, args...);
    c->timing.kinds.push_back(kind);
  } else {
    hipLaunchKernelGGL(kernel, dim3(G), dim3(wg), 0, s, args...);
  }
}

template <typename K, typename... Args>
void launch_timed(piso_ctx* c, hipStream_t s, int kind, K kernel, int G, Args... args) {
  launch_timed_wg(c, s, kind, kernel, G, kWG, args...);
}

inline int grid_cells(int N) { return (N + kWG - 1) / kWG; }
// Work-groups of the Krylov and reduction kernels.  Every work-group of a kernel
// re-reduces the previous kernel's per-group partials, so more groups cost a longer
// prologue; fewer leave the chip idle.  Measured on the 96^3, 192x128x192, 256^2 and
// cylinder workloads: best with whole loop trips of 256 work units (quads or cells) per
// group, as few trips as keep the grid at or below 1536 groups, and at least 256 groups
// (then 64 units each).  (A fixed 512 groups for the one-shot sums left 128 cells per
// thread at 256^3, with too few waves in flight: k_div 0.50 ms there.)
inline int solver_groups(long units) {
  const long trips = std::max(1L, (units + 256L * 1536 - 1) / (256L * 1536));
  long g = (units + 256 * trips - 1) / (256 * trips);
  if (g < 256) g = std::min(256L, (units + 63) / 64);
  return (int)std::max(1L, std::min(g, (long)kRedGrid));
}
inline int grid_red(int N) { return solver_groups(N); }
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
// max over cells of |face-flux divergence| of a corrected flux F [d][N] (+ Dirichlet fluxes
// of u_b) into *out (device)
template <typename R>
int launch_flux_div(piso_ctx* c, hipStream_t s, const R* F, const R* ub, double* out);
// Cell and side (2 axis + high) of every Dirichlet face, from the face map.
int bface_cells(piso_ctx* c, std::vector<int>& bcell, std::vector<int>& bside);
// y = 2 p - q over ncomp fields of N cells
template <typename R>
int launch_extrapolate(piso_ctx* c, hipStream_t s, const R* p, const R* q, R* y, int ncomp = 1);
// y = a + b - q
template <typename R>
int launch_add_diff(piso_ctx* c, hipStream_t s, const R* a, const R* b, const R* q, R* y);
template <typename R>
int launch_add_scalar(piso_ctx* c, hipStream_t s, const double* v, R* y);
template <typename R>
int launch_fill(piso_ctx* c, hipStream_t s, int n, R v, R* y);
template <typename R>
int launch_jt_field(piso_ctx* c, hipStream_t s, const R* S, R* W);
template <typename TI, typename TO>
int launch_sum(piso_ctx* c, hipStream_t s, const TI* x, int n, double scale, double* out);
template <typename TI, typename TO>
int launch_sub_mean(piso_ctx* c, hipStream_t s, const TI* x, const double* mean, TO* y, int n);
template <typename TI, typename TO>
int launch_copy(piso_ctx* c, hipStream_t s, const TI* x, TO* y, int n);

// ---- multigrid preconditioner (piso_mg.hip) ----
// Host construction of the aggregation hierarchy from the block table and face map.
int mg_build(piso_ctx* c);
// Coarse operators of every level from the fine face coefficients Pf.
template <typename R>
int mg_setup(piso_ctx* c, hipStream_t s, const R* Pf);
// z = B r (one V-cycle, zero initial guess) and the partial sums of r.z and r.r over
// G work-groups into partB; every kernel returns at once when st->done is set.
// y = omega D^-1 r for a fresh residual (the PCG update writes it in the iterations).
template <typename R>
int mg_prescale(piso_ctx* c, hipStream_t s, const R* Dinv, const R* r, R* y);
template <typename R>
int mg_apply(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* r, const R* y, R* z, CgState* st,
             double* partB, int G);
// One PCG update (alpha from the Gp partials of d.q in partA, x += alpha d, rout = rin -
// alpha q, y = omega D^-1 rout) fused with the fine-grid restriction, then the rest of
// the V-cycle as mg_apply on rout.
template <typename R>
int mg_update_apply(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, R* x, const R* rin, R* rout,
                    const R* dnew, const R* q, R* y, R* z, CgState* st, const double* partA, int Gp, int par,
                    double* partB, int G);

// ---- plane-marching fine-grid kernels (piso_zmarch.hip) ----
// Tiles for 3D grids of quads with a multigrid hierarchy (sets zm_on).  PISO_ZMARCH=0 keeps
// the one-quad-per-thread kernels, PISO_ZMARCH=1 takes the marching ones at every size.
int zm_setup(piso_ctx* c);
int zm_groups(const piso_ctx* c);
// For Krylov vectors of es bytes per element: tiles built, point smoothing, and a large grid.
inline bool zm_use(const piso_ctx* c, size_t es) {
  return c->zm_on && c->mg_line_axis == 0 && (c->zm_force || (size_t)c->N * es >= kZmMinStreamBytes);
}
// The PCG update fused with the fine-level pre-smoothing and restriction (as k_mg_down0uq).
template <typename R>
int zm_launch_down(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, R* x, const R* rin, R* rout,
                   const R* dnew, const R* q, R* y, R* rc, CgState* st, const double* partA, int Gp, int par);
// The direction update and M d with the d.q partials (as k_cg_spmv_q with z as operand).
template <typename R>
int zm_launch_spmv(piso_ctx* c, hipStream_t s, const R* Pf, const R* z, const R* dold, R* dnew, R* q, CgState* st,
                   const double* partB, double* partA, int Gp, int par);
// The prolongation with the fine-level post-smoothing and the r.z, r.r partials (as k_mg_up0_q).
template <typename R>
int zm_launch_up(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* r, const R* y, const int* parent,
                 const R* e1, R* z, double* partB, const CgState* st);

// ---- fine-level line smoothing (piso_line.hip) ----
// Chooses the line axis for a single-block grid whose metric is strongly anisotropic
// along one transverse axis (y or z), else leaves point Jacobi.
int line_choose(piso_ctx* c, const piso_domain_desc* desc);
// Work-groups of the line kernels (32 lines each); their partial sums use this count.
int line_groups(const piso_ctx* c);
// y = omega T^-1 r' (T: tridiagonal part of M along the line axis), after the PCG update
// x += alpha d, r' = rin - alpha q into rout when `update`, else r' = rin.
template <typename R>
int line_pre(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, R* x, const R* rin, R* rout, const R* dnew,
             const R* q, R* y, CgState* st, const double* partA, int Gp, int par, bool update);
// z = z1 + omega T^-1 (r - M z1), z1 = y + e1[parent]; partial sums of r.z, r.r into partB
// (line_groups work-groups).
template <typename R>
int line_post(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const R* r, const R* y, const R* e1, R* z,
              double* partB, CgState* st);
// Level-1 residual R (r - M y) into mg[0].r in the quad layout; returns 1 without
// launching where that layout does not apply (the tile kernel is used then).
template <typename R>
int line_restrict(piso_ctx* c, hipStream_t s, const R* Pf, const R* r, const R* y, CgState* st);

// ---- advective outflow boundary (piso_outflow.hip) ----
struct OutflowUm {
  double v[3];
};
int outflow_build(piso_ctx* c);
template <typename R>
int outflow_update(piso_ctx* c, hipStream_t s, const R* u, const R* ub, const int* outflow, OutflowUm um,
                   double dt, R* ub_out);
template <typename R>
int outflow_update_bwd(piso_ctx* c, hipStream_t s, const R* u, const R* ub, const int* outflow, OutflowUm um,
                       double dt, const R* gbar, R* du, R* dub);

// ---- online plane statistics (piso_stats.hip) ----
int stats_planes(const piso_ctx* c, int axis, int* n_planes, int* m);
template <typename R>
int stats_accumulate(piso_ctx* c, hipStream_t s, const R* u, int axis, double* state);
int stats_finalize(piso_ctx* c, hipStream_t s, int axis, const double* state, double* mean, double* cov);
template <typename R>
int stats_backward(piso_ctx* c, hipStream_t s, const R* u, int axis, const double* state, const double* mbar,
                   const double* cbar, R* du);

// ---- arbitrary-order moments, field gradients, budget terms (piso_moments.hip) ----
int moments_layout(const piso_ctx* c, int axis, int m, int order, int* n_planes, int* samples, int* n_alpha);
template <typename R>
int moments_accumulate(piso_ctx* c, hipStream_t s, const R* x, int m, int order, int axis, double* state);
int moments_finalize(piso_ctx* c, hipStream_t s, int m, int order, int axis, const double* state, double* mean,
                     double* mom);
template <typename R>
int moments_backward(piso_ctx* c, hipStream_t s, const R* x, int m, int order, int axis, const double* state,
                     const double* mbar, const double* obar, R* dx);
template <typename R>
int field_gradient(piso_ctx* c, hipStream_t s, const R* phi, int nc, const R* phib, R* out);
template <typename R>
int budget(piso_ctx* c, hipStream_t s, int axis, int order_u, const double* su, const double* sg, const double* sup,
           const double* wall_mean, double* out);

// ---- Krylov solvers (piso_krylov.hip) ----
// Zero-mean solution of P x = rhs - mean: rhs of type BT, mean a device scalar or null.
template <typename R, typename BT>
int pressure_solve(piso_ctx* c, hipStream_t s, const R* Pf, const R* Dinv, const BT* rhs,
                   const double* mean, R* x, const piso_solve_opts* o, piso_solve_info* info);
// MIXED form: double residual with the double Pf and rhs64, inner float PCG, refinement
// of the double x64 (pressure_solve<double, double> comes here in a MIXED context).
int pressure_solve_mixed(piso_ctx* c, hipStream_t s, const double* Pf, const double* Dinv,
                         const double* rhs64, const double* mean, double* x64,
                         const piso_solve_opts* o, piso_solve_info* info);
template <typename R>
int velocity_solve(piso_ctx* c, hipStream_t s, bool trans, const R* A, const R* C, const R* b, R* x,
                   const piso_solve_opts* o, piso_solve_info* info);
// Workspace of one BiCGStab solve (F64 / F32 contexts): the vectors r, r-hat, p (two),
// v (two), s, t ([d][N] each) and 1/A ([N]) in the context's element type (with ILU(0)
// also M^-1 p, M^-1 s and the pivots), the partial-sum regions (3, 6 and 9 values of
// kRedGrid doubles each) and the solver state.
struct BiWork {
  void *r, *rh, *p0, *p1, *v0, *v1, *s, *t, *iA;
  void *ph, *sh, *sinv;   // ILU(0) only: M^-1 p, M^-1 s ([d][N]) and the pivots ([N])
  double *part1, *part2, *part3;
  BiState* st;
};
BiWork bi_work_ctx(piso_ctx* c);   // the context's own workspaces
template <typename R>
int velocity_solve_ws(piso_ctx* c, hipStream_t s, bool trans, const R* A, const R* C, const R* b, R* x,
                      const piso_solve_opts* o, piso_solve_info* info, const BiWork& w);
// The fixed device array of the allocation-free entry point on the context's device
// (piso_noalloc.hip): its address, looked up once per device at context creation.
int noalloc_bind(piso_ctx* c);

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
