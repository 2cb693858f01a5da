/*
 * piso.h - C-ABI of a multi-block PISO time step for incompressible flow on
 * AMD Instinct MI355X (gfx950), with its hand-written adjoint.
 *
 * The method is the PISO algorithm with a collocated finite-volume discretisation on
 * multi-block structured grids with precomputed cell-centre transformations, as given
 * in arXiv 2505.16992 (PICT), Sec. 2.1-2.3 and App. A.2-A.5.  One step:
 *
 *   predictor   C(u^n) u* = b,  b = b_u - grad p^n            (App. A.2, eq. advectionMat)
 *   corrector   h = A^-1 (b_u - H u);  P p = div h;  u = h - A^-1 grad p
 *               applied twice (u = u*, then u**)                (eqs. pressureRHS, pressure,
 *                                                                  correction)
 *   output      u^{n+1} = u***,  p^{n+1} = p**
 *
 * with A = diag(C), H = C - A, P the pressure matrix of eq. pMatDiscrete, b_u the
 * predictor right-hand side of eq. velRHSdiscrete (plus deferred non-orthogonal terms,
 * App. A.3.5).  Rows of C are per unit volume (temporal term 1/dt).
 *
 * Data layout (all calls):
 *   - cells of block b are numbered off_b + i + nx*(j + ny*k) (x fastest), blocks
 *     concatenated in block order; N = total cells, d = 2 or 3;
 *   - fields are structure-of-arrays: a vector field is [d][N], a scalar [N];
 *   - face arrays are [d][N]: entry [j][P] belongs to the face between P and its
 *     +j neighbour (zero where that face is a boundary);
 *   - the matrix C is stored as its diagonal A [N] and the face array C [2][d][N]:
 *     C[0][j][P] = C(P, P+j) and C[1][j][P] = C(P+j, P);
 *   - Dirichlet boundary values u_b are [d][NB]: Dirichlet segments in the order they
 *     were given to piso_create, faces of a segment in tangential order (first
 *     tangential axis fastest).
 *   - element type of every field, intermediate and gradient: float for PISO_F32,
 *     double for PISO_F64 and PISO_MIXED.
 *
 * Pointers: "device" pointers must point to memory of the device that was current at
 * piso_create; "host" pointers are read during the call only.  The caller owns every
 * field, intermediate, tape and gradient buffer; the context owns its topology tables,
 * metric copies and solver workspaces (allocated in piso_create, freed in
 * piso_destroy).  A context is not thread-safe; calls on one context must not overlap.
 *
 * Streams: work is enqueued on the given stream (hipStream_t, may be 0).  The Krylov
 * solves read their convergence state back to the host every check_every iterations,
 * which synchronises that stream; everything else is asynchronous.
 *
 * Errors: a negative return is a hard error (outputs unspecified, message from
 * piso_last_error); a positive return is a soft status (outputs written; see the
 * piso_solve_info).  No call allocates device memory after piso_create.
 */
#ifndef PISO_H
#define PISO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct piso_ctx piso_ctx;

typedef enum {
  PISO_F64 = 0,    /* all storage and arithmetic in double */
  PISO_F32 = 1,    /* float storage and stencil arithmetic; Krylov dot products in double */
  PISO_MIXED = 2   /* double storage and double stencil arithmetic outside the Krylov
                      iterations; both linear solves run as iterative refinement: the
                      residual of the double system in double, a float inner Krylov solve
                      (float operator copies, float vectors, double dot products) for the
                      correction, the correction added in double */
} piso_precision;

typedef enum {
  PISO_OK = 0,
  PISO_NOT_CONVERGED = 1,   /* solve stopped at max_iter above its tolerance */
  PISO_BREAKDOWN = 2,       /* BiCGStab breakdown (rho or omega vanished) */
  PISO_E_ARG = -1,          /* invalid argument (null pointer, bad size, bad option) */
  PISO_E_TOPOLOGY = -2,     /* invalid block layout (see piso_create) */
  PISO_E_HIP = -3,          /* a HIP runtime call failed */
  PISO_E_NAN = -4,          /* a residual became NaN or infinite */
  PISO_E_OOM = -5           /* device allocation failed in piso_create */
} piso_status;

typedef enum {
  PISO_SIDE_CONNECT = 0,    /* conformal connection to the opposite side of another (or the
                               same, for periodicity) block with the same axis orientation */
  PISO_SIDE_DIRICHLET = 1   /* prescribed velocity u_b; implies zero-Neumann pressure (App. A.4) */
} piso_side_kind;

/* One segment of one block side (Sec. 2.2: each side carries a connection or a prescribed
 * value; a side may be tiled by several segments).  side: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z,
 * 5 +z.  Tangential axes of a side are the two other axes in increasing order.  */
typedef struct {
  int32_t block, side, kind;
  int32_t begin[2], end[2];        /* tangential cell range [begin, end); 2D: begin[1]=0, end[1]=1 */
  int32_t other_block;             /* CONNECT: block entered through this segment */
  int32_t other_begin[2];          /* CONNECT: tangential position of begin on the other side */
} piso_side_desc;

typedef struct {
  int32_t dim;                     /* 2 or 3 */
  int32_t n_blocks;                /* 1 .. 16 */
  int32_t n_sides;
  const int32_t* block_cells;      /* host [n_blocks][3] (nx, ny, nz); nz = 1 in 2D */
  const piso_side_desc* sides;     /* host [n_sides]; must tile every block side exactly once */
  const double* T;                 /* host [d][d][N]: T[(j*d + i)*N + P] = d xi^j / d x_i at centres */
  const double* J;                 /* host [N]: det(d x / d xi) > 0 (cell volume) */
  /* Metrics on the Dirichlet faces (App. A.4: a prescribed boundary carries its values
     and metrics on the face itself; eq. velRHSdiscrete takes alpha and U there without
     interpolation).  Both NULL: every Dirichlet face takes the metrics of its boundary
     cell.  Otherwise both given, in the face order of u_b: Tb[(j*d + i)*NB + f] =
     d xi^j / d x_i and Jb[f] > 0 on face f.  They enter the 2 alpha_jj nu diagonal and
     the boundary terms of the predictor (eqs. difMatDiscrete, velRHSdiscrete), the
     deferred cross terms through the face (eq. velRHSnonOrtho), the Dirichlet flux
     N (J T_j) . u_b of the pressure right-hand side and of the outflow balance, and
     their adjoints.  Non-finite values or Jb <= 0: PISO_E_ARG. */
  const double* Tb;                /* host [d][d][NB] or NULL */
  const double* Jb;                /* host [NB] or NULL */
} piso_domain_desc;

/* Preconditioner of a Krylov solve (piso_solve_opts.precond). */
typedef enum {
  PISO_PRECOND_JACOBI = 0,  /* diagonal scaling (pressure CG and velocity BiCGStab) */
  PISO_PRECOND_MG = 1,      /* pressure CG only: one V-cycle of aggregation multigrid per
                               iteration (2^d cells per aggregate inside each block, Galerkin
                               coarse operators, damped Jacobi smoothing).  The paper names
                               multigrid for the pressure as the way to a faster solver
                               (Sec. 6, App. A.6); the converged solution is the same. */
  PISO_PRECOND_ILU0 = 2,    /* velocity BiCGStab only: ILU(0) of C in red-black order (App. A.6
                               names ILU for BiCGStab).  Cells of one colour couple only to the
                               other colour, so the factors need no fill-in except on the
                               diagonal of the second colour: S_P = A_P - sum_F C_PF C_FP / A_F,
                               and M^-1 r is two colour sweeps.  Needs a grid that two colours
                               tile with every face between colours (even periodic extents,
                               consistent across block connections): PISO_E_ARG otherwise. */
  PISO_PRECOND_JACOBI_ILU0 = 3   /* velocity BiCGStab only: Jacobi first; if that solve ends
                               without converging (max_iter, breakdown, or a non-finite
                               residual) it is restarted with PISO_PRECOND_ILU0 (App. A.6:
                               ILU only where the plain solve fails), from the last iterate,
                               or from zero after a non-finite one.  On a grid that two
                               colours cannot tile the Jacobi result stands. */
} piso_precond;

typedef struct {
  double rtol;                     /* stop when ||b - M x||_2 <= rtol ||b||_2 (per component) */
  int32_t max_iter;                /* Krylov iterations (MIXED: inner iterations per sweep) */
  int32_t check_every;             /* iterations between convergence read-backs */
  double inner_rtol;               /* MIXED only: smallest inner float Krylov tolerance;
                                      each sweep asks for the residual reduction still
                                      needed (with a factor-2 margin), but not below this */
  int32_t max_refine;              /* MIXED only: refinement sweeps (0: the initial guess is
                                      returned with PISO_NOT_CONVERGED unless it already
                                      meets rtol) */
  int32_t precond;                 /* piso_precond; PISO_PRECOND_MG for the pressure only,
                                      PISO_PRECOND_ILU0 / _JACOBI_ILU0 for the velocity only
                                      (PISO_E_ARG otherwise) */
} piso_solve_opts;

typedef struct {
  int32_t status;                  /* PISO_OK, PISO_NOT_CONVERGED, PISO_BREAKDOWN or < 0 */
  int32_t iters;                   /* Krylov iterations (summed over components / sweeps) */
  int32_t refinements;             /* MIXED: refinement sweeps */
  int32_t fallback;                /* velocity, PISO_PRECOND_JACOBI_ILU0: 1 if the ILU(0)
                                      restart ran (iters then counts both solves) */
  double rel_residual;             /* final relative residual (max over components) */
} piso_solve_info;

typedef struct {
  piso_solve_opts vel, pres;
  int32_t n_correctors;            /* pressure correctors per step; 2 in PISO (App. A.2) */
  int32_t grad_p_in_predictor;     /* 1: b = b_u - grad p^n (eq. implEuler1); 0: b = b_u */
  int32_t grad_path_flags;         /* backward only: 1 = skip the adjoint velocity solve,
                                      2 = skip the adjoint pressure solves (Sec. 2.4) */
  int32_t adjoint_warm_start;      /* backward only: 1 = each adjoint pressure solve of
                                      piso_step_backward starts from the solution of the same
                                      corrector's solve in the previous call, or from the linear
                                      extrapolation 2 l_1 - l_2 of the solutions of the two
                                      previous calls once there are two (consecutive steps of a
                                      backward rollout have similar adjoint pressures); 0 = from
                                      zero.  The result then depends on that history within the
                                      solver tolerance; piso_adjoint_reset clears it. */
  int32_t report_flux_div;         /* forward only: 1 = fill piso_step_info.flux_div_linf (one
                                      extra flux and divergence sweep per corrector, and a
                                      synchronisation of the stream); 0 = leave it 0 */
  /* Starts of the linear solves from earlier steps of the same rollout (forward only, per
     call; device arrays of the context's element type, NULL = not given).  They change
     only where the Krylov solves start, so the result changes only within the solver
     tolerance; p_n stays the lagged pressure of eqs. implEuler1 and velCorrDiscrete.
       corrector 1 starts from  p*_{n-1} + (p_n - p_prev)   with p_prev and p_prev_star,
                                2 p_n - p_prev               with p_prev alone,
                                p_n                          otherwise;
       corrector 2 starts from  p* + (p_n - p*_{n-1})        with p_prev_star,
                                p* (corrector 1's pressure)  otherwise;
       later correctors start from the pressure of the corrector before them.
     p_star_out receives this step's p* (with one corrector: its only pressure) for the next
     step's p_prev_star.  p_star_out must not alias p_n, p_np1, p_prev or p_prev_star
     (PISO_E_ARG).  With u_prev (device [d][N]) the velocity solve starts from
     2 u_n - u_prev instead of u_n. */
  const void* p_prev;              /* the previous step's pressure p_{n-1} */
  const void* p_prev_star;         /* the previous step's first-corrector pressure p*_{n-1} */
  void* p_star_out;                /* NULL, or device [N] for this step's p* */
  const void* u_prev;              /* the previous step's velocity u_{n-1} */
} piso_step_opts;

typedef struct {
  piso_solve_info vel;
  piso_solve_info pres[2];
  /* max over cells of |sum_f N_f F_f| for the corrected face flux F of corrector 1 and of
   * the last corrector (eq. divtheorem, with the Dirichlet boundary fluxes): the
   * face-flux divergence that the correction drives to the pressure solve's residual
   * (App. A.3.5).  Filled when report_flux_div is set. */
  double flux_div_linf[2];
} piso_step_info;

/* Intermediates of the fine-grained calls; every pointer is a caller-owned device
 * buffer of the context's element type. */
typedef struct {
  void* A;      /* [N]      diagonal of C */
  void* C;      /* [2][d][N] off-diagonal face coefficients of C */
  void* b_u;    /* [d][N]   predictor right-hand side without the pressure gradient */
  void* b;      /* [d][N]   predictor right-hand side b = b_u - grad p^n */
  void* Pf;     /* [d][N]   pressure face coefficients lerp(alpha_jj / A) */
  void* Dinv;   /* [N]      inverse of the pressure matrix diagonal (Jacobi) */
  void* h;      /* [d][N]   A^-1 (b_u - H u) of the latest piso_solve_pressure */
  void* rhs;    /* [N]      divergence of h (+ boundary flux, + lag term), before mean removal */
} piso_system;

/* Gradients of the intermediates, accumulated (+=) by the backward calls. */
typedef struct {
  void* dA;     /* [N] */
  void* dC;     /* [2][d][N] */
  void* db_u;   /* [d][N] */
  void* db;     /* [d][N] */
} piso_system_grad;

/* Build a context for a block layout (Sec. 2.2, App. A.4).  Validates that every block
 * side is tiled exactly once, connections are conformal and reciprocal (matching
 * resolution, opposite sides, same orientation), J > 0; returns PISO_E_TOPOLOGY
 * otherwise.  Derives alpha_jk = J T_j . T_k (App. A.3.3) on the device and detects
 * non-orthogonal grids (max |alpha_jk| / alpha_jj > 1e-12).  Uses the current HIP device.
 * On failure *out is NULL and piso_create_error() returns the message.
 *
 * Environment read at creation (all optional; for measurement and comparison):
 *   PISO_MG_LINE=0     point Jacobi on the fine multigrid level; =1 lines wherever the
 *                      grid allows them (see piso_mg_smoother)
 *   PISO_MG_GRAPH=1    table-driven coarse-level kernels on single-block grids too
 *   PISO_NO_QUAD=1     no vectorised (four cells per thread) kernels
 *   PISO_NO_GRAPH=1    launch the PCG iterations one by one instead of replaying a graph
 *   PISO_CG_GROUPS=n   work-groups of the Krylov kernels (0 or unset: sized to the grid,
 *                      at most 2048) */
int piso_create(const piso_domain_desc* desc, int32_t precision, piso_ctx** out);
void piso_destroy(piso_ctx* ctx);
const char* piso_last_error(const piso_ctx* ctx);
const char* piso_create_error(void);

/* Sizes: cells, Dirichlet faces, bytes of one step tape (see piso_step), element bytes,
 * non-orthogonal flag. Any output pointer may be NULL. */
int piso_sizes(const piso_ctx* ctx, int64_t* n_cells, int64_t* n_bfaces, int64_t* tape_bytes,
               int64_t* elem_bytes, int32_t* non_orthogonal);

/* Shape of the multigrid hierarchy of the pressure preconditioner, built in piso_create:
 * n_levels coarse levels (0 when the grid cannot be coarsened: PISO_PRECOND_MG then
 * runs as Jacobi), and for level l = 1 .. n_levels the cell count cells[l-1] and graph
 * slots per cell slots[l-1] (host arrays of at least 16 entries, may be NULL). */
int piso_mg_info(const piso_ctx* ctx, int32_t* n_levels, int64_t* cells, int32_t* slots);

/* Fine-level smoother of the multigrid preconditioner: *line_axis = 0 for damped point
 * Jacobi, or 1 (y) / 2 (z) for damped line Jacobi along that axis (tridiagonal solves
 * along the lines).  Lines are chosen at context creation for single-block grids whose
 * sides are walls or wrap onto the block, with lines of at most 128 cells, and whose
 * metric weight along one transverse axis is on average more than 3x the largest other
 * (a grid stretched towards walls normal to that axis); PISO_MG_LINE=0 in the
 * environment at creation keeps point Jacobi, PISO_MG_LINE=1 takes lines wherever the
 * grid allows them. */
int piso_mg_smoother(const piso_ctx* ctx, int32_t* line_axis);

/* Work-groups of the plane-marching fine-grid kernels of the multigrid PCG: *groups > 0
 * when they run for this context's pressure solves, else 0.  They run on 3D grids whose
 * blocks all have nx % 4 == 0, with point smoothing on the fine level, when one field of
 * the pressure Krylov vectors (float in the F32 and MIXED forms, double in F64) takes at
 * least 8 MiB.  They compute the same iteration as the one-quad-per-thread kernels (the
 * PCG of App. A.6 with the multigrid preconditioner) in another summation order; a tile of
 * rows marches through a run of planes, its neighbours in x and y shared in LDS and those
 * in z carried from plane to plane.  PISO_ZMARCH=0 in the environment at creation keeps
 * the one-quad-per-thread kernels, PISO_ZMARCH=1 takes the marching ones at every size. */
int piso_mg_marching(const piso_ctx* ctx, int32_t* groups);

/* Default options for a precision: vel rtol 1e-7 (F32) / 1e-10 (F64, MIXED), Jacobi with
 * the ILU(0) restart on failure (PISO_PRECOND_JACOBI_ILU0);
 * pres rtol 1e-10 (F64), 1e-6 (F32), 1e-8 (MIXED), multigrid-preconditioned; MIXED inner
 * floors 1e-5 and at most 20 (pressure) / 10 (velocity) refinement sweeps; read back every
 * 4 iterations; 2 correctors, grad_p_in_predictor = 1. */
void piso_default_step_opts(int32_t precision, piso_step_opts* opts);

/* Predictor assembly (App. A.3.3-A.3.5, eqs. advMatDiscrete, difMatDiscrete,
 * velRHSdiscrete, velRHSnonOrtho) and pressure coefficients (eq. pMatDiscrete):
 * writes sys->A, C, b_u, b, Pf, Dinv.  nu: device [N] if nu_is_field else [1].
 * u_n [d][N], p_n [N], S [d][N], u_b [d][NB] (may be NULL if NB = 0).
 * grad_p_in_predictor: 1 subtracts the central gradient of p_n from b. */
int piso_assemble(piso_ctx* ctx, void* stream, const void* u_n, const void* p_n, const void* nu,
                  int32_t nu_is_field, const void* S, const void* u_b, double dt,
                  int32_t grad_p_in_predictor, const piso_system* sys);

/* Velocity predictor solve C u* = b (App. A.6: BiCGStab) for the d components at once,
 * Jacobi-preconditioned on the right, from x0 = u_star (in) to rtol; u_star [d][N]. */
int piso_solve_velocity(piso_ctx* ctx, void* stream, const piso_system* sys, void* u_star,
                        const piso_solve_opts* opts, piso_solve_info* info);

/* For callers that cannot allocate device memory at the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): piso_solve_velocity
 * with the same kernels and results, but its BiCGStab workspace (the vectors r, r-hat,
 * p, p', v, v', s, t, M^-1 p, M^-1 s [d][N], 1/A and the ILU(0) pivots [N] in the
 * context's element type, 18 partial-sum rows of 2048 doubles and the solver state)
 * taken from one fixed device array of
 * PISO_NOALLOC_SCRATCH_BYTES per GPU instead of the context's buffers.  The array is
 * part of the library's device code: each GPU the library runs on holds its own copy
 * until the process ends.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU race (serialise them, e.g. on one stream); nothing carries over
 * from one call to the next.  Needs 256-byte-aligned (10 d + 2) N elements plus the
 * partial sums and state within the array (an F64 3D grid: 256 bytes per cell, about
 * 260k cells; F32 3D: about 520k cells): PISO_E_ARG beyond that, and for PISO_MIXED
 * contexts (whose solves need the context's refinement buffers).  Calls no hipMalloc,
 * hipFree or allocating library routine. */
#define PISO_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
int piso_solve_velocity_noalloc(piso_ctx* ctx, void* stream, const piso_system* sys, void* u_star,
                                const piso_solve_opts* opts, piso_solve_info* info);

/* Pressure corrector: h = A^-1 (b_u - H u_in) (eq. pressureRHS), rhs = div h + Dirichlet
 * face flux + deferred non-orthogonal term of p_lag (eqs. pressureRHSdivDiscrete,
 * pressureRHSnonOrtho), then the zero-mean solution of P p = rhs - mean(rhs) by PCG on
 * -P (App. A.6: CG; opts->precond: Jacobi or multigrid) from x0 = p (in).  Writes
 * sys->h, sys->rhs and p. */
int piso_solve_pressure(piso_ctx* ctx, void* stream, const piso_system* sys, const void* u_in,
                        const void* u_b, const void* p_lag, void* p, const piso_solve_opts* opts,
                        piso_solve_info* info);

/* Velocity correction u_out = h - A^-1 grad p (eq. velCorrDiscrete) with central
 * differences and boundary value p_b = p_P.  If F_out [d][N] is not NULL it receives the
 * corrected face flux lerp(J T_j . h) - P_f (p_F - p_P) - cross(p_lag) of every +j face;
 * its divergence equals the pressure residual. */
int piso_correct(piso_ctx* ctx, void* stream, const piso_system* sys, const void* p,
                 const void* p_lag, const void* u_b, void* u_out, void* F_out);

/* One full PISO step (App. A.2): assemble, velocity solve from u_n, correctors with
 * pressure initial guesses p_n then p*.  Outputs u_np1 [d][N], p_np1 [N].  If tape is
 * not NULL (tape_bytes from piso_sizes), everything piso_step_backward needs is stored
 * there.  info may be NULL. */
int piso_step(piso_ctx* ctx, void* stream, const void* u_n, const void* p_n, const void* nu,
              int32_t nu_is_field, const void* S, const void* u_b, double dt, void* u_np1,
              void* p_np1, void* tape, const piso_step_opts* opts, piso_step_info* info);

/* ---- adjoint (App. A.5; each linear solve A x = b is differentiated by solving
 * A^T db = dx and dA = -db (x) x on A's sparsity, Sec. 2.3).  All gradient outputs
 * are accumulated (+=); NULL means "not requested" where stated. */

/* Adjoint of piso_correct: dh += du_out; dp += -G^T (du_out / A); dA += (grad p) . du_out / A^2. */
int piso_correct_backward(piso_ctx* ctx, void* stream, const piso_system* sys, const void* p,
                          const void* du_out, void* dh, void* dp, void* dA);

/* Adjoint of piso_solve_pressure given the gradients dh (of sys->h) and dp (of p):
 * solves P lambda = dp - mean(dp) (same PCG), then accumulates du_in, dp_lag (may be
 * NULL on orthogonal grids), du_b (may be NULL), and g->db_u, g->dA, g->dC.  p is the
 * forward solution, u_in the forward input, sys->h the forward h.  skip_solve = 1
 * takes lambda = 0 (gradient path without the pressure solve, Sec. 2.4). */
int piso_solve_pressure_backward(piso_ctx* ctx, void* stream, const piso_system* sys,
                                 const void* u_in, const void* p_lag, const void* p,
                                 const void* dh, const void* dp, void* du_in, void* dp_lag,
                                 void* du_b, const piso_system_grad* g, int32_t skip_solve,
                                 const piso_solve_opts* opts, piso_solve_info* info);

/* Adjoint of piso_solve_velocity: solves C^T mu = du_star (transposed BiCGStab), then
 * g->db += mu, g->dA += -mu . u*, g->dC += -mu (x) u* on the stencil.  skip_solve = 1
 * takes mu = 0 (Sec. 2.4). */
int piso_solve_velocity_backward(piso_ctx* ctx, void* stream, const piso_system* sys,
                                 const void* u_star, const void* du_star,
                                 const piso_system_grad* g, int32_t skip_solve,
                                 const piso_solve_opts* opts, piso_solve_info* info);

/* Adjoint of piso_assemble for the gradients in g (dA, dC, db_u, db; dPf is folded into
 * dA by piso_solve_pressure_backward): accumulates du_n, dp_n, dS, dnu ([N] if
 * nu_is_field else [1]) and du_b; any output may be NULL. */
int piso_assemble_backward(piso_ctx* ctx, void* stream, const void* u_n, const void* nu,
                           int32_t nu_is_field, const void* u_b, double dt,
                           int32_t grad_p_in_predictor, const piso_system_grad* g, void* du_n,
                           void* dp_n, void* dS, void* dnu, void* du_b);

/* Adjoint of piso_step from its tape: given du_np1 [d][N] and dp_np1 [N] (either may be
 * NULL = zero), accumulates du_n, dp_n, dS, dnu, du_b (any may be NULL).  u_n, p_n, nu,
 * u_b, dt must be the forward inputs.  opts->grad_path_flags selects Sec. 2.4 paths. */
int piso_step_backward(piso_ctx* ctx, void* stream, const void* tape, const void* u_n,
                       const void* p_n, const void* nu, int32_t nu_is_field, const void* u_b,
                       double dt, const void* du_np1, const void* dp_np1, void* du_n, void* dp_n,
                       void* dS, void* dnu, void* du_b, const piso_step_opts* opts,
                       piso_step_info* info);

/* Forget the adjoint pressure solutions kept for adjoint_warm_start: the next
 * piso_step_backward starts its adjoint pressure solves from zero.  Call at the start of
 * every backward rollout whose gradients must not depend on earlier calls (results are
 * then a function of the rollout alone, e.g. bit-identical with and without
 * checkpointing). */
int piso_adjoint_reset(piso_ctx* ctx);

/* Advective outflow boundary (App. A.4, eq. advOut), applied between steps: on the
 * Dirichlet faces with outflow[f] != 0 (device int32 [NB]) the value is advanced
 * implicitly and upwind from the face's boundary cell P,
 *     u_b* = (u_b + c u_P) / (1 + c),   c = 2 dt |T_j(P) . u_m|   (j: the face's axis),
 * with u_m the characteristic velocity (host [d]); then every outflow value is scaled
 * by s = -Q_rest / Q_out so that the net boundary flux sum_f N_f J_P T_j(P) . u_b (the
 * Dirichlet flux of the pressure right-hand side; N_f = +1 on high sides) vanishes
 * (s = 1 if Q_out = 0).  Faces without the flag keep their value.  The printed update
 * factor has the opposite sign inside its fraction, which would be anti-upwind for an
 * outflow; this is the upwind reading.  u_n [d][N], u_b and u_b_out [d][NB] (may be the
 * same buffer).  Deterministic. */
int piso_outflow_update(piso_ctx* ctx, void* stream, const void* u_n, const void* u_b,
                        const int32_t* outflow, const double* u_m, double dt, void* u_b_out);

/* Adjoint of piso_outflow_update for the gradient du_b_out of u_b_out: writes du_b
 * [d][NB] and ADDS the gradient with respect to u_n into du_n [d][N] (may be NULL to
 * skip it).  du_b must not alias du_b_out. */
int piso_outflow_update_backward(piso_ctx* ctx, void* stream, const void* u_n, const void* u_b,
                                 const int32_t* outflow, const double* u_m, double dt,
                                 const void* du_b_out, void* du_n, void* du_b);

/* Divergence-free gradient modification (Sec. 3.1, eq. SgradPsgrad) for a learned
 * source (or velocity correction) S [d][N] with incoming gradient dS [d][N]: solves the
 * extra pressure equation with the step's operators at A = 1,
 *     P(A = 1) p_S = div lerp(J T . S) - mean   (no Dirichlet flux, zero lagged
 *     pressure, x0 = 0, opts as for piso_solve_pressure),
 * and writes dS_out = dS + lambda grad p_S (the correction's central gradient with
 * p_b = p_P).  S - grad p_S then has zero corrected face-flux divergence.  p_S [N] is
 * written if not NULL.  Uses the context's step workspaces; dS_out may alias dS, not S. */
int piso_divfree_gradient(piso_ctx* ctx, void* stream, const void* S, const void* dS, double lambda,
                          const piso_solve_opts* opts, void* dS_out, void* p_S, piso_solve_info* info);

/* Online turbulence statistics over homogeneous planes (Sec. 2.5), for single-block
 * contexts (PISO_E_ARG otherwise).  The planes are normal to `axis` (0 .. d-1); every
 * accumulated step adds its cells' d velocity components to their plane.  The state is
 * a caller-owned device array of n_planes records of record_len doubles,
 * [n, mu_0 .. mu_{d-1}, C_ij for i <= j (row-major)]: sample count, mean and central
 * comoment sums; all zeros is the empty state.  piso_stats_size gives both sizes. */
int piso_stats_size(const piso_ctx* ctx, int32_t axis, int64_t* n_planes, int64_t* record_len);

/* Merge one field u [d][N] into the state: per plane, the step's mean and central sums
 * are taken in two passes and merged with the pairwise update for central comoments
 * (no raw second moments).  Deterministic. */
int piso_stats_accumulate(piso_ctx* ctx, void* stream, const void* u, int32_t axis, double* state);

/* mean [n_planes][d] and population covariance C / n [n_planes][d(d+1)/2] (i <= j,
 * row-major), device doubles. */
int piso_stats_finalize(piso_ctx* ctx, void* stream, int32_t axis, const double* state, double* mean,
                        double* cov);

/* For a non-empty final state and the gradients mean_bar, cov_bar of the finalized
 * statistics, ADDS to du [d][N] the gradient with respect to one accumulated field u:
 * mean_bar_k / n + sum_{i<=j} cov_bar_ij (delta_ik (u_j - mu_j) + delta_jk (u_i - mu_i)) / n. */
int piso_stats_backward(piso_ctx* ctx, void* stream, const void* u, int32_t axis, const double* state,
                        const double* mean_bar, const double* cov_bar, void* du);

/* Arbitrary-order online (co)moments (Sec. 2.5: differentiable moments of any order
 * accumulated without storing the sequence), for single-block contexts.  m variables per
 * sample, given as fields x [m][N] of the context's element type (m in {2, 3, 4, 6}: the
 * velocity components, or velocity and a vector such as grad p side by side), central
 * comoments of every total order 2 .. order (order 2 .. 4, at most 32 multi-indices: m <= 6
 * at order 2, m <= 4 at order 3, m <= 3 at order 4), per plane normal to `axis`.  State:
 * caller-owned device doubles, n_planes records of record_len = 1 + m + n_alpha:
 * [n, mu_0 .. mu_{m-1}, S_alpha] with S_alpha = sum over the plane's samples of
 * prod_i (x_i - mu_i)^alpha_i; a multi-index is its sorted tuple of variable indices,
 * stored by order and then lexicographically (order 2 first: (0,0), (0,1), .., the
 * covariance pairs; then (0,0,0), (0,0,1), ..).  All zeros is the empty state.  Each step
 * merges by the binomial expansion of the deviations about the combined mean (no raw
 * moments).  PISO_E_ARG for other layouts.  Deterministic. */
int piso_moments_size(const piso_ctx* ctx, int32_t axis, int32_t m, int32_t order, int64_t* n_planes,
                      int64_t* record_len);
int piso_moments_accumulate(piso_ctx* ctx, void* stream, const void* x, int32_t m, int32_t order, int32_t axis,
                            double* state);
/* mean [n_planes][m] and central moments S_alpha / n [n_planes][n_alpha], device doubles. */
int piso_moments_finalize(piso_ctx* ctx, void* stream, int32_t m, int32_t order, int32_t axis,
                          const double* state, double* mean, double* moments);
/* For a non-empty final state and the gradients mean_bar, moments_bar of the finalized
 * statistics, ADDS to dx [m][N] the gradient with respect to one accumulated field x:
 * mean_bar_k / n + sum_alpha moments_bar_alpha (alpha_k / n)
 * (dev^(alpha - e_k) - M_(alpha - e_k)), dev = x - mu, M of order 1 being zero. */
int piso_moments_backward(piso_ctx* ctx, void* stream, const void* x, int32_t m, int32_t order, int32_t axis,
                          const double* state, const double* mean_bar, const double* moments_bar, void* dx);

/* Cell-centred gradient of a field phi [ncomp][N]: out [d][ncomp][N] with
 * out[i][c] = sum_j T_ji (phi_c(P + e_j) - phi_c(P - e_j)) / 2; across a Dirichlet face
 * the neighbour is the ghost 2 phi_b - phi_P with phi_b [ncomp][NB] the face values (a
 * velocity and its u_b), or phi_P when phi_b is NULL (the pressure: the step's own
 * gradient, boundary value p_b = p_P).  The inputs of the dissipation and
 * pressure-gradient budget terms. */
int piso_field_gradient(piso_ctx* ctx, void* stream, const void* phi, int32_t ncomp, const void* phi_b,
                        void* out);

/* Turbulent energy-budget terms of Sec. 2.5 per plane normal to `axis` (the other axes
 * homogeneous; for grids whose metric is constant over each plane), from accumulated
 * moment states: state_u of u (m = d, order_u >= 3), state_grad the d states of
 * g_k = du/dx_k (m = d, order 2; [d][n_planes][record] contiguous), state_up of
 * (u, grad p) side by side (m = 2 d, order 2); wall_mean host [2][d]: the mean velocity on
 * the low and high wall of the axis (ignored on a periodic axis).  out [5][n_planes][d(d+1)/2]
 * (i <= j): production P_ij = -(R_ia dU_j/dx_a + R_ja dU_i/dx_a), dissipation
 * eps_ij = 2 sum_k cov(g_k,i, g_k,j), turbulent transport T_ij = -d<u_i'u_j'u_a'>/dx_a,
 * viscous diffusion D_ij = d^2 R_ij/dx_a^2 (without nu, as printed), velocity
 * pressure-gradient term Pi_ij = -(cov(u_i, dp/dx_j) + cov(u_j, dp/dx_i)).  Profile
 * derivatives: T_aa (f_+ - f_-)/2 and (1/J)(alpha_+ (f_+ - f) + alpha_- (f_- - f)),
 * alpha = J T_aa^2 with face weights lerp(alpha), from the plane's first cell; at a wall
 * the ghost 2 f_w - f and the face weight 2 alpha, f_w the wall mean for U and zero for
 * the fluctuation statistics.  Forward only. */
int piso_budget(piso_ctx* ctx, void* stream, int32_t axis, int32_t order_u, const double* state_u,
                const double* state_grad, const double* state_up, const double* wall_mean, double* out);

/* Diagnostics used by tests and benchmarks.  While timing is enabled, the pressure
 * solver's kernels are launched with HIP events attached to the dispatch
 * (hipExtLaunchKernelGGL) and their durations summed per kernel class; enabling resets
 * the sums.  Timing adds host work per launch: leave it off outside measurements. */
typedef enum {
  PISO_TIME_CG_STENCIL = 0,  /* PCG direction update and stencil product q = M d */
  PISO_TIME_CG_UPDATE = 1,   /* PCG x, r update */
  PISO_TIME_MG_DOWN0 = 2,    /* multigrid restriction from the fine grid */
  PISO_TIME_MG_UP0 = 3,      /* multigrid prolongation and smoothing on the fine grid */
  PISO_TIME_MG_COARSE = 4,   /* multigrid kernels on the coarse levels */
  PISO_TIME_CG_UPDATE_MG = 5, /* multigrid PCG: x, r update fused with the fine-grid
                                 pre-smoothing (point smoothing: and the restriction) */
  PISO_TIME_MG_SMOOTH0 = 6,  /* line smoothing: first pre-smoothing of a solve on the fine grid */
  PISO_TIME_KINDS = 7
} piso_time_kind;

int piso_set_timing(piso_ctx* ctx, int32_t enable);
/* Total milliseconds and launch count of one kernel class since timing was enabled. */
int piso_get_timing(piso_ctx* ctx, int32_t kind, double* ms, int64_t* calls);

#ifdef __cplusplus
}
#endif

#endif /* PISO_H */
