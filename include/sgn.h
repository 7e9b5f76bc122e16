/*
 * sgn.h -- C ABI of libsgn.so, the MI355X (gfx950) hot path of the
 * Serre-Green-Naghdi constraint solver of Feng, Shirokoff and Choi,
 * "Preconditioning and Linearly Implicit Time Integration for the
 * Serre-Green-Naghdi Equations" (arXiv 2506.16045).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are DEVICE pointers owned by the caller (for example
 *    PyTorch tensors).  The library never frees them and never keeps them past
 *    the call, except the sgn_state object, which keeps the pointers given to
 *    sgn_state_create until sgn_state_destroy.
 *  - Fields are FP64, contiguous, in the layout of section 6.1 of the paper:
 *    1D scalar fields [nx], 2D scalar fields [ny][nx] with x the fast index,
 *    x_i = i Lx / nx, y_j = j Ly / ny (doubly periodic).  Vector fields
 *    (velocity u, U = G u, grad h) are component-major: [d][ny][nx].
 *  - Grid sizes must be powers of two: 1D 2 <= nx <= 16384; 2D 2 <= nx <= 4096
 *    and 2 <= ny <= 1024.
 *  - Every call enqueues its device work on the context's HIP stream.  Calls
 *    that return scalars to the host (coefficients, solve and step info)
 *    synchronise that stream before returning.
 *  - Errors are returned as sgn_status, never thrown; sgn_last_error gives a
 *    message.  Invalid arguments are rejected before any device work starts.
 *  - A workspace (d_ws) is caller-allocated device memory of at least
 *    sgn_workspace_bytes() bytes, 256-byte aligned; its contents are scratch
 *    between calls.  Two calls that overlap in time must not share one.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef SGN_H
#define SGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sgn_status {
    SGN_OK = 0,
    SGN_EINVAL = -1,        /* bad argument (null pointer, size, option) */
    SGN_EDOMAIN = -2,       /* total depth not strictly positive, or NaN/Inf data */
    SGN_ENOCONV = -3,       /* Krylov solve hit max_iter; output holds the last iterate */
    SGN_ENOMEM = -4,        /* device allocation inside sgn_create failed */
    SGN_EDEVICE = -5,       /* a HIP runtime call failed */
    SGN_EUNSUPPORTED = -6   /* size not a power of two or above the limits */
} sgn_status;

typedef struct sgn_ctx sgn_ctx;
typedef struct sgn_state sgn_state;

/* Boundary conditions of a grid. */
typedef enum sgn_bc {
    SGN_BC_PERIODIC = 0,  /* periodic, points x_j = j L / n (section 6.1) */
    SGN_BC_WALLS = 1      /* homogeneous Neumann n.u = 0 on the walls of [0, Lx] (x [0, Ly])
                           * (Subsec:DAEform, Subsec:linop), points at the cell centres
                           * x_j = (j + 1/2) L / n; scalar fields are cosine series, each
                           * velocity component a sine series along its own axis.  Taken by
                           * sgn_bathy_prepare, sgn_precond_coeffs, sgn_apply_constraint,
                           * sgn_precond_solve, sgn_krylov_solve, sgn_rhs and the stepping
                           * states (sgn_state_create and the sgn_step_* calls; the state then
                           * keeps the reflected fields and the stepping history of the twin),
                           * and their workspace queries; the de-aliasing calls, the batched
                           * solver and the server return SGN_EUNSUPPORTED.  Sizes: 1D
                           * nx <= 8192, 2D nx <= 2048 and ny <= 512.  On 2D grids the FP64
                           * PCG solve (sgn_krylov_solve, sgn_krylov_solve_noalloc), sgn_rhs
                           * and the FP64 PCG calls of sgn_step_rk4 and sgn_step_ab run on
                           * the grid's own points in cosine / sine amplitudes; every other
                           * call (1D, mixed precision, GMRES, sgn_apply_constraint,
                           * sgn_precond_solve, the linearly implicit steps) reflects the
                           * fields (even / odd) onto the periodic grid of twice the length
                           * per axis, where the periodic path runs.  A stepping state holds
                           * both forms; a call that uses the other form than the call before
                           * restarts the initial-guess history.  The workspace queries cover
                           * both. */
} sgn_bc;

/* Grid (section 6.1): dim 1 or 2; ny and Ly are ignored when dim = 1; bc takes
 * a value of the enum above (periodic when the struct is zero-initialised). */
typedef struct sgn_grid {
    int32_t dim;
    int32_t nx;
    int32_t ny;
    double Lx;
    double Ly;
    int32_t bc;
} sgn_grid;

/* Coefficients of the preconditioner A = sigma I - alpha grad(div)  (Def:A),
 * and the bound kappa_ub of Theorem 4.1.  flat = 1 selects the flat-bottom
 * formulas (Eq:FlatbathCoeff), 0 the variable-bathymetry ones
 * (Eq:Optcoeff, Eq:Optcoeffb). */
typedef struct sgn_coeffs {
    double sigma;
    double alpha;
    double kappa_ub;
    int32_t flat;
} sgn_coeffs;

typedef enum sgn_method { SGN_PCG = 0, SGN_GMRES = 1 } sgn_method;
typedef enum sgn_precision {
    SGN_FP64 = 0,   /* every operation in FP64 */
    SGN_MIXED = 1   /* FP32 operator, FFT and preconditioner inside an FP64
                       iterative refinement: residual, dots, update in FP64 */
} sgn_precision;
typedef enum sgn_coeff_kind {
    SGN_COEFF_OPTIMAL = 0,     /* Eq:Optcoeff */
    SGN_COEFF_REPLACEMENT = 1  /* sigma**, alpha** of Remark 4.2 */
} sgn_coeff_kind;
/* Initial guesses of the solves inside the steppers (the paper leaves them
 * open).  Every such solve has a slot (RK4 stages 2, 3, 4, the final RK4
 * solve, the Adams-Bashforth solve) and a base, the most recent velocity.
 * PREVIOUS starts from the base.  EXTRAPOLATE records the slot's offset
 * o_n = solution - base and starts from base + o_{n-1} (one recorded) or
 * base + 2 o_{n-1} - o_{n-2}; the offsets are cleared when dt changes.  The
 * guess moves the start of the iteration only: every solve still stops on
 * its residual. */
typedef enum sgn_guess {
    SGN_GUESS_PREVIOUS = 0,
    SGN_GUESS_EXTRAPOLATE = 1
} sgn_guess;

typedef struct sgn_solve_opts {
    int32_t method;        /* sgn_method */
    int32_t precision;     /* sgn_precision */
    double tol;            /* stop when ||r||_2 <= tol ||b||_2 */
    int32_t max_iter;      /* Krylov iterations (inner iterations in mixed mode) */
    int32_t x0_is_guess;   /* 1: u_inout is the initial guess; 0: start from 0 */
    int32_t gmres_restart; /* GMRES restart length m, 1 <= m <= 256 */
    double inner_tol;      /* mixed mode: tightest relative tolerance of an FP32 inner solve;
                              each inner solve stops at max(inner_tol, tol ||b|| / (2 ||r||))
                              relative to the current outer residual r (at most 1/2) */
    int32_t max_outer;     /* mixed mode: refinement steps */
    int32_t check_every;   /* convergence flag read back every this many iterations (>= 1) */
    int32_t coeff_kind;    /* sgn_coeff_kind, used when coefficients are computed */
    int32_t guess;         /* sgn_guess, read by the steppers only */
} sgn_solve_opts;

typedef struct sgn_solve_info {
    int32_t iters;         /* Krylov iterations (all inner iterations in mixed mode) */
    int32_t outer_iters;   /* refinement steps (0 in FP64 mode) */
    int32_t converged;
    double relres;         /* ||b - G u||_2 / ||b||_2 as tracked by the solver */
    sgn_coeffs coeffs;     /* coefficients of A that were used */
} sgn_solve_info;

typedef struct sgn_step_info {
    int64_t solves;        /* Krylov solves performed */
    int64_t iters;         /* Krylov iterations summed over the solves */
    int32_t max_iters;     /* largest iteration count of one solve */
    int32_t converged;     /* 1 if every solve converged */
    double t;              /* simulated time of the state after the call */
    int64_t steps_done;    /* steps taken by the state since creation */
} sgn_step_info;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Allocates the FFT twiddle tables
 * and a small pinned readback buffer.  SGN_ENOMEM / SGN_EDEVICE on failure. */
sgn_status sgn_create(sgn_ctx **ctx, int device, void *hip_stream);
void sgn_destroy(sgn_ctx *ctx);
sgn_status sgn_set_stream(sgn_ctx *ctx, void *hip_stream);
const char *sgn_last_error(const sgn_ctx *ctx);
/* Library version string. */
const char *sgn_version(void);

/* Kernel timing for measurement (off by default).  Between sgn_profile_begin
 * and sgn_profile_end every launch of the kernel families below is bracketed
 * by HIP events on the context's stream; sgn_profile_end synchronises the
 * stream and returns, per family index k < nkinds, the launch count and the
 * summed event time in milliseconds (host arrays of nkinds entries).
 * The events may add a few microseconds per launch. */
typedef enum sgn_kernel_kind {
    SGN_KERNEL_PCG_C1 = 0,   /* FP64: A^{-1}, search direction, y-IFFT (column pass) */
    SGN_KERNEL_PCG_R1 = 1,   /* FP64: x-IFFT, pointwise operator, p.Gp, x-FFT (row pass) */
    SGN_KERNEL_PCG_C2 = 2,   /* FP64: y-FFT, q = G p, x and r update, r.z, r.r (column pass) */
    SGN_KERNEL_PCG_INIT = 3, /* FP64: initial residual pass */
    SGN_KERNEL_ROWS = 4,     /* generic FP64 row transforms (right-hand side etc.) */
    SGN_KERNEL_COLS = 5,     /* generic FP64 column operators */
    SGN_KERNEL_PCG_C1_F32 = 6,   /* the same PCG passes in FP32 (mixed precision) */
    SGN_KERNEL_PCG_R1_F32 = 7,
    SGN_KERNEL_PCG_C2_F32 = 8,
    SGN_KERNEL_PCG_INIT_F32 = 9,
    SGN_KERNEL_BATCH = 10,   /* batched 1D solves (one launch per call) */
    SGN_KERNEL_RHS_ROWS_FWD = 11,  /* 2D right-hand side: products and their row transforms */
    SGN_KERNEL_RHS_COLS = 12,      /* 2D right-hand side: derivative column operators */
    SGN_KERNEL_RHS_ROWS_INV = 13,  /* 2D right-hand side: inverse row transforms, pointwise eta_t, U_t, S */
    SGN_KERNEL_RHS_FLUX = 14,      /* 2D right-hand side: grad S - div(eta u (x) u) column operators */
    SGN_KERNEL_BATCH_STEP = 15,    /* whole 1D RK4 runs, one workgroup per state (one launch per call) */
    SGN_KERNEL_WALL_ORDER = 16,    /* 2D fields between walls to and from the cosine / sine transform order */
    SGN_KERNEL_KINDS = 17
} sgn_kernel_kind;
sgn_status sgn_profile_begin(sgn_ctx *ctx);
sgn_status sgn_profile_end(sgn_ctx *ctx, int64_t *launches, double *total_ms, int32_t nkinds);
/* The individual launches timed between the last sgn_profile_begin and
 * sgn_profile_end, in launch order: kinds[i] (an sgn_kernel_kind) and ms[i]
 * (event time in milliseconds) for i < min(cap, count), host arrays of cap
 * entries; *count receives the number recorded.  A Krylov pass launched after
 * its solve has converged returns at once, so a family's durations are
 * bimodal: callers that price launches by the bytes a full pass moves can
 * tell the two apart here.  SGN_EINVAL on null pointers or cap < 0. */
sgn_status sgn_profile_launches(const sgn_ctx *ctx, int32_t *kinds, float *ms, int64_t cap, int64_t *count);

/* Bytes of workspace any single call below needs for this grid and precision. */
size_t sgn_workspace_bytes(const sgn_grid *grid, int32_t precision);

/* ---- bathymetry and coefficients (section 4) --------------------------- */

/* grad h on the grid and the flat flag.  grad h is the spectral gradient D h
 * (section 6.1); a bathymetry that is exactly constant on the grid is flat and
 * gets grad h = 0 exactly (|grad h|_max = 0 selects Eq:FlatbathCoeff).
 * d_h: [ny][nx]; d_grad_h: [d][ny][nx] output; *flat: host output. */
sgn_status sgn_bathy_prepare(sgn_ctx *ctx, const sgn_grid *grid, const double *d_h,
                             double *d_grad_h, int32_t *flat, void *d_ws);

/* sigma*, alpha*, kappa_ub from eta and grad h (Eq:MaxMinWaveFields,
 * Eq:FlatbathCoeff, Eq:Optcoeff, Eq:Optcoeffb; Remark 4.2 for kind = 1).
 * SGN_EDOMAIN if min eta <= 0 or any value is not finite. */
sgn_status sgn_precond_coeffs(sgn_ctx *ctx, const sgn_grid *grid, const double *d_eta,
                              const double *d_grad_h, int32_t flat, int32_t kind,
                              sgn_coeffs *out, void *d_ws);

/* ---- operators (sections 2.2, 4, 6.1) ---------------------------------- */

/* out = G_{eta,h} u  (Def:G) with spectral derivatives.  d_eta is the total
 * depth ("h" of the operator's name), d_grad_h the bathymetry gradient
 * ("b").  d_u, d_out: [d][ny][nx]; d_out may not alias the inputs. */
sgn_status sgn_apply_constraint(sgn_ctx *ctx, const sgn_grid *grid, const double *d_eta,
                                const double *d_grad_h, const double *d_u, double *d_out,
                                void *d_ws);

/* out = A^{-1} rhs with A = sigma I - alpha grad(div)  (Def:A), diagonal in
 * Fourier space with each Nyquist wavenumber set to zero (section 6.1).
 * Only sigma and alpha of *coeffs are read; both must be > 0. */
sgn_status sgn_precond_solve(sgn_ctx *ctx, const sgn_grid *grid, const sgn_coeffs *coeffs,
                             const double *d_rhs, double *d_out, void *d_ws);

/* Solve G_{eta,h} u = rhs by a Krylov method preconditioned with A (section
 * 3.2, Eq:PCGLinSyst).  method = SGN_PCG: preconditioned conjugate gradients
 * (FP64, or FP32 inner solves with FP64 refinement for SGN_MIXED).
 * method = SGN_GMRES: right-preconditioned restarted GMRES(m) with
 * m = opts->gmres_restart, FP64 only (SGN_EUNSUPPORTED otherwise); the stop
 * test is the same, the residual estimate of the Arnoldi step ends a cycle and
 * the true residual of each restart decides; info->iters counts operator
 * applications inside Arnoldi steps.  GMRES needs the larger workspace of
 * sgn_gmres_workspace_bytes(grid, m) (the size is not checked: d_ws must be
 * at least that).  coeffs = NULL computes the coefficients from eta
 * (opts->coeff_kind).  On SGN_ENOCONV d_u_inout holds the last iterate and
 * *info is filled.  opts = NULL uses PCG, FP64, tol 1e-12, max_iter 1000, zero
 * initial guess. */
sgn_status sgn_krylov_solve(sgn_ctx *ctx, const sgn_grid *grid, const double *d_eta,
                            const double *d_grad_h, const double *d_rhs, double *d_u_inout,
                            const sgn_coeffs *coeffs, const sgn_solve_opts *opts,
                            sgn_solve_info *info, void *d_ws);

/* sgn_krylov_solve without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The call allocates nothing: its workspace
 * is a static device array of 48 MiB (50331648 bytes) that the library holds on
 * every device it runs on until the process ends (its device address is looked up
 * once per device by sgn_create).  Arguments, results and errors are those of
 * sgn_krylov_solve; in addition SGN_EINVAL if the workspace the call needs
 * (sgn_workspace_bytes, or sgn_gmres_workspace_bytes for GMRES) exceeds 48 MiB:
 * every 1D grid fits, and 2D grids up to 512 x 512.  Iteration chunks run
 * eagerly (no graph capture).  All calls on one device share the array, which
 * keeps the last call's contents (nothing in it needs to start at zero): calls
 * that overlap in time on one device race and must not be issued. */
sgn_status sgn_krylov_solve_noalloc(sgn_ctx *ctx, const sgn_grid *grid, const double *d_eta,
                                    const double *d_grad_h, const double *d_rhs, double *d_u_inout,
                                    const sgn_coeffs *coeffs, const sgn_solve_opts *opts,
                                    sgn_solve_info *info);

/* Bytes of workspace sgn_krylov_solve needs with method = SGN_GMRES and
 * restart length m (m + 1 basis vectors of the grid's half spectrum); 0 for an
 * unsupported grid or m outside [1, 256]. */
size_t sgn_gmres_workspace_bytes(const sgn_grid *grid, int32_t restart);

/* ---- batched independent 1D solves ----------------------------------------- */

/* Bytes of device workspace sgn_batch_solve needs for nitems systems of sizes
 * h_n[i] (host array) in the given precision; 0 if a size is unsupported. */
size_t sgn_batch_workspace_bytes(int32_t nitems, const int32_t *h_n, int32_t precision);

/* Solve nitems independent 1D systems G_{eta_i,h_i} u_i = rhs_i (Def:G in 1D)
 * by PCG with the preconditioner A of Def:A built per system from eta_i
 * (section 3.2, coefficients of section 4 by opts->coeff_kind, the flat
 * formulas iff h_x is identically zero), all in one kernel launch: each
 * workgroup takes whole systems, largest first, and iterates each to its own
 * stop test ||r||_2 <= tol ||rhs||_2.  opts->precision = SGN_MIXED runs FP32
 * inner solves (tolerance as for inner_tol above) inside an FP64 iterative refinement (residual,
 * stop test and u in FP64); SGN_FP64 iterates in FP64.
 *   h_n[i]   points of system i: a power of two in [2, 8192] (host array)
 *   h_L[i]   its period (host array)
 *   d_eta, d_grad_h (h_x), d_rhs, d_u_inout: device arrays packed in system
 *            order, system i at offset sum_{j<i} h_n[j]; u is the initial
 *            guess when opts->x0_is_guess (else 0) and the result on return
 *   h_info   nitems results (host array, may be NULL)
 *   d_ws     sgn_batch_workspace_bytes(...) bytes, 256-byte aligned
 * Synchronises the stream.  Every system is solved even if another fails:
 * SGN_EDOMAIN if a system had non-positive depth or non-finite data (its u
 * is left unchanged, relres NaN), else SGN_ENOCONV if a system stopped at
 * max_iter (inner) / max_outer, else SGN_OK.  opts = NULL: FP64, tol 1e-12. */
sgn_status sgn_batch_solve(sgn_ctx *ctx, int32_t nitems, const int32_t *h_n, const double *h_L,
                           const double *d_eta, const double *d_grad_h, const double *d_rhs,
                           double *d_u_inout, const sgn_solve_opts *opts, sgn_solve_info *h_info,
                           void *d_ws);

/* Bytes of device workspace sgn_batch_step_rk4 needs for nitems states of
 * sizes h_n[i] (host array) in the given precision (each state's h_x, U, stage
 * values, right-hand sides, guess offsets and solve scratch, about 40 h_n[i]
 * doubles); 0 if a size is unsupported. */
size_t sgn_batch_step_workspace_bytes(int32_t nitems, const int32_t *h_n, int32_t precision);

/* Advance nitems independent periodic 1D states by RK4 (Eq:ERK, with the
 * constraint solve of section 3.2 for the velocity of every stage and of the
 * new level), all in one kernel launch: each workgroup takes whole runs,
 * largest first, and carries its state through all of its steps.  State i
 * starts from (eta_i, u_i) over bathymetry h_i: h_x = D h (zero, and the flat
 * coefficient formulas, iff h_i is constant) and U = G_{eta,h} u are formed
 * first, and every solve starts from the guess opts->guess selects, its history
 * starting empty.  The steps are those of sgn_step_rk4 (which runs a 1D state of
 * up to 8192 points through the same kernel), and a state's result is the same,
 * bit for bit, whatever else shares the launch.
 *   h_n[i]      points of state i: a power of two in [2, 8192] (host array)
 *   h_L[i], h_dt[i], h_nsteps[i] (>= 0): its period, step and step count (host)
 *   d_h         bathymetry, device, packed in state order (state i at offset
 *               sum_{j<i} h_n[j]), read only
 *   d_eta, d_u  total depth and velocity, device, packed the same way: the
 *               initial state on entry, the state after the run on return
 *   h_info      nitems results (host array, may be NULL): solves, iterations,
 *               t = the simulated time advanced, steps_done = steps taken
 *   h_status    nitems statuses (host array, may be NULL): SGN_OK, SGN_EDOMAIN
 *               (non-positive depth or non-finite data; the run stops there)
 *               or SGN_ENOCONV (a solve missed tol; the run stops after it)
 *   d_ws        sgn_batch_step_workspace_bytes(...) bytes, 256-byte aligned
 * Synchronises the stream.  Every run proceeds even if another fails; a run
 * that stops leaves the state it reached (a failed last solve counts its step,
 * as sgn_step_rk4 does).  Returns SGN_EDOMAIN if a run met bad data, else
 * SGN_ENOCONV if a solve missed tol, else SGN_OK.  opts = NULL: FP64, tol
 * 1e-12, extrapolated guesses; method must be SGN_PCG, precision SGN_FP64 or
 * SGN_MIXED. */
sgn_status sgn_batch_step_rk4(sgn_ctx *ctx, int32_t nitems, const int32_t *h_n, const double *h_L,
                              const double *h_dt, const int32_t *h_nsteps, const double *d_h,
                              double *d_eta, double *d_u, const sgn_solve_opts *opts,
                              sgn_step_info *h_info, sgn_status *h_status, void *d_ws);

/* Right-hand side of the constraint form (Eq:DSWEcf, Def:bigF, Eq:DAE_DSWE):
 * eta_t = -div(eta u), U_t = -eta grad(zeta) - div(eta u (x) u) + F with
 * zeta = eta - h and (u.grad)^2 h read as u.grad(u.grad h).  Always FP64.
 * d_eta_t: [ny][nx]; d_U_t: [d][ny][nx]. */
sgn_status sgn_rhs(sgn_ctx *ctx, const sgn_grid *grid, const double *d_eta, const double *d_h,
                   const double *d_grad_h, const double *d_u, double *d_eta_t, double *d_U_t,
                   void *d_ws);

/* ---- time stepping (section 5) ----------------------------------------- */

/* Bytes of state workspace (stage buffers and multistep history). */
size_t sgn_state_workspace_bytes(const sgn_grid *grid, int32_t precision);

/* Bind a time-stepping state to caller-owned device fields: bathymetry h and
 * grad h (read), and eta, U = G u, u (advanced in place by the step calls).
 * U must already equal G_{eta,h} u (sgn_apply_constraint).  d_state_ws holds
 * sgn_state_workspace_bytes() bytes and d_ws sgn_workspace_bytes() bytes; both
 * stay owned by the caller and bound to the state until sgn_state_destroy. */
sgn_status sgn_state_create(sgn_ctx *ctx, const sgn_grid *grid, const double *d_h,
                            const double *d_grad_h, int32_t flat, double *d_eta, double *d_U,
                            double *d_u, void *d_state_ws, void *d_ws, sgn_state **state);
void sgn_state_destroy(sgn_state *state);

/* nsteps steps of classical RK4 (Eq:ERK) with one Krylov solve per stage
 * (4 per step).  Each solve starts from the guess opts->guess selects (opts =
 * NULL: SGN_GUESS_EXTRAPOLATE) and builds A from the current eta.  The guess
 * history stays with the state across calls with the same dt.  A failed stage
 * solve (SGN_ENOCONV, SGN_EDOMAIN) leaves the state at the last completed step;
 * a failed final solve of a step still counts the step: eta and U hold the new
 * level, u the last iterate of that solve, and t, steps_done describe them.
 * On a periodic 1D grid of up to 8192 points (plain right-hand side, PCG in
 * FP64 or mixed precision) the whole call runs in one workgroup of one kernel
 * launch (the kernel of sgn_batch_step_rk4, on this state's buffers and guess
 * history). */
sgn_status sgn_step_rk4(sgn_ctx *ctx, sgn_state *state, double dt, int32_t nsteps,
                        const sgn_solve_opts *opts, sgn_step_info *info);

/* nsteps steps of Adams-Bashforth of order 2..4 (Eq:AB, Table LMMCoeffs), one
 * Krylov solve per step.  Missing history is filled by RK4 steps with the
 * same dt; changing order or dt restarts the history, and so does a failed
 * solve (whose step counts, as in sgn_step_rk4). */
sgn_status sgn_step_ab(sgn_ctx *ctx, sgn_state *state, int32_t order, double dt,
                       int32_t nsteps, const sgn_solve_opts *opts, sgn_step_info *info);

/* nsteps steps of the linearly implicit SBDF2 scheme (Eq:MM): one A-solve per
 * step, no Krylov iteration.  fixed = NULL takes sigma*, alpha* from the
 * state's current eta (section 6.5 uses the initial data) and keeps them for
 * the life of the history; fixed coefficients other than the history's, a
 * new dt or a failed start-up step start a new history.  The first step of a
 * history is an RK4 step (solver options opts). */
sgn_status sgn_step_linimp(sgn_ctx *ctx, sgn_state *state, double dt, int32_t nsteps,
                           const sgn_coeffs *fixed, const sgn_solve_opts *opts,
                           sgn_step_info *info);

/* Third-order linearly implicit steps (Eq:IMEX_DAE; section 5.4 on
 * zero-stability): the one-parameter family
 *     c(z) = (z - r)^3,  b(z) = c(z) - (z - 1)^3,  a(z) from the third-order
 *     conditions sum_j a_j j^k = k sum_j c_j j^(k-1), k = 0..3
 * (r = 0 is SBDF3), with A scaled to theta A.  Every step is one A-solve and no
 * Krylov iteration; a history starts with the current level and two RK4 steps
 * (solver options opts).  fixed = NULL takes sigma*, alpha* from the state's eta
 * when a history starts (section 6.5) and keeps theta times them for its life;
 * another r, theta, dt or fixed starts a new history.  The scheme is zero-stable
 * (roots of Eq:CharEq inside the unit disk) for eigenvalues of (theta A)^{-1} G
 * in (1/(1 + (1+r)^3), 1/(1 - ((1+r)/2)^3)); sgn_linimp3_choose gives (r, theta)
 * covering Theorem 4.1's interval [1/kappa_ub, 1].  SGN_EINVAL unless
 * 0 <= r < 1 and theta > 0. */
sgn_status sgn_step_linimp3(sgn_ctx *ctx, sgn_state *state, double r, double theta, double dt,
                            int32_t nsteps, const sgn_coeffs *fixed, const sgn_solve_opts *opts,
                            sgn_step_info *info);

/* Joint choice of the scheme and of A's scale for sgn_step_linimp3 (host only):
 * the smallest r whose stable interval is at least kappa margin^2 wide, and theta
 * placing [1/(theta kappa), 1/theta] (the eigenvalues of (theta A)^{-1} G when
 * those of A^{-1} G lie in [1/kappa, 1]) at the interval's geometric centre, a
 * factor of at least `margin` from either end.  kappa >= 1, margin >= 1. */
sgn_status sgn_linimp3_choose(double kappa, double margin, double *r, double *theta);

/* ---- de-aliased right-hand side ------------------------------------------
 * The nonlinear terms of f(w, p) formed on a grid padded with zero modes
 * (subsec:dswe_1d, the remark on aliasing after Test 2, which reports that
 * padding the high wavenumbers with zeros helps long runs of large solitary
 * waves).  eta, u and grad h are interpolated onto the grid twice as fine per
 * axis (same domain) by zero-padding their spectra, f is evaluated there by the
 * same kernels as sgn_rhs, and eta_t, U_t are truncated back to the modes of
 * the original grid.  Both transfers keep the modes |m| < n/2 of the original
 * axis and drop its Nyquist mode (which the spectral derivative already maps to
 * zero).  Always FP64.  Grids: 1D nx <= 8192, 2D nx <= 2048 and ny <= 1024. */

/* Bytes of device workspace for the two calls below (fields on the padded grid,
 * the transfer spectra and the padded grid's right-hand-side workspace); 0 for
 * a grid that is unsupported or too large to pad. */
size_t sgn_dealias_workspace_bytes(const sgn_grid *grid);

/* The de-aliased eta_t, U_t; arguments as sgn_rhs, with d_dws of
 * sgn_dealias_workspace_bytes() bytes (contents not kept between calls).
 * SGN_EUNSUPPORTED for a grid above the limits or closed by walls. */
sgn_status sgn_rhs_dealiased(sgn_ctx *ctx, const sgn_grid *grid, const double *d_eta,
                             const double *d_h, const double *d_grad_h, const double *d_u,
                             double *d_eta_t, double *d_U_t, void *d_dws);

/* Make every later step call of the state use the de-aliased right-hand side,
 * with d_dws (sgn_dealias_workspace_bytes() bytes, owned by the caller) bound
 * to the state until it is destroyed or this is called again; d_dws = NULL goes
 * back to the plain form.  Either way a multistep (Adams-Bashforth or SBDF2)
 * history is cleared, since it holds right-hand sides of the form used so far.
 * The padded grad h is computed here, once.  SGN_EUNSUPPORTED (and the plain
 * form kept) for a grid above the limits. */
sgn_status sgn_state_set_dealias(sgn_ctx *ctx, sgn_state *state, void *d_dws);

/* ---- served execution --------------------------------------------------
 * A request server on one device.  Requests (constraint solves and RK4
 * time-steps of 1D or 2D grids) are submitted from any host thread with host
 * input arrays (copied at submission) and host output arrays (written when the
 * request completes).  A request is admitted once its device footprint (its
 * fields, Krylov workspace and stepping state) fits in the server's HBM budget
 * beside the admitted ones; admitted requests keep their fields and Krylov
 * state on the device until they complete, then release their memory.
 * Continuous batching: admitted 1D solves with nx <= 8192 are gathered into
 * one sgn_batch_solve launch whenever their batching lane is free, and admitted
 * 1D RK4 requests with nx <= 8192 into one sgn_batch_step_rk4 launch on a
 * second batching lane, so requests that arrive while a batch runs join the
 * next launch (a group shares its options; dt and nsteps may differ); every
 * other request runs on one of the worker lanes (each its own context and HIP
 * stream), so batches, solves and steps overlap on the device.  A request's
 * result does not depend on what it was batched or overlapped with (one
 * workgroup carries each batched request, and the kernels reduce in a fixed
 * order).  The lanes overlap on the device only if the process has a hardware
 * queue for each of them (lanes + 2); HIP gives a process 4 unless
 * GPU_MAX_HW_QUEUES, read when the HIP runtime starts, says otherwise. */
typedef struct sgn_server sgn_server;

typedef struct sgn_server_opts {
    size_t hbm_budget;      /* bytes; 0 = 80% of the device memory free at creation */
    int32_t lanes;          /* worker lanes (>= 1; 0 = 3) */
    int32_t max_batch;      /* most requests per batched launch (0 = 1024) */
} sgn_server_opts;

typedef enum sgn_request_kind {
    SGN_REQ_SOLVE = 0,      /* G_{eta,h} u = rhs (sgn_krylov_solve / sgn_batch_solve) */
    SGN_REQ_STEP_RK4 = 1    /* nsteps RK4 steps of (eta, u) over bathymetry h (sgn_step_rk4) */
} sgn_request_kind;

typedef struct sgn_request {
    int32_t kind;            /* sgn_request_kind */
    sgn_grid grid;
    sgn_solve_opts opts;     /* Krylov options of the solve or of every stage solve */
    const double *h_eta;     /* [N] total depth (both kinds) */
    const double *h_grad_h;  /* [d][N] bathymetry gradient (SOLVE) */
    const double *h_rhs;     /* [d][N] right-hand side (SOLVE) */
    const double *h_h;       /* [N] bathymetry (STEP) */
    const double *h_u0;      /* [d][N] initial guess (SOLVE, read iff opts.x0_is_guess) or initial velocity (STEP) */
    double dt;               /* STEP */
    int32_t nsteps;          /* STEP */
    double *h_eta_out;       /* [N] eta after the steps (STEP; may be NULL) */
    double *h_u_out;         /* [d][N] solution (SOLVE) or velocity after the steps (STEP) */
} sgn_request;

typedef struct sgn_result {
    int32_t done;            /* 1 once the outputs are written */
    int32_t status;          /* sgn_status of the request */
    int64_t iters;           /* Krylov iterations (summed over the solves of a STEP) */
    int64_t solves;
    double relres;           /* SOLVE: final relative residual */
    double t_submit, t_admit, t_start, t_done;  /* seconds on the server's clock */
    int32_t batched;         /* 1 if solved inside a batched launch */
    int32_t batch_size;      /* systems in that launch */
} sgn_result;

/* Create a server on `device`.  opts = NULL: defaults.  Starts the lanes. */
sgn_status sgn_server_create(sgn_server **server, int device, const sgn_server_opts *opts);
/* Stop accepting requests, finish the admitted and queued ones, join the lanes
 * and free every device buffer. */
void sgn_server_destroy(sgn_server *server);
/* Device bytes charged to a request while admitted (0 if the request is
 * invalid): the pooled block a worker-lane request occupies (its fields, Krylov
 * workspace and stepping state, rounded up to the pool's power-of-two size class),
 * or the fields and one-system workspace of a batched 1D solve or RK4 run. */
size_t sgn_request_footprint(const sgn_request *req);
/* Queue a request; *id identifies it.  SGN_EINVAL for an invalid request,
 * SGN_ENOMEM if its footprint exceeds the whole budget. */
sgn_status sgn_server_submit(sgn_server *server, const sgn_request *req, uint64_t *id);
/* Result of a request (done = 0 while it is queued or running); after a done
 * result has been returned the request is forgotten. */
sgn_status sgn_server_poll(sgn_server *server, uint64_t id, sgn_result *result);
/* Block until the request is done (timeout_s < 0: no limit); on timeout
 * returns SGN_OK with result->done = 0. */
sgn_status sgn_server_wait(sgn_server *server, uint64_t id, double timeout_s, sgn_result *result);
/* Requests queued, admitted and completed so far; bytes_in_use: the footprints of
 * the admitted requests not yet finished; bytes_held: the device memory the server
 * holds (pooled blocks in use or cached for reuse, and the batching lane's buffer),
 * never more than the budget (cached blocks are freed before an allocation would
 * pass it).  Any output pointer may be NULL. */
sgn_status sgn_server_stats(sgn_server *server, int64_t *queued, int64_t *admitted, int64_t *completed,
                            size_t *bytes_in_use, size_t *bytes_held, size_t *budget);

#ifdef __cplusplus
}
#endif
#endif /* SGN_H */
