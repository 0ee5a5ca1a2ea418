/*
 * mgrit.h -- C ABI of the MI355X (gfx950) library for multigrid reduction in
 * time (MGRIT) applied to method-of-lines discretizations of periodic linear
 * advection, following De Sterck, Falgout, Krzysik and Schroder,
 * "Efficient multigrid reduction-in-time for method-of-lines discretizations
 * of linear advection" (arXiv 2209.06916).
 *
 * Problem (Sec. 2.1, eq. ad):  u_t + alpha u_x = 0 on the periodic interval
 * [x_lo, x_hi), u(x,0) = u0(x).  Mesh x_i = x_lo + i h, i = 0..nx-1,
 * h = (x_hi - x_lo)/nx; time points t_n = n dt, n = 0..nt, dt = cfl*h/alpha.
 * Fine time-stepper (Sec. 4.3, eq. MOL_M_def): one Runge-Kutta step (ERKq or
 * SDIRKq) of the p-th order upwind semi-discretisation (Sec. 4.1), giving the
 * one-step system u_{n+1} = Phi u_n (eq. one-step-general).
 * Coarse time-steppers (Sec. 6.1-6.2, eqs. MOL-SL-corrected and
 * MOL-SL-corrected-multilevel): a semi-Lagrangian step followed by one
 * implicit periodic banded solve with I - phi_l D^(p+1).
 * Solver (Sec. 2.2): linear MGRIT, two-level or V-cycle, F(CF)^nu relaxation.
 *
 * Conventions for every entry point:
 *  - Every array is float64, row-major, time-major: row n of a space-time
 *    array [nt+1][nx] is time point t_n, contiguous in space.
 *  - Pointers named *_dev are device (HBM) pointers, owned by the caller and
 *    valid for the duration of the call; the library never frees them.
 *  - Work is queued on the HIP stream given to mgrit_setup (NULL = the
 *    default stream).  Calls that return host-visible results (stats, norms)
 *    synchronise that stream before returning.
 *  - A handle may be used by one host thread at a time.
 *  - Errors: a negative mgrit_status; mgrit_last_error(handle) describes the
 *    most recent failure on that handle.  Device-side failures are reported as
 *    MGRIT_EDEVICE with the HIP error string.
 */
#ifndef MGRIT_H
#define MGRIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGRIT_MAX_LEVELS 16
#define MGRIT_MAX_NX 16384 /* one spatial slab per workgroup, kept in LDS */
#define MGRIT_NOALLOC_BYTES (64u << 20) /* workspace of mgrit_solve_noalloc, per device */

typedef enum {
  MGRIT_OK = 0,
  MGRIT_ENOTCONVERGED = 1, /* max_iter reached; stats and outputs valid       */
  MGRIT_EINVAL = -1,       /* invalid argument or unsupported combination     */
  MGRIT_EUNSTABLE = -2,    /* explicit scheme above its CFL limit (Table 2)   */
  MGRIT_ENOMEM = -3,       /* device allocation failed                        */
  MGRIT_EDEVICE = -4,      /* HIP runtime error                               */
  MGRIT_EDIVERGED = -5     /* non-finite residual or growth past the limit    */
} mgrit_status;

typedef enum { MGRIT_ERK = 0, MGRIT_SDIRK = 1 } mgrit_rk_kind;

typedef enum {
  /* Psi_l = (I - phi_l D^(p+1))^{-1} S_p^(Delta_l), eq. MOL-SL-corrected-multilevel */
  MGRIT_CG_SL_CORRECTED = 0,
  /* Psi = Phi^m, the ideal coarse operator (Sec. 2.2); two levels only        */
  MGRIT_CG_IDEAL = 1,
  /* Psi_l = S_p^(Delta_l) with phi = 0 (uncorrected semi-Lagrangian)          */
  MGRIT_CG_SL_PLAIN = 2,
  /* Psi_l = the fine Runge-Kutta + upwind step at the level's step Delta_l
     (rediscretisation; Sec. 5, the comparison of Fig. 2 and Theorem 1).
     Explicit schemes must stay below their CFL limit at c * m_0 * ... * m_{l-1}. */
  MGRIT_CG_REDISC = 3
} mgrit_cg_kind;

/* The paper's problem statement (Sec. 2.1, 4.1-4.3). */
typedef struct {
  double velocity;      /* alpha > 0                                          */
  double x_lo, x_hi;    /* periodic domain [x_lo, x_hi), x_hi > x_lo          */
  int64_t nx;           /* spatial points, 1 <= nx <= MGRIT_MAX_NX            */
  int64_t nt;           /* fine time steps; nt+1 time points                  */
  double cfl;           /* c = alpha dt / h > 0                               */
  int32_t upwind_order; /* p in 1..5; the SL coarse operators need odd p      */
  int32_t rk_kind;      /* mgrit_rk_kind                                      */
  int32_t rk_order;     /* q: ERK 1..5, SDIRK 1..3 (built-in tableaux); with
                           rk_stages > 0 the order the tableau claims        */
  int32_t rk_stages;    /* 0: the built-in tableau of (rk_kind, rk_order);
                           s in 1..7: the Butcher tableau below (Sec. 4.2).
                           MGRIT_ERK needs rk_A strictly lower triangular,
                           MGRIT_SDIRK lower triangular with one diagonal
                           value gamma > 0 (singly diagonally implicit).  It
                           must satisfy the linear order conditions
                           b^T A^{j-1} 1 = 1/j!, j = 1..rk_order, to 1e-12,
                           else setup returns MGRIT_EINVAL.  Both arrays are
                           host memory, read during setup only.             */
  const double *rk_A;   /* [s][s] row-major Butcher matrix                   */
  const double *rk_b;   /* [s] weights                                        */
} mgrit_problem;

/* MGRIT parameters (Sec. 2.2, 6.3). */
typedef struct {
  int32_t max_levels;    /* 2 = two-level; more = V-cycle (<= MGRIT_MAX_LEVELS) */
  int32_t m[MGRIT_MAX_LEVELS - 1]; /* m[l] coarsens level l to l+1; a zero entry
                                      repeats the previous factor; m[0] >= 2   */
  int32_t min_coarse_nt; /* stop coarsening once nt_l <= min_coarse_nt       */
  int32_t nu;            /* CF sweeps after the first F: 0 = F, 1 = FCF      */
  int32_t cg_kind;       /* mgrit_cg_kind                                     */
  double rtol;           /* stop when ||r_it|| <= rtol ||r_0|| (e.g. 1e-10)   */
  int32_t max_iter;      /* upper bound on coarse-grid corrections           */
  double diverge_factor; /* ||r_it|| > diverge_factor ||r_0|| => EDIVERGED;
                            <= 0 disables the check                          */
  int32_t coarse_launch; /* 0: the coarse part of each V-cycle as one
                            persistent launch when it applies (it assumes its
                            workgroups are the only persistent ones resident);
                            1: one launch per pass (for handles that run
                            concurrently on several streams)                 */
  int32_t precision;     /* mgrit_precision                                   */
  double inner_rtol;     /* MGRIT_PREC_MIXED: each inner solve stops once its
                            C-point residual falls by this factor (> 0)      */
  int32_t inner_max_iter; /* MGRIT_PREC_MIXED: cap on each inner solve's
                            iterations (>= 1)                                 */
  int32_t tile_tune;     /* explicit schemes, level 0: 0 = tile width from the
                            launch-cost model; 1 = time the candidate widths
                            on the device at setup and keep the fastest
                            (cached per process by nx, m, scheme and N_c)    */
  uint64_t init_seed;    /* initial iterate when mgrit_solve gets no v_init:
                            0 = zero; otherwise every point (n, i), n >= 1,
                            that the solve reads (the C-points; in mixed
                            precision every point) is U[0,1) from SplitMix64
                            seeded with init_seed: the k-th output,
                            k = (n-1) nx + i, mixes init_seed + (k+1) *
                            0x9E3779B97F4A7C15 and keeps its top 53 bits
                            (the paper's random initial iterate, Sec. 5.3) */
  int32_t coarse_solve;  /* MGRIT_CG_SL_CORRECTED's periodic solves: 0 =
                            exact (factorised banded recurrences); 1 =
                            approximate, GMRES from a zero start on every
                            coarse-step application until the residual falls
                            by gmres_rtol or after gmres_max_iter iterations
                            (Sec. 6.3; float64 1D solves only, nx a
                            multiple of 128)                                */
  double gmres_rtol;     /* e.g. 1e-2 (two orders of magnitude)              */
  int32_t gmres_max_iter; /* 1..32; the paper: 10 (ERK1+U1), 20 (ERK3+U3,
                            ERK5+U5)                                        */
} mgrit_options;

/* Arithmetic of mgrit_solve.
 * MGRIT_PREC_FP64: the whole solve in float64.
 * MGRIT_PREC_MIXED: iterative refinement.  The outer loop runs in float64 on
 *   the device: the full space-time residual r = g - A u (one fine step per
 *   time point, all in parallel), its norm and the convergence test, and the
 *   update u += e.  Between them, MGRIT solves A e = r in float32 (every
 *   level's relaxation, residual and coarse solve; zero initial guess) until
 *   its C-point residual falls by inner_rtol, or stalls at float32 rounding
 *   (an iteration that gains less than a factor 2), or inner_max_iter.  res0 / res_final / the history
 *   are then norms of the full space-time residual, iterations counts outer
 *   iterations and inner_iterations the float32 MGRIT iterations. */
typedef enum { MGRIT_PREC_FP64 = 0, MGRIT_PREC_MIXED = 1 } mgrit_precision;

typedef struct {
  int32_t iterations;   /* coarse-grid corrections performed                 */
  double res0;          /* ||r_0||: 2-norm over all C-points, first residual */
  double res_final;     /* ||r|| at the stop                                 */
  double conv_factor;   /* res_final / previous residual (NaN if none)      */
  double *res_history;  /* caller-owned host array or NULL                   */
  int32_t res_history_cap;
  int32_t res_history_len; /* entries written (iterations + 1, capped)       */
  double t_solve_s;     /* host wall time of the solve call                  */
  int32_t inner_iterations; /* MGRIT_PREC_MIXED: float32 MGRIT iterations, all
                               outer iterations together (0 otherwise)       */
} mgrit_stats;

typedef struct {
  int64_t nt;           /* time steps on this level                          */
  int32_t m;            /* coarsening factor to the next level (0 = coarsest) */
  double shift;         /* semi-Lagrangian shift alpha*Delta_l/h (level >= 1) */
  int64_t K;            /* floor(shift)                                       */
  double eps;           /* shift - K, in [0,1)  (Sec. 3)                     */
  double phi_p;         /* coefficient of D^(p+1) in Psi_l                    */
  double phi_q;         /* coefficient of D^(q+1) (q != p only)               */
  int32_t tile_p;       /* level 0, explicit schemes: points per lane of the
                           relaxation tiles (0: no tiles)                      */
  int32_t win_L;        /* points per thread of the windowed step kernel,
                           which takes each periodic recurrence of the
                           level's banded solves by truncated carries: the
                           state entering a chunk is summed from the
                           zero-state end states of the win_D chunks before
                           it, exact to rounding because the recurrence
                           decays (setup checks the bound); 0: the step runs
                           with an exact workgroup-wide scan                 */
  int32_t win_D[2];     /* those chunk counts for the causal and the
                           anti-causal recurrence (0: none)                  */
  int32_t gmres_max_iter; /* level >= 1 with coarse_solve = 1: the GMRES
                           iteration cap of its approximate solves (0: the
                           periodic solve is exact)                          */
} mgrit_level_desc;

/* Phases timed by the optional profiler (mgrit_profile_enable). */
typedef enum {
  MGRIT_PROF_FINE_RELAX = 0, /* level-0 F/C relaxation and C-point residual   */
  MGRIT_PROF_COARSE = 1,     /* relaxation, residual and correction, levels >= 1 */
  MGRIT_PROF_FINAL = 2,      /* final F-relaxation writing the solution        */
  MGRIT_PROF_SEQUENTIAL = 3, /* mgrit_sequential                               */
  MGRIT_PROF_RESIDUAL = 4,   /* mgrit_residual                                 */
  MGRIT_PROF_OTHER = 5,      /* norm reductions, copies                        */
  MGRIT_PROF_NPHASES = 6
} mgrit_prof_phase;

typedef struct {
  int64_t launches[MGRIT_PROF_NPHASES]; /* kernel launches timed             */
  double total_ms[MGRIT_PROF_NPHASES];  /* sum of their GPU durations         */
} mgrit_profile;

typedef struct mgrit_handle mgrit_handle;

/* Validate the problem and options, build the level hierarchy (nt_0 = nt,
 * nt_{l+1} = nt_l / m_l), compute the time-stepper coefficients of every
 * level (eqs. MOL_M_def, varphi-constant-MOL-SL, MOL-SL-corrected-multilevel),
 * factorise every periodic banded operator that a step solves with, upload
 * them, and allocate the per-level device workspace (owned by the handle).
 * Returns MGRIT_EINVAL for nt % m[0] != 0, nx outside 1..MGRIT_MAX_NX, even p
 * with a semi-Lagrangian coarse operator, or an unsupported (kind, order);
 * MGRIT_EUNSTABLE for ERK above its CFL limit (on the fine level, or on a
 * rediscretised coarse level).  *out is NULL on failure. */
mgrit_status mgrit_setup(const mgrit_problem *problem, const mgrit_options *options,
                         void *hip_stream, mgrit_handle **out);

/* As mgrit_setup, with the handle's device workspace carved from the
 * caller's buffer instead of allocated: workspace_dev must be 256-byte
 * aligned and hold workspace_bytes >= mgrit_workspace_bytes(problem, options)
 * bytes; it stays owned by the caller, must stay valid until mgrit_destroy,
 * and must not be used by anything else meanwhile.  The tables are uploaded
 * on hip_stream.  MGRIT_EINVAL for a null, misaligned or too small
 * workspace; otherwise as mgrit_setup.  Neither this call nor mgrit_destroy
 * frees device memory, so neither waits for other work on the device: the
 * form for request loops that keep many solves in flight. */
mgrit_status mgrit_setup_ws(const mgrit_problem *problem, const mgrit_options *options, void *hip_stream,
                            void *workspace_dev, uint64_t workspace_bytes, mgrit_handle **out);

/* Solve the one-step system u_{n+1} = Phi u_n, u_0 = u0 (eq. one-step-general)
 * with MGRIT.
 *   u0_dev      [nx], required.
 *   v_init_dev  [nt+1][nx] initial iterate; only its C-points (rows
 *               k*m[0]) are read, row 0 is replaced by u0.  NULL: the
 *               seeded U[0,1) iterate of options.init_seed, or zero when
 *               init_seed is 0 (the 2D solve always takes zero).
 *   u_out_dev   [nt+1][nx] receives the final iterate at every time point,
 *               or NULL.
 *   u_final_dev [nx] receives row nt of the final iterate, or NULL.
 *   stats       optional.
 * Returns MGRIT_OK on convergence, MGRIT_ENOTCONVERGED at max_iter (outputs
 * hold the last iterate), MGRIT_EDIVERGED on a non-finite or growing residual.
 * With MGRIT_PREC_MIXED the iterate is the whole space-time array: v_init
 * (every row, row 0 replaced by u0) or zero, kept in u_out_dev when given
 * (else in the handle's workspace); max_iter bounds the outer iterations. */
mgrit_status mgrit_solve(mgrit_handle *h, const double *u0_dev, const double *v_init_dev,
                         double *u_out_dev, double *u_final_dev, mgrit_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * float64 solve as mgrit_setup + mgrit_solve + mgrit_destroy in one call that
 * allocates nothing.  Its workspace is one file-scope device array of
 * MGRIT_NOALLOC_BYTES per GPU, kept until the process ends; every call on a
 * GPU reuses that GPU's array, so calls that overlap on one GPU (from several
 * threads or streams) race and must be serialised by the caller.  Arguments
 * as mgrit_setup and mgrit_solve (the caller owns u0_dev, v_init_dev,
 * u_out_dev, u_final_dev and stats); work runs on hip_stream and the call
 * synchronises it, the host waiting for each iteration's stopping decision.
 * MGRIT_EINVAL, with mgrit_last_error(NULL) saying why, for a problem whose
 * workspace (mgrit_workspace_bytes) exceeds MGRIT_NOALLOC_BYTES, for
 * MGRIT_PREC_MIXED and for tile_tune != 0; other outcomes as mgrit_solve. */
mgrit_status mgrit_solve_noalloc(const mgrit_problem *problem, const mgrit_options *options, void *hip_stream,
                                 const double *u0_dev, const double *v_init_dev, double *u_out_dev,
                                 double *u_final_dev, mgrit_stats *stats);

/* The same solve in steps, for request loops that keep several solves in
 * flight (one handle and one stream each).  mgrit_solve_start queues the
 * start and the first iteration; mgrit_solve_advance never blocks: once the
 * last queued iteration's stopping test has run it queues the next iteration,
 * or the outputs and sets *done = 1; mgrit_solve_finish waits for the solve to
 * end (driving it if needed), fills stats and returns the status mgrit_solve
 * would have returned.  Arguments as for mgrit_solve; the device buffers must
 * stay valid until mgrit_solve_finish returns.  One solve at a time per handle
 * (MGRIT_EINVAL otherwise).  mgrit_solve is start + finish.  Mixed-precision
 * handles advance one float32 inner iteration (or one outer step) per
 * decision; stats.iterations counts the outer steps. */
mgrit_status mgrit_solve_start(mgrit_handle *h, const double *u0_dev, const double *v_init_dev, double *u_out_dev,
                               double *u_final_dev);
mgrit_status mgrit_solve_advance(mgrit_handle *h, int32_t *done);
mgrit_status mgrit_solve_finish(mgrit_handle *h, mgrit_stats *stats);

/* Host-only: an upper bound on the device memory (bytes) the handle of
 * (problem, options) allocates, in one piece, at mgrit_setup (C-point and
 * residual arrays of every level, norm partials, tables); the caller's own
 * buffers (u0, v_init, outputs) are not included. */
mgrit_status mgrit_workspace_bytes(const mgrit_problem *problem, const mgrit_options *options, uint64_t *bytes);

/* Space-time residual of an arbitrary iterate u_dev [nt+1][nx] of the fine
 * system: r_n = Phi u_{n-1} - u_n, n = 1..nt, one fine step per time point,
 * all in parallel.  r_dev [nt][nx] (row n-1 holds r_n) or NULL;
 * *norm2_host (optional) receives ||r||_2 over all n and i. */
mgrit_status mgrit_residual(mgrit_handle *h, const double *u_dev, double *r_dev, double *norm2_host);

/* Sequential time-stepping (eq. one-step-general): u_out_dev [nt+1][nx] with
 * row 0 = u0 and row n = Phi row n-1.  The baseline MGRIT is compared with. */
mgrit_status mgrit_sequential(mgrit_handle *h, const double *u0_dev, double *u_out_dev);

/* Apply the level-l time-stepper nsteps times to each of `count` independent
 * vectors: v_out[b] = Phi_l^nsteps v_in[b]; v_in_dev, v_out_dev [count][nx]
 * (may alias).  Level 0 is the fine step; level l >= 1 is Psi_l. */
mgrit_status mgrit_apply_step(mgrit_handle *h, int32_t level, const double *v_in_dev,
                              double *v_out_dev, int64_t count, int32_t nsteps);

/* Number of levels of the hierarchy built by mgrit_setup (>= 2). */
int32_t mgrit_num_levels(const mgrit_handle *h);

/* Description of level `level` (0 = fine). */
mgrit_status mgrit_level_info(const mgrit_handle *h, int32_t level, mgrit_level_desc *out);

/* Host-only: two-level LFA convergence estimate of eq. (rho-asym) for the
 * problem's fine step and the options' first coarsening factor and coarse
 * operator, with 2^11 spatial frequencies minus the 11 nearest omega = 0. */
mgrit_status mgrit_lfa_rho(const mgrit_problem *problem, const mgrit_options *options, double *rho);

/* Tracing: time every kernel launch of the phases in `phase_mask` (bit
 * 1 << mgrit_prof_phase) with a pair of HIP events on the handle's stream;
 * 0 disables.  Durations are collected whenever the library synchronises the
 * stream.  Adds two event records per timed launch, nothing else. */
mgrit_status mgrit_profile_enable(mgrit_handle *h, uint32_t phase_mask);
/* Copy the accumulated counts and durations; reset them if reset != 0. */
mgrit_status mgrit_profile_read(mgrit_handle *h, mgrit_profile *out, int32_t reset);

const char *mgrit_status_string(mgrit_status s);
const char *mgrit_last_error(const mgrit_handle *h);
/* Waits for the work queued on the handle's stream, then releases the handle
 * (its own workspace with hipFree; a caller's workspace stays the caller's). */
void mgrit_destroy(mgrit_handle *h);

/* ------------------------------------------------------------------------
 * 2D extension: u_t + a_x u_x + a_y u_y = 0 on a periodic rectangle.  The
 * paper is one-dimensional; this follows one reading of it:
 *  - fine step: one explicit Runge-Kutta step (ERK1..5) of the
 *    dimension-split semi-discretisation -(c_x L_p^(x) + c_y L_p^(y)), the 1D
 *    upwind stencil of Sec. 4.1 along each axis, c_x = a_x dt / h_x,
 *    c_y = a_y dt / h_y;
 *  - coarse step on level l: the 1D corrected semi-Lagrangian step of eq.
 *    (MOL-SL-corrected-multilevel) along x with the coefficients of the 1D
 *    problem at CFL c_x, then the same along y for c_y (a tensor-product
 *    semi-Lagrangian step and one periodic banded solve per grid line in
 *    each direction);
 *  - MGRIT as in the 1D solver (Sec. 2.2): F(CF)^nu relaxation, C-point
 *    residual, V-cycle, sequential coarsest level, float64 throughout.
 * Space-time arrays are [nt+1][ny][nx] float64, x contiguous.
 * ---------------------------------------------------------------------- */
typedef struct {
  double velocity_x, velocity_y; /* a_x, a_y > 0                              */
  double x_lo, x_hi, y_lo, y_hi; /* periodic rectangle                        */
  int64_t nx, ny;                /* points per axis, 1 <= n <= MGRIT_MAX_NX   */
  int64_t nt;                    /* time steps                                */
  double dt;                     /* time step > 0                             */
  int32_t upwind_order;          /* p in {1, 3, 5} (the coarse step needs odd p) */
  int32_t rk_order;              /* ERK order q in 1..5                       */
} mgrit2d_problem;

typedef struct mgrit2d_handle mgrit2d_handle;

/* Validate, build the hierarchy from options (max_levels, m, min_coarse_nt,
 * nu, rtol, max_iter, diverge_factor, precision, inner_rtol, inner_max_iter;
 * cg_kind must be MGRIT_CG_SL_CORRECTED, else MGRIT_EINVAL),
 * factorise the x- and y-line operators of every coarse level and allocate
 * the workspace (owned by the handle).  MGRIT_EUNSTABLE when the fine step's
 * amplification factor exceeds 1 on a 256 x 256 grid of frequencies. */
mgrit_status mgrit2d_setup(const mgrit2d_problem *problem, const mgrit_options *options, void *hip_stream,
                           mgrit2d_handle **out);
/* MGRIT solve; arguments and statuses as mgrit_solve, with [ny][nx] slabs:
 * u0_dev [ny][nx]; v_init_dev [nt+1][ny][nx] or NULL (zero; only C-points
 * are read); u_out_dev [nt+1][ny][nx] or NULL; u_final_dev [ny][nx] or NULL.
 * MGRIT_PREC_MIXED as for mgrit_solve: float32 2D MGRIT on the correction
 * equation inside float64 refinement (the whole space-time array is the
 * iterate, v_init's every row is read). */
mgrit_status mgrit2d_solve(mgrit2d_handle *h, const double *u0_dev, const double *v_init_dev, double *u_out_dev,
                           double *u_final_dev, mgrit_stats *stats);
/* Sequential time-stepping of the fine step: u_out_dev [nt+1][ny][nx]. */
mgrit_status mgrit2d_sequential(mgrit2d_handle *h, const double *u0_dev, double *u_out_dev);
/* count slabs: v_out = step_level(v_in) (level 0 = fine; v_in and v_out may
 * not overlap). */
mgrit_status mgrit2d_apply_step(mgrit2d_handle *h, int32_t level, const double *v_in_dev, double *v_out_dev,
                                int64_t count);
int32_t mgrit2d_num_levels(const mgrit2d_handle *h);
const char *mgrit2d_last_error(const mgrit2d_handle *h);
void mgrit2d_destroy(mgrit2d_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* MGRIT_H */
