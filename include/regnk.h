/*
 * regnk.h -- C ABI of the MI355X (gfx950) reduced-space Gauss-Newton-Krylov library for 2D
 * diffeomorphic image registration (Mang & Biros, "Constrained H1-regularization schemes for
 * diffeomorphic image registration", SIAM J. Imaging Sci. 9(3), 2016).
 *
 * Problem (Sec. 2, eq. (opt-prob-v)): find a stationary velocity v on the periodic domain
 * [0, 2 pi)^2 that minimises
 *     J[v] = 1/2 ||m_R - m_1||^2 + 1/2 beta_v |v|^2_V + gamma 1/2 beta_w ||div v||^2_{H1}
 * subject to the transport equation d_t m + grad m . v = 0, m(0) = m_T (eq. (transport-eq)) and,
 * for gamma = 1, the divergence constraint (eq. (constraint-divv)), which is eliminated through the
 * projection K of Sec. 3.3, eq. (project-body-force).
 *
 * Conventions shared by every entry point
 *  - Return value: reg_status (REG_OK = 0).  No C++ exception crosses the ABI; on error
 *    reg_last_error() returns a thread-local message.
 *  - Array arguments are DEVICE pointers (HIP global memory) owned by the caller.  They must stay
 *    valid until the call's work on the problem's stream has finished.  Calls that return host
 *    scalars synchronise that stream before returning; the others only enqueue work.
 *  - Layout: a scalar field is double[n1][n2], row-major (i2 fastest), sample (i1, i2) at
 *    x = (2 pi i1 / n1, 2 pi i2 / n2).  A vector field is double[2][n1][n2] (component-major).
 *  - Every velocity-like input (v, v~, r) has its Nyquist row and column (k1 = n1/2, k2 = n2/2)
 *    removed before use, and every velocity-like output has none (spectral derivatives use the
 *    Nyquist wavenumber 0 so that they are exactly skew-symmetric).
 *  - Sizes: n1, n2 even in [8, 2048]; nt >= 1; beta_v > 0; beta_w > 0 exactly when
 *    constraint == REG_MASS_SOURCE.  Anything else is REG_EINVAL.  Powers of two take the
 *    register FFT kernels; other lengths of the form 2^a 3^b 5^c take mixed-radix (2, 3, 4, 5, 8)
 *    FFTs staged in LDS; the remaining even lengths take direct O(n^2)-per-line spectral sums along
 *    that axis (same operators, slower).
 */
#ifndef REGNK_H
#define REGNK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    REG_OK = 0,
    REG_EINVAL = -1,      /* bad argument, size or parameter combination */
    REG_ENOMEM = -2,      /* workspace too small */
    REG_EDEVICE = -3,     /* a HIP runtime call failed */
    REG_ENOTCONV = -4,    /* line search failed / iteration limit with a failure condition */
    REG_ENONFINITE = -5,  /* a reduction produced NaN or Inf */
    REG_ESTATE = -6       /* Hessian matvec requested before any linearisation point was set */
} reg_status;

/* Seminorm on v (Sec. 2, eq. (reg-v)); A = -Lap (H1) or Lap^2 (H2), eq. (var-reg-v); REG_H3 is the
 * H3 seminorm the paper names as an option (A = -Lap^3, a triharmonic reduced gradient). */
enum { REG_H1 = 1, REG_H2 = 2, REG_H3 = 3, REG_STOKES = 4 };
/* REG_STOKES: the nonlinear Stokes (shear-control) model of eq. (shear-control-reg-v),
 * beta_v R(v) with R(v) = 2nu/(nu+1) int (E:E + eps)^{(1+nu)/(2nu)}, E = sym grad v; its first
 * variation -div(2 eta E) (eq. (1st-var-reg-v-nls)) and second variation (eq. (2nd-var-reg-v-nls))
 * enter the gradient and the Hessian, projected together with the body force under
 * REG_DIVFREE; the preconditioner is the inverse vector Laplacian (App. E.2).  nu = stokes_nu > 0
 * (nu > 1 thins, nu < 1 thickens under shear), eps = stokes_eps > 0 keeps eta finite where the
 * strain vanishes.  With REG_MASS_SOURCE (relaxed incompressibility, App. A) the projection is
 * K[b, v] with M = 2 beta_v eta_bar (beta_w(-Lap + I))^{-1} + I, eta_bar the mean viscosity at the
 * linearisation point, applied to b, beta_v times the first (second) variation and the gradient
 * (Hessian) of 1/2 beta_w <div v, (1 - Lap) div v>; PCG then uses <K^{-1} ., .> with that K, and the
 * low-rank preconditioner correction is not available (REG_EINVAL). */
/* Constraint on div v (Sec. 2): gamma = 0; gamma = 1 with w = 0 (incompressible); gamma = 1 with a
 * mass source w penalised by its H1 norm (eq. (reg-w)), beta_w > 0. */
enum { REG_UNCONSTRAINED = 0, REG_DIVFREE = 1, REG_MASS_SOURCE = 2 };
/* Arithmetic of the transport solves and FFTs: FP64 throughout, or FP32 transport with FP64
 * spectral assembly, reductions and Krylov vectors. */
enum { REG_FP64 = 0, REG_FP32_TRANSPORT = 1 };
/* Time quadrature of the body forces (Sec. 4): REG_ADJ_DISCRETE uses the quadrature that is the
 * exact transpose of the discrete RK2 forward map (exact gradient, symmetric Hessian);
 * REG_ADJ_PAPER uses the trapezoidal rule as printed. */
enum { REG_ADJ_DISCRETE = 0, REG_ADJ_PAPER = 1 };

/* Hessian of the matvec and of the solve's Newton steps.  REG_HESS_GN: the Gauss-Newton
 * approximation of Sec. 4 (every term that carries lam dropped; positive definite).  REG_HESS_FULL:
 * an extension -- eq. (inc-control-eq-elim) with the div(lam v~) term of eq. (inc-adj-eq-elim) and the
 * lam grad m~ term of the incremental body force kept, discretised as the exact derivative of the
 * REG_ADJ_DISCRETE gradient (the Hessian of the discrete objective: symmetric, possibly indefinite
 * away from a minimiser, where PCG stops at the first direction of non-positive curvature).  Needs
 * REG_ADJ_DISCRETE; the workspace also holds the adjoint stage values (2 n_t fields) and the
 * incremental-state gradients (2 n_t vector fields) in the transport precision. */
enum { REG_HESS_GN = 0, REG_HESS_FULL = 1 };

typedef struct {
    int32_t n1, n2;       /* grid (even, 8..2048; powers of two are the fast path) */
    int32_t nt;           /* RK2 time steps on [0, 1] */
    int32_t norm;         /* REG_H1 | REG_H2 | REG_H3 | REG_STOKES */
    int32_t constraint;   /* REG_UNCONSTRAINED | REG_DIVFREE | REG_MASS_SOURCE */
    int32_t precision;    /* REG_FP64 | REG_FP32_TRANSPORT */
    int32_t adjoint;      /* REG_ADJ_DISCRETE | REG_ADJ_PAPER */
    int32_t hessian;      /* REG_HESS_GN | REG_HESS_FULL */
    int32_t lowrank_capacity; /* 0..64: directions the low-rank preconditioner correction of
                                 reg_solve can hold (workspace grows by 2 vector fields per direction,
                                 4 for REG_MASS_SOURCE); 0 = no correction */
    int32_t nt_max;       /* 0, or nt..4096: the largest n_t that reg_solve's CFL adaptation
                             (reg_solve_opts.cfl_max) may raise n_t to; the workspace holds the
                             trajectory of max(nt, nt_max) steps */
    double beta_v;        /* weight of the v seminorm (> 0) */
    double beta_w;        /* weight of the mass-source norm (> 0 iff REG_MASS_SOURCE) */
    double stokes_nu;     /* REG_STOKES: nu > 0; otherwise 0 */
    double stokes_eps;    /* REG_STOKES: eps > 0; otherwise 0 */
} reg_params;

typedef struct reg_problem reg_problem;   /* opaque handle */

/* Bytes of device workspace a problem with these parameters needs (host-only, no device work). */
reg_status reg_workspace_bytes(const reg_params* params, size_t* bytes);

/* Create a problem.  m_T (template) and m_R (reference) are device scalar fields; they are copied
 * into `workspace` (device memory of at least reg_workspace_bytes bytes, 256-byte aligned, owned
 * by the caller and kept alive until reg_destroy).  The template is used as given (callers
 * normalise intensities to [0, 1] as in Sec. 4).  All work is enqueued on `hip_stream`
 * (hipStream_t; NULL = default stream).  The library allocates no device memory of its own. */
reg_status reg_create(const reg_params* params, const double* m_T, const double* m_R,
                      void* workspace, size_t workspace_bytes, void* hip_stream,
                      reg_problem** out);

/* Release the handle (the workspace stays the caller's). */
reg_status reg_destroy(reg_problem* h);

/* Replace the image pair of an existing problem (same grid and parameters): m_T, m_R are copied
 * and checked as in reg_create; the linearisation point is dropped.  Captured launch graphs and
 * tuned launch shapes stay valid, so one handle can serve a stream of pairs.  Synchronises. */
reg_status reg_set_images(reg_problem* h, const double* m_T, const double* m_R);

/* Change the stream subsequent calls enqueue on. */
reg_status reg_set_stream(reg_problem* h, void* hip_stream);

/* Deformed template m_1 = m(t = 1): one state solve forward in time (Sec. 3.3, eq. (state-eq-elim),
 * RK2 as in Sec. 4).  v: device vector field; m1: device scalar field (output). */
reg_status reg_state_forward(reg_problem* h, const double* v, double* m1);

/* Objective J(v) of Sec. 2, eq. (objective): one state solve.  J_host: host double (output);
 * terms3_host (nullable): host double[3] = {data, reg_v, reg_w}.  Synchronises the stream. */
reg_status reg_objective(reg_problem* h, const double* v, double* J_host, double* terms3_host);

/* Reduced gradient g = beta_v A v + K[b], b = int_0^1 lam grad m dt (Sec. 3.3, eq. (control-eq-elim)):
 * state solve forward, adjoint solve backward (eq. (adj-eq-elim)) and the body-force quadrature.
 * Also makes v the linearisation point of later Hessian matvecs (the state trajectory and its
 * gradients stay in the workspace).  g: device vector field (output); J_host (nullable) receives
 * J(v) (then the stream is synchronised). */
reg_status reg_gradient(reg_problem* h, const double* v, double* g, double* J_host);

/* Gauss-Newton reduced Hessian matvec at the current linearisation point (Sec. 3.3,
 * eq. (inc-control-eq-elim) with B = A and L = K; Gauss-Newton as in Sec. 4: the lam terms are
 * dropped):  H v~ = beta_v A v~ + K[b~], where b~ = int_0^1 lam~ grad m dt comes from one incremental
 * state solve forward (eq. (inc-state-eq-elim)) and one incremental adjoint solve backward
 * (eq. (inc-adj-eq-elim)).  vtilde, Hvtilde: device vector fields (may not alias).
 * REG_ESTATE if no linearisation point has been set by reg_gradient / reg_solve. */
reg_status reg_hessian_matvec(reg_problem* h, const double* vtilde, double* Hvtilde);

/* Preconditioner of App. E.2: z = (beta_v A)^{-1} r, with the kernel of A (the mean, k = 0)
 * scaled by 1/beta_v.  r, z: device vector fields (may alias). */
reg_status reg_precond_apply(reg_problem* h, const double* r, double* z);

/* Newton step of Alg. 2: PCG on H x = rhs at the current linearisation point, x_0 = 0, stopping at
 * ||r|| <= eta ||rhs|| or after max_iters iterations; fixed_iters > 0 runs exactly that many.
 * For REG_MASS_SOURCE the PCG inner product is <K^{-1} a, b>, in which H is self-adjoint.
 * Where the assembly's column pass can form P^{-1} H s (power-of-two grids with 64..512-point
 * columns, no low-rank correction), z = P^{-1} r and K^{-1} r follow r by recurrence and are formed
 * from r afresh at the start and every eighth iteration; the iterates equal those of the textbook
 * iteration up to rounding.  If <s, H s>_W <= 0 the iteration stops (a fixed schedule keeps
 * launching with x and r held).
 * x: device vector field (output).  iters_host, relres_host: host outputs (nullable).
 * Synchronises the stream. */
reg_status reg_pcg(reg_problem* h, const double* rhs, double eta, int32_t max_iters,
                   int32_t fixed_iters, double* x, int32_t* iters_host, double* relres_host);

typedef struct {
    int32_t max_newton;       /* outer iterations (Alg. 1) */
    int32_t max_pcg;          /* inner iterations per Newton step (Alg. 2) */
    int32_t fixed_pcg_iters;  /* > 0: exactly this many PCG iterations, no forcing-term test */
    int32_t max_backtracks;   /* Armijo halvings before REG_ENOTCONV */
    double gtol_rel;          /* stop when ||g(v_k)|| / ||g(0)|| <= gtol_rel */
    double armijo_c1;         /* sufficient-decrease constant (1e-4) */
    double armijo_rho;        /* backtracking factor (0.5) */
    const double* v0;         /* nullable device vector field: warm start (kept if J(v0) < J(0),
                                 otherwise the solve starts from v = 0: stats.fallback_used) */
    /* Low-rank correction of the PCG preconditioner (an extension; the paper uses the spectral
     * preconditioner alone).  A set of directions z_k with H z_k and e_k = <z_k, H z_k>_W > 0 turns
     * M^{-1} = (beta_v A)^{-1} into the balancing (deflation) preconditioner
     *   P r = Pi M^{-1} Pi^* r + sum_k z_k <z_k, r>_W / e_k,   Pi = I - sum_k z_k <H z_k, .>_W / e_k,
     * which is SPD in <., .>_W for any such set and maps span{z_k} to itself under P H.  The set is
     * built in two ways, both bounded by params.lowrank_capacity: */
    const double* precond_U;  /* nullable device [rank][2][n1][n2]: caller directions.  At the
                                 point where the first Newton step is taken their admissible parts
                                 (Nyquist-free; Leray-projected for REG_DIVFREE) are orthonormalised
                                 in <., M .>_W (near-dependent ones dropped), H is applied to that
                                 basis (one matvec each, counted in stats) and Rayleigh-Ritz gives the
                                 z_k; Ritz values <= 0 are dropped. */
    double* precond_d;        /* nullable host [rank] (output): the kept Ritz values theta_k of H
                                 relative to M, ascending, then zeros */
    int32_t rank;             /* 0..min(8, lowrank_capacity) caller directions */
    int32_t recycle;          /* >= 0: the first `recycle` search directions of each Newton step's
                                 PCG solve (mutually H-conjugate) are added to the set for the later
                                 steps, until it is full; no extra matvecs.  Needs capacity > 0. */
    /* CFL-adapted n_t (Sec. 4 adapts the number of time steps by monitoring the CFL condition of the
     * explicit RK2 steps; Sec. 5 starts from n_t = 2 max(n1, n2)).  cfl_max > 0: before the first
     * Newton step and after every accepted one, C(v) = h_t (max|v_1| n1/2 + max|v_2| n2/2) of the
     * iterate is checked; when C > cfl_max, n_t is raised to the smallest value with C <= cfl_max
     * (at most params.nt_max) and the problem is re-linearised at the same v (J and g change with
     * n_t; g(0) does not).  n_t never decreases; the new n_t stays with the handle after the solve.
     * 0 = n_t fixed. */
    double cfl_max;
    /* Per-Newton-step records (nullable): step k < max_steps fills steps[k] (host memory) once the
     * step ends, also a step whose line search fails (alpha = 0).  Costs one host round trip per
     * step for C(v). */
    struct reg_step_record* steps;
    int32_t max_steps;        /* >= 0; 0 = no records */
} reg_solve_opts;

/* One Newton step of reg_solve (Alg. 1): the quantities the paper reports per iteration and the
 * step's cost. */
typedef struct reg_step_record {
    int32_t newton_iter;      /* k, from 0 */
    int32_t pcg_iters;        /* PCG iterations of the step's Newton system */
    int32_t backtracks;       /* Armijo reductions of the step length */
    int32_t nt;               /* n_t after the step's CFL check */
    double J;                 /* objective at the new iterate (the old one if the search failed) */
    double g_rel;             /* ||g|| / ||g(0)|| at that iterate */
    double alpha;             /* accepted step length; 0 if the line search failed */
    double cfl;               /* C(v) of that iterate at n_t (see reg_cfl) */
    double ms;                /* host wall time of the step, host round trips included */
} reg_step_record;

typedef struct {
    int32_t newton_iters, pcg_iters, n_matvec, n_pde, backtracks, status;
    int32_t fallback_used;    /* 1: the warm start v0 did not lower J below J(0); solved from v = 0 */
    int32_t lowrank_dim;      /* directions in the preconditioner correction when the solve ended */
    double g0_norm;           /* ||g(0)|| at v = 0 (also for a warm start) */
    double g_rel;             /* final ||g|| / ||g(0)|| */
    double J;                 /* final objective */
    double cfl;               /* CFL number of the final velocity (see reg_cfl) at the final n_t */
    int32_t nt;               /* n_t at the end of the solve (differs from params.nt after a CFL
                                 adaptation) */
    int32_t nt_changes;       /* how many times the CFL adaptation raised n_t */
} reg_solve_stats;

/* Alg. 1: globalised inexact reduced-space Gauss-Newton-Krylov solve from v0 (or 0): PCG Newton
 * steps (Alg. 2, forcing term eta_k = min(1/2, sqrt(||g_k|| / ||g(0)||))) and Armijo backtracking
 * (Sec. 4).  v_out: device vector field (output); stats_host: host (nullable).  Leaves the final
 * v as the linearisation point.  Synchronises the stream. */
reg_status reg_solve(reg_problem* h, const reg_solve_opts* opts, double* v_out,
                     reg_solve_stats* stats_host);

/* Batched Alg. 1: solve `count` independent problems (any mix of sizes, steps and weights), pair i
 * with opts[i] into v_out[i] (device vector field of that problem's size), stats into
 * stats_host[i] (nullable).  Pairs run concurrently on up to eight internal streams (the environment
 * variable REGNK_BATCH_WORKERS, 1..32, sets another count), largest first; each problem's own stream is synchronised before its solve starts, and every solve has
 * finished when the call returns.  A problem may appear only once.  Returns the first failure
 * (REG_ENOTCONV after all others); stats carry each pair's own status. */
reg_status reg_batch_solve(int32_t count, reg_problem* const* problems, const reg_solve_opts* opts,
                           double* const* v_out, reg_solve_stats* stats_host);

/* CFL number of a velocity for this problem's current n_t (Sec. 4: the explicit RK2 steps are only
 * conditionally stable, and the paper monitors the CFL condition to adapt n_t):
 * C = h_t (max|v_1| n1/2 + max|v_2| n2/2), the largest |h_t k . v| over the resolved modes, of the
 * Nyquist-projected v.  reg_solve adapts n_t itself with reg_solve_opts.cfl_max.  v: device vector
 * field; cfl_host: host double.  Synchronises the stream. */
reg_status reg_cfl(reg_problem* h, const double* v, double* cfl_host);

/* Leading generalised eigenpairs of (H, M) at the current linearisation point, H the Hessian of
 * reg_hessian_matvec and M the preconditioner of reg_precond_apply (an extension: the training
 * targets of the learned low-rank correction, regnet.h).  Subspace iteration: Rayleigh-Ritz on
 * span(U) exactly as reg_solve does for precond_U (admissible parts, orthonormal in <., M .>_W,
 * Ritz pairs with theta <= 0 dropped), then U <- M^{-1} H z_k, repeated `iters` times (0..100);
 * each repetition damps the components along smaller theta by their ratio to the kept ones.
 * U: device [rank][2][n1][n2], in: the starting directions, out: the Ritz vectors in descending
 * order of theta, M-orthonormal with plain grid sums (sum over points of z_i . M z_j = delta_ij, the
 * M image K^{-1}-weighted for REG_MASS_SOURCE as in <., .>_W; slots of dropped directions zeroed).  theta_host
 * (nullable): host [rank], the Ritz values, descending, then zeros.  1 <= rank <= min(8,
 * lowrank_capacity); REG_ESTATE before reg_gradient; REG_EINVAL for REG_STOKES with
 * REG_MASS_SOURCE.  Costs (iters + 1) rank matvecs; overwrites the low-rank correction slots and
 * synchronises the stream. */
reg_status reg_ritz_directions(reg_problem* h, double* U, int32_t rank, int32_t iters, double* theta_host);

/* Deformation diagnostics of a velocity (appendix "Illustration of Deformation Map"): the
 * displacement u with u(0) = 0 transported by v with source v (eq. (displacement); the Eulerian map
 * is y = x - u_1) and the deformation gradient F with F(0) = I transported by v with source
 * (grad v) F (eq. (def-grad)), integrated with the state equation's Heun steps (n_t) in FP64 for the
 * Nyquist-projected v.  v: device vector field.  workspace: device memory of at least
 * reg_deformation_workspace_bytes (37 FP64 scalar fields), 256-byte aligned, owned by the caller.
 * Outputs, all nullable: u1 (device vector field), F1 (device [2][2][n1][n2], F1[i][k] = F_ik),
 * detF1 (device scalar field det F_1), stats_host (host double[3]: min, max and mean of det F_1;
 * then the stream is synchronised).  Does not change the linearisation point. */
reg_status reg_deformation_workspace_bytes(const reg_params* params, size_t* bytes);
reg_status reg_deformation(reg_problem* h, const double* v, void* workspace, size_t workspace_bytes,
                           double* u1, double* F1, double* detF1, double* stats_host);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): reg_deformation without the workspace argument.  Its 37 FP64
 * scratch fields live in a library-owned static device array (one per GPU, about 18.5 MiB, held
 * until the process ends), so grids are limited to n1 * n2 <= 65536 (256 x 256); larger grids give
 * REG_EINVAL.  The call allocates nothing.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race and must be serialised by the caller.
 * Outputs and their meaning as for reg_deformation. */
reg_status reg_deformation_static(reg_problem* h, const double* v, double* u1, double* F1, double* detF1,
                                  double* stats_host);

/* Measurement hook: run `reps` (1..1000, reps * nt <= 512) Hessian matvecs at the current
 * linearisation point and time every launch of one of the four RK2-stage launches of a time step:
 * ms_per_launch_host = mean dispatch interval, from start / end events that the dispatch itself
 * stamps (what a profiler reports as the kernel's duration); exec_ms_host (nullable) = mean
 * execution interval of its blocks on the device wall clock (latest block end, after its stores
 * completed, minus earliest block start); the difference is the workgroup dispatch ramp and the
 * end-of-kernel completion.  bytes_per_launch_host = the launch's compulsory HBM bytes (each
 * operand field read once, each result written once).  Overwrites PCG scratch.
 * which: 0 GN incremental-adjoint stage 2 (the busiest launch: it also accumulates the body force),
 * 1 incremental-state stage 2, 2 GN incremental-adjoint stage 1, 3 incremental-state stage 1.
 * REG_ESTATE before the first reg_hessian_matvec.  Synchronises the stream. */
reg_status reg_time_pass(reg_problem* h, int32_t which, int32_t reps, double* ms_per_launch_host,
                         double* bytes_per_launch_host, double* exec_ms_host);

/* Measurement hook, phase mode: as reg_time_pass (same `which`; reps * nt <= 256), but every block of
 * the timed launches also stamps, on the device wall clock, the arrival of all its loads and the end
 * of its transforms, each after waiting for all its waves' memory operations, so the three phases
 * run one after another instead of overlapping.  phase_us_host[6] receives, in microseconds per
 * launch: [0] dispatch interval, [1] block execution interval, [2] spread of the block starts (latest
 * minus earliest), and the means over blocks of [3] start -> loads arrived, [4] -> forward and inverse
 * transforms done, [5] -> stores acknowledged.  [3..5] cover the one-launch stages of square
 * power-of-two FP32 grids (64+ points) and are 0 for the others.  REG_ESTATE before the first reg_hessian_matvec.  Synchronises
 * the stream. */
reg_status reg_time_phases(reg_problem* h, int32_t which, int32_t reps, double* phase_us_host);

/* Launch-shape autotuner for the FP32 transport stages on square grids of 64+ points (elements per
 * thread of the row and column register FFTs, threads per block), at the current linearisation
 * point and on the last reg_hessian_matvec input.  The first pass times every shape that fits the
 * grid's line length for each of the four matvec stage launches in isolation (`reps` launches); the
 * second times whole graph-replayed matvecs and, one stage at a time, keeps whichever of that stage's
 * four fastest first-pass shapes makes the matvec fastest (a change must save more than 0.1%).  The choice
 * stays in the handle; `report` (nullable, truncated to report_bytes) receives JSON with the first-pass
 * timings (microseconds per launch), the matvec time of the first-pass picks and of the final choice
 * (milliseconds) and the choice.  Results are identical for every shape up to rounding; only speed
 * differs.  REG_ESTATE before the first reg_hessian_matvec.  FP64 problems use fixed shapes
 * (no-op).  Synchronises the stream. */
reg_status reg_autotune(reg_problem* h, int32_t reps, char* report, size_t report_bytes);

/* Apply launch shapes chosen earlier (e.g. cached from a reg_autotune report): one shape index in
 * [0, 20) per stage op {state 1, state 2, adjoint 1, adjoint 2, incremental state 1, incremental
 * state 2, gradient}; count must be 7.  A shape that does not fit the grid's line length (too few
 * threads for a 2048-point line, say) runs as the grid's default shape. */
reg_status reg_set_pass_variants(reg_problem* h, const int32_t* variants, int32_t count);

/* Thread-local description of the last error (never NULL). */
const char* reg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* REGNK_H */
