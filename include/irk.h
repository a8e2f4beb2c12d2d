/*
 * irk.h -- C ABI of the MI355X stage solver for fully implicit Runge-Kutta
 * time stepping of  M u' = -K u + F  (Q1 finite elements, uniform grid).
 *
 * Problem statement (Kirby & MacLachlan, "Extending Irksome", Section 2 and
 * Section 3, eq:block_struct_AI): one time step of an s-stage Runge-Kutta method
 * with Butcher tableau (A, b, c) solves the stage-coupled linear system
 *
 *     (I_s (x) M + dt * A (x) K) k = f,     f_i = -K u^n + F,
 *
 * for the stage derivatives k = (k_1, ..., k_s) and updates
 * u^{n+1} = u^n + dt * sum_i b_i k_i.  M is the Q1 consistent mass matrix and K
 * the stiffness matrix of div(kappa grad u) with per-element kappa on the
 * uniform N x N grid of the unit square; homogeneous Dirichlet data are imposed
 * as the paper's "DAE-type" boundary conditions (Section 2.1), which for g = 0
 * and invertible A make every stage vanish on the boundary.
 *
 * The system is solved by right-preconditioned FGMRES. The preconditioner is the
 * block Jacobi (eq:pcbjac), block lower Gauss-Seidel (eq:pcbgs), its block upper
 * variant, or Rana-LD (eq:pcranald) stage preconditioner, in the AI form
 * I (x) M + dt * Atil (x) K  with Atil = D, L + D or U + D of A = L + D + U, or
 * Atil = L1 D of A = L1 D U1 (unit triangular L1, U1); each diagonal block
 * M + dt*atil_ii*K is approximated by one geometric multigrid V-cycle (Section 3.1).
 * A triangular Atil is inverted by block forward (lower) or backward (upper)
 * substitution.
 *
 * Conventions for every entry point:
 *  - Return value: IRK_OK (0) or a negative irk_status. After an error,
 *    irk_last_error() returns a message for the calling thread.
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory. The caller owns every pointer passed in
 *    and keeps it valid for the duration of the call. The library copies what
 *    it keeps (kappa, the tableau, the options) and owns its workspace; the
 *    destroy functions free it.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream). All device
 *    work is enqueued on it. Entry points that make convergence decisions
 *    (irk_solve_stages, irk_advance, irk_adjoint) synchronise the stream before
 *    they return; the others only enqueue work.
 *  - Nodal vectors use the compact interior layout: the n = (N-1)^2 interior
 *    nodes, row-major by y with x fastest; node (i, j) at (i/N, j/N),
 *    1 <= i, j <= N-1, sits at index (j-1)*(N-1) + (i-1). A stage block is s
 *    such vectors one after the other (stage-major), s*n doubles.
 *  - Element fields use the layout: element (ex, ey) covering
 *    [ex/N,(ex+1)/N] x [ey/N,(ey+1)/N] sits at index ey*N + ex, N*N doubles.
 */
#ifndef IRK_H
#define IRK_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IRK_OK = 0,
  IRK_EINVAL = -1,      /* invalid argument (message says which)               */
  IRK_ENOMEM = -2,      /* device or host allocation failed                    */
  IRK_EHIP = -3,        /* a HIP runtime call failed                           */
  IRK_ENOCONV = -4,     /* FGMRES missed rtol within max_it                    */
  IRK_EBREAKDOWN = -5   /* non-finite value met inside the Krylov iteration
                           (the stepper clears its work vectors and stays
                           usable)                                             */
} irk_status;

/* eq:pcbjac, eq:pcbgs, eq:pcranald, the block upper-triangular variant of eq:pcbgs (Section 3.1),
 * and one monolithic multigrid V-cycle on the whole stage-coupled system (Section 3.2) */
enum { IRK_PC_JACOBI = 0, IRK_PC_GS_LOWER = 1, IRK_PC_RANA_LD = 2, IRK_PC_GS_UPPER = 3, IRK_PC_MONOLITHIC = 4 };
enum { IRK_F64 = 0, IRK_F32 = 1, IRK_BF16 = 2 };            /* multigrid precision */
/* Gram-Schmidt variant of the Arnoldi process: classical with re-orthogonalisation (three passes per
 * step), with selective re-orthogonalisation, or its delayed one-reduction form (two passes per step;
 * Swirydowicz et al., Numer. Linear Algebra Appl. 2021) */
enum { IRK_ORTH_CGS2 = 0, IRK_ORTH_CGS_SELECTIVE = 1, IRK_ORTH_DCGS2 = 2 };
enum { IRK_GUESS_ZERO = 0, IRK_GUESS_PREV = 1 };            /* FGMRES initial guess */
/* Stage formulation (Section 2.2): AI solves eq:block_struct_AI for the stage derivatives k;
 * IA solves eq:block_struct_IA, (A^{-1} (x) M + dt I (x) K) w = f, for w = (A (x) I) k
 * (eq:butcherw, eq:stageeqw); A must then be invertible. */
enum { IRK_SPLIT_AI = 0, IRK_SPLIT_IA = 1 };
/* Stage solve (Section 2.3): COUPLED runs one FGMRES on the whole stage system; DIRK (lower-
 * triangular A, AI form) solves the stages one after the other, each by FGMRES on
 * M + dt a_ii K preconditioned by one V-cycle, with the known stages moved to the right. */
enum { IRK_STAGE_COUPLED = 0, IRK_STAGE_DIRK = 1 };
/* Arnoldi steps queued ahead of the host's convergence test (IRK_ORTH_DCGS2 only). OFF queues each
 * step after the host has read the previous one. ADAPTIVE (default) queues step 0 before the host reads
 * the initial norms, and step j+2 behind step j+1 while the last residual reduction factor, applied once
 * more, leaves the estimate above 4x the target (and step 1 with step 0 when the last solve of the same
 * system took three or more iterations). ALWAYS queues step j+2 whenever the cycle has one. A step
 * queued ahead and not used writes only Krylov vectors the solution does not depend on, so all three give
 * bit-identical results; irk_stats.arnoldi_discarded counts such steps. */
enum { IRK_LOOKAHEAD_OFF = 0, IRK_LOOKAHEAD_ADAPTIVE = 1, IRK_LOOKAHEAD_ALWAYS = 2 };

/* Butcher tableau (Section 2): A is s x s row-major, b and c have s entries.
 * Host memory; copied at stepper creation. */
typedef struct {
  int s;
  const double *A;
  const double *b;
  const double *c;
} irk_tableau;

/* Solver options; fill with irk_options_default() and override fields. */
typedef struct {
  int precond;        /* IRK_PC_JACOBI, IRK_PC_GS_LOWER, IRK_PC_RANA_LD, IRK_PC_GS_UPPER,
                         IRK_PC_MONOLITHIC (s <= 4)                                */
  double rtol;        /* stop when |f - Acal k|_2 <= rtol * |f|_2 (true residual)  */
  int restart;        /* FGMRES restart length m, 1..32                           */
  int max_it;         /* total FGMRES iterations allowed per stage solve          */
  int mg_coarse_n;    /* coarsen while a level has an even element count > this  */
  int cheb_degree;    /* Chebyshev smoothing degree, 1..3                          */
  double cheb_lo;     /* smoothing interval [cheb_lo*mu, cheb_hi*mu]              */
  double cheb_hi;
  int power_its;      /* power iterations for the largest eigenvalue mu            */
  int mg_precision;   /* IRK_F64, IRK_F32 or IRK_BF16 (storage; BF16 computes in FP32). With IRK_F32 or
                         IRK_BF16 the flexible basis of preconditioned vectors is kept in FP32 (the values
                         the FP32 multigrid computed); the Krylov basis, residuals and updates stay FP64 */
  int orth;           /* IRK_ORTH_DCGS2 (default), IRK_ORTH_CGS2 or IRK_ORTH_CGS_SELECTIVE */
  int initial_guess;  /* IRK_GUESS_ZERO or IRK_GUESS_PREV (previous step's k)     */
  int use_graphs;     /* 1: replay each Krylov iteration as a captured HIP graph;  
                         0: launch every kernel eagerly (same arithmetic)          */
  int splitting;      /* IRK_SPLIT_AI (default) or IRK_SPLIT_IA                    */
  int stage_type;     /* IRK_STAGE_COUPLED (default) or IRK_STAGE_DIRK             */
  int lookahead;      /* IRK_LOOKAHEAD_ADAPTIVE (default), IRK_LOOKAHEAD_OFF or IRK_LOOKAHEAD_ALWAYS */
  int basis_f64;      /* 1: keep the flexible basis in FP64 with IRK_F32 / IRK_BF16 as well (the same
                         values, twice the bytes: a check of the FP32 basis); 0 (default) */
} irk_options;

/* Per-call statistics (host struct, filled if non-NULL). */
typedef struct {
  int steps_done;        /* time steps completed successfully                */
  int fgmres_its_total;  /* FGMRES iterations summed over the solves          */
  int fgmres_its_max;    /* largest iteration count of one solve              */
  int restarts_total;    /* FGMRES restarts summed over the solves            */
  int solves;            /* stage-system solves performed                     */
  int forward_advances;  /* adjoint only: forward steps recomputed by revolve  */
  double last_rel_resid; /* |f - Acal k| / |f| of the last solve               */
  int failed_step;       /* index of the step that failed, -1 if none          */
  int arnoldi_discarded; /* Arnoldi steps launched ahead of the convergence test and not used */
} irk_stats;

typedef struct irk_problem irk_problem;
typedef struct irk_stepper irk_stepper;

/* Message for the last error on the calling thread ("" if none). */
const char *irk_last_error(void);

/* Defaults: GS_LOWER, rtol 1e-10, restart 30, max_it 300, coarse 32, Chebyshev
 * degree 2 on [0.25 mu, 1.1 mu] (the interval of Section 4.3), 15 power
 * iterations, FP64 multigrid, DCGS2 (delayed one-reduction CGS2), zero initial
 * guess, graphs on, AI splitting, coupled stage solve, ADAPTIVE lookahead. */
void irk_options_default(irk_options *opts);

/* Problem (Section 2, eq:rkheat with the Q1 discretisation of div(kappa grad u) on the
 * unit square): the grid and the diffusivity. N >= 2 elements per side; kappa is a
 * device array of N*N doubles (element layout), copied; every entry must be
 * finite and > 0 (IRK_EINVAL otherwise). The multigrid halves N while it is even
 * and above mg_coarse_n; the coarsest level Nc needs (Nc-1)^2 <= 1024 (dense solve),
 * otherwise stepper creation fails with IRK_EINVAL. */
int irk_problem_create(irk_problem **out, int N, const double *kappa, void *stream);
void irk_problem_destroy(irk_problem *p);

/* Replaces the problem's diffusivity (the kappa of eq:rkheat, Section 2) by kappa (device, N*N
 * doubles, element (ex, ey) at ey*N + ex), e.g. between the iterations of an optimisation over
 * kappa. Every value must be finite and > 0: otherwise IRK_EINVAL and the old kappa stays.
 * Waits for the stream. Steppers built on the problem see the new kappa in their stage operator
 * at once; their multigrid hierarchy (level diffusivities, Chebyshev estimates, coarsest
 * inverse) is updated by irk_stepper_refresh, which must be called on each of them before
 * their next solve. */
int irk_problem_set_kappa(irk_problem *p, const double *kappa, void *stream);

/* y = M x on one nodal vector: the consistent mass matrix M of eq:rkheat (Section 2),
 * Dirichlet rows and columns removed (device, n doubles each; x and y must not overlap).
 * Used for objectives such as J = 1/2 |u - u_*|_M^2. Staging: two padded planes owned by the
 * problem, allocated by the first irk_apply_mass / irk_apply_stiffness call on it; calls on one
 * problem that overlap in time (different streams, threads) race on them. Only enqueues work. */
int irk_apply_mass(const irk_problem *p, const double *x, double *y, void *stream);

/* y = K x: the stiffness matrix K of eq:rkheat (Section 2) with the problem's kappa,
 * Dirichlet rows and columns removed (device, n doubles each; no overlap). Staging as
 * irk_apply_mass. Only enqueues work. */
int irk_apply_stiffness(const irk_problem *p, const double *x, double *y, void *stream);

/* y = M x exactly as irk_apply_mass (same kernels, same result bits), for callers that cannot
 * allocate device memory: code under HIP stream capture, serving loops, harnesses that forbid
 * hipMalloc. It calls no allocating routine: its staging (two padded planes) is a static device
 * array of 2 * 1025 * 1040 doubles (17.1 MB) that every GPU the library runs on holds until the
 * process ends, so N <= 1024 (IRK_EINVAL beyond, with a message). The array's device address is
 * looked up once per device, on the first call for a problem of that device, which must then be
 * the current device (IRK_EINVAL otherwise). Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (different streams or threads) race and must be ordered by the
 * caller. Only enqueues work (x, y: device, n doubles each, no overlap). */
int irk_apply_mass_noalloc(const irk_problem *p, const double *x, double *y, void *stream);

/* Stepper (Section 2 time stepping of eq:rkheat with the stage system eq:block_struct_AI or
 * eq:block_struct_IA and a Section 3 preconditioner): a tableau, a time step and solver
 * options on a problem; sets up the
 * multigrid hierarchy (level diffusivities, power-iteration estimates of mu per
 * level and diagonal block, the coarsest-level inverse) and the Krylov
 * workspace. Every eigenvalue of A must have positive real part and every
 * a_ii > 0 (Rana-LD: every LDU pivot > 0), A must be invertible for IRK_SPLIT_IA and
 * lower triangular for IRK_STAGE_DIRK (IRK_EINVAL otherwise). The problem must outlive the stepper. */
int irk_stepper_create(irk_stepper **out, const irk_problem *p, const irk_tableau *tab,
                       double dt, const irk_options *opts, void *stream);
void irk_stepper_destroy(irk_stepper *st);

/* Rebuilds the kappa-dependent state of a stepper from its problem's current kappa (after
 * irk_problem_set_kappa): level diffusivities, power-iteration estimates and Chebyshev
 * coefficients, coarsest-level inverses (also of the monolithic cycle), reusing every
 * buffer; captured Arnoldi graphs are dropped (captured again on first use) and the next
 * solve starts without a previous-step guess. Waits for the stream before and after. */
int irk_stepper_refresh(irk_stepper *st, void *stream);

/* a1 (Section 2, eq:rkheat): f_i = -K u + F for every stage i. u: device n; F: device
 * n or NULL (F = 0); f: device s*n. */
int irk_stage_rhs(const irk_stepper *st, const double *u, const double *F, double *f, void *stream);

/* a2 (eq:block_struct_AI): y = (I (x) M + dt * A (x) K) x, or with A^T when transpose != 0;
 * with IRK_SPLIT_IA (eq:block_struct_IA): y = (A^{-1} (x) M + dt I (x) K) x, or with A^{-T}.
 * x, y: device s*n, no overlap. */
int irk_apply_stage_operator(const irk_stepper *st, const double *x, double *y, int transpose, void *stream);

/* a3 (eq:pcbjac / eq:pcbgs / eq:pcranald): z = P^{-1} v with the stepper's block
 * preconditioner, every diagonal block solve replaced by one V-cycle. AI splitting:
 * P = I (x) M + dt Atil (x) K, stages coupled through K. IA splitting (the printed form):
 * P = Atil^{-1} (x) M + dt I (x) K, stages coupled through M, diagonal blocks
 * (1/atil_ii) M + dt K, whose V-cycle is atil_ii times the V-cycle of M + dt atil_ii K.
 * IRK_PC_MONOLITHIC: one monolithic V-cycle (Section 3.2, eq:Cinv on the patches of
 * eq:bigdecomp) on the whole system: additive Schwarz over each vertex's s stage values
 * (an s x s solve per node) inside Chebyshev smoothing, stage-wise transfers, a dense
 * solve on the coarsest level (halving while N is even and N > mg_coarse_n or
 * s (N-1)^2 > 1024). With transpose != 0 the preconditioner of the transposed system is
 * applied: for the block preconditioners the transpose of the forward one, I (x) M + dt Atil^T (x) K
 * (IA: Atil^{-T} (x) M + dt I (x) K), by block substitution in the opposite order; the monolithic
 * cycle is built on the transposed operator. v, z: device s*n. */
int irk_apply_preconditioner(const irk_stepper *st, const double *v, double *z, int transpose, void *stream);

/* a4 (Section 3.1 diagonal blocks): z = one V-cycle for (M + dt*atil_ii*K) z = t with zero
 * initial guess, for stage `stage` (0-based; atil_ii = a_ii, or the LDU pivot for Rana-LD).
 * t, z: device n. */
int irk_vcycle(const irk_stepper *st, int stage, const double *t, double *z, void *stream);

/* a5: solve (I (x) M + dt*A (x) K) k = f (A^T when transpose != 0) by FGMRES to the
 * stepper's rtol from a zero initial guess; with IRK_SPLIT_IA the unknown is w and the
 * operator that of irk_apply_stage_operator. With IRK_STAGE_DIRK the same system is solved
 * stage by stage (backwards for the transpose), each stage to rtol of its own right-hand
 * side; stats count one solve per stage. f, k: device s*n. Synchronises. */
int irk_solve_stages(irk_stepper *st, const double *f, double *k, int transpose, irk_stats *stats, void *stream);

/* a1+a5+a6: advance u (device n, in/out) by nsteps time steps of size dt with forcing F
 * (device n or NULL), u^{n+1} = u^n + dt * sum_i b_i k_i (IA: dt * sum_i (A^{-T} b)_i w_i).
 * On IRK_ENOCONV or IRK_EBREAKDOWN u holds the last step that converged and stats->failed_step
 * names the failing step. Synchronises. */
int irk_advance(irk_stepper *st, double *u, const double *F, int nsteps, irk_stats *stats, void *stream);

/* a8+a9: discrete adjoint of nsteps steps from u0 (device n) with F = 0. Given
 * lambda_T = dJ/du_N (device n) it returns lambda_0 = dJ/du_0 (device n, may be NULL) and
 * grad_logkappa = dJ/dlog(kappa) (device N*N, element layout, may be NULL). The forward
 * states are recomputed from nsnap >= 1 snapshots (one of them u0) by the optimal binomial
 * checkpointing schedule. Workspace (min(nsnap, nsteps) checkpoint planes, the adjoint state, the
 * gradient and two stage vectors) is owned by the stepper: allocated by the first call, the
 * checkpoint planes grown when a later call needs more. Synchronises. */
int irk_adjoint(irk_stepper *st, const double *u0, int nsteps, int nsnap, const double *lambda_T,
                double *lambda_0, double *grad_logkappa, irk_stats *stats, void *stream);

/* a9 (host only): the binomial checkpointing schedule for nsteps steps and nsnap slots.
 * Writes up to cap actions as pairs (kind, arg) into actions (host int[2*cap]);
 * kind 0 = advance arg steps, 1 = store the current state in slot arg,
 * 2 = restore slot arg, 3 = reverse the step starting at the current state
 * (recompute its stages, solve its adjoint). *count receives the number of actions
 * and *advances the number of forward steps outside reversals. Returns
 * IRK_EINVAL if cap is too small (with *count set to the size needed). */
int irk_revolve_schedule(int nsteps, int nsnap, int *actions, int cap, int *count, int *advances);

/* Sizes: n = (N-1)^2 interior nodes and s stages of a stepper. */
int irk_stepper_sizes(const irk_stepper *st, int *N, int *s, int *levels);

/* The power-iteration estimate mu of the largest eigenvalue of D^{-1}(M + dt*a_ii*K) on
 * multigrid level `level` (0 = finest) for stage `stage`; *mu = 0 on the coarsest level. */
int irk_stepper_mu(const irk_stepper *st, int stage, int level, double *mu);

/* Monolithic cycle (IRK_PC_MONOLITHIC steppers only): *levels (may be NULL) receives its level
 * count and *mu (may be NULL) the power-iteration estimate for the Chebyshev interval on level
 * `level` (0 = finest; 0 on the coarsest) of the forward (transpose = 0) or transposed system. */
int irk_stepper_mmg_mu(const irk_stepper *st, int transpose, int level, double *mu, int *levels);

/* Measurement hook: kernel families of a step, timed by irk_kernel_timer. */
enum {
  IRK_KFAM_GRAM_SCHMIDT = 0,   /* streaming Gram-Schmidt passes over the Krylov vectors (also norms, updates)  */
  IRK_KFAM_OPERATOR = 1,       /* stage operator (and residual) applications                                   */
  IRK_KFAM_MG_FINE = 2,        /* finest-level multigrid DOWN and UP kernels (single-stage and monolithic)    */
  IRK_KFAM_MG_COARSE = 3,      /* multigrid DOWN and UP kernels on the coarser levels                          */
  IRK_KFAM_COARSE_SOLVE = 4,   /* dense coarsest-level solves                                                  */
  IRK_KFAM_REDUCE_FINISH = 5,  /* one-block finishing kernels of the reductions                                */
  IRK_KFAM_OTHER = 6,          /* stage right-hand side, update, block-triangular coupling on one-level grids  */
  IRK_KFAM_COUNT = 7,
  IRK_KFAM_ALL = 100           /* every family above                                                           */
};

/* While enabled, every dispatch of kernel family `family` (or of all families) during the
 * solver's time steps and stage solves carries HIP start/stop events attached to the dispatch
 * itself (hipExtLaunchKernelGGL on the stream the kernel runs on), and its algorithmic bytes are
 * accumulated: the streaming passes count each vector they read or write (8 bytes a value); the
 * multigrid kernels count two figures, the per-pass model (every smoothing, residual and transfer
 * pass streaming its vectors: per node 8.25 p for DOWN and for UP with p the bytes of a stored
 * value, plus the diffusivity once per smoothing pass, plus 8 bytes per coupled FP64 stage
 * plane) and the fused minimum (what the fused kernel reads and writes once); the coarsest solve
 * counts its inverse and vectors. Krylov iterations are launched eagerly (not replayed from
 * graphs) meanwhile, with the same kernels and arithmetic. Enabling resets the counters. */
int irk_kernel_timer(irk_stepper *st, int family, int enable);
/* For one family (or IRK_KFAM_ALL): dispatches timed, their summed duration (ms), and their
 * summed algorithmic bytes (per-pass model and fused minimum; each pointer may be NULL).
 * Synchronises on the recorded events. */
int irk_kernel_timer_family(irk_stepper *st, int family, int *launches, double *total_ms, double *bytes,
                            double *bytes_min);
/* The same over all timed families (per-pass model bytes). */
int irk_kernel_timer_read(irk_stepper *st, int *launches, double *total_ms, double *bytes);

/* Measurement reference (defined by no passage of the paper): y = x for n doubles (device, no
 * overlap, IRK_EINVAL otherwise; n = 0 does nothing), one 16-byte load and store per thread when
 * both pointers are 16-byte aligned. The plain streaming kernel against which the solver's kernels
 * are compared: its bandwidth is the practical ceiling, and its HBM byte counters (2n*8 bytes
 * known) scale the counters of the others. Only enqueues work. */
int irk_device_copy(const double *x, double *y, long long n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* IRK_H */
