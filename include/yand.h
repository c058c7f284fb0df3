/*
 * libyand -- MI355X-native hot path of YAND-MVSK (Yau's affine-normal descent
 * for unrestricted mean-variance-skewness-kurtosis portfolios).
 *
 * Problem (Section 2, equation (mvsk)): minimise over portfolio weights w
 *     f(w) = -c1 m1(w) + c2 m2(w) - c3 m3(w) + c4 m4(w),
 * with m1 = mu^T w and m_p = T^-1 sum_t ((R w)_t - mu^T w)^p, where R (T x n)
 * holds one row of asset returns per bar, mu = T^-1 R^T 1 and A = R - 1 mu^T.
 * Weights satisfy the budget 1^T w = 1 (BUDGET set: its affine hull, the
 * reduced parametrisation of Section 4.2) and optionally a return target
 * mu^T w = r; the SIMPLEX set additionally keeps w_i >= tau through the
 * feasibility cap of Section 4.3 (up to the rounding of a step that ends on
 * the bound, a few ulps of the largest weight).
 *
 * Conventions for every entry point:
 *  - Scalars and small fixed-size arrays (c[4], coef[5], mom[4], f, target)
 *    are HOST memory.  Vectors of length n or T (w, v, d, grad, hv, w_out)
 *    are DEVICE memory on the context's device, FP64, contiguous.
 *  - The caller owns every buffer it passes in; the library never frees or
 *    retains them.  The context owns its copy of A (centered, at the chosen
 *    storage precision), mu and all workspaces.
 *  - Work is enqueued on the context's HIP stream.  Every call returns after
 *    the stream has finished the call's work (host outputs are valid).
 *  - Return value: 0 success, > 0 warning, < 0 error (YAND_* codes below).
 *    Nothing is thrown across the ABI.  A context is not thread-safe: calls
 *    on one context must be serialised by the caller.
 *  - c must satisfy c_i >= 0 (Section 2) or YAND_ERR_ARG is returned.
 */
#ifndef YAND_H
#define YAND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  YAND_OK = 0,
  YAND_WARN_MAXITER = 1,     /* iteration / time budget ended above eps      */
  YAND_WARN_STALL = 2,       /* stalled above eps: the objective decreased by
                                less than 1e-14 of |f| on 3 iterations in a
                                row, or the stall restarts ran and the solve
                                is still above eps                           */
  YAND_ERR_ARG = -1,         /* bad size, negative c, infeasible start/target */
  YAND_ERR_NONFINITE = -2,   /* NaN or Inf in R or in an iterate             */
  YAND_ERR_HIP = -3,         /* a HIP runtime call failed                    */
  YAND_ERR_OOM = -4,         /* device allocation failed                     */
  YAND_ERR_INDEFINITE = -5,  /* tangent Hessian indefinite after escalation  */
  YAND_ERR_UNBOUNDED = -6,   /* quartic line model unbounded below           */
  YAND_ERR_TOO_LARGE = -7    /* instance exceeds the fixed scratch array of
                                yand_mvsk_solve_R_noalloc                    */
};

/* Storage precision of the centered matrix A inside the context. */
enum { YAND_FP64 = 0, YAND_FP32 = 1, YAND_BF16 = 2 };
/* Reduced tangent solve: dense Cholesky ("small") or projected PCG ("large"),
 * Appendix D, Table "YAND-MVSK parameter settings". */
enum { YAND_SOLVER_DIRECT = 0, YAND_SOLVER_PCG = 1 };
/* Feasible set: affine budget hull (no cap) or the slice Delta(tau). */
enum { YAND_SET_BUDGET = 0, YAND_SET_SIMPLEX = 1 };
/* Trace of the affine-normal correction in the PCG configuration: exact
 * (the dense route, or the T x T push-through when 2 T <= n) or estimated
 * from random sign probes (Hutchinson's diagonal estimator with the probe
 * solves by the same PCG: the Krylov reduced solve of Appendix C). */
enum { YAND_TRACE_EXACT = 0, YAND_TRACE_PROBE = 1 };
/* Step rule on the quartic line model: the exact rule (Proposition "Quartic
 * exact line search from sample power sums") or Armijo backtracking (the
 * rule of the convergence theory; sigma = 1e-4, halving from min(1,
 * alpha_max), the Armijo diagnostic of Table "YAND-MVSK parameter
 * settings"). */
enum { YAND_LS_EXACT = 0, YAND_LS_ARMIJO = 1 };

typedef struct yand_ctx yand_ctx;

/* Solver parameters (Appendix D, Table "YAND-MVSK parameter settings").
 * regularization is relative: lambda = regularization * (mean diagonal of the
 * tangent Hessian).  yand_default_opts fills the direct configuration. */
typedef struct yand_opts {
  int solver;             /* YAND_SOLVER_*                                    */
  int feasible_set;       /* YAND_SET_*                                       */
  double eps;             /* stop when ||reduced gradient||_2 <= eps (1e-8)   */
  int max_iter;           /* outer budget (direct 300, PCG 40)                */
  double max_elapsed;     /* seconds per phase (PCG 60; <= 0 means unlimited):
                             checked before each direction; the direct
                             configuration and batched solves measure it
                             from the start of the call                     */
  double regularization;  /* relative lambda (direct 0, PCG 1e-4)             */
  double krylov_tol;      /* relative PCG residual (1e-3; must be > 0)        */
  int krylov_maxit;       /* PCG iterations (15)                              */
  double tau;             /* interior margin of Delta(tau) (1e-8)             */
  int stall_recovery;     /* PCG: restart twice when a phase ends above eps
                             (stall test, iteration or time budget): budget
                             set, twice the Krylov budget, then the direct
                             solve; simplex boundary block, projected trial
                             steps 0.045, then 0.02                         */
  int restart_max_iter;   /* outer budget of each restart (120)               */
  double eta;             /* simplex boundary block: nominal projected trial
                             step (0.05; 0 = capped raw steps only).  Active
                             on YAND_SET_SIMPLEX without a return target.    */
  int linesearch;         /* YAND_LS_EXACT (default) or YAND_LS_ARMIJO        */
  int dense_fp64;         /* FP32 / BF16 storage of A: 0 (default) forms the
                             exact trace's products (B = A^T diag(psi'') A / T
                             and the rows of L^-1 A^T) on the matrix cores
                             with FP32 / BF16 inputs and FP32 accumulation;
                             1 forms them in FP64.  The factorisation, the
                             passes' reductions, the line-search sums and
                             the PCG inner products are FP64 either way.     */
  int trace_mode;         /* YAND_TRACE_EXACT (default) or YAND_TRACE_PROBE;
                             the probe estimate applies to PCG phases only:
                             q_t = k^-1 sum_j xi_tj (A K A^T xi_j)_t with
                             K = P_S (H + lambda)^-1 P_S applied by k PCG
                             solves (krylov_tol, krylov_maxit) whose
                             products with A run as block passes on the
                             matrix cores; no n x n matrix is formed        */
  int probes;             /* k, sign vectors per direction (1..64; 64)        */
  uint64_t probe_seed;    /* xi_tj = sign bit of SplitMix64 at the Weyl state
                             probe_seed + gamma (d 2^42 + t 2^10 + j), d the
                             direction count of the solve (0 for
                             yand_affine_normal), gamma = 0x9E3779B97F4A7C15 */
} yand_opts;

/* Per-solve report: counters follow the oracle-query accounting of the
 * implementation appendix (value/gradient, Hessian-vector, third-order,
 * line-search passes, Krylov iterations). */
typedef struct yand_info {
  int status;             /* return code of the solve                         */
  int iterations;         /* outer iterations performed                       */
  int restarts;           /* stall-recovery restarts                          */
  int cg_iters;           /* total PCG iterations                             */
  double f;               /* objective at w_out                               */
  double gnorm;           /* ||reduced gradient||_2 at w_out (own precision)  */
  double elapsed;         /* seconds                                          */
  double lambda_used;     /* absolute regularisation of the last direction    */
  int64_t oracle_passes;  /* value/gradient passes over A                     */
  int64_t hvp_passes;     /* Hessian-vector passes over A                     */
  int64_t third_passes;   /* third-order back-projection passes over A        */
  int64_t ls_passes;      /* line-search passes over A                        */
  int64_t dense_traces;   /* exact-trace factorisations                       */
  double kkt;             /* projected-simplex KKT residual at w_out
                             |w - Pi_Delta(tau)(w - grad f(w))|_2 (simplex
                             set; NaN on the budget set)                     */
  int projected_steps;    /* iterations that took the projected trial segment */
  int phase_iterations[3];/* iterations of the baseline phase and of each
                             stall-recovery restart                          */
  int64_t probe_traces;   /* directions whose trace came from probes          */
  int64_t probe_cg_iters; /* PCG iterations of the probe solves (all columns) */
  int64_t thin_traces;    /* exact traces by the T < n push-through (of
                             dense_traces; no n x n matrix formed)           */
} yand_info;

/* Fill *opts with the direct configuration (YAND-MVSK small). */
void yand_default_opts(yand_opts* opts);
/* Fill *opts with the PCG configuration with stall recovery (YAND-MVSK large). */
void yand_large_opts(yand_opts* opts);

/* Create a context from device returns R (T x n, FP64, row stride ldr >= n).
 * Computes mu = T^-1 R^T 1 and A = R - 1 mu^T (Section 2; Algorithm 1 setup),
 * rounds A to `precision` and keeps it; R is not retained.
 * hip_stream: a hipStream_t (NULL = default stream).  Requires n >= 2, T >= 2.
 * Errors: YAND_ERR_ARG, YAND_ERR_NONFINITE (R has NaN/Inf), YAND_ERR_OOM,
 * YAND_ERR_HIP.  On error *out is set to NULL. */
int yand_create(const double* R, int64_t T, int64_t n, int64_t ldr,
                int precision, void* hip_stream, yand_ctx** out);
int yand_destroy(yand_ctx* ctx);

/* Copy mu (n, FP64) to a device buffer. */
int yand_get_mu(yand_ctx* ctx, double* mu_out);

/* Exact sample oracle (Proposition "Exact operator representation"):
 * f(w) (host), grad = -c1 mu + A^T psi'(Aw)/T (device, nullable) and the
 * moments m1..m4 (host, nullable).  One pass over A. */
int yand_eval(yand_ctx* ctx, const double c[4], const double* w, double* f,
              double* grad, double mom[4]);

/* Hessian-vector product hv = A^T (psi''(Aw) * Av) / T (equation
 * (operator-hvp)); w, v, hv device.  A value pass caches z = Aw, then one
 * fused pass over A forms the product. */
int yand_hvp(yand_ctx* ctx, const double c[4], const double* w,
             const double* v, double* hv);

/* Quartic line-search coefficients coef[0..4] = A0..A4 of f(w + alpha d)
 * (Proposition "Quartic exact line search from sample power sums"), built
 * from the FP64 power sums s_rs = T^-1 sum z^r (Ad)^s.  w, d device. */
int yand_linesearch_coeffs(yand_ctx* ctx, const double c[4], const double* w,
                           const double* d, double coef[5]);

/* Exact step (same proposition): the argmin of the quartic over 0, alpha_max
 * (if finite; pass INFINITY for the budget set) and the real roots of its
 * derivative in (0, alpha_max), computed on the device.  Ties go to the
 * smallest step within 1e-15 * sum_{i>=1} |A_i| alpha^i.  A constant model
 * (A1..A4 zero) gives alpha = 0.  Returns YAND_ERR_UNBOUNDED when alpha_max
 * is infinite and the quartic does not grow at infinity. */
int yand_select_step(yand_ctx* ctx, const double coef[5], double alpha_max,
                     double* alpha);

/* Euclidean projection onto Delta(tau) = {x : x_i >= tau, sum_i x_i = 1}
 * (the projected trial step of the implementation appendix's reduced-simplex
 * wrapper): x = Pi(y).  y, x device (n doubles; may not overlap).  One
 * workgroup on the null stream: bisection for the threshold theta of
 * x_i = max(y_i - tau - theta, 0) + tau, then theta formed from the
 * support.  Returns after the projection is done.  YAND_ERR_ARG when
 * n < 1, tau < 0 or tau >= 1/n, or a pointer is NULL. */
int yand_project_simplex(const double* y, int64_t n, double tau, double* x);

/* Projected-simplex KKT residual |w - Pi_Delta(tau)(w - grad f(w))|_2 at
 * w (device, n), the solution-quality metric of the computational study
 * (the paper gives no formula; this is the projected-gradient residual on
 * the slice), written to *kkt (host).  yand_mvsk_solve reports it with the
 * solve's tau.  YAND_ERR_ARG when tau < 0 or tau >= 1/n. */
int yand_kkt_residual(yand_ctx* ctx, const double c[4], const double* w,
                      double tau, double* kkt);

/* Affine-normal direction with the exact log-det trace at the feasible point
 * w (Section 4.2 and Section 4.4; factor 1/(m+1) of Appendix B, Proposition
 * "A sufficient condition for the imported bounded-direction hypothesis"),
 * written to d_out (device, n).  target: NULL for the budget constraint only,
 * else a host pointer to r in mu^T w = r.  gnorm (host, nullable) receives
 * the reduced-gradient norm.  opts selects direct or PCG solve (NULL: direct,
 * no regularisation). */
int yand_affine_normal(yand_ctx* ctx, const double c[4], const double* target,
                       const double* w, const yand_opts* opts, double* d_out,
                       double* gnorm);

/* Algorithm 1: solve from w0 (device, n; NULL = equal weights moved onto the
 * target constraint) and write w_out (device, n).  info (host) is nullable.
 * On YAND_SET_SIMPLEX without a target and with opts->eta > 0 the boundary
 * block of Algorithm 1 runs: the direction lives on the current face of
 * Delta(tau) (bound coordinates with a negative multiplier are released);
 * a step capped below eta is replaced by the line search on the corrected
 * segment Pi_{Delta(tau)}(w + eta d) - w when that is a descent direction
 * whose step covers at least a tenth of it; otherwise the face solver holds
 * the coordinates that stop the raw step (and released ones the direction
 * drives down) at the bound and the capped raw step is taken.  The run also
 * stops when the projected-KKT residual is <= eps.  A failed Cholesky
 * factorisation escalates lambda tenfold up to 16 times before
 * YAND_ERR_INDEFINITE. */
int yand_mvsk_solve(yand_ctx* ctx, const double c[4], const double* target,
                    const double* w0, const yand_opts* opts, double* w_out,
                    yand_info* info);

/* Return-floor protocol of the real-data comparison (Section "Computational
 * Study"): the long-only MVSK portfolio whose in-sample mean return
 * mu^T w lies as close as possible to the floor, the q-th percentile of the
 * asset means (linear interpolation between order statistics at (n-1) q).
 *  - Normalisation: c_k = profile[k-2] / |m_k(1/n)| for k = 2, 3, 4, the
 *    moments of the equal-weight portfolio (profile = (p2, p3, p4), host).
 *  - Calibration of c1 (the paper gives no rule; this one leans on mu^T w
 *    of the minimiser being nondecreasing in c1, which holds when f is
 *    convex): c1 = 0 first, kept when it meets the floor (or when all asset
 *    means are equal); else c1 = 1 / (max mu - min mu), times 4 until the
 *    floor is met; then geometric bisection of the bracket (c_hi / 2 while
 *    the lower end is 0).  Each phase takes at most max_rounds solves; the
 *    bisection stops once |mu^T w - floor| <= 1e-9 (max mu - min mu).
 *    Every solve is yand_mvsk_solve from equal weights with opts (NULL: the
 *    direct configuration on YAND_SET_SIMPLEX; a non-NULL opts must select
 *    YAND_SET_SIMPLEX).
 * Outputs (all but w_out nullable): the closest solve (ties to the larger
 * c1): c_out[4] and floor_out, ret_out (host), its weights w_out (device, n)
 * and info (host), and the number of solves (host).  Returns that solve's
 * status (0 or a warning).  YAND_ERR_ARG for q outside [0, 1], a negative
 * or non-finite profile entry, max_rounds < 0, a nonzero profile entry
 * whose equal-weight moment is 0, or opts not on the simplex; a solve's
 * error (YAND_ERR_INDEFINITE outside the convexity certificate) ends the
 * protocol and is returned, with the outputs left unset.  Allocates one
 * n-vector of device memory for the duration of the call. */
int yand_return_floor(yand_ctx* ctx, const double profile[3], double q,
                      const yand_opts* opts, int max_rounds, double c_out[4],
                      double* floor_out, double* ret_out, double* w_out,
                      yand_info* info, int* solves);

/* Batched efficient-frontier solve on one context (shared A): instance b
 * minimises with preference vector C4[4b..4b+3] (host) and, when targets
 * (host, length B) is not NULL, the return target targets[b].  W0 (device,
 * B x n, nullable) holds the starting weights, each moved onto the
 * instance's constraints (NULL: equal weights moved there).  Weights go to
 * row b of W_out (device, B x n row-major); infos (host, length B) is
 * nullable.  Instances advance together in lanes of up to 64 solves; after
 * the first iteration one outer iteration of all lanes is replayed from a
 * captured HIP graph, with one host synchronisation per iteration.  Both
 * configurations: with opts->solver = YAND_SOLVER_PCG (exact trace only;
 * trace_mode = YAND_TRACE_PROBE is YAND_ERR_ARG) the lanes' tangent solves
 * advance together too, every CG step one pair of block products over A
 * for all lanes (the search directions as the 64 columns of one block), and
 * instances that neither converge nor fail continue through the single
 * solve's stall recovery (twice the Krylov budget, then the direct solve;
 * on the simplex face solver the projected trial steps 0.045 then 0.02),
 * counted in infos[b].restarts and phase_iterations.  Returns the first
 * error; per-instance status is in infos[b].status. */
int yand_frontier_solve(yand_ctx* ctx, int64_t B, const double* C4,
                        const double* targets, const double* W0,
                        const yand_opts* opts, double* W_out,
                        yand_info* infos);

/* Batched solve over contexts that may differ (universes of uneven n):
 * instance b runs on ctxs[b] (host array of B contexts on one device) and
 * writes W_out[b] (host array of B device pointers, each n_b long); W0
 * (nullable host array of B device pointers, entries nullable) gives starts.
 * max_lanes bounds the solves advancing together (<= 0: 64).  use_graph:
 * bit 0 replays captured iterations; bit 1 keeps the lanes on separate
 * streams.  Without bit 1, instances that all run on one context with the
 * exact trace's products in FP64 advance in lockstep on one stream: the
 * SYRK, the factorisation with its inverse and the trace GEMM of all lanes
 * run as single grouped launches (the same kernels and tile order per lane,
 * so in the direct configuration the results are those of separate lanes
 * bit for bit; the PCG configuration's batched Hessian products sum in
 * another order than the per-lane passes, so there they agree to rounding).
 * The PCG configuration is accepted as in yand_frontier_solve. */
int yand_batch_solve(int64_t B, yand_ctx* const* ctxs, const double* C4,
                     const double* targets, const double* const* W0,
                     const yand_opts* opts, double* const* W_out,
                     yand_info* infos, int max_lanes, int use_graph);

/* Kernel timing on the context stream (instrumentation): enable != 0 starts
 * recording HIP events around the main kernels; yand_profile_read(ctx, -1,
 * ...) returns the number of recorded kernel names, and index i >= 0 fills
 * the name, the total milliseconds and the launch count. */
int yand_profile_enable(yand_ctx* ctx, int enable);
int yand_profile_read(yand_ctx* ctx, int index, char* name, int name_len,
                      double* total_ms, int64_t* count);

/* A launch-shape record (yand_tuning, yand_autotune) holds
 * YAND_TUNING_INTS ints, 0 selecting the built-in default in every slot:
 *   [0..5]   workgroups per streaming pass, for the oracle, value, HVP,
 *            line-search, dot and third-order passes (rows per workgroup);
 *   [6]      128-column blocks per group of the two-level Cholesky;
 *   [7..12]  rows per block of the same six passes (1, 2 or 4; a height
 *            above the pass's register budget takes that budget's);
 *   [13]     sub-block width of the Cholesky's in-group updates (32 or 64);
 *   [14]     band width of its panel step (32 or 64).
 * Results change only in rounding order: the workgroup count and block
 * height regroup the FP64 sums of a pass; the widths leave the factor and
 * its inverse bit for bit the same. */
#define YAND_TUNING_INTS 15
/* Doubles of an autotune report: the chosen record, then the best mean
 * times in ms of the six passes and of the factorisation with inverse. */
#define YAND_AUTOTUNE_REPORT (YAND_TUNING_INTS + 7)

/* Launch-shape autotuner (an extension for serving).  Times candidate
 * launch shapes on this context's own A at equal weights with c = (1,5,2,10):
 * for each pass kind the workgroup count (256, 384, 512, 768 or 1024), then
 * the block height at that count; the group size of the Cholesky (2, 3, 4,
 * 5, 6 or 8), then the in-group sub-block and panel band widths at that
 * size.  The fastest are kept in the context and used by every later call
 * on it (and by batched solves over it).  report (host, nullable, YAND_AUTOTUNE_REPORT
 * doubles): see above.  Overwrites the context's scratch state. */
int yand_autotune(yand_ctx* ctx, double* report);

/* Read (get, host, YAND_TUNING_INTS ints, nullable) and/or set (set, host,
 * YAND_TUNING_INTS ints, nullable) the launch-shape record.  A value outside
 * the sets above gives YAND_ERR_ARG and changes nothing. */
int yand_tuning(yand_ctx* ctx, const int* set, int* get);

/* Stateless wrapper: returns R (device, T x n contiguous) -> w_out (device),
 * FP64 storage, direct solver, budget set. */
int yand_mvsk_solve_R(const double* R, int64_t T, int64_t n, double c1,
                      double c2, double c3, double c4, const double* target,
                      double* w_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * stateless solve of yand_mvsk_solve_R (same arguments, kernels and results;
 * from 16 tile columns, n > 1920, the SYRK keeps its plain tile order instead
 * of the balanced schedule, and results agree to rounding), with every
 * workspace -- the centered copy of A, mu, the pass
 * partials, the n x n factor buffers -- carved from one fixed 256 MiB device
 * array that the library holds on each device it runs on until the process
 * ends.  It calls no hipMalloc, hipFree or other allocating routine and uses
 * the null stream.  The instance needs about 8 (T n + 3 n^2) bytes plus
 * 8 MiB per 1024 columns of pass partials (padded to multiples of 128);
 * larger instances (for example n = 2000 at T = 12000) return
 * YAND_ERR_TOO_LARGE with a message on stderr, before any device work.
 * The array keeps the last call's contents and every call clears the part it
 * uses; calls that overlap on one device (several host threads) race on it
 * and must be serialised by the caller.  Errors otherwise as
 * yand_mvsk_solve_R. */
int yand_mvsk_solve_R_noalloc(const double* R, int64_t T, int64_t n,
                              double c1, double c2, double c3, double c4,
                              const double* target, double* w_out);

/* Corollary "coefficient-only convexity certificate": 1 if c4 > 0 and
 * 8 c2 c4 > 3 c3^2, else 0. */
int yand_is_certified_convex(const double c[4]);

/* Storage precision, T, n of a context (host outputs, nullable). */
int yand_shape(yand_ctx* ctx, int64_t* T, int64_t* n, int* precision);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension; the paper trains no model).  A small
 * fully connected network maps instance features (preferences c, return
 * target, moment summaries of the equal-weight portfolio) to the solution in
 * reduced coordinates of the fixed Householder basis U of {1^T x = 0}:
 * H = I - 2 v v^T / v^T v with v = e_n - 1/sqrt(n) 1; U = first n-1 columns
 * of H, and w = 1/n + U y.  The plain iteration always finishes the solve;
 * the first-order stationarity residual ||reduced gradient|| decides whether
 * the proposal or the plain start is used.
 * FP32 network buffers are DEVICE memory; the handle owns its weights, Adam
 * moments and activations.  Calls on one handle must be serialised.
 * ---------------------------------------------------------------------- */
typedef struct yand_mlp yand_mlp;

/* Features per instance built by the warm start (see yand_warmstart_features). */
#define YAND_WS_FEATURES 11

typedef struct yand_mlp_opts {
  int hidden;      /* width of every hidden layer (512)                       */
  int layers;      /* weight layers: hidden layers + 1 (4)                    */
  int epochs;      /* full-batch Adam steps (2000)                            */
  double lr;       /* Adam step size (1e-3)                                   */
  uint64_t seed;   /* initial weights N(0, 1/fan_in), counter-based           */
} yand_mlp_opts;

void yand_default_mlp_opts(yand_mlp_opts* opts);

/* Network in_dim -> hidden (tanh) x (layers-1) -> out_dim (linear), FP32,
 * weights initialised from seed, Adam moments zero.  Work runs on hip_stream
 * (NULL = default).  Errors: YAND_ERR_ARG, YAND_ERR_OOM, YAND_ERR_HIP. */
int yand_mlp_create(int64_t in_dim, int64_t out_dim, int hidden, int layers,
                    uint64_t seed, void* hip_stream, yand_mlp** out);
int yand_mlp_destroy(yand_mlp* mlp);
/* Number of FP32 parameters: for each layer l, W_l (fan_in x fan_out,
 * row-major, x W convention) followed by b_l (fan_out). -1 for NULL. */
int64_t yand_mlp_num_params(const yand_mlp* mlp);
/* Copy the parameter vector to / from a device buffer of num_params floats. */
int yand_mlp_get_params(const yand_mlp* mlp, float* dst);
int yand_mlp_set_params(yand_mlp* mlp, const float* src);
/* out (N x out_dim) = network(X (N x in_dim)); device, row-major. */
int yand_mlp_forward(yand_mlp* mlp, int64_t N, const float* X, float* out);
/* Gradient of (1/2N) sum_i |out_i - Y_i|^2 with respect to the parameters by
 * backpropagation; grad (device, num_params) and loss (host) are nullable.
 * The gradient is also kept in the handle for yand_mlp_adam_step. */
int yand_mlp_loss_grad(yand_mlp* mlp, int64_t N, const float* X,
                       const float* Y, float* grad, double* loss);
/* One bias-corrected Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the
 * handle's step counter; grad NULL uses the last yand_mlp_loss_grad result. */
int yand_mlp_adam_step(yand_mlp* mlp, const float* grad, double lr);

/* Reduced coordinates, FP64 device rows: Y[b] = U^T (W[b] - 1/n)
 * (N x n -> N x (n-1)) and its inverse W[b] = 1/n + U Y[b]. */
int yand_reduced_coords(int64_t N, int64_t n, const double* W, double* Y,
                        void* hip_stream);
int yand_from_reduced(int64_t N, int64_t n, const double* Y, double* W,
                      void* hip_stream);

/* Features of N instances (C4 host N x 4, targets host N or NULL) on ctx,
 * into F (host, N x YAND_WS_FEATURES): log1p(c1..c4), has_target,
 * (r - mean(mu)) / |mu - mean(mu)|, and from the equal-weight portfolio
 * z = A 1/n: log m2, m3 / m2^1.5, log(m4 / m2^2), mean(mu) / sqrt(m2),
 * |mu - mean(mu)| / sqrt(n m2).  One value pass over A. */
int yand_warmstart_features(yand_ctx* ctx, int64_t N, const double* C4,
                            const double* targets, double* F);

/* Train a warm-start network on N solved instances of ctx: W_solved (device,
 * N x n) holds their weights.  Features are standardised per column and the
 * reduced coordinates per column mean and one global scale; training is
 * full-batch Adam for opts->epochs steps on the context's stream.  final_loss
 * (host, nullable) receives the last loss.  *out is NULL on error. */
int yand_warmstart_train(yand_ctx* ctx, int64_t N, const double* C4,
                         const double* targets, const double* W_solved,
                         const yand_mlp_opts* opts, yand_mlp** out,
                         double* final_loss);

/* Warm starts for B instances on ctx (same n as in training): each proposal
 * w = 1/n + U y is moved onto the budget (and target) constraint, then its
 * reduced-gradient norm is compared with that of the plain start (equal
 * weights moved onto the constraints); the smaller wins and goes to row b of
 * W0_out (device, B x n).  used_mlp (host, B, nullable) is 1 where the
 * proposal won; gnorms (host, B x 2, nullable) receives both norms.  For the
 * BUDGET set (the proposal may hold negative weights). */
int yand_warmstart_predict(yand_ctx* ctx, yand_mlp* mlp, int64_t B,
                           const double* C4, const double* targets,
                           double* W0_out, int* used_mlp, double* gnorms);

#ifdef __cplusplus
}
#endif

#endif /* YAND_H */
