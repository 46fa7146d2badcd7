/*
 * libslse — SLSE-FRS (Sequential Least-Squares Estimators with Fast Randomized
 * Sketching, Chen, Xie and Yang) on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every call returns an slse_status; on failure slse_last_error()
 * returns a message for the calling thread.  No C++ exception crosses the ABI.
 *
 * Conventions
 *  - X is row-major N x d with leading dimension ldx >= d (elements); Y is a
 *    contiguous length-N vector.  [X|Y] is the tall data of the linear model
 *    Y = X beta + zeta (problem statement, Sec. 1).
 *  - Pointers to X, Y, sketch buffers, beta, gradients and factors are DEVICE
 *    pointers owned by the caller unless stated otherwise.  Structs passed by
 *    pointer (problem, params, layout, report) live in HOST memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are enqueued on it and return before the work finishes, except
 *    where a call fills a host report.
 *  - A context (slse_ctx) is bound to one device.  It owns scratch device
 *    memory (grown on demand, freed by slse_ctx_destroy), cached
 *    preconditioners and captured hipGraphs.  One context must not be used by
 *    two host threads at once.
 */
#ifndef SLSE_H
#define SLSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLSE_OK = 0,
  SLSE_EINVAL = -1,       /* bad argument (null pointer, size, alignment, ordering) */
  SLSE_ENOMEM = -2,       /* device allocation failed */
  SLSE_EDEVICE = -3,      /* a HIP runtime call failed */
  SLSE_ESINGULAR = -4,    /* zero, negative or non-finite pivot in the factorization */
  SLSE_ENOTCONV = -5,     /* tolerance not met within s_max steps (beta holds the last iterate) */
  SLSE_ENONFINITE = -6,   /* NaN/Inf met in the iteration */
  SLSE_EUNSUPPORTED = -7  /* valid request this library does not implement */
} slse_status;

typedef enum { SLSE_F32 = 0, SLSE_F64 = 1, SLSE_BF16 = 2 } slse_dtype;

/* Sketch families (Sec. 1.2; SRHT of Sec. 3; CountSketch of Sec. 5.4). */
typedef enum { SLSE_SRHT = 0, SLSE_COUNTSKETCH = 1, SLSE_GAUSSIAN = 2 } slse_sketch_kind;

/* Factorization of the Hessian sketch (implementation-details appendix):
 *  SLSE_FACTOR_CHOL  through the Gram matrix (Cholesky; inside the solve the
 *                    Gram matrix is inverted directly).  Fine while the
 *                    sketch's condition number is well below u^{-1/2} ~ 1e8.
 *  SLSE_FACTOR_QR    the R factor of the QR of the sketch by shifted
 *                    CholeskyQR3 (Fukaya et al., SIAM J. Sci. Comput. 2020),
 *                    for condition numbers up to about u^{-1}. */
typedef enum { SLSE_FACTOR_CHOL = 0, SLSE_FACTOR_QR = 1 } slse_factor_method;

/* SLSE_PREC_F64: everything in FP64.  SLSE_PREC_MIXED: data stored, sketched
 * and streamed in FP32; FP64 factorization, preconditioner and update; the
 * full-data sweeps accumulate in FP32 for the first `fp32_sweeps` stage-2
 * steps and in FP64 afterwards. */
typedef enum { SLSE_PREC_F64 = 0, SLSE_PREC_MIXED = 1 } slse_precision;

#define SLSE_MAX_LEVELS 40

/* Where slse_sketch_apply put each nested sketch (S_i X, S_i Y), i = 1..K
 * (Sec. 2: (S_i X, S_i Y) is extracted from (S_{i+1} X, S_{i+1} Y)).
 * Level i occupies rows [offset[i], offset[i] + m[i]) of A; its M-IHS
 * gradient is scale[i] * B^T (b - B beta) with [B | b] those rows.
 * H_hat = hat_scale * Ahat[:, :d]^T Ahat[:, :d]. */
typedef struct {
  int32_t K;
  int64_t m[SLSE_MAX_LEVELS];
  int64_t offset[SLSE_MAX_LEVELS];
  double scale[SLSE_MAX_LEVELS];
  int64_t rows_A;
  int64_t r;
  double hat_scale;
  int64_t n_pad; /* N' = 2^ceil(log2 N) for SRHT, N otherwise */
} slse_sketch_layout;

const char* slse_last_error(void);
const char* slse_version(void);

typedef struct slse_ctx slse_ctx;

/* Create a context on HIP device `device`.  *out receives a new context. */
slse_status slse_ctx_create(slse_ctx** out, int device);
/* Free the context, its scratch memory and graphs.  NULL is accepted. */
slse_status slse_ctx_destroy(slse_ctx* ctx);
/* Release the context's scratch memory and cached graphs (they regrow on use). */
slse_status slse_ctx_trim(slse_ctx* ctx);
/* The launch shapes the context has tuned (residual-gradient pass and batched
 * steps, per shape) saved to / loaded from a text file, so a later process skips
 * the timing runs.  The file names the device architecture and compute-unit
 * count; loading a file of another part loads nothing (*loaded = 0).  Shapes only
 * set launch parameters, never what is computed.
 *  loaded   host, may be NULL: the number of entries taken from the file.
 * Errors: EINVAL for null pointers or an unreadable / unwritable / malformed file. */
slse_status slse_ctx_save_tuning(slse_ctx* ctx, const char* path);
slse_status slse_ctx_load_tuning(slse_ctx* ctx, const char* path, int32_t* loaded);

/*
 * slse_sketch_apply — apply the nested sketches S_1..S_K and the Hessian
 * sketch S_hat to [X|Y] (Alg. 2 input (S_0 X, S_0 Y); the efficient
 * construction of Sec. 3; CountSketch and Gaussian of Sec. 1.2).
 *
 *  kind, seed   sketch family and the key of every random choice it makes
 *               (D signs, permutation P, sample orders, hashes, Gaussian
 *               entries all come from Philox4x64-10 keyed by (seed, stream)).
 *  N, d         rows and columns of X (N > d >= 1).
 *  X, ldx, Y    device data in dtype in_t (SLSE_F32 or SLSE_F64).
 *  m[0..K-1]    strictly increasing sketch sizes m_1 < ... < m_K (host array,
 *               1 <= K <= SLSE_MAX_LEVELS).  SRHT: m_K <= N'.  CountSketch:
 *               every m_i a power of 2 and m_{i+1} = 2 m_i.
 *  r            rows of S_hat (d < r; SRHT: r <= N').
 *  A, lda       device output, rows_A x (d+1) in out_t, lda >= d+1.
 *               SRHT/Gaussian: rows_A = m_K and level i is the prefix of m_i
 *               rows (unscaled transform rows; scale c_i = 1/m_i).
 *               CountSketch: rows_A = m_1 + ... + m_K, levels back to back,
 *               c_i = 1.
 *  Ahat, ldah   device output, r x (d+1) in out_t, ldah >= d+1.
 *  out_t        SLSE_F32 or SLSE_F64, equal to in_t; or SLSE_BF16 for a Gaussian
 *               sketch of F32 data computed on the matrix cores with BF16 operands
 *               (G and [X|Y] rounded to BF16) and FP32 accumulation: A and Ahat are
 *               then written as F32.
 *  layout_out   host, filled with the level offsets and scales (may be NULL).
 * Errors: EINVAL for null pointers, sizes or orderings above; EUNSUPPORTED for
 * dtype pairs not listed; ENOMEM when scratch cannot grow.
 */
slse_status slse_sketch_apply(slse_ctx* ctx, slse_sketch_kind kind, uint64_t seed, int64_t N,
                              int64_t d, const void* X, int64_t ldx, const void* Y,
                              slse_dtype in_t, const int64_t* m, int32_t K, int64_t r, void* A,
                              int64_t lda, void* Ahat, int64_t ldah, slse_dtype out_t,
                              slse_sketch_layout* layout_out, void* stream);

/*
 * slse_factor — factor the Hessian sketch H_hat = (S_hat X)^T S_hat X
 * (Sec. 3) applied through R (the QR route of the implementation-details
 * appendix): R upper triangular d x d with nonnegative diagonal and
 * R^T R = scale * A[:, :d]^T A[:, :d].
 *  rows, d    size of the sketch block (rows >= d).
 *  A, lda     device, rows x d (only the first d columns are read), dtype a_t
 *             (SLSE_F32 or SLSE_F64).
 *  R, ldr     device FP64 output, upper triangle written, strict lower zeroed.
 *  M, ldm     optional device FP64 output (may be NULL): the preconditioner
 *             matrix M = (R^T R)^{-1}, d x d, symmetric.
 * Errors: EINVAL; ESINGULAR when a pivot is zero, negative or non-finite
 * (the status is read back from the device, so this call synchronizes the
 * stream).
 */
slse_status slse_factor(slse_ctx* ctx, int64_t rows, int64_t d, const void* A, int64_t lda,
                        slse_dtype a_t, double scale, slse_factor_method method, double* R,
                        int64_t ldr, double* M, int64_t ldm, void* stream);

/*
 * slse_fused_resid_grad — g = scale * X[0:n]^T (Y[0:n] - X[0:n] beta), the
 * negative gradient -scale * grad f(beta; X, Y) with grad f = X^T (X beta - Y)
 * (Sec. 1), read in one pass over X (each row is loaded once; its residual is
 * formed in registers and immediately folded into g).
 *  n, d           rows and columns (n >= 0; n = 0 gives g = 0).
 *  X, ldx         device, dtype storage (SLSE_F32 or SLSE_F64).
 *  Y              device, length n, same dtype; NULL means Y = 0.
 *  beta           device FP64, length d.
 *  accum          SLSE_F32 or SLSE_F64: type of the residual and of the
 *                 per-thread sums (cross-block sums are FP64 in a fixed order,
 *                 so results are bit-reproducible for a given launch shape).
 *  g_out          device FP64, length d.
 *  rnorm2_out     device FP64 scalar, scale * ||Y - X beta||^2, or NULL.
 */
slse_status slse_fused_resid_grad(slse_ctx* ctx, int64_t n, int64_t d, const void* X, int64_t ldx,
                                  const void* Y, slse_dtype storage, const double* beta,
                                  double scale, slse_dtype accum, double* g_out,
                                  double* rnorm2_out, void* stream);

/*
 * slse_fused_resid_grad_noalloc — slse_fused_resid_grad for callers that cannot
 * allocate device memory (code under hipGraph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, result and errors; the
 * call allocates nothing: the pass's partial sums live in a fixed device array
 * of the library (about 4.4 MB per device, held until the process ends) that
 * slse_ctx_create locates on its device.  Limits: d <= 1024 (EINVAL above) and
 * grids of at most 512 blocks (the tuned launch shape of slse_fused_resid_grad
 * is reused when known and capped there).  Every call on one device uses the
 * same array, so calls that overlap on a device (other streams, other host
 * threads) race; the array keeps the last call's partials.
 */
slse_status slse_fused_resid_grad_noalloc(slse_ctx* ctx, int64_t n, int64_t d, const void* X,
                                          int64_t ldx, const void* Y, slse_dtype storage,
                                          const double* beta, double scale, slse_dtype accum,
                                          double* g_out, double* rnorm2_out, void* stream);

typedef struct {
  int64_t N, d;
  const void* X;
  int64_t ldx;
  const void* Y;
  slse_dtype dtype; /* storage of X and Y: SLSE_F32 or SLSE_F64 */
} slse_problem;

typedef struct {
  slse_sketch_kind kind;
  uint64_t seed;
  int32_t K;
  int64_t m[SLSE_MAX_LEVELS]; /* sketch sizes m_1 < ... < m_K */
  int32_t a[SLSE_MAX_LEVELS]; /* M-IHS steps a_i on subproblem i (Alg. 2) */
  int64_t r;                  /* Hessian sketch rows */
  double mu, eta;             /* step sizes; Sec. 5 uses eta = d/r, mu = (1-eta)^2 */
  int32_t s_max;              /* stage-2 (full-data) steps, or the cap when tol > 0 */
  double tol;                 /* > 0: stop stage 2 at the first step whose estimate
                                 ||H_hat^{-1} g_t|| / ||beta_{t+1}|| of the relative error of
                                 beta_t (beta_hat - beta_t = H^{-1} g_t) is <= tol */
  slse_precision precision;
  int32_t fp32_sweeps;        /* MIXED only, see slse_precision */
  int32_t momentum_reset;     /* 1: beta_{t-1} := beta_t at each subproblem and stage start */
  slse_factor_method factor;
  const double* beta0;        /* device, d; NULL = 0 */
  double* trajectory;         /* device, (sum a_i + s_max + 1) x d, row t = beta_t; or NULL */
  double* surrogate;          /* device, (sum a_i + s_max): the estimate above, per step; or NULL */
  int32_t use_graph;          /* 1: capture the whole solve once and replay it as a hipGraph */
  /* Per-iterate error accounting against a caller's reference vector (for example
   * the OLS solution, or the true coefficients of a synthetic model), written for
   * t = 0..T (T = sum a_i + s_max), row t describing beta_t.  With tol > 0 the
   * entries after the step that met tol are unspecified. */
  const double* beta_ref;     /* device, d; required when rel_err or pred_err is set */
  double* rel_err;            /* device, T+1: ||beta_t - beta_ref|| / ||beta_ref||; or NULL */
  double* pred_err;           /* device, T+1: ||X (beta_t - beta_ref)||^2, the prediction error
                                 Delta_t of the experiments (Sec. 5) when beta_ref is the true
                                 beta; or NULL.  Costs one extra read of X per iterate. */
  /* Checkpoint and resume.  The sketch is a function of the seed, so the whole
   * state of the iteration after step t - 1 is (beta_t, beta_{t-1}).  Steps are
   * numbered t = 0..T-1 over the whole solve (stage 1 subproblem by subproblem,
   * then stage 2; T = sum a_i + s_max).  The call sketches and factors, then
   * runs steps start_step .. stop_step - 1 from beta_{start_step} = beta0 and
   * beta_{start_step - 1} = beta_prev.  A momentum reset (momentum_reset) at the
   * start of a subproblem or of stage 2 happens when its first step is run.
   * trajectory rows and the surrogate and error entries keep their indices t;
   * those of steps not run are not written.  A stopped run resumed from its
   * state_out retraces the uninterrupted run (Alg. 2 keeps one global t). */
  int32_t start_step;         /* first step to run, 0 <= start_step <= stop */
  int32_t stop_step;          /* run the steps t < stop_step; 0 = T */
  const double* beta_prev;    /* device, d: beta_{start_step - 1}; NULL = beta0 */
  double* state_out;          /* device, 2 x d: (beta_{t-1}, beta_t) for the last iterate t
                                 computed, the checkpoint to resume from; or NULL.  After a
                                 stop on tol the pair is unspecified. */
} slse_params;

typedef struct {
  slse_status status;
  int32_t stage1_steps; /* stage-1 steps run by this call */
  int32_t stage2_steps; /* stage-2 steps run by this call (up to the tol stop) */
  double surrogate0;    /* error estimate at the first stage-2 step */
  double surrogate_final; /* error estimate at the last step taken */
  double ms_total;      /* device time of the call (hipEvents) */
  /* device time of each phase of Alg. 2 (hipEvents between the phases); filled
   * when use_graph = 0 (a replayed graph is timed only as a whole: zeros) */
  double ms_sketch;     /* S_0 [X|Y]: every nested sketch and the Hessian sketch */
  double ms_factor;     /* H_hat = (S_hat X)^T S_hat X and its inverse */
  double ms_stage1;     /* the a_i M-IHS steps on the sketched subproblems (eq. (98)) */
  double ms_stage2;     /* the full-data M-IHS steps (eq. (99)), with any error accounting */
} slse_report;

/*
 * slse_solve — Alg. 2 (An Efficient SLSE-FRS): sketch once, factor H_hat,
 * run a_i M-IHS steps (eq. (98)) on each nested sketched subproblem, then
 * s_max full-data M-IHS steps (eq. (99)).  beta_{-1} = beta_0; momentum
 * carries across subproblems unless momentum_reset.
 *  beta_out   device FP64, length d: beta_T.
 *  rep        host report or NULL.  When non-NULL the call synchronizes the
 *             stream to fill it.
 * Errors: EINVAL (see slse_sketch_apply for the sizes; also start_step or
 * stop_step outside 0..T, or start_step > stop), ESINGULAR from the
 * factorization, ENOTCONV when tol > 0 was not met (beta_out still holds
 * the last iterate), ENONFINITE when the surrogate is not finite.
 */
slse_status slse_solve(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                       double* beta_out, slse_report* rep, void* stream);

/*
 * slse_workspace_size — device bytes that slse_solve_ws needs for this problem
 * and these parameters (the sketch levels and the Hessian sketch, the SRHT /
 * CountSketch / Gaussian scratch, the factor buffers, the iterate ring and the
 * reduction partials of Alg. 2).  No device work, no allocation.
 *  bytes   host, receives the size.
 * Errors: EINVAL for the same argument errors slse_solve reports.
 */
slse_status slse_workspace_size(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                                size_t* bytes);

/*
 * slse_solve_ws — slse_solve with every scratch buffer carved from the caller's
 * device workspace ws[0 .. ws_bytes) (256-byte aligned regions, in a fixed
 * order) instead of the context's own memory, so the call allocates no device
 * memory.  The workspace is the caller's: it must stay valid until the stream
 * has finished the call, and calls that share one workspace must not overlap.
 * The context still keeps the launch-shape cache and, with use_graph, a graph
 * per (problem, params, beta_out, ws) that is replayed on later calls.  A solve
 * through a workspace does not leave a preconditioner for slse_backward.
 *  ws, ws_bytes   device workspace, at least slse_workspace_size bytes.
 * Errors: as slse_solve; EINVAL when ws is NULL or ws_bytes is too small.
 */
slse_status slse_solve_ws(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                          double* beta_out, slse_report* rep, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * slse_ihs — the iterative Hessian sketch baseline (the IHS update of Sec. 1):
 * s_max full-data steps
 *     beta_{t+1} = beta_t + H_t^{-1} X^T (Y - X beta_t),  H_t = (S_t X)^T S_t X,
 * each with a Hessian sketch S_t of r rows drawn anew from the key seed + t (the
 * Hessian-sketch rows of slse_sketch_apply under that key; the call also forms one
 * nested level of the power of 2 >= r rows, which IHS does not use).  It is
 * eq. (99) with mu = 1 and eta = 0 and a fresh H_hat per step.  Read from q: kind,
 * seed, r, s_max, precision, factor, beta0, trajectory, use_graph; m, a, mu, eta,
 * tol, the error-accounting and the checkpoint fields are ignored.
 *  beta_out   device FP64, length d: beta_{s_max}.
 * Errors: as slse_solve.
 */
slse_status slse_ihs(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                     double* beta_out, slse_report* rep, void* stream);

/*
 * Parameter helpers (host only, no device work, no context).
 *
 * slse_paper_schedule — the sketch sizes of the experiments (Sec. 5): m_1 =
 * m1_factor * d (8d in the paper) rounded up to a power of 2, m_{i+1} = 2 m_i
 * (the constant ratio of the nested construction, Sec. 3), up to m_K = N/2
 * rounded down to a power of 2.
 *  m_out   host array of cap entries; *K_out receives K.
 * Errors: EINVAL for N <= d, d < 1, m1_factor < 1, null pointers, an empty
 * schedule (m_1 > N/2) or cap < K.
 */
slse_status slse_paper_schedule(int64_t N, int64_t d, int64_t m1_factor, int64_t* m_out,
                                int32_t cap, int32_t* K_out);

/*
 * slse_paper_params — the Hessian-sketch size and step sizes of the experiments
 * (Sec. 5): r = 6d when r_in <= 0 (else r_in), eta = d/r, mu = (1 - eta)^2.
 * Errors: EINVAL for d < 1, r <= d or null pointers.
 */
slse_status slse_paper_params(int64_t d, int64_t r_in, int64_t* r_out, double* mu, double* eta);

/*
 * slse_stage1_counts — stage-1 step counts from the lower bound of Thm
 * lowerBoundai (Sec. 4): for i >= 2, a_i is the smallest integer >= 1 with
 *     3^{a_i} >= ((1 + omega) r(i-1, i) + 1) / omega,
 *     r(i-1, i) = sqrt((m_i - d) / (m_{i-1} - d)).
 * a_1 (whose bound, Thm a1, needs the first subproblem's unknown errors) is a1
 * when a1 >= 1, else a_2 (2 when K = 1).
 *  m       host, K sizes with m_{i-1} > d for i >= 2.
 *  a_out   host, K counts.
 * Errors: EINVAL for K < 1, null pointers, omega not in (0, 1], or m_{i-1} <= d.
 */
slse_status slse_stage1_counts(const int64_t* m, int32_t K, int64_t d, double omega, int32_t a1,
                               int32_t* a_out);

/*
 * slse_backward — adjoint of beta_hat(X, Y) for a loss L with
 * dL/dbeta_hat = w: lambda solves (X^T X) lambda = w by the same
 * sketch-preconditioned M-IHS iteration (lambda_0 = H_hat^{-1} w, then s_max
 * full-data steps), then one fused pass writes
 *     dY = X lambda,   dX = r lambda^T - (X lambda) beta_hat^T,  r = Y - X beta_hat
 * (from differentiating the normal equations of the problem statement).
 * The preconditioner of the last slse_solve on the same data, seed and sizes
 * is reused when the context still holds it; otherwise it is rebuilt.  The
 * error-accounting and checkpoint fields of q are ignored.
 *  beta_hat      device FP64, length d.
 *  w, incw       device FP64, entry k at w[k * incw] (incw >= 0; 0 repeats w[0]).
 *  dX, lddx      device output N x d in grad_t (F32 or F64), or NULL.
 *  dY            device output length N in grad_t, or NULL.
 *  lambda_out    device FP64 length d, or NULL.
 */
slse_status slse_backward(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                          const double* beta_hat, const double* w, int64_t incw, void* dX,
                          int64_t lddx, void* dY, slse_dtype grad_t, double* lambda_out,
                          slse_report* rep, void* stream);

/*
 * slse_solve_batched — B independent problems (any N_b, d_b) solved as one
 * launch sequence: the sketch, factor and every M-IHS step of all problems
 * run in shared persistent kernels over a (problem, row-tile) work list, the
 * whole sequence captured once as a hipGraph and replayed.  Problems whose
 * schedule is shorter idle through the extra steps.
 *  ps, qs      host arrays of B problems and parameters (trajectory,
 *              surrogate and use_graph fields are ignored; the checkpoint
 *              fields must be zero / NULL: EINVAL otherwise).
 *  betas       host array of B device pointers (FP64, length d_b each).
 *  reps        host array of B reports, or NULL.
 * Every problem of a batch shares one storage dtype and has d_b <= 512
 * (d_b <= 256 when some problem's rows are not 16-byte aligned); EINVAL
 * otherwise.
 * Returns the worst status of the batch.
 */
slse_status slse_solve_batched(slse_ctx* ctx, int32_t B, const slse_problem* ps,
                               const slse_params* qs, double* const* betas, slse_report* reps,
                               void* stream);

/*
 * Test hooks: the library's own counter-based streams, written to a device
 * buffer so that they can be compared bit for bit with an independent
 * implementation.
 *  what: 0 Philox words (4 per counter c0 = start + i, c1 = aux, key (seed, stream_id))
 *        1 permutation pi(x) of [0, 2^aux) for x = start + i (stream_id selects P, sigma,
 *          sigma_hat), 2 its inverse,
 *        3 Rademacher sign D_j (+1/-1) for j = start + i,
 *        4 CountSketch bucket h(j) mod aux (aux a power of 2), 5 its sign,
 *        6 Hessian CountSketch bucket into [0, aux), 7 its sign.
 *  out: device int64 (uint64 bit patterns for what = 0), count entries (4*count for what 0).
 */
slse_status slse_debug_stream(slse_ctx* ctx, int32_t what, uint64_t seed, int32_t stream_id,
                              int64_t aux, int64_t start, int64_t count, int64_t* out,
                              void* stream);
/* Tiles of one batched step, as slse_solve_batched cuts them (host only, no
 * device work): problem b has n[b] rows (0: idle) of row_bytes[b] bytes and
 * a main loop of step_rows[b] rows per block step; slots = grid x tiles per
 * block; min_tile_bytes is the smallest tile.  Writes tile_rows[b] and
 * ntiles[b] (host arrays of B).  EINVAL on null pointers or sizes <= 0. */
slse_status slse_debug_batch_tiles(int32_t B, const int64_t* n, const int64_t* row_bytes,
                                   const int64_t* step_rows, int64_t slots, int64_t min_tile_bytes,
                                   int32_t* tile_rows, int32_t* ntiles);
/* The host plan of slse_solve_batched for these problems, made without any
 * device work or allocation (every buffer is placed at an offset from a fake
 * base), then checked: each problem's regions lie inside their pools, the
 * per-step tile tables cover every row once, and the SRHT index and record
 * tables stay inside their sizes.  A failed check returns EINVAL with a
 * message.  bytes_out (host, may be NULL) receives the device bytes the batch
 * needs.  The betas of the problems are not read. */
slse_status slse_debug_batch_plan(int32_t B, const slse_problem* ps, const slse_params* qs,
                                  size_t* bytes_out);
/* Reference streams for measurement (no method arithmetic): mode 0 reads bytes of src
 * with 16-byte non-temporal loads, one contiguous chunk per block, and writes one word per
 * block to dst (device, >= 4 * blocks bytes); mode 1 copies src to dst (device, bytes).
 * bytes a multiple of 16, src and dst 16-byte aligned; blocks <= 0 means one per compute
 * unit. */
slse_status slse_debug_bandwidth(slse_ctx* ctx, int32_t mode, const void* src, void* dst,
                                 int64_t bytes, int32_t blocks, void* stream);
/* Gaussian sketch entries G[k0 + a, j0 + b] (a < nk, b < nj) of stream 7 (S) or 8 (S_hat),
 * written row-major to `out` (device, FP64) as the library computes them: form 0 as the
 * FP32/FP64 sketch kernels do (FP32 Box-Muller), form 1 as the BF16 matrix-core kernel
 * does (FP32 Box-Muller on the hardware transcendentals, rounded to BF16). */
slse_status slse_debug_gaussian(slse_ctx* ctx, uint64_t seed, int32_t stream_id, int32_t form,
                                int64_t k0, int64_t nk, int64_t j0, int64_t nj, double* out,
                                void* stream);
/* Reference for measurement: the matrix-core Gaussian sketch's generation of the m x N
 * entries of G alone (Philox block, Box-Muller, BF16 rounding), with no data read and no
 * product formed; one checksum word per thread into sink (device, >= 256 * blocks words).
 * Its time is the floor that generating G sets for a sketch of m rows of N data rows. */
slse_status slse_debug_gaussian_generate(slse_ctx* ctx, uint64_t seed, int32_t stream_id,
                                        int64_t m, int64_t N, int32_t blocks, uint32_t* sink,
                                        void* stream);
/* Data-row splits the Gaussian sketch of N x (d+1) data into m sketch rows uses (host only):
 * bf16 = 1 for the matrix-core form on F32 data, 0 for the FP32/FP64 form.  Each split sums
 * its own contiguous range of data rows; the ranges are added in split order. */
slse_status slse_debug_gaussian_plan(int64_t N, int64_t d, int64_t m, int32_t bf16,
                                     int32_t* splits);

#ifdef __cplusplus
}
#endif

#endif /* SLSE_H */
