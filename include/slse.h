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
  SLSE_EUNSUPPORTED = -7  /* valid request this build does not implement */
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
} slse_params;

typedef struct {
  slse_status status;
  int32_t stage1_steps;
  int32_t stage2_steps; /* steps actually taken */
  double surrogate0;    /* error estimate at the first stage-2 step */
  double surrogate_final; /* error estimate at the last step taken */
  double ms_total;      /* device time of the call (hipEvents), when requested */
} slse_report;

/*
 * slse_solve — Alg. 2 (An Efficient SLSE-FRS): sketch once, factor H_hat,
 * run a_i M-IHS steps (eq. (98)) on each nested sketched subproblem, then
 * s_max full-data M-IHS steps (eq. (99)).  beta_{-1} = beta_0; momentum
 * carries across subproblems unless momentum_reset.
 *  beta_out   device FP64, length d: beta_T.
 *  rep        host report or NULL.  When non-NULL the call synchronizes the
 *             stream to fill it.
 * Errors: EINVAL (see slse_sketch_apply for the sizes), ESINGULAR from the
 * factorization, ENOTCONV when tol > 0 was not met (beta_out still holds
 * the last iterate), ENONFINITE when the surrogate is not finite.
 */
slse_status slse_solve(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                       double* beta_out, slse_report* rep, void* stream);

/*
 * slse_backward — adjoint of beta_hat(X, Y) for a loss L with
 * dL/dbeta_hat = w: lambda solves (X^T X) lambda = w by the same
 * sketch-preconditioned M-IHS iteration (lambda_0 = H_hat^{-1} w, then s_max
 * full-data steps), then one fused pass writes
 *     dY = X lambda,   dX = r lambda^T - (X lambda) beta_hat^T,  r = Y - X beta_hat
 * (from differentiating the normal equations of the problem statement).
 * The preconditioner of the last slse_solve on the same data, seed and sizes
 * is reused when the context still holds it; otherwise it is rebuilt.
 *  beta_hat, w   device FP64, length d.
 *  dX, lddx      device output N x d in grad_t (F32 or F64), or NULL.
 *  dY            device output length N in grad_t, or NULL.
 *  lambda_out    device FP64 length d, or NULL.
 */
slse_status slse_backward(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                          const double* beta_hat, const double* w, void* dX, int64_t lddx,
                          void* dY, slse_dtype grad_t, double* lambda_out, slse_report* rep,
                          void* stream);

/*
 * slse_solve_batched — B independent problems (any N_b, d_b) solved as one
 * launch sequence: the sketch, factor and every M-IHS step of all problems
 * run in shared persistent kernels over a (problem, row-tile) work list, the
 * whole sequence captured once as a hipGraph and replayed.  Problems whose
 * schedule is shorter idle through the extra steps.
 *  ps, qs      host arrays of B problems and parameters (trajectory,
 *              surrogate and use_graph fields are ignored).
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
/* Gaussian sketch entries G[k0 + a, j0 + b] (a < nk, b < nj) of stream 7 (S) or 8 (S_hat),
 * written row-major to `out` (device, FP64) as the library computes them in FP32. */
slse_status slse_debug_gaussian(slse_ctx* ctx, uint64_t seed, int32_t stream_id, int64_t k0,
                                int64_t nk, int64_t j0, int64_t nj, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SLSE_H */
