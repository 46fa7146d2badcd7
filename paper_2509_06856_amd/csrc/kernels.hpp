// Internal launchers of libslse's device kernels.  Every launcher enqueues on
// `stream` and checks the launch; shapes are validated by the caller.
#pragma once

#include <vector>

#include "common.hpp"

namespace slse {

// --------------------------------------------------------------------------
// Fused residual-gradient (one pass over X): per-group partial sums of
//   X[0:n]^T (Y - X beta)   and   ||Y - X beta||^2
// written to gpart[group][0..d] (index d holds the residual norm).  The
// launch reduces its block partials to `groups` rows itself (the last block
// of each group sums its group's blocks in a fixed order).
// --------------------------------------------------------------------------
struct ResidGradPlan {
  int blocks = 0;
  int groups = 0;
  int group_size = 0;
  int lpr = 0;   // lanes per row
  int vec = 0;   // elements per vector load
  int nch = 0;   // vector chunks per lane
  int ldp = 0;   // leading dimension of partial rows (>= d + 1)
  bool full = false;  // d = nch * lpr * vec: every lane's chunks are whole vectors
};

// lpr_hint > 0 picks the lane-group width (else a default); grid_blocks is the
// target grid, capped by `capacity` (the rows allocated for block partials).
ResidGradPlan plan_resid_grad(int64_t n, int d, slse_dtype storage, const void* X, int64_t ldx,
                              int grid_blocks, int capacity, int lpr_hint = 0);

struct ResidGradArgs {
  int64_t n = 0;
  int d = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  const void* Y = nullptr;  // may be null (Y = 0)
  int64_t incy = 1;
  slse_dtype storage = SLSE_F64;
  slse_dtype accum = SLSE_F64;
  const double* beta = nullptr;
  double* partial = nullptr;  // [blocks][ldp]
  double* gpart = nullptr;    // [groups][ldp]
  int* counters = nullptr;    // [groups], zero before the first launch; left zero
  int capacity_blocks = 0;    // rows allocated in `partial` (groups: ceil(capacity / 32))
  const int* done = nullptr;  // optional early-exit flag
};

void launch_resid_grad(const ResidGradPlan& pl, const ResidGradArgs& a, hipStream_t s);

// g = scale * sum_g gpart[g][0..d) (and rnorm2 = scale * sum_g gpart[g][d]).
void launch_finalize_grad(const double* gpart, int groups, int ldp, int d, double scale,
                          double* g_out, double* rnorm2_out, hipStream_t s);

// --------------------------------------------------------------------------
// M-IHS update (eqs. (98)/(99)) with the preconditioner M = H_hat^{-1}:
//   g      = scale * sum_groups gpart (+ w)
//   p      = M g
//   beta'  = beta + mu p + eta (beta - beta_prev)
// surrogate ||R^{-T} g||^2 = g . p is reduced into sur_out[0] (if given);
// when tol2 > 0 the step that brings it to <= tol2 * sur_ref[0] raises
// `done`, and later steps are skipped.
// --------------------------------------------------------------------------
struct UpdateArgs {
  const double* gpart = nullptr;
  int groups = 0;
  int ldp = 0;
  int d = 0;
  double scale = 1.0;
  const double* w = nullptr;  // added to g (adjoint right-hand side), may be null
  int64_t incw = 1;           // stride of w (0: w[0] for every k)
  const double* M = nullptr;
  int64_t ldm = 0;
  const double* beta = nullptr;
  const double* beta_prev = nullptr;
  double* beta_next = nullptr;
  double mu = 1.0;
  double eta = 0.0;
  double* beta_out = nullptr;     // copy of beta_next (may be null)
  double* traj_row = nullptr;     // copy of beta_next (may be null)
  double* sur_partial = nullptr;  // [blocks] scratch
  int* sur_counter = nullptr;     // zero before first use; left zero
  double* sur_out = nullptr;      // surrogate of this step (may be null)
  const double* sur_ref = nullptr;
  double tol2 = 0.0;
  int* done = nullptr;            // early-exit flag (may be null)
  int* status = nullptr;          // set to 1 on a non-finite surrogate (may be null)
};

int update_blocks(int d);
void launch_update(const UpdateArgs& a, hipStream_t s);

// rel_out[0] = ||beta - ref|| / ||ref|| and delta = beta - ref (either may be null).
void launch_iter_error(const double* beta, const double* ref, int d, double* rel_out,
                       double* delta, hipStream_t s);
void launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t s);
void launch_fill_i32(int* dst, int value, int64_t n, hipStream_t s);
void launch_fill_f64(double* dst, double value, int64_t n, hipStream_t s);

// --------------------------------------------------------------------------
// SRHT: index maps and Walsh-Hadamard passes.
// --------------------------------------------------------------------------
struct SrhtArgs {
  slse_dtype t = SLSE_F64;
  int64_t N = 0;
  int d = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  const void* Y = nullptr;
  uint64_t seed = 0;
  int p = 0;  // N' = 2^p
  int64_t mK = 0;
  int64_t r = 0;
  void* A = nullptr;
  int64_t lda = 0;
  void* Ahat = nullptr;
  int64_t ldah = 0;
  // scratch
  int32_t* pi_sgn = nullptr;  // [N']
  int32_t* slotA = nullptr;   // [N']
  int32_t* slotH = nullptr;   // [N']
  void* Z = nullptr;          // [N'][ldz]
  int64_t ldz = 0;
  int ct = 0;                 // column tile (chosen by srht_plan)
  int bmax = 0;               // stages per pass cap
  bool xcd_swizzle = true;    // contiguous work runs per XCD
  bool indices_ready = false; // pi_sgn / slotA / slotH already built (batched)
  bool split_y = false;       // Y transformed on its own: Z = X's d columns, then N' values of Y
  bool y_pregathered = false; // (set at launch) Y gathered through P by the index-map kernel
};

void srht_plan(SrhtArgs& a, int prefer_ct);
// Single transforms whose X columns fill whole column tiles (d a multiple of
// the tile) take Y through its own one-column passes instead of a tile that
// would hold Y and padding (no-op otherwise; SLSE_SRHT_SPLIT_Y=0 disables).
void srht_split_y(SrhtArgs& a);

// Index maps of many SRHTs in two launches (rows of every job, then the r
// Hessian samples of every job).  base/hbase: first global index of the job.
struct SrhtIndexJob {
  int64_t npad;
  int64_t r;
  int64_t mK;
  uint64_t seed;
  int p;
  int s0_last;
  int b_last;
  int pad_;
  int64_t base;
  int64_t hbase;
  int32_t* pi_sgn;
  int32_t* slotA;
  int32_t* slotH;
};
// b_last / s0_last of the pass split srht_plan chooses for `a` (a.p, a.bmax set)
void srht_last_pass(const SrhtArgs& a, int* s0_last, int* b_last);
// index maps of B jobs (max_npad / max_r: the largest npad and r among them)
void launch_srht_index_batched(const SrhtIndexJob* jobs, int B, int64_t max_npad, int64_t max_r,
                               hipStream_t s);
size_t srht_z_bytes(const SrhtArgs& a);
void launch_srht(const SrhtArgs& a, hipStream_t s);

// SRHT passes of many transforms in shared launches (index maps already
// built, one workspace Z per multi-pass transform).  srht_batch_plan writes
// the device parameter records into `records` (host bytes, to be uploaded by
// the caller) and returns the launches; launch_srht_batched enqueues them.
struct SrhtBatchLaunch {
  int b = 0;     // butterfly stages of the pass
  int mode = 0;  // first / last pass flags
  int first = 0;  // first record of the launch
  int count = 0;  // transforms in the launch
  int64_t max_blocks = 0;
};
std::vector<SrhtBatchLaunch> srht_batch_plan(const std::vector<SrhtArgs>& as, slse_dtype t,
                                             std::vector<char>& records);
void launch_srht_batched(const std::vector<SrhtBatchLaunch>& L, const void* d_records, slse_dtype t,
                         hipStream_t s);
// --------------------------------------------------------------------------
// CountSketch and Gaussian sketches.
// --------------------------------------------------------------------------
struct CountSketchArgs {
  slse_dtype t = SLSE_F64;
  int64_t N = 0;
  int d = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  const void* Y = nullptr;
  uint64_t seed = 0;
  const int64_t* m = nullptr;
  int K = 0;
  int64_t r = 0;
  void* A = nullptr;  // levels back to back, m_1 first
  int64_t lda = 0;
  void* Ahat = nullptr;
  int64_t ldah = 0;
  void* scratch = nullptr;  // countsketch_scratch_bytes(*this) bytes: the bucket lists
};
size_t countsketch_scratch_bytes(const CountSketchArgs& a);
void launch_countsketch(const CountSketchArgs& a, hipStream_t s);

struct GaussianArgs {
  slse_dtype t = SLSE_F64;
  int64_t N = 0;
  int d = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  const void* Y = nullptr;
  uint64_t seed = 0;
  int64_t m = 0;
  uint64_t stream_id = 7;
  void* A = nullptr;
  int64_t lda = 0;
  float* partial = nullptr;   // split-K scratch
  double* partial64 = nullptr;
  int splits = 0;
  bool bf16 = false;          // BF16 operands on the matrix cores, FP32 accumulation
  bool tiles_ready = false;   // BF16: the scratch already holds this [X|Y]'s staged tiles
};
size_t gaussian_scratch_bytes(const GaussianArgs& a);
void gaussian_plan(GaussianArgs& a);
void launch_gaussian(const GaussianArgs& a, hipStream_t s);
void launch_debug_gaussian(uint64_t seed, uint64_t stream_id, int64_t k0, int64_t nk, int64_t j0,
                           int64_t nj, int form, double* out, hipStream_t s);
// the matrix-core form's generation of m x N entries of G alone (one checksum
// word per thread of `blocks` x 256 into sink)
void launch_gauss_generate(uint64_t seed, uint64_t stream_id, int64_t m, int64_t N, int blocks,
                           unsigned* sink, hipStream_t s);

// --------------------------------------------------------------------------
// Dense FP64 helpers for the factorization.
// --------------------------------------------------------------------------
// C[MxN] = alpha * op(A) * op(B) + beta * C, all FP64 row-major.  Small outputs
// with long K are split over K into `scratch` (gemm_scratch_doubles entries)
// and summed in split order.
size_t gemm_scratch_doubles(int64_t M, int64_t N, int64_t K);
void launch_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                     bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
                     int64_t ldc, hipStream_t s, double* scratch = nullptr,
                     size_t scratch_doubles = 0);
// out[i][k] = s * A[i][k] for i < rows, k < d (A in F32 or F64).
void launch_convert_scale(int64_t rows, int d, const void* A, int64_t lda, slse_dtype at, double s,
                          double* out, int64_t ldo, hipStream_t st);
// R = upper Cholesky factor of the SPD d x d matrix G (R^T R = G); info[0] = 0 or (j+1) of the
// first bad pivot.  G is read only.
void launch_cholesky(int d, const double* G, int64_t ldg, double* R, int64_t ldr, int* info,
                     hipStream_t s);
// G = G^{-1} in place for SPD G (d x d, ld = d) by blocked Gauss-Jordan; colp
// is d x 32 scratch.  info[0] (zero on entry) becomes k0 + 1 of the first
// pivot block with a non-positive or non-finite pivot.
void launch_spd_inverse(int d, double* G, double* colp, int* info, hipStream_t s);
// G += coef * trace(G) * I (d x d, ld = d).
void launch_shift_diag(int d, double* G, double coef, hipStream_t s);
// Rinv = R^{-1} (upper triangular, row-major d x d) for upper triangular R.
void launch_tri_inv(int d, const double* R, int64_t ldr, double* Rinv, int64_t ldi, hipStream_t s);

// One Cholesky-route factorization of a batch: Ad = scale * A[:, :d] (FP64),
// G = Ad^T Ad, then M = G^{-1} by the blocked Gauss-Jordan steps of the
// single-problem route (info[0]: first non-positive pivot block + 1).  Every
// buffer is the job's own, row-major with leading dimension d (A: lda); G may
// be M (the Gram is then inverted in place).
struct FactorJob {
  const void* A = nullptr;
  int64_t lda = 0;
  int64_t rows = 0;
  int d = 0;
  double scale = 1.0;
  double* Ad = nullptr;
  double* G = nullptr;
  double* M = nullptr;
  double* colp = nullptr;  // d x 32 Gauss-Jordan column panel
  double* part = nullptr;  // splits x d x d partial Grams (factor_batched_splits > 1)
  int* info = nullptr;
};
// row splits of the batched Gram for sketches of at most rows_max rows
int factor_batched_splits(int64_t rows_max);
// All jobs at once (jobs in device memory; dmax, rows_max bound every job).
void launch_factor_batched(const FactorJob* jobs, int B, int dmax, int64_t rows_max,
                           slse_dtype at, hipStream_t s);

// --------------------------------------------------------------------------
// Adjoint rank-2 pass: dY = X lambda, dX = r lambda^T - (X lambda) beta^T.
// --------------------------------------------------------------------------
struct AdjointArgs {
  int64_t n = 0;
  int d = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  const void* Y = nullptr;
  slse_dtype t = SLSE_F64;
  const double* beta = nullptr;
  const double* lambda = nullptr;
  void* dX = nullptr;
  int64_t lddx = 0;
  void* dY = nullptr;
  slse_dtype gt = SLSE_F64;
};
void launch_adjoint(const AdjointArgs& a, hipStream_t s);

// --------------------------------------------------------------------------
// Batched M-IHS steps (many problems per launch).
// --------------------------------------------------------------------------
// batched residual-gradient pass: threads per block, and 16-byte vectors of
// [X|Y] a lane has in flight (a lane group's rows per step of its main loop
// are kBatchSlots / ch)
constexpr int kBatchThreads = 256;
constexpr int kBatchSlots = 8;
struct BatchStep {  // one problem at one global step
  const void* X;
  int64_t ldx;
  const void* Y;
  int64_t incy;
  int64_t n;  // rows of this step (0: the problem is idle)
  double scale;
  const double* beta;
  const double* beta_prev;
  double* beta_next;
  int ntiles;
  int tile_rows;  // rows per tile in this step (the last tile may be short)
};
struct BatchProblem {
  int d;
  int lpr;  // lanes per row (a power of 2 <= 64)
  int ch;   // 16-byte vectors per lane per row (1, 2 or 4)
  int64_t part_off;  // first partial row of this problem in the pool
  const double* M;
  double* beta_out;
  double mu, eta;
  const double* beta0;  // initial iterate (device) or null for 0
  double* beta_init;    // the iterate buffer the first step reads
};
void launch_batched_resid_grad(const BatchStep* steps, const BatchProblem* probs, const int* prefix,
                               int B, int total_tiles, int grid, double* pool, slse_dtype t, bool vec,
                               int chmax, hipStream_t s);
void launch_batched_update(const BatchStep* steps, const BatchProblem* probs, int B, int dmax,
                           const double* pool, int* flags, hipStream_t s);
// beta_init = beta_out = beta0 (or 0) for every problem
void launch_batched_init(const BatchProblem* probs, int B, int dmax, hipStream_t s);

// --------------------------------------------------------------------------
// Test hooks.
// --------------------------------------------------------------------------
// Reference streams (no method arithmetic): mode 0 reads `bytes` of src (one
// word per block into dst[0..blocks)), mode 1 copies src to dst.
void launch_stream_reference(int mode, const void* src, void* dst, int64_t bytes, int blocks,
                             hipStream_t s);
void launch_debug_stream(int what, uint64_t seed, int stream_id, int64_t aux, int64_t start,
                         int64_t count, int64_t* out, hipStream_t s);

}  // namespace slse
