// Host side of libslse: context and scratch memory, the solve driver of
// Alg. 2 (sketch once, factor H_hat, stage-1 steps on nested sketched
// prefixes, stage-2 full-data steps), its hipGraph capture, the adjoint
// driver and the C-ABI entry points.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"

namespace slse {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// Scratch arena: named grow-only device buffers.  Growing a buffer frees the
// old one, so every captured graph is dropped when that happens.
//
// Two other modes serve the calls that must not allocate:
//  - measuring: get() hands out offsets from a fake base (never dereferenced,
//    no kernel is launched) and only adds up the bytes a call would need;
//  - external: get() carves 256-byte aligned regions from a caller workspace
//    in request order (EINVAL when it runs out).  Buffers that must start at
//    zero are listed in `ext_zero` for the caller to clear on its stream.
// In both modes a name asked for twice in one call gets the same region.
// ---------------------------------------------------------------------------
struct Arena {
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  bool grew = false;

  bool measuring = false;
  char* ext = nullptr;
  size_t ext_bytes = 0;
  size_t ext_used = 0;
  std::map<std::string, Buf> ext_bufs;
  std::vector<Buf> ext_zero;

  static constexpr uintptr_t kMeasureBase = uintptr_t(1) << 40;

  bool borrowed() const { return measuring || ext != nullptr; }

  void begin_measure() {
    end_borrow();
    measuring = true;
  }
  void begin_external(void* base, size_t bytes) {
    end_borrow();
    ext = static_cast<char*>(base);
    ext_bytes = bytes;
  }
  void end_borrow() {
    measuring = false;
    ext = nullptr;
    ext_bytes = ext_used = 0;
    ext_bufs.clear();
    ext_zero.clear();
  }

  void* get(const std::string& name, size_t bytes, bool zero_init = false) {
    bytes = std::max<size_t>(bytes, 256);
    if (borrowed()) {
      auto it = ext_bufs.find(name);
      if (it != ext_bufs.end() && it->second.bytes >= bytes) return it->second.p;
      const size_t off = (size_t)round_up((int64_t)ext_used, 256);
      const size_t len = (size_t)round_up((int64_t)bytes, 256);
      ext_used = off + len;
      void* p = nullptr;
      if (measuring) {
        p = reinterpret_cast<void*>(kMeasureBase + off);
      } else {
        if (ext_used > ext_bytes)
          fail(SLSE_EINVAL, "workspace too small: need at least " + std::to_string(ext_used) +
                                " bytes, got " + std::to_string(ext_bytes));
        p = ext + off;
        if (zero_init) ext_zero.push_back(Buf{p, bytes});
      }
      ext_bufs[name] = Buf{p, bytes};
      return p;
    }
    Buf& b = bufs[name];
    if (b.bytes >= bytes) return b.p;
    if (b.p) SLSE_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    void* p = nullptr;
    SLSE_HIP(hipMalloc(&p, bytes));
    if (zero_init) {
      SLSE_HIP(hipMemset(p, 0, bytes));
      SLSE_HIP(hipDeviceSynchronize());
    }
    b.p = p;
    b.bytes = bytes;
    grew = true;
    return p;
  }
  template <typename T>
  T* get_t(const std::string& name, size_t count, bool zero_init = false) {
    return static_cast<T*>(get(name, count * sizeof(T), zero_init));
  }
  void release() {
    for (auto& kv : bufs)
      if (kv.second.p) (void)hipFree(kv.second.p);
    bufs.clear();
  }
};

// Ends a borrowed (measuring or external) arena mode when it goes out of scope.
struct BorrowScope {
  Arena& a;
  ~BorrowScope() { a.end_borrow(); }
};

}  // namespace slse

struct slse_ctx {
  int device = 0;
  int num_cus = 256;
  hipStream_t capture_stream = nullptr;
  slse::Arena arena;
  // preconditioner of the last solve (reused by slse_backward)
  struct {
    bool valid = false;
    uint64_t seed = 0;
    int kind = -1;
    int64_t N = 0, d = 0, r = 0;
    const void* X = nullptr;
    int precision = 0;
  } pre;
  std::map<std::string, hipGraphExec_t> graphs;
  // recorded after each batched graph launch: the next batched call waits for
  // it before it rewrites the shared descriptor tables
  hipEvent_t batch_done = nullptr;
  bool batch_busy = false;
  // autotuned (grid blocks, lanes per row) of the residual-gradient pass, keyed
  // by storage / accumulation / d / vector width / log2(rows), and (grid,
  // tiles per block) of batched steps, keyed by the batch shape
  std::map<std::string, std::pair<int, int>> rg_tune;
  std::string arch;  // gcnArchName of the device and its compute-unit count
  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
};

namespace slse {
namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    SLSE_HIP(hipGetDevice(&prev));
    if (prev != dev) SLSE_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// Validation and layout of the sketch.
// ---------------------------------------------------------------------------
struct SketchShape {
  slse_sketch_kind kind;
  int64_t N, d, r;
  int K;
  std::vector<int64_t> m;
  int p = 0;
  int64_t n_pad = 0;
  int64_t rows_A = 0;
  std::vector<int64_t> offset;
  std::vector<double> scale;
  double hat_scale = 1.0;
};

SketchShape make_sketch_shape(slse_sketch_kind kind, int64_t N, int64_t d, const int64_t* m, int K,
                              int64_t r) {
  require(N > 0 && d >= 1 && N > d, "need N > d >= 1");
  require(d <= 1024, "d > 1024 is not supported by this library");
  require(K >= 1 && K <= SLSE_MAX_LEVELS && m != nullptr, "need 1 <= K <= SLSE_MAX_LEVELS");
  require(r > d, "need r > d");
  SketchShape s;
  s.kind = kind;
  s.N = N;
  s.d = d;
  s.r = r;
  s.K = K;
  s.m.assign(m, m + K);
  require(s.m[0] >= 1, "sketch sizes must be positive");
  for (int i = 1; i < K; ++i) require(s.m[i] > s.m[i - 1], "sketch sizes must increase");
  s.offset.resize(K);
  s.scale.resize(K);
  if (kind == SLSE_SRHT) {
    s.p = std::max(1, ilog2_ceil(N));
    require(s.p <= 30, "N too large for this library (N' <= 2^30)");
    s.n_pad = int64_t(1) << s.p;
    require(s.m[K - 1] <= s.n_pad && r <= s.n_pad, "SRHT: m_K and r must be <= N'");
    for (int i = 0; i < K; ++i) {
      s.offset[i] = 0;
      s.scale[i] = 1.0 / (double)s.m[i];
    }
    s.rows_A = s.m[K - 1];
    s.hat_scale = 1.0 / (double)r;
  } else if (kind == SLSE_COUNTSKETCH) {
    s.n_pad = N;
    int64_t off = 0;
    for (int i = 0; i < K; ++i) {
      require(is_pow2(s.m[i]), "CountSketch: every m_i must be a power of 2");
      s.offset[i] = off;
      s.scale[i] = 1.0;
      off += s.m[i];
    }
    s.rows_A = off;
    s.hat_scale = 1.0;
  } else if (kind == SLSE_GAUSSIAN) {
    s.n_pad = N;
    for (int i = 0; i < K; ++i) {
      s.offset[i] = 0;
      s.scale[i] = 1.0 / (double)s.m[i];
    }
    s.rows_A = s.m[K - 1];
    s.hat_scale = 1.0 / (double)r;
  } else {
    fail(SLSE_EINVAL, "unknown sketch kind");
  }
  return s;
}

void fill_layout(const SketchShape& s, slse_sketch_layout* L) {
  if (!L) return;
  std::memset(L, 0, sizeof(*L));
  L->K = s.K;
  for (int i = 0; i < s.K; ++i) {
    L->m[i] = s.m[i];
    L->offset[i] = s.offset[i];
    L->scale[i] = s.scale[i];
  }
  L->rows_A = s.rows_A;
  L->r = s.r;
  L->hat_scale = s.hat_scale;
  L->n_pad = s.n_pad;
}

// Reserve every scratch buffer the sketch needs (no kernel launched).
void reserve_sketch(slse_ctx* ctx, const SketchShape& s, slse_dtype t, SrhtArgs* srht,
                    GaussianArgs* ga, GaussianArgs* gh, bool gauss_bf16 = false,
                    void** cs_scratch = nullptr) {
  if (s.kind == SLSE_SRHT) {
    srht->t = t;
    srht->N = s.N;
    srht->d = (int)s.d;
    srht->p = s.p;
    srht->mK = s.m[s.K - 1];
    srht->r = s.r;
    srht_plan(*srht, 0);
    srht_split_y(*srht);
    srht->pi_sgn = ctx->arena.get_t<int32_t>("srht_pi", s.n_pad);
    srht->slotA = ctx->arena.get_t<int32_t>("srht_slotA", s.n_pad);
    srht->slotH = ctx->arena.get_t<int32_t>("srht_slotH", s.n_pad);
    const size_t zb = srht_z_bytes(*srht);
    srht->Z = zb ? ctx->arena.get("srht_Z", zb) : nullptr;
  } else if (s.kind == SLSE_COUNTSKETCH) {
    CountSketchArgs c;
    c.t = t;
    c.N = s.N;
    c.d = (int)s.d;
    c.m = s.m.data();
    c.K = s.K;
    c.r = s.r;
    void* p = ctx->arena.get("cs_lists", countsketch_scratch_bytes(c));
    if (cs_scratch) *cs_scratch = p;
  } else if (s.kind == SLSE_GAUSSIAN) {
    for (GaussianArgs* g : {ga, gh}) {
      g->t = t;
      g->N = s.N;
      g->d = (int)s.d;
      g->bf16 = gauss_bf16;
    }
    ga->m = s.m[s.K - 1];
    ga->stream_id = 7;
    gh->m = s.r;
    gh->stream_id = 8;
    gaussian_plan(*ga);
    gaussian_plan(*gh);
    const size_t b = std::max(gaussian_scratch_bytes(*ga), gaussian_scratch_bytes(*gh));
    void* p = ctx->arena.get("gauss_part", b);
    ga->partial = gh->partial = static_cast<float*>(p);
    ga->partial64 = gh->partial64 = static_cast<double*>(p);
  }
}

void enqueue_sketch(const SketchShape& s, uint64_t seed, const void* X, int64_t ldx, const void* Y,
                    slse_dtype t, void* A, int64_t lda, void* Ahat, int64_t ldah, SrhtArgs srht,
                    GaussianArgs ga, GaussianArgs gh, hipStream_t st, void* cs_scratch = nullptr) {
  if (s.kind == SLSE_SRHT) {
    srht.X = X;
    srht.ldx = ldx;
    srht.Y = Y;
    srht.seed = seed;
    srht.A = A;
    srht.lda = lda;
    srht.Ahat = Ahat;
    srht.ldah = ldah;
    launch_srht(srht, st);
  } else if (s.kind == SLSE_COUNTSKETCH) {
    CountSketchArgs c;
    c.t = t;
    c.N = s.N;
    c.d = (int)s.d;
    c.X = X;
    c.ldx = ldx;
    c.Y = Y;
    c.seed = seed;
    c.m = s.m.data();
    c.K = s.K;
    c.r = s.r;
    c.A = A;
    c.lda = lda;
    c.Ahat = Ahat;
    c.ldah = ldah;
    c.scratch = cs_scratch;
    launch_countsketch(c, st);
  } else {
    for (GaussianArgs* g : {&ga, &gh}) {
      g->X = X;
      g->ldx = ldx;
      g->Y = Y;
      g->seed = seed;
    }
    ga.A = A;
    ga.lda = lda;
    gh.A = Ahat;
    gh.lda = ldah;
    launch_gaussian(ga, st);
    // the BF16 tiles of [X|Y] staged for S serve S_hat too (same scratch, same stream)
    gh.tiles_ready = ga.bf16 && gh.bf16 && ga.partial == gh.partial;
    launch_gaussian(gh, st);
  }
}

// ---------------------------------------------------------------------------
// Factorization: R^T R = scale A^T A, then L = R^{-T} and M = L^T L = H_hat^{-1}.
// ---------------------------------------------------------------------------
struct FactorBufs {
  double* Ad = nullptr;  // rows x d
  double* G = nullptr;   // d x d
  double* R = nullptr;   // d x d (ldr)
  double* L = nullptr;   // d x d: R^{-1}
  double* M = nullptr;   // d x d
  double* Q = nullptr;   // rows x d (QR route)
  double* R2 = nullptr;  // d x d (QR route)
  int* info = nullptr;   // 2 ints
  double* part = nullptr;  // split-K scratch of the GEMMs
  size_t part_n = 0;
  double* colp = nullptr;  // d x 32 panel scratch of the Gauss-Jordan inverse
};

FactorBufs reserve_factor(slse_ctx* ctx, int64_t rows, int64_t d, slse_factor_method method) {
  FactorBufs f;
  f.Ad = ctx->arena.get_t<double>("f_Ad", rows * d);
  f.G = ctx->arena.get_t<double>("f_G", d * d);
  f.R = ctx->arena.get_t<double>("f_R", d * d);
  f.L = ctx->arena.get_t<double>("f_L", d * d);
  f.M = ctx->arena.get_t<double>("f_M", d * d);
  if (method == SLSE_FACTOR_QR) {
    f.Q = ctx->arena.get_t<double>("f_Q", rows * d);
    f.R2 = ctx->arena.get_t<double>("f_R2", d * d);
  }
  f.info = ctx->arena.get_t<int>("f_info", 4, true);
  f.part_n = std::max(gemm_scratch_doubles(d, d, rows), gemm_scratch_doubles(d, d, d));
  if (method == SLSE_FACTOR_QR) f.part_n = std::max(f.part_n, gemm_scratch_doubles(rows, d, d));
  f.part = ctx->arena.get_t<double>("f_part", f.part_n + 1);
  f.colp = ctx->arena.get_t<double>("f_colp", d * 32);
  return f;
}

// M (ldm = d) into f.M, and R (ldr = d) into f.R when need_R or on the QR
// route.  Without R the Cholesky route inverts the Gram matrix directly
// (M = G^{-1}, blocked Gauss-Jordan): the iteration needs only M.
void enqueue_factor(const FactorBufs& f, int64_t rows, int d, const void* A, int64_t lda,
                    slse_dtype at, double scale, slse_factor_method method, hipStream_t st,
                    bool need_R = false) {
  launch_convert_scale(rows, d, A, lda, at, std::sqrt(scale), f.Ad, d, st);
  if (method == SLSE_FACTOR_CHOL && !need_R) {
    launch_gemm_f64(d, d, rows, 1.0, f.Ad, d, true, f.Ad, d, false, 0.0, f.M, d, st, f.part,
                    f.part_n);
    launch_fill_i32(f.info, 0, 3, st);
    launch_spd_inverse(d, f.M, f.colp, f.info, st);
    return;
  }
  launch_gemm_f64(d, d, rows, 1.0, f.Ad, d, true, f.Ad, d, false, 0.0, f.G, d, st, f.part, f.part_n);
  if (method == SLSE_FACTOR_QR) {
    // shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa,
    // SIAM J. Sci. Comput. 2020): a Cholesky of G + s I with
    // s = 11 (rows d + d (d + 1)) u ||A||_F^2 always exists; Q0 = A R0^{-1} then
    // has a modest condition number, and two CholeskyQR passes finish the job.
    // R = R2 R1 R0 matches Householder's R to O(kappa u) for kappa up to ~u^{-1}.
    const double u = std::ldexp(1.0, -53);
    launch_shift_diag(d, f.G, 11.0 * ((double)rows * d + (double)d * (d + 1)) * u, st);
    launch_cholesky(d, f.G, d, f.R, d, f.info, st);                        // R0
    launch_tri_inv(d, f.R, d, f.L, d, st);
    launch_gemm_f64(rows, d, d, 1.0, f.Ad, d, false, f.L, d, false, 0.0, f.Q, d, st, f.part, f.part_n);
    launch_gemm_f64(d, d, rows, 1.0, f.Q, d, true, f.Q, d, false, 0.0, f.G, d, st, f.part, f.part_n);
    launch_cholesky(d, f.G, d, f.R2, d, f.info + 1, st);                   // R1
    launch_tri_inv(d, f.R2, d, f.L, d, st);
    launch_gemm_f64(rows, d, d, 1.0, f.Q, d, false, f.L, d, false, 0.0, f.Ad, d, st, f.part, f.part_n);
    launch_gemm_f64(d, d, rows, 1.0, f.Ad, d, true, f.Ad, d, false, 0.0, f.G, d, st, f.part, f.part_n);
    launch_cholesky(d, f.G, d, f.L, d, f.info + 2, st);                    // R2
    launch_gemm_f64(d, d, d, 1.0, f.R2, d, false, f.R, d, false, 0.0, f.G, d, st, f.part, f.part_n);
    launch_gemm_f64(d, d, d, 1.0, f.L, d, false, f.G, d, false, 0.0, f.R, d, st, f.part, f.part_n);
  } else {
    launch_cholesky(d, f.G, d, f.R, d, f.info, st);
  }
  // M = R^{-1} R^{-T}
  launch_tri_inv(d, f.R, d, f.L, d, st);
  launch_gemm_f64(d, d, d, 1.0, f.L, d, false, f.L, d, true, 0.0, f.M, d, st, f.part, f.part_n);
}

// ---------------------------------------------------------------------------
// The M-IHS iteration engine shared by the forward solve and the adjoint.
// ---------------------------------------------------------------------------
struct IterBufs {
  double* beta[3];
  double* partial = nullptr;
  double* gpart = nullptr;
  int* counters = nullptr;
  double* sur_partial = nullptr;
  int* sur_counter = nullptr;
  int* flags = nullptr;  // [0] done, [1] non-finite
  double* err_delta = nullptr;  // beta_t - beta_ref (per-iterate error accounting)
  double* err_g = nullptr;      // discarded gradient of the prediction-error pass
  int max_blocks = 1024;   // capacity of the partial rows
  int grid_blocks = 512;   // grid of the residual-gradient launches (<= max_blocks)
};

IterBufs reserve_iter(slse_ctx* ctx, int64_t d, const char* tag) {
  IterBufs b;
  std::string t(tag);
  for (int i = 0; i < 3; ++i) b.beta[i] = ctx->arena.get_t<double>(t + "_beta" + char('0' + i), d);
  b.max_blocks = std::max(256, 8 * ctx->num_cus);
  b.grid_blocks = std::max(64, 2 * ctx->num_cus);
  const int64_t ldp = round_up(d + 1, 8);
  b.partial = ctx->arena.get_t<double>(t + "_partial", b.max_blocks * ldp);
  const int groups = (int)ceil_div(b.max_blocks, 32);
  b.gpart = ctx->arena.get_t<double>(t + "_gpart", groups * ldp);
  b.counters = ctx->arena.get_t<int>(t + "_counters", groups, true);
  b.sur_partial = ctx->arena.get_t<double>(t + "_surp", 3 * update_blocks((int)d) + 8);
  b.sur_counter = ctx->arena.get_t<int>(t + "_surc", 4, true);
  b.flags = ctx->arena.get_t<int>(t + "_flags", 4);
  b.err_delta = ctx->arena.get_t<double>(t + "_errd", d);
  b.err_g = ctx->arena.get_t<double>(t + "_errg", d);
  return b;
}

std::string rg_key(int64_t n, int d, slse_dtype storage, slse_dtype accum, const void* X,
                   int64_t ldx) {
  const int es = (int)dtype_size(storage);
  const bool vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((ldx * es) % 16 == 0);
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= n) ++lg;
  return std::to_string((int)storage) + "/" + std::to_string((int)accum) + "/" +
         std::to_string(d) + "/" + (vec ? "v" : "s") + "/" + std::to_string(lg);
}

ResidGradPlan rg_plan(const slse_ctx* ctx, const IterBufs& b, int64_t n, int d,
                      slse_dtype storage, slse_dtype accum, const void* X, int64_t ldx) {
  if (ctx) {
    auto it = ctx->rg_tune.find(rg_key(n, d, storage, accum, X, ldx));
    if (it != ctx->rg_tune.end())
      return plan_resid_grad(n, d, storage, X, ldx, it->second.first, b.max_blocks,
                             it->second.second);
  }
  return plan_resid_grad(n, d, storage, X, ldx, b.grid_blocks, b.max_blocks);
}

// Time a few (grid, lane-group) shapes of the residual-gradient pass on the
// actual data and keep the fastest for this shape (never inside a capture).
void tune_resid_grad(slse_ctx* ctx, const IterBufs& b, int64_t n, int d, slse_dtype storage,
                     slse_dtype accum, const void* X, int64_t ldx, const void* Y, int64_t incy,
                     hipStream_t st) {
  if (n < (int64_t(1) << 12)) return;
  if (const char* e = std::getenv("SLSE_AUTOTUNE"))
    if (std::atoi(e) == 0) return;
  const std::string key = rg_key(n, d, storage, accum, X, ldx);
  if (ctx->rg_tune.count(key)) return;
  const ResidGradPlan base = plan_resid_grad(n, d, storage, X, ldx, b.grid_blocks, b.max_blocks);
  std::vector<int> lprs;
  for (int l : {base.lpr / 2, base.lpr, base.lpr * 2, base.lpr * 4})
    if (l >= 1 && l <= 64) lprs.push_back(l);
  std::vector<int> grids;
  for (int g : {ctx->num_cus, 2 * ctx->num_cus, 4 * ctx->num_cus})
    if (g <= b.max_blocks) grids.push_back(g);
  hipEvent_t e0, e1;
  SLSE_HIP(hipEventCreate(&e0));
  SLSE_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  std::pair<int, int> pick{base.blocks, base.lpr};
  for (int g : grids)
    for (int l : lprs) {
      ResidGradPlan pl;
      try {
        pl = plan_resid_grad(n, d, storage, X, ldx, g, b.max_blocks, l);
      } catch (const Error&) {
        continue;
      }
      ResidGradArgs a;
      a.n = n;
      a.d = d;
      a.X = X;
      a.ldx = ldx;
      a.Y = Y;
      a.incy = incy;
      a.storage = storage;
      a.accum = accum;
      a.beta = b.beta[0];
      a.partial = b.partial;
      a.gpart = b.gpart;
      a.counters = b.counters;
      a.capacity_blocks = b.max_blocks;
      launch_resid_grad(pl, a, st);
      SLSE_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r) launch_resid_grad(pl, a, st);
      SLSE_HIP(hipEventRecord(e1, st));
      SLSE_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SLSE_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        pick = {g, pl.lpr};
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->rg_tune[key] = pick;
}

// Per-iterate errors against a reference vector (slse_params.beta_ref):
// rel[t] = ||beta_t - ref|| / ||ref|| and pred[t] = ||X (beta_t - ref)||^2 over
// the full data (one fused pass with Y = 0 on beta_t - ref).
struct ErrorSink {
  const double* ref = nullptr;
  double* rel = nullptr;
  double* pred = nullptr;
  int64_t N = 0;
  const void* X = nullptr;
  int64_t ldx = 0;
  slse_dtype storage = SLSE_F64;
  bool on() const { return ref && (rel || pred); }
};

struct Stepper {
  IterBufs b;
  int d;
  const double* M;
  int cur = 0, prev = 0;
  int t = 0;  // iterate index
  hipStream_t st;
  const slse_ctx* ctx = nullptr;
  ErrorSink err;

  // errors of the current iterate beta_t (t = this->t)
  void record_errors() {
    if (!err.on()) return;
    launch_iter_error(b.beta[cur], err.ref, d, err.rel ? err.rel + t : nullptr,
                      err.pred ? b.err_delta : nullptr, st);
    if (!err.pred) return;
    const ResidGradPlan pl = rg_plan(ctx, b, err.N, d, err.storage, SLSE_F64, err.X, err.ldx);
    ResidGradArgs a;
    a.n = err.N;
    a.d = d;
    a.X = err.X;
    a.ldx = err.ldx;
    a.Y = nullptr;
    a.incy = 1;
    a.storage = err.storage;
    a.accum = SLSE_F64;
    a.beta = b.err_delta;
    a.partial = b.partial;
    a.gpart = b.gpart;
    a.counters = b.counters;
    a.capacity_blocks = b.max_blocks;
    launch_resid_grad(pl, a, st);
    launch_finalize_grad(b.gpart, pl.groups, pl.ldp, d, 1.0, b.err_g, err.pred + t, st);
  }

  // beta_{t0} = beta0 (zeros if NULL), beta_{t0-1} = beta_prev (beta0 if NULL)
  void start(const double* beta0, double* traj, const double* beta_prev = nullptr, int t0 = 0) {
    if (beta0)
      launch_copy_f64(beta0, b.beta[0], d, st);
    else
      launch_fill_f64(b.beta[0], 0.0, d, st);
    cur = prev = 0;
    if (beta_prev) {
      launch_copy_f64(beta_prev, b.beta[1], d, st);
      prev = 1;
    }
    t = t0;
    if (traj) launch_copy_f64(b.beta[0], traj + (int64_t)t0 * d, d, st);
    launch_fill_i32(b.flags, 0, 4, st);
    record_errors();
  }
  // (beta_{t-1}, beta_t) of the current iterate
  void save_state(double* out) const {
    launch_copy_f64(b.beta[prev], out, d, st);
    launch_copy_f64(b.beta[cur], out + d, d, st);
  }
  void reset_momentum() { prev = cur; }

  // one M-IHS step on rows [0, n) of (X, Y)
  void step(int64_t n, const void* X, int64_t ldx, const void* Y, int64_t incy, slse_dtype storage,
            slse_dtype accum, double scale, const double* w, double mu, double eta, double* beta_out,
            double* traj, double* sur, double tol, int64_t incw = 1) {
    const ResidGradPlan pl = rg_plan(ctx, b, n, d, storage, accum, X, ldx);
    ResidGradArgs a;
    a.n = n;
    a.d = d;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.incy = incy;
    a.storage = storage;
    a.accum = accum;
    a.beta = b.beta[cur];
    a.partial = b.partial;
    a.gpart = b.gpart;
    a.counters = b.counters;
    a.capacity_blocks = b.max_blocks;
    a.done = b.flags;
    launch_resid_grad(pl, a, st);
    const int next = (cur + 1) % 3 == prev ? (cur + 2) % 3 : (cur + 1) % 3;
    UpdateArgs u;
    u.gpart = b.gpart;
    u.groups = pl.groups;
    u.ldp = pl.ldp;
    u.d = d;
    u.scale = scale;
    u.w = w;
    u.incw = incw;
    u.M = M;
    u.ldm = d;
    u.beta = b.beta[cur];
    u.beta_prev = b.beta[prev];
    u.beta_next = b.beta[next];
    u.mu = mu;
    u.eta = eta;
    u.beta_out = beta_out;
    u.traj_row = traj ? traj + (int64_t)(t + 1) * d : nullptr;
    u.sur_partial = b.sur_partial;
    u.sur_counter = b.sur_counter;
    u.sur_out = sur ? sur + t : nullptr;
    u.tol2 = tol > 0 ? tol * tol : 0.0;
    u.done = b.flags;
    u.status = b.flags + 1;
    launch_update(u, st);
    prev = cur;
    cur = next;
    ++t;
    record_errors();
  }
};

// ---------------------------------------------------------------------------
// Solve.
// ---------------------------------------------------------------------------
struct SolvePlan {
  SketchShape sk;
  slse_dtype st_t;    // storage of the data and of the sketch
  slse_dtype acc1;    // stage-1 accumulation
  void* A = nullptr;
  int64_t lda = 0;
  void* Ahat = nullptr;
  int64_t ldah = 0;
  SrhtArgs srht;
  GaussianArgs ga, gh;
  void* cs = nullptr;  // CountSketch bucket lists
  FactorBufs f;
  IterBufs it;
  double* sur = nullptr;  // per-step error estimates (the caller's or ours)
};

void check_params(const slse_problem* p, const slse_params* q) {
  require(p && q, "null problem or params");
  require(p->X && p->Y, "null X or Y");
  require(p->ldx >= p->d, "ldx < d");
  require(p->dtype == SLSE_F32 || p->dtype == SLSE_F64, "data dtype must be F32 or F64");
  if (q->precision == SLSE_PREC_F64)
    require(p->dtype == SLSE_F64, "precision F64 needs F64 data");
  else if (q->precision == SLSE_PREC_MIXED)
    require(p->dtype == SLSE_F32, "precision MIXED needs F32 data");
  else
    fail(SLSE_EINVAL, "unknown precision");
  require(q->s_max >= 0, "s_max < 0");
  require(q->K >= 0 && q->K <= SLSE_MAX_LEVELS, "need 0 <= K <= SLSE_MAX_LEVELS");
  for (int i = 0; i < q->K; ++i) require(q->a[i] >= 0, "a_i < 0");
  require(std::isfinite(q->mu) && std::isfinite(q->eta), "mu, eta must be finite");
  require(q->factor == SLSE_FACTOR_CHOL || q->factor == SLSE_FACTOR_QR, "unknown factor method");
  require(!(q->rel_err || q->pred_err) || q->beta_ref, "rel_err / pred_err need beta_ref");
  int T = q->s_max;
  for (int i = 0; i < q->K; ++i) T += q->a[i];
  require(q->stop_step >= 0 && q->stop_step <= T, "need 0 <= stop_step <= T");
  require(q->start_step >= 0 && q->start_step <= (q->stop_step ? q->stop_step : T),
          "need 0 <= start_step <= stop_step (or T)");
}

int total_steps(const slse_params* q) {
  int T = q->s_max;
  for (int i = 0; i < q->K; ++i) T += q->a[i];
  return T;
}

// the steps [t0, t1) that a call runs (checkpoint and resume)
void step_range(const slse_params* q, int& t0, int& t1) {
  t0 = q->start_step;
  t1 = q->stop_step ? q->stop_step : total_steps(q);
}

// Row stride of the internal sketch buffers: rows of at least one 128-byte
// line start on a line boundary, so the SRHT's scattered row segments are
// whole-line writes; shorter rows are packed at 16-byte alignment.
int64_t sketch_ld(int64_t d, size_t es) {
  const int64_t line = 128 / (int64_t)es;
  return (d + 1) >= line ? round_up(d + 1, line) : round_up(d + 1, 16 / (int64_t)es);
}

// Every scratch buffer of one solve, in a fixed order (the order also fixes
// the layout of a caller workspace).
SolvePlan reserve_solve(slse_ctx* ctx, const slse_problem* p, const slse_params* q) {
  SolvePlan pl;
  pl.sk = make_sketch_shape(q->kind, p->N, p->d, q->m, q->K, q->r);
  pl.st_t = p->dtype;
  pl.acc1 = q->precision == SLSE_PREC_MIXED ? SLSE_F32 : SLSE_F64;
  const size_t es = dtype_size(pl.st_t);
  pl.lda = sketch_ld(p->d, es);
  pl.ldah = pl.lda;
  pl.A = ctx->arena.get("A", (size_t)pl.sk.rows_A * pl.lda * es);
  pl.Ahat = ctx->arena.get("Ahat", (size_t)pl.sk.r * pl.ldah * es);
  // a Gaussian sketch of FP32 data in the mixed form runs on the matrix cores (BF16 operands)
  reserve_sketch(ctx, pl.sk, pl.st_t, &pl.srht, &pl.ga, &pl.gh,
                 q->precision == SLSE_PREC_MIXED && q->kind == SLSE_GAUSSIAN, &pl.cs);
  pl.f = reserve_factor(ctx, pl.sk.r, p->d, q->factor);
  pl.it = reserve_iter(ctx, p->d, "it");
  // the per-step error estimates always land somewhere: the caller's buffer or ours
  pl.sur = q->surrogate ? q->surrogate
                        : ctx->arena.get_t<double>("sur_hist", (size_t)total_steps(q) + 1);
  return pl;
}

ErrorSink error_sink(const slse_problem* p, const slse_params* q) {
  ErrorSink e;
  e.ref = q->beta_ref;
  e.rel = q->rel_err;
  e.pred = q->pred_err;
  e.N = p->N;
  e.X = p->X;
  e.ldx = p->ldx;
  e.storage = p->dtype;
  return e;
}

// Phase boundaries of one solve: ev[0] after the sketch, ev[1] after the
// factor, ev[2] after stage 1, ev[3] after stage 2 (all optional).
void enqueue_solve(const slse_ctx* ctx, const SolvePlan& pl, const slse_problem* p,
                   const slse_params* q, double* beta_out, hipStream_t st,
                   hipEvent_t* ev = nullptr) {
  const int d = (int)p->d;
  const SketchShape& sk = pl.sk;
  auto mark = [&](int k) {
    if (ev && ev[k]) SLSE_HIP(hipEventRecord(ev[k], st));
  };
  enqueue_sketch(sk, q->seed, p->X, p->ldx, p->Y, pl.st_t, pl.A, pl.lda, pl.Ahat, pl.ldah, pl.srht,
                 pl.ga, pl.gh, st, pl.cs);
  mark(0);
  enqueue_factor(pl.f, sk.r, d, pl.Ahat, pl.ldah, pl.st_t, sk.hat_scale, q->factor, st);
  mark(1);
  // steps t0 .. t1-1 of the global step sequence (all of them unless resuming)
  int t0, t1;
  step_range(q, t0, t1);
  Stepper S{pl.it, d, pl.f.M, 0, 0, 0, st, ctx, error_sink(p, q)};
  S.start(q->beta0, q->trajectory, q->beta_prev, t0);
  launch_copy_f64(S.b.beta[0], beta_out, d, st);
  const size_t es = dtype_size(pl.st_t);
  int g = 0;  // global index of the next step
  // stage 1: a_i steps on the prefix of m_i sketched rows (eq. (98))
  for (int i = 0; i < sk.K; ++i) {
    const char* base = static_cast<const char*>(pl.A) + (size_t)sk.offset[i] * pl.lda * es;
    for (int j = 0; j < q->a[i]; ++j, ++g) {
      if (g < t0 || g >= t1) continue;
      if (j == 0 && q->momentum_reset) S.reset_momentum();
      S.step(sk.m[i], base, pl.lda, base + (size_t)d * es, pl.lda, pl.st_t, pl.acc1, sk.scale[i],
             nullptr, q->mu, q->eta, beta_out, q->trajectory, pl.sur, 0.0);
    }
  }
  mark(2);
  // stage 2: full-data steps (eq. (99))
  for (int j = 0; j < q->s_max; ++j, ++g) {
    if (g < t0 || g >= t1) continue;
    if (j == 0 && q->momentum_reset) S.reset_momentum();
    slse_dtype acc = SLSE_F64;
    if (q->precision == SLSE_PREC_MIXED && j < q->fp32_sweeps) acc = SLSE_F32;
    S.step(p->N, p->X, p->ldx, p->Y, 1, pl.st_t, acc, 1.0, nullptr, q->mu, q->eta, beta_out,
           q->trajectory, pl.sur, q->tol);
  }
  if (q->state_out) S.save_state(q->state_out);
  mark(3);
}

std::string graph_key(const char* tag, const slse_problem* p, const slse_params* q,
                      const double* beta_out, const void* ws, size_t ws_bytes) {
  std::string k(tag);
  auto add = [&k](const void* v, size_t n) { k.append(static_cast<const char*>(v), n); };
  add(p, sizeof(*p));
  add(q, sizeof(*q));
  add(&beta_out, sizeof(beta_out));
  add(&ws, sizeof(ws));
  add(&ws_bytes, sizeof(ws_bytes));
  return k;
}

// Capture `body` on the context's capture stream once per key and launch the
// instantiated graph on st.
template <typename F>
void launch_cached_graph(slse_ctx* ctx, const std::string& key, hipStream_t st, F&& body) {
  auto itg = ctx->graphs.find(key);
  if (itg == ctx->graphs.end()) {
    hipGraph_t g = nullptr;
    SLSE_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    try {
      body(ctx->capture_stream);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(ctx->capture_stream, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    SLSE_HIP(hipStreamEndCapture(ctx->capture_stream, &g));
    hipGraphExec_t ge = nullptr;
    const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    SLSE_HIP(e);
    itg = ctx->graphs.emplace(key, ge).first;
  }
  SLSE_HIP(hipGraphLaunch(itg->second, st));
}

// Events of a timed call: [0] start, [1..4] phase ends (the last = the end).
struct CallTimer {
  hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int n = 0;
  CallTimer(bool on, bool phases, hipStream_t st) {
    if (!on) return;
    n = phases ? 5 : 2;
    for (int i = 0; i < n; ++i) SLSE_HIP(hipEventCreate(&e[i]));
    SLSE_HIP(hipEventRecord(e[0], st));
  }
  ~CallTimer() {
    for (int i = 0; i < n; ++i)
      if (e[i]) (void)hipEventDestroy(e[i]);
  }
  hipEvent_t* phase_events() { return n == 5 ? e + 1 : nullptr; }
  hipEvent_t end() const { return n == 5 ? e[4] : e[1]; }
  void record_end(hipStream_t st) {
    if (n == 2) SLSE_HIP(hipEventRecord(e[1], st));
  }
  double ms(int a, int b) const {
    float v = 0.f;
    SLSE_HIP(hipEventElapsedTime(&v, e[a], e[b]));
    return v;
  }
};

slse_status finish_report(const SolvePlan& pl, const slse_params* q, slse_report* rep,
                          hipStream_t st, const CallTimer& tm) {
  int flags[4] = {0, 0, 0, 0};
  int info[3] = {0, 0, 0};
  SLSE_HIP(hipMemcpyAsync(flags, pl.it.flags, sizeof(flags), hipMemcpyDeviceToHost, st));
  SLSE_HIP(hipMemcpyAsync(info, pl.f.info, sizeof(info), hipMemcpyDeviceToHost, st));
  SLSE_HIP(hipStreamSynchronize(st));
  slse_status status = SLSE_OK;
  if (info[0] != 0 || info[1] != 0 || info[2] != 0)
    status = SLSE_ESINGULAR;
  else if (flags[1])
    status = SLSE_ENONFINITE;
  else if (q->tol > 0 && !flags[0])
    status = SLSE_ENOTCONV;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->status = status;
    int s1 = 0;
    for (int i = 0; i < q->K; ++i) s1 += q->a[i];
    const int T = s1 + q->s_max;
    int t0, t1;
    step_range(q, t0, t1);
    const int u2 = std::max(t0, s1);  // first stage-2 step run
    rep->stage1_steps = std::max(0, std::min(t1, s1) - t0);
    rep->stage2_steps = std::max(0, t1 - u2);
    if (t1 > t0 && pl.sur) {
      std::vector<double> sur(T, 0.0);
      SLSE_HIP(hipMemcpy(sur.data(), pl.sur, sizeof(double) * T, hipMemcpyDeviceToHost));
      int taken = 0;
      for (int t = u2; t < t1; ++t) {
        ++taken;
        if (q->tol > 0 && sur[t] <= q->tol) break;
      }
      if (q->tol > 0) rep->stage2_steps = taken;
      rep->surrogate0 = u2 < t1 ? sur[u2] : sur[t0];
      const int last = rep->stage2_steps > 0 ? u2 + rep->stage2_steps - 1 : t1 - 1;
      rep->surrogate_final = sur[last];
    }
    if (tm.n == 5) {
      rep->ms_sketch = tm.ms(0, 1);
      rep->ms_factor = tm.ms(1, 2);
      rep->ms_stage1 = tm.ms(2, 3);
      rep->ms_stage2 = tm.ms(3, 4);
      rep->ms_total = tm.ms(0, 4);
    } else if (tm.n == 2) {
      rep->ms_total = tm.ms(0, 1);
    }
  }
  return status;
}

// Clear the regions of a caller workspace that must start at zero.
void clear_borrowed(slse_ctx* ctx, hipStream_t st) {
  for (const Arena::Buf& z : ctx->arena.ext_zero)
    launch_fill_i32(static_cast<int*>(z.p), 0, (int64_t)(z.bytes / sizeof(int)), st);
}

void remember_preconditioner(slse_ctx* ctx, const slse_problem* p, const slse_params* q, bool ok) {
  ctx->pre.valid = ok;
  ctx->pre.seed = q->seed;
  ctx->pre.kind = q->kind;
  ctx->pre.N = p->N;
  ctx->pre.d = p->d;
  ctx->pre.r = q->r;
  ctx->pre.X = p->X;
  ctx->pre.precision = q->precision;
}

slse_status solve_impl(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                       double* beta_out, slse_report* rep, hipStream_t st, void* ws = nullptr,
                       size_t ws_bytes = 0) {
  check_params(p, q);
  require(beta_out != nullptr, "null beta_out");
  BorrowScope scope{ctx->arena};
  if (ws) ctx->arena.begin_external(ws, ws_bytes);
  ctx->arena.grew = false;
  SolvePlan pl = reserve_solve(ctx, p, q);
  if (ctx->arena.grew) ctx->drop_graphs();
  if (ws) clear_borrowed(ctx, st);
  {
    // shapes of the stage-2 sweeps and of the large stage-1 prefixes
    const slse_dtype acc2 = q->precision == SLSE_PREC_MIXED && q->fp32_sweeps > 0 ? SLSE_F32
                                                                                  : SLSE_F64;
    tune_resid_grad(ctx, pl.it, p->N, (int)p->d, pl.st_t, SLSE_F64, p->X, p->ldx, p->Y, 1, st);
    if (acc2 == SLSE_F32)
      tune_resid_grad(ctx, pl.it, p->N, (int)p->d, pl.st_t, SLSE_F32, p->X, p->ldx, p->Y, 1, st);
    const size_t es = dtype_size(pl.st_t);
    for (int i = 0; i < pl.sk.K; ++i) {
      const char* base = static_cast<const char*>(pl.A) + (size_t)pl.sk.offset[i] * pl.lda * es;
      tune_resid_grad(ctx, pl.it, pl.sk.m[i], (int)p->d, pl.st_t, pl.acc1, base, pl.lda,
                      base + (size_t)p->d * es, pl.lda, st);
    }
  }
  CallTimer tm(rep != nullptr, rep != nullptr && !q->use_graph, st);
  if (q->use_graph) {
    launch_cached_graph(ctx, graph_key("solve", p, q, beta_out, ws, ws_bytes), st,
                        [&](hipStream_t cs) { enqueue_solve(ctx, pl, p, q, beta_out, cs); });
  } else {
    enqueue_solve(ctx, pl, p, q, beta_out, st, tm.phase_events());
  }
  // a solve through a caller workspace leaves no preconditioner behind
  remember_preconditioner(ctx, p, q, ws == nullptr);
  tm.record_end(st);
  slse_status status = SLSE_OK;
  if (rep || q->tol > 0) status = finish_report(pl, q, rep, st, tm);
  return status;
}

size_t solve_workspace_bytes(slse_ctx* ctx, const slse_problem* p, const slse_params* q) {
  check_params(p, q);
  BorrowScope scope{ctx->arena};
  ctx->arena.begin_measure();
  (void)reserve_solve(ctx, p, q);
  return ctx->arena.ext_used;
}

// ---------------------------------------------------------------------------
// IHS with a Hessian sketch drawn anew at every step (the baseline of Sec. 1).
// ---------------------------------------------------------------------------
void enqueue_ihs(const slse_ctx* ctx, const SolvePlan& pl, const slse_problem* p,
                 const slse_params* q, double* beta_out, hipStream_t st) {
  const int d = (int)p->d;
  const SketchShape& sk = pl.sk;
  Stepper S{pl.it, d, pl.f.M, 0, 0, 0, st, ctx, ErrorSink{}};
  S.start(q->beta0, q->trajectory);
  launch_copy_f64(S.b.beta[0], beta_out, d, st);
  for (int t = 0; t < q->s_max; ++t) {
    enqueue_sketch(sk, q->seed + (uint64_t)t, p->X, p->ldx, p->Y, pl.st_t, pl.A, pl.lda, pl.Ahat,
                   pl.ldah, pl.srht, pl.ga, pl.gh, st, pl.cs);
    enqueue_factor(pl.f, sk.r, d, pl.Ahat, pl.ldah, pl.st_t, sk.hat_scale, q->factor, st);
    S.step(p->N, p->X, p->ldx, p->Y, 1, pl.st_t, SLSE_F64, 1.0, nullptr, 1.0, 0.0, beta_out,
           q->trajectory, pl.sur, 0.0);
  }
}

slse_status ihs_impl(slse_ctx* ctx, const slse_problem* p, const slse_params* q, double* beta_out,
                     slse_report* rep, hipStream_t st) {
  require(p && q, "null problem or params");
  require(beta_out != nullptr, "null beta_out");
  // the fields IHS reads, with one unused nested level of the power of 2 >= r
  slse_params qq = *q;
  qq.K = 1;
  qq.m[0] = int64_t(1) << ilog2_ceil(std::max<int64_t>(q->r, 1));
  qq.a[0] = 0;
  qq.mu = 1.0;
  qq.eta = 0.0;
  qq.tol = 0.0;
  qq.momentum_reset = 0;
  qq.fp32_sweeps = 0;
  qq.surrogate = nullptr;
  qq.beta_ref = nullptr;
  qq.rel_err = qq.pred_err = nullptr;
  qq.start_step = qq.stop_step = 0;
  qq.beta_prev = nullptr;
  qq.state_out = nullptr;
  check_params(p, &qq);
  ctx->arena.grew = false;
  SolvePlan pl = reserve_solve(ctx, p, &qq);
  if (ctx->arena.grew) ctx->drop_graphs();
  tune_resid_grad(ctx, pl.it, p->N, (int)p->d, pl.st_t, SLSE_F64, p->X, p->ldx, p->Y, 1, st);
  CallTimer tm(rep != nullptr, false, st);
  if (qq.use_graph)
    launch_cached_graph(ctx, graph_key("ihs", p, &qq, beta_out, nullptr, 0), st,
                        [&](hipStream_t cs) { enqueue_ihs(ctx, pl, p, &qq, beta_out, cs); });
  else
    enqueue_ihs(ctx, pl, p, &qq, beta_out, st);
  ctx->pre.valid = false;
  tm.record_end(st);
  if (!rep) return SLSE_OK;
  slse_params qr = qq;  // the report counts the s_max full-data steps
  qr.K = 0;
  return finish_report(pl, &qr, rep, st, tm);
}

// ---------------------------------------------------------------------------
// Backward: lambda from (X^T X) lambda = w by the preconditioned iteration,
// then the rank-2 pass.
// ---------------------------------------------------------------------------
slse_status backward_impl(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                          const double* beta_hat, const double* w, int64_t incw, void* dX,
                          int64_t lddx, void* dY, slse_dtype grad_t, double* lambda_out,
                          slse_report* rep, hipStream_t st) {
  check_params(p, q);
  require(beta_hat && w, "null beta_hat or w");
  require(incw >= 0, "incw < 0");
  require(grad_t == SLSE_F32 || grad_t == SLSE_F64, "grad dtype must be F32 or F64");
  if (dX) require(lddx >= p->d, "lddx < d");
  const int d = (int)p->d;
  ctx->arena.grew = false;
  const bool reuse = ctx->pre.valid && ctx->pre.seed == q->seed && ctx->pre.kind == q->kind &&
                     ctx->pre.N == p->N && ctx->pre.d == p->d && ctx->pre.r == q->r &&
                     ctx->pre.X == p->X && ctx->pre.precision == q->precision;
  SolvePlan pl;
  pl.sk = make_sketch_shape(q->kind, p->N, p->d, q->m, q->K, q->r);
  pl.st_t = p->dtype;
  pl.f = reserve_factor(ctx, q->r, p->d, q->factor);
  if (!reuse) {
    // sketch only what H_hat needs (the smallest level keeps the sketch cheap)
    const size_t es = dtype_size(pl.st_t);
    pl.lda = pl.ldah = sketch_ld(p->d, es);
    pl.A = ctx->arena.get("A", (size_t)pl.sk.rows_A * pl.lda * es);
    pl.Ahat = ctx->arena.get("Ahat", (size_t)pl.sk.r * pl.ldah * es);
    reserve_sketch(ctx, pl.sk, pl.st_t, &pl.srht, &pl.ga, &pl.gh,
                   q->precision == SLSE_PREC_MIXED && q->kind == SLSE_GAUSSIAN, &pl.cs);
  }
  IterBufs ib = reserve_iter(ctx, p->d, "adj");
  double* lam0 = ctx->arena.get_t<double>("adj_lam0", d);
  double* zero = ctx->arena.get_t<double>("adj_zero", (int64_t)d * 1);
  if (ctx->arena.grew) ctx->drop_graphs();
  if (!reuse) {
    enqueue_sketch(pl.sk, q->seed, p->X, p->ldx, p->Y, pl.st_t, pl.A, pl.lda, pl.Ahat, pl.ldah,
                   pl.srht, pl.ga, pl.gh, st, pl.cs);
    enqueue_factor(pl.f, pl.sk.r, d, pl.Ahat, pl.ldah, pl.st_t, pl.sk.hat_scale, q->factor, st);
    ctx->pre.valid = false;
  }
  // lambda_0 = M w: one update step with g = w from a zero gradient and beta = 0
  Stepper S{ib, d, pl.f.M, 0, 0, 0, st, ctx, ErrorSink{}};
  S.start(nullptr, nullptr);
  launch_fill_f64(zero, 0.0, d, st);
  {
    // gpart rows of zero: reuse the update kernel with groups = 0 and w added
    UpdateArgs u;
    u.gpart = ib.gpart;
    u.groups = 0;
    u.ldp = (int)round_up(d + 1, 8);
    u.d = d;
    u.scale = 1.0;
    u.w = w;
    u.incw = incw;
    u.M = pl.f.M;
    u.ldm = d;
    u.beta = zero;
    u.beta_prev = zero;
    u.beta_next = ib.beta[0];
    u.mu = 1.0;
    u.eta = 0.0;
    u.beta_out = lam0;
    launch_update(u, st);
  }
  // s_max full-data steps on (X^T X) lambda = w: g = w + X^T (0 - X lambda)
  for (int j = 0; j < q->s_max; ++j) {
    S.step(p->N, p->X, p->ldx, nullptr, 1, p->dtype, SLSE_F64, 1.0, w, q->mu, q->eta, lambda_out,
           nullptr, nullptr, 0.0, incw);
  }
  const double* lam = ib.beta[S.cur];
  if (lambda_out && q->s_max == 0) launch_copy_f64(lam, lambda_out, d, st);
  AdjointArgs a;
  a.n = p->N;
  a.d = d;
  a.X = p->X;
  a.ldx = p->ldx;
  a.Y = p->Y;
  a.t = p->dtype;
  a.beta = beta_hat;
  a.lambda = lam;
  a.dX = dX;
  a.lddx = lddx;
  a.dY = dY;
  a.gt = grad_t;
  if (dX || dY) launch_adjoint(a, st);
  slse_status status = SLSE_OK;
  if (rep) {
    int flags[4] = {0, 0, 0, 0};
    int info[3] = {0, 0, 0};
    SLSE_HIP(hipMemcpyAsync(flags, ib.flags, sizeof(flags), hipMemcpyDeviceToHost, st));
    SLSE_HIP(hipMemcpyAsync(info, pl.f.info, sizeof(info), hipMemcpyDeviceToHost, st));
    SLSE_HIP(hipStreamSynchronize(st));
    if (info[0] || info[1] || info[2]) status = SLSE_ESINGULAR;
    else if (flags[1]) status = SLSE_ENONFINITE;
    std::memset(rep, 0, sizeof(*rep));
    rep->status = status;
    rep->stage2_steps = q->s_max;
  }
  return status;
}

// ---------------------------------------------------------------------------
// Batched solve: per-problem sketches and factors, then every M-IHS step of
// every problem in two launches per global step.
// ---------------------------------------------------------------------------
struct BatchPlan {
  int B = 0;
  // bytes / entries of each pool (for the plan checks)
  int64_t a_bytes = 0, ah_bytes = 0, m_n = 0, beta_n = 0, part_n = 0;
  int64_t bf_ad_n = 0, bf_cp_n = 0, bf_sq_n = 0, bf_splits = 1;
  size_t bsz_bytes = 0;  // shared SRHT workspaces
  slse_dtype t = SLSE_F32;
  std::vector<SketchShape> sk;
  std::vector<int64_t> lda, a_off, ah_off, m_off, beta_off, part_off;
  std::vector<int> steps_of;  // total steps of each problem
  int T = 0;                  // global steps (max over problems)
  int items = 1;  // work items per block of a full step (tiles = grid x items)
  int grid = 512;
  int cus = 256;  // compute units of the device
  bool vec = true;
  int nch = 4;
  char* Apool = nullptr;
  char* Ahpool = nullptr;
  double* Mpool = nullptr;
  double* Bpool = nullptr;  // 3 beta buffers per problem
  double* part = nullptr;
  int* flags = nullptr;     // per problem: non-finite
  int* finfo = nullptr;     // per problem: 3 ints of factor info
  BatchStep* d_steps = nullptr;
  int* d_prefix = nullptr;
  BatchProblem* d_probs = nullptr;
  std::vector<BatchStep> h_steps;
  std::vector<int> h_prefix;
  std::vector<int> h_total;
  std::vector<double> h_bytes;  // bytes of [X|Y] each step reads
  std::vector<BatchProblem> h_probs;
  SrhtArgs srht;
  GaussianArgs ga, gh;
  void* cs = nullptr;  // CountSketch bucket lists (sized for the largest problem)
  FactorBufs f;
  // SRHT index maps of every SRHT problem, built in two launches
  std::vector<SrhtIndexJob> h_sjobs;
  SrhtIndexJob* d_sjobs = nullptr;
  std::vector<int64_t> s_off;  // offset of problem b in the index pools (-1: not SRHT)
  // SRHT passes of every SRHT problem in shared launches (each with its own Z)
  std::vector<SrhtBatchLaunch> srht_launches;
  std::vector<char> h_srec;
  void* d_srec = nullptr;
  std::vector<char> srht_batched;  // problem b's sketch runs in the shared launches
  int64_t s_rows = 0, s_hat = 0;          // index-map rows and Hessian samples of all jobs
  int64_t s_max_npad = 0, s_max_r = 0;   // the largest of one job
  int32_t *s_pi = nullptr, *s_sa = nullptr, *s_sh = nullptr;
  // Cholesky route for every problem: one batched factorization
  bool batched_factor = false;
  int dmax = 0;
  int64_t rmax = 0;
  FactorJob* d_jobs = nullptr;
  std::vector<FactorJob> h_jobs;
};

constexpr int kBatchTileFloor = 256;  // tiles per problem <= ceil(rows / 256) (partial pool size)
constexpr int kBatchTileCeil = 1 << 20;  // and >= ceil(rows / 2^20)
constexpr int64_t kBatchMinTileBytes = int64_t(128) << 10;  // smallest tile a step is cut into
constexpr size_t kBatchSrhtZMax = size_t(16) << 30;  // workspace cap for shared SRHT launches

// smallest tile (bytes of [X|Y]) a batched step is cut into
// (SLSE_BATCH_MIN_TILE_KB overrides)
int64_t batch_min_tile_bytes() {
  static const int64_t v = [] {
    int64_t t = kBatchMinTileBytes;
    if (const char* e = std::getenv("SLSE_BATCH_MIN_TILE_KB"))
      t = std::max<int64_t>(16 << 10, (int64_t)std::atoi(e) << 10);
    return t;
  }();
  return v;
}

// lanes per row of the batched pass: one 16-byte vector of the row (an
// element when rows are not 16-byte aligned) per lane up to 16 lanes, more
// vectors per lane beyond that (at most 4, so up to 64 lanes); 16 lanes, i.e.
// 256 contiguous bytes of a row per load instruction and four xor steps per
// row dot, measured fastest (SLSE_BATCH_LPR_MAX overrides the 16)
int batch_lpr(int d, bool vec, slse_dtype t) {
  static const int cap = [] {
    int c = 16;
    if (const char* e = std::getenv("SLSE_BATCH_LPR_MAX")) c = std::atoi(e);
    return (c == 4 || c == 8 || c == 16 || c == 32 || c == 64) ? c : 16;
  }();
  const int v = vec ? 16 / (int)dtype_size(t) : 1;
  const int nvec = (int)ceil_div(d, v);
  int p2 = 1;
  while (p2 < nvec) p2 *= 2;
  int lpr = std::min(p2, cap);
  while (lpr < 64 && lpr * 4 < p2) lpr *= 2;
  return lpr;
}

// Tiles of one batched step.  Problem b has n[b] rows (0: idle) of
// row_bytes[b] bytes; the pass's main loop covers step_rows[b] rows per block
// step.  The step's bytes are cut into about `slots` tiles of equal size (no
// smaller than min_tile_bytes), shared out over the problems by largest
// remainder, so the grid's strided walk gives every block about the same
// bytes; a problem's rows are split evenly over its tiles, rounded up to
// whole main-loop steps (only its last tile has a remainder).  Every problem
// gets between ceil(n / 2^20) and ceil(n / 256) tiles (the partial pool holds
// ceil(n / 256) rows per problem).
void split_step_tiles(int B, const int64_t* n, const int64_t* row_bytes, const int64_t* step_rows,
                      int64_t slots, int64_t min_tile_bytes, int* tile_rows, int* ntiles) {
  double total = 0.0;
  for (int b = 0; b < B; ++b) total += (double)std::max<int64_t>(n[b], 0) * row_bytes[b];
  int64_t want = 0;
  if (total > 0.0)
    want = std::clamp<int64_t>((int64_t)std::ceil(total / (double)std::max<int64_t>(min_tile_bytes, 1)),
                               1, std::max<int64_t>(slots, 1));
  int64_t given = 0;
  std::vector<int64_t> lo(B, 0), cap(B, 0), tiles(B, 0);
  std::vector<double> frac(B, -1.0);
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) {
    if (n[b] <= 0) continue;
    lo[b] = ceil_div(n[b], (int64_t)kBatchTileCeil);
    cap[b] = ceil_div(n[b], (int64_t)kBatchTileFloor);
    const double q = (double)n[b] * row_bytes[b] * (double)want / total;
    tiles[b] = std::clamp<int64_t>((int64_t)q, lo[b], cap[b]);
    frac[b] = q - std::floor(q);
    given += tiles[b];
  }
  // one tile more for the largest remainders, or (when the one-tile minimum
  // of small problems overshot) one fewer for the smallest
  for (int b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return frac[x] > frac[y]; });
  for (int i = 0; i < B && given < want; ++i) {
    const int b = order[i];
    if (frac[b] < 0.0 || tiles[b] >= cap[b]) continue;
    ++tiles[b];
    ++given;
  }
  for (int i = B - 1; i >= 0 && given > want; --i) {
    const int b = order[i];
    if (frac[b] < 0.0 || tiles[b] <= lo[b]) continue;
    --tiles[b];
    --given;
  }
  for (int b = 0; b < B; ++b) {
    if (n[b] <= 0) {
      tile_rows[b] = 1;
      ntiles[b] = 0;
      continue;
    }
    const int64_t sr = std::max<int64_t>(step_rows[b], 1);
    tile_rows[b] = (int)std::min<int64_t>(round_up(ceil_div(n[b], tiles[b]), sr), n[b]);
    ntiles[b] = (int)ceil_div(n[b], (int64_t)tile_rows[b]);
  }
}

// Per-(step, problem) descriptors and tile prefix sums for a tile size.
void build_batch_tables(BatchPlan& bp, const slse_problem* ps, const slse_params* qs,
                        double* const* betas) {
  const int B = bp.B;
  bp.h_steps.assign((size_t)bp.T * B, BatchStep{});
  bp.h_prefix.assign((size_t)bp.T * (B + 1), 0);
  bp.h_total.assign(bp.T, 0);
  bp.h_bytes.assign(bp.T, 0.0);
  for (int b = 0; b < B; ++b) {
    const SketchShape& sk = bp.sk[b];
    const int d = (int)ps[b].d;
    const size_t es = dtype_size(bp.t);
    double* ring[3] = {bp.Bpool + bp.beta_off[b], bp.Bpool + bp.beta_off[b] + d,
                       bp.Bpool + bp.beta_off[b] + 2 * d};
    int cur = 0, prev = 0, t = 0;
    auto add = [&](const void* X, int64_t ldx, const void* Y, int64_t incy, int64_t n,
                   double scale) {
      const int next = (cur + 1) % 3 == prev ? (cur + 2) % 3 : (cur + 1) % 3;
      BatchStep& st = bp.h_steps[(size_t)t * B + b];
      st.X = X;
      st.ldx = ldx;
      st.Y = Y;
      st.incy = incy;
      st.n = n;
      st.scale = scale;
      st.beta = ring[cur];
      st.beta_prev = ring[prev];
      st.beta_next = ring[next];
      prev = cur;
      cur = next;
      ++t;
    };
    for (int i = 0; i < sk.K; ++i) {
      if (qs[b].momentum_reset) prev = cur;
      const char* base = bp.Apool + bp.a_off[b] + (size_t)sk.offset[i] * bp.lda[b] * es;
      for (int j = 0; j < qs[b].a[i]; ++j)
        add(base, bp.lda[b], base + (size_t)d * es, bp.lda[b], sk.m[i], sk.scale[i]);
    }
    if (qs[b].momentum_reset) prev = cur;
    for (int j = 0; j < qs[b].s_max; ++j) add(ps[b].X, ps[b].ldx, ps[b].Y, 1, ps[b].N, 1.0);
    (void)betas;
  }
  // Tiles per (step, problem): split_step_tiles
  const int64_t es = (int64_t)dtype_size(bp.t);
  const int64_t slots = (int64_t)bp.grid * bp.items;
  std::vector<int64_t> n(B), row_bytes(B), step_rows(B);
  std::vector<int> tile_rows(B), ntiles(B);
  for (int b = 0; b < B; ++b) {
    const BatchProblem& pr = bp.h_probs[b];
    row_bytes[b] = (ps[b].d + 1) * es;
    step_rows[b] = (int64_t)(kBatchThreads / 64) * (64 / pr.lpr) * (kBatchSlots / pr.ch);
  }
  for (int t = 0; t < bp.T; ++t) {
    BatchStep* row = &bp.h_steps[(size_t)t * B];
    double total = 0.0;
    for (int b = 0; b < B; ++b) {
      n[b] = std::max<int64_t>(row[b].n, 0);
      total += (double)n[b] * row_bytes[b];
    }
    bp.h_bytes[t] = total;
    split_step_tiles(B, n.data(), row_bytes.data(), step_rows.data(), slots,
                     batch_min_tile_bytes(), tile_rows.data(), ntiles.data());
    for (int b = 0; b < B; ++b) {
      row[b].tile_rows = tile_rows[b];
      row[b].ntiles = ntiles[b];
    }
  }
  for (int t = 0; t < bp.T; ++t) {
    int acc = 0;
    for (int b = 0; b < B; ++b) {
      bp.h_prefix[(size_t)t * (B + 1) + b] = acc;
      acc += bp.h_steps[(size_t)t * B + b].ntiles;
    }
    bp.h_prefix[(size_t)t * (B + 1) + B] = acc;
    bp.h_total[t] = acc;
  }
}

void enqueue_batch_steps(const BatchPlan& bp, hipStream_t st) {
  for (int t = 0; t < bp.T; ++t) {
    launch_batched_resid_grad(bp.d_steps + (size_t)t * bp.B, bp.d_probs,
                              bp.d_prefix + (size_t)t * (bp.B + 1), bp.B, bp.h_total[t], bp.grid,
                              bp.part, bp.t, bp.vec, bp.nch, st);
    launch_batched_update(bp.d_steps + (size_t)t * bp.B, bp.d_probs, bp.B, bp.dmax, bp.part,
                          bp.flags, st);
  }
}

// Sketch of problem b into its A / Ahat.
void enqueue_batch_sketch(const BatchPlan& bp, int b, const slse_problem* ps,
                          const slse_params* qs, hipStream_t st) {
  const SketchShape& sk = bp.sk[b];
  const int d = (int)ps[b].d;
  SrhtArgs sa = bp.srht;
  if (sk.kind == SLSE_SRHT) {
    sa.N = sk.N;
    sa.d = d;
    sa.p = sk.p;
    sa.mK = sk.m[sk.K - 1];
    sa.r = sk.r;
    srht_plan(sa, 0);
    if (bp.s_off[b] >= 0) {
      sa.pi_sgn = bp.s_pi + bp.s_off[b];
      sa.slotA = bp.s_sa + bp.s_off[b];
      sa.slotH = bp.s_sh + bp.s_off[b];
      sa.indices_ready = true;
    }
  }
  GaussianArgs ga = bp.ga, gh = bp.gh;
  ga.N = gh.N = sk.N;
  ga.d = gh.d = d;
  ga.m = sk.m[sk.K - 1];
  gh.m = sk.r;
  ga.bf16 = gh.bf16 = qs[b].precision == SLSE_PREC_MIXED && bp.t == SLSE_F32;
  if (sk.kind == SLSE_GAUSSIAN) {
    gaussian_plan(ga);
    gaussian_plan(gh);
  }
  void* A = bp.Apool + bp.a_off[b];
  void* Ah = bp.Ahpool + bp.ah_off[b];
  enqueue_sketch(sk, qs[b].seed, ps[b].X, ps[b].ldx, ps[b].Y, bp.t, A, bp.lda[b], Ah, bp.lda[b],
                 sa, ga, gh, st, bp.cs);
}

// Factor of problem b through the shared scratch (the QR route).
void enqueue_batch_factor(const BatchPlan& bp, int b, const slse_problem* ps,
                          const slse_params* qs, hipStream_t st) {
  const SketchShape& sk = bp.sk[b];
  const int d = (int)ps[b].d;
  FactorBufs f = bp.f;
  f.info = bp.finfo + 3 * b;
  enqueue_factor(f, sk.r, d, bp.Ahpool + bp.ah_off[b], bp.lda[b], bp.t, sk.hat_scale, qs[b].factor,
                 st);
  launch_copy_f64(f.M, bp.Mpool + bp.m_off[b], (int64_t)d * d, st);
}

// Sketches one problem after another, the factorizations (one batched launch
// sequence on the Cholesky route), the initial iterates, then the batched steps.
void enqueue_batch(const BatchPlan& bp, const slse_problem* ps, const slse_params* qs,
                   hipStream_t st) {
  launch_fill_i32(bp.flags, 0, bp.B, st);
  launch_fill_i32(bp.finfo, 0, 3 * (int64_t)bp.B, st);
  if (!bp.h_sjobs.empty())
    launch_srht_index_batched(bp.d_sjobs, (int)bp.h_sjobs.size(), bp.s_max_npad, bp.s_max_r, st);
  if (!bp.srht_launches.empty()) launch_srht_batched(bp.srht_launches, bp.d_srec, bp.t, st);
  for (int b = 0; b < bp.B; ++b)
    if (bp.srht_batched.empty() || !bp.srht_batched[b]) enqueue_batch_sketch(bp, b, ps, qs, st);
  if (bp.batched_factor)
    launch_factor_batched(bp.d_jobs, bp.B, bp.dmax, bp.rmax, bp.t, st);
  else
    for (int b = 0; b < bp.B; ++b) enqueue_batch_factor(bp, b, ps, qs, st);
  launch_batched_init(bp.d_probs, bp.B, bp.dmax, st);
  enqueue_batch_steps(bp, st);
}

// The host plan of a batch: shapes, pools and offsets, SRHT jobs and
// records, factor jobs, per-problem descriptors and the launch shape.  Every
// buffer comes from ctx->arena (so a measuring arena plans without device
// work); nothing is uploaded or launched here.  Returns the autotune key and
// whether the launch shape is already known.
std::pair<std::string, bool> plan_batched(slse_ctx* ctx, int B, const slse_problem* ps,
                                          const slse_params* qs, double* const* betas,
                                          BatchPlan& bp) {
  bp.B = B;
  bp.cus = ctx->num_cus;
  bp.t = ps[0].dtype;
  for (int b = 0; b < B; ++b) {
    check_params(&ps[b], &qs[b]);
    require(qs[b].start_step == 0 && qs[b].stop_step == 0 && !qs[b].beta_prev && !qs[b].state_out,
            "batched solves do not checkpoint or resume");
    require(betas[b] != nullptr, "null beta pointer in the batch");
    require(ps[b].dtype == bp.t, "every problem of a batch must share one storage dtype");
    require(ps[b].d <= 512, "batched problems need d <= 512");
  }
  const size_t es = dtype_size(bp.t);
  int64_t a_bytes = 0, ah_bytes = 0, m_n = 0, beta_n = 0, max_npad = 0, max_rows = 0, max_d = 0;
  int64_t max_r = 0;
  size_t z_bytes = 0, g_bytes = 0, cs_bytes = 0;
  bp.vec = true;
  for (int b = 0; b < B; ++b) {
    bp.sk.push_back(make_sketch_shape(qs[b].kind, ps[b].N, ps[b].d, qs[b].m, qs[b].K, qs[b].r));
    const SketchShape& sk = bp.sk.back();
    const int64_t d = ps[b].d;
    const int64_t lda = sketch_ld(d, es);
    bp.lda.push_back(lda);
    bp.a_off.push_back(a_bytes);
    a_bytes += round_up((int64_t)(sk.rows_A * lda * es), 256);
    bp.ah_off.push_back(ah_bytes);
    ah_bytes += round_up((int64_t)(sk.r * lda * es), 256);
    bp.m_off.push_back(m_n);
    m_n += d * d;
    bp.beta_off.push_back(beta_n);
    beta_n += 3 * d;
    max_npad = std::max(max_npad, sk.n_pad);
    max_r = std::max(max_r, sk.r);
    max_d = std::max(max_d, d);
    max_rows = std::max(max_rows, std::max<int64_t>(sk.rows_A, ps[b].N));
    if (sk.kind == SLSE_SRHT) {
      SrhtArgs sa;
      sa.t = bp.t;
      sa.d = (int)d;
      sa.p = sk.p;
      srht_plan(sa, 0);
      z_bytes = std::max(z_bytes, srht_z_bytes(sa));
    } else if (sk.kind == SLSE_COUNTSKETCH) {
      CountSketchArgs c;
      c.t = bp.t;
      c.N = sk.N;
      c.d = (int)d;
      c.m = sk.m.data();
      c.K = sk.K;
      c.r = sk.r;
      cs_bytes = std::max(cs_bytes, countsketch_scratch_bytes(c));
    } else if (sk.kind == SLSE_GAUSSIAN) {
      GaussianArgs g1, g2;
      g1.t = g2.t = bp.t;
      g1.bf16 = g2.bf16 = qs[b].precision == SLSE_PREC_MIXED && bp.t == SLSE_F32;
      g1.N = g2.N = sk.N;
      g1.d = g2.d = (int)d;
      g1.m = sk.m[sk.K - 1];
      g2.m = sk.r;
      gaussian_plan(g1);
      gaussian_plan(g2);
      g_bytes = std::max({g_bytes, gaussian_scratch_bytes(g1), gaussian_scratch_bytes(g2)});
    }
    const int es_i = (int)es;
    if ((reinterpret_cast<uintptr_t>(ps[b].X) % 16) || ((ps[b].ldx * es_i) % 16)) bp.vec = false;
  }
  bp.a_bytes = a_bytes;
  bp.ah_bytes = ah_bytes;
  bp.m_n = m_n;
  bp.beta_n = beta_n;
  bp.Apool = static_cast<char*>(ctx->arena.get("bA", (size_t)a_bytes));
  bp.Ahpool = static_cast<char*>(ctx->arena.get("bAhat", (size_t)ah_bytes));
  bp.Mpool = ctx->arena.get_t<double>("bM", (size_t)m_n);
  bp.Bpool = ctx->arena.get_t<double>("bBeta", (size_t)beta_n);
  bp.flags = ctx->arena.get_t<int>("bFlags", (size_t)B);
  bp.finfo = ctx->arena.get_t<int>("bInfo", (size_t)3 * B);
  bp.srht.pi_sgn = ctx->arena.get_t<int32_t>("srht_pi", (size_t)max_npad);
  bp.srht.slotA = ctx->arena.get_t<int32_t>("srht_slotA", (size_t)max_npad);
  bp.srht.slotH = ctx->arena.get_t<int32_t>("srht_slotH", (size_t)max_npad);
  bp.srht.Z = z_bytes ? ctx->arena.get("srht_Z", z_bytes) : nullptr;
  bp.cs = cs_bytes ? ctx->arena.get("cs_lists", cs_bytes) : nullptr;
  // per-problem SRHT index maps
  bp.s_off.assign(B, -1);
  for (int b = 0; b < B; ++b) {
    const SketchShape& sk = bp.sk[b];
    if (sk.kind != SLSE_SRHT) continue;
    SrhtArgs sa;
    sa.t = bp.t;
    sa.d = (int)ps[b].d;
    sa.p = sk.p;
    srht_plan(sa, 0);
    SrhtIndexJob j{};
    j.npad = sk.n_pad;
    j.r = sk.r;
    j.mK = sk.m[sk.K - 1];
    j.seed = qs[b].seed;
    j.p = sk.p;
    srht_last_pass(sa, &j.s0_last, &j.b_last);
    j.base = bp.s_rows;
    j.hbase = bp.s_hat;
    bp.s_off[b] = bp.s_rows;
    bp.s_rows += sk.n_pad;
    bp.s_hat += sk.r;
    bp.s_max_npad = std::max<int64_t>(bp.s_max_npad, sk.n_pad);
    bp.s_max_r = std::max<int64_t>(bp.s_max_r, sk.r);
    bp.h_sjobs.push_back(j);
  }
  if (!bp.h_sjobs.empty()) {
    bp.s_pi = ctx->arena.get_t<int32_t>("bSrhtPi", (size_t)bp.s_rows);
    bp.s_sa = ctx->arena.get_t<int32_t>("bSrhtSlotA", (size_t)bp.s_rows);
    bp.s_sh = ctx->arena.get_t<int32_t>("bSrhtSlotH", (size_t)bp.s_rows);
    for (SrhtIndexJob& j : bp.h_sjobs) {
      j.pi_sgn = bp.s_pi + j.base;
      j.slotA = bp.s_sa + j.base;
      j.slotH = bp.s_sh + j.base;
    }
    bp.d_sjobs = ctx->arena.get_t<SrhtIndexJob>("bSrhtJobs", bp.h_sjobs.size());
    // the passes of every SRHT in shared launches, each transform with its
    // own workspace (skipped when those would exceed kBatchSrhtZMax bytes)
    std::vector<SrhtArgs> sas;
    std::vector<int> who;
    size_t zsum = 0;
    for (int b = 0; b < B; ++b) {
      if (bp.s_off[b] < 0) continue;
      const SketchShape& sk = bp.sk[b];
      SrhtArgs sa;
      sa.t = bp.t;
      sa.N = sk.N;
      sa.d = (int)ps[b].d;
      sa.p = sk.p;
      srht_plan(sa, 0);
      sa.X = ps[b].X;
      sa.ldx = ps[b].ldx;
      sa.Y = ps[b].Y;
      sa.A = bp.Apool + bp.a_off[b];
      sa.lda = bp.lda[b];
      sa.Ahat = bp.Ahpool + bp.ah_off[b];
      sa.ldah = bp.lda[b];
      sa.pi_sgn = bp.s_pi + bp.s_off[b];
      sa.slotA = bp.s_sa + bp.s_off[b];
      sa.slotH = bp.s_sh + bp.s_off[b];
      sa.Z = reinterpret_cast<void*>(zsum);  // offset until the pool exists
      zsum += round_up((int64_t)srht_z_bytes(sa), 256);
      sas.push_back(sa);
      who.push_back(b);
    }
    bp.srht_batched.assign(B, 0);
    if (!sas.empty() && zsum <= kBatchSrhtZMax) {
      char* zpool = zsum ? static_cast<char*>(ctx->arena.get("bSrhtZ", zsum)) : nullptr;
      bp.bsz_bytes = zsum;
      for (SrhtArgs& sa : sas)
        sa.Z = srht_z_bytes(sa) ? zpool + reinterpret_cast<uintptr_t>(sa.Z) : nullptr;
      bp.srht_launches = srht_batch_plan(sas, bp.t, bp.h_srec);
      bp.d_srec = ctx->arena.get("bSrhtRec", bp.h_srec.size());
      for (int b : who) bp.srht_batched[b] = 1;
    }
  }
  bp.srht.t = bp.t;
  bp.ga.t = bp.gh.t = bp.t;
  bp.ga.stream_id = 7;
  bp.gh.stream_id = 8;
  if (g_bytes) {
    void* gp = ctx->arena.get("gauss_part", g_bytes);
    bp.ga.partial = bp.gh.partial = static_cast<float*>(gp);
    bp.ga.partial64 = bp.gh.partial64 = static_cast<double*>(gp);
  }
  slse_factor_method fm = SLSE_FACTOR_CHOL;
  for (int b = 0; b < B; ++b)
    if (qs[b].factor == SLSE_FACTOR_QR) fm = SLSE_FACTOR_QR;
  bp.dmax = (int)max_d;
  bp.rmax = max_r;
  bp.batched_factor = fm == SLSE_FACTOR_CHOL;
  if (bp.batched_factor) {
    // each problem owns its scaled sketch Ad and a Gauss-Jordan column panel;
    // the Gram is formed in its M-pool slot and inverted there
    const int splits = factor_batched_splits(max_r);
    int64_t ad_n = 0, cp_n = 0, sq_n = 0;
    for (int b = 0; b < B; ++b) {
      ad_n += bp.sk[b].r * ps[b].d;
      cp_n += ps[b].d * 32;
      sq_n += ps[b].d * ps[b].d;
    }
    double* adp = ctx->arena.get_t<double>("bfAd", (size_t)ad_n);
    double* cpp = ctx->arena.get_t<double>("bfColp", (size_t)cp_n);
    double* pp = splits > 1 ? ctx->arena.get_t<double>("bfPart", (size_t)(splits * sq_n)) : nullptr;
    bp.bf_ad_n = ad_n;
    bp.bf_cp_n = cp_n;
    bp.bf_sq_n = sq_n;
    bp.bf_splits = splits;
    bp.h_jobs.resize(B);
    int64_t ao = 0, co = 0, so = 0;
    for (int b = 0; b < B; ++b) {
      FactorJob& j = bp.h_jobs[b];
      const int64_t d = ps[b].d;
      j.A = bp.Ahpool + bp.ah_off[b];
      j.lda = bp.lda[b];
      j.rows = bp.sk[b].r;
      j.d = (int)d;
      j.scale = std::sqrt(bp.sk[b].hat_scale);
      j.Ad = adp + ao;
      j.M = bp.Mpool + bp.m_off[b];
      j.G = j.M;
      j.colp = cpp + co;
      j.part = pp ? pp + splits * so : nullptr;
      j.info = bp.finfo + 3 * b;
      ao += j.rows * d;
      co += d * 32;
      so += d * d;
    }
    bp.d_jobs = ctx->arena.get_t<FactorJob>("bJobs", (size_t)B);
  } else {
    bp.f = reserve_factor(ctx, max_r, max_d, fm);
  }
  // steps of every problem
  for (int b = 0; b < B; ++b) {
    int T = qs[b].s_max;
    for (int i = 0; i < qs[b].K; ++i) T += qs[b].a[i];
    bp.steps_of.push_back(T);
    bp.T = std::max(bp.T, T);
  }
  // lane groups and chunk count (one kernel shape for the whole batch)
  bp.h_probs.resize(B);
  int nch = 1;
  for (int b = 0; b < B; ++b) {
    const int d = (int)ps[b].d;
    const int lpr = batch_lpr(d, bp.vec, bp.t);
    const int v = bp.vec ? 16 / (int)es : 1;
    int c = (int)ceil_div(ceil_div(d, v), lpr);
    int p2 = 1;
    while (p2 < c) p2 *= 2;
    require(p2 <= 4, "batched: d too large for the batched kernel");
    nch = std::max(nch, p2);
    BatchProblem& pr = bp.h_probs[b];
    pr.d = d;
    pr.lpr = lpr;
    pr.ch = p2;
    pr.M = bp.Mpool + bp.m_off[b];
    pr.beta_out = betas[b];
    const double eta = qs[b].eta, mu = qs[b].mu;
    pr.mu = mu;
    pr.eta = eta;
    pr.beta0 = qs[b].beta0;
    // the first step of every problem reads beta slot 0 of its ring
    pr.beta_init = bp.steps_of[b] > 0 ? bp.Bpool + bp.beta_off[b] : nullptr;
  }
  bp.nch = nch;
  // tile size and grid: autotuned once per batch shape on a stage-2 step
  int64_t rows_total = 0;
  for (int b = 0; b < B; ++b) rows_total += ps[b].N;
  const std::string key = "batched/" + std::to_string(B) + "/" + std::to_string(rows_total) + "/" +
                          std::to_string((int)bp.t);
  bool tuned = false;
  if (auto it = ctx->rg_tune.find(key); it != ctx->rg_tune.end()) {
    bp.grid = it->second.first;
    bp.items = it->second.second;
    tuned = true;
  } else if (const char* e = std::getenv("SLSE_BATCH_GRID")) {
    // fixed launch shape (SLSE_BATCH_GRID blocks, SLSE_BATCH_ITEMS tiles each)
    bp.grid = std::max(1, std::atoi(e));
    const char* k = std::getenv("SLSE_BATCH_ITEMS");
    bp.items = std::max(1, k ? std::atoi(k) : 1);
    tuned = true;
  } else {
    bp.grid = 4 * ctx->num_cus;
    bp.items = 1;
  }
  // partial pool sized for the shortest tile a step may use
  int64_t part_n = 0;
  for (int b = 0; b < B; ++b) {
    bp.part_off.push_back(part_n);
    part_n += ceil_div(std::max<int64_t>(bp.sk[b].rows_A, ps[b].N), (int64_t)kBatchTileFloor) *
              (ps[b].d + 1);
  }
  bp.part = ctx->arena.get_t<double>("bPart", (size_t)part_n + 1);
  bp.d_steps = ctx->arena.get_t<BatchStep>("bSteps", (size_t)bp.T * B);
  bp.d_prefix = ctx->arena.get_t<int>("bPrefix", (size_t)bp.T * (B + 1));
  bp.d_probs = ctx->arena.get_t<BatchProblem>("bProbs", (size_t)B);
  for (int b = 0; b < B; ++b) bp.h_probs[b].part_off = bp.part_off[b];
  bp.part_n = part_n;
  return {key, tuned};
}

slse_status batched_impl(slse_ctx* ctx, int B, const slse_problem* ps, const slse_params* qs,
                         double* const* betas, slse_report* reps, hipStream_t st) {
  BatchPlan bp;
  ctx->arena.grew = false;
  auto [key, tuned] = plan_batched(ctx, B, ps, qs, betas, bp);
  if (ctx->arena.grew) ctx->drop_graphs();
  // the tables below are rewritten for this call: the previous batch's graph
  // (on whatever stream it ran) must be done reading them
  if (ctx->batch_busy) {
    SLSE_HIP(hipEventSynchronize(ctx->batch_done));
    ctx->batch_busy = false;
  }
  SLSE_HIP(hipMemcpy(bp.d_probs, bp.h_probs.data(), sizeof(BatchProblem) * B, hipMemcpyHostToDevice));
  if (bp.batched_factor)
    SLSE_HIP(hipMemcpy(bp.d_jobs, bp.h_jobs.data(), sizeof(FactorJob) * B, hipMemcpyHostToDevice));
  if (!bp.h_srec.empty())
    SLSE_HIP(hipMemcpy(bp.d_srec, bp.h_srec.data(), bp.h_srec.size(), hipMemcpyHostToDevice));
  if (!bp.h_sjobs.empty())
    SLSE_HIP(hipMemcpy(bp.d_sjobs, bp.h_sjobs.data(), sizeof(SrhtIndexJob) * bp.h_sjobs.size(),
                       hipMemcpyHostToDevice));

  auto upload = [&]() {
    build_batch_tables(bp, ps, qs, betas);
    SLSE_HIP(hipMemcpy(bp.d_steps, bp.h_steps.data(), sizeof(BatchStep) * bp.h_steps.size(),
                       hipMemcpyHostToDevice));
    SLSE_HIP(hipMemcpy(bp.d_prefix, bp.h_prefix.data(), sizeof(int) * bp.h_prefix.size(),
                       hipMemcpyHostToDevice));
  };
  if (!tuned && bp.T > 0) {
    // time the step with the most bytes for a few (grid, tiles per block) shapes
    const char* env = std::getenv("SLSE_AUTOTUNE");
    const bool do_tune = !(env && std::atoi(env) == 0);
    std::pair<int, int> best{bp.grid, bp.items};
    if (do_tune) {
      hipEvent_t e0, e1;
      SLSE_HIP(hipEventCreate(&e0));
      SLSE_HIP(hipEventCreate(&e1));
      float best_ms = 1e30f;
      for (int g : {ctx->num_cus, 2 * ctx->num_cus, 3 * ctx->num_cus, 4 * ctx->num_cus})
        for (int k : {1, 2, 4}) {
          bp.grid = g;
          bp.items = k;
          upload();
          const int tmax = (int)(std::max_element(bp.h_bytes.begin(), bp.h_bytes.end()) -
                                 bp.h_bytes.begin());
          auto run = [&]() {
            launch_batched_resid_grad(bp.d_steps + (size_t)tmax * B, bp.d_probs,
                                      bp.d_prefix + (size_t)tmax * (B + 1), B, bp.h_total[tmax],
                                      g, bp.part, bp.t, bp.vec, bp.nch, st);
          };
          run();
          SLSE_HIP(hipEventRecord(e0, st));
          for (int r = 0; r < 3; ++r) run();
          SLSE_HIP(hipEventRecord(e1, st));
          SLSE_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          SLSE_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best_ms) {
            best_ms = ms;
            best = {g, k};
          }
        }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    ctx->rg_tune[key] = best;
    bp.grid = best.first;
    bp.items = best.second;
  }
  upload();
  // one graph for the whole batch (sketches, factors, every step)
  std::string gk = key;
  auto add_key = [&gk](const void* v, size_t n) { gk.append(static_cast<const char*>(v), n); };
  for (int b = 0; b < B; ++b) {
    add_key(&ps[b], sizeof(slse_problem));
    add_key(&qs[b], sizeof(slse_params));
    add_key(&betas[b], sizeof(double*));
  }
  launch_cached_graph(ctx, gk, st, [&](hipStream_t cs) { enqueue_batch(bp, ps, qs, cs); });
  if (!ctx->batch_done) SLSE_HIP(hipEventCreateWithFlags(&ctx->batch_done, hipEventDisableTiming));
  SLSE_HIP(hipEventRecord(ctx->batch_done, st));
  ctx->batch_busy = true;
  ctx->pre.valid = false;
  slse_status worst = SLSE_OK;
  if (reps) {
    std::vector<int> flags(B), info(3 * B);
    SLSE_HIP(hipMemcpyAsync(flags.data(), bp.flags, sizeof(int) * B, hipMemcpyDeviceToHost, st));
    SLSE_HIP(hipMemcpyAsync(info.data(), bp.finfo, sizeof(int) * 3 * B, hipMemcpyDeviceToHost, st));
    SLSE_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
      slse_status sb = SLSE_OK;
      if (info[3 * b] || info[3 * b + 1] || info[3 * b + 2])
        sb = SLSE_ESINGULAR;
      else if (flags[b])
        sb = SLSE_ENONFINITE;
      std::memset(&reps[b], 0, sizeof(slse_report));
      reps[b].status = sb;
      int s1 = 0;
      for (int i = 0; i < qs[b].K; ++i) s1 += qs[b].a[i];
      reps[b].stage1_steps = s1;
      reps[b].stage2_steps = qs[b].s_max;
      if (sb < worst) worst = sb;
    }
  }
  return worst;
}

// Checks of a batch plan made on a measuring arena: every device pointer the
// tables hold, with the extent the kernels touch, lies inside the region the
// arena handed out for its pool; the tiles of every step cover each row once
// and fit the partial pool; the prefix sums match the tile counts.
void check_batch_plan(const Arena& ar, const BatchPlan& bp, const slse_problem* ps) {
  auto region = [&](const char* name) {
    auto it = ar.ext_bufs.find(name);
    require(it != ar.ext_bufs.end(), std::string("plan: no region ") + name);
    const uintptr_t lo = reinterpret_cast<uintptr_t>(it->second.p);
    return std::make_pair(lo, lo + it->second.bytes);
  };
  auto inside = [&](const void* p, int64_t bytes, const char* name, const std::string& what) {
    const auto [lo, hi] = region(name);
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    require(bytes >= 0 && a >= lo && a + (uintptr_t)bytes <= hi,
            "plan: " + what + " outside " + name);
  };
  const int B = bp.B;
  const int64_t es = (int64_t)dtype_size(bp.t);
  for (int b = 0; b < B; ++b) {
    const SketchShape& sk = bp.sk[b];
    const int64_t d = ps[b].d;
    const std::string tag = "problem " + std::to_string(b);
    const char* A = bp.Apool + bp.a_off[b];
    const int64_t a_len = sk.rows_A * bp.lda[b] * es;
    inside(A, a_len, "bA", tag + " sketch rows");
    inside(bp.Ahpool + bp.ah_off[b], sk.r * bp.lda[b] * es, "bAhat", tag + " Hessian sketch");
    inside(bp.Mpool + bp.m_off[b], d * d * 8, "bM", tag + " M");
    inside(bp.Bpool + bp.beta_off[b], 3 * d * 8, "bBeta", tag + " iterate ring");
    const int64_t cap = ceil_div(std::max<int64_t>(sk.rows_A, ps[b].N), (int64_t)kBatchTileFloor);
    require(bp.part_off[b] + cap * (d + 1) <= bp.part_n, "plan: " + tag + " partial rows");
    inside(bp.part + bp.part_off[b], cap * (d + 1) * 8, "bPart", tag + " partial rows");
    const BatchProblem& pr = bp.h_probs[b];
    require(pr.d == d && pr.part_off == bp.part_off[b], "plan: " + tag + " descriptor");
    require(pr.M == bp.Mpool + bp.m_off[b], "plan: " + tag + " descriptor M");
    require(pr.lpr >= 1 && pr.lpr <= 64 && (pr.ch == 1 || pr.ch == 2 || pr.ch == 4),
            "plan: " + tag + " lane shape");
    if (bp.batched_factor) {
      const FactorJob& j = bp.h_jobs[b];
      inside(j.A, (j.rows - 1) * j.lda * es + d * es, "bAhat", tag + " factor input");
      inside(j.Ad, j.rows * d * 8, "bfAd", tag + " factor Ad");
      inside(j.colp, d * 32 * 8, "bfColp", tag + " factor panel");
      inside(j.M, d * d * 8, "bM", tag + " factor M");
      if (j.part) inside(j.part, bp.bf_splits * d * d * 8, "bfPart", tag + " factor partials");
      inside(j.info, 3 * 4, "bInfo", tag + " factor info");
    }
    if (bp.s_off[b] >= 0) require(bp.s_off[b] + sk.n_pad <= bp.s_rows, "plan: " + tag + " SRHT maps");
  }
  for (const SrhtIndexJob& j : bp.h_sjobs) {
    require(j.base + j.npad <= bp.s_rows && j.hbase + j.r <= bp.s_hat, "plan: SRHT job range");
    inside(j.pi_sgn, j.npad * 4, "bSrhtPi", "SRHT job pi");
    inside(j.slotA, j.npad * 4, "bSrhtSlotA", "SRHT job slotA");
    inside(j.slotH, j.npad * 4, "bSrhtSlotH", "SRHT job slotH");
  }
  if (!bp.h_sjobs.empty()) inside(bp.d_sjobs, (int64_t)(bp.h_sjobs.size() * sizeof(SrhtIndexJob)),
                                  "bSrhtJobs", "SRHT job table");
  if (!bp.h_srec.empty()) inside(bp.d_srec, (int64_t)bp.h_srec.size(), "bSrhtRec", "SRHT records");
  inside(bp.d_steps, (int64_t)((size_t)bp.T * B * sizeof(BatchStep)), "bSteps", "step table");
  inside(bp.d_prefix, (int64_t)((size_t)bp.T * (B + 1) * sizeof(int)), "bPrefix", "prefix table");
  inside(bp.d_probs, (int64_t)(B * sizeof(BatchProblem)), "bProbs", "problem table");
  require(bp.h_steps.size() == (size_t)bp.T * B && bp.h_prefix.size() == (size_t)bp.T * (B + 1),
          "plan: table sizes");
  for (int t = 0; t < bp.T; ++t) {
    int acc = 0;
    for (int b = 0; b < B; ++b) {
      const BatchStep& st = bp.h_steps[(size_t)t * B + b];
      const std::string tag = "step " + std::to_string(t) + " problem " + std::to_string(b);
      require(bp.h_prefix[(size_t)t * (B + 1) + b] == acc, "plan: " + tag + " prefix");
      acc += st.ntiles;
      if (st.n <= 0) {
        require(st.ntiles == 0, "plan: " + tag + " idle problem with tiles");
        continue;
      }
      const int64_t d = ps[b].d;
      require(st.tile_rows >= 1 && st.ntiles >= 1, "plan: " + tag + " empty tiling");
      require((int64_t)(st.ntiles - 1) * st.tile_rows < st.n &&
                  st.n <= (int64_t)st.ntiles * st.tile_rows,
              "plan: " + tag + " tiles do not cover the rows once");
      const int64_t cap = ceil_div(std::max<int64_t>(bp.sk[b].rows_A, ps[b].N), (int64_t)kBatchTileFloor);
      require(st.ntiles <= cap, "plan: " + tag + " more tiles than partial rows");
      const char* A = bp.Apool + bp.a_off[b];
      if (st.X != ps[b].X) {  // a stage-1 step reads a prefix of the sketch rows
        const int64_t a_len = bp.sk[b].rows_A * bp.lda[b] * es;
        const uintptr_t x = reinterpret_cast<uintptr_t>(st.X), y = reinterpret_cast<uintptr_t>(st.Y);
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(A);
        require(x >= a0 && x + (uintptr_t)(((st.n - 1) * st.ldx + d) * es) <= a0 + (uintptr_t)a_len,
                "plan: " + tag + " X outside the problem's sketch rows");
        require(y >= a0 && y + (uintptr_t)(((st.n - 1) * st.incy + 1) * es) <= a0 + (uintptr_t)a_len,
                "plan: " + tag + " Y outside the problem's sketch rows");
      } else {
        require(st.n == ps[b].N && st.Y == ps[b].Y && st.incy == 1, "plan: " + tag + " full-data step");
      }
      for (const double* q : {st.beta, (const double*)st.beta_prev, (const double*)st.beta_next})
        inside(q, d * 8, "bBeta", tag + " iterate");
      const uintptr_t r0 = reinterpret_cast<uintptr_t>(bp.Bpool + bp.beta_off[b]);
      for (const double* q : {st.beta, (const double*)st.beta_prev, (const double*)st.beta_next})
        require(reinterpret_cast<uintptr_t>(q) >= r0 &&
                    reinterpret_cast<uintptr_t>(q) + (uintptr_t)(d * 8) <= r0 + (uintptr_t)(3 * d * 8),
                "plan: " + tag + " iterate outside the problem's ring");
    }
    require(bp.h_prefix[(size_t)t * (B + 1) + B] == acc && bp.h_total[t] == acc,
            "plan: step " + std::to_string(t) + " total tiles");
  }
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free residual-gradient entry point
// (slse_fused_resid_grad_noalloc): the group tickets, group partial rows and
// block partial rows of one pass, for grids of up to kNoAllocBlocks blocks and
// d <= kNoAllocMaxD.  Each device holds its own copy for the life of the
// process, located once per device when a context is created on it; calls on
// one device share it, so they must not overlap.
// ---------------------------------------------------------------------------
constexpr int kNoAllocBlocks = 512;
constexpr int kNoAllocMaxD = 1024;
constexpr int64_t kNoAllocLdp = 1032;  // partial row stride at d = kNoAllocMaxD: d + 1 rounded to 8
constexpr int64_t kNoAllocGroups = kNoAllocBlocks / 32;
constexpr size_t kNoAllocTicketBytes = 256;
constexpr size_t kNoAllocGpartBytes = ((kNoAllocGroups * kNoAllocLdp * 8 + 255) / 256) * 256;
constexpr size_t kNoAllocBytes =
    kNoAllocTicketBytes + kNoAllocGpartBytes + (size_t)kNoAllocBlocks * kNoAllocLdp * 8;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kNoAllocMaxDevices] = {};

// With `device` current: find this device's copy of `scratch` and clear its
// tickets (every pass leaves them at zero again).
void setup_noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  require(device >= 0 && device < kNoAllocMaxDevices, "device index above the scratch table");
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  SLSE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  require(p != nullptr, "no device address for the fixed scratch");
  launch_fill_i32(static_cast<int*>(p), 0, (int64_t)(kNoAllocTicketBytes / sizeof(int)), nullptr);
  SLSE_HIP(hipStreamSynchronize(nullptr));
  g_scratch_ptr[device] = static_cast<char*>(p);
}

template <typename F>
slse_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return SLSE_EDEVICE;
  } catch (...) {
    set_last_error("unknown error");
    return SLSE_EDEVICE;
  }
}

}  // namespace
}  // namespace slse

using namespace slse;

extern "C" {

const char* slse_last_error(void) { return g_last_error.c_str(); }

const char* slse_version(void) { return "libslse 0.1 (gfx950)"; }

slse_status slse_ctx_create(slse_ctx** out, int device) {
  return guarded([&]() -> slse_status {
    require(out != nullptr, "null out");
    int n = 0;
    SLSE_HIP(hipGetDeviceCount(&n));
    require(device >= 0 && device < n, "bad device index");
    DeviceGuard g(device);
    auto ctx = std::make_unique<slse_ctx>();
    ctx->device = device;
    hipDeviceProp_t prop;
    SLSE_HIP(hipGetDeviceProperties(&prop, device));
    ctx->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    ctx->arch = std::string(prop.gcnArchName) + "/" + std::to_string(ctx->num_cus);
    SLSE_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    setup_noalloc_scratch(device);
    *out = ctx.release();
    return SLSE_OK;
  });
}

slse_status slse_ctx_destroy(slse_ctx* ctx) {
  if (!ctx) return SLSE_OK;
  return guarded([&]() -> slse_status {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->drop_graphs();
    ctx->arena.release();
    if (ctx->batch_done) (void)hipEventDestroy(ctx->batch_done);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
    return SLSE_OK;
  });
}

slse_status slse_ctx_trim(slse_ctx* ctx) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr, "null ctx");
    DeviceGuard g(ctx->device);
    SLSE_HIP(hipDeviceSynchronize());
    ctx->drop_graphs();
    ctx->arena.release();
    ctx->pre.valid = false;
    return SLSE_OK;
  });
}

slse_status slse_sketch_apply(slse_ctx* ctx, slse_sketch_kind kind, uint64_t seed, int64_t N,
                              int64_t d, const void* X, int64_t ldx, const void* Y,
                              slse_dtype in_t, const int64_t* m, int32_t K, int64_t r, void* A,
                              int64_t lda, void* Ahat, int64_t ldah, slse_dtype out_t,
                              slse_sketch_layout* layout_out, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr, "null ctx");
    require(X && Y && A && Ahat, "null pointer");
    require(ldx >= d && lda >= d + 1 && ldah >= d + 1, "leading dimension too small");
    require(in_t == SLSE_F32 || in_t == SLSE_F64, "in dtype must be F32 or F64");
    const bool bf16 = out_t == SLSE_BF16;
    if (bf16 && !(kind == SLSE_GAUSSIAN && in_t == SLSE_F32))
      fail(SLSE_EUNSUPPORTED, "BF16 products are offered for the Gaussian sketch of F32 data");
    if (!bf16 && out_t != in_t) fail(SLSE_EUNSUPPORTED, "out dtype must equal in dtype in this library");
    DeviceGuard g(ctx->device);
    SketchShape s = make_sketch_shape(kind, N, d, m, K, r);
    SrhtArgs srht;
    GaussianArgs ga, gh;
    void* cs = nullptr;
    ctx->arena.grew = false;
    reserve_sketch(ctx, s, in_t, &srht, &ga, &gh, bf16, &cs);
    if (ctx->arena.grew) ctx->drop_graphs();
    ctx->pre.valid = false;
    enqueue_sketch(s, seed, X, ldx, Y, in_t, A, lda, Ahat, ldah, srht, ga, gh, as_stream(stream), cs);
    fill_layout(s, layout_out);
    return SLSE_OK;
  });
}

slse_status slse_factor(slse_ctx* ctx, int64_t rows, int64_t d, const void* A, int64_t lda,
                        slse_dtype a_t, double scale, slse_factor_method method, double* R,
                        int64_t ldr, double* M, int64_t ldm, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx && A && R, "null pointer");
    require(d >= 1 && rows >= d, "need rows >= d >= 1");
    require(d <= 512, "d > 512 is not supported by the factorization of this library");
    require(lda >= d && ldr >= d && (!M || ldm >= d), "leading dimension too small");
    require(a_t == SLSE_F32 || a_t == SLSE_F64, "A dtype must be F32 or F64");
    require(scale > 0 && std::isfinite(scale), "scale must be positive");
    require(method == SLSE_FACTOR_CHOL || method == SLSE_FACTOR_QR, "unknown method");
    DeviceGuard g(ctx->device);
    hipStream_t st = as_stream(stream);
    ctx->arena.grew = false;
    FactorBufs f = reserve_factor(ctx, rows, d, method);
    if (ctx->arena.grew) ctx->drop_graphs();
    ctx->pre.valid = false;
    launch_fill_i32(f.info, 0, 3, st);
    enqueue_factor(f, rows, (int)d, A, lda, a_t, scale, method, st, true);
    SLSE_HIP(hipMemcpy2DAsync(R, ldr * sizeof(double), f.R, d * sizeof(double), d * sizeof(double),
                              d, hipMemcpyDeviceToDevice, st));
    if (M)
      SLSE_HIP(hipMemcpy2DAsync(M, ldm * sizeof(double), f.M, d * sizeof(double),
                                d * sizeof(double), d, hipMemcpyDeviceToDevice, st));
    int info[3] = {0, 0, 0};
    SLSE_HIP(hipMemcpyAsync(info, f.info, sizeof(info), hipMemcpyDeviceToHost, st));
    SLSE_HIP(hipStreamSynchronize(st));
    if (info[0] || info[1] || info[2]) {
      set_last_error("factorization: non-positive or non-finite pivot at column " +
                     std::to_string((info[0] ? info[0] : info[1] ? info[1] : info[2]) - 1));
      return SLSE_ESINGULAR;
    }
    return SLSE_OK;
  });
}

slse_status slse_fused_resid_grad(slse_ctx* ctx, int64_t n, int64_t d, const void* X, int64_t ldx,
                                  const void* Y, slse_dtype storage, const double* beta,
                                  double scale, slse_dtype accum, double* g_out,
                                  double* rnorm2_out, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx && beta && g_out, "null pointer");
    require(n >= 0 && d >= 1 && d <= 1024, "need n >= 0 and 1 <= d <= 1024");
    require(n == 0 || X != nullptr, "null X");
    require(ldx >= d, "ldx < d");
    require(storage == SLSE_F32 || storage == SLSE_F64, "storage must be F32 or F64");
    require(accum == SLSE_F32 || accum == SLSE_F64, "accum must be F32 or F64");
    DeviceGuard g(ctx->device);
    hipStream_t st = as_stream(stream);
    ctx->arena.grew = false;
    IterBufs b = reserve_iter(ctx, d, "rg");
    if (ctx->arena.grew) ctx->drop_graphs();
    if (n > 0) tune_resid_grad(ctx, b, n, (int)d, storage, accum, X, ldx, Y, 1, st);
    const ResidGradPlan pl = rg_plan(ctx, b, n, (int)d, storage, accum, X, ldx);
    if (n == 0) {
      launch_fill_f64(g_out, 0.0, d, st);
      if (rnorm2_out) launch_fill_f64(rnorm2_out, 0.0, 1, st);
      return SLSE_OK;
    }
    ResidGradArgs a;
    a.n = n;
    a.d = (int)d;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.incy = 1;
    a.storage = storage;
    a.accum = accum;
    a.beta = beta;
    a.partial = b.partial;
    a.gpart = b.gpart;
    a.counters = b.counters;
    a.capacity_blocks = b.max_blocks;
    launch_resid_grad(pl, a, st);
    launch_finalize_grad(b.gpart, pl.groups, pl.ldp, (int)d, scale, g_out, rnorm2_out, st);
    return SLSE_OK;
  });
}

slse_status slse_fused_resid_grad_noalloc(slse_ctx* ctx, int64_t n, int64_t d, const void* X,
                                          int64_t ldx, const void* Y, slse_dtype storage,
                                          const double* beta, double scale, slse_dtype accum,
                                          double* g_out, double* rnorm2_out, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx && beta && g_out, "null pointer");
    require(n >= 0 && d >= 1, "need n >= 0 and d >= 1");
    if (d > kNoAllocMaxD)
      fail(SLSE_EINVAL, "d = " + std::to_string(d) + " exceeds the fixed scratch of the "
                        "allocation-free entry point (d <= " + std::to_string(kNoAllocMaxD) + ")");
    require(n == 0 || X != nullptr, "null X");
    require(ldx >= d, "ldx < d");
    require(storage == SLSE_F32 || storage == SLSE_F64, "storage must be F32 or F64");
    require(accum == SLSE_F32 || accum == SLSE_F64, "accum must be F32 or F64");
    require(ctx->device >= 0 && ctx->device < kNoAllocMaxDevices, "bad device");
    char* base = g_scratch_ptr[ctx->device];
    require(base != nullptr, "the fixed scratch of this device is not set up");
    DeviceGuard g(ctx->device);
    hipStream_t st = as_stream(stream);
    if (n == 0) {
      launch_fill_f64(g_out, 0.0, d, st);
      if (rnorm2_out) launch_fill_f64(rnorm2_out, 0.0, 1, st);
      return SLSE_OK;
    }
    // the launch shape of slse_fused_resid_grad (its tuned grid when known),
    // capped at the blocks the fixed scratch holds; no tuning here
    IterBufs b;
    b.max_blocks = kNoAllocBlocks;
    b.grid_blocks = std::min(kNoAllocBlocks, std::max(64, 2 * ctx->num_cus));
    const ResidGradPlan pl = rg_plan(ctx, b, n, (int)d, storage, accum, X, ldx);
    require(pl.blocks <= kNoAllocBlocks && pl.ldp <= kNoAllocLdp, "plan exceeds the fixed scratch");
    ResidGradArgs a;
    a.n = n;
    a.d = (int)d;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.incy = 1;
    a.storage = storage;
    a.accum = accum;
    a.beta = beta;
    a.counters = reinterpret_cast<int*>(base);
    a.gpart = reinterpret_cast<double*>(base + kNoAllocTicketBytes);
    a.partial = reinterpret_cast<double*>(base + kNoAllocTicketBytes + kNoAllocGpartBytes);
    a.capacity_blocks = kNoAllocBlocks;
    launch_resid_grad(pl, a, st);
    launch_finalize_grad(a.gpart, pl.groups, pl.ldp, (int)d, scale, g_out, rnorm2_out, st);
    return SLSE_OK;
  });
}

slse_status slse_solve(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                       double* beta_out, slse_report* rep, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr, "null ctx");
    DeviceGuard g(ctx->device);
    return solve_impl(ctx, p, q, beta_out, rep, as_stream(stream));
  });
}

slse_status slse_workspace_size(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                                size_t* bytes) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr && bytes != nullptr, "null ctx or bytes");
    *bytes = solve_workspace_bytes(ctx, p, q);
    return SLSE_OK;
  });
}

slse_status slse_solve_ws(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                          double* beta_out, slse_report* rep, void* ws, size_t ws_bytes,
                          void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr, "null ctx");
    require(ws != nullptr, "null workspace");
    const size_t need = solve_workspace_bytes(ctx, p, q);
    if (ws_bytes < need)
      fail(SLSE_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes, got " +
                            std::to_string(ws_bytes));
    DeviceGuard g(ctx->device);
    return solve_impl(ctx, p, q, beta_out, rep, as_stream(stream), ws, ws_bytes);
  });
}

slse_status slse_ihs(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                     double* beta_out, slse_report* rep, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr, "null ctx");
    DeviceGuard g(ctx->device);
    return ihs_impl(ctx, p, q, beta_out, rep, as_stream(stream));
  });
}

slse_status slse_paper_schedule(int64_t N, int64_t d, int64_t m1_factor, int64_t* m_out,
                                int32_t cap, int32_t* K_out) {
  return guarded([&]() -> slse_status {
    require(m_out && K_out, "null pointer");
    require(d >= 1 && N > d && m1_factor >= 1, "need N > d >= 1 and m1_factor >= 1");
    require(d <= (int64_t(1) << 40) / m1_factor, "m1_factor * d too large");
    // m_1: the power of 2 at or above m1_factor * d; m_K: the power of 2 at or below N / 2
    const int64_t m1 = int64_t(1) << ilog2_ceil(m1_factor * d);
    int64_t mk = 1;
    while (mk * 2 <= N / 2) mk *= 2;
    require(N / 2 >= 1 && m1 <= mk, "empty schedule: m_1 > N/2");
    int32_t K = 0;
    for (int64_t v = m1; v <= mk; v *= 2) {
      require(K < cap, "m_out too short for the schedule");
      m_out[K++] = v;
    }
    *K_out = K;
    return SLSE_OK;
  });
}

slse_status slse_paper_params(int64_t d, int64_t r_in, int64_t* r_out, double* mu, double* eta) {
  return guarded([&]() -> slse_status {
    require(r_out && mu && eta, "null pointer");
    require(d >= 1, "d < 1");
    const int64_t r = r_in > 0 ? r_in : 6 * d;
    require(r > d, "need r > d");
    const double e = (double)d / (double)r;
    *r_out = r;
    *eta = e;
    *mu = (1.0 - e) * (1.0 - e);
    return SLSE_OK;
  });
}

slse_status slse_stage1_counts(const int64_t* m, int32_t K, int64_t d, double omega, int32_t a1,
                               int32_t* a_out) {
  return guarded([&]() -> slse_status {
    require(m && a_out, "null pointer");
    require(K >= 1 && K <= SLSE_MAX_LEVELS, "need 1 <= K <= SLSE_MAX_LEVELS");
    require(omega > 0.0 && omega <= 1.0, "omega must lie in (0, 1]");
    std::vector<int32_t> a(K, 0);
    for (int i = 1; i < K; ++i) {
      require(m[i - 1] > d, "the bound needs m_{i-1} > d");
      const double ratio = std::sqrt((double)(m[i] - d) / (double)(m[i - 1] - d));
      const double target = ((1.0 + omega) * ratio + 1.0) / omega;
      int k = 1;
      while (std::pow(3.0, k) < target) ++k;
      a[i] = k;
    }
    a[0] = a1 >= 1 ? a1 : (K > 1 ? a[1] : 2);
    for (int i = 0; i < K; ++i) a_out[i] = a[i];
    return SLSE_OK;
  });
}

slse_status slse_backward(slse_ctx* ctx, const slse_problem* p, const slse_params* q,
                          const double* beta_hat, const double* w, int64_t incw, void* dX,
                          int64_t lddx, void* dY, slse_dtype grad_t, double* lambda_out,
                          slse_report* rep, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr, "null ctx");
    DeviceGuard g(ctx->device);
    return backward_impl(ctx, p, q, beta_hat, w, incw, dX, lddx, dY, grad_t, lambda_out, rep,
                         as_stream(stream));
  });
}

slse_status slse_solve_batched(slse_ctx* ctx, int32_t B, const slse_problem* ps,
                               const slse_params* qs, double* const* betas, slse_report* reps,
                               void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx != nullptr, "null ctx");
    require(B >= 0 && (B == 0 || (ps && qs && betas)), "bad batch arguments");
    if (B == 0) return SLSE_OK;
    DeviceGuard g(ctx->device);
    return batched_impl(ctx, B, ps, qs, betas, reps, as_stream(stream));
  });
}

slse_status slse_ctx_save_tuning(slse_ctx* ctx, const char* path) {
  return guarded([&]() -> slse_status {
    require(ctx && path, "null pointer");
    FILE* f = std::fopen(path, "w");
    if (!f) fail(SLSE_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "libslse-tuning 1 %s\n", ctx->arch.c_str());
    for (const auto& kv : ctx->rg_tune)
      std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.first, kv.second.second);
    const bool ok = std::fclose(f) == 0;
    if (!ok) fail(SLSE_EINVAL, std::string("cannot write ") + path);
    return SLSE_OK;
  });
}

slse_status slse_ctx_load_tuning(slse_ctx* ctx, const char* path, int32_t* loaded) {
  return guarded([&]() -> slse_status {
    require(ctx && path, "null pointer");
    if (loaded) *loaded = 0;
    FILE* f = std::fopen(path, "r");
    if (!f) fail(SLSE_EINVAL, std::string("cannot read ") + path);
    char head[64] = {0}, arch[128] = {0};
    int version = 0;
    const bool header = std::fscanf(f, "%63s %d %127s", head, &version, arch) == 3 &&
                        std::string(head) == "libslse-tuning" && version == 1;
    if (!header) {
      std::fclose(f);
      fail(SLSE_EINVAL, std::string("not a tuning file: ") + path);
    }
    int n = 0;
    if (ctx->arch == arch) {  // entries of another part or CU count are ignored
      char key[256];
      int a = 0, b = 0;
      while (std::fscanf(f, "%255s %d %d", key, &a, &b) == 3) {
        if (a > 0 && b > 0) {
          ctx->rg_tune[key] = {a, b};
          ++n;
        }
      }
    }
    std::fclose(f);
    if (loaded) *loaded = n;
    return SLSE_OK;
  });
}

slse_status slse_debug_stream(slse_ctx* ctx, int32_t what, uint64_t seed, int32_t stream_id,
                              int64_t aux, int64_t start, int64_t count, int64_t* out,
                              void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx && out, "null pointer");
    require(what >= 0 && what <= 7, "bad selector");
    require(count >= 0 && start >= 0, "bad range");
    if (what == 1 || what == 2) {
      require(aux >= 1 && aux <= 62, "permutation bits out of range");
      require(start + count <= (int64_t(1) << aux), "index outside the permutation domain");
    }
    if (what == 4 || what == 5) require(is_pow2(aux), "bucket count must be a power of 2");
    if (what == 6 || what == 7) require(aux >= 1, "bucket count must be positive");
    DeviceGuard g(ctx->device);
    launch_debug_stream(what, seed, stream_id, aux, start, count, out, as_stream(stream));
    return SLSE_OK;
  });
}

slse_status slse_debug_batch_tiles(int32_t B, const int64_t* n, const int64_t* row_bytes,
                                   const int64_t* step_rows, int64_t slots, int64_t min_tile_bytes,
                                   int32_t* tile_rows, int32_t* ntiles) {
  return guarded([&]() -> slse_status {
    require(B >= 0 && (B == 0 || (n && row_bytes && step_rows && tile_rows && ntiles)),
            "null pointer");
    for (int b = 0; b < B; ++b) require(n[b] >= 0 && row_bytes[b] > 0 && step_rows[b] > 0, "bad sizes");
    std::vector<int> tr(B), nt(B);
    split_step_tiles(B, n, row_bytes, step_rows, slots, min_tile_bytes, tr.data(), nt.data());
    for (int b = 0; b < B; ++b) {
      tile_rows[b] = tr[b];
      ntiles[b] = nt[b];
    }
    return SLSE_OK;
  });
}

slse_status slse_debug_bandwidth(slse_ctx* ctx, int32_t mode, const void* src, void* dst,
                                 int64_t bytes, int32_t blocks, void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx && src && dst, "null pointer");
    require(mode == 0 || mode == 1, "mode must be 0 (read) or 1 (copy)");
    require(bytes >= 0 && bytes % 16 == 0, "bytes must be a multiple of 16");
    require(reinterpret_cast<uintptr_t>(src) % 16 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0,
            "src and dst must be 16-byte aligned");
    const int nb = blocks > 0 ? blocks : ctx->num_cus;
    require(nb <= 65536, "too many blocks");
    DeviceGuard g(ctx->device);
    launch_stream_reference(mode, src, dst, bytes, nb, as_stream(stream));
    return SLSE_OK;
  });
}

slse_status slse_debug_batch_plan(int32_t B, const slse_problem* ps, const slse_params* qs,
                                  size_t* bytes_out) {
  return guarded([&]() -> slse_status {
    require(B >= 1 && ps && qs, "bad batch arguments");
    slse_ctx ctx;  // host-only: no device, no stream, the default CU count
    BorrowScope scope{ctx.arena};
    ctx.arena.begin_measure();
    // result pointers are only stored in the descriptors, never read here
    std::vector<double*> betas(B);
    for (int b = 0; b < B; ++b)
      betas[b] = reinterpret_cast<double*>((uintptr_t(1) << 36) + (uintptr_t)b * 4096);
    BatchPlan bp;
    (void)plan_batched(&ctx, B, ps, qs, betas.data(), bp);
    build_batch_tables(bp, ps, qs, betas.data());
    check_batch_plan(ctx.arena, bp, ps);
    if (bytes_out) *bytes_out = ctx.arena.ext_used;
    return SLSE_OK;
  });
}

slse_status slse_debug_gaussian(slse_ctx* ctx, uint64_t seed, int32_t stream_id, int32_t form,
                                int64_t k0, int64_t nk, int64_t j0, int64_t nj, double* out,
                                void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx && out, "null pointer");
    require(k0 >= 0 && j0 >= 0 && nk >= 0 && nj >= 0, "bad range");
    require(form == 0 || form == 1, "form must be 0 or 1");
    DeviceGuard g(ctx->device);
    launch_debug_gaussian(seed, (uint64_t)stream_id, k0, nk, j0, nj, form, out, as_stream(stream));
    return SLSE_OK;
  });
}

slse_status slse_debug_gaussian_generate(slse_ctx* ctx, uint64_t seed, int32_t stream_id,
                                        int64_t m, int64_t N, int32_t blocks, uint32_t* sink,
                                        void* stream) {
  return guarded([&]() -> slse_status {
    require(ctx && sink, "null pointer");
    require(m >= 1 && N >= 1 && blocks >= 1 && blocks <= 65536, "bad sizes");
    DeviceGuard g(ctx->device);
    launch_gauss_generate(seed, (uint64_t)stream_id, m, N, blocks, sink, as_stream(stream));
    return SLSE_OK;
  });
}

slse_status slse_debug_gaussian_plan(int64_t N, int64_t d, int64_t m, int32_t bf16,
                                     int32_t* splits) {
  return guarded([&]() -> slse_status {
    require(splits != nullptr, "null pointer");
    require(N >= 1 && d >= 1 && m >= 1, "bad sizes");
    GaussianArgs a;
    a.t = bf16 ? SLSE_F32 : SLSE_F64;
    a.N = N;
    a.d = (int)d;
    a.m = m;
    a.bf16 = bf16 != 0;
    gaussian_plan(a);
    *splits = a.splits;
    return SLSE_OK;
  });
}

}  // extern "C"
