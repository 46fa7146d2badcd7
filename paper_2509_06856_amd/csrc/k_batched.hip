// Batched M-IHS steps for many independent regressions of uneven size (one
// launch per step for the whole batch instead of one per problem).
//
// Residual gradient: the bytes of [X|Y] a step reads are cut into tiles of
// about equal size (grid x items tiles, shared out over the active problems;
// a problem's rows split evenly over its tiles); one flat list of (problem,
// tile) work items is walked by a persistent grid.  A block takes a tile and
// streams its rows with the problem's own lane groups (a row split over `lpr`
// lanes, one to four 16-byte vectors per lane, several rows in flight),
// reduces the tile's partial gradient in LDS and writes it to the tile's own
// partial row, so the result does not depend on which block ran which tile.
//
// Update: blocks per (problem, 64 rows) sum the problem's tile partials in a
// fixed order, apply M = H_hat^{-1} (GEMV) and take the heavy-ball step of
// eqs. (98)/(99).
#include <algorithm>

#include "kernels.hpp"

namespace slse {
namespace {

constexpr int kThreads = kBatchThreads;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxD = 1024;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// [X|Y] rows live in global memory: loads through global (address space 1)
// pointers, not flat ones (the descriptors holding the pointers come from
// memory, so the compiler cannot infer it)
template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T* p, T (&v)[VEC]) {
  if constexpr (VEC == 1) {
    v[0] = __builtin_nontemporal_load(gptr(p));
  } else if constexpr (sizeof(T) == 4) {
    f32x4 x = __builtin_nontemporal_load((const SLSE_GLOBAL f32x4*)p);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = x[i];
  } else {
    f64x2 x = __builtin_nontemporal_load((const SLSE_GLOBAL f64x2*)p);
    v[0] = x[0];
    v[1] = x[1];
  }
}

// FP32 -> FP64 as an instruction the compiler cannot merge with an earlier
// conversion of the same value, so widened rows are not kept alive from a
// row's dot to its gradient update (that would double the registers held)
template <typename T>
__device__ __forceinline__ double widen_f64(T x) {
  if constexpr (sizeof(T) == 4) {
    double r;
    asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
  } else {
    return (double)x;
  }
}

constexpr int kPrefixLds = 512;  // problems whose tile prefix is searched in LDS
constexpr int kSlots = kBatchSlots;

// the problem b with prefix[b] <= tile < prefix[b + 1]; *first = prefix[b]
// (prefix[0] = 0)
template <typename P>
__device__ __forceinline__ int find_problem(P prefix, int B, int tile, int* first) {
  int lo = 0, hi = B, vlo = 0;  // prefix[lo] = vlo <= tile < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    const int v = prefix[mid];
    if (v <= tile) {
      lo = mid;
      vlo = v;
    } else {
      hi = mid;
    }
  }
  *first = vlo;
  return lo;
}

// Rows of one tile: lane group `grp` of `lpr` lanes covers a row with CH
// vectors per lane (vector k*lpr + l), so every load instruction of a wave
// reads gpw consecutive rows as one contiguous range; a lane keeps kSlots
// vectors in flight, i.e. kSlots / CH rows.  The tile's partial gradient is
// reduced over the lane groups, then over the waves in LDS, and written to
// the tile's own partial row.

// RU rows per lane group: the dots (row by row, so that the widened values
// of a row die with its dot), the lane-group sums of all RU dots interleaved,
// then the residuals and the gradient update
template <typename T, int VEC, int CH, int RU>
__device__ __forceinline__ void rows_update(const T (&x)[RU][CH][VEC], const T (&y)[RU],
                                            const double (&bv)[CH][VEC], int lpr,
                                            double (&acc)[CH][VEC], double& rr) {
  double dot[RU];
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    __builtin_amdgcn_sched_barrier(0);
    double p = 0.0;
#pragma unroll
    for (int k = 0; k < CH; ++k)
#pragma unroll
      for (int v = 0; v < VEC; ++v) p = fma((double)x[u][k][v], bv[k][v], p);
    dot[u] = p;
  }
  __builtin_amdgcn_sched_barrier(0);
  for (int m = lpr >> 1; m > 0; m >>= 1) {
    double o[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) o[u] = wave_xor(dot[u], m);
#pragma unroll
    for (int u = 0; u < RU; ++u) dot[u] += o[u];
  }
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    const double r = (double)y[u] - dot[u];
#pragma unroll
    for (int k = 0; k < CH; ++k)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[k][v] = fma(r, widen_f64(x[u][k][v]), acc[k][v]);
    rr = fma(r, r, rr);
  }
}

template <typename T, int VEC, int CH>
__device__ __forceinline__ void batched_tile(const BatchStep& st, int d, int lpr, int lt,
                                             double* __restrict__ prow,
                                             double (*s_red)[kMaxD + 1]) {
  constexpr int RU = kSlots / CH;         // rows per lane group in flight
  constexpr int RG = RU < 2 ? RU : 2;     // the same in the guarded loop
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gpw = 64 / lpr;
  const int grp = lane / lpr;
  const int l = lane - grp * lpr;
  const T* X = static_cast<const T*>(st.X);
  const T* Y = static_cast<const T*>(st.Y);
  const double* beta = st.beta;
  double bv[CH][VEC];
  bool full[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int col0 = (k * lpr + l) * VEC;
    full[k] = col0 + VEC <= d;
#pragma unroll
    for (int v = 0; v < VEC; ++v) bv[k][v] = (col0 + v < d) ? gptr(beta)[col0 + v] : 0.0;
  }
  double acc[CH][VEC];
#pragma unroll
  for (int k = 0; k < CH; ++k)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[k][v] = 0.0;
  double rr = 0.0;
  const int64_t r0 = (int64_t)lt * st.tile_rows;
  const int64_t r1 = min(st.n, r0 + st.tile_rows);
  const int rs = kWaves * gpw;
  int64_t base = r0 + wave * gpw + grp;
  if (lpr * CH * VEC == d) {
    // every lane's vectors lie inside the row: while all RU rows of every
    // lane group of the wave are in range (a wave-uniform test), no guards
    // (row pointers advance by uniform strides: no per-row 64-bit products)
    const int64_t last = (int64_t)(gpw - 1) + (int64_t)(RU - 1) * rs;
    const int64_t xs = (int64_t)rs * st.ldx;   // between a group's rows in flight
    const int64_t ys = (int64_t)rs * st.incy;
    int64_t wb = r0 + wave * gpw;
    const T* xp = X + (wb + grp) * st.ldx + l * VEC;
    const T* yp = Y + (wb + grp) * st.incy;
    for (; wb + last < r1; wb += (int64_t)rs * RU, xp += RU * xs, yp += RU * ys) {
      T x[RU][CH][VEC];
      T y[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
#pragma unroll
        for (int k = 0; k < CH; ++k) load_vec<T, VEC>(xp + u * xs + k * lpr * VEC, x[u][k]);
        y[u] = __builtin_nontemporal_load(gptr(yp + u * ys));
      }
      rows_update<T, VEC, CH, RU>(x, y, bv, lpr, acc, rr);
    }
    base = wb + grp;
  }
  // guarded rows: the rest of the tile, or all of it when a lane's vectors
  // may pass the end of the row
  for (; base < r1; base += (int64_t)rs * RG) {
    T x[RG][CH][VEC];
    T y[RG];
#pragma unroll
    for (int u = 0; u < RG; ++u) {
      const int64_t row = base + (int64_t)u * rs;
      const bool ok = row < r1;
      const T* xr = X + (ok ? row : r0) * st.ldx;
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int col0 = (k * lpr + l) * VEC;
        if (ok && full[k]) {
          load_vec<T, VEC>(xr + col0, x[u][k]);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) x[u][k][v] = (ok && col0 + v < d) ? gptr(xr)[col0 + v] : (T)0;
        }
      }
      y[u] = ok ? gptr(Y)[(ok ? row : r0) * st.incy] : (T)0;
    }
    rows_update<T, VEC, CH, RG>(x, y, bv, lpr, acc, rr);
  }
#pragma unroll
  for (int k = 0; k < CH; ++k)
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      double t = acc[k][v];
      for (int m = lpr; m < 64; m <<= 1) t += wave_xor(t, m);
      acc[k][v] = t;
    }
  rr = (l == 0) ? rr : 0.0;
  for (int m = 1; m < 64; m <<= 1) rr += wave_xor(rr, m);
  __syncthreads();  // s_red of the previous tile is consumed
  if (grp == 0) {
#pragma unroll
    for (int k = 0; k < CH; ++k)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int col = (k * lpr + l) * VEC + v;
        if (col < d) s_red[wave][col] = acc[k][v];
      }
    if (l == 0) s_red[wave][d] = rr;
  }
  __syncthreads();
  for (int col = threadIdx.x; col <= d; col += kThreads) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += s_red[w][col];
    gptr(prow)[col] = t;
  }
}

// Persistent grid over the step's (problem, tile) items; CHMAX is the most
// vectors per lane of any problem's row in the batch.
template <typename T, int VEC, int CHMAX>
__global__ __launch_bounds__(kThreads) void batched_resid_grad_kernel(
    const BatchStep* __restrict__ steps, const BatchProblem* __restrict__ probs,
    const int* __restrict__ prefix, int B, int total_tiles, double* __restrict__ pool) {
  __shared__ double s_red[kWaves][kMaxD + 1];
  __shared__ int s_prefix[kPrefixLds + 1];
  // the tile prefix of this step, searched in LDS (global if the batch is large)
  const bool lds_prefix = B <= kPrefixLds;
  if (lds_prefix) {
    for (int i = threadIdx.x; i <= B; i += kThreads) s_prefix[i] = prefix[i];
    __syncthreads();
  }
  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    // the problem and tile are block-uniform: in scalar registers, the step
    // and problem descriptors come in through scalar loads (the LDS and the
    // global search are kept apart so that neither becomes a flat access)
    int first;
    const int b = __builtin_amdgcn_readfirstlane(lds_prefix ? find_problem(s_prefix, B, tile, &first)
                                                            : find_problem(prefix, B, tile, &first));
    const BatchStep st = steps[b];
    const BatchProblem pr = probs[b];
    const int lt = __builtin_amdgcn_readfirstlane(tile - first);
    double* prow = pool + pr.part_off + (int64_t)lt * (pr.d + 1);
    if (CHMAX >= 4 && pr.ch == 4)
      batched_tile<T, VEC, (CHMAX >= 4 ? 4 : 1)>(st, pr.d, pr.lpr, lt, prow, s_red);
    else if (CHMAX >= 2 && pr.ch == 2)
      batched_tile<T, VEC, (CHMAX >= 2 ? 2 : 1)>(st, pr.d, pr.lpr, lt, prow, s_red);
    else
      batched_tile<T, VEC, 1>(st, pr.d, pr.lpr, lt, prow, s_red);
  }
}

// Blocks (problem, 64-row block): g = scale * sum_tiles partial (every block of
// a problem forms all of g), p = M g for the block's rows,
// beta' = beta + mu p + eta (beta - beta_prev) on those rows.  The tile sum is
// split over (column, tile residue class) pairs and the classes are combined
// in a fixed order, so the result does not depend on timing; the GEMV runs
// four rows per wave at once so that their loads overlap.
constexpr int kUpdThreads = 1024;
constexpr int kUpdWaves = kUpdThreads / 64;
constexpr int kUpdRows = 4 * kUpdWaves;  // rows of p = M g per block (blockIdx.y)

__global__ __launch_bounds__(kUpdThreads) void batched_update_kernel(
    const BatchStep* __restrict__ steps, const BatchProblem* __restrict__ probs,
    const double* __restrict__ pool, int* __restrict__ flags) {
  __shared__ double s_g[kMaxD];
  __shared__ double s_part[kUpdThreads];
  const int b = blockIdx.x;
  const BatchStep st = steps[b];
  if (st.n <= 0) return;  // this problem has finished its schedule
  const BatchProblem pr = probs[b];
  const int d = pr.d;
  const int row_lo = blockIdx.y * kUpdRows;  // this block's rows of p and beta
  if (row_lo >= d) return;
  const int row_hi = min(d, row_lo + kUpdRows);
  const int ntiles = st.ntiles;
  const double* part = pool + pr.part_off;
  // classes of tiles per column: nq = 1024 / d rounded down to a power of 2
  int nq = 1;
  while (nq * 2 * d <= kUpdThreads) nq *= 2;
  {
    const int k = threadIdx.x % d;
    const int q = threadIdx.x / d;
    if (q < nq) {
      double t = 0.0;
      int j = q;
      for (; j + 7 * nq < ntiles; j += 8 * nq) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = gptr(part)[(int64_t)(j + u * nq) * (d + 1) + k];
#pragma unroll
        for (int u = 0; u < 8; ++u) t += v[u];
      }
      for (; j < ntiles; j += nq) t += gptr(part)[(int64_t)j * (d + 1) + k];
      s_part[q * d + k] = t;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < d; k += kUpdThreads) {
    double t = 0.0;
    for (int q = 0; q < nq; ++q) t += s_part[q * d + k];
    s_g[k] = st.scale * t;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  bool bad = false;
  for (int i0 = row_lo + 4 * wave; i0 < row_hi; i0 += 4 * kUpdWaves) {
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = lane; k < d; k += 64) {
      const double gk = s_g[k];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u < row_hi) p[u] = fma(gptr(pr.M)[(int64_t)(i0 + u) * d + k], gk, p[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      for (int m = 32; m > 0; m >>= 1) p[u] += wave_xor(p[u], m);
    if (lane < 4 && i0 + lane < row_hi) {
      const int i = i0 + lane;
      const double pi = lane == 0 ? p[0] : lane == 1 ? p[1] : lane == 2 ? p[2] : p[3];
      const double bi = gptr(st.beta)[i];
      const double bn = bi + pr.mu * pi + pr.eta * (bi - gptr(st.beta_prev)[i]);
      *gptr(st.beta_next + i) = bn;
      *gptr(pr.beta_out + i) = bn;
      bad |= !isfinite(bn);
    }
  }
  if (bad && flags) atomicExch(flags + b, 1);
}

__global__ void batched_init_kernel(const BatchProblem* __restrict__ probs) {
  const BatchProblem pr = probs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pr.d) return;
  const double v = pr.beta0 ? gptr(pr.beta0)[i] : 0.0;
  if (pr.beta_init) *gptr(pr.beta_init + i) = v;
  *gptr(pr.beta_out + i) = v;
}

template <typename T, int VEC>
void launch_rg(const BatchStep* steps, const BatchProblem* probs, const int* prefix, int B,
               int total, int grid, double* pool, int chmax, hipStream_t s) {
  switch (chmax) {
    case 1:
      batched_resid_grad_kernel<T, VEC, 1><<<grid, kThreads, 0, s>>>(steps, probs, prefix, B, total,
                                                                      pool);
      break;
    case 2:
      batched_resid_grad_kernel<T, VEC, 2><<<grid, kThreads, 0, s>>>(steps, probs, prefix, B, total,
                                                                      pool);
      break;
    default:
      batched_resid_grad_kernel<T, VEC, 4><<<grid, kThreads, 0, s>>>(steps, probs, prefix, B, total,
                                                                      pool);
      break;
  }
}

}  // namespace

void launch_batched_resid_grad(const BatchStep* steps, const BatchProblem* probs, const int* prefix,
                               int B, int total_tiles, int grid, double* pool,
                               slse_dtype t, bool vec, int chmax, hipStream_t s) {
  if (total_tiles <= 0) return;
  grid = std::max(1, std::min(grid, total_tiles));
  if (t == SLSE_F32) {
    if (vec)
      launch_rg<float, 4>(steps, probs, prefix, B, total_tiles, grid, pool, chmax, s);
    else
      launch_rg<float, 1>(steps, probs, prefix, B, total_tiles, grid, pool, chmax, s);
  } else {
    if (vec)
      launch_rg<double, 2>(steps, probs, prefix, B, total_tiles, grid, pool, chmax, s);
    else
      launch_rg<double, 1>(steps, probs, prefix, B, total_tiles, grid, pool, chmax, s);
  }
  SLSE_LAUNCH_CHECK();
}

void launch_batched_init(const BatchProblem* probs, int B, int dmax, hipStream_t s) {
  if (B <= 0 || dmax <= 0) return;
  batched_init_kernel<<<dim3((unsigned)ceil_div(dmax, 256), (unsigned)B), 256, 0, s>>>(probs);
  SLSE_LAUNCH_CHECK();
}

void launch_batched_update(const BatchStep* steps, const BatchProblem* probs, int B, int dmax,
                           const double* pool, int* flags, hipStream_t s) {
  if (B <= 0 || dmax <= 0) return;
  const dim3 grid((unsigned)B, (unsigned)ceil_div(dmax, kUpdRows));
  batched_update_kernel<<<grid, kUpdThreads, 0, s>>>(steps, probs, pool, flags);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
