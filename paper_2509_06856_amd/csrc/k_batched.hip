// Batched M-IHS steps for many independent regressions of uneven size (one
// launch per step for the whole batch instead of one per problem).
//
// Residual gradient: the rows of every active problem are cut into tiles (the
// tile height is chosen per step, smaller when few rows are active, so the
// grid stays busy); one flat list of (problem, tile) work items is walked by a
// persistent grid.  A block takes a tile, streams its rows with the problem's
// own lane-group width (as in the single-problem pass: a row split over
// `lpr` lanes, many rows in flight), reduces the tile's partial gradient in
// LDS and writes it to the problem's partial rows.  Tiles never share a
// partial row, so the result does not depend on which block ran which tile.
//
// Update: one block per problem sums its tile partials in tile order, applies
// M = H_hat^{-1} (GEMV) and takes the heavy-ball step of eqs. (98)/(99).
#include <algorithm>

#include "kernels.hpp"

namespace slse {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxD = 1024;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&v)[VEC]) {
  if constexpr (VEC == 1) {
    v[0] = __builtin_nontemporal_load(p);
  } else if constexpr (sizeof(T) == 4) {
    f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = x[i];
  } else {
    f64x2 x = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
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

__device__ __forceinline__ int find_problem(const int* __restrict__ prefix, int B, int tile) {
  int lo = 0, hi = B;  // prefix[lo] <= tile < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= tile)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename T, int VEC, int NCH>
__global__ __launch_bounds__(kThreads) void batched_resid_grad_kernel(
    const BatchStep* __restrict__ steps, const BatchProblem* __restrict__ probs,
    const int* __restrict__ prefix, int B, int total_tiles, double* __restrict__ pool) {
  // rows in flight per lane group: two with four chunks per lane (fewer
  // registers, measured faster than four), else four
  constexpr int UNROLL = NCH >= 4 ? 2 : 4;
  __shared__ double s_red[kWaves][kMaxD + 1];
  __shared__ int s_prefix[kPrefixLds + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // the tile prefix of this step, searched in LDS (global if the batch is large)
  const bool lds_prefix = B <= kPrefixLds;
  if (lds_prefix) {
    for (int i = threadIdx.x; i <= B; i += kThreads) s_prefix[i] = prefix[i];
    __syncthreads();
  }
  const int* pfx = lds_prefix ? s_prefix : prefix;
  for (int tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const int b = find_problem(pfx, B, tile);
    const BatchStep st = steps[b];
    const BatchProblem pr = probs[b];
    const int lt = tile - pfx[b];
    const int d = pr.d;
    const int lpr = pr.lpr;
    const int gpw = 64 / lpr;
    const int grp = lane / lpr;
    const int l = lane - grp * lpr;
    const T* X = static_cast<const T*>(st.X);
    const T* Y = static_cast<const T*>(st.Y);
    const double* beta = st.beta;
    double bv[NCH][VEC];
    bool full[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int col0 = (c * lpr + l) * VEC;
      full[c] = col0 + VEC <= d;
#pragma unroll
      for (int v = 0; v < VEC; ++v) bv[c][v] = (col0 + v < d) ? beta[col0 + v] : 0.0;
    }
    double acc[NCH][VEC];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[c][v] = 0.0;
    double rr = 0.0;
    const int64_t r0 = (int64_t)lt * st.tile_rows;
    const int64_t r1 = min(st.n, r0 + st.tile_rows);
    const int rs = kWaves * gpw;
    for (int64_t base = r0 + wave * gpw + grp; base < r1; base += (int64_t)rs * UNROLL) {
      T x[UNROLL][NCH][VEC];
      T y[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int64_t row = base + (int64_t)u * rs;
        const bool ok = row < r1;
        const T* xr = X + (ok ? row : r0) * st.ldx;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int col0 = (c * lpr + l) * VEC;
          if (ok && full[c]) {
            load_vec<T, VEC>(xr + col0, x[u][c]);
          } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) x[u][c][v] = (ok && col0 + v < d) ? xr[col0 + v] : (T)0;
          }
        }
        y[u] = ok ? Y[(ok ? row : r0) * st.incy] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        double dot = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
          for (int v = 0; v < VEC; ++v) dot = fma((double)x[u][c][v], bv[c][v], dot);
        dot = lane_group_sum(dot, lpr);
        const double r = (double)y[u] - dot;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[c][v] = fma(r, widen_f64(x[u][c][v]), acc[c][v]);
        rr = fma(r, r, rr);
      }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        double t = acc[c][v];
        for (int m = lpr; m < 64; m <<= 1) t += wave_xor(t, m);
        acc[c][v] = t;
      }
    rr = (l == 0) ? rr : 0.0;
    for (int m = 1; m < 64; m <<= 1) rr += wave_xor(rr, m);
    __syncthreads();  // s_red of the previous tile is consumed
    if (grp == 0) {
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int col = (c * lpr + l) * VEC + v;
          if (col < d) s_red[wave][col] = acc[c][v];
        }
      if (l == 0) s_red[wave][d] = rr;
    }
    __syncthreads();
    double* prow = pool + pr.part_off + (int64_t)lt * (d + 1);
    for (int col = threadIdx.x; col <= d; col += kThreads) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += s_red[w][col];
      prow[col] = t;
    }
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
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(j + u * nq) * (d + 1) + k];
#pragma unroll
        for (int u = 0; u < 8; ++u) t += v[u];
      }
      for (; j < ntiles; j += nq) t += part[(int64_t)j * (d + 1) + k];
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
        if (i0 + u < row_hi) p[u] = fma(pr.M[(int64_t)(i0 + u) * d + k], gk, p[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      for (int m = 32; m > 0; m >>= 1) p[u] += wave_xor(p[u], m);
    if (lane < 4 && i0 + lane < row_hi) {
      const int i = i0 + lane;
      const double pi = lane == 0 ? p[0] : lane == 1 ? p[1] : lane == 2 ? p[2] : p[3];
      const double bi = st.beta[i];
      const double bn = bi + pr.mu * pi + pr.eta * (bi - st.beta_prev[i]);
      st.beta_next[i] = bn;
      pr.beta_out[i] = bn;
      bad |= !isfinite(bn);
    }
  }
  if (bad && flags) atomicExch(flags + b, 1);
}

__global__ void batched_init_kernel(const BatchProblem* __restrict__ probs) {
  const BatchProblem pr = probs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pr.d) return;
  const double v = pr.beta0 ? pr.beta0[i] : 0.0;
  if (pr.beta_init) pr.beta_init[i] = v;
  pr.beta_out[i] = v;
}

template <typename T, int VEC>
void launch_rg(const BatchStep* steps, const BatchProblem* probs, const int* prefix, int B,
               int total, int grid, double* pool, int nch, hipStream_t s) {
  switch (nch) {
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
                               slse_dtype t, bool vec, int nch, hipStream_t s) {
  if (total_tiles <= 0) return;
  grid = std::max(1, std::min(grid, total_tiles));
  if (t == SLSE_F32) {
    if (vec)
      launch_rg<float, 4>(steps, probs, prefix, B, total_tiles, grid, pool, nch, s);
    else
      launch_rg<float, 1>(steps, probs, prefix, B, total_tiles, grid, pool, nch, s);
  } else {
    if (vec)
      launch_rg<double, 2>(steps, probs, prefix, B, total_tiles, grid, pool, nch, s);
    else
      launch_rg<double, 1>(steps, probs, prefix, B, total_tiles, grid, pool, nch, s);
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
