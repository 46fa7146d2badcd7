// CountSketch and Gaussian sketches of [X|Y] (Sec. 1.2; CountSketch as the
// alternative sketching matrix of Sec. 5.4).
//
// CountSketch: column j of S_K has the single entry s(j) in row h(j), so
// S_K [X|Y] adds s(j) [x_j | y_j] into bucket h(j).  One lane group per row
// reads the row once and scatters it with float atomics into the largest
// level (m_K buckets) and into the Hessian sketch (r buckets).  Smaller levels
// use the bucket h(j) mod m_i, so level i is level i+1 folded in halves:
// A_i[k] = sum_{t = k mod m_i} A_{i+1}[t].  Sums land in an order set by the
// atomics: results agree with any other order to rounding, not bit for bit.
//
// Gaussian: A = G [X|Y] with G_kj iid N(0, 1) drawn on the fly (Philox block
// (j, k >> 3) -> four Box-Muller pairs).  Tiled 64 (sketch rows) x 64
// (columns) per block with the N rows split over blocks; partial tiles are
// summed in split order by a second kernel.  FP64 data accumulates in FP64,
// FP32 data in FP32.
#include <algorithm>

#include "kernels.hpp"
#include "rng.hpp"

namespace slse {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t n = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, c = e % cols;
    p[i * ld + c] = (T)0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void cs_scatter_kernel(int64_t n, int d, const T* __restrict__ X,
                                                              int64_t ldx, const T* __restrict__ Y,
                                                              uint64_t seed, uint64_t mK_mask,
                                                              T* __restrict__ AK, int64_t lda,
                                                              int64_t r, T* __restrict__ Ahat,
                                                              int64_t ldah, int lpr) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gpw = 64 / lpr;
  const int grp = lane / lpr;
  const int l = lane - grp * lpr;
  const int64_t stride = (int64_t)gridDim.x * kWaves * gpw;
  for (int64_t row = ((int64_t)blockIdx.x * kWaves + wave) * gpw + grp; row < n; row += stride) {
    uint64_t h, hh;
    int sg, sh;
    rng::cs_hash(seed, (uint64_t)row, mK_mask, h, sg);
    rng::cs_hash_hat(seed, (uint64_t)row, (uint64_t)r, hh, sh);
    T* a = AK + (int64_t)h * lda;
    T* b = Ahat + (int64_t)hh * ldah;
    for (int col = l; col <= d; col += lpr) {
      const T v = col < d ? X[row * ldx + col] : Y[row];
      atomicAdd(a + col, sg > 0 ? v : -v);
      atomicAdd(b + col, sh > 0 ? v : -v);
    }
  }
}

// dst[k][c] = sum_{q < ratio} src[k + q*m][c], k < m
template <typename T>
__global__ void cs_fold_kernel(const T* __restrict__ src, T* __restrict__ dst, int64_t m, int ratio,
                               int cols, int64_t ld) {
  const int64_t n = m * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / cols;
    const int c = (int)(e % cols);
    T t = 0;
    for (int q = 0; q < ratio; ++q) t += src[(k + q * m) * ld + c];
    dst[k * ld + c] = t;
  }
}

// ---------------------------------------------------------------------------
// Gaussian entries: u = (w32 + 1/2) 2^-32, z = sqrt(-2 ln u1) (cos | sin)(2 pi u2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void box_muller8(uint64_t seed, uint64_t stream, uint64_t j,
                                            uint64_t kblk, float (&z)[8]) {
  const rng::Words w = rng::philox(j, kblk, 0, 0, seed, stream);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (uint32_t)(w.w[q] & 0xffffffffu);
    const uint32_t hi = (uint32_t)(w.w[q] >> 32);
    const float u1 = fmaf((float)lo, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
    const float u2 = fmaf((float)hi, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
    const float rad = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincosf(6.283185307179586f * u2, &sn, &cs);
    z[2 * q] = rad * cs;
    z[2 * q + 1] = rad * sn;
  }
}

constexpr int kGT = 64;   // tile (sketch rows and columns)
constexpr int kGK = 16;   // data rows per step

template <typename T, typename Acc>
__global__ __launch_bounds__(kThreads) void gauss_kernel(int64_t N, int d, const T* __restrict__ X,
                                                         int64_t ldx, const T* __restrict__ Y,
                                                         uint64_t seed, uint64_t stream, int64_t m,
                                                         int splits, Acc* __restrict__ part,
                                                         int64_t ldp) {
  __shared__ Acc Gs[kGK][kGT + 1];
  __shared__ Acc Ws[kGK][kGT + 1];
  const int tx = threadIdx.x % 16;
  const int ty = threadIdx.x / 16;
  const int64_t k0 = (int64_t)blockIdx.y * kGT;  // sketch rows
  const int c0 = blockIdx.x * kGT;               // columns of [X|Y]
  const int split = blockIdx.z;
  const int64_t per = ceil_div(N, (int64_t)splits);
  const int64_t j_begin = split * per;
  const int64_t j_end = min(N, j_begin + per);
  Acc acc[4][4] = {};
  for (int64_t j0 = j_begin; j0 < j_end; j0 += kGK) {
    // G tile: kGT rows x kGK data rows = 8 row blocks x 16 columns of Philox blocks
    if (threadIdx.x < (kGT / 8) * kGK) {
      const int kb = threadIdx.x / kGK;  // which group of 8 sketch rows
      const int jj = threadIdx.x % kGK;
      const int64_t j = j0 + jj;
      float z[8];
      if (j < j_end) {
        box_muller8(seed, stream, (uint64_t)j, (uint64_t)((k0 >> 3) + kb), z);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) z[q] = 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) Gs[jj][kb * 8 + q] = (Acc)z[q];
    }
    for (int e = threadIdx.x; e < kGK * kGT; e += kThreads) {
      const int jj = e / kGT, cc = e % kGT;
      const int64_t j = j0 + jj;
      const int col = c0 + cc;
      Acc v = 0;
      if (j < j_end) {
        if (col < d)
          v = (Acc)X[j * ldx + col];
        else if (col == d)
          v = (Acc)Y[j];
      }
      Ws[jj][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < kGK; ++jj) {
      Acc a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Gs[jj][ty + 16 * u];
        b[u] = Ws[jj][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t k = k0 + ty + 16 * u;
      const int col = c0 + tx + 16 * v;
      if (k < m && col <= d) part[((int64_t)split * m + k) * ldp + col] = acc[u][v];
    }
}

template <typename T, typename Acc>
__global__ void gauss_reduce_kernel(const Acc* __restrict__ part, int splits, int64_t m, int cols,
                                    int64_t ldp, T* __restrict__ A, int64_t lda) {
  const int64_t n = m * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / cols;
    const int c = (int)(e % cols);
    Acc t = 0;
    for (int s = 0; s < splits; ++s) t += part[((int64_t)s * m + k) * ldp + c];
    A[k * lda + c] = (T)t;
  }
}

// ---------------------------------------------------------------------------
// Gaussian sketch on the matrix cores: G and [X|Y] rounded to BF16 (nearest
// even), products accumulated in FP32 by v_mfma_f32_32x32x16_bf16.  Block
// tile 128 sketch rows x 128 columns, one wave per 32 rows, four 32 x 32
// accumulators per wave; 16 data rows per step, G generated into LDS by the
// block (one Philox block per thread per step), [X|Y] staged transposed so
// that every lane reads its 8 consecutive k as one 16-byte load.
// Lane layout (checked by an in-bounds probe): lane l holds A[l%32][8(l/32)+j]
// and B[8(l/32)+j][l%32], j < 8; accumulator r of lane l is
// C[(r%4) + 8(r/4) + 4(l/32)][l%32].
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kMT = 128;  // sketch rows per block
constexpr int kNT = 128;  // columns per block
constexpr int kKT = 16;   // data rows per step
constexpr int kKP = kKT + 8;  // padded LDS row (bf16 elements)

__device__ __forceinline__ __bf16 to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  return __builtin_bit_cast(__bf16, (uint16_t)u);
}

template <typename T>
__global__ __launch_bounds__(256) void gauss_mfma_kernel(int64_t N, int d, const T* __restrict__ X,
                                                         int64_t ldx, const T* __restrict__ Y,
                                                         uint64_t seed, uint64_t stream, int64_t m,
                                                         int splits, float* __restrict__ part,
                                                         int64_t ldp) {
  __shared__ __attribute__((aligned(16))) __bf16 Gs[kMT][kKP];
  __shared__ __attribute__((aligned(16))) __bf16 Ws[kNT][kKP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t k0 = (int64_t)blockIdx.y * kMT;
  const int c0 = blockIdx.x * kNT;
  const int split = blockIdx.z;
  const int64_t per = round_up(ceil_div(N, (int64_t)splits), kKT);
  const int64_t j_begin = (int64_t)split * per;
  const int64_t j_end = min(N, j_begin + per);
  f32x16_t acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  for (int64_t j0 = j_begin; j0 < j_end; j0 += kKT) {
    {  // G tile: thread -> (row block of 8, data row)
      const int kb = threadIdx.x / kKT;  // 0..15
      const int jj = threadIdx.x % kKT;
      const int64_t j = j0 + jj;
      float z[8];
      if (j < j_end) {
        box_muller8(seed, stream, (uint64_t)j, (uint64_t)((k0 >> 3) + kb), z);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) z[q] = 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) Gs[kb * 8 + q][jj] = to_bf16_rne(z[q]);
    }
    for (int e = threadIdx.x; e < kKT * kNT; e += 256) {  // [X|Y] tile, stored transposed
      const int jj = e / kNT, cc = e % kNT;
      const int64_t j = j0 + jj;
      const int col = c0 + cc;
      float v = 0.0f;
      if (j < j_end) {
        if (col < d)
          v = (float)X[j * ldx + col];
        else if (col == d)
          v = (float)Y[j];
      }
      Ws[cc][jj] = to_bf16_rne(v);
    }
    __syncthreads();
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&Gs[wave * 32 + (lane & 31)][8 * (lane >> 5)]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(&Ws[q * 32 + (lane & 31)][8 * (lane >> 5)]);
      acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[q], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t k = k0 + wave * 32 + (r % 4) + 8 * (r / 4) + 4 * (lane >> 5);
      const int col = c0 + q * 32 + (lane & 31);
      if (k < m && col <= d) part[((int64_t)split * m + k) * ldp + col] = acc[q][r];
    }
}

__global__ void debug_gauss_kernel(uint64_t seed, uint64_t stream, int64_t k0, int64_t nk,
                                   int64_t j0, int64_t nj, double* __restrict__ out) {
  const int64_t n = nk * nj;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / nj, b = e % nj;
    const int64_t k = k0 + a, j = j0 + b;
    float z[8];
    box_muller8(seed, stream, (uint64_t)j, (uint64_t)(k >> 3), z);
    out[e] = (double)z[k & 7];
  }
}

int grid1(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 8192)); }

template <typename T>
void countsketch_t(const CountSketchArgs& a, hipStream_t s) {
  T* A = static_cast<T*>(a.A);
  T* Ah = static_cast<T*>(a.Ahat);
  int64_t rows_A = 0;
  for (int i = 0; i < a.K; ++i) rows_A += a.m[i];
  fill_kernel<T><<<grid1(rows_A * (a.d + 1)), 256, 0, s>>>(A, rows_A, a.d + 1, a.lda);
  fill_kernel<T><<<grid1(a.r * (a.d + 1)), 256, 0, s>>>(Ah, a.r, a.d + 1, a.ldah);
  SLSE_LAUNCH_CHECK();
  const int64_t offK = rows_A - a.m[a.K - 1];
  int lpr = 1;
  while (lpr < 64 && lpr * 4 <= a.d + 1) lpr *= 2;
  const int rows_per_block = kWaves * (64 / lpr);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(a.N, rows_per_block), 8192));
  cs_scatter_kernel<T><<<blocks, kThreads, 0, s>>>(a.N, a.d, static_cast<const T*>(a.X), a.ldx,
                                                   static_cast<const T*>(a.Y), a.seed,
                                                   (uint64_t)a.m[a.K - 1] - 1, A + offK * a.lda,
                                                   a.lda, a.r, Ah, a.ldah, lpr);
  SLSE_LAUNCH_CHECK();
  int64_t off_hi = offK;
  for (int i = a.K - 2; i >= 0; --i) {
    const int64_t off_lo = off_hi - a.m[i];
    const int ratio = (int)(a.m[i + 1] / a.m[i]);
    cs_fold_kernel<T><<<grid1(a.m[i] * (a.d + 1)), 256, 0, s>>>(
        A + off_hi * a.lda, A + off_lo * a.lda, a.m[i], ratio, a.d + 1, a.lda);
    SLSE_LAUNCH_CHECK();
    off_hi = off_lo;
  }
}

template <typename T>
void gaussian_mfma_t(const GaussianArgs& a, hipStream_t s) {
  const int cols = a.d + 1;
  const int64_t ldp = round_up(cols, 4);
  dim3 grid((unsigned)ceil_div(cols, kNT), (unsigned)ceil_div(a.m, kMT), (unsigned)a.splits);
  gauss_mfma_kernel<T><<<grid, 256, 0, s>>>(a.N, a.d, static_cast<const T*>(a.X), a.ldx,
                                            static_cast<const T*>(a.Y), a.seed, a.stream_id, a.m,
                                            a.splits, a.partial, ldp);
  SLSE_LAUNCH_CHECK();
  gauss_reduce_kernel<float, float><<<grid1(a.m * cols), 256, 0, s>>>(
      a.partial, a.splits, a.m, cols, ldp, static_cast<float*>(a.A), a.lda);
  SLSE_LAUNCH_CHECK();
}

template <typename T, typename Acc>
void gaussian_t(const GaussianArgs& a, hipStream_t s) {
  const int cols = a.d + 1;
  const int64_t ldp = round_up(cols, 4);
  Acc* part = std::is_same<Acc, double>::value ? reinterpret_cast<Acc*>(a.partial64)
                                               : reinterpret_cast<Acc*>(a.partial);
  dim3 grid((unsigned)ceil_div(cols, kGT), (unsigned)ceil_div(a.m, kGT), (unsigned)a.splits);
  gauss_kernel<T, Acc><<<grid, kThreads, 0, s>>>(a.N, a.d, static_cast<const T*>(a.X), a.ldx,
                                                  static_cast<const T*>(a.Y), a.seed, a.stream_id,
                                                  a.m, a.splits, part, ldp);
  SLSE_LAUNCH_CHECK();
  gauss_reduce_kernel<T, Acc><<<grid1(a.m * cols), 256, 0, s>>>(part, a.splits, a.m, cols, ldp,
                                                                 static_cast<T*>(a.A), a.lda);
  SLSE_LAUNCH_CHECK();
}

}  // namespace

void launch_countsketch(const CountSketchArgs& a, hipStream_t s) {
  if (a.t == SLSE_F64)
    countsketch_t<double>(a, s);
  else if (a.t == SLSE_F32)
    countsketch_t<float>(a, s);
  else
    fail(SLSE_EUNSUPPORTED, "countsketch: dtype");
}

void gaussian_plan(GaussianArgs& a) {
  const int64_t tiles = a.bf16 ? ceil_div(a.d + 1, kNT) * ceil_div(a.m, kMT)
                               : ceil_div(a.d + 1, kGT) * ceil_div(a.m, kGT);
  // enough blocks to fill the chip, each split at least a few thousand rows
  int64_t splits = std::max<int64_t>(1, 2048 / std::max<int64_t>(tiles, 1));
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, a.N / 4096));
  a.splits = (int)splits;
}

size_t gaussian_scratch_bytes(const GaussianArgs& a) {
  const size_t es = (a.t == SLSE_F64 && !a.bf16) ? 8 : 4;
  return (size_t)a.splits * (size_t)a.m * (size_t)round_up(a.d + 1, 4) * es;
}

void launch_gaussian(const GaussianArgs& a, hipStream_t s) {
  if (a.bf16) {
    if (a.t != SLSE_F32) fail(SLSE_EUNSUPPORTED, "gaussian: BF16 products need F32 data");
    gaussian_mfma_t<float>(a, s);
    return;
  }
  if (a.t == SLSE_F64)
    gaussian_t<double, double>(a, s);
  else if (a.t == SLSE_F32)
    gaussian_t<float, float>(a, s);
  else
    fail(SLSE_EUNSUPPORTED, "gaussian: dtype");
}

void launch_debug_gaussian(uint64_t seed, uint64_t stream_id, int64_t k0, int64_t nk, int64_t j0,
                           int64_t nj, double* out, hipStream_t s) {
  if (nk * nj <= 0) return;
  debug_gauss_kernel<<<grid1(nk * nj), 256, 0, s>>>(seed, stream_id, k0, nk, j0, nj, out);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
