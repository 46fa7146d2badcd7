// Dense FP64 kernels behind slse_factor: the Hessian sketch
// H_hat = (S_hat X)^T S_hat X (Sec. 3) is applied through its triangular
// factor R (R^T R = H_hat; QR route of the implementation-details appendix).
//
//  gemm        C = alpha op(A) op(B) + beta C, 64x64 tiles, 4x4 per thread
//  cholesky    one block, blocked upper Cholesky: for each 32-row panel the
//              rows are first updated with all earlier rows of R (a GEMM
//              staged through LDS), then factored in LDS
//  tri_inv_t   L = R^{-T}: one wave per row of L (back substitution of
//              R x = e_j, x kept in LDS)
#include <algorithm>

#include "kernels.hpp"

namespace slse {
namespace {

constexpr int kTile = 64;
constexpr int kKStep = 16;

__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const double* __restrict__ A, int64_t lda,
                                                   int transA, const double* __restrict__ B,
                                                   int64_t ldb, int transB, double beta,
                                                   double* __restrict__ C, int64_t ldc) {
  __shared__ double As[kKStep][kTile + 1];
  __shared__ double Bs[kKStep][kTile + 1];
  const int tx = threadIdx.x % 16;
  const int ty = threadIdx.x / 16;
  const int64_t i0 = (int64_t)blockIdx.y * kTile;
  const int64_t j0 = (int64_t)blockIdx.x * kTile;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += kKStep) {
    for (int e = threadIdx.x; e < kKStep * kTile; e += 256) {
      int kk, ii;
      if (transA) {  // A stored K x M: contiguous along i
        kk = e / kTile;
        ii = e % kTile;
      } else {  // A stored M x K: contiguous along k
        ii = e / kKStep;
        kk = e % kKStep;
      }
      const int64_t gi = i0 + ii, gk = k0 + kk;
      double v = 0.0;
      if (gi < M && gk < K) v = transA ? A[gk * lda + gi] : A[gi * lda + gk];
      As[kk][ii] = v;
      int kb, jj;
      if (transB) {  // B stored N x K
        jj = e / kKStep;
        kb = e % kKStep;
      } else {
        kb = e / kTile;
        jj = e % kTile;
      }
      const int64_t gj = j0 + jj, gkb = k0 + kb;
      double w = 0.0;
      if (gj < N && gkb < K) w = transB ? B[gj * ldb + gkb] : B[gkb * ldb + gj];
      Bs[kb][jj] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKStep; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty + 16 * u];
        b[u] = Bs[kk][tx + 16 * u];
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
      const int64_t gi = i0 + ty + 16 * u, gj = j0 + tx + 16 * v;
      if (gi < M && gj < N) {
        double c = alpha * acc[u][v];
        if (beta != 0.0) c += beta * C[gi * ldc + gj];
        C[gi * ldc + gj] = c;
      }
    }
}

__global__ void convert_scale_kernel(int64_t rows, int d, const void* __restrict__ A, int64_t lda,
                                     int is_f32, double s, double* __restrict__ out, int64_t ldo) {
  const int64_t n = rows * d;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / d, k = e % d;
    const double v = is_f32 ? (double)static_cast<const float*>(A)[i * lda + k]
                            : static_cast<const double*>(A)[i * lda + k];
    out[i * ldo + k] = s * v;
  }
}

constexpr int kCholNB = 32;
constexpr int kCholThreads = 1024;
constexpr int kCholMaxD = 512;
constexpr int kCholKC = 32;

__global__ __launch_bounds__(kCholThreads) void cholesky_kernel(int d, const double* __restrict__ G,
                                                                int64_t ldg, double* __restrict__ R,
                                                                int64_t ldr, int* __restrict__ info) {
  __shared__ double P[kCholNB][kCholMaxD + 1];
  __shared__ double Kb[kCholKC][kCholNB];
  __shared__ double s_diag;
  __shared__ int s_bad;
  const int t = threadIdx.x;
  if (t == 0) s_bad = 0;
  for (int J = 0; J < d; J += kCholNB) {
    const int w = min(kCholNB, d - J);
    const int ncols = d - J;
    // 1. panel rows J..J+w of G, columns J..d
    for (int e = t; e < w * ncols; e += kCholThreads) {
      const int a = e / ncols, c = e % ncols;
      P[a][c] = G[(int64_t)(J + a) * ldg + J + c];
    }
    // 2. subtract sum_{k<J} R[k][J+a] R[k][J+c]
    {
      double acc[kCholNB];
#pragma unroll
      for (int a = 0; a < kCholNB; ++a) acc[a] = 0.0;
      const int c = t;
      for (int k0 = 0; k0 < J; k0 += kCholKC) {
        const int kc = min(kCholKC, J - k0);
        __syncthreads();
        for (int e = t; e < kc * w; e += kCholThreads) {
          const int kk = e / w, a = e % w;
          Kb[kk][a] = R[(int64_t)(k0 + kk) * ldr + J + a];
        }
        __syncthreads();
        if (c < ncols) {
          for (int kk = 0; kk < kc; ++kk) {
            const double rc = R[(int64_t)(k0 + kk) * ldr + J + c];
#pragma unroll
            for (int a = 0; a < kCholNB; ++a)
              if (a < w) acc[a] = fma(Kb[kk][a], rc, acc[a]);
          }
        }
      }
      __syncthreads();
      if (c < ncols) {
#pragma unroll
        for (int a = 0; a < kCholNB; ++a)
          if (a < w) P[a][c] -= acc[a];
      }
    }
    // 3. factor the panel: row a of R is row a of the panel scaled by 1/sqrt(pivot)
    for (int a = 0; a < w; ++a) {
      __syncthreads();
      if (t == 0) {
        double piv = P[a][a];
        if (!(piv > 0.0) || !isfinite(piv)) {
          if (!s_bad) s_bad = J + a + 1;
          piv = 1.0;
        }
        s_diag = sqrt(piv);
      }
      __syncthreads();
      const double inv = 1.0 / s_diag;
      for (int c = a + t; c < ncols; c += kCholThreads) P[a][c] = (c == a) ? s_diag : P[a][c] * inv;
      __syncthreads();
      const int rows_left = w - a - 1;
      for (int e = t; e < rows_left * ncols; e += kCholThreads) {
        const int b = a + 1 + e / ncols, c = e % ncols;
        if (c >= b) P[b][c] -= P[a][b] * P[a][c];
      }
    }
    __syncthreads();
    // 4. write the panel rows of R (zero below the diagonal)
    for (int e = t; e < w * d; e += kCholThreads) {
      const int a = e / d, c = e % d;
      const int rc = c - J;
      R[(int64_t)(J + a) * ldr + c] = (rc >= a) ? P[a][rc] : 0.0;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (t == 0) info[0] = s_bad;
}

// L[j][i] = (R^{-1})[i][j]: one wave per j
__global__ __launch_bounds__(256) void tri_inv_t_kernel(int d, const double* __restrict__ R,
                                                        int64_t ldr, double* __restrict__ L,
                                                        int64_t ldl) {
  extern __shared__ double xs_all[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 4 + wave;
  if (j >= d) return;
  double* xs = xs_all + (int64_t)wave * d;
  for (int i = lane; i < d; i += 64) xs[i] = 0.0;
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) xs[j] = 1.0 / R[(int64_t)j * ldr + j];
  __builtin_amdgcn_wave_barrier();
  for (int i = j - 1; i >= 0; --i) {
    const double* Ri = R + (int64_t)i * ldr;
    double s = 0.0;
    for (int k = i + 1 + lane; k <= j; k += 64) s = fma(Ri[k], xs[k], s);
    for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) xs[i] = -s / Ri[i];
    __builtin_amdgcn_wave_barrier();
  }
  for (int i = lane; i < d; i += 64) L[(int64_t)j * ldl + i] = (i <= j) ? xs[i] : 0.0;
}

}  // namespace

void launch_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                     bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
                     int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((unsigned)ceil_div(N, kTile), (unsigned)ceil_div(M, kTile));
  gemm_kernel<<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, transA ? 1 : 0, B, ldb, transB ? 1 : 0,
                                   beta, C, ldc);
  SLSE_LAUNCH_CHECK();
}

void launch_convert_scale(int64_t rows, int d, const void* A, int64_t lda, slse_dtype at, double s,
                          double* out, int64_t ldo, hipStream_t st) {
  const int64_t n = rows * d;
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>(ceil_div(n, 256), 8192);
  convert_scale_kernel<<<blocks, 256, 0, st>>>(rows, d, A, lda, at == SLSE_F32 ? 1 : 0, s, out,
                                                ldo);
  SLSE_LAUNCH_CHECK();
}

void launch_cholesky(int d, const double* G, int64_t ldg, double* R, int64_t ldr, int* info,
                     hipStream_t s) {
  if (d > kCholMaxD) fail(SLSE_EUNSUPPORTED, "cholesky: d > 512 not supported by this build");
  cholesky_kernel<<<1, kCholThreads, 0, s>>>(d, G, ldg, R, ldr, info);
  SLSE_LAUNCH_CHECK();
}

void launch_tri_inv_t(int d, const double* R, int64_t ldr, double* L, int64_t ldl, hipStream_t s) {
  const size_t shm = (size_t)4 * d * sizeof(double);
  if (shm > 64 * 1024) fail(SLSE_EUNSUPPORTED, "tri_inv: d too large for this build");
  tri_inv_t_kernel<<<(int)ceil_div(d, 4), 256, shm, s>>>(d, R, ldr, L, ldl);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
