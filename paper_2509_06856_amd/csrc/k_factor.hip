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

// value of `v` held by lane `lane` (uniform), broadcast to the wave
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// One 64 x 64 output tile of C = alpha op(A) op(B) + beta C over k in
// [kb0, kend); with `part` the raw sums go to split slot `zpart` instead.
// (the pointer types are generic, or global ones from a batched kernel's
// job descriptors)
template <typename CP, typename MP>
__device__ __forceinline__ void gemm_tile(int64_t M, int64_t N, double alpha, CP __restrict__ A,
                                          int64_t lda, int transA, CP __restrict__ B, int64_t ldb,
                                          int transB, double beta, MP __restrict__ C, int64_t ldc,
                                          MP __restrict__ part, int zpart, int64_t i0,
                                          int64_t j0, int64_t kb0, int64_t kend) {
  __shared__ double As[kKStep][kTile + 1];
  __shared__ double Bs[kKStep][kTile + 1];
  const int tx = threadIdx.x % 16;
  const int ty = threadIdx.x / 16;
  double acc[4][4] = {};
  // Each thread copies kL entries of A and of B per k step.  Their loads are
  // unconditional (entries outside the matrices read a clamped, valid address
  // and are replaced by zero when written to LDS) and the next step's are
  // issued before the current step's products, so they are all in flight
  // together and overlap the arithmetic.
  constexpr int kL = kKStep * kTile / 256;
  double va[kL], vb[kL];
  unsigned oka = 0, okb = 0;
  auto fetch = [&](int64_t k0) {
    oka = okb = 0;
#pragma unroll
    for (int u = 0; u < kL; ++u) {
      const int e = threadIdx.x + 256 * u;
      int kk, ii;
      if (transA) {  // A stored K x M: contiguous along i
        kk = e / kTile;
        ii = e % kTile;
      } else {  // A stored M x K: contiguous along k
        ii = e / kKStep;
        kk = e % kKStep;
      }
      const int64_t gi = i0 + ii, gk = k0 + kk;
      oka |= (unsigned)(gi < M && gk < kend) << u;
      const int64_t ci = min(gi, M - 1), ck = min(gk, kend - 1);
      va[u] = transA ? A[ck * lda + ci] : A[ci * lda + ck];
      int kb, jj;
      if (transB) {  // B stored N x K
        jj = e / kKStep;
        kb = e % kKStep;
      } else {
        kb = e / kTile;
        jj = e % kTile;
      }
      const int64_t gj = j0 + jj, gkb = k0 + kb;
      okb |= (unsigned)(gj < N && gkb < kend) << u;
      const int64_t cj = min(gj, N - 1), ckb = min(gkb, kend - 1);
      vb[u] = transB ? B[cj * ldb + ckb] : B[ckb * ldb + cj];
    }
  };
  if (kb0 < kend) fetch(kb0);
  for (int64_t k0 = kb0; k0 < kend; k0 += kKStep) {
#pragma unroll
    for (int u = 0; u < kL; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (transA)
        As[e / kTile][e % kTile] = ((oka >> u) & 1) ? va[u] : 0.0;
      else
        As[e % kKStep][e / kKStep] = ((oka >> u) & 1) ? va[u] : 0.0;
      if (transB)
        Bs[e % kKStep][e / kKStep] = ((okb >> u) & 1) ? vb[u] : 0.0;
      else
        Bs[e / kTile][e % kTile] = ((okb >> u) & 1) ? vb[u] : 0.0;
    }
    __syncthreads();
    if (k0 + kKStep < kend) fetch(k0 + kKStep);
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
        if (part) {
          part[((int64_t)zpart * M + gi) * N + gj] = acc[u][v];
        } else {
          double c = alpha * acc[u][v];
          if (beta != 0.0) c += beta * C[gi * ldc + gj];
          C[gi * ldc + gj] = c;
        }
      }
    }
}

__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const double* __restrict__ A, int64_t lda,
                                                   int transA, const double* __restrict__ B,
                                                   int64_t ldb, int transB, double beta,
                                                   double* __restrict__ C, int64_t ldc,
                                                   double* __restrict__ part, int64_t kper) {
  const int64_t kb0 = (int64_t)blockIdx.z * kper;
  gemm_tile(M, N, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc, part, (int)blockIdx.z,
            (int64_t)blockIdx.y * kTile, (int64_t)blockIdx.x * kTile, kb0, min(K, kb0 + kper));
}

// Batched products of the factor jobs (blockIdx.z = job):
//   which = 0: G = Ad^T Ad    which = 1: M = L L^T
// G = Ad^T Ad of every job (blockIdx.z = job x splits + split): with splits > 1
// each split sums its share of the rows into the job's partial slot
__global__ __launch_bounds__(256) void factor_gemm_batched_kernel(const FactorJob* __restrict__ jobs,
                                                                  int splits) {
  const int z = blockIdx.z / splits, sp = blockIdx.z % splits;
  const FactorJob jb = jobs[z];
  const int64_t d = jb.d;
  const int64_t i0 = (int64_t)blockIdx.y * kTile, j0 = (int64_t)blockIdx.x * kTile;
  if (i0 >= d || j0 >= d) return;
  const int64_t kper = round_up(ceil_div(jb.rows, (int64_t)splits), kKStep);
  const int64_t kb0 = sp * kper;
  gemm_tile(d, d, 1.0, gptr((const double*)jb.Ad), d, 1, gptr((const double*)jb.Ad), d, 0, 0.0,
            gptr(jb.G), d, splits > 1 ? gptr(jb.part) : nullptr, sp, i0, j0, kb0,
            min(jb.rows, kb0 + kper));
}

// G = sum of the job's split slots, in split order (blockIdx.y = job)
__global__ void factor_reduce_batched_kernel(const FactorJob* __restrict__ jobs, int splits) {
  const FactorJob jb = jobs[blockIdx.y];
  const int64_t n = (int64_t)jb.d * jb.d;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < splits; ++q) t += gptr(jb.part)[(int64_t)q * n + e];
    *gptr(jb.G + e) = t;
  }
}

// C = alpha * sum_s part[s] + beta * C (splits summed in order)
__global__ void gemm_reduce_kernel(int64_t M, int64_t N, int splits, const double* __restrict__ part,
                                   double alpha, double beta, double* __restrict__ C, int64_t ldc) {
  const int64_t n = M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < splits; ++q) t += part[(int64_t)q * n + e];
    const int64_t i = e / N, j = e % N;
    double c = alpha * t;
    if (beta != 0.0) c += beta * C[i * ldc + j];
    C[i * ldc + j] = c;
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

constexpr int kCholNB = 32;       // panel height
constexpr int kCholThreads = 512;  // one thread per column of the panel
constexpr int kCholMaxD = 512;
constexpr int kCholKC = 32;       // rows of R staged per update step

// Upper Cholesky R^T R = G by row panels of height 32.  Thread c owns column
// J + c of the panel rows J..J+31 in registers.  Each panel is first reduced by
// the rows of R above it (a GEMM against rows staged through LDS), its 32 x 32
// diagonal block is then factored in LDS by the whole block, and the rest of
// the panel is a triangular solve with that block, one column per thread.
__device__ __forceinline__ void cholesky_block(int d, const double* __restrict__ G, int64_t ldg,
                                               double* __restrict__ R, int64_t ldr,
                                               int* __restrict__ info) {
  __shared__ double Kb[kCholKC][kCholNB];
  __shared__ double D[kCholNB][kCholNB + 1];
  __shared__ int s_bad;
  const int t = threadIdx.x;
  if (t == 0) s_bad = 0;
  for (int J = 0; J < d; J += kCholNB) {
    const int w = min(kCholNB, d - J);
    const int ncols = d - J;
    const bool mine = t < ncols;
    double acc[kCholNB];
#pragma unroll
    for (int a = 0; a < kCholNB; ++a) acc[a] = (mine && a < w) ? G[(int64_t)(J + a) * ldg + J + t] : 0.0;
    // 1. subtract sum_{k < J} R[k][J+a] R[k][J+t]
    for (int k0 = 0; k0 < J; k0 += kCholKC) {
      const int kc = min(kCholKC, J - k0);
      __syncthreads();
      for (int e = t; e < kCholKC * kCholNB; e += kCholThreads) {
        const int kk = e / kCholNB, a = e % kCholNB;
        Kb[kk][a] = (kk < kc && a < w) ? R[(int64_t)(k0 + kk) * ldr + J + a] : 0.0;
      }
      double rc[kCholKC];
#pragma unroll
      for (int kk = 0; kk < kCholKC; ++kk)
        rc[kk] = (mine && kk < kc) ? R[(int64_t)(k0 + kk) * ldr + J + t] : 0.0;
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kCholKC; ++kk)
#pragma unroll
        for (int a = 0; a < kCholNB; ++a) acc[a] = fma(-Kb[kk][a], rc[kk], acc[a]);
    }
    // 2. factor the diagonal block: wave 0, lane c holds column c in registers,
    //    rows of the block are broadcast lane to lane
    if (t < 64) {
      double col[kCholNB];
#pragma unroll
      for (int a = 0; a < kCholNB; ++a) col[a] = acc[a];
#pragma unroll
      for (int a = 0; a < kCholNB; ++a) {
        if (a < w) {
          double piv = readlane_f64(col[a], a);
          if (!(piv > 0.0) || !isfinite(piv)) {
            if (t == 0 && !s_bad) s_bad = J + a + 1;
            piv = 1.0;
          }
          const double rd = sqrt(piv);
          const double inv = 1.0 / rd;
          col[a] = (t == a) ? rd : col[a] * inv;  // row a of R: R[a][c]
#pragma unroll
          for (int b = a + 1; b < kCholNB; ++b) {
            if (b < w) col[b] = fma(-readlane_f64(col[a], b), col[a], col[b]);
          }
        }
      }
      if (t < w) {
#pragma unroll
        for (int a = 0; a < kCholNB; ++a)
          if (a < w) D[a][t] = col[a];
      }
    }
    __syncthreads();
    // 3. the rest of the panel: solve D^T x = acc for each column t >= w
    if (mine) {
      if (t < w) {
#pragma unroll
        for (int a = 0; a < kCholNB; ++a) acc[a] = (a < w && a <= t) ? D[a][t] : 0.0;
      } else {
#pragma unroll
        for (int a = 0; a < kCholNB; ++a) {
          if (a < w) {
            double x = acc[a];
#pragma unroll
            for (int b = 0; b < kCholNB; ++b)
              if (b < a) x = fma(-D[b][a], acc[b], x);
            acc[a] = x / D[a][a];
          }
        }
      }
    }
    // 4. write panel rows J..J+w of R (zero left of the diagonal)
    for (int a = 0; a < w; ++a) {
      double* Rr = R + (int64_t)(J + a) * ldr;
      for (int c = t; c < J; c += kCholThreads) Rr[c] = 0.0;
    }
    if (mine) {
#pragma unroll
      for (int a = 0; a < kCholNB; ++a)
        if (a < w) R[(int64_t)(J + a) * ldr + J + t] = acc[a];
    }
    __threadfence_block();
    __syncthreads();
  }
  if (t == 0) info[0] = s_bad;
}

__global__ __launch_bounds__(kCholThreads) void cholesky_kernel(int d, const double* __restrict__ G,
                                                                int64_t ldg, double* __restrict__ R,
                                                                int64_t ldr, int* __restrict__ info) {
  cholesky_block(d, G, ldg, R, ldr, info);
}

// Rinv = R^{-1} row by row: row i solves x^T R = e_i^T by forward
// substitution over j with running sums s_l = -sum_{k<j} x_k R_kl, so each
// step reads one row of R (contiguous).  Lane l keeps s for the columns
// l, l+64, ... in registers; x_j is read from its owner lane.  A block's four
// waves take rows i0..i0+3 and share rows of R staged through LDS.
constexpr int kInvRows = 16;
constexpr int kInvMaxD = 512;
constexpr int kInvPer = kInvMaxD / 64;

__device__ __forceinline__ void tri_inv_rows(int d, const double* __restrict__ R, int64_t ldr,
                                             double* __restrict__ Rinv, int64_t ldi, int i0) {
  __shared__ double Rs[kInvRows][kInvMaxD];
  __shared__ double rdiag[kInvMaxD];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i = i0 + wave;
  for (int l = threadIdx.x; l < d; l += 256) rdiag[l] = 1.0 / R[(int64_t)l * ldr + l];
  double s[kInvPer];
#pragma unroll
  for (int k = 0; k < kInvPer; ++k) s[k] = 0.0;
  for (int j0 = i0; j0 < d; j0 += kInvRows) {
    const int jc = min(kInvRows, d - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < jc * d; e += 256) {
      const int rr = e / d, c = e % d;
      Rs[rr][c] = R[(int64_t)(j0 + rr) * ldr + c];
    }
    __syncthreads();
    if (i < d) {
      for (int jj = 0; jj < jc; ++jj) {
        const int j = j0 + jj;
        if (j < i) continue;
        // x_j = (delta_ij + s_j) / R_jj, s_j held by lane j % 64 in slot j / 64
        double sj = 0.0;
#pragma unroll
        for (int k = 0; k < kInvPer; ++k)
          if (k == (j >> 6)) sj = readlane_f64(s[k], j & 63);
        const double xj = ((j == i) ? 1.0 + sj : sj) * rdiag[j];
#pragma unroll
        for (int k = 0; k < kInvPer; ++k) {
          const int l = lane + 64 * k;
          if (l == j) {
            s[k] = xj;  // slot j now holds x_j
          } else if (l > j && l < d) {
            s[k] = fma(-xj, Rs[jj][l], s[k]);
          }
        }
      }
    }
  }
  if (i < d) {
#pragma unroll
    for (int k = 0; k < kInvPer; ++k) {
      const int l = lane + 64 * k;
      if (l < d) Rinv[(int64_t)i * ldi + l] = (l < i) ? 0.0 : s[k];
    }
  }
}

__global__ __launch_bounds__(256) void tri_inv_kernel(int d, const double* __restrict__ R,
                                                      int64_t ldr, double* __restrict__ Rinv,
                                                      int64_t ldi) {
  tri_inv_rows(d, R, ldr, Rinv, ldi, blockIdx.x * 4);
}

// Ad = scale * A[:, :d] of every job (blockIdx.y = job)
__global__ void convert_scale_batched_kernel(const FactorJob* __restrict__ jobs, int is_f32) {
  const FactorJob jb = jobs[blockIdx.y];
  const int64_t n = jb.rows * jb.d;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / jb.d, k = e % jb.d;
    const double v = is_f32 ? (double)gptr(static_cast<const float*>(jb.A))[i * jb.lda + k]
                            : gptr(static_cast<const double*>(jb.A))[i * jb.lda + k];
    *gptr(jb.Ad + e) = jb.scale * v;
  }
}

// ---------------------------------------------------------------------------
// M = G^{-1} for SPD G by blocked Gauss-Jordan elimination in place, 32 rows
// per step (no pivoting: the pivots of an SPD matrix are positive).  Step k
// with pivot block P = G[K, K], K = [k0, k0 + 32):
//   panel  : Pinv = P^{-1} (every block; block 0 stores it in colp rows K);
//            G[K, j] = Pinv G[K, j] (j outside K); the old column panel
//            G[i, K] (i outside K) is saved to colp rows i
//   update : G[i, j] -= colp[i, :] G[K, j]   (i, j outside K)
//            G[i, K]  = -colp[i, :] Pinv      (i outside K)
//            G[K, K]  = Pinv
// G[K, K] is written only in the update, after every panel block has read P.
// ---------------------------------------------------------------------------
constexpr int kGJ = 32;
constexpr int kGJChunk = 64;  // columns (and saved rows) per panel block

template <typename DP, typename IP>
__device__ __forceinline__ void gj_panel(int d, int k0, DP __restrict__ G, DP __restrict__ colp,
                                         IP __restrict__ info, int bx) {
  __shared__ double Pinv[kGJ][kGJ + 1];
  __shared__ double Rp[kGJ][kGJChunk + 1];
  const int t = threadIdx.x;
  const int kw = min(kGJ, d - k0);
  // Every thread moves a fixed number of entries in each of 1-3, so the
  // loops have compile-time trip counts and all their loads are in flight
  // together (a runtime-bounded loop waits for each load in turn).
  constexpr int kP = kGJ * kGJ / 256;       // pivot-block entries per thread
  constexpr int kC = kGJChunk * kGJ / 256;  // column- and row-panel entries per thread
  // (loads outside the matrix read a clamped, valid address and are
  // replaced afterwards, so that no load sits behind a branch)
  // 1. the pivot block into LDS, padded with the identity past d
  {
    double v[kP];
#pragma unroll
    for (int u = 0; u < kP; ++u) {
      const int e = t + 256 * u;
      const int a = min(e / kGJ, kw - 1), c = min(e % kGJ, kw - 1);
      v[u] = G[(int64_t)(k0 + a) * d + k0 + c];
    }
#pragma unroll
    for (int u = 0; u < kP; ++u) {
      const int e = t + 256 * u;
      const int a = e / kGJ, c = e % kGJ;
      Pinv[a][c] = (a < kw && c < kw) ? v[u] : (a == c ? 1.0 : 0.0);
    }
  }
  // 2. save the old column panel for rows [64 b, 64 b + 64) outside K
  const int r0 = bx * kGJChunk;
  {
    double v[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const int e = t + 256 * u;
      const int i = min(r0 + e / kGJ, d - 1), a = min(e % kGJ, kw - 1);
      v[u] = G[(int64_t)i * d + k0 + a];
    }
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const int e = t + 256 * u;
      const int i = r0 + e / kGJ, a = e % kGJ;
      if (i < d && (i < k0 || i >= k0 + kw) && a < kw) colp[(int64_t)i * kGJ + a] = v[u];
    }
  }
  // 3. row panel of this block's columns [64 b, 64 b + 64)
  const int c0 = bx * kGJChunk;
  {
    double v[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const int e = t + 256 * u;
      const int a = min(e / kGJChunk, kw - 1), j = min(c0 + e % kGJChunk, d - 1);
      v[u] = G[(int64_t)(k0 + a) * d + j];
    }
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const int e = t + 256 * u;
      const int a = e / kGJChunk, j = c0 + e % kGJChunk;
      Rp[a][e % kGJChunk] = (a < kw && j < d) ? v[u] : 0.0;
    }
  }
  __syncthreads();
  // 1b. Gauss-Jordan on the pivot block in place, every thread on four entries
  // of one row (row i = t / 8, columns 4 (t % 8) ..): at step s the pivot row
  // becomes P[s][.] / P[s][s] (1 / P[s][s] in column s), and every other row
  // loses P[i][s] times it (-P[i][s] / P[s][s] in column s).  The old values
  // of the step are read before a barrier and written after it.  A
  // non-positive or non-finite pivot is reported.
  {
    static_assert(kGJ * kGJ == 4 * 256, "four entries per thread");
    const int i = t >> 3;
    const int j0 = (t & 7) * 4;
    bool bad = false;
    for (int s = 0; s < kGJ; ++s) {
      double piv = Pinv[s][s];
      if (!(piv > 0.0) || !isfinite(piv)) {
        bad = true;
        piv = 1.0;
      }
      const double inv = 1.0 / piv;
      const double f = Pinv[i][s];
      double rs[4], cur[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + u;
        rs[u] = (j == s) ? inv : Pinv[s][j] * inv;
        cur[u] = Pinv[i][j];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + u;
        Pinv[i][j] = (i == s) ? rs[u] : (j == s) ? -f * inv : fma(-f, rs[u], cur[u]);
      }
      __syncthreads();
    }
    if (bad && t == 0) atomicCAS(info, 0, k0 + 1);
  }
  if (bx == 0)
    for (int e = t; e < kGJ * kGJ; e += 256) {
      const int a = e / kGJ, c = e % kGJ;
      if (a < kw && c < kw) colp[(int64_t)(k0 + a) * kGJ + c] = Pinv[a][c];
    }
  for (int e = t; e < kGJ * kGJChunk; e += 256) {
    const int a = e / kGJChunk, jj = e % kGJChunk, j = c0 + jj;
    if (a >= kw || j >= d || (j >= k0 && j < k0 + kw)) continue;
    double v = 0.0;
#pragma unroll 8
    for (int q = 0; q < kGJ; ++q) v = fma(Pinv[a][q], Rp[q][jj], v);
    G[(int64_t)(k0 + a) * d + j] = v;
  }
}

__global__ __launch_bounds__(256) void gj_panel_kernel(int d, int k0, double* __restrict__ G,
                                                       double* __restrict__ colp,
                                                       int* __restrict__ info) {
  gj_panel(d, k0, G, colp, info, blockIdx.x);
}

// the panel step of every job (blockIdx.y), past the end of a smaller job: nothing
__global__ __launch_bounds__(256) void gj_panel_batched_kernel(const FactorJob* __restrict__ jobs,
                                                               int k0) {
  const FactorJob jb = jobs[blockIdx.y];
  if (k0 >= jb.d || (int)blockIdx.x * kGJChunk >= jb.d) return;
  gj_panel(jb.d, k0, gptr(jb.M), gptr(jb.colp), jb.info, blockIdx.x);
}

// one 32 x 32 output tile per block (by = row tile, bx = column tile)
template <typename DP, typename CP>
__device__ __forceinline__ void gj_update(int d, int k0, DP __restrict__ G, CP __restrict__ colp,
                                          int bx, int by) {
  __shared__ double Cp[kGJ][kGJ + 1];  // colp rows of this tile
  __shared__ double Rw[kGJ][kGJ + 1];  // new row panel columns of this tile
  const int kw = min(kGJ, d - k0);
  const int i0 = by * kGJ, j0 = bx * kGJ;
  const int t = threadIdx.x;
  const bool pivcols = j0 == k0;
  if (i0 == k0) {  // the pivot rows were finished by the panel step, but for G[K, K]
    if (pivcols)
      for (int e = t; e < kGJ * kGJ; e += 256) {
        const int r = e / kGJ, c = e % kGJ;
        if (r < kw && c < kw) G[(int64_t)(k0 + r) * d + k0 + c] = colp[(int64_t)(k0 + r) * kGJ + c];
      }
    return;
  }
  // a fixed count per thread, every load from a clamped valid address (the
  // entries outside the matrix are replaced afterwards): all of the two
  // tiles' loads in flight together
  {
    constexpr int kT = kGJ * kGJ / 256;
    double cv[kT], rv[kT];
#pragma unroll
    for (int u = 0; u < kT; ++u) {
      const int e = t + 256 * u;
      const int r = e / kGJ, c = min(e % kGJ, kw - 1);
      cv[u] = colp[(int64_t)min(i0 + r, d - 1) * kGJ + c];
      // Pinv (colp rows K) for the pivot columns, else the new row panel
      const int rr = min(r, kw - 1);
      rv[u] = pivcols ? colp[(int64_t)(k0 + rr) * kGJ + c]
                      : G[(int64_t)(k0 + rr) * d + min(j0 + e % kGJ, d - 1)];
    }
#pragma unroll
    for (int u = 0; u < kT; ++u) {
      const int e = t + 256 * u;
      const int r = e / kGJ, c = e % kGJ;
      Cp[r][c] = (i0 + r < d && c < kw) ? cv[u] : 0.0;
      Rw[r][c] = (r < kw && j0 + c < d) ? rv[u] : 0.0;
    }
  }
  __syncthreads();
  // the tile's old values first (all in flight), then the products
  constexpr int kU = kGJ * kGJ / 256;
  double old[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int e = t + 256 * u;
    const int i = i0 + e / kGJ, j = j0 + e % kGJ;
    old[u] = G[(int64_t)min(i, d - 1) * d + min(j, d - 1)];
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int e = t + 256 * u;
    const int r = e / kGJ, c = e % kGJ;
    const int i = i0 + r, j = j0 + c;
    if (i >= d || j >= d) continue;
    double v = 0.0;
#pragma unroll 8
    for (int q = 0; q < kGJ; ++q) v = fma(Cp[r][q], Rw[q][c], v);
    G[(int64_t)i * d + j] = pivcols ? -v : old[u] - v;  // Rw holds Pinv for the pivot columns
  }
}

__global__ __launch_bounds__(256) void gj_update_kernel(int d, int k0, double* __restrict__ G,
                                                        const double* __restrict__ colp) {
  gj_update(d, k0, G, colp, blockIdx.x, blockIdx.y);
}

// the update step of every job (blockIdx.z)
__global__ __launch_bounds__(256) void gj_update_batched_kernel(const FactorJob* __restrict__ jobs,
                                                                int k0) {
  const FactorJob jb = jobs[blockIdx.z];
  const int nt = (int)ceil_div(jb.d, kGJ);
  if (k0 >= jb.d || (int)blockIdx.x >= nt || (int)blockIdx.y >= nt) return;
  gj_update(jb.d, k0, gptr(jb.M), gptr((const double*)jb.colp), blockIdx.x, blockIdx.y);
}

// G += coef trace(G) I (one block): the diagonal shift of shifted CholeskyQR
__global__ __launch_bounds__(256) void shift_diag_kernel(int d, double* __restrict__ G, double coef) {
  __shared__ double red[256];
  double t = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) t += G[(int64_t)i * d + i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double shift = coef * red[0];
  for (int i = threadIdx.x; i < d; i += 256) G[(int64_t)i * d + i] += shift;
}

}  // namespace

void launch_shift_diag(int d, double* G, double coef, hipStream_t s) {
  shift_diag_kernel<<<1, 256, 0, s>>>(d, G, coef);
  SLSE_LAUNCH_CHECK();
}

void launch_spd_inverse(int d, double* G, double* colp, int* info, hipStream_t s) {
  if (d <= 0) return;
  const unsigned nt = (unsigned)ceil_div(d, kGJ);
  for (int k0 = 0; k0 < d; k0 += kGJ) {
    gj_panel_kernel<<<(unsigned)ceil_div(d, kGJChunk), 256, 0, s>>>(d, k0, G, colp, info);
    SLSE_LAUNCH_CHECK();
    gj_update_kernel<<<dim3(nt, nt), 256, 0, s>>>(d, k0, G, colp);
    SLSE_LAUNCH_CHECK();
  }
}

int gemm_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ceil_div(M, kTile) * ceil_div(N, kTile);
  int64_t sp = std::max<int64_t>(1, 512 / std::max<int64_t>(tiles, 1));
  sp = std::min<int64_t>(sp, std::max<int64_t>(1, K / 128));
  return (int)std::min<int64_t>(sp, 32);
}

size_t gemm_scratch_doubles(int64_t M, int64_t N, int64_t K) {
  const int sp = gemm_splits(M, N, K);
  return sp > 1 ? (size_t)sp * M * N : 0;
}

void launch_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                     bool transA, const double* B, int64_t ldb, bool transB, double beta, double* C,
                     int64_t ldc, hipStream_t s, double* scratch, size_t scratch_doubles) {
  if (M <= 0 || N <= 0) return;
  int sp = gemm_splits(M, N, K);
  if (sp > 1 && (!scratch || scratch_doubles < (size_t)sp * M * N)) sp = 1;
  const int64_t kper = sp > 1 ? round_up(ceil_div(K, sp), kKStep) : std::max<int64_t>(K, 1);
  sp = (int)std::max<int64_t>(1, ceil_div(K, kper));
  dim3 grid((unsigned)ceil_div(N, kTile), (unsigned)ceil_div(M, kTile), (unsigned)sp);
  gemm_kernel<<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, transA ? 1 : 0, B, ldb, transB ? 1 : 0,
                                   beta, C, ldc, sp > 1 ? scratch : nullptr, kper);
  SLSE_LAUNCH_CHECK();
  if (sp > 1) {
    const int blocks = (int)std::min<int64_t>(ceil_div(M * N, 256), 4096);
    gemm_reduce_kernel<<<blocks, 256, 0, s>>>(M, N, sp, scratch, alpha, beta, C, ldc);
    SLSE_LAUNCH_CHECK();
  }
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
  if (d > kCholMaxD) fail(SLSE_EUNSUPPORTED, "cholesky: d > 512 not supported by this library");
  cholesky_kernel<<<1, kCholThreads, 0, s>>>(d, G, ldg, R, ldr, info);
  SLSE_LAUNCH_CHECK();
}

int factor_batched_splits(int64_t rows_max) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, rows_max / 256));
}

void launch_factor_batched(const FactorJob* jobs, int B, int dmax, int64_t rows_max,
                           slse_dtype at, hipStream_t s) {
  if (B <= 0) return;
  if (dmax > kCholMaxD) fail(SLSE_EUNSUPPORTED, "cholesky: d > 512 not supported by this library");
  const unsigned cb = (unsigned)std::min<int64_t>(ceil_div(rows_max * dmax, 256), 1024);
  convert_scale_batched_kernel<<<dim3(cb, (unsigned)B), 256, 0, s>>>(jobs, at == SLSE_F32 ? 1 : 0);
  SLSE_LAUNCH_CHECK();
  const unsigned tiles = (unsigned)ceil_div(dmax, kTile);
  // the scaled Gram into M (G points at M), then M = G^{-1} in place by the
  // blocked Gauss-Jordan steps of every job at once
  if (B > 65535) fail(SLSE_EUNSUPPORTED, "factor: too many batched jobs");
  const int splits = factor_batched_splits(rows_max);
  if ((int64_t)B * splits > 65535) fail(SLSE_EUNSUPPORTED, "factor: too many batched jobs");
  factor_gemm_batched_kernel<<<dim3(tiles, tiles, (unsigned)(B * splits)), 256, 0, s>>>(jobs, splits);
  SLSE_LAUNCH_CHECK();
  if (splits > 1) {
    const unsigned rb = (unsigned)std::min<int64_t>(ceil_div((int64_t)dmax * dmax, 256), 256);
    factor_reduce_batched_kernel<<<dim3(rb, (unsigned)B), 256, 0, s>>>(jobs, splits);
    SLSE_LAUNCH_CHECK();
  }
  const unsigned nt = (unsigned)ceil_div(dmax, kGJ);
  for (int k0 = 0; k0 < dmax; k0 += kGJ) {
    gj_panel_batched_kernel<<<dim3((unsigned)ceil_div(dmax, kGJChunk), (unsigned)B), 256, 0, s>>>(jobs,
                                                                                                k0);
    SLSE_LAUNCH_CHECK();
    gj_update_batched_kernel<<<dim3(nt, nt, (unsigned)B), 256, 0, s>>>(jobs, k0);
    SLSE_LAUNCH_CHECK();
  }
}

void launch_tri_inv(int d, const double* R, int64_t ldr, double* Rinv, int64_t ldi, hipStream_t s) {
  if (d > kInvMaxD) fail(SLSE_EUNSUPPORTED, "tri_inv: d > 512 not supported by this library");
  tri_inv_kernel<<<(int)ceil_div(d, 4), 256, 0, s>>>(d, R, ldr, Rinv, ldi);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
