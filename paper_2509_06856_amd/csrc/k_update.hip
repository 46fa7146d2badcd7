// M-IHS step with a fixed Hessian sketch (eqs. (98) and (99)):
//   beta_{t+1} = beta_t + mu * H_hat^{-1} g_t + eta * (beta_t - beta_{t-1}),
// g_t = c X^T (Y - X beta_t) being the negative gradient produced by the fused
// residual-gradient pass (its per-group partial rows are summed here, in a
// fixed order).  H_hat^{-1} is applied as the dense symmetric matrix
// M = R^{-1} R^{-T} (a GEMV spread over blocks).  The step also reduces
//   ||M g_t||^2 and ||beta_{t+1}||^2,
// whose ratio estimates the relative error of beta_t against the fixed point
// (beta_hat - beta_t = H^{-1} g_t and M ~ H^{-1}); the last block to finish
// writes it, flags non-finite values and raises `done` when it meets tol.
#include <algorithm>

#include "kernels.hpp"

namespace slse {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__global__ __launch_bounds__(kThreads) void mihs_update_kernel(UpdateArgs a, int rows_per_block) {
  if (a.done && *a.done) return;
  extern __shared__ double s_g[];
  __shared__ double s_red[3][kWaves];
  __shared__ int s_ticket;
  const int d = a.d;
  for (int k = threadIdx.x; k < d; k += kThreads) {
    // fixed-order sum over the groups, loads issued eight at a time
    double t = 0.0;
    int q = 0;
    for (; q + 8 <= a.groups; q += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = a.gpart[(int64_t)(q + u) * a.ldp + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) t += v[u];
    }
    for (; q < a.groups; ++q) t += a.gpart[(int64_t)q * a.ldp + k];
    double g = a.scale * t;
    if (a.w) g += a.w[k * a.incw];
    s_g[k] = g;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double gp = 0.0, pp = 0.0, bb = 0.0;
  const int row0 = blockIdx.x * rows_per_block;
  for (int j = wave; j < rows_per_block; j += kWaves) {
    const int i = row0 + j;
    if (i >= d) break;
    const double* Mi = a.M + (int64_t)i * a.ldm;
    double p = 0.0;
    for (int k = lane; k < d; k += 64) p = fma(Mi[k], s_g[k], p);
    for (int m = 32; m > 0; m >>= 1) p += wave_xor(p, m);
    if (lane == 0) {
      const double bi = a.beta[i];
      const double bn = bi + a.mu * p + a.eta * (bi - a.beta_prev[i]);
      a.beta_next[i] = bn;
      if (a.beta_out) a.beta_out[i] = bn;
      if (a.traj_row) a.traj_row[i] = bn;
      gp += s_g[i] * p;
      pp += p * p;
      bb += bn * bn;
    }
  }
  if (!a.sur_partial) return;
  if (lane == 0) {
    s_red[0][wave] = gp;
    s_red[1][wave] = pp;
    s_red[2][wave] = bb;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += s_red[threadIdx.x][w];
    store_device(a.sur_partial + 3 * blockIdx.x + threadIdx.x, t);
  }
  wait_memory();
  __syncthreads();
  if (threadIdx.x == 0) {
    s_ticket = take_ticket(a.sur_counter);
    if (s_ticket == (int)gridDim.x - 1) acquire_partials();
  }
  __syncthreads();
  if (s_ticket != (int)gridDim.x - 1) return;
  // the last block: every thread sums a fixed subset of the block partials,
  // then a fixed tree over the threads (deterministic)
  __shared__ double s_tail[3][kThreads];
  double tgp = 0.0, tpp = 0.0, tbb = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kThreads) {
    tgp += load_device(a.sur_partial + 3 * b + 0);
    tpp += load_device(a.sur_partial + 3 * b + 1);
    tbb += load_device(a.sur_partial + 3 * b + 2);
  }
  s_tail[0][threadIdx.x] = tgp;
  s_tail[1][threadIdx.x] = tpp;
  s_tail[2][threadIdx.x] = tbb;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int c = 0; c < 3; ++c) s_tail[c][threadIdx.x] += s_tail[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tgp = s_tail[0][0];
    tpp = s_tail[1][0];
    tbb = s_tail[2][0];
    const double est = tbb > 0.0 ? sqrt(tpp / tbb) : sqrt(tpp);
    if (a.sur_out) a.sur_out[0] = est;
    const bool finite = isfinite(tgp) && isfinite(tpp) && isfinite(tbb);
    if (!finite && a.status) atomicExch(a.status, 1);
    if (a.done && a.tol2 > 0.0 && (!finite || est * est <= a.tol2)) atomicExch(a.done, 1);
    atomicExch(a.sur_counter, 0);
  }
}

// Per-iterate error accounting: rel_out[0] = ||beta - ref|| / ||ref|| (||beta - ref||
// when ref = 0) and delta = beta - ref, either output optional.  One block; the
// sums run over a fixed thread order and a fixed tree.
__global__ __launch_bounds__(kThreads) void iter_error_kernel(const double* __restrict__ beta,
                                                              const double* __restrict__ ref, int d,
                                                              double* __restrict__ rel_out,
                                                              double* __restrict__ delta) {
  __shared__ double s_e[kThreads], s_r[kThreads];
  double e = 0.0, r = 0.0;
  for (int k = threadIdx.x; k < d; k += kThreads) {
    const double x = beta[k] - ref[k];
    if (delta) delta[k] = x;
    e += x * x;
    r += ref[k] * ref[k];
  }
  s_e[threadIdx.x] = e;
  s_r[threadIdx.x] = r;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_e[threadIdx.x] += s_e[threadIdx.x + h];
      s_r[threadIdx.x] += s_r[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && rel_out)
    rel_out[0] = s_r[0] > 0.0 ? sqrt(s_e[0] / s_r[0]) : sqrt(s_e[0]);
}

__global__ void fill_i32_kernel(int* __restrict__ p, int v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_f64_kernel(double* __restrict__ p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void copy_f64_kernel(const double* __restrict__ s, double* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 4096)); }

int rows_per_block_for(int d) {
  // about 64 blocks: each block re-reads the group partials, so fewer blocks
  // for larger d keep that traffic near the size of M itself
  int rpb = (int)ceil_div(d, 64);
  return (int)round_up(std::max(rpb, kWaves), kWaves);
}

}  // namespace

int update_blocks(int d) { return (int)ceil_div(d, rows_per_block_for(d)); }

void launch_update(const UpdateArgs& a, hipStream_t s) {
  const int rpb = rows_per_block_for(a.d);
  const int blocks = (int)ceil_div(a.d, rpb);
  const size_t shm = (size_t)a.d * sizeof(double);
  if (shm > 64 * 1024) fail(SLSE_EUNSUPPORTED, "update: d too large for this library");
  mihs_update_kernel<<<blocks, kThreads, shm, s>>>(a, rpb);
  SLSE_LAUNCH_CHECK();
}

void launch_iter_error(const double* beta, const double* ref, int d, double* rel_out,
                       double* delta, hipStream_t s) {
  iter_error_kernel<<<1, kThreads, 0, s>>>(beta, ref, d, rel_out, delta);
  SLSE_LAUNCH_CHECK();
}

void launch_fill_i32(int* dst, int value, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_i32_kernel<<<grid_for(n), 256, 0, s>>>(dst, value, n);
  SLSE_LAUNCH_CHECK();
}

void launch_fill_f64(double* dst, double value, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_f64_kernel<<<grid_for(n), 256, 0, s>>>(dst, value, n);
  SLSE_LAUNCH_CHECK();
}

void launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  copy_f64_kernel<<<grid_for(n), 256, 0, s>>>(src, dst, n);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
