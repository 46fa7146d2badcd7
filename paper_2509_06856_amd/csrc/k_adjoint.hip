// Fused rank-2 adjoint pass.  For L with dL/dbeta_hat = w and
// lambda = (X^T X)^{-1} w, differentiating the normal equations X^T X
// beta_hat = X^T Y (problem statement, Sec. 1) gives per row j
//     u_j = x_j . lambda,  r_j = y_j - x_j . beta_hat,
//     dY_j = u_j,          dX_j = r_j lambda^T - u_j beta_hat^T.
// One read of [x_j | y_j], one write of [dX_j | dY_j]; both dots accumulate in
// FP64.  Row split over lane groups as in the residual-gradient pass.
#include <algorithm>

#include "kernels.hpp"
#include "rng.hpp"

namespace slse {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename T, typename G, int NCH>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(int64_t n, int d, const T* __restrict__ X,
                                                           int64_t ldx, const T* __restrict__ Y,
                                                           const double* __restrict__ beta,
                                                           const double* __restrict__ lambda,
                                                           int lpr, G* __restrict__ dX, int64_t lddx,
                                                           G* __restrict__ dY) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gpw = 64 / lpr;
  const int grp = lane / lpr;
  const int l = lane - grp * lpr;
  double b[NCH], lam[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int col = c * lpr + l;
    b[c] = col < d ? beta[col] : 0.0;
    lam[c] = col < d ? lambda[col] : 0.0;
  }
  const int64_t stride = (int64_t)gridDim.x * kWaves * gpw;
  for (int64_t row = ((int64_t)blockIdx.x * kWaves + wave) * gpw + grp; row < n; row += stride) {
    const T* xr = X + row * ldx;
    double x[NCH];
    double d1 = 0.0, d2 = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int col = c * lpr + l;
      x[c] = col < d ? (double)__builtin_nontemporal_load(xr + col) : 0.0;
      d1 = fma(x[c], b[c], d1);
      d2 = fma(x[c], lam[c], d2);
    }
    d1 = lane_group_sum(d1, lpr);
    d2 = lane_group_sum(d2, lpr);
    const double r = (Y ? (double)Y[row] : 0.0) - d1;
    if (dX) {
      G* out = dX + row * lddx;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int col = c * lpr + l;
        if (col < d) __builtin_nontemporal_store((G)(r * lam[c] - d2 * b[c]), out + col);
      }
    }
    if (dY && l == 0) dY[row] = (G)d2;
  }
}

template <typename T, typename G, int NCH>
void launch3(const AdjointArgs& a, int lpr, hipStream_t s) {
  const int rows_per_block = kWaves * (64 / lpr);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(a.n, rows_per_block), 4096));
  adjoint_kernel<T, G, NCH><<<blocks, kThreads, 0, s>>>(
      a.n, a.d, static_cast<const T*>(a.X), a.ldx, static_cast<const T*>(a.Y), a.beta, a.lambda,
      lpr, static_cast<G*>(a.dX), a.lddx, static_cast<G*>(a.dY));
  SLSE_LAUNCH_CHECK();
}

template <typename T, typename G>
void launch2(const AdjointArgs& a, hipStream_t s) {
  int lpr = 1;
  while (lpr < 64 && lpr * 4 <= a.d) lpr *= 2;
  const int nch = (int)ceil_div(a.d, lpr);
  if (nch <= 4)
    launch3<T, G, 4>(a, lpr, s);
  else if (nch <= 8)
    launch3<T, G, 8>(a, lpr, s);
  else if (nch <= 16)
    launch3<T, G, 16>(a, lpr, s);
  else if (nch <= 32)
    launch3<T, G, 32>(a, lpr, s);
  else
    fail(SLSE_EUNSUPPORTED, "adjoint: d too large for this build");
}

// ---------------------------------------------------------------------------
// Test hook: the counter streams as the device computes them.
// ---------------------------------------------------------------------------
__global__ void debug_stream_kernel(int what, uint64_t seed, int stream_id, int64_t aux,
                                    int64_t start, int64_t count, int64_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t x = (uint64_t)(start + i);
    switch (what) {
      case 0: {
        rng::Words w = rng::philox(x, (uint64_t)aux, 0, 0, seed, (uint64_t)stream_id);
        for (int k = 0; k < 4; ++k) out[4 * i + k] = (int64_t)w.w[k];
        break;
      }
      case 1: out[i] = (int64_t)rng::prp(x, seed, (uint64_t)stream_id, (int)aux); break;
      case 2: out[i] = (int64_t)rng::prp_inv(x, seed, (uint64_t)stream_id, (int)aux); break;
      case 3: out[i] = rng::rademacher(seed, x); break;
      case 4:
      case 5: {
        uint64_t bkt;
        int sg;
        rng::cs_hash(seed, x, (uint64_t)aux - 1, bkt, sg);
        out[i] = what == 4 ? (int64_t)bkt : sg;
        break;
      }
      default: {
        uint64_t bkt;
        int sg;
        rng::cs_hash_hat(seed, x, (uint64_t)aux, bkt, sg);
        out[i] = what == 6 ? (int64_t)bkt : sg;
        break;
      }
    }
  }
}

}  // namespace

void launch_adjoint(const AdjointArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  if (a.t == SLSE_F64 && a.gt == SLSE_F64)
    launch2<double, double>(a, s);
  else if (a.t == SLSE_F32 && a.gt == SLSE_F32)
    launch2<float, float>(a, s);
  else if (a.t == SLSE_F32 && a.gt == SLSE_F64)
    launch2<float, double>(a, s);
  else if (a.t == SLSE_F64 && a.gt == SLSE_F32)
    launch2<double, float>(a, s);
  else
    fail(SLSE_EUNSUPPORTED, "adjoint: dtype");
}

void launch_debug_stream(int what, uint64_t seed, int stream_id, int64_t aux, int64_t start,
                         int64_t count, int64_t* out, hipStream_t s) {
  if (count <= 0) return;
  const int blocks = (int)std::min<int64_t>(ceil_div(count, 256), 4096);
  debug_stream_kernel<<<blocks, 256, 0, s>>>(what, seed, stream_id, aux, start, count, out);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
