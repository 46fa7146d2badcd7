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

template <typename T, int VEC>
using vec_of = T __attribute__((ext_vector_type(VEC)));

// VEC elements at p (16-byte vector loads/stores when VEC > 1), streamed past
// the caches
template <typename T, int VEC>
__device__ __forceinline__ void load_chunk(const T* __restrict__ p, T (&v)[VEC]) {
  if constexpr (VEC == 1) {
    v[0] = __builtin_nontemporal_load(p);
  } else {
    const vec_of<T, VEC> t = __builtin_nontemporal_load(reinterpret_cast<const vec_of<T, VEC>*>(p));
#pragma unroll
    for (int k = 0; k < VEC; ++k) v[k] = t[k];
  }
}
template <typename G, int VEC>
__device__ __forceinline__ void store_chunk(G* __restrict__ p, const G (&v)[VEC]) {
  if constexpr (VEC == 1) {
    __builtin_nontemporal_store(v[0], p);
  } else {
    vec_of<G, VEC> t;
#pragma unroll
    for (int k = 0; k < VEC; ++k) t[k] = v[k];
    __builtin_nontemporal_store(t, reinterpret_cast<vec_of<G, VEC>*>(p));
  }
}

// rows of [X|Y] a lane keeps in flight: about 128 bytes of X per lane
template <typename T, int VEC, int NCH>
constexpr int adjoint_unroll() {
  constexpr int u = 128 / (NCH * VEC * (int)sizeof(T));
  return u < 1 ? 1 : (u > 8 ? 8 : u);
}

// A row is split over `lpr` lanes, each holding NCH chunks of VEC columns
// (column (c lpr + l) VEC + k); a block handles tiles of UNROLL x (rows per
// block step) rows, every lane group keeping UNROLL rows in flight.  With
// VEC > 1, d is a multiple of VEC and X, dX rows are VEC-aligned.
template <typename T, typename G, int VEC, int NCH>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(int64_t n, int d, const T* __restrict__ X,
                                                           int64_t ldx, const T* __restrict__ Y,
                                                           const double* __restrict__ beta,
                                                           const double* __restrict__ lambda,
                                                           int lpr, G* __restrict__ dX, int64_t lddx,
                                                           G* __restrict__ dY) {
  constexpr int UNROLL = adjoint_unroll<T, VEC, NCH>();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gpw = 64 / lpr;
  const int grp = lane / lpr;
  const int l = lane - grp * lpr;
  double b[NCH][VEC], lam[NCH][VEC];
  bool inside[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int col0 = (c * lpr + l) * VEC;
    inside[c] = col0 < d;
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      b[c][k] = inside[c] ? beta[col0 + k] : 0.0;
      lam[c][k] = inside[c] ? lambda[col0 + k] : 0.0;
    }
  }
  const int step = kWaves * gpw;  // rows per block step
  const int64_t tile = (int64_t)step * UNROLL;
  const int my = wave * gpw + grp;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    T x[UNROLL][NCH][VEC];
    double y[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t row = base + (int64_t)u * step + my;
      const bool ok = row < n;
      const T* xr = X + (ok ? row : 0) * ldx;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        if (ok && inside[c]) {
          load_chunk<T, VEC>(xr + (c * lpr + l) * VEC, x[u][c]);
        } else {
#pragma unroll
          for (int k = 0; k < VEC; ++k) x[u][c][k] = (T)0;
        }
      }
      y[u] = (Y && ok) ? (double)Y[row] : 0.0;
    }
    double d1[UNROLL], d2[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          s1 = fma((double)x[u][c][k], b[c][k], s1);
          s2 = fma((double)x[u][c][k], lam[c][k], s2);
        }
      d1[u] = s1;
      d2[u] = s2;
    }
    for (int m = lpr >> 1; m > 0; m >>= 1) {
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        d1[u] += wave_xor(d1[u], m);
        d2[u] += wave_xor(d2[u], m);
      }
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t row = base + (int64_t)u * step + my;
      if (row >= n) continue;
      const double r = y[u] - d1[u];
      if (dX) {
        G* out = dX + row * lddx;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          if (!inside[c]) continue;
          G o[VEC];
#pragma unroll
          for (int k = 0; k < VEC; ++k) o[k] = (G)(r * lam[c][k] - d2[u] * b[c][k]);
          store_chunk<G, VEC>(out + (c * lpr + l) * VEC, o);
        }
      }
      if (dY && l == 0) dY[row] = (G)d2[u];
    }
  }
}

template <typename T, typename G, int VEC, int NCH>
void launch4(const AdjointArgs& a, int lpr, hipStream_t s) {
  const int64_t tile = (int64_t)kWaves * (64 / lpr) * adjoint_unroll<T, VEC, NCH>();
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(a.n, tile), 2048));
  adjoint_kernel<T, G, VEC, NCH><<<blocks, kThreads, 0, s>>>(
      a.n, a.d, static_cast<const T*>(a.X), a.ldx, static_cast<const T*>(a.Y), a.beta, a.lambda,
      lpr, static_cast<G*>(a.dX), a.lddx, static_cast<G*>(a.dY));
  SLSE_LAUNCH_CHECK();
}

template <typename T, typename G, int VEC>
void launch3(const AdjointArgs& a, hipStream_t s) {
  // lane groups of at most a wave, about four chunks per lane
  const int nvec = (int)ceil_div(a.d, VEC);
  int lpr = 1;
  while (lpr < 64 && lpr * 4 < nvec) lpr *= 2;
  const int nch = (int)ceil_div(nvec, lpr);
  if (nch <= 1)
    launch4<T, G, VEC, 1>(a, lpr, s);
  else if (nch <= 2)
    launch4<T, G, VEC, 2>(a, lpr, s);
  else if (nch <= 4)
    launch4<T, G, VEC, 4>(a, lpr, s);
  else if (nch <= 8)
    launch4<T, G, VEC, 8>(a, lpr, s);
  else if (nch <= 16)
    launch4<T, G, VEC, 16>(a, lpr, s);
  else
    fail(SLSE_EUNSUPPORTED, "adjoint: d too large for this library");
}

template <typename T, typename G>
void launch2(const AdjointArgs& a, hipStream_t s) {
  // 16-byte chunks when every row of X and dX starts on such a boundary
  constexpr int V = 16 / (int)sizeof(T);
  auto aligned = [](const void* p, int64_t ld, size_t es) {
    return p == nullptr ||
           (reinterpret_cast<uintptr_t>(p) % (V * es) == 0 && (ld * (int64_t)es) % (V * (int64_t)es) == 0);
  };
  if (a.d % V == 0 && aligned(a.X, a.ldx, sizeof(T)) && aligned(a.dX, a.lddx, sizeof(G)))
    launch3<T, G, V>(a, s);
  else
    launch3<T, G, 1>(a, s);
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
