// Fused residual-gradient pass g = X^T (Y - X beta) (the full-data gradient
// of eq. (99), and of eq. (98) on a sketched prefix), reading X once.
//
// Layout: a row of X is split over a group of `lpr` lanes; lane l of the group
// owns the vector chunks c*lpr + l (c < NCH) of VEC consecutive elements, so a
// wave's loads of one row are contiguous.  Per row the group forms the partial
// dot x_j . beta, all-reduces it across its lanes (xor shuffles), and every
// lane folds r_j = y_j - x_j . beta into its own slice of g.  A wave streams
// 64/lpr rows per step, UNROLL steps in flight, over one contiguous chunk of
// rows per block.  At the end the wave's row
// groups, then the block's waves, are summed; the block writes one partial
// row; the last block of every group of `group_size` blocks adds its group's
// rows in block order (deterministic for a fixed launch shape).
#include <algorithm>
#include <cstdlib>

#include "kernels.hpp"

namespace slse {
namespace {

// Build-time launch shape: threads per block and bytes in flight per lane (in
// units of 256 B) of the fully vectorised main loop.
#ifndef SLSE_RG_THREADS
#define SLSE_RG_THREADS 256
#endif
#ifndef SLSE_RG_DEPTH
#define SLSE_RG_DEPTH 1
#endif
constexpr int kThreads = SLSE_RG_THREADS;
constexpr int kWaves = kThreads / 64;
constexpr int kGroupSize = 32;  // blocks summed by the last block of each group

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T, int VEC>
struct VecT;
template <>
struct VecT<double, 2> {
  using type = f64x2;
};
template <>
struct VecT<float, 4> {
  using type = f32x4;
};
template <>
struct VecT<double, 1> {
  using type = double;
};
template <>
struct VecT<float, 1> {
  using type = float;
};

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&v)[VEC]) {
  using V = typename VecT<T, VEC>::type;
  V x = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  if constexpr (VEC == 1) {
    v[0] = x;
  } else {
#pragma unroll
    for (int i = 0; i < VEC; ++i) v[i] = x[i];
  }
}

// x widened to the accumulation type
template <typename Acc, typename T>
__device__ __forceinline__ Acc widen(T x) {
  return (Acc)x;
}

// The same, as a separate instruction the compiler cannot merge with `widen`:
// the widened row is then not kept alive from the dot to the update.
template <typename Acc, typename T>
__device__ __forceinline__ Acc widen_again(T x) {
  if constexpr (sizeof(Acc) == 8 && sizeof(T) == 4) {
    double r;
    asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
  } else {
    return (Acc)x;
  }
}

// value of lane (lane ^ m) for 32- or 64-bit values (m < 64, no width clamp)
template <typename V>
__device__ __forceinline__ V lane_xor(V v, int m, int lane) {
  const int addr = (lane ^ m) << 2;
  if constexpr (sizeof(V) == 8) {
    const long long u = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(u & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(u >> 32));
    return __builtin_bit_cast(V, ((long long)hi << 32) | (unsigned int)lo);
  } else {
    return __builtin_bit_cast(V, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
  }
}

template <typename T, int VEC, int NCH, int DEPTH = 1>
constexpr int unroll_for() {
  constexpr int bytes = NCH * VEC * (int)sizeof(T);
  constexpr int u = 256 * DEPTH / bytes;
  return u < 1 ? 1 : (u > 16 * DEPTH ? 16 * DEPTH : u);
}

// FULL: d = NCH * lpr * VEC, so every chunk is a whole vector inside the row.
template <typename T, typename Acc, int VEC, int NCH, bool HAS_Y, bool FULL>
__global__ __launch_bounds__(kThreads) void resid_grad_kernel(
    int64_t n, int d, const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y, int64_t incy,
    const double* __restrict__ beta, int lpr, double* __restrict__ partial,
    double* __restrict__ gpart, int* __restrict__ counters, int ldp,
    const int* __restrict__ done) {
  constexpr int UNROLL = unroll_for<T, VEC, NCH, FULL ? SLSE_RG_DEPTH : 1>();
  if (done && *done) return;
  __shared__ double s_red[kWaves][1025];
  __shared__ int s_ticket;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gpw = 64 / lpr;  // row groups per wave
  const int grp = lane / lpr;
  const int l = lane - grp * lpr;

  // beta slice of this lane
  Acc b[NCH][VEC];
  bool full[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int col0 = (c * lpr + l) * VEC;
    full[c] = col0 + VEC <= d;
#pragma unroll
    for (int v = 0; v < VEC; ++v) b[c][v] = (col0 + v < d) ? (Acc)beta[col0 + v] : (Acc)0;
  }

  Acc acc[NCH][VEC];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[c][v] = 0;
  Acc rr = 0;

  // each block streams one contiguous chunk of rows; at every unroll step its
  // lane groups cover `rs` consecutive rows
  const int rs = kWaves * gpw;
  const int64_t chunk = round_up(ceil_div(n, (int64_t)gridDim.x), rs);
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(n, r0 + chunk);

  int64_t base = r0 + wave * gpw + grp;
  if constexpr (FULL) {
    // main loop: every row of the step is in range for the whole wave (the
    // bound is wave-uniform), so the loads carry no guards and no branches
    const int64_t wave_base0 = r0 + wave * gpw;
    const int64_t last_off = (int64_t)(gpw - 1) + (int64_t)(UNROLL - 1) * rs;
    int64_t wb = wave_base0;
    for (; wb + last_off < r1; wb += (int64_t)rs * UNROLL) {
      const int64_t row0 = wb + grp;
      T x[UNROLL][NCH][VEC];
      T y[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const T* xr = X + (row0 + (int64_t)u * rs) * ldx;
#pragma unroll
        for (int c = 0; c < NCH; ++c) load_vec<T, VEC>(xr + (c * lpr + l) * VEC, x[u][c]);
        if constexpr (HAS_Y) {
          y[u] = __builtin_nontemporal_load(Y + (row0 + (int64_t)u * rs) * incy);
        } else {
          y[u] = 0;
        }
      }
      // partial dots row by row (the widened values of a row die with its dot)
      Acc dot[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        __builtin_amdgcn_sched_barrier(0);
        Acc p0 = 0, p1 = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            if ((c * VEC + v) & 1)
              p1 = fma(widen<Acc>(x[u][c][v]), b[c][v], p1);
            else
              p0 = fma(widen<Acc>(x[u][c][v]), b[c][v], p0);
          }
        dot[u] = p0 + p1;
      }
      __builtin_amdgcn_sched_barrier(0);
      // all-reduce the rows' dots inside each lane group, the rows interleaved
      for (int m = lpr >> 1; m > 0; m >>= 1) {
        Acc o[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) o[u] = lane_xor(dot[u], m, lane);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) dot[u] += o[u];
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const Acc r = (Acc)y[u] - dot[u];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[c][v] = fma(r, widen_again<Acc>(x[u][c][v]), acc[c][v]);
        rr = fma(r, r, rr);
      }
    }
    // tail: one row per lane group at a time, whole vectors, row guard only
    for (int64_t row = wb + grp; row < r1; row += rs) {
      const T* xr = X + row * ldx;
      T x[NCH][VEC];
#pragma unroll
      for (int c = 0; c < NCH; ++c) load_vec<T, VEC>(xr + (c * lpr + l) * VEC, x[c]);
      T y0 = 0;
      if constexpr (HAS_Y) y0 = Y[row * incy];
      Acc dot = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) dot = fma((Acc)x[c][v], b[c][v], dot);
      // lanes of a group share the row, so the group's shuffles stay inside
      // lanes that are all active
      dot = lane_group_sum(dot, lpr);
      const Acc r = (Acc)y0 - dot;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[c][v] = fma(r, (Acc)x[c][v], acc[c][v]);
      rr = fma(r, r, rr);
    }
    base = r1;  // nothing left for the guarded loop
  }
  // guarded loop (every row when not FULL)
  for (; base < r1; base += (int64_t)rs * UNROLL) {
    T x[UNROLL][NCH][VEC];
    T y[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t row = base + (int64_t)u * rs;
      const bool ok = row < r1;
      const T* xr = X + (ok ? row : 0) * ldx;
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
      if constexpr (HAS_Y) {
        y[u] = ok ? Y[row * incy] : (T)0;
      } else {
        y[u] = 0;
      }
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      Acc dot = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) dot = fma((Acc)x[u][c][v], b[c][v], dot);
      dot = lane_group_sum(dot, lpr);
      const Acc r = (Acc)y[u] - dot;  // zero for rows past n (x = y = 0)
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[c][v] = fma(r, (Acc)x[u][c][v], acc[c][v]);
      rr = fma(r, r, rr);
    }
  }

  // sum the wave's row groups: lanes with equal l hold the same columns
  double accd[NCH][VEC];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      double t = (double)acc[c][v];
      for (int m = lpr; m < 64; m <<= 1) t += wave_xor(t, m);
      accd[c][v] = t;
    }
  double rrd = (double)rr;  // every lane of a group holds the same r: count lane l == 0 only
  rrd = (l == 0) ? rrd : 0.0;
  for (int m = 1; m < 64; m <<= 1) rrd += wave_xor(rrd, m);

  // block reduction through LDS (columns d.. handled by the spill loop below)
  double* prow = partial + (int64_t)blockIdx.x * ldp;
  for (int c0 = 0; c0 < d + 1; c0 += 1024) {
    if (grp == 0) {
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int col = (c * lpr + l) * VEC + v;
          if (col >= c0 && col < c0 + 1024 && col < d) s_red[wave][col - c0] = accd[c][v];
        }
      if (l == 0 && d >= c0 && d < c0 + 1024) s_red[wave][d - c0] = rrd;
    }
    __syncthreads();
    for (int col = c0 + threadIdx.x; col < min(d + 1, c0 + 1024); col += kThreads) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += s_red[w][col - c0];
      store_device(prow + col, t);
    }
    __syncthreads();
  }

  // last block of the group sums the group's partial rows in block order
  wait_memory();
  __syncthreads();
  const int group = blockIdx.x / kGroupSize;
  const int g0 = group * kGroupSize;
  const int gsz = min(kGroupSize, (int)gridDim.x - g0);
  if (threadIdx.x == 0) {
    s_ticket = take_ticket(&counters[group]);
    if (s_ticket == gsz - 1) acquire_partials();
  }
  __syncthreads();
  if (s_ticket == gsz - 1) {
    for (int col = threadIdx.x; col < d + 1; col += kThreads) {
      double v[kGroupSize];
#pragma unroll
      for (int bk = 0; bk < kGroupSize; ++bk)
        v[bk] = bk < gsz ? load_device(partial + (int64_t)(g0 + bk) * ldp + col) : 0.0;
      double t = 0.0;
#pragma unroll
      for (int bk = 0; bk < kGroupSize; ++bk) t += v[bk];
      gpart[(int64_t)group * ldp + col] = t;
    }
    if (threadIdx.x == 0) atomicExch(&counters[group], 0);
  }
}

__global__ void finalize_grad_kernel(const double* __restrict__ gpart, int groups, int ldp, int d,
                                     double scale, double* __restrict__ g, double* __restrict__ rn) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col > d) return;
  double t = 0.0;
  for (int k = 0; k < groups; ++k) t += gpart[(int64_t)k * ldp + col];
  if (col < d) {
    g[col] = scale * t;
  } else if (rn) {
    rn[0] = scale * t;
  }
}

template <typename T, typename Acc, int VEC, int NCH, bool FULL>
void launch_t(const ResidGradPlan& pl, const ResidGradArgs& a, hipStream_t s) {
  const T* X = static_cast<const T*>(a.X);
  const T* Y = static_cast<const T*>(a.Y);
  if (Y) {
    resid_grad_kernel<T, Acc, VEC, NCH, true, FULL><<<pl.blocks, kThreads, 0, s>>>(
        a.n, a.d, X, a.ldx, Y, a.incy, a.beta, pl.lpr, a.partial, a.gpart, a.counters, pl.ldp,
        a.done);
  } else {
    resid_grad_kernel<T, Acc, VEC, NCH, false, FULL><<<pl.blocks, kThreads, 0, s>>>(
        a.n, a.d, X, a.ldx, Y, a.incy, a.beta, pl.lpr, a.partial, a.gpart, a.counters, pl.ldp,
        a.done);
  }
}

template <typename T, typename Acc, int VEC, bool FULL>
void launch_nch(const ResidGradPlan& pl, const ResidGradArgs& a, hipStream_t s) {
  switch (pl.nch) {
    case 1: launch_t<T, Acc, VEC, 1, FULL>(pl, a, s); break;
    case 2: launch_t<T, Acc, VEC, 2, FULL>(pl, a, s); break;
    case 4: launch_t<T, Acc, VEC, 4, FULL>(pl, a, s); break;
    case 8: launch_t<T, Acc, VEC, 8, FULL>(pl, a, s); break;
    case 16: launch_t<T, Acc, VEC, 16, FULL>(pl, a, s); break;
    default: fail(SLSE_EUNSUPPORTED, "resid_grad: unsupported chunk count");
  }
}

template <typename T, typename Acc>
void launch_vec(const ResidGradPlan& pl, const ResidGradArgs& a, hipStream_t s) {
  constexpr int V = 16 / sizeof(T);
  if (pl.vec == V) {
    if (pl.full)
      launch_nch<T, Acc, V, true>(pl, a, s);
    else
      launch_nch<T, Acc, V, false>(pl, a, s);
  } else {
    launch_nch<T, Acc, 1, false>(pl, a, s);
  }
}

}  // namespace

ResidGradPlan plan_resid_grad(int64_t n, int d, slse_dtype storage, const void* X, int64_t ldx,
                              int grid_blocks, int capacity, int lpr_hint) {
  ResidGradPlan pl;
  const int es = (int)dtype_size(storage);
  const int vfull = 16 / es;
  const bool aligned = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((ldx * es) % 16 == 0);
  pl.vec = aligned ? vfull : 1;
  const int nvec = (int)ceil_div(d, pl.vec);
  // default: about eight vector chunks per lane (measured best for wide rows);
  // lane groups are powers of 2 up to a wave
  int lpr = 1;
  while (lpr < 64 && lpr * 16 <= nvec) lpr *= 2;
  if (lpr_hint > 0) lpr = lpr_hint;
  if (const char* e = std::getenv("SLSE_RG_LPR")) lpr = std::atoi(e);
  lpr = std::max(1, std::min(64, lpr));
  while (lpr & (lpr - 1)) lpr &= lpr - 1;
  int nch = (int)ceil_div(nvec, lpr);
  int p2 = 1;
  while (p2 < nch) p2 *= 2;
  while (p2 > 16 && lpr < 64) {  // too many chunks: widen the lane group
    lpr *= 2;
    nch = (int)ceil_div(nvec, lpr);
    p2 = 1;
    while (p2 < nch) p2 *= 2;
  }
  if (p2 > 16) fail(SLSE_EUNSUPPORTED, "resid_grad: d too large for this build");
  pl.lpr = lpr;
  pl.nch = p2;
  pl.full = pl.vec > 1 && d % pl.vec == 0 && (int64_t)p2 * lpr * pl.vec == d;
  if (const char* e = std::getenv("SLSE_RG_FULL")) pl.full = pl.full && std::atoi(e) != 0;
  pl.ldp = (int)round_up(d + 1, 8);
  const int rows_per_block_step = kWaves * (64 / lpr);
  const int bytes_per_vec = pl.vec * es;
  const int unroll = std::max(1, std::min(16, 256 / (p2 * bytes_per_vec)));
  // an override may choose another grid, never one above the capacity the
  // partial rows and group counters were allocated for
  int target = std::min(grid_blocks, capacity);
  if (const char* e = std::getenv("SLSE_RG_BLOCKS"))
    target = std::max(1, std::min(capacity, std::atoi(e)));
  int64_t want = ceil_div(std::max<int64_t>(n, 1), (int64_t)rows_per_block_step * unroll);
  pl.blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, target));
  pl.group_size = kGroupSize;
  pl.groups = (int)ceil_div(pl.blocks, pl.group_size);
  return pl;
}

void launch_resid_grad(const ResidGradPlan& pl, const ResidGradArgs& a, hipStream_t s) {
  if (pl.blocks > a.capacity_blocks || pl.groups > ceil_div(a.capacity_blocks, pl.group_size))
    fail(SLSE_EINVAL, "resid_grad: plan exceeds the scratch capacity");
  if (a.storage == SLSE_F64) {
    if (a.accum == SLSE_F64)
      launch_vec<double, double>(pl, a, s);
    else
      launch_vec<double, float>(pl, a, s);
  } else if (a.storage == SLSE_F32) {
    if (a.accum == SLSE_F64)
      launch_vec<float, double>(pl, a, s);
    else
      launch_vec<float, float>(pl, a, s);
  } else {
    fail(SLSE_EUNSUPPORTED, "resid_grad: storage must be F32 or F64");
  }
  SLSE_LAUNCH_CHECK();
}

void launch_finalize_grad(const double* gpart, int groups, int ldp, int d, double scale,
                          double* g_out, double* rnorm2_out, hipStream_t s) {
  const int threads = 256;
  finalize_grad_kernel<<<(int)ceil_div(d + 1, threads), threads, 0, s>>>(gpart, groups, ldp, d,
                                                                         scale, g_out, rnorm2_out);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
