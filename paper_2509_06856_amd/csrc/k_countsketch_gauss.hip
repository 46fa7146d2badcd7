// CountSketch and Gaussian sketches of [X|Y] (Sec. 1.2; CountSketch as the
// alternative sketching matrix of Sec. 5.4).
//
// CountSketch: column j of S_K has the single entry s(j) in row h(j), so
// S_K [X|Y] adds s(j) [x_j | y_j] into bucket h(j).  Instead of scattering
// rows with float atomics, the rows are first listed per bucket (integer
// counts, an exclusive scan, a fill that writes each row's index with its
// sign folded in), and each output row is then gathered: one wave per bucket
// of the largest level (m_K buckets, a few rows each) and several waves per
// bucket of the Hessian sketch (r buckets, about N/r rows each; their partial
// rows are added in a fixed order).  Smaller levels use the bucket h(j) mod
// m_i, so level i is level i+1 folded in halves: A_i[k] = sum_{t = k mod m_i}
// A_{i+1}[t].  The order of the rows inside a bucket list is set by the fill's
// atomics, so sums agree with any other order to rounding, not bit for bit.
//
// Gaussian: A = G [X|Y] with G_kj iid N(0, 1) drawn on the fly (Philox block
// (j, k >> 3) -> four Box-Muller pairs).  Tiled 64 (sketch rows) x 64
// (columns) per block with the N rows split over blocks; partial tiles are
// summed in split order by a second kernel.  FP64 data accumulates in FP64,
// FP32 data in FP32.
#include <algorithm>
#include <cstdlib>

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

constexpr int kHistLds = 8192;  // Hessian buckets counted in LDS up to this many

// bucket sizes of the largest level (DO_K) and of S_hat (HAT)
template <bool LDS_H, bool HAT, bool DO_K = true>
__global__ __launch_bounds__(kThreads) void cs_count_kernel(int64_t n, uint64_t seed,
                                                            uint64_t mK_mask, int64_t r,
                                                            int* __restrict__ cntK,
                                                            int* __restrict__ cntH) {
  __shared__ int hist[LDS_H && HAT ? kHistLds : 1];
  if constexpr (LDS_H && HAT) {
    for (int k = threadIdx.x; k < r; k += kThreads) hist[k] = 0;
    __syncthreads();
  }
  for (int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kThreads) {
    if constexpr (DO_K) {
      uint64_t h;
      int sg;
      rng::cs_hash(seed, (uint64_t)j, mK_mask, h, sg);
      atomicAdd(cntK + h, 1);
    }
    if constexpr (HAT) {
      uint64_t hh;
      int sh;
      rng::cs_hash_hat(seed, (uint64_t)j, (uint64_t)r, hh, sh);
      if constexpr (LDS_H)
        atomicAdd(hist + hh, 1);
      else
        atomicAdd(cntH + hh, 1);
    }
  }
  if constexpr (LDS_H && HAT) {
    __syncthreads();
    for (int k = threadIdx.x; k < r; k += kThreads)
      if (hist[k]) atomicAdd(cntH + k, hist[k]);
  }
}

// The Hessian buckets' lists in row order, without atomics on their (hot)
// cursors: wave w owns the contiguous rows [w C, (w + 1) C).  It counts its
// rows per bucket; a scan over the waves of every bucket gives each wave the
// first slot of its rows in every bucket; the wave then lists its rows in
// order, 64 at a time (a row's place among the batch's rows of its bucket
// comes from comparing buckets across the lanes).  Up to kHistLds buckets.
constexpr int kHatWaves = 1024;

// per wave: its rows' counts per bucket (cntW row w), and the bucket sizes
// (integer sums: the order of the additions does not matter)
__global__ __launch_bounds__(64) void cs_hat_count_kernel(int64_t n, int64_t chunk, uint64_t seed,
                                                          int64_t r, int* __restrict__ cntW,
                                                          int* __restrict__ cntH) {
  __shared__ int hist[kHistLds];
  for (int k = threadIdx.x; k < r; k += 64) hist[k] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 64) {
    uint64_t hh;
    int sh;
    rng::cs_hash_hat(seed, (uint64_t)j, (uint64_t)r, hh, sh);
    atomicAdd(hist + hh, 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < r; k += 64) {
    const int c = hist[k];
    cntW[(int64_t)blockIdx.x * r + k] = c;
    if (c) atomicAdd(cntH + k, c);
  }
}

// per bucket: the exclusive scan of the bucket totals (written to off, with
// off[r] = their sum) and the first slot of every wave's rows (in place over
// the counts).  A block takes 64 buckets: its threads first sum the totals
// before them and one wave scans its 64; then its 16 waves each sum a
// sixteenth of the waves' rows (lanes on consecutive buckets: coalesced), the
// sixteen partial sums are scanned in LDS, and every wave writes its rows'
// running starts.  Integer sums: exact in any order.
constexpr int kColTile = 64;
__global__ __launch_bounds__(1024) void cs_colscan_kernel(int64_t r, int waves,
                                                          int* __restrict__ cntW,
                                                          const int* __restrict__ tot,
                                                          int* __restrict__ off) {
  __shared__ int part[16][kColTile];
  __shared__ int red[16];
  __shared__ int base[kColTile];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kColTile;
  const int64_t k = c0 + lane;
  int pre = 0;
  for (int64_t e = threadIdx.x; e < c0; e += 1024) pre += tot[e];
  for (int m = 32; m > 0; m >>= 1) pre += __shfl_xor(pre, m, 64);
  if (lane == 0) red[g] = pre;
  __syncthreads();
  if (g == 0) {
    int p0 = 0;
    for (int h = 0; h < 16; ++h) p0 += red[h];
    const int t = k < r ? tot[k] : 0;
    int incl = t;
    for (int m = 1; m < 64; m <<= 1) {
      const int v = __shfl_up(incl, m, 64);
      if (lane >= m) incl += v;
    }
    base[lane] = p0 + incl - t;
    if (k < r) off[k] = p0 + incl - t;
    if (k == r - 1) off[r] = p0 + incl;
  }
  // (both walks over the waves' rows load 16 counts at a time, so that their
  // loads are in flight together instead of one after another)
  constexpr int kB = 16;
  const int per = (waves + 15) / 16;
  const int w0 = g * per, w1 = min(waves, w0 + per);
  int t = 0;
  if (k < r) {
    int w = w0;
    for (; w + kB <= w1; w += kB) {
      int v[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) v[u] = cntW[(int64_t)(w + u) * r + k];
#pragma unroll
      for (int u = 0; u < kB; ++u) t += v[u];
    }
    for (; w < w1; ++w) t += cntW[(int64_t)w * r + k];
  }
  part[g][lane] = t;
  __syncthreads();
  if (k < r) {
    int run = base[lane];
    for (int h = 0; h < g; ++h) run += part[h][lane];
    int w = w0;
    for (; w + kB <= w1; w += kB) {
      int v[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) v[u] = cntW[(int64_t)(w + u) * r + k];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        cntW[(int64_t)(w + u) * r + k] = run;
        run += v[u];
      }
    }
    for (; w < w1; ++w) {
      const int c = cntW[(int64_t)w * r + k];
      cntW[(int64_t)w * r + k] = run;
      run += c;
    }
  }
}

// The largest level's lists by a stable two-pass counting sort of the rows
// on their bucket h(j) (low digit, then high digit of at most kDigitBits
// bits each), each pass in the per-wave scheme above: every wave owns a
// contiguous range of positions, counts it per digit, a scan over the waves
// of every digit gives it its first slots, and it writes its positions in
// order.  The result lists every bucket's rows in increasing row order with
// no atomic slot claims.
constexpr int kDigitBits = 11;
constexpr int kDigits = 1 << kDigitBits;
constexpr int64_t kRadixRows = int64_t(1) << 21;  // the sort pays off from here (measured)

// the rank of this lane among the batch's lanes with the same digit, and
// whether it is the last of them (one ballot per digit bit)
__device__ __forceinline__ void digit_rank(int dg, bool valid, int bits, int& before, bool& last) {
  const int lane = threadIdx.x & 63;
  uint64_t same = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const uint64_t ones = __ballot((dg >> b) & 1);
    same &= ((dg >> b) & 1) ? ones : ~ones;
  }
  const uint64_t below = (uint64_t(1) << lane) - 1;
  before = __popcll(same & below);
  last = (same & ~below & ~(uint64_t(1) << lane)) == 0;
}

// PASS 0 draws the rows' buckets (digit = low bits); PASS 1 reads the first
// pass's keys (digit = the bits above shift)
template <int PASS>
__global__ __launch_bounds__(64) void cs_digit_count_kernel(int64_t n, int64_t chunk, uint64_t seed,
                                                            uint64_t mK_mask, int shift, int bits,
                                                            const int* __restrict__ keys,
                                                            int* __restrict__ cntW,
                                                            int* __restrict__ tot) {
  __shared__ int hist[kDigits];
  const int nd = 1 << bits;
  for (int k = threadIdx.x; k < nd; k += 64) hist[k] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  if constexpr (PASS == 0) {
    for (int64_t j = j0 + threadIdx.x; j < j1; j += 64) {
      uint64_t h;
      int sg;
      rng::cs_hash(seed, (uint64_t)j, mK_mask, h, sg);
      atomicAdd(hist + (((int)h >> shift) & (nd - 1)), 1);
    }
  } else {
    // four rows per thread per round, their loads in flight together
    for (int64_t jb = j0 + threadIdx.x; jb < j1; jb += 256) {
      int key[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) key[u] = jb + 64 * u < j1 ? keys[jb + 64 * u] : -1;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (key[u] >= 0) atomicAdd(hist + ((key[u] >> shift) & (nd - 1)), 1);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nd; k += 64) {
    const int c = hist[k];
    cntW[(int64_t)blockIdx.x * nd + k] = c;
    if (c) atomicAdd(tot + k, c);
  }
}

// PASS 0: writes (bucket, entry) of every row in low-digit order; PASS 1:
// moves them into high-digit order, writing the entries (the lists) and the
// buckets in the final order
template <int PASS>
__global__ __launch_bounds__(64) void cs_digit_fill_kernel(int64_t n, int64_t chunk, uint64_t seed,
                                                           uint64_t mK_mask, int shift, int bits,
                                                           const int* __restrict__ offW,
                                                           const int* __restrict__ keys_in,
                                                           const int* __restrict__ vals_in,
                                                           int* __restrict__ keys_out,
                                                           int* __restrict__ vals_out) {
  __shared__ int cur[kDigits];
  const int lane = threadIdx.x;
  const int nd = 1 << bits;
  for (int k = lane; k < nd; k += 64) cur[k] = offW[(int64_t)blockIdx.x * nd + k];
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  for (int64_t jb = j0; jb < j1; jb += 64) {
    const int64_t j = jb + lane;
    const bool valid = j < j1;
    int key = 0, val = 0;
    if (valid) {
      if constexpr (PASS == 0) {
        uint64_t h;
        int sg;
        rng::cs_hash(seed, (uint64_t)j, mK_mask, h, sg);
        key = (int)h;
        val = sg > 0 ? (int)j : ~(int)j;
      } else {
        key = keys_in[j];
        val = vals_in[j];
      }
    }
    const int dg = (key >> shift) & (nd - 1);
    int before;
    bool last;
    digit_rank(dg, valid, bits, before, last);
    if (valid) {
      // every lane reads its cursor before any lane writes one (one wave)
      const int slot = cur[dg] + before;
      keys_out[slot] = key;
      vals_out[slot] = val;
      if (last) cur[dg] = slot + 1;
    }
  }
}

// bucket starts from the bucket-sorted keys: position i starts every bucket
// in (key[i-1], key[i]], and the buckets past the last key start at n
__global__ void cs_starts_kernel(int64_t n, int64_t nb, const int* __restrict__ keys,
                                 int* __restrict__ off) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = i == 0 ? 0 : (int64_t)keys[i - 1] + 1;
    const int64_t hi = i == n ? nb : (int64_t)keys[i];
    for (int64_t k = lo; k <= hi; ++k) off[k] = (int)i;
  }
}

__global__ __launch_bounds__(64) void cs_hat_fill_kernel(int64_t n, int64_t chunk, uint64_t seed,
                                                         int64_t r, int bits,
                                                         const int* __restrict__ offW,
                                                         int* __restrict__ listH) {
  __shared__ int cur[kHistLds];
  const int lane = threadIdx.x;
  for (int k = lane; k < r; k += 64) cur[k] = offW[(int64_t)blockIdx.x * r + k];
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  for (int64_t jb = j0; jb < j1; jb += 64) {
    const int64_t j = jb + lane;
    int hh = -1, sh = 1;
    if (j < j1) {
      uint64_t b;
      rng::cs_hash_hat(seed, (uint64_t)j, (uint64_t)r, b, sh);
      hh = (int)b;
    }
    // lanes with the same bucket: one ballot per bucket bit, and the valid lanes
    uint64_t same = __ballot(hh >= 0);
    for (int b = 0; b < bits; ++b) {
      const uint64_t ones = __ballot((hh >> b) & 1);
      same &= ((hh >> b) & 1) ? ones : ~ones;
    }
    const uint64_t below = (uint64_t(1) << lane) - 1;
    const int before = __popcll(same & below);
    const int after = __popcll(same & ~below & ~(uint64_t(1) << lane));
    if (hh >= 0) {
      // every lane reads its cursor before any lane writes one (one wave:
      // its LDS accesses take effect in program order)
      const int slot = cur[hh] + before;
      listH[slot] = sh > 0 ? (int)j : ~(int)j;
      if (after == 0) cur[hh] = slot + 1;  // the batch's last row in this bucket
    }
  }
}

// The Hessian lists and the first (low-digit) pass of the largest level's
// counting sort in one pass over the rows: both walk the same per-wave row
// ranges, so one kernel hashes each row once for the count and once for the
// fill.  Count: per wave, its rows per Hessian bucket (cntW) and per low
// digit (cntWd), and the totals of both.
__global__ __launch_bounds__(64) void cs_lists_count_kernel(int64_t n, int64_t chunk, uint64_t seed,
                                                            int64_t r, uint64_t mK_mask, int bits,
                                                            int* __restrict__ cntW,
                                                            int* __restrict__ cntH,
                                                            int* __restrict__ cntWd,
                                                            int* __restrict__ dtot) {
  __shared__ int hist[kHistLds];
  __shared__ int histd[kDigits];
  const int nd = 1 << bits;
  for (int k = threadIdx.x; k < r; k += 64) hist[k] = 0;
  for (int k = threadIdx.x; k < nd; k += 64) histd[k] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 64) {
    uint64_t hh, h;
    int sh, sg;
    rng::cs_hash_hat(seed, (uint64_t)j, (uint64_t)r, hh, sh);
    rng::cs_hash(seed, (uint64_t)j, mK_mask, h, sg);
    atomicAdd(hist + hh, 1);
    atomicAdd(histd + ((int)h & (nd - 1)), 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < r; k += 64) {
    const int c = hist[k];
    cntW[(int64_t)blockIdx.x * r + k] = c;
    if (c) atomicAdd(cntH + k, c);
  }
  for (int k = threadIdx.x; k < nd; k += 64) {
    const int c = histd[k];
    cntWd[(int64_t)blockIdx.x * nd + k] = c;
    if (c) atomicAdd(dtot + k, c);
  }
}

// Fill: every row into its Hessian bucket's list (listH) and, by its low
// digit, its (bucket, entry) into the first pass's order (keys_out, vals_out)
__global__ __launch_bounds__(64) void cs_lists_fill_kernel(
    int64_t n, int64_t chunk, uint64_t seed, int64_t r, int hbits, const int* __restrict__ offW,
    int* __restrict__ listH, uint64_t mK_mask, int bits, const int* __restrict__ offWd,
    int* __restrict__ keys_out, int* __restrict__ vals_out) {
  __shared__ int cur[kHistLds];
  __shared__ int curd[kDigits];
  const int lane = threadIdx.x;
  const int nd = 1 << bits;
  for (int k = lane; k < r; k += 64) cur[k] = offW[(int64_t)blockIdx.x * r + k];
  for (int k = lane; k < nd; k += 64) curd[k] = offWd[(int64_t)blockIdx.x * nd + k];
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(n, j0 + chunk);
  for (int64_t jb = j0; jb < j1; jb += 64) {
    const int64_t j = jb + lane;
    const bool valid = j < j1;
    int hh = 0, sh = 1, key = 0, sg = 1;
    if (valid) {
      uint64_t b, h;
      rng::cs_hash_hat(seed, (uint64_t)j, (uint64_t)r, b, sh);
      rng::cs_hash(seed, (uint64_t)j, mK_mask, h, sg);
      hh = (int)b;
      key = (int)h;
    }
    int before, beforeD;
    bool last, lastD;
    digit_rank(hh, valid, hbits, before, last);
    const int dg = key & (nd - 1);
    digit_rank(dg, valid, bits, beforeD, lastD);
    if (valid) {
      // every lane reads its cursors before any lane writes one (one wave)
      const int slot = cur[hh] + before;
      const int slotD = curd[dg] + beforeD;
      listH[slot] = sh > 0 ? (int)j : ~(int)j;
      keys_out[slotD] = key;
      vals_out[slotD] = sg > 0 ? (int)j : ~(int)j;
      if (last) cur[hh] = slot + 1;
      if (lastD) curd[dg] = slotD + 1;
    }
  }
}

// exclusive scan of n ints in three steps: per-block scans of kScanTile
// elements with block totals, one block scanning the totals, then the carry
constexpr int kScanTile = kThreads * 8;

__global__ __launch_bounds__(kThreads) void scan_tiles_kernel(const int* __restrict__ in,
                                                              int* __restrict__ out, int64_t n,
                                                              int* __restrict__ totals) {
  __shared__ int s_w[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  int v[8];
  int run = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    v[q] = base + q < n ? in[base + q] : 0;
    const int t = v[q];
    v[q] = run;  // exclusive inside the thread
    run += t;
  }
  // inclusive scan of the thread totals across the block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  int wave_off = 0;
  for (int w = 0; w < wave; ++w) wave_off += s_w[w];
  const int excl = x - run + wave_off;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (base + q < n) out[base + q] = v[q] + excl;
  if (threadIdx.x == kThreads - 1) totals[blockIdx.x] = excl + run;
}

// one block: exclusive scan of the tile totals in place, grand total to *total
__global__ __launch_bounds__(kThreads) void scan_totals_kernel(int* __restrict__ totals, int64_t nt,
                                                               int* __restrict__ total) {
  __shared__ int s_w[kWaves];
  __shared__ int s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t b0 = 0; b0 < nt; b0 += kThreads) {
    const int64_t i = b0 + threadIdx.x;
    const int v = i < nt ? totals[i] : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    int wave_off = 0;
    for (int w = 0; w < wave; ++w) wave_off += s_w[w];
    const int carry = s_carry;
    if (i < nt) totals[i] = carry + wave_off + x - v;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) s_carry = carry + wave_off + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = s_carry;
}

__global__ void scan_carry_kernel(int* __restrict__ out, int64_t n, const int* __restrict__ totals) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += totals[i / kScanTile];
}

// list every row in its bucket of the largest level (DO_K) and of S_hat
// (HAT): entry = j, or ~j when the sign is -1
template <bool HAT, bool DO_K = true>
__global__ __launch_bounds__(kThreads) void cs_fill_kernel(int64_t n, uint64_t seed, uint64_t mK_mask,
                                                           int64_t r, int* __restrict__ curK,
                                                           int* __restrict__ listK,
                                                           int* __restrict__ curH,
                                                           int* __restrict__ listH) {
  for (int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kThreads) {
    if constexpr (DO_K) {
      uint64_t h;
      int sg;
      rng::cs_hash(seed, (uint64_t)j, mK_mask, h, sg);
      listK[atomicAdd(curK + h, 1)] = sg > 0 ? (int)j : ~(int)j;
    }
    if constexpr (HAT) {
      uint64_t hh;
      int sh;
      rng::cs_hash_hat(seed, (uint64_t)j, (uint64_t)r, hh, sh);
      listH[atomicAdd(curH + hh, 1)] = sh > 0 ? (int)j : ~(int)j;
    }
  }
}

// The fill claims slots with atomics, so the order of a bucket's rows varies
// from run to run, and with it the rounding of the bucket's sum.  Sorting
// every bucket's entries by row index afterwards makes the lists, and every
// sum over them, the same on every run.  An entry is j or ~j (negative sign).
__device__ __forceinline__ int cs_row(int e) { return e < 0 ? ~e : e; }

// one thread per bucket: insertion sort in place (the largest level's buckets
// hold about N / m_K rows, two on average)
__global__ void cs_sort_small_kernel(int64_t nb, const int* __restrict__ off, int* __restrict__ list) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nb;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int a = off[k], b = off[k + 1];
    for (int i = a + 1; i < b; ++i) {
      const int e = list[i];
      const int key = cs_row(e);
      int p = i - 1;
      while (p >= a && cs_row(list[p]) > key) {
        list[p + 1] = list[p];
        --p;
      }
      list[p + 1] = e;
    }
  }
}

// One block per bucket: a sorting network whose compare-exchanges all put the
// smaller key at the lower index (each merge first compares mirrored
// positions, then halves), so the length need not be a power of 2: missing
// positions act as +infinity and never move.  Segments up to kSortLds entries
// are sorted in LDS, longer ones in place in global memory.
constexpr int kSortLds = 16384;
constexpr int kSortThreads = 1024;

// LOCAL: v is in LDS, where a wave's accesses take effect in program order,
// so the sub-steps that stay inside one wave's 128 positions (t <= 128: the
// wave's 64 consecutive pairs) need no block barrier.
template <bool LOCAL, typename P>
__device__ __forceinline__ void cs_block_sort(P v, int len) {
  int span = 1;
  while (span < len) span <<= 1;
  for (int s = 2; s <= span; s <<= 1) {
    for (int t = s, lh = __builtin_ctz((unsigned)s) - 1; t >= 2; t >>= 1, --lh) {
      const bool sync = !LOCAL || t > 128;
      if (sync) __syncthreads();
      // first sub-step of a merge of size s: mirrored pairs; then half-cleaners
      // (pair q: block q >> lh of t positions, offset q mod t / 2 in it)
      const int half = t >> 1;
      for (int q = threadIdx.x; q < span / 2; q += kSortThreads) {
        const int r = q & (half - 1);
        const int i = ((q >> lh) << (lh + 1)) + r;
        const int l = (t == s) ? i - r + t - 1 - r : i + half;
        if (l < len) {
          const int x = v[i], y = v[l];
          if (cs_row(x) > cs_row(y)) {
            v[i] = y;
            v[l] = x;
          }
        }
      }
      if (sync) __syncthreads();
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSortThreads) void cs_sort_large_kernel(int64_t nb,
                                                                     const int* __restrict__ off,
                                                                     int* __restrict__ list) {
  __shared__ int tile[kSortLds];
  for (int64_t k = blockIdx.x; k < nb; k += gridDim.x) {
    const int a = off[k], len = off[k + 1] - a;
    if (len <= 1) continue;
    if (len <= kSortLds) {
      for (int i = threadIdx.x; i < len; i += kSortThreads) tile[i] = list[a + i];
      __syncthreads();
      cs_block_sort<true>(tile, len);
      for (int i = threadIdx.x; i < len; i += kSortThreads) list[a + i] = tile[i];
      __syncthreads();
    } else {
      cs_block_sort<false>(list + a, len);
    }
  }
}

// out row (bucket b, part p of P): sum of s(j) [x_j | y_j] over list entries
// [off[b] + p len / P, off[b] + (p + 1) len / P), len = off[b+1] - off[b].
// One wave per (bucket, part); a lane holds VEC columns of a 64 VEC-column
// chunk, eight list entries in flight.
template <typename T, int VEC, int CH>
__global__ __launch_bounds__(kThreads) void cs_gather_kernel(int64_t nb, int parts, int d,
                                                             const T* __restrict__ X, int64_t ldx,
                                                             const T* __restrict__ Y,
                                                             const int* __restrict__ off,
                                                             const int* __restrict__ list,
                                                             T* __restrict__ out, int64_t ldo) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = nb * parts;
  for (int64_t w = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); w < nw;
       w += (int64_t)gridDim.x * kWaves) {
    const int64_t b = w / parts;
    const int p = (int)(w % parts);
    const int o0 = off[b], len = off[b + 1] - o0;
    const int e0 = o0 + (int)((int64_t)len * p / parts);
    const int e1 = o0 + (int)((int64_t)len * (p + 1) / parts);
    T* orow = out + w * ldo;
    // CH chunks of 64 VEC columns per pass: a row's chunks are loaded together
    constexpr int U = 8 / CH;  // list entries per batch: eight loads in flight
    for (int c0 = 0; c0 < d; c0 += 64 * VEC * CH) {
      T acc[CH][VEC];
#pragma unroll
      for (int h = 0; h < CH; ++h)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[h][v] = 0;
      for (int e = e0; e < e1; e += U) {
        T x[U][CH][VEC];
        int neg = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int ent = e + u < e1 ? list[e + u] : 0;
          const bool ok = e + u < e1;
          const int64_t j = ent < 0 ? (int64_t)~ent : (int64_t)ent;
          neg |= (ent < 0 ? 1 : 0) << u;
#pragma unroll
          for (int h = 0; h < CH; ++h) {
            const int col = c0 + h * 64 * VEC + lane * VEC;
            const T* xr = X + j * ldx + col;
            if (ok && col + VEC <= d) {
              if constexpr (VEC > 1) {
                typedef T V __attribute__((ext_vector_type(VEC)));
                const V t = __builtin_nontemporal_load(reinterpret_cast<const V*>(xr));
#pragma unroll
                for (int v = 0; v < VEC; ++v) x[u][h][v] = t[v];
              } else {
                x[u][h][0] = __builtin_nontemporal_load(xr);
              }
            } else {
#pragma unroll
              for (int v = 0; v < VEC; ++v) x[u][h][v] = (ok && col + v < d) ? xr[v] : (T)0;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int h = 0; h < CH; ++h)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[h][v] += ((neg >> u) & 1) ? -x[u][h][v] : x[u][h][v];
      }
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        const int col = c0 + h * 64 * VEC + lane * VEC;
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          if (col + v < d) orow[col + v] = acc[h][v];
      }
    }
    // the Y column: lanes split the list, then a wave sum in lane order
    T yacc = 0;
    for (int e = e0 + lane; e < e1; e += 64) {
      const int ent = list[e];
      const int64_t j = ent < 0 ? (int64_t)~ent : (int64_t)ent;
      const T y = Y[j];
      yacc += ent < 0 ? -y : y;
    }
    for (int m = 32; m > 0; m >>= 1) yacc += __shfl_xor(yacc, m, 64);
    if (lane == 0) orow[d] = yacc;
  }
}

// Level K straight from [X|Y] together with the L levels below it (levels
// of m_K / 2, .., m_K / 2^L buckets, when the schedule has them).  One wave
// per family of B = 2^L level-K buckets k_q = f + q mf (q < B, mf = m_K / B):
// by h(j) mod m_i, the rows of the whole family land in bucket f of level
// K - L.  The wave gathers the family's rows (about 2B of them, eight loads in
// flight), keeps the B bucket sums of a chunk of 64 VEC columns in registers
// and writes them with their halvings: level K - l receives the B / 2^l sums
// A_{K-l}[f + q mf] = A_{K-l+1}[f + q mf] + A_{K-l+1}[f + (q + B / 2^l) mf],
// the fold fold(A)[k] = A[k] + A[k + m/2] of the smaller levels.
struct FamilyTargets {
  int64_t off[4];  // off[l]: first row (in A) of level K - l, l = 0..L
};

template <typename T, int VEC, int L, int CH>
__global__ __launch_bounds__(kThreads) void cs_gather_family_kernel(
    int64_t mf, int d, const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y,
    const int* __restrict__ off, const int* __restrict__ list, T* __restrict__ A, int64_t lda,
    FamilyTargets tg, bool a_vec) {
  constexpr int B = 1 << L;
  constexpr int U = 8 / CH;  // rows per batch: eight loads in flight
  const int lane = threadIdx.x & 63;
  for (int64_t f = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); f < mf;
       f += (int64_t)gridDim.x * kWaves) {
    // lane q < B: the list range of bucket k_q, and its start in the family's entries
    int o0 = 0, len = 0;
    if (lane < B) {
      const int64_t k = f + (int64_t)lane * mf;
      o0 = off[k];
      len = off[k + 1] - o0;
    }
    // every lane keeps each bucket's list offset and first entry index
    int oo[B], st[B];
    int E = 0;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      oo[q] = __shfl(o0, q, 64);
      st[q] = E;
      E += __shfl(len, q, 64);
    }
    // CH chunks of 64 VEC columns per pass: a row's chunks are loaded together
    for (int c0 = 0; c0 < d; c0 += 64 * VEC * CH) {
      T acc[CH][B][VEC];
#pragma unroll
      for (int h = 0; h < CH; ++h)
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[h][q][v] = (T)0;
      for (int r0 = 0; r0 < E; r0 += 64) {
        // lane e of this round holds entry r0 + e and its bucket
        const int e = r0 + lane;
        int qe = 0, oq = oo[0], sq = st[0];
#pragma unroll
        for (int q = 1; q < B; ++q)
          if (e >= st[q]) {
            qe = q;
            oq = oo[q];
            sq = st[q];
          }
        const int ent = e < E ? list[oq + (e - sq)] : 0;
        const int n = min(64, E - r0);
        for (int u0 = 0; u0 < n; u0 += U) {
          T x[U][CH][VEC];
          int qu[U];
          int neg = 0;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const bool ok = u0 + u < n;
            const int eu = __shfl(ent, (u0 + u) & 63, 64);
            qu[u] = ok ? __shfl(qe, (u0 + u) & 63, 64) : -1;
            const int64_t j = eu < 0 ? (int64_t)~eu : (int64_t)eu;
            neg |= (eu < 0 ? 1 : 0) << u;
#pragma unroll
            for (int h = 0; h < CH; ++h) {
              const int col = c0 + h * 64 * VEC + lane * VEC;
              const T* xr = X + j * ldx + col;
              if (ok && col + VEC <= d) {
                if constexpr (VEC > 1) {
                  typedef T V __attribute__((ext_vector_type(VEC)));
                  const V t = __builtin_nontemporal_load(reinterpret_cast<const V*>(xr));
#pragma unroll
                  for (int v = 0; v < VEC; ++v) x[u][h][v] = t[v];
                } else {
                  x[u][h][0] = __builtin_nontemporal_load(xr);
                }
              } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v) x[u][h][v] = (ok && col + v < d) ? xr[v] : (T)0;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < B; ++q)
#pragma unroll
              for (int h = 0; h < CH; ++h)
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                  if (qu[u] == q) acc[h][q][v] += ((neg >> u) & 1) ? -x[u][h][v] : x[u][h][v];
        }
      }
      // level K, then the halvings down to level K - L
#pragma unroll
      for (int l = 0; l <= L; ++l) {
        const int nq = B >> l;
        if (l > 0) {
#pragma unroll
          for (int q = 0; q < (B >> 1); ++q)
            if (q < nq)
#pragma unroll
              for (int h = 0; h < CH; ++h)
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[h][q][v] += acc[h][q + nq][v];
        }
#pragma unroll
        for (int q = 0; q < B; ++q) {
          if (q >= nq) continue;
          T* orow = A + (tg.off[l] + f + (int64_t)q * mf) * lda;
#pragma unroll
          for (int h = 0; h < CH; ++h) {
            const int col = c0 + h * 64 * VEC + lane * VEC;
            if constexpr (VEC > 1) {
              if (a_vec && col + VEC <= d) {
                typedef T V __attribute__((ext_vector_type(VEC)));
                V t;
#pragma unroll
                for (int v = 0; v < VEC; ++v) t[v] = acc[h][q][v];
                // streaming stores: the levels are not read again by this
                // pass, and keeping them out of L2 leaves it to the gathers
                __builtin_nontemporal_store(t, reinterpret_cast<V*>(orow + col));
                continue;
              }
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v)
              if (col + v < d) orow[col + v] = acc[h][q][v];
          }
        }
      }
    }
    // the Y column: lanes split the entries, then one wave sum per bucket in lane order
    T ys[B];
#pragma unroll
    for (int q = 0; q < B; ++q) ys[q] = (T)0;
    for (int e = lane; e < E; e += 64) {
      int qe = 0, oq = oo[0], sq = st[0];
#pragma unroll
      for (int q = 1; q < B; ++q)
        if (e >= st[q]) {
          qe = q;
          oq = oo[q];
          sq = st[q];
        }
      const int ent = list[oq + (e - sq)];
      const int64_t j = ent < 0 ? (int64_t)~ent : (int64_t)ent;
      const T y = Y[j];
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (qe == q) ys[q] += ent < 0 ? -y : y;
    }
#pragma unroll
    for (int q = 0; q < B; ++q)
      for (int m = 32; m > 0; m >>= 1) ys[q] += __shfl_xor(ys[q], m, 64);
#pragma unroll
    for (int l = 0; l <= L; ++l) {
      const int nq = B >> l;
      if (l > 0) {
#pragma unroll
        for (int q = 0; q < (B >> 1); ++q)
          if (q < nq) ys[q] += ys[q + nq];
      }
      if (lane < nq) {
        T yv = ys[0];
#pragma unroll
        for (int q = 1; q < B; ++q)
          if (lane == q) yv = ys[q];
        A[(tg.off[l] + f + (int64_t)lane * mf) * lda + d] = yv;
      }
    }
  }
}

// dst[b] = sum over the parts of bucket b in part order
template <typename T>
__global__ void cs_parts_kernel(const T* __restrict__ part, int parts, int64_t nb, int cols,
                                int64_t ldp, T* __restrict__ dst, int64_t ldd) {
  const int64_t n = nb * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / cols;
    const int c = (int)(e % cols);
    T t = 0;
    for (int q = 0; q < parts; ++q) t += part[(b * parts + q) * ldp + c];
    dst[b * ldd + c] = t;
  }
}

// dst[k][c] = sum_{q < ratio} src[k + q*m][c], k < m: rows over blocks,
// columns over threads (every access coalesced along the row)
template <typename T>
__global__ void cs_fold_kernel(const T* __restrict__ src, T* __restrict__ dst, int64_t m, int ratio,
                               int cols, int64_t ld) {
  for (int64_t k = blockIdx.x; k < m; k += gridDim.x) {
    for (int c = threadIdx.x; c < cols; c += blockDim.x) {
      T t = 0;
      for (int q = 0; q < ratio; ++q) t += src[(k + (int64_t)q * m) * ld + c];
      dst[k * ld + c] = t;
    }
  }
}

// Several levels at once by repeated halving, fold(A)[k] = A[k] + A[k + m/2]:
// work item (group g < mT, column tile) holds rows g + q mT, q < R, of the
// source level (R = m_S / mT rows, a power of 2 up to kFoldMax) in LDS and
// halves them down to one row; after the halving to s rows, the level of
// s mT rows (when the schedule has it) gets rows g + q mT, q < s.  Work
// items are dealt to the XCDs in contiguous runs, so the column tiles of one
// group (the same rows) run back to back on one XCD.  The LDS tile is sized
// for the R rows at launch: a small R leaves room for many blocks per CU,
// whose loads are then in flight together.
constexpr int kFoldMax = 512;  // source rows per group
template <typename T, int VEC>
struct FoldVec {
  using type = T __attribute__((ext_vector_type(VEC)));
};
template <typename T>
struct FoldVec<T, 1> {
  using type = T;
};
struct FoldTargets {
  int64_t off[10];  // off[lg]: first row (in A) of the level of 2^lg mT rows, or -1
};

template <typename T, int VEC>
__global__ __launch_bounds__(256) void cs_fold_tree_kernel(const T* __restrict__ src,
                                                           T* __restrict__ A, int64_t lda,
                                                           int64_t mT, int lgR, int cols, int n_ct,
                                                           int64_t xcd_q, FoldTargets tg) {
  constexpr int CT = 128 / (int)sizeof(T);  // columns per tile (128 bytes)
  constexpr int NV = CT / VEC;              // vectors per row segment
  extern __shared__ __attribute__((aligned(16))) char fold_lds[];  // R x CT values
  T* tile = reinterpret_cast<T*>(fold_lds);
  int64_t bid = blockIdx.x;
  if (xcd_q > 0 && bid < 8 * xcd_q) bid = (bid & 7) * xcd_q + (bid >> 3);
  const int ct = (int)(bid % n_ct);
  const int64_t g = bid / n_ct;
  const int c0 = ct * CT;
  const int R = 1 << lgR;
  using V = typename FoldVec<T, VEC>::type;
  // load the group's R rows of this column tile (whole vectors inside the
  // row), eight vectors per thread in flight
  constexpr int U = 8;
  for (int base = threadIdx.x; base < R * NV; base += 256 * U) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * 256;
      const int q = e / NV, cv = (e % NV) * VEC;
      const int col = c0 + cv;
      const T* p = src + (g + (int64_t)(e < R * NV ? q : 0) * mT) * lda + col;
      if (e < R * NV && col + VEC <= cols) {
        if constexpr (VEC == 1) {
          v[u] = __builtin_nontemporal_load(p);
        } else {
          v[u] = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
        }
      } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          const T x = (e < R * NV && col + k < cols) ? p[k] : (T)0;
          if constexpr (VEC == 1) {
            v[u] = x;
          } else {
            v[u][k] = x;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * 256;
      if (e < R * NV) *reinterpret_cast<V*>(&tile[(e / NV) * CT + (e % NV) * VEC]) = v[u];
    }
  }
  __syncthreads();
  for (int lg = lgR - 1; lg >= 0; --lg) {
    const int sz = 1 << lg;
    const int64_t off = tg.off[lg];
    for (int e = threadIdx.x; e < sz * NV; e += 256) {
      const int q = e / NV, cv = (e % NV) * VEC;
      V a = *reinterpret_cast<const V*>(&tile[q * CT + cv]);
      const V b = *reinterpret_cast<const V*>(&tile[(q + sz) * CT + cv]);
      a = a + b;
      *reinterpret_cast<V*>(&tile[q * CT + cv]) = a;
      if (off >= 0) {
        const int col = c0 + cv;
        T* p = A + (off + g + (int64_t)q * mT) * lda + col;
        if (col + VEC <= cols) {
          if constexpr (VEC == 1) {
            __builtin_nontemporal_store(a, p);
          } else {
            __builtin_nontemporal_store(a, reinterpret_cast<V*>(p));
          }
        } else {
#pragma unroll
          for (int k = 0; k < VEC; ++k) {
            if constexpr (VEC == 1) {
              if (col + k < cols) p[k] = a;
            } else {
              if (col + k < cols) p[k] = a[k];
            }
          }
        }
      }
    }
    __syncthreads();
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

// Box-Muller with the hardware transcendentals (v_log_f32 is log2, v_sin_f32
// and v_cos_f32 take revolutions): about 1e-6 relative, far below the BF16
// rounding the matrix-core path applies to G afterwards.
__device__ __forceinline__ void box_muller8_words(const uint64_t (&w)[4], float (&z)[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (uint32_t)(w[q] & 0xffffffffu);
    const uint32_t hi = (uint32_t)(w[q] >> 32);
    const float u1 = fmaf((float)lo, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
    const float u2 = fmaf((float)hi, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
    const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    z[2 * q] = rad * __builtin_amdgcn_cosf(u2);
    z[2 * q + 1] = rad * __builtin_amdgcn_sinf(u2);
  }
}
__device__ __forceinline__ void box_muller8_fast(uint64_t seed, uint64_t stream, uint64_t j,
                                                 uint64_t kblk, float (&z)[8]) {
  const rng::Words w = rng::philox(j, kblk, 0, 0, seed, stream);
  box_muller8_words(w.w, z);
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
// even), products accumulated in FP32 by v_mfma_f32_16x16x32_bf16.  A block
// computes kMT sketch rows x kNT columns over one split of the data rows, in
// steps of kKT data rows.  [X|Y] is converted to BF16 once, by a stage pass,
// into tiles laid out column by column (every lane reads its 8 consecutive k
// as one 16-byte load).
//
// The generation of G (Philox4x64-10 and Box-Muller, about 350 VALU
// instructions per 8 entries) is the largest cost, so the waves specialise:
// on every SIMD one wave generates G and one runs the MFMAs.  A wave issues
// in order, so a wave that did both would leave the matrix core idle while it
// generates and the VALU idle while it multiplies; with one job per wave the
// SIMD issues the MFMAs of some waves between the VALU instructions of the
// others.  During step s the generator waves write the G tile of step s + 1
// into the second of two LDS buffers while the MFMA waves multiply the tiles
// of step s and copy the [X|Y] tile of step s + 1 into the second [X|Y]
// buffer (global_load_lds: straight into LDS, no registers); one barrier per
// step swaps the buffers.  The LDS tiles are unpadded: the 16-byte chunk q of
// row c sits at chunk q ^ (c % 8) of that row, so the lanes that read one
// chunk of consecutive rows hit 8 distinct 16-byte slots of every 128-byte
// line (no bank conflicts), and a wave-wide copy still fills 1 KB of LDS in
// order (each lane picks the source chunk of its slot).  Every block of
// columns generates G again, so one block covers every column of [X|Y] when
// d < kNT.
// Lane layout of v_mfma_f32_16x16x32_bf16 (pinned by the element-wise parity
// tests): lane l holds A[l%16][8(l/16)+j] and B[8(l/16)+j][l%16], j < 8;
// accumulator r of lane l is C[4(l/16)+r][l%16].
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// 64 sketch rows x 576 columns per block (every column of a d <= 575 problem
// in one block, so G is generated once), 64 data rows per step.  Eight
// waves, two per SIMD: 4 MFMA waves, each all four 16-row tiles x nine
// 16-column tiles of v_mfma_f32_16x16x32_bf16 (36 accumulators of four
// registers; every [X|Y] element is read from LDS by one wave only), and 4
// generator waves, two Philox blocks per thread per step with their rounds
// interleaved (two independent chains keep one wave's VALU issue busy).
constexpr int kMT = 64;             // sketch rows per block
constexpr int kNT = 576;            // columns per block
constexpr int kKT = 64;             // data rows per step: 8 chunks of 8 per LDS row
constexpr int kMW = 4;              // MFMA waves: 4 column quarters of all 64 rows
constexpr int kGW = 4;              // generator waves
constexpr int kRT = 4;              // 16-row tiles per MFMA wave
constexpr int kGThreads = 64 * (kMW + kGW);
constexpr int kRH = kMT / (16 * kRT);  // row groups of MFMA waves
constexpr int kCQ = kMW / kRH;         // column groups of MFMA waves
constexpr int kCT = kNT / 16 / kCQ;    // 16-column tiles per MFMA wave (9)
constexpr int kGB = kMT / 8 * kKT / (64 * kGW);  // Philox blocks per generator thread per step
static_assert(kRH * kCQ == kMW && kCT * 16 * kCQ == kNT, "MFMA waves tile the block");
static_assert(kGB * 64 * kGW == kMT / 8 * kKT, "whole Philox blocks per generator thread");
static_assert((2 * kNT + 2 * kMT) * kKT * 2 <= 163840, "two [X|Y] tiles and two G tiles fit in LDS");

// FP32 -> BF16, round to nearest even: gfx950 converts two values per
// instruction (v_cvt_pk_bf16_f32), which the compiler forms from adjacent
// conversions
__device__ __forceinline__ __bf16 to_bf16_rne(float f) { return (__bf16)f; }

// element offset of (row, k) in an unpadded swizzled LDS tile of kKT columns
__device__ __forceinline__ int swz(int row, int k) {
  return row * kKT + ((((k >> 3) ^ row) & 7) << 3) + (k & 7);
}

// [X|Y] in BF16 (nearest even), cut into tiles of kKT data rows x kNT
// columns stored column by column (tile[c][k]), tiles ordered by column block
// then data-row chunk, so that every block copies its tiles with 16-byte
// loads instead of converting and transposing [X|Y] again.  Rows past N and
// columns past d are zeros.
constexpr int kStageThreads = 256;
// columns held by the tiles of column block cb: whole 32-column MFMA tiles up
// to the last one with a column of [X|Y] (cols = d + 1)
__host__ __device__ inline int gauss_tile_cols(int cols, int cb) {
  const int left = (int)round_up(cols, 32) - cb * kNT;
  return left < kNT ? left : kNT;
}
__global__ __launch_bounds__(kStageThreads) void gauss_stage_kernel(
    int64_t N, int d, const float* __restrict__ X, int64_t ldx, const float* __restrict__ Y,
    int64_t nchunks, __bf16* __restrict__ tiles) {
  const int64_t chunk = blockIdx.x;
  const int cb = blockIdx.y;
  const int64_t j0 = chunk * kKT;
  const int wc = gauss_tile_cols(d + 1, cb);
  __bf16* t = tiles + (int64_t)cb * nchunks * (kNT * kKT) + chunk * (wc * kKT);
  // FP32 rows on 16-byte boundaries: four columns per load
  const bool vec4 = (reinterpret_cast<uintptr_t>(X) % 16) == 0 && ldx % 4 == 0;
  // item (4 columns from 4 c4, 8 data rows from 8 q): eight row loads, four
  // 16-byte stores (the 8 k values of each column); consecutive threads take
  // the row groups of one column group, so that each store instruction
  // fills whole 128-byte column segments of the tile
  const int ncg = wc / 4;
  constexpr int NQG = kKT / 8;
  for (int e = threadIdx.x; e < ncg * NQG; e += kStageThreads) {
    const int q = e % NQG, c4 = e / NQG;
    const int col = cb * kNT + 4 * c4;
    float v[8][4];
    const int64_t jq = j0 + 8 * q;
    if (vec4 && col + 4 <= d && jq + 8 <= N) {
      // the common case: eight whole 16-byte loads, all in flight at once
      f32x4_t x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
        x[r] = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(X + (jq + r) * ldx + col));
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[r][i] = x[r][i];
    } else {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t j = jq + r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = col + i;
          v[r][i] = j < N ? (c < d ? X[j * ldx + c] : (c == d ? Y[j] : 0.0f)) : 0.0f;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bf16x8_t w;
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = to_bf16_rne(v[r][i]);
      __builtin_nontemporal_store(w, reinterpret_cast<bf16x8_t*>(t + (int64_t)(4 * c4 + i) * kKT + 8 * q));
    }
  }
}

// one step of the generator waves: kGB Philox blocks of 8 sketch rows at
// data row j per thread, rounded to BF16 and written to the G tile (rows past
// the split are zeros)
__device__ __forceinline__ void gauss_gen_step(uint64_t seed, uint64_t stream, int64_t k0,
                                               int64_t j, int64_t j_end, int gt, __bf16* Gb) {
  const int kb = gt / kKT, jj = gt % kKT;
  // the blocks' rounds side by side: independent chains for the one
  // generator wave of a SIMD to issue back to back
  rng::PhiloxState st[kGB];
#pragma unroll
  for (int b = 0; b < kGB; ++b)
    st[b] = rng::PhiloxState{{(uint64_t)j, (uint64_t)((k0 >> 3) + kb + b * (64 * kGW / kKT)), 0, 0},
                             seed,
                             stream};
#pragma unroll
  for (int r = 0; r < 10; ++r)
#pragma unroll
    for (int b = 0; b < kGB; ++b) rng::philox_round(st[b], r);
  const bool live = j < j_end;
#pragma unroll
  for (int b = 0; b < kGB; ++b) {
    const int rb = kb + b * (64 * kGW / kKT);  // group of 8 sketch rows
    float z[8];
    box_muller8_words(st[b].c, z);
#pragma unroll
    for (int q = 0; q < 8; ++q) Gb[swz(rb * 8 + q, jj)] = to_bf16_rne(live ? z[q] : 0.0f);
  }
}

// the staged [X|Y] tile of one step copied straight into LDS by the MFMA
// waves (16 bytes per lane, placed in order from the wave's LDS base; no
// registers): slot p of row c receives the tile's chunk p ^ (c % 8)
__device__ __forceinline__ void gauss_copy_step(const __bf16* tb, int wc, __bf16* Wb, int wave,
                                                int lane) {
  const int copies = wc / 8;  // 8 rows of 128 bytes per wave-wide copy
  const int c_in = lane >> 3, p = lane & 7;
  for (int g = wave; g < copies; g += kMW) {
    const int c = 8 * g + c_in;
    const __bf16* src = tb + (int64_t)c * kKT + 8 * (p ^ c_in);
    __builtin_amdgcn_global_load_lds(
        (const SLSE_GLOBAL void*)src,
        (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(Wb) + 1024 * g), 16, 0,
        0);
  }
}

__global__ __launch_bounds__(kGThreads) void gauss_mfma_kernel(int64_t N, int d,
                                                         const __bf16* __restrict__ tiles,
                                                         int64_t nchunks, uint64_t seed,
                                                         uint64_t stream, int64_t m, int splits,
                                                         float* __restrict__ part, int64_t ldp) {
  __shared__ __attribute__((aligned(1024))) __bf16 Ws[2][kNT * kKT];
  __shared__ __attribute__((aligned(1024))) __bf16 Gs[2][kMT * kKT];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t k0 = (int64_t)blockIdx.x * kMT;
  const int split = blockIdx.z;
  const int cblk = blockIdx.y;
  const int c0 = cblk * kNT;
  const int64_t per = round_up(ceil_div(N, (int64_t)splits), kKT);
  const int64_t j_begin = (int64_t)split * per;
  const int64_t j_end = min(N, j_begin + per);
  const __bf16* tcol = tiles + (int64_t)cblk * nchunks * (kNT * kKT);
  const int wc = gauss_tile_cols(d + 1, cblk);  // columns of this block's tiles
  const int64_t steps = j_end > j_begin ? ceil_div(j_end - j_begin, kKT) : 0;
  const bool mfma_wave = wave < kMW;
  const int gt = threadIdx.x - 64 * kMW;  // generator thread index
  // step 0's tiles.  A split past the last data row (the rounding of the
  // split length can leave the last ones empty) runs no step but still
  // writes its zero partials; steps is the same for the whole block, so
  // every wave meets the same barriers.
  if (steps > 0) {
    if (mfma_wave) {
      gauss_copy_step(tcol + (j_begin / kKT) * (wc * kKT), wc, Ws[0], wave, lane);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    } else {
      gauss_gen_step(seed, stream, k0, j_begin + gt % kKT, j_end, gt, Gs[0]);
    }
    __syncthreads();
  }
  if (mfma_wave) {
    const int rh = wave % kRH;  // row group: kRT 16-row tiles
    const int cq = wave / kRH;  // column group: kCT 16-column tiles
    f32x4_t acc[kRT][kCT];
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
      for (int q = 0; q < kCT; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][q][r] = 0.0f;
    for (int64_t s = 0; s < steps; ++s) {
      const int b = (int)(s & 1);
      if (s + 1 < steps)
        gauss_copy_step(tcol + ((j_begin + (s + 1) * kKT) / kKT) * (wc * kKT), wc, Ws[b ^ 1],
                        wave, lane);
      const __bf16* Gb = Gs[b];
      const __bf16* Wb = Ws[b];
#pragma unroll
      for (int ks = 0; ks < kKT / 32; ++ks) {
        const int kk = 32 * ks + 8 * (lane >> 4);
        bf16x8_t a[kRT];
#pragma unroll
        for (int i = 0; i < kRT; ++i)
          a[i] = *reinterpret_cast<const bf16x8_t*>(&Gb[swz(rh * 16 * kRT + i * 16 + (lane & 15), kk)]);
#pragma unroll
        for (int q = 0; q < kCT; ++q) {
          // tiles past [X|Y] multiply stale LDS and are never stored (a
          // wave-uniform skip measured slower: it splits the unrolled loop)
          const int col = (cq * kCT + q) * 16 + (lane & 15);
          const bf16x8_t bv = *reinterpret_cast<const bf16x8_t*>(&Wb[swz(col, kk)]);
#pragma unroll
          for (int i = 0; i < kRT; ++i)
            acc[i][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv, acc[i][q], 0, 0, 0);
        }
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // next [X|Y] tile is in LDS
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kRT; ++i)
#pragma unroll
      for (int q = 0; q < kCT; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t k = k0 + rh * 16 * kRT + i * 16 + 4 * (lane >> 4) + r;
          const int t = cq * kCT + q;
          const int col = c0 + t * 16 + (lane & 15);
          if (k < m && col <= d && t * 16 < wc)
            part[((int64_t)split * m + k) * ldp + col] = acc[i][q][r];
        }
  } else {
    for (int64_t s = 0; s < steps; ++s) {
      // G of step s + 1 (zeros after the last step: never read)
      const int64_t j = j_begin + (s + 1) * kKT + gt % kKT;
      gauss_gen_step(seed, stream, k0, j, j_end, gt, Gs[(s + 1) & 1]);
      __syncthreads();
    }
  }
}

// Reference for measurement: the matrix-core kernel's generation of G alone
// (Philox block -> eight Box-Muller values -> BF16) for entries k < m, j < N,
// folded into one checksum word per thread; no data is read and no product
// formed.  Its time is the floor the VALU work of the Gaussian sketch sets.
__global__ __launch_bounds__(256) void gauss_generate_kernel(uint64_t seed, uint64_t stream,
                                                             int64_t kblocks, int64_t N,
                                                             unsigned* __restrict__ sink) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // entry e = kb N + j, walked with a carry instead of a division per entry
  int64_t kb = tid / N, j = tid % N;
  const int64_t skb = stride / N, sj = stride % N;
  unsigned acc = 0;
  while (kb < kblocks) {
    float z[8];
    box_muller8_fast(seed, stream, (uint64_t)j, (uint64_t)kb, z);
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += __builtin_bit_cast(uint16_t, to_bf16_rne(z[q]));
    kb += skb;
    j += sj;
    if (j >= N) {
      j -= N;
      ++kb;
    }
  }
  sink[tid] = acc;
}

// form 0: the entries of the VALU kernels; form 1: those of the matrix-core
// kernel (hardware transcendentals, then rounded to BF16 as its operands are)
__global__ void debug_gauss_kernel(uint64_t seed, uint64_t stream, int64_t k0, int64_t nk,
                                   int64_t j0, int64_t nj, int form, double* __restrict__ out) {
  const int64_t n = nk * nj;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / nj, b = e % nj;
    const int64_t k = k0 + a, j = j0 + b;
    float z[8];
    if (form == 1) {
      box_muller8_fast(seed, stream, (uint64_t)j, (uint64_t)(k >> 3), z);
      out[e] = (double)(float)(__bf16)z[k & 7];
    } else {
      box_muller8(seed, stream, (uint64_t)j, (uint64_t)(k >> 3), z);
      out[e] = (double)z[k & 7];
    }
  }
}

int grid1(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 8192)); }

// parts of each Hessian bucket: about 1024 listed rows per wave
int cs_hat_parts(int64_t N, int64_t r) {
  const int64_t per = ceil_div(std::max<int64_t>(N, 1), std::max<int64_t>(r, 1));
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, ceil_div(per, 1024)));
}

__global__ void copy_i32_kernel(const int* __restrict__ src, int* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

void copy_i32(const int* src, int* dst, int64_t n, hipStream_t s) {
  copy_i32_kernel<<<grid1(n), 256, 0, s>>>(src, dst, n);
  SLSE_LAUNCH_CHECK();
}

// Scratch of the bucket lists, carved from CountSketchArgs::scratch.
struct CsScratch {
  int *cntK, *offK, *listK, *cntH, *offH, *listH, *totals;
  int* cntW;   // per (wave, Hessian bucket) counts, then first slots (row-order fills)
  int* cntWd;  // the same per (wave, digit) for the counting sort
  int waves;
  int64_t chunk;
  bool radix;                    // the largest level's lists by the counting sort
  int *keysA, *valsA, *keysB;    // its passes' buckets and entries
  int *dtot, *doff;              // per-digit totals and their scan
  void* partH;
  size_t bytes;
};

CsScratch cs_scratch(const CountSketchArgs& a) {
  const int64_t mK = a.m[a.K - 1];
  const int parts = cs_hat_parts(a.N, a.r);
  const int64_t ntiles = ceil_div(std::max<int64_t>({mK, a.r, 1}), (int64_t)kScanTile);
  const size_t es = dtype_size(a.t);
  char* p = static_cast<char*>(a.scratch);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* q = p ? p + o : nullptr;
    o += (size_t)round_up((int64_t)bytes, 256);
    return q;
  };
  CsScratch c;
  c.cntK = reinterpret_cast<int*>(take(sizeof(int) * mK));
  c.offK = reinterpret_cast<int*>(take(sizeof(int) * (mK + 1)));
  c.listK = reinterpret_cast<int*>(take(sizeof(int) * a.N));
  c.cntH = reinterpret_cast<int*>(take(sizeof(int) * a.r));
  c.offH = reinterpret_cast<int*>(take(sizeof(int) * (a.r + 1)));
  c.listH = reinterpret_cast<int*>(take(sizeof(int) * a.N));
  c.totals = reinterpret_cast<int*>(take(sizeof(int) * ntiles));
  c.partH = parts > 1 ? take(es * (size_t)a.r * parts * (a.d + 1)) : nullptr;
  // per-wave row ranges: the Hessian lists in row order when their counts fit
  // in a wave's LDS; the largest level's by the counting sort when its
  // buckets take at most two digits
  const int64_t w = std::min<int64_t>(kHatWaves, ceil_div(std::max<int64_t>(a.N, 1), 64));
  c.chunk = round_up(ceil_div(std::max<int64_t>(a.N, 1), w), 64);
  c.waves = (int)ceil_div(std::max<int64_t>(a.N, 1), c.chunk);
  const bool hat_rows = a.r <= kHistLds;
  c.radix = ilog2_ceil(mK) <= 2 * kDigitBits;
  c.cntW = hat_rows ? reinterpret_cast<int*>(take(sizeof(int) * (size_t)c.waves * a.r)) : nullptr;
  c.cntWd = c.radix ? reinterpret_cast<int*>(take(sizeof(int) * (size_t)c.waves * kDigits)) : nullptr;
  c.keysA = c.valsA = c.keysB = c.dtot = c.doff = nullptr;
  if (c.radix) {
    c.keysA = reinterpret_cast<int*>(take(sizeof(int) * a.N));
    c.valsA = reinterpret_cast<int*>(take(sizeof(int) * a.N));
    c.keysB = reinterpret_cast<int*>(take(sizeof(int) * a.N));
    c.dtot = reinterpret_cast<int*>(take(sizeof(int) * (kDigits + 1)));
    c.doff = reinterpret_cast<int*>(take(sizeof(int) * (kDigits + 1)));
  }
  c.bytes = o;
  return c;
}

void scan_exclusive(const int* in, int* out, int64_t n, int* totals, hipStream_t s) {
  const int64_t nt = ceil_div(std::max<int64_t>(n, 1), (int64_t)kScanTile);
  scan_tiles_kernel<<<(unsigned)nt, kThreads, 0, s>>>(in, out, n, totals);
  scan_totals_kernel<<<1, kThreads, 0, s>>>(totals, nt, out + n);
  scan_carry_kernel<<<(unsigned)ceil_div(std::max<int64_t>(n, 1), 256), 256, 0, s>>>(out, n, totals);
  SLSE_LAUNCH_CHECK();
}

template <typename T>
void gather(int64_t nb, int parts, const CountSketchArgs& a, const int* off, const int* list, T* out,
            int64_t ldo, hipStream_t s) {
  const int64_t waves = nb * parts;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(waves, kWaves), 65536));
  const T* X = static_cast<const T*>(a.X);
  const T* Y = static_cast<const T*>(a.Y);
  constexpr int V = 16 / sizeof(T);
  const bool vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((a.ldx * (int64_t)sizeof(T)) % 16 == 0);
  if (vec && a.d > 64 * V)  // rows wider than one chunk: two chunks of a row per pass
    cs_gather_kernel<T, V, 2><<<blocks, kThreads, 0, s>>>(nb, parts, a.d, X, a.ldx, Y, off, list, out, ldo);
  else if (vec)
    cs_gather_kernel<T, V, 1><<<blocks, kThreads, 0, s>>>(nb, parts, a.d, X, a.ldx, Y, off, list, out, ldo);
  else
    cs_gather_kernel<T, 1, 1><<<blocks, kThreads, 0, s>>>(nb, parts, a.d, X, a.ldx, Y, off, list, out, ldo);
  SLSE_LAUNCH_CHECK();
}

// Level K (at row offK of A) and the L levels below it, one wave per family.
template <typename T>
void gather_family(int L, const CountSketchArgs& a, const int* off, const int* list, T* A,
                   int64_t offK, hipStream_t s) {
  const int64_t mK = a.m[a.K - 1];
  const int64_t mf = mK >> L;
  FamilyTargets tg;
  int64_t o = offK;
  for (int l = 0; l < 4; ++l) tg.off[l] = -1;
  for (int l = 0; l <= L; ++l) {
    tg.off[l] = o;
    if (l < L) o -= a.m[a.K - 2 - l];
  }
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(mf, kWaves), 65536));
  const T* X = static_cast<const T*>(a.X);
  const T* Y = static_cast<const T*>(a.Y);
  constexpr int V = 16 / sizeof(T);
  const bool vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((a.ldx * (int64_t)sizeof(T)) % 16 == 0);
  const bool a_vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && ((a.lda * (int64_t)sizeof(T)) % 16 == 0);
#define SLSE_FAMILY(VV, LL, CC)                                                                 \
  cs_gather_family_kernel<T, VV, LL, CC><<<blocks, kThreads, 0, s>>>(mf, a.d, X, a.ldx, Y, off,   \
                                                                     list, A, a.lda, tg, a_vec)
  // rows wider than one chunk of 64 V columns: two chunks of a row per pass
  const bool two = a.d > 64 * V;
  if (vec && two) {
    if (L == 3) SLSE_FAMILY(V, 3, 2);
    else if (L == 2) SLSE_FAMILY(V, 2, 2);
    else if (L == 1) SLSE_FAMILY(V, 1, 2);
    else SLSE_FAMILY(V, 0, 2);
  } else if (vec) {
    if (L == 3) SLSE_FAMILY(V, 3, 1);
    else if (L == 2) SLSE_FAMILY(V, 2, 1);
    else if (L == 1) SLSE_FAMILY(V, 1, 1);
    else SLSE_FAMILY(V, 0, 1);
  } else {
    if (L == 3) SLSE_FAMILY(1, 3, 1);
    else if (L == 2) SLSE_FAMILY(1, 2, 1);
    else if (L == 1) SLSE_FAMILY(1, 1, 1);
    else SLSE_FAMILY(1, 0, 1);
  }
#undef SLSE_FAMILY
  SLSE_LAUNCH_CHECK();
}

// Levels top-1 .. 0 from level `top` (level i sits just before level i + 1
// in A, level K-1 at row offK).  Each pass folds a source level down as far as
// kFoldMax rows per group allow and writes every level on the way; a step
// between two levels wider than that falls back to the one-level fold.
template <typename T>
void fold_levels(const CountSketchArgs& a, T* A, int64_t offK, int top, hipStream_t s) {
  std::vector<int64_t> off(a.K);
  off[a.K - 1] = offK;
  for (int i = a.K - 2; i >= 0; --i) off[i] = off[i + 1] - a.m[i];
  const int cols = a.d + 1;
  constexpr int CT = 128 / (int)sizeof(T);
  const int n_ct = (int)ceil_div(cols, CT);
  const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && ((a.lda * (int64_t)sizeof(T)) % 16 == 0);
  int S = top;
  while (S > 0) {
    int Tl = S;
    while (Tl > 0 && a.m[S] / a.m[Tl - 1] <= kFoldMax) --Tl;
    if (Tl == S) {  // the next level is more than kFoldMax times smaller
      const int i = S - 1;
      cs_fold_kernel<T><<<(unsigned)std::min<int64_t>(a.m[i], 65536), 256, 0, s>>>(
          A + off[S] * a.lda, A + off[i] * a.lda, a.m[i], (int)(a.m[S] / a.m[i]), cols, a.lda);
      SLSE_LAUNCH_CHECK();
      S = i;
      continue;
    }
    const int64_t mT = a.m[Tl];
    const int lgR = ilog2_ceil(a.m[S] / mT);
    FoldTargets tg;
    for (int k = 0; k < 10; ++k) tg.off[k] = -1;
    for (int i = Tl; i < S; ++i) tg.off[ilog2_ceil(a.m[i] / mT)] = off[i];
    const int64_t blocks = mT * n_ct;
    if (blocks > 0x7fffffffLL) fail(SLSE_EUNSUPPORTED, "countsketch: too many fold work items");
    const int64_t xq = blocks / 8;
    const size_t lds = (size_t)(int64_t(1) << lgR) * CT * sizeof(T);  // at most 64 KiB
    if (vec)
      cs_fold_tree_kernel<T, 16 / sizeof(T)><<<(unsigned)blocks, 256, lds, s>>>(
          A + off[S] * a.lda, A, a.lda, mT, lgR, cols, n_ct, xq, tg);
    else
      cs_fold_tree_kernel<T, 1><<<(unsigned)blocks, 256, lds, s>>>(A + off[S] * a.lda, A, a.lda, mT,
                                                                   lgR, cols, n_ct, xq, tg);
    SLSE_LAUNCH_CHECK();
    S = Tl;
  }
}

template <typename T>
void countsketch_t(const CountSketchArgs& a, hipStream_t s) {
  if (a.N >= (int64_t(1) << 31)) fail(SLSE_EUNSUPPORTED, "countsketch: N >= 2^31 rows");
  T* A = static_cast<T*>(a.A);
  T* Ah = static_cast<T*>(a.Ahat);
  int64_t rows_A = 0;
  for (int i = 0; i < a.K; ++i) rows_A += a.m[i];
  const int64_t mK = a.m[a.K - 1];
  const CsScratch sc = cs_scratch(a);
  const unsigned rb = (unsigned)grid1(a.N);
  const uint64_t mK_mask = (uint64_t)mK - 1;
  // 1. the largest level's lists, every bucket's rows in increasing row order:
  // by the counting sort from 2^21 rows, below that by atomic slot claims and
  // a sort of each list (fewer launches; the two give the same lists).
  // SLSE_CS_SORT=1 / 0 forces one of them, for measurement and tests.
  bool radix = sc.radix && a.N >= kRadixRows;
  if (const char* e = std::getenv("SLSE_CS_SORT")) radix = sc.radix && std::atoi(e) != 0;
  const bool hat_rows = a.r <= kHistLds;
  const unsigned ncs = (unsigned)ceil_div(kDigits, kColTile);
  auto digit_pass1 = [&](int shift, int bits) {  // high digit: counts, first slots, fill
    fill_kernel<int><<<grid1(kDigits), 256, 0, s>>>(sc.dtot, 1, kDigits, kDigits);
    cs_digit_count_kernel<1><<<(unsigned)sc.waves, 64, 0, s>>>(a.N, sc.chunk, a.seed, mK_mask, shift,
                                                              bits, sc.keysA, sc.cntWd, sc.dtot);
    cs_colscan_kernel<<<ncs, 1024, 0, s>>>(int64_t(1) << bits, sc.waves, sc.cntWd, sc.dtot, sc.doff);
    cs_digit_fill_kernel<1><<<(unsigned)sc.waves, 64, 0, s>>>(
        a.N, sc.chunk, a.seed, mK_mask, shift, bits, sc.cntWd, sc.keysA, sc.valsA, sc.keysB, sc.listK);
  };
  if (radix && hat_rows) {
    // the Hessian lists and the low-digit pass together, then the high digit
    const int p = ilog2_ceil(mK);
    const int b0 = std::min(p, kDigitBits), b1 = p - b0;
    fill_kernel<int><<<grid1(kDigits), 256, 0, s>>>(sc.dtot, 1, kDigits, kDigits);
    fill_kernel<int><<<grid1(a.r), 256, 0, s>>>(sc.cntH, 1, a.r, a.r);
    cs_lists_count_kernel<<<(unsigned)sc.waves, 64, 0, s>>>(a.N, sc.chunk, a.seed, a.r, mK_mask, b0,
                                                            sc.cntW, sc.cntH, sc.cntWd, sc.dtot);
    cs_colscan_kernel<<<ncs, 1024, 0, s>>>(int64_t(1) << b0, sc.waves, sc.cntWd, sc.dtot, sc.doff);
    cs_colscan_kernel<<<(unsigned)ceil_div(a.r, kColTile), 1024, 0, s>>>(a.r, sc.waves, sc.cntW,
                                                                        sc.cntH, sc.offH);
    cs_lists_fill_kernel<<<(unsigned)sc.waves, 64, 0, s>>>(
        a.N, sc.chunk, a.seed, a.r, ilog2_ceil(a.r), sc.cntW, sc.listH, mK_mask, b0, sc.cntWd,
        b1 ? sc.keysA : sc.keysB, b1 ? sc.valsA : sc.listK);
    if (b1) digit_pass1(b0, b1);
    cs_starts_kernel<<<grid1(a.N + 1), 256, 0, s>>>(a.N, mK, sc.keysB, sc.offK);
    SLSE_LAUNCH_CHECK();
  } else {
    if (radix) {
      const int p = ilog2_ceil(mK);
      const int b0 = std::min(p, kDigitBits), b1 = p - b0;
      fill_kernel<int><<<grid1(kDigits), 256, 0, s>>>(sc.dtot, 1, kDigits, kDigits);
      cs_digit_count_kernel<0><<<(unsigned)sc.waves, 64, 0, s>>>(a.N, sc.chunk, a.seed, mK_mask, 0,
                                                                b0, nullptr, sc.cntWd, sc.dtot);
      cs_colscan_kernel<<<ncs, 1024, 0, s>>>(int64_t(1) << b0, sc.waves, sc.cntWd, sc.dtot, sc.doff);
      cs_digit_fill_kernel<0><<<(unsigned)sc.waves, 64, 0, s>>>(
          a.N, sc.chunk, a.seed, mK_mask, 0, b0, sc.cntWd, nullptr, nullptr,
          b1 ? sc.keysA : sc.keysB, b1 ? sc.valsA : sc.listK);
      if (b1) digit_pass1(b0, b1);
      cs_starts_kernel<<<grid1(a.N + 1), 256, 0, s>>>(a.N, mK, sc.keysB, sc.offK);
    } else {
      fill_kernel<int><<<grid1(mK), 256, 0, s>>>(sc.cntK, 1, mK, mK);
      cs_count_kernel<false, false, true><<<rb, kThreads, 0, s>>>(a.N, a.seed, mK_mask, a.r, sc.cntK,
                                                                  nullptr);
      scan_exclusive(sc.cntK, sc.offK, mK, sc.totals, s);
      copy_i32(sc.offK, sc.cntK, mK, s);
      cs_fill_kernel<false, true><<<rb, kThreads, 0, s>>>(a.N, a.seed, mK_mask, a.r, sc.cntK,
                                                          sc.listK, nullptr, nullptr);
      cs_sort_small_kernel<<<grid1(mK), 256, 0, s>>>(mK, sc.offK, sc.listK);
    }
    SLSE_LAUNCH_CHECK();
    // 2. the Hessian buckets' lists, in row order too
    fill_kernel<int><<<grid1(a.r), 256, 0, s>>>(sc.cntH, 1, a.r, a.r);
    if (hat_rows) {
      cs_hat_count_kernel<<<(unsigned)sc.waves, 64, 0, s>>>(a.N, sc.chunk, a.seed, a.r, sc.cntW,
                                                            sc.cntH);
      cs_colscan_kernel<<<(unsigned)ceil_div(a.r, kColTile), 1024, 0, s>>>(a.r, sc.waves, sc.cntW,
                                                                          sc.cntH, sc.offH);
      cs_hat_fill_kernel<<<(unsigned)sc.waves, 64, 0, s>>>(a.N, sc.chunk, a.seed, a.r,
                                                           ilog2_ceil(a.r), sc.cntW, sc.listH);
    } else {
      cs_count_kernel<false, true, false><<<rb, kThreads, 0, s>>>(a.N, a.seed, mK_mask, a.r, nullptr,
                                                                  sc.cntH);
      scan_exclusive(sc.cntH, sc.offH, a.r, sc.totals, s);
      copy_i32(sc.offH, sc.cntH, a.r, s);
      cs_fill_kernel<true, false><<<rb, kThreads, 0, s>>>(a.N, a.seed, mK_mask, a.r, nullptr,
                                                          nullptr, sc.cntH, sc.listH);
      cs_sort_large_kernel<<<(unsigned)std::min<int64_t>(a.r, 65535), kSortThreads, 0, s>>>(
          a.r, sc.offH, sc.listH);
    }
    SLSE_LAUNCH_CHECK();
  }
  // 3. gathers: the largest level and up to three below it straight into A,
  //    S_hat through its parts
  const int64_t offK = rows_A - mK;
  // fuse the levels below K that halve it step by step (up to three)
  int L = 0;
  while (L < 3 && L < a.K - 1 && a.m[a.K - 2 - L] == (mK >> (L + 1))) ++L;
  gather_family<T>(L, a, sc.offK, sc.listK, A, offK, s);
  const int parts = cs_hat_parts(a.N, a.r);
  if (parts == 1) {
    gather<T>(a.r, 1, a, sc.offH, sc.listH, Ah, a.ldah, s);
  } else {
    T* part = static_cast<T*>(sc.partH);
    const int64_t ldp = a.d + 1;
    gather<T>(a.r, parts, a, sc.offH, sc.listH, part, ldp, s);
    cs_parts_kernel<T><<<grid1(a.r * (a.d + 1)), 256, 0, s>>>(part, parts, a.r, a.d + 1, ldp, Ah,
                                                             a.ldah);
    SLSE_LAUNCH_CHECK();
  }
  // 4. smaller levels by folding, several levels per pass
  fold_levels<T>(a, A, offK, a.K - 1 - L, s);
}

// BF16 path scratch: the staged tiles (shared by the two sketches of one
// [X|Y]: they depend only on N and d), then, at a 256-byte boundary, the split
// partial sums
size_t gauss_partial_bytes(const GaussianArgs& a) {
  const size_t es = (a.t == SLSE_F64 && !a.bf16) ? 8 : 4;
  return (size_t)a.splits * (size_t)a.m * (size_t)round_up(a.d + 1, 4) * es;
}
size_t gauss_tile_bytes(const GaussianArgs& a) {
  if (!a.bf16) return 0;
  return (size_t)ceil_div(a.d + 1, kNT) * (size_t)ceil_div(std::max<int64_t>(a.N, 1), kKT) *
         (size_t)(kNT * kKT) * sizeof(__bf16);
}

void gaussian_mfma(const GaussianArgs& a, hipStream_t s) {
  const int cols = a.d + 1;
  const int64_t ldp = round_up(cols, 4);
  const int64_t nchunks = ceil_div(std::max<int64_t>(a.N, 1), kKT);
  __bf16* tiles = reinterpret_cast<__bf16*>(a.partial);
  float* part = reinterpret_cast<float*>(reinterpret_cast<char*>(a.partial) +
                                         round_up((int64_t)gauss_tile_bytes(a), 256));
  if (!a.tiles_ready) {
    gauss_stage_kernel<<<dim3((unsigned)nchunks, (unsigned)ceil_div(cols, kNT)), kStageThreads,
                         0, s>>>(a.N, a.d, static_cast<const float*>(a.X), a.ldx,
                                 static_cast<const float*>(a.Y), nchunks, tiles);
    SLSE_LAUNCH_CHECK();
  }
  // blockIdx.x is the sketch-row block: the blocks that read the same data
  // rows and columns run side by side and share them through the caches
  const int ncb = (int)ceil_div(cols, kNT);
  dim3 grid((unsigned)ceil_div(a.m, kMT), (unsigned)ncb, (unsigned)a.splits);
  gauss_mfma_kernel<<<grid, kGThreads, 0, s>>>(a.N, a.d, tiles, nchunks, a.seed, a.stream_id, a.m,
                                               a.splits, part, ldp);
  SLSE_LAUNCH_CHECK();
  gauss_reduce_kernel<float, float><<<grid1(a.m * cols), 256, 0, s>>>(
      part, a.splits, a.m, cols, ldp, static_cast<float*>(a.A), a.lda);
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

size_t countsketch_scratch_bytes(const CountSketchArgs& a) { return cs_scratch(a).bytes; }

void launch_countsketch(const CountSketchArgs& a, hipStream_t s) {
  if (!a.scratch) fail(SLSE_EINVAL, "countsketch: no scratch buffer");
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
  const size_t t = gauss_tile_bytes(a);
  return t ? (size_t)round_up((int64_t)t, 256) + gauss_partial_bytes(a) : gauss_partial_bytes(a);
}

void launch_gaussian(const GaussianArgs& a, hipStream_t s) {
  if (a.bf16) {
    if (a.t != SLSE_F32) fail(SLSE_EUNSUPPORTED, "gaussian: BF16 products need F32 data");
    gaussian_mfma(a, s);
    return;
  }
  if (a.t == SLSE_F64)
    gaussian_t<double, double>(a, s);
  else if (a.t == SLSE_F32)
    gaussian_t<float, float>(a, s);
  else
    fail(SLSE_EUNSUPPORTED, "gaussian: dtype");
}

void launch_gauss_generate(uint64_t seed, uint64_t stream_id, int64_t m, int64_t N, int blocks,
                           unsigned* sink, hipStream_t s) {
  gauss_generate_kernel<<<blocks, 256, 0, s>>>(seed, stream_id, ceil_div(m, 8), N, sink);
  SLSE_LAUNCH_CHECK();
}

void launch_debug_gaussian(uint64_t seed, uint64_t stream_id, int64_t k0, int64_t nk, int64_t j0,
                           int64_t nj, int form, double* out, hipStream_t s) {
  if (nk * nj <= 0) return;
  debug_gauss_kernel<<<grid1(nk * nj), 256, 0, s>>>(seed, stream_id, k0, nk, j0, nj, form, out);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
