// Subsampled randomized Hadamard transform of [X|Y] (Sec. 3: S = (N/m)^{1/2}
// B H D P with H the normalised Sylvester Hadamard matrix, and the efficient
// construction S_i = (N/m_i)^{1/2} B_i (H D P)).  The transform H D P [X|Y] is
// computed once over the zero-padded length N' = 2^p and only its sampled rows
// are written: row sigma(t) of the transform goes to A[t] for t < m_K (every
// level i is the prefix of m_i rows) and row sigma_hat(t) to Ahat[t] for t < r.
//
// Design.  The p butterfly stages along the rows are split into passes of at
// most 10-11 stages.  A pass works on groups of 2^b rows that differ only in
// the pass's b bits (stride 2^s0 in the row index) and on a tile of CT
// columns, so every row segment it touches is CT contiguous elements (128 B)
// of one row of [X|Y] or of the workspace Z.  Inside a block the group is
// held twice in registers and once in LDS: phase A keeps 2^BA rows of one
// column per thread and runs the stages on the high BA bits, writes LDS;
// phase B reads 2^BB consecutive rows per thread and runs the low BB stages.
// The first pass gathers rows through the permutation P and applies the
// signs D on load; the last pass scatters only the sampled rows.
#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "rng.hpp"

namespace slse {
namespace {

constexpr int kPassThreads = 512;
enum { kFirst = 1, kLast = 2 };

template <typename T>
struct PassParams {
  const T* X;
  int64_t ldx;
  const T* Y;
  int64_t N;
  int d;
  const int32_t* pi_sgn;
  T* Z;
  int64_t ldz;
  const int32_t* slotA;
  const int32_t* slotH;
  T* A;
  int64_t lda;
  T* Ahat;
  int64_t ldah;
  int s0;
  int n_ct;
};

template <typename T, int CT, int BA, int BB, int MODE>
__global__ __launch_bounds__(kPassThreads) void fwht_pass_kernel(PassParams<T> P) {
  constexpr int RA = 1 << BA;
  constexpr int RB = 1 << BB;
  constexpr int B = BA + BB;
  constexpr int PAD = CT;  // one padded row per 2^BB rows spreads phase-B reads over the banks
  __shared__ T tile[(1 << B) * CT + RA * PAD];

  // index maps of this group, fetched once (contiguous: the first pass has
  // s0 = 0 and the slot maps are stored in the last pass's group order)
  __shared__ int32_t s_pi[(MODE & kFirst) ? (1 << B) : 1];
  __shared__ int32_t s_slot[(MODE & kLast) ? 2 * (1 << B) : 1];

  const int ct = blockIdx.x % P.n_ct;
  const int64_t g = blockIdx.x / P.n_ct;
  const int64_t lo = g & ((int64_t(1) << P.s0) - 1);
  const int64_t hi = g >> P.s0;
  const int64_t hi_part = hi << (P.s0 + B);
  const int col_base = ct * CT;
  if constexpr ((MODE & kFirst) != 0) {
    for (int k = threadIdx.x; k < (1 << B); k += kPassThreads) s_pi[k] = P.pi_sgn[hi_part | k];
  }
  if constexpr ((MODE & kLast) != 0) {
    const int64_t gb = g << B;
    for (int k = threadIdx.x; k < (1 << B); k += kPassThreads) {
      s_slot[k] = P.slotA[gb + k];
      s_slot[(1 << B) + k] = P.slotH[gb + k];
    }
  }
  if constexpr ((MODE & (kFirst | kLast)) != 0) __syncthreads();

  // phase A: 2^BA rows {q + k 2^BB} of one column per item; stages on the high BA bits
  for (int it = threadIdx.x; it < RB * CT; it += kPassThreads) {
    const int c = it % CT;
    const int q = it / CT;
    const int col = col_base + c;
    T v[RA];
    if constexpr ((MODE & kFirst) != 0) {
      // gather through P with D applied; branch-free so that all 2^BA loads
      // are in flight together (out-of-range rows and padding columns read a
      // valid address and are zeroed afterwards)
      int32_t ps[RA];
#pragma unroll
      for (int k = 0; k < RA; ++k) ps[k] = s_pi[q + (k << BB)];
#pragma unroll
      for (int k = 0; k < RA; ++k) {
        const bool neg = ps[k] < 0;
        const int64_t src = neg ? (int64_t)(~ps[k]) : (int64_t)ps[k];
        const bool in_rows = src < P.N;
        const int64_t srow = in_rows ? src : 0;
        // select the address as an integer so that the load stays unconditional
        const uintptr_t ax = reinterpret_cast<uintptr_t>(P.X + srow * P.ldx + col);
        const uintptr_t ay = reinterpret_cast<uintptr_t>(P.Y + srow);
        const T* addr = reinterpret_cast<const T*>(col < P.d ? ax : ay);
        const T val = __builtin_nontemporal_load(addr);
        // zero / negate with bit masks: a select here would let the compiler
        // move the load under a branch and wait for it
        using U = typename std::conditional<sizeof(T) == 8, uint64_t, uint32_t>::type;
        const U keep = (in_rows && col <= P.d) ? ~U(0) : U(0);
        const U sgn = neg ? (U(1) << (8 * sizeof(T) - 1)) : U(0);
        v[k] = __builtin_bit_cast(T, (U)((__builtin_bit_cast(U, val) ^ sgn) & keep));
      }
    } else {
#pragma unroll
      for (int k = 0; k < RA; ++k) {
        const int64_t pos = q + (k << BB);
        const int64_t j = hi_part | (pos << P.s0) | lo;
        v[k] = __builtin_nontemporal_load(P.Z + j * P.ldz + col);
      }
    }
#pragma unroll
    for (int h = 1; h < RA; h <<= 1)
#pragma unroll
      for (int k = 0; k < RA; ++k)
        if ((k & h) == 0) {
          const T a0 = v[k], a1 = v[k + h];
          v[k] = a0 + a1;
          v[k + h] = a0 - a1;
        }
#pragma unroll
    for (int k = 0; k < RA; ++k) tile[(q + (k << BB)) * CT + c + k * PAD] = v[k];
  }
  __syncthreads();

  // phase B: 2^BB consecutive rows {qq 2^BB + k} per item; stages on the low BB bits
  for (int it = threadIdx.x; it < RA * CT; it += kPassThreads) {
    const int c = it % CT;
    const int qq = it / CT;
    const int col = col_base + c;
    T v[RB];
    int32_t sa[RB], sh[RB];
    if constexpr ((MODE & kLast) != 0) {
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        sa[k] = s_slot[(qq << BB) + k];
        sh[k] = s_slot[(1 << B) + (qq << BB) + k];
      }
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) v[k] = tile[((qq << BB) + k) * CT + c + qq * PAD];
#pragma unroll
    for (int h = 1; h < RB; h <<= 1)
#pragma unroll
      for (int k = 0; k < RB; ++k)
        if ((k & h) == 0) {
          const T a0 = v[k], a1 = v[k + h];
          v[k] = a0 + a1;
          v[k + h] = a0 - a1;
        }
    if constexpr ((MODE & kLast) != 0) {
      if (col <= P.d) {
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          if (sa[k] >= 0) __builtin_nontemporal_store(v[k], P.A + (int64_t)sa[k] * P.lda + col);
          if (sh[k] >= 0) P.Ahat[(int64_t)sh[k] * P.ldah + col] = v[k];
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        const int64_t pos = ((int64_t)qq << BB) + k;
        const int64_t j = hi_part | (pos << P.s0) | lo;
        __builtin_nontemporal_store(v[k], P.Z + j * P.ldz + col);
      }
    }
  }
}

// Position of row j in the last pass's order: group g = (hi, lo), slot pos.
__device__ __forceinline__ int64_t last_pass_index(int64_t j, int s0, int B) {
  const int64_t hi = j >> (s0 + B);
  const int64_t lo = j & ((int64_t(1) << s0) - 1);
  const int64_t pos = (j >> s0) & ((int64_t(1) << B) - 1);
  return (hi << (s0 + B)) | (lo << B) | pos;
}

// pi_sgn[j] = pi(j) (or ~pi(j) when D_j = -1), in row order (the first pass reads it
// contiguously); slotA = sigma^{-1}(j) if < m_K else -1, in the last pass's order
__global__ void srht_index_kernel(int64_t npad, int p, uint64_t seed, int64_t mK, int s0_last,
                                  int b_last, int32_t* __restrict__ pi_sgn,
                                  int32_t* __restrict__ slotA) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < npad;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t src = rng::prp((uint64_t)j, seed, rng::kStreamP, p);
    const int D = rng::rademacher(seed, (uint64_t)j);
    pi_sgn[j] = D > 0 ? (int32_t)src : ~(int32_t)src;
    const uint64_t t = rng::prp_inv((uint64_t)j, seed, rng::kStreamS, p);
    slotA[last_pass_index(j, s0_last, b_last)] = t < (uint64_t)mK ? (int32_t)t : -1;
  }
}

// slotH (pre-filled with -1): the row sigma_hat(t) carries slot t, for t < r
__global__ void srht_hat_kernel(int64_t r, int p, uint64_t seed, int s0_last, int b_last,
                                int32_t* __restrict__ slotH) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < r;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = (int64_t)rng::prp((uint64_t)t, seed, rng::kStreamShat, p);
    slotH[last_pass_index(j, s0_last, b_last)] = (int32_t)t;
  }
}

template <typename T>
constexpr int ct_max() {
  return 128 / (int)sizeof(T);
}

// Column tile: 128 B row segments while the tile fits 128 KB of LDS; the
// narrow variant halves the tile so that two blocks share a CU.
template <typename T, bool NARROW>
constexpr int ct_for(int b) {
  return (b <= 10 ? ct_max<T>() : ct_max<T>() / 2) / (NARROW ? 2 : 1);
}

template <typename T, int B, int MODE, bool NARROW>
void launch_pass(PassParams<T> P, int64_t npad, hipStream_t s) {
  constexpr int BA = (B + 1) / 2;
  constexpr int BB = B / 2;
  constexpr int CT = ct_for<T, NARROW>(B);
  const int64_t groups = npad >> B;
  P.n_ct = (int)(P.ldz / CT);
  const int64_t blocks = groups * P.n_ct;
  if (blocks > 0x7fffffffLL) fail(SLSE_EUNSUPPORTED, "srht: grid too large");
  fwht_pass_kernel<T, CT, BA, BB, MODE><<<(unsigned)blocks, kPassThreads, 0, s>>>(P);
  SLSE_LAUNCH_CHECK();
}

template <typename T, int MODE, bool NARROW>
void dispatch_b(int b, PassParams<T> P, int64_t npad, hipStream_t s) {
  switch (b) {
#define SLSE_CASE(BV) \
  case BV: launch_pass<T, BV, MODE, NARROW>(P, npad, s); break;
    SLSE_CASE(1)
    SLSE_CASE(2)
    SLSE_CASE(3)
    SLSE_CASE(4)
    SLSE_CASE(5)
    SLSE_CASE(6)
    SLSE_CASE(7)
    SLSE_CASE(8)
    SLSE_CASE(9)
    SLSE_CASE(10)
    SLSE_CASE(11)
#undef SLSE_CASE
    default: fail(SLSE_EUNSUPPORTED, "srht: bad pass size");
  }
}

template <typename T, bool NARROW>
void dispatch_mode(int mode, int b, PassParams<T> P, int64_t npad, hipStream_t s) {
  switch (mode) {
    case 0: dispatch_b<T, 0, NARROW>(b, P, npad, s); break;
    case kFirst: dispatch_b<T, kFirst, NARROW>(b, P, npad, s); break;
    case kLast: dispatch_b<T, kLast, NARROW>(b, P, npad, s); break;
    default: dispatch_b<T, kFirst | kLast, NARROW>(b, P, npad, s); break;
  }
}

std::vector<int> pass_sizes(int p, int bmax) {
  const int npass = (int)ceil_div(p, bmax);
  std::vector<int> b(npass, p / npass);
  for (int i = 0; i < p % npass; ++i) b[i] += 1;
  return b;
}

template <typename T>
void run_passes(const SrhtArgs& a, hipStream_t s) {
  const int64_t npad = int64_t(1) << a.p;
  PassParams<T> P{};
  P.X = static_cast<const T*>(a.X);
  P.ldx = a.ldx;
  P.Y = static_cast<const T*>(a.Y);
  P.N = a.N;
  P.d = a.d;
  P.pi_sgn = a.pi_sgn;
  P.Z = static_cast<T*>(a.Z);
  P.ldz = a.ldz;
  P.slotA = a.slotA;
  P.slotH = a.slotH;
  P.A = static_cast<T*>(a.A);
  P.lda = a.lda;
  P.Ahat = static_cast<T*>(a.Ahat);
  P.ldah = a.ldah;
  const std::vector<int> bs = pass_sizes(a.p, a.bmax);
  int s0 = 0;
  for (size_t i = 0; i < bs.size(); ++i) {
    int mode = (i == 0 ? kFirst : 0) | (i + 1 == bs.size() ? kLast : 0);
    P.s0 = s0;
    if (a.narrow)
      dispatch_mode<T, true>(mode, bs[i], P, npad, s);
    else
      dispatch_mode<T, false>(mode, bs[i], P, npad, s);
    s0 += bs[i];
  }
}

}  // namespace

void srht_plan(SrhtArgs& a, int prefer_bmax) {
  const int es = (int)dtype_size(a.t);
  const int ctm = 128 / es;
  a.ct = ctm;
  a.ldz = round_up(a.d + 1, ctm);
  int bmax = prefer_bmax > 0 ? prefer_bmax : 10;
  if (const char* e = std::getenv("SLSE_SRHT_BMAX")) bmax = std::atoi(e);
  a.bmax = std::min(11, std::max(1, bmax));
  a.narrow = false;
  if (const char* e = std::getenv("SLSE_SRHT_NARROW")) a.narrow = std::atoi(e) != 0;
}

size_t srht_z_bytes(const SrhtArgs& a) {
  if (a.p <= a.bmax) return 0;  // a single pass needs no workspace
  return (size_t)(int64_t(1) << a.p) * (size_t)a.ldz * dtype_size(a.t);
}

void launch_srht(const SrhtArgs& a, hipStream_t s) {
  const int64_t npad = int64_t(1) << a.p;
  const int threads = 256;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(npad, threads), 16384));
  const std::vector<int> bs = pass_sizes(a.p, a.bmax);
  const int b_last = bs.back();
  const int s0_last = a.p - b_last;
  srht_index_kernel<<<blocks, threads, 0, s>>>(npad, a.p, a.seed, a.mK, s0_last, b_last,
                                               a.pi_sgn, a.slotA);
  SLSE_LAUNCH_CHECK();
  launch_fill_i32(a.slotH, -1, npad, s);
  srht_hat_kernel<<<(int)ceil_div(a.r, threads), threads, 0, s>>>(a.r, a.p, a.seed, s0_last,
                                                                  b_last, a.slotH);
  SLSE_LAUNCH_CHECK();
  if (a.t == SLSE_F64)
    run_passes<double>(a, s);
  else if (a.t == SLSE_F32)
    run_passes<float>(a, s);
  else
    fail(SLSE_EUNSUPPORTED, "srht: dtype");
}

}  // namespace slse
