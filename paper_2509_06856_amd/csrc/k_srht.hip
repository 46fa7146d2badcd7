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
#include <cstring>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "rng.hpp"

namespace slse {
namespace {

// kGroupOrder (two-pass transforms): the workspace Z holds its rows in the
// last pass's group order, so the last pass reads each group as contiguous
// rows and the first pass writes them at a stride instead
// kPregathered (first pass of Y's own transform): the rows were gathered
// through P with D applied by the index-map kernel, so they are read in order
enum { kFirst = 1, kLast = 2, kGroupOrder = 4, kPregathered = 8 };

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
  int64_t xcd_q;  // > 0: blocks [0, 8 xcd_q) are remapped so that each XCD walks a contiguous range
  int64_t blocks;  // work items (row groups x column tiles) of this pass
  int zb;          // kGroupOrder: stages of the last pass
};

// Threads per block: one phase-A item (a column of 2^BA rows) per thread when
// the group is small, at most 512 (up to 256 registers per thread).
template <int CT, int BB, int ROUNDS>
constexpr int pass_threads() {
  return (CT << BB) < 64 ? 64 : ((CT << BB) > 512 ? 512 : (CT << BB));
}

// ROUNDS > 1 exchanges the tile through LDS in ROUNDS slices of the high
// (phase-A) index, so a group of 2^B rows x CT columns needs only 1/ROUNDS of
// it in LDS; every thread keeps all its phase-A values in registers meanwhile.
// One work item (row group x column tile) `bid` of a pass.
template <typename T, int CT, int BA, int BB, int MODE, int ROUNDS>
__device__ __forceinline__ void fwht_pass(const PassParams<T>& P, int64_t bid) {
  constexpr int NT = pass_threads<CT, BB, ROUNDS>();
  constexpr int RA = 1 << BA;
  constexpr int RB = 1 << BB;
  constexpr int B = BA + BB;
  constexpr int RA_R = RA / ROUNDS;                  // phase-B row blocks per round
  constexpr int NA = RB * CT;                        // phase-A items
  constexpr int NB = RA_R * CT;                      // phase-B items per round
  constexpr int IA = (NA + NT - 1) / NT;
  constexpr int IB = (NB + NT - 1) / NT;
  constexpr int PAD = CT;  // one padded row per 2^BB rows spreads phase-B reads over the banks
  static_assert(RA_R * ROUNDS == RA, "rounds must divide 2^BA");
  __shared__ T tile[(RA_R << BB) * CT + RA_R * PAD];

  // index maps of this group, fetched once (contiguous: the first pass has
  // s0 = 0 and the slot maps are stored in the last pass's group order)
  __shared__ int32_t s_pi[((MODE & kFirst) && !(MODE & kPregathered)) ? (1 << B) : 1];
  __shared__ int32_t s_slot[(MODE & kLast) ? 2 * (1 << B) : 1];

  const int ct = (int)(bid % P.n_ct);
  const int64_t g = bid / P.n_ct;
  const int64_t lo = g & ((int64_t(1) << P.s0) - 1);
  const int64_t hi = g >> P.s0;
  const int64_t hi_part = hi << (P.s0 + B);
  const int col_base = ct * CT;
  if constexpr ((MODE & kFirst) != 0 && (MODE & kPregathered) == 0) {
    for (int k = threadIdx.x; k < (1 << B); k += NT) s_pi[k] = gptr(P.pi_sgn)[hi_part | k];
  }
  if constexpr ((MODE & kLast) != 0) {
    const int64_t gb = g << B;
    for (int k = threadIdx.x; k < (1 << B); k += NT) {
      s_slot[k] = gptr(P.slotA)[gb + k];
      s_slot[(1 << B) + k] = gptr(P.slotH)[gb + k];
    }
  }
  if constexpr ((MODE & kLast) != 0 || ((MODE & kFirst) != 0 && (MODE & kPregathered) == 0))
    __syncthreads();

  // phase A: 2^BA rows {q + k 2^BB} of one column per item; stages on the high BA bits
  T v[IA][RA];
#pragma unroll
  for (int ia = 0; ia < IA; ++ia) {
    const int it = ia * NT + threadIdx.x;
    if (NA % NT != 0 && it >= NA) break;
    const int c = it % CT;
    const int q = it / CT;
    const int col = col_base + c;
    if constexpr ((MODE & kPregathered) != 0) {
      // rows hi_part | (q + k 2^BB) of the pregathered values, in order
#pragma unroll
      for (int k = 0; k < RA; ++k) v[ia][k] = __builtin_nontemporal_load(gptr(P.X + (hi_part | (q + (k << BB)))));
    } else if constexpr ((MODE & kFirst) != 0) {
      // gather through P with D applied; branch-free so that all 2^BA loads
      // are in flight together (out-of-range rows and padding columns read a
      // valid address and are zeroed afterwards)
      // The sign and keep flags of the 2^BA rows are packed into two
      // per-thread bit masks, so that no per-load state pins registers and
      // every load is issued before the first one is consumed.
      static_assert(RA <= 64, "flag masks hold 64 rows");
      using U = typename std::conditional<sizeof(T) == 8, uint64_t, uint32_t>::type;
      uint64_t negm = 0, keepm = 0;
      U raw[RA];
#pragma unroll
      for (int k = 0; k < RA; ++k) {
        const int32_t ps = s_pi[q + (k << BB)];
        const bool neg = ps < 0;
        const int64_t src = neg ? (int64_t)(~ps) : (int64_t)ps;
        const bool in_rows = src < P.N;
        const int64_t srow = in_rows ? src : 0;
        // select the address as an integer so that the load stays unconditional
        const uintptr_t ax = reinterpret_cast<uintptr_t>(P.X + srow * P.ldx + col);
        const uintptr_t ay = reinterpret_cast<uintptr_t>(P.Y + srow);
        const T* addr = reinterpret_cast<const T*>(col < P.d ? ax : ay);
        raw[k] = __builtin_bit_cast(U, __builtin_nontemporal_load(gptr(addr)));
        negm |= (uint64_t)neg << k;
        keepm |= (uint64_t)(in_rows && col <= P.d) << k;
      }
      // keep the scheduler from consuming early loads while later ones are
      // still to be issued (it would cap the loads in flight at a handful)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < RA; ++k) {
        const U sgn = (U)((negm >> k) & 1) << (8 * sizeof(T) - 1);
        const U keep = (U)0 - (U)((keepm >> k) & 1);
        v[ia][k] = __builtin_bit_cast(T, (U)((raw[k] ^ sgn) & keep));
      }
    } else {
#pragma unroll
      for (int k = 0; k < RA; ++k) {
        const int64_t pos = q + (k << BB);
        const int64_t j = (MODE & kGroupOrder) ? ((g << B) | pos) : (hi_part | (pos << P.s0) | lo);
        v[ia][k] = __builtin_nontemporal_load(gptr(P.Z + j * P.ldz + col));
      }
    }
#pragma unroll
    for (int h = 1; h < RA; h <<= 1)
#pragma unroll
      for (int k = 0; k < RA; ++k)
        if ((k & h) == 0) {
          const T a0 = v[ia][k], a1 = v[ia][k + h];
          v[ia][k] = a0 + a1;
          v[ia][k + h] = a0 - a1;
        }
  }

#pragma unroll
  for (int rho = 0; rho < ROUNDS; ++rho) {
    if (rho > 0) __syncthreads();  // the previous round's phase-B reads are done
    // rows q + k 2^BB with k in this round's slice go to LDS (local k)
#pragma unroll
    for (int ia = 0; ia < IA; ++ia) {
      const int it = ia * NT + threadIdx.x;
      if (NA % NT != 0 && it >= NA) break;
      const int c = it % CT;
      const int q = it / CT;
#pragma unroll
      for (int kl = 0; kl < RA_R; ++kl)
        tile[(q + (kl << BB)) * CT + c + kl * PAD] = v[ia][rho * RA_R + kl];
    }
    __syncthreads();

    // phase B: 2^BB consecutive rows {qq 2^BB + k} per item; stages on the low BB bits
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
      const int it = ib * NT + threadIdx.x;
      if (NB % NT != 0 && it >= NB) break;
      const int c = it % CT;
      const int ql = it / CT;
      const int qq = rho * RA_R + ql;
      const int col = col_base + c;
      T w[RB];
#pragma unroll
      for (int k = 0; k < RB; ++k) w[k] = tile[((ql << BB) + k) * CT + c + ql * PAD];
#pragma unroll
      for (int h = 1; h < RB; h <<= 1)
#pragma unroll
        for (int k = 0; k < RB; ++k)
          if ((k & h) == 0) {
            const T a0 = w[k], a1 = w[k + h];
            w[k] = a0 + a1;
            w[k + h] = a0 - a1;
          }
      if constexpr ((MODE & kLast) != 0) {
        if (col <= P.d) {
          // slots are read from LDS at the store, not held in registers
#pragma unroll
          for (int k = 0; k < RB; ++k) {
            const int32_t sa = s_slot[(qq << BB) + k];
            const int32_t sh = s_slot[(1 << B) + (qq << BB) + k];
            if (sa >= 0) __builtin_nontemporal_store(w[k], gptr(P.A + (int64_t)sa * P.lda + col));
            if (sh >= 0) *gptr(P.Ahat + (int64_t)sh * P.ldah + col) = w[k];
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          const int64_t pos = ((int64_t)qq << BB) + k;
          // group order: the first pass (s0 = 0) holds rows (g, pos), which
          // the last pass's group pos reads at slot g
          const int64_t j = (MODE & kGroupOrder) ? ((pos << P.zb) | g) : (hi_part | (pos << P.s0) | lo);
          __builtin_nontemporal_store(w[k], gptr(P.Z + j * P.ldz + col));
        }
      }
    }
  }
}

template <typename T, int CT, int BA, int BB, int MODE, int ROUNDS>
__global__ __launch_bounds__((pass_threads<CT, BB, ROUNDS>())) void fwht_pass_kernel(PassParams<T> P) {
  // Workgroups are dealt to the 8 XCDs round-robin.  Remapping block b to
  // (b % 8) q + b / 8 hands each XCD a contiguous run of work items, so the
  // column tiles of one row group run back to back on the same XCD: the
  // partial cache lines they write meet in that XCD's L2 and the DRAM pages
  // of the rows they touch are reused while open.
  int64_t bid = blockIdx.x;
  if (P.xcd_q > 0 && bid < 8 * P.xcd_q) bid = (bid & 7) * P.xcd_q + (bid >> 3);
  fwht_pass<T, CT, BA, BB, MODE, ROUNDS>(P, bid);
}

// The same pass for several transforms at once: blockIdx.y picks the
// transform's parameters, blockIdx.x its work item (blocks past the
// transform's own count return at once).
template <typename T, int CT, int BA, int BB, int MODE, int ROUNDS>
__global__ __launch_bounds__((pass_threads<CT, BB, ROUNDS>())) void fwht_pass_batched_kernel(
    const PassParams<T>* __restrict__ Ps) {
  const PassParams<T> P = Ps[blockIdx.y];
  if ((int64_t)blockIdx.x >= P.blocks) return;
  fwht_pass<T, CT, BA, BB, MODE, ROUNDS>(P, blockIdx.x);
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
// The permutation of [0, 2^p) (INV: its inverse) of every index j = j0,
// j0 + stride, .. < n, handed to emit(j, value).  Cycle walking (an odd p
// walks twice on average) would hold a wave for its longest walk; here every
// iteration evaluates the Feistel network once per lane, on the lane's next
// index as soon as its current one has left the walking range.  The values
// are those of rng::prp / rng::prp_inv.
template <bool INV, typename Emit>
__device__ __forceinline__ void prp_each(int64_t j0, int64_t n, int64_t stride, uint64_t seed,
                                         uint64_t stream, int p, Emit&& emit) {
  if (j0 >= n) return;
  const int h = (p + 1) >> 1;
  const uint64_t lim = uint64_t(1) << p;
  int64_t j = j0;
  uint64_t x = (uint64_t)j;
  while (true) {
    const uint64_t y =
        INV ? rng::feistel_dec(x, seed, stream, h) : rng::feistel_enc(x, seed, stream, h);
    if (y < lim) {
      emit(j, y);
      j += stride;
      if (j >= n) break;
      x = (uint64_t)j;
    } else {
      x = y;
    }
  }
}

// pi_sgn and slotA of the indices j0, j0 + stride, .. < npad
__device__ __forceinline__ void srht_index_range(int64_t j0, int64_t stride, int64_t npad, int p,
                                                 uint64_t seed, int64_t mK, int s0_last, int b_last,
                                                 int32_t* __restrict__ pi_sgn,
                                                 int32_t* __restrict__ slotA) {
  prp_each<false>(j0, npad, stride, seed, rng::kStreamP, p,
                  [&](int64_t j, uint64_t src) { gptr(pi_sgn)[j] = (int32_t)src; });
  // the signs D over the same indices (each thread rereads its own writes)
  for (int64_t j = j0; j < npad; j += stride)
    if (rng::rademacher(seed, (uint64_t)j) < 0) gptr(pi_sgn)[j] = ~gptr(pi_sgn)[j];
  prp_each<true>(j0, npad, stride, seed, rng::kStreamS, p, [&](int64_t j, uint64_t t) {
    gptr(slotA)[last_pass_index(j, s0_last, b_last)] = t < (uint64_t)mK ? (int32_t)t : -1;
  });
}

__global__ void srht_index_kernel(int64_t npad, int p, uint64_t seed, int64_t mK, int s0_last,
                                  int b_last, int32_t* __restrict__ pi_sgn,
                                  int32_t* __restrict__ slotA) {
  srht_index_range(blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x,
                   npad, p, seed, mK, s0_last, b_last, pi_sgn, slotA);
}

// The same maps, and Y gathered through P with D applied, in row order:
// yp[j] = D_j Y[pi(j)] (+0 past N), the bits the first pass's gather would
// form; Y's own first pass then reads its rows in order, and the random reads
// of Y overlap the Feistel arithmetic here.
template <typename T>
__global__ void srht_index_y_kernel(int64_t npad, int p, uint64_t seed, int64_t mK, int s0_last,
                                    int b_last, int32_t* __restrict__ pi_sgn,
                                    int32_t* __restrict__ slotA, const T* __restrict__ Y, int64_t N,
                                    T* __restrict__ yp) {
  const int64_t j0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  srht_index_range(j0, stride, npad, p, seed, mK, s0_last, b_last, pi_sgn, slotA);
  for (int64_t j = j0; j < npad; j += stride) {
    const int32_t ps = gptr(pi_sgn)[j];
    const bool neg = ps < 0;
    const int64_t src = neg ? (int64_t)(~ps) : (int64_t)ps;
    const T v = src < N ? gptr(Y)[src] : (T)0;
    gptr(yp)[j] = src < N ? (neg ? -v : v) : (T)0;
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
constexpr int ct_of() {
  return 128 / (int)sizeof(T);  // 128-byte row segments
}

// Passes of up to 10 stages exchange the whole 2^B x CT tile through LDS at
// once (128 KB at B = 10); an 11-stage pass does it in two rounds.
template <typename T, int B, int MODE, int CT = ct_of<T>()>
void launch_pass(PassParams<T> P, int64_t npad, hipStream_t s) {
  constexpr int BA = (B + 1) / 2;
  constexpr int BB = B / 2;
  constexpr int ROUNDS = B > 10 ? 2 : 1;
  const int64_t groups = npad >> B;
  P.n_ct = (int)(P.ldz / CT);
  const int64_t blocks = groups * P.n_ct;
  if (blocks > 0x7fffffffLL) fail(SLSE_EUNSUPPORTED, "srht: grid too large");
  P.blocks = blocks;
  P.xcd_q = P.xcd_q != 0 ? blocks / 8 : 0;
  fwht_pass_kernel<T, CT, BA, BB, MODE, ROUNDS>
      <<<(unsigned)blocks, pass_threads<CT, BB, ROUNDS>(), 0, s>>>(P);
  SLSE_LAUNCH_CHECK();
}

template <typename T, int MODE>
void dispatch_b(int b, PassParams<T> P, int64_t npad, hipStream_t s) {
  switch (b) {
#define SLSE_CASE(BV) \
  case BV: launch_pass<T, BV, MODE>(P, npad, s); break;
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

// the one-column passes of Y (two-pass transforms in group order only)
template <typename T, int MODE>
void dispatch_b_y(int b, PassParams<T> P, int64_t npad, hipStream_t s) {
  switch (b) {
#define SLSE_CASE(BV) \
  case BV: launch_pass<T, BV, MODE, 1>(P, npad, s); break;
    SLSE_CASE(6)
    SLSE_CASE(7)
    SLSE_CASE(8)
    SLSE_CASE(9)
    SLSE_CASE(10)
    SLSE_CASE(11)
#undef SLSE_CASE
    default: fail(SLSE_EUNSUPPORTED, "srht: bad pass size for the Y passes");
  }
}

template <typename T>
void dispatch_mode(int mode, int b, PassParams<T> P, int64_t npad, hipStream_t s) {
  switch (mode) {
    case 0: dispatch_b<T, 0>(b, P, npad, s); break;
    case kFirst: dispatch_b<T, kFirst>(b, P, npad, s); break;
    case kLast: dispatch_b<T, kLast>(b, P, npad, s); break;
    case kFirst | kGroupOrder: dispatch_b<T, kFirst | kGroupOrder>(b, P, npad, s); break;
    case kLast | kGroupOrder: dispatch_b<T, kLast | kGroupOrder>(b, P, npad, s); break;
    default: dispatch_b<T, kFirst | kLast>(b, P, npad, s); break;
  }
}

template <typename T, int B, int MODE>
void launch_pass_batched(const PassParams<T>* d_params, int count, int64_t max_blocks, hipStream_t s) {
  constexpr int BA = (B + 1) / 2;
  constexpr int BB = B / 2;
  constexpr int CT = ct_of<T>();
  constexpr int ROUNDS = B > 10 ? 2 : 1;
  fwht_pass_batched_kernel<T, CT, BA, BB, MODE, ROUNDS>
      <<<dim3((unsigned)max_blocks, (unsigned)count), pass_threads<CT, BB, ROUNDS>(), 0, s>>>(d_params);
  SLSE_LAUNCH_CHECK();
}

template <typename T, int MODE>
void dispatch_b_batched(int b, const PassParams<T>* d, int count, int64_t max_blocks, hipStream_t s) {
  switch (b) {
#define SLSE_CASE(BV) \
  case BV: launch_pass_batched<T, BV, MODE>(d, count, max_blocks, s); break;
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

template <typename T>
void dispatch_mode_batched(int mode, int b, const PassParams<T>* d, int count, int64_t max_blocks,
                           hipStream_t s) {
  switch (mode) {
    case 0: dispatch_b_batched<T, 0>(b, d, count, max_blocks, s); break;
    case kFirst: dispatch_b_batched<T, kFirst>(b, d, count, max_blocks, s); break;
    case kLast: dispatch_b_batched<T, kLast>(b, d, count, max_blocks, s); break;
    case kFirst | kGroupOrder:
      dispatch_b_batched<T, kFirst | kGroupOrder>(b, d, count, max_blocks, s);
      break;
    case kLast | kGroupOrder:
      dispatch_b_batched<T, kLast | kGroupOrder>(b, d, count, max_blocks, s);
      break;
    default: dispatch_b_batched<T, kFirst | kLast>(b, d, count, max_blocks, s); break;
  }
}

std::vector<int> pass_sizes(int p, int bmax) {
  const int npass = (int)ceil_div(p, bmax);
  std::vector<int> b(npass, p / npass);
  for (int i = 0; i < p % npass; ++i) b[i] += 1;
  return b;
}

// whether two-pass transforms keep Z in the last pass's group order
// (SLSE_SRHT_GROUP_ORDER overrides)
bool srht_group_order() {
  static const bool v = [] {
    const char* e = std::getenv("SLSE_SRHT_GROUP_ORDER");
    return e ? std::atoi(e) != 0 : true;
  }();
  return v;
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
  P.xcd_q = a.xcd_swizzle ? 1 : 0;
  const std::vector<int> bs = pass_sizes(a.p, a.bmax);
  int s0 = 0;
  for (size_t i = 0; i < bs.size(); ++i) {
    int mode = (i == 0 ? kFirst : 0) | (i + 1 == bs.size() ? kLast : 0);
    if (bs.size() == 2 && srht_group_order()) mode |= kGroupOrder;
    P.zb = bs.back();
    P.s0 = s0;
    dispatch_mode<T>(mode, bs[i], P, npad, s);
    s0 += bs[i];
  }
  if (a.split_y) {
    // Y on its own: a one-column transform with the same index maps, its
    // workspace after X's, its sampled values into column d of A and A_hat
    PassParams<T> Q = P;
    Q.X = static_cast<const T*>(a.Y);  // not read: every column is past d = 0
    Q.ldx = 1;
    Q.d = 0;
    Q.Z = static_cast<T*>(a.Z) + npad * a.ldz;
    Q.ldz = 1;
    Q.A = static_cast<T*>(a.A) + a.d;
    Q.Ahat = static_cast<T*>(a.Ahat) + a.d;
    Q.zb = bs.back();
    Q.s0 = 0;
    if (a.y_pregathered) {
      Q.X = static_cast<const T*>(a.Z) + npad * (a.ldz + 1);  // yp, written with the index maps
      dispatch_b_y<T, kFirst | kGroupOrder | kPregathered>(bs[0], Q, npad, s);
    } else {
      dispatch_b_y<T, kFirst | kGroupOrder>(bs[0], Q, npad, s);
    }
    Q.s0 = bs[0];
    dispatch_b_y<T, kLast | kGroupOrder>(bs[1], Q, npad, s);
  }
}

// Parameter records of every pass of every transform, ordered by pass round
// (a transform's passes run in order), then by pass shape; one launch per
// (round, shape) covers every transform with that pass.
template <typename T>
std::vector<SrhtBatchLaunch> batch_plan_t(const std::vector<SrhtArgs>& as, std::vector<char>& rec) {
  struct Item {
    int round, mode, b;
    PassParams<T> P;
  };
  std::vector<Item> items;
  constexpr int CT = ct_of<T>();
  for (const SrhtArgs& a : as) {
    if (a.ldz % CT != 0) fail(SLSE_EINVAL, "srht batch: workspace rows must be whole column tiles");
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
    P.xcd_q = 0;
    P.n_ct = (int)(a.ldz / CT);
    const std::vector<int> bs = pass_sizes(a.p, a.bmax);
    if (bs.size() > 1 && a.Z == nullptr) fail(SLSE_EINVAL, "srht batch: missing workspace");
    int s0 = 0;
    for (size_t i = 0; i < bs.size(); ++i) {
      int mode = (i == 0 ? kFirst : 0) | (i + 1 == bs.size() ? kLast : 0);
      if (bs.size() == 2 && srht_group_order()) mode |= kGroupOrder;
      P.zb = bs.back();
      P.s0 = s0;
      P.blocks = ((int64_t(1) << a.p) >> bs[i]) * P.n_ct;
      if (P.blocks > 0x7fffffffLL) fail(SLSE_EUNSUPPORTED, "srht: grid too large");
      items.push_back({(int)i, mode, bs[i], P});
      s0 += bs[i];
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) {
    if (x.round != y.round) return x.round < y.round;
    if (x.mode != y.mode) return x.mode < y.mode;
    return x.b < y.b;
  });
  std::vector<SrhtBatchLaunch> L;
  rec.assign(items.size() * sizeof(PassParams<T>), 0);
  for (size_t k = 0; k < items.size(); ++k) {
    std::memcpy(rec.data() + k * sizeof(PassParams<T>), &items[k].P, sizeof(PassParams<T>));
    const bool same = !L.empty() && k > 0 && items[k - 1].round == items[k].round &&
                      items[k - 1].mode == items[k].mode && items[k - 1].b == items[k].b &&
                      L.back().count < 65535;
    if (!same) {
      SrhtBatchLaunch l;
      l.b = items[k].b;
      l.mode = items[k].mode;
      l.first = (int)k;
      L.push_back(l);
    }
    L.back().count += 1;
    L.back().max_blocks = std::max(L.back().max_blocks, items[k].P.blocks);
  }
  return L;
}

}  // namespace

std::vector<SrhtBatchLaunch> srht_batch_plan(const std::vector<SrhtArgs>& as, slse_dtype t,
                                             std::vector<char>& records) {
  if (t == SLSE_F64) return batch_plan_t<double>(as, records);
  if (t == SLSE_F32) return batch_plan_t<float>(as, records);
  fail(SLSE_EUNSUPPORTED, "srht: dtype");
}

void launch_srht_batched(const std::vector<SrhtBatchLaunch>& L, const void* d_records, slse_dtype t,
                         hipStream_t s) {
  for (const SrhtBatchLaunch& l : L) {
    if (t == SLSE_F64) {
      const auto* d = static_cast<const PassParams<double>*>(d_records) + l.first;
      dispatch_mode_batched<double>(l.mode, l.b, d, l.count, l.max_blocks, s);
    } else if (t == SLSE_F32) {
      const auto* d = static_cast<const PassParams<float>*>(d_records) + l.first;
      dispatch_mode_batched<float>(l.mode, l.b, d, l.count, l.max_blocks, s);
    } else {
      fail(SLSE_EUNSUPPORTED, "srht: dtype");
    }
  }
}

void srht_plan(SrhtArgs& a, int prefer_bmax) {
  const int es = (int)dtype_size(a.t);
  const int ctm = 128 / es;
  a.ct = ctm;
  a.ldz = round_up(a.d + 1, ctm);
  // 11-stage passes (two LDS rounds) keep FP32 in registers; FP64 would spill
  int bmax = prefer_bmax > 0 ? prefer_bmax : (es == 4 ? 11 : 10);
  if (const char* e = std::getenv("SLSE_SRHT_BMAX")) bmax = std::atoi(e);
  a.bmax = std::min(11, std::max(1, bmax));
  a.xcd_swizzle = true;
  if (const char* e = std::getenv("SLSE_SRHT_XCD")) a.xcd_swizzle = std::atoi(e) != 0;
}

void srht_split_y(SrhtArgs& a) {
  a.split_y = false;
  if (const char* e = std::getenv("SLSE_SRHT_SPLIT_Y"))
    if (std::atoi(e) == 0) return;
  if (a.d <= 0 || a.d % a.ct != 0 || pass_sizes(a.p, a.bmax).size() != 2 || !srht_group_order())
    return;
  a.split_y = true;
  a.ldz = a.d;
}

size_t srht_z_bytes(const SrhtArgs& a) {
  if (a.p <= a.bmax) return 0;  // a single pass needs no workspace
  // X's columns, then Y's own column and Y gathered through P (split_y)
  return (size_t)(int64_t(1) << a.p) * (size_t)(a.ldz + (a.split_y ? 2 : 0)) * dtype_size(a.t);
}

namespace {

// Index maps of many transforms: blockIdx.y picks the job (its fields are
// uniform over the block), blockIdx.x and the threads stride over its rows.
// Every row index: pi_sgn, slotA (as srht_index_kernel) and slotH = -1.
__global__ void srht_index_batched_kernel(const SrhtIndexJob* __restrict__ jobs) {
  const SrhtIndexJob jb = jobs[blockIdx.y];
  const int64_t j0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  srht_index_range(j0, stride, jb.npad, jb.p, jb.seed, jb.mK, jb.s0_last, jb.b_last, jb.pi_sgn,
                   jb.slotA);
  for (int64_t j = j0; j < jb.npad; j += stride) gptr(jb.slotH)[j] = -1;
}

// every Hessian sample of every job (after the kernel above)
__global__ void srht_hat_batched_kernel(const SrhtIndexJob* __restrict__ jobs) {
  const SrhtIndexJob jb = jobs[blockIdx.y];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < jb.r;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = (int64_t)rng::prp((uint64_t)t, jb.seed, rng::kStreamShat, jb.p);
    gptr(jb.slotH)[last_pass_index(j, jb.s0_last, jb.b_last)] = (int32_t)t;
  }
}

}  // namespace

void srht_last_pass(const SrhtArgs& a, int* s0_last, int* b_last) {
  const std::vector<int> bs = pass_sizes(a.p, a.bmax);
  *b_last = bs.back();
  *s0_last = a.p - bs.back();
}

void launch_srht_index_batched(const SrhtIndexJob* jobs, int B, int64_t max_npad, int64_t max_r,
                               hipStream_t s) {
  if (B <= 0) return;
  const int threads = 256;
  // about four rows per thread in the largest job; blocks past a smaller
  // job's rows return at once
  for (int j0 = 0; j0 < B; j0 += 65535) {
    const int nb = std::min(65535, B - j0);
    const int bx = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(max_npad, 4 * threads), 4096));
    srht_index_batched_kernel<<<dim3(bx, nb), threads, 0, s>>>(jobs + j0);
    SLSE_LAUNCH_CHECK();
    const int hx = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(max_r, 4 * threads), 4096));
    srht_hat_batched_kernel<<<dim3(hx, nb), threads, 0, s>>>(jobs + j0);
    SLSE_LAUNCH_CHECK();
  }
}

void launch_srht(const SrhtArgs& a, hipStream_t s) {
  if (a.indices_ready) {
    if (a.t == SLSE_F64)
      run_passes<double>(a, s);
    else if (a.t == SLSE_F32)
      run_passes<float>(a, s);
    else
      fail(SLSE_EUNSUPPORTED, "srht: dtype");
    return;
  }
  const int64_t npad = int64_t(1) << a.p;
  const int threads = 256;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(npad, threads), 16384));
  const std::vector<int> bs = pass_sizes(a.p, a.bmax);
  const int b_last = bs.back();
  const int s0_last = a.p - b_last;
  // with Y on its own, Y is gathered through P together with the maps
  // (SLSE_SRHT_Y_PREGATHER=0: in its first pass instead)
  SrhtArgs b = a;
  b.y_pregathered = a.split_y;
  if (const char* e = std::getenv("SLSE_SRHT_Y_PREGATHER"))
    if (std::atoi(e) == 0) b.y_pregathered = false;
  if (b.y_pregathered && a.t == SLSE_F32) {
    srht_index_y_kernel<float><<<blocks, threads, 0, s>>>(
        npad, a.p, a.seed, a.mK, s0_last, b_last, a.pi_sgn, a.slotA, static_cast<const float*>(a.Y),
        a.N, static_cast<float*>(a.Z) + npad * (a.ldz + 1));
  } else if (b.y_pregathered && a.t == SLSE_F64) {
    srht_index_y_kernel<double><<<blocks, threads, 0, s>>>(
        npad, a.p, a.seed, a.mK, s0_last, b_last, a.pi_sgn, a.slotA, static_cast<const double*>(a.Y),
        a.N, static_cast<double*>(a.Z) + npad * (a.ldz + 1));
  } else {
    b.y_pregathered = false;
    srht_index_kernel<<<blocks, threads, 0, s>>>(npad, a.p, a.seed, a.mK, s0_last, b_last,
                                                 a.pi_sgn, a.slotA);
  }
  SLSE_LAUNCH_CHECK();
  launch_fill_i32(a.slotH, -1, npad, s);
  srht_hat_kernel<<<(int)ceil_div(a.r, threads), threads, 0, s>>>(a.r, a.p, a.seed, s0_last,
                                                                  b_last, a.slotH);
  SLSE_LAUNCH_CHECK();
  if (a.t == SLSE_F64)
    run_passes<double>(b, s);
  else if (a.t == SLSE_F32)
    run_passes<float>(b, s);
  else
    fail(SLSE_EUNSUPPORTED, "srht: dtype");
}

}  // namespace slse
