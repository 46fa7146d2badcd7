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

  const int ct = blockIdx.x % P.n_ct;
  const int64_t g = blockIdx.x / P.n_ct;
  const int64_t lo = g & ((int64_t(1) << P.s0) - 1);
  const int64_t hi = g >> P.s0;
  const int64_t hi_part = hi << (P.s0 + B);
  const int col_base = ct * CT;

  // phase A: 2^BA rows {q + k 2^BB} of one column per item; stages on the high BA bits
  for (int it = threadIdx.x; it < RB * CT; it += kPassThreads) {
    const int c = it % CT;
    const int q = it / CT;
    const int col = col_base + c;
    T v[RA];
#pragma unroll
    for (int k = 0; k < RA; ++k) {
      const int64_t pos = q + (k << BB);
      const int64_t j = hi_part | (pos << P.s0) | lo;
      if constexpr ((MODE & kFirst) != 0) {
        const int32_t ps = P.pi_sgn[j];
        const bool neg = ps < 0;
        const int64_t src = neg ? (int64_t)(~ps) : (int64_t)ps;
        T val = (T)0;
        if (src < P.N) {
          if (col < P.d)
            val = P.X[src * P.ldx + col];
          else if (col == P.d)
            val = P.Y[src];
        }
        v[k] = neg ? -val : val;
      } else {
        v[k] = P.Z[j * P.ldz + col];
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
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int64_t pos = ((int64_t)qq << BB) + k;
      const int64_t j = hi_part | (pos << P.s0) | lo;
      if constexpr ((MODE & kLast) != 0) {
        if (col <= P.d) {
          const int32_t sa = P.slotA[j];
          if (sa >= 0) P.A[(int64_t)sa * P.lda + col] = v[k];
          const int32_t sh = P.slotH[j];
          if (sh >= 0) P.Ahat[(int64_t)sh * P.ldah + col] = v[k];
        }
      } else {
        P.Z[j * P.ldz + col] = v[k];
      }
    }
  }
}

// pi_sgn[j] = pi(j) (or ~pi(j) when D_j = -1); slotA[j] = sigma^{-1}(j) if < m_K else -1
__global__ void srht_index_kernel(int64_t npad, int p, uint64_t seed, int64_t mK,
                                  int32_t* __restrict__ pi_sgn, int32_t* __restrict__ slotA) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < npad;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t src = rng::prp((uint64_t)j, seed, rng::kStreamP, p);
    const int D = rng::rademacher(seed, (uint64_t)j);
    pi_sgn[j] = D > 0 ? (int32_t)src : ~(int32_t)src;
    const uint64_t t = rng::prp_inv((uint64_t)j, seed, rng::kStreamS, p);
    slotA[j] = t < (uint64_t)mK ? (int32_t)t : -1;
  }
}

// slotH[sigma_hat(t)] = t for t < r (slotH pre-filled with -1)
__global__ void srht_hat_kernel(int64_t r, int p, uint64_t seed, int32_t* __restrict__ slotH) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < r;
       t += (int64_t)gridDim.x * blockDim.x) {
    slotH[rng::prp((uint64_t)t, seed, rng::kStreamShat, p)] = (int32_t)t;
  }
}

template <typename T>
constexpr int ct_max() {
  return 128 / (int)sizeof(T);
}

template <typename T>
constexpr int ct_for(int b) {
  return b <= 10 ? ct_max<T>() : ct_max<T>() / 2;
}

template <typename T, int B, int MODE>
void launch_pass(PassParams<T> P, int64_t npad, hipStream_t s) {
  constexpr int BA = (B + 1) / 2;
  constexpr int BB = B / 2;
  constexpr int CT = ct_for<T>(B);
  const int64_t groups = npad >> B;
  P.n_ct = (int)(P.ldz / CT);
  const int64_t blocks = groups * P.n_ct;
  if (blocks > 0x7fffffffLL) fail(SLSE_EUNSUPPORTED, "srht: grid too large");
  fwht_pass_kernel<T, CT, BA, BB, MODE><<<(unsigned)blocks, kPassThreads, 0, s>>>(P);
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

template <typename T>
void dispatch_mode(int mode, int b, PassParams<T> P, int64_t npad, hipStream_t s) {
  switch (mode) {
    case 0: dispatch_b<T, 0>(b, P, npad, s); break;
    case kFirst: dispatch_b<T, kFirst>(b, P, npad, s); break;
    case kLast: dispatch_b<T, kLast>(b, P, npad, s); break;
    default: dispatch_b<T, kFirst | kLast>(b, P, npad, s); break;
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
    dispatch_mode<T>(mode, bs[i], P, npad, s);
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
}

size_t srht_z_bytes(const SrhtArgs& a) {
  if (a.p <= a.bmax) return 0;  // a single pass needs no workspace
  return (size_t)(int64_t(1) << a.p) * (size_t)a.ldz * dtype_size(a.t);
}

void launch_srht(const SrhtArgs& a, hipStream_t s) {
  const int64_t npad = int64_t(1) << a.p;
  const int threads = 256;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(npad, threads), 16384));
  srht_index_kernel<<<blocks, threads, 0, s>>>(npad, a.p, a.seed, a.mK, a.pi_sgn, a.slotA);
  SLSE_LAUNCH_CHECK();
  launch_fill_i32(a.slotH, -1, npad, s);
  srht_hat_kernel<<<(int)ceil_div(a.r, threads), threads, 0, s>>>(a.r, a.p, a.seed, a.slotH);
  SLSE_LAUNCH_CHECK();
  if (a.t == SLSE_F64)
    run_passes<double>(a, s);
  else if (a.t == SLSE_F32)
    run_passes<float>(a, s);
  else
    fail(SLSE_EUNSUPPORTED, "srht: dtype");
}

}  // namespace slse
