// Counter-based randomness of the sketches (host and device).
//
// The SRHT draws a Rademacher diagonal D, a uniform permutation P and a row
// sampling B (Sec. 3, the SRHT definition); the CountSketch one +-1 per column
// and the Gaussian sketch iid entries (Sec. 1.2).  Every draw here is a pure
// function of (seed, stream, index) through Philox4x64-10 (Salmon, Moraes,
// Dror, Shaw, SC'11), so any entry can be recomputed where it is consumed.
//
// Stream ids (key word 1): 1 D, 2 P, 3 sigma, 4 sigma_hat, 5 CountSketch of
// S_K, 6 CountSketch of S_hat, 7 Gaussian S, 8 Gaussian S_hat.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace slse {
namespace rng {

enum : uint64_t {
  kStreamD = 1,
  kStreamP = 2,
  kStreamS = 3,
  kStreamShat = 4,
  kStreamCS = 5,
  kStreamCShat = 6,
  kStreamG = 7,
  kStreamGhat = 8,
};

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
constexpr int kFeistelRounds = 4;

struct Words {
  uint64_t w[4];
};

// The 128-bit product a * b.  On the device it is built from 32 x 32 -> 64-bit
// multiply-adds (v_mad_u64_u32, whose scalar destination is the carry out of
// the 64-bit add): with a = a1 2^32 + a0 and b = b1 2^32 + b0,
//   t1 = a0 b1 + hi32(a0 b0)      (cannot overflow),
//   s  = a1 b0 + t1               (its carry c is kept),
//   lo = lo32(s) 2^32 + lo32(a0 b0),  hi = a1 b1 + (c 2^32 + hi32(s)).
// The compiler's own lowering splits s into 32-bit halves and spends register
// moves and a 64-bit add on them.
__host__ __device__ __forceinline__ void mulhilo(uint64_t a, uint64_t b, uint64_t& hi,
                                                 uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p0 = (uint64_t)a0 * b0;
  const uint64_t t1 = (uint64_t)a0 * b1 + (p0 >> 32);
  uint64_t s, c;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(s), "=s"(c) : "v"(a1), "v"(b0), "v"(t1));
  uint32_t cbit;
  asm("v_cndmask_b32_e64 %0, 0, 1, %1" : "=v"(cbit) : "s"(c));
  lo = (s << 32) | (p0 & 0xffffffffu);
  hi = (uint64_t)a1 * b1 + ((s >> 32) | ((uint64_t)cbit << 32));
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  lo = (uint64_t)p;
  hi = (uint64_t)(p >> 64);
#endif
}

// Philox4x64-10 state between rounds: counter words and key.
struct PhiloxState {
  uint64_t c[4];
  uint64_t k0, k1;
};

// round r (0..9) of Philox4x64-10: the key is bumped by the Weyl constants
// before every round but the first
__host__ __device__ __forceinline__ void philox_round(PhiloxState& s, int r) {
  if (r) {
    s.k0 += kW0;
    s.k1 += kW1;
  }
  uint64_t hi0, lo0, hi1, lo1;
  mulhilo(kM0, s.c[0], hi0, lo0);
  mulhilo(kM1, s.c[2], hi1, lo1);
  const uint64_t n0 = hi1 ^ s.c[1] ^ s.k0;
  const uint64_t n2 = hi0 ^ s.c[3] ^ s.k1;
  s.c[0] = n0;
  s.c[1] = lo1;
  s.c[2] = n2;
  s.c[3] = lo0;
}

// Philox4x64-10 block: 10 rounds, key bumped by the Weyl constants between them.
__host__ __device__ __forceinline__ Words philox(uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t c3, uint64_t k0, uint64_t k1) {
  PhiloxState s{{c0, c1, c2, c3}, k0, k1};
#pragma unroll
  for (int r = 0; r < 10; ++r) philox_round(s, r);
  return Words{{s.c[0], s.c[1], s.c[2], s.c[3]}};
}

__host__ __device__ __forceinline__ uint64_t feistel_round(uint64_t x, int i, uint64_t seed,
                                                           uint64_t stream, uint64_t mask) {
  return philox(x, (uint64_t)i, 0, 0, seed, stream).w[0] & mask;
}

// Balanced Feistel network on 2h bits (h = ceil(p/2)); the permutation of
// [0, 2^p) is obtained by cycle walking (Black and Rogaway, CT-RSA 2002).
__host__ __device__ __forceinline__ uint64_t feistel_enc(uint64_t x, uint64_t seed,
                                                         uint64_t stream, int h) {
  const uint64_t mask = (uint64_t(1) << h) - 1;
  uint64_t L = x >> h, R = x & mask;
#pragma unroll
  for (int i = 0; i < kFeistelRounds; ++i) {
    uint64_t f = feistel_round(R, i, seed, stream, mask);
    uint64_t nl = R;
    R = L ^ f;
    L = nl;
  }
  return (L << h) | R;
}

__host__ __device__ __forceinline__ uint64_t feistel_dec(uint64_t y, uint64_t seed,
                                                         uint64_t stream, int h) {
  const uint64_t mask = (uint64_t(1) << h) - 1;
  uint64_t L = y >> h, R = y & mask;
#pragma unroll
  for (int i = kFeistelRounds - 1; i >= 0; --i) {
    uint64_t f = feistel_round(L, i, seed, stream, mask);
    uint64_t nr = L;
    L = R ^ f;
    R = nr;
  }
  return (L << h) | R;
}

// pi(x) for the keyed permutation of [0, 2^p), x < 2^p.
__host__ __device__ __forceinline__ uint64_t prp(uint64_t x, uint64_t seed, uint64_t stream,
                                                 int p) {
  const int h = (p + 1) >> 1;
  const uint64_t lim = uint64_t(1) << p;
  uint64_t y = feistel_enc(x, seed, stream, h);
  while (y >= lim) y = feistel_enc(y, seed, stream, h);
  return y;
}

__host__ __device__ __forceinline__ uint64_t prp_inv(uint64_t y, uint64_t seed, uint64_t stream,
                                                     int p) {
  const int h = (p + 1) >> 1;
  const uint64_t lim = uint64_t(1) << p;
  uint64_t x = feistel_dec(y, seed, stream, h);
  while (x >= lim) x = feistel_dec(x, seed, stream, h);
  return x;
}

// D_j in {+1,-1}: bit (j & 63) of word ((j >> 6) & 3) of block j >> 8 (0 -> +1).
__host__ __device__ __forceinline__ int rademacher(uint64_t seed, uint64_t j) {
  Words w = philox(j >> 8, 0, 0, 0, seed, kStreamD);
  uint64_t word = w.w[(j >> 6) & 3];
  return ((word >> (j & 63)) & 1) ? -1 : 1;
}

// CountSketch of S_K: bucket = word0 mod m (m a power of 2), sign from word1.
__host__ __device__ __forceinline__ void cs_hash(uint64_t seed, uint64_t j, uint64_t m_mask,
                                                 uint64_t& bucket, int& sign) {
  Words w = philox(j, 0, 0, 0, seed, kStreamCS);
  bucket = w.w[0] & m_mask;
  sign = (w.w[1] & 1) ? -1 : 1;
}

// CountSketch of S_hat: bucket = ((word0 >> 32) * r) >> 32 in [0, r), sign from word1.
__host__ __device__ __forceinline__ void cs_hash_hat(uint64_t seed, uint64_t j, uint64_t r,
                                                     uint64_t& bucket, int& sign) {
  Words w = philox(j, 0, 0, 0, seed, kStreamCShat);
  bucket = ((w.w[0] >> 32) * r) >> 32;
  sign = (w.w[1] & 1) ? -1 : 1;
}

}  // namespace rng
}  // namespace slse
