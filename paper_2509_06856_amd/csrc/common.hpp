// Shared host/device helpers of libslse: status plumbing, HIP checks, small
// device utilities.  Internal header.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/slse.h"

namespace slse {

// ---------------------------------------------------------------------------
// Errors.  Internal code throws slse::Error; the C-ABI entry points catch it
// and turn it into a status plus a thread-local message.
// ---------------------------------------------------------------------------
struct Error {
  slse_status status;
  std::string msg;
};

void set_last_error(const std::string& msg);

[[noreturn]] inline void fail(slse_status st, const std::string& msg) { throw Error{st, msg}; }

inline void require(bool ok, const std::string& msg) {
  if (!ok) fail(SLSE_EINVAL, msg);
}

#define SLSE_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::slse::fail(e_ == hipErrorOutOfMemory ? SLSE_ENOMEM : SLSE_EDEVICE,             \
                   std::string(#call) + " failed: " + hipGetErrorString(e_));          \
    }                                                                                  \
  } while (0)

#define SLSE_LAUNCH_CHECK() SLSE_HIP(hipGetLastError())

inline size_t dtype_size(slse_dtype t) {
  switch (t) {
    case SLSE_F32: return 4;
    case SLSE_F64: return 8;
    case SLSE_BF16: return 2;
  }
  return 0;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// smallest p with 2^p >= v (the exact log for a power of 2)
inline int ilog2_ceil(int64_t v) {
  int p = 0;
  while ((int64_t(1) << p) < v) ++p;
  return p;
}

inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// ---------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------
// Global-memory (address space 1) pointers.  A pointer that a kernel reads
// from a descriptor in memory (not a kernel argument) is generic to the
// compiler, and its accesses become flat instructions, which also count
// against the LDS counter: every wait for an LDS result then waits for the
// memory accesses in flight too.  Casting such pointers at their accesses
// keeps them global.
#define SLSE_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const SLSE_GLOBAL T* gptr(const T* p) {
  return (const SLSE_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ SLSE_GLOBAL T* gptr(T* p) {
  return (SLSE_GLOBAL T*)p;
}

template <typename T>
__device__ __forceinline__ T wave_xor(T v, int mask) {
  return __shfl_xor(v, mask, 64);
}

template <typename T>
__device__ __forceinline__ T lane_group_sum(T v, int group) {
  // all-reduce inside aligned groups of `group` lanes (power of 2 <= 64)
  for (int m = group >> 1; m > 0; m >>= 1) v += wave_xor(v, m);
  return v;
}

// Block partials handed to the last block of a grid (or of a block group).
// Each XCD has its own L2, so a plain store may sit in the writer's L2 where
// a block on another XCD does not see it.  The partials are stored and loaded
// with agent-scope (sc1) accesses, which go past the non-coherent L2 level.
__device__ __forceinline__ void store_device(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_device(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait for this thread's outstanding memory operations (stores included)
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The ticket of a hand-off.  After its partial stores, a wait for their
// completion (wait_memory) and a block barrier, one thread per block draws a
// ticket with release semantics at agent scope, so in the memory model the
// block's stores happen before its ticket; the block that draws the last
// ticket issues an agent-scope acquire fence (acquire_partials) before its
// threads read the partials.  The release costs each block one write-back of
// its L2's dirty lines (about 16 us per residual-gradient pass of 256 blocks).
__device__ __forceinline__ int take_ticket(int* counter) {
  return __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void acquire_partials() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

}  // namespace slse
