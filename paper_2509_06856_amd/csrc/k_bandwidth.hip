// Reference streams for measurement: a plain streaming read and a plain copy
// of a device buffer.  They hold none of the method's arithmetic; the
// benchmark times them on the same data as the path's kernels, so that those
// can be stated as a fraction of what a bare read (or read + write) reaches on
// the part.  Each block streams one contiguous chunk with 16-byte
// non-temporal accesses, four in flight per lane.
#include "kernels.hpp"

namespace slse {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRdThreads = 256;
constexpr int kRdDepth = 8;
constexpr int kCpThreads = 1024;
constexpr int kCpDepth = 4;

__global__ __launch_bounds__(kRdThreads) void stream_read_kernel(const u32x4* __restrict__ src,
                                                                 int64_t n16, int64_t per_block,
                                                                 unsigned* __restrict__ sink) {
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = min(n16, b0 + per_block);
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (int64_t i = b0 + threadIdx.x; i < b1; i += (int64_t)kRdThreads * kRdDepth) {
    u32x4 v[kRdDepth];
#pragma unroll
    for (int u = 0; u < kRdDepth; ++u) {
      const int64_t k = i + (int64_t)u * kRdThreads;
      v[u] = k < b1 ? __builtin_nontemporal_load(src + k) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < kRdDepth; ++u) acc ^= v[u];
  }
  // one word per block keeps the loads live
  __shared__ unsigned s[kRdThreads];
  s[threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
  __syncthreads();
  for (int h = kRdThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] ^= s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sink[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kCpThreads) void stream_copy_kernel(const u32x4* __restrict__ src,
                                                                 u32x4* __restrict__ dst,
                                                                 int64_t n16, int64_t per_block) {
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = min(n16, b0 + per_block);
  for (int64_t i = b0 + threadIdx.x; i < b1; i += (int64_t)kCpThreads * kCpDepth) {
    u32x4 v[kCpDepth];
#pragma unroll
    for (int u = 0; u < kCpDepth; ++u) {
      const int64_t k = i + (int64_t)u * kCpThreads;
      if (k < b1) v[u] = __builtin_nontemporal_load(src + k);
    }
#pragma unroll
    for (int u = 0; u < kCpDepth; ++u) {
      const int64_t k = i + (int64_t)u * kCpThreads;
      if (k < b1) __builtin_nontemporal_store(v[u], dst + k);
    }
  }
}

}  // namespace

void launch_stream_reference(int mode, const void* src, void* dst, int64_t bytes, int blocks,
                             hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return;
  const int64_t per = ceil_div(n16, (int64_t)blocks);
  if (mode == 0)
    stream_read_kernel<<<blocks, kRdThreads, 0, s>>>(static_cast<const u32x4*>(src), n16, per,
                                                     static_cast<unsigned*>(dst));
  else
    stream_copy_kernel<<<blocks, kCpThreads, 0, s>>>(static_cast<const u32x4*>(src),
                                                     static_cast<u32x4*>(dst), n16, per);
  SLSE_LAUNCH_CHECK();
}

}  // namespace slse
