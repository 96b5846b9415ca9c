// Measurement kernels: a plain streaming read and a plain copy of HBM-resident
// bytes, with the load form of the scan kernels (16-byte non-temporal vector
// loads, each wavefront reading one contiguous 1 KB stretch per step, several
// steps in flight).  The read rate they reach on the device is the achievable
// ceiling the aggregation kernels are held against beside the datasheet peak;
// their known byte counts calibrate the hardware traffic counters.
#include <algorithm>

#include "pac_internal.h"

namespace pac {

typedef unsigned int s4u32 __attribute__((ext_vector_type(4)));

constexpr int kStreamUnroll = 4;

__global__ __launch_bounds__(256) void stream_read_kernel(const s4u32 *__restrict__ p, int64_t n16, uint64_t *out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  s4u32 acc = {0u, 0u, 0u, 0u};
  for (; i + (kStreamUnroll - 1) * stride < n16; i += kStreamUnroll * stride) {
    s4u32 x[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) x[u] = __builtin_nontemporal_load(&p[i + u * stride]);
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) acc ^= x[u];
  }
  for (; i < n16; i += stride) acc ^= __builtin_nontemporal_load(&p[i]);
  uint64_t v = ((uint64_t)(acc[0] ^ acc[2]) << 32) | (acc[1] ^ acc[3]);
  for (int o = 32; o > 0; o >>= 1) v ^= (uint64_t)__shfl_xor((long long)v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicXor((unsigned long long *)out, (unsigned long long)v);
}

__global__ __launch_bounds__(256) void stream_copy_kernel(const s4u32 *__restrict__ p, s4u32 *__restrict__ q,
                                                          int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(&p[i]), &q[i]);
}

hipError_t launch_stream_read(const LaunchEnv &env, const void *buf, int64_t bytes, uint64_t *out) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n16 + 255) / 256, (int64_t)env.n_cu * 8));
  hipLaunchKernelGGL(stream_read_kernel, dim3(blocks), dim3(256), 0, env.stream, (const s4u32 *)buf, n16, out);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const LaunchEnv &env, const void *src, void *dst, int64_t bytes) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n16 + 255) / 256, (int64_t)env.n_cu * 8));
  hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(256), 0, env.stream, (const s4u32 *)src, (s4u32 *)dst,
                     n16);
  return hipGetLastError();
}

}  // namespace pac
