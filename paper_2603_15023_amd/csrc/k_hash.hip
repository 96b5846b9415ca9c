// a1: keyed PU hash (Sec. 2 "SIMD-PAC-DB", Sec. 4.2 "PAC Hash") and small fill kernels.
//
// One thread per key; word w of key k is the (w+1)-th splitmix64 output from
// state k ^ K.  Reads 8 B and writes 8*W B per key: HBM-bound, coalesced.
#include "pac_internal.h"

namespace pac {

template <int W>
__global__ __launch_bounds__(256) void hash_kernel(const int64_t *__restrict__ keys, int64_t n, uint64_t qk,
                                                   uint32_t balanced, uint64_t *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t k = __builtin_nontemporal_load(&keys[i]);
#pragma unroll
    for (int w = 0; w < W; ++w) out[i * W + w] = pu_word(k, qk, w, balanced != 0);
  }
}

hipError_t launch_hash(const LaunchEnv &env, const int64_t *keys, int64_t n, uint64_t qk, int m, bool balanced,
                       uint64_t *out) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks_needed = (n + 255) / 256;
  const int blocks = (int)(blocks_needed < (int64_t)env.n_cu * 16 ? blocks_needed : (int64_t)env.n_cu * 16);
  if (m == 64)
    hipLaunchKernelGGL(hash_kernel<1>, dim3(blocks), dim3(256), 0, env.stream, keys, n, qk, balanced ? 1u : 0u, out);
  else
    hipLaunchKernelGGL(hash_kernel<2>, dim3(blocks), dim3(256), 0, env.stream, keys, n, qk, balanced ? 1u : 0u, out);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T *p, int64_t n, T v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T>
static hipError_t launch_fill(const LaunchEnv &env, T *p, int64_t n, T v) {
  if (n <= 0 || !p) return hipSuccess;
  const int64_t need = (n + 255) / 256;
  const int blocks = (int)(need < (int64_t)env.n_cu * 8 ? need : (int64_t)env.n_cu * 8);
  hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks), dim3(256), 0, env.stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i64(const LaunchEnv &env, int64_t *p, int64_t n, int64_t v) { return launch_fill(env, p, n, v); }

// Several fills in one launch: grid row y sets segment y's n[y] 64-bit words
// at p[y] to the bit pattern v[y].
__global__ __launch_bounds__(256) void fill_multi_kernel(FillSegs f) {
  const int s = blockIdx.y;
  int64_t *p = f.p[s];
  const int64_t n = f.n[s], v = f.v[s];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_multi(const LaunchEnv &env, const FillSegs &in) {
  FillSegs f{};
  int64_t max_n = 0;
  for (int i = 0; i < in.count && i < kMaxFillSegs; ++i) {  // empty segments dropped
    if (in.n[i] <= 0 || !in.p[i]) continue;
    f.p[f.count] = in.p[i];
    f.n[f.count] = in.n[i];
    f.v[f.count] = in.v[i];
    max_n = in.n[i] > max_n ? in.n[i] : max_n;
    ++f.count;
  }
  if (f.count == 0) return hipSuccess;
  const int64_t need = (max_n + 255) / 256, cap = (int64_t)env.n_cu * 8 / f.count;
  const int blocks = (int)(need < cap ? need : (cap > 0 ? cap : 1));
  hipLaunchKernelGGL(fill_multi_kernel, dim3(blocks, f.count), dim3(256), 0, env.stream, f);
  return hipGetLastError();
}

// Occupied slots of a sparse-key table: per-wave ballot counts, summed per
// workgroup in LDS, one atomic add per workgroup (n_used cleared first).
__global__ __launch_bounds__(256) void count_used_kernel(const int64_t *slot_keys, int64_t cap, int64_t *n_used) {
  __shared__ uint32_t part[4];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride)
    c += slot_keys[i] != PAC_EMPTY_KEY ? 1u : 0u;
  for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t sum = (uint64_t)part[0] + part[1] + part[2] + part[3];
    if (sum) atomicAdd((unsigned long long *)n_used, (unsigned long long)sum);
  }
}

hipError_t launch_count_used(const LaunchEnv &env, const int64_t *slot_keys, int64_t cap, int64_t *n_used) {
  hipError_t e = launch_fill(env, n_used, (int64_t)1, (int64_t)0);
  if (e != hipSuccess || cap <= 0) return e;
  const int64_t need = (cap + 255) / 256;
  const int blocks = (int)(need < (int64_t)env.n_cu * 4 ? need : (int64_t)env.n_cu * 4);
  hipLaunchKernelGGL(count_used_kernel, dim3(blocks), dim3(256), 0, env.stream, slot_keys, cap, n_used);
  return hipGetLastError();
}
hipError_t launch_fill_f64(const LaunchEnv &env, double *p, int64_t n, double v) { return launch_fill(env, p, n, v); }

}  // namespace pac
