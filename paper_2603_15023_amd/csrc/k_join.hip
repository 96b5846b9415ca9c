// PU-key join index (Sec. 3.2: the rewriter adds the joins that lead each
// sensitive table to the PU table along its foreign keys; Sec. 2 relational
// privacy unit).  The aggregation kernels follow foreign keys given as row
// indices; a table whose foreign keys are key values is first mapped to row
// indices here: an open-addressing table key -> row (linear probing over a
// power-of-two capacity of at least twice the keys) is built with one CAS per
// key, then every referencing key is probed.
#include <algorithm>

#include "pac_join.h"

namespace pac {

constexpr uint64_t kJoinSalt = 0x2545F4914F6CDD1Dull;

__global__ __launch_bounds__(256) void join_build_kernel(const int64_t *keys, int64_t n_keys, int64_t *tk, int32_t *ti,
                                                         uint64_t mask, uint32_t *status) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_keys; i += stride) {
    const int64_t k = keys[i];
    if (k == PAC_EMPTY_KEY) continue;  // not a valid key: that row is not indexed
    uint64_t h = mix64((uint64_t)k ^ kJoinSalt) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
      const unsigned long long prev =
          atomicCAS((unsigned long long *)&tk[h], (unsigned long long)PAC_EMPTY_KEY, (unsigned long long)k);
      if (prev == (unsigned long long)PAC_EMPTY_KEY) {
        ti[h] = (int32_t)i;
        break;
      }
      if ((int64_t)prev == k) {
        atomicOr(status, PAC_STATUS_DUPLICATE_KEY);
        break;
      }
      h = (h + 1) & mask;
    }
  }
}

__global__ __launch_bounds__(256) void join_probe_kernel(const int64_t *fk, int64_t n, const int64_t *tk,
                                                         const int32_t *ti, uint64_t mask, int32_t *out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int64_t k = fk[r];
    int32_t found = -1;
    if (k != PAC_EMPTY_KEY) {
      uint64_t h = mix64((uint64_t)k ^ kJoinSalt) & mask;
      for (uint64_t probe = 0; probe <= mask; ++probe) {
        const int64_t t = tk[h];
        if (t == k) {
          found = ti[h];
          break;
        }
        if (t == PAC_EMPTY_KEY) break;
        h = (h + 1) & mask;
      }
    }
    out[r] = found;
  }
}

int64_t join_capacity(int64_t n_keys) {
  int64_t cap = 16;
  while (cap < 2 * n_keys) cap <<= 1;
  return cap;
}

size_t join_scratch_bytes(int64_t n_keys) {
  const int64_t cap = join_capacity(n_keys);
  return (size_t)cap * 8 + (size_t)cap * 4 + 256;
}

hipError_t launch_key_index(const LaunchEnv &env, const int64_t *keys, int64_t n_keys, const int64_t *fk, int64_t n,
                            int32_t *out, void *scratch) {
  const int64_t cap = join_capacity(n_keys);
  int64_t *tk = (int64_t *)scratch;
  int32_t *ti = (int32_t *)(tk + cap);
  hipError_t e = launch_fill_i64(env, tk, cap, PAC_EMPTY_KEY);
  if (e != hipSuccess) return e;
  const uint64_t mask = (uint64_t)cap - 1;
  if (n_keys > 0) {
    const int blocks = (int)std::min<int64_t>((n_keys + 255) / 256, (int64_t)env.n_cu * 16);
    hipLaunchKernelGGL(join_build_kernel, dim3(blocks), dim3(256), 0, env.stream, keys, n_keys, tk, ti, mask,
                       env.status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (n > 0) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, (int64_t)env.n_cu * 16);
    hipLaunchKernelGGL(join_probe_kernel, dim3(blocks), dim3(256), 0, env.stream, fk, n, tk, ti, mask, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace pac
