// a2-a6, ballot form: world bits transposed across the wavefront, counts by popcount.
//
// Per 64-row chunk, lane r holds row r's PU word; a 64x64 bit transpose
// (six exchange stages) leaves in lane j the 64-bit set T_j of chunk rows that
// are in world j.  With the row set of group g as a ballot G_g and the bit
// planes of the offset values x = v - lo as ballots V_b:
//   COUNT[g][j] += popcount(T_j & G_g)
//   SUM[g][c][j] += sum_b 2^b popcount(T_j & G_g & V_{c,b}) + lo_c * popcount(T_j & G_g)
// This is exact for integers and costs G * (1 + sum of value bits) popcounts
// per chunk: far cheaper than per-row adds when values have few significant
// bits (the 1..50 values of the ungrouped count/sum workload use 6 bits), and
// more expensive than the matrix-core form for wide values.
#include <algorithm>

#include "pac_internal.h"

namespace pac {

__device__ __forceinline__ uint64_t xor_shfl64(uint64_t x, int mask) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, mask, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), mask, 64);
  return ((uint64_t)hi << 32) | lo;
}

// After the call, bit r of lane j's word = bit j of lane r's word.
__device__ __forceinline__ uint64_t transpose64(uint64_t x, int lane) {
  const uint64_t lo_masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int b = 32 >> s;
    const uint64_t partner = xor_shfl64(x, b);
    const uint64_t lm = lo_masks[s];
    if ((lane & b) == 0)
      x = (x & lm) | ((partner & lm) << b);
    else
      x = (x & ~lm) | ((partner & ~lm) >> b);
  }
  return x;
}

template <int W>
__global__ __launch_bounds__(256) void agg_ballot(DevInput in, DevState st, uint32_t *status, int waves_per_block) {
  extern __shared__ uint64_t lds[];
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ni = in.n_icols, A = 1 + ni;
  const int64_t G = in.n_groups;
  const int64_t gstride = (int64_t)A * m + 1;
  const int64_t region = G * gstride;
  for (int64_t i = threadIdx.x; i < region * waves_per_block; i += blockDim.x) lds[i] = 0;
  __syncthreads();
  uint64_t *my = lds + (int64_t)wave * region;
  const int64_t n = in.n_rows;
  const int64_t n_chunks = (n + 63) >> 6;
  const int64_t total_waves = (int64_t)gridDim.x * waves_per_block;
  for (int64_t chunk = (int64_t)blockIdx.x * waves_per_block + wave; chunk < n_chunks; chunk += total_waves) {
    const int64_t r = chunk * 64 + lane;
    int64_t g = -1;
    uint64_t mk[W];
    uint64_t x[kMaxCols];
#pragma unroll
    for (int w = 0; w < W; ++w) mk[w] = 0;
    if (r < n) {
      g = row_group(in, st, r, status);
      int64_t idx = 0;
      if (g >= 0 && !chain_index(in, r, &idx, status)) g = -1;
      if (g >= 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) mk[w] = pu_of_index(in, idx, w);
      }
    }
    // values outside the stated statistics would lose bits above icol_bits:
    // such a row updates nothing and reports PAC_STATUS_OUT_OF_RANGE
    bool out_of_range = false;
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c)
      if (c < ni) {
        x[c] = g >= 0 ? (uint64_t)load_icol(in.icols[c], in.icol_type[c], r) - (uint64_t)in.icol_lo[c] : 0;
        out_of_range |= x[c] > in.icol_range[c];
      }
    if (out_of_range) {
      atomicOr(status, PAC_STATUS_OUT_OF_RANGE);
      g = -1;
#pragma unroll
      for (int w = 0; w < W; ++w) mk[w] = 0;
#pragma unroll
      for (int c = 0; c < kMaxCols; ++c) x[c] = 0;
    }
    uint64_t T[W];
#pragma unroll
    for (int w = 0; w < W; ++w) T[w] = transpose64(mk[w], lane);
    uint64_t live = __ballot(g >= 0);
    while (live) {
      // next group present in this chunk (uniform)
      const int rr = __ffsll((unsigned long long)live) - 1;
      const int64_t gg = (int64_t)(((uint64_t)__builtin_amdgcn_readlane((uint32_t)((uint64_t)g >> 32), rr) << 32) |
                                   (uint32_t)__builtin_amdgcn_readlane((uint32_t)g, rr));
      const uint64_t Gb = __ballot(g == gg);
      live &= ~Gb;
      uint64_t *base = my + gg * gstride;
      if (lane == 0) base[(int64_t)A * m] += (uint64_t)__popcll(Gb);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint64_t Tg = T[w] & Gb;
        const uint64_t cnt = (uint64_t)__popcll(Tg);
        const int j = w * 64 + lane;
        base[j] += cnt;
#pragma unroll
        for (int c = 0; c < kMaxCols; ++c) {
          if (c >= ni) continue;
          uint64_t s = (uint64_t)in.icol_lo[c] * cnt;
          for (int b = 0; b < in.icol_bits[c]; ++b) {
            const uint64_t Vb = __ballot((x[c] >> b) & 1ull);
            s += (uint64_t)__popcll(Tg & Vb) << b;
          }
          base[(int64_t)(1 + c) * m + j] += s;
        }
      }
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < region; i += blockDim.x) {
    uint64_t s = 0;
    for (int w = 0; w < waves_per_block; ++w) s += lds[(int64_t)w * region + i];
    if (!s) continue;
    const int64_t gg = i / gstride, off = i % gstride;
    if (off == (int64_t)A * m) {
      atomicAdd((unsigned long long *)&st.nrows[gg], (unsigned long long)s);
      continue;
    }
    const int a = (int)(off / m), j = (int)(off % m);
    unsigned long long *dst = a == 0 ? (unsigned long long *)&st.count[gg * m + j]
                                     : (unsigned long long *)&st.isum[(gg * ni + (a - 1)) * m + j];
    atomicAdd(dst, (unsigned long long)s);
  }
}

bool ballot_supported(const DevInput &in) {
  if (in.group_keys || in.n_fcols > 0) return false;
  const int64_t region = in.n_groups * ((int64_t)(1 + in.n_icols) * in.m + 1) * 8;
  return region <= 160 * 1024;
}

hipError_t launch_agg_ballot(const LaunchEnv &env, const DevInput &in, const DevState &st) {
  if (in.n_rows <= 0) return hipSuccess;
  const int64_t region = in.n_groups * ((int64_t)(1 + in.n_icols) * in.m + 1) * 8;
  const int wpb = (int)std::max<int64_t>(1, std::min<int64_t>(4, (160 * 1024) / region));
  const int64_t lds = region * wpb;
  const void *fn = in.W == 1 ? (const void *)agg_ballot<1> : (const void *)agg_ballot<2>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int per_cu = (int)std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / lds));
  const int64_t n_chunks = (in.n_rows + 63) / 64;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n_chunks + wpb - 1) / wpb, (int64_t)env.n_cu * per_cu));
  if (in.W == 1)
    hipLaunchKernelGGL(agg_ballot<1>, dim3(blocks), dim3(64 * wpb), (size_t)lds, env.stream, in, st, env.status, wpb);
  else
    hipLaunchKernelGGL(agg_ballot<2>, dim3(blocks), dim3(64 * wpb), (size_t)lds, env.stream, in, st, env.status, wpb);
  return hipGetLastError();
}

}  // namespace pac
