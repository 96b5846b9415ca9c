// Approximate integer SUM (Sec. 5, Approximation): per-world 16-bit counters
// in levels that cascade every 4 bits, one state for the positive values and
// one for the negated negative values (the two-sided SUM).
//
// A value v != 0 with a = |v| goes to level l = floor((msb(a) - 8) / 4) (0
// below 256) as x = a >> 4l (< 2^12).  Adding x to a counter that would pass
// 65535 first moves the counter's upper 12 bits one level up (carry = C >> 4,
// which may cascade further) and restarts it at 0; the lower 4 bits are lost,
// at most 15 / 61441 < 2^-12 of what moved.  A state is worth
// sum_k C[k] 2^(4k); the result is pos - neg.
//
// Decomposition: rows are taken in blocks of PAC_APPROX_BLOCK_ROWS consecutive
// indices.  For each block, group and world, a fresh state takes the block's
// rows of that group with the world bit set, in row order; its value is then
// added exactly (mod 2^64, like the exact sums) to isum.  COUNT and nrows are
// exact.
//
// One workgroup per block: the rows' groups, PU words and routed values are
// staged in LDS and the (group, row) keys sorted (bitonic), so that each
// group's rows form one run in row order.  A task is one (run, column): one
// wave with lane = world, its 2 x 16 level counters in registers (indexed by
// the row's level, which is the same in every lane), the run's rows read 64 at
// a time (one per lane) and broadcast with readlane.  A run has at most 1024
// rows, so one side holds at most 2^73: a level k overflows only with
// 61441 * 2^(4k) <= 2^73, i.e. k <= 14, and no carry goes past level 15.
// Sixteen levels are kept (the paper's 25 cover 2^112 for unbounded row
// counts).
#include <algorithm>

#include "pac_internal.h"

namespace pac {

constexpr int kApproxRows = PAC_APPROX_BLOCK_ROWS;  // rows per block (a power of two)
constexpr int kApproxRowBits = 10;
static_assert((1 << kApproxRowBits) == kApproxRows, "block rows");
constexpr int kApproxLevels = 16;
constexpr int kApproxWaves = 4;
constexpr uint64_t kNoKey = ~0ull;

// Level and shifted value of a (> 0).
__device__ __forceinline__ uint32_t approx_route(uint64_t a, bool neg) {
  const int msb = 63 - __clzll(a);
  const int l = msb < 8 ? 0 : (msb - 8) >> 2;
  const uint32_t x = (uint32_t)(a >> (4 * l));
  return x | ((uint32_t)l << 12) | ((uint32_t)neg << 17);
}

// Adds `add` (0 in lanes whose world bit is clear) at counter index `idx`
// (side * 16 + level, the same in every lane) with the cascade of overflows;
// returns the highest counter index written.
__device__ __forceinline__ int approx_add(uint32_t (&S)[2 * kApproxLevels], int idx, uint32_t add) {
  uint32_t C = S[idx];
  uint32_t sum = C + add;
  bool ovf = sum > 0xFFFFu;
  S[idx] = ovf ? add : sum;  // an overflowing counter restarts at 0, then takes the update
  if (__ballot(ovf) == 0ull) return idx;  // the usual case: no lane overflows
  uint32_t carry = ovf ? C >> 4 : 0u;  // its upper 12 bits move up a level (never 0: C > 61440)
  const int last = (idx / kApproxLevels) * kApproxLevels + kApproxLevels - 1;
  do {
    ++idx;
    C = S[idx];
    sum = C + carry;
    ovf = sum > 0xFFFFu;
    S[idx] = carry == 0u ? C : (ovf ? carry : sum);
    carry = ovf ? C >> 4 : 0u;
  } while (__ballot(carry != 0u) != 0ull && idx < last);
  return idx;
}

template <int W>
__global__ __launch_bounds__(64 * kApproxWaves) void agg_approx(DevInput in, DevState st, uint32_t *status) {
  extern __shared__ uint64_t lds[];
  constexpr int R = kApproxRows, L = kApproxLevels;
  constexpr int m = 64 * W;
  const int nc = in.n_icols, tasks_per_run = nc > 0 ? nc : 1;
  uint64_t *keys = lds;                                        // [R] (group << 10) | row, sorted
  uint64_t *words = keys + R;                                  // [R][W] by row
  uint32_t *vals = (uint32_t *)(words + (size_t)R * W);        // [nc][R] routed values by row
  int32_t *runs = (int32_t *)(vals + (size_t)nc * R);          // [R] run starts (positions in keys)
  int32_t *n_runs = runs + R;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int T = 64 * kApproxWaves;

  const int64_t n = in.n_rows;
  const int64_t n_blocks = (n + R - 1) / R;
  for (int64_t b = blockIdx.x; b < n_blocks; b += gridDim.x) {
    const int64_t base = b * R;
    if (tid == 0) *n_runs = 0;
    // ---- stage: group, PU words and routed values of every row of the block
    for (int t = tid; t < R; t += T) {
      const int64_t r = base + t;
      int64_t g = -1, idx = 0;
      if (r < n) {
        g = row_group(in, st, r, status);
        if (g >= 0 && !chain_index(in, r, &idx, status)) g = -1;
      }
      keys[t] = g >= 0 ? ((uint64_t)g << kApproxRowBits) | (uint64_t)t : kNoKey;
      if (g >= 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) words[t * W + w] = pu_of_index(in, idx, w);
        for (int c = 0; c < nc; ++c) {
          const int64_t v = load_icol(in.icols[c], in.icol_type[c], r);
          vals[c * R + t] = v == 0 ? 0u : approx_route(v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v, v < 0);
        }
      }
    }
    __syncthreads();
    // ---- bitonic sort of the keys: each group's rows become one run, in row order
    for (int k = 2; k <= R; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < R; i += T) {
          const int p = i ^ j;
          if (p > i) {
            const uint64_t a = keys[i], c = keys[p];
            if ((a > c) == ((i & k) == 0)) {
              keys[i] = c;
              keys[p] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = tid; i < R; i += T) {
      const uint64_t k = keys[i];
      if (k != kNoKey && (i == 0 || (keys[i - 1] >> kApproxRowBits) != (k >> kApproxRowBits)))
        runs[atomicAdd(n_runs, 1)] = i;
    }
    __syncthreads();
    // ---- tasks (run, column), one per wave at a time; lane = world
    const int n_tasks = *n_runs * tasks_per_run;
    for (int task = wave; task < n_tasks; task += kApproxWaves) {
      const int q = task / tasks_per_run, c = task - q * tasks_per_run;
      // run bounds and group in scalar registers (the same in every lane)
      const int s = __builtin_amdgcn_readfirstlane(runs[q]);
      const uint64_t gk = readlane_u64(keys[s], 0) >> kApproxRowBits;
      const int64_t g = (int64_t)gk;
      int e = s + 1;
      while (e < R) {
        const uint64_t k = readlane_u64(keys[e], 0);
        if (k == kNoKey || (k >> kApproxRowBits) != gk) break;
        ++e;
      }
      const bool counts = c == 0;  // the first task of a run also takes COUNT and nrows
      // one counter array per PU word, each small enough to stay in registers
      uint32_t S0[2 * L], S1[2 * L];
#pragma unroll
      for (int k = 0; k < 2 * L; ++k) S0[k] = S1[k] = 0;
      int top = -1;  // highest level written on either side (uniform)
      int cnt[W];
#pragma unroll
      for (int w = 0; w < W; ++w) cnt[w] = 0;
      for (int i0 = s; i0 < e; i0 += 64) {
        // one row per lane, then broadcast row by row in order
        const int i = i0 + lane;
        uint64_t wd[W];
        uint32_t pv = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) wd[w] = 0;
        if (i < e) {
          const int t = (int)(keys[i] & (R - 1));
#pragma unroll
          for (int w = 0; w < W; ++w) wd[w] = words[t * W + w];
          pv = nc > 0 ? vals[c * R + t] : 0u;
        }
        const int nn = min(64, e - i0);
        for (int k = 0; k < nn; ++k) {
          const uint32_t p = __builtin_amdgcn_readlane(pv, k);
          uint32_t bit[W];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            bit[w] = (uint32_t)(readlane_u64(wd[w], k) >> lane) & 1u;
            cnt[w] += (int)bit[w];
          }
          const uint32_t x = p & 0xFFFu;
          if (x == 0u) continue;
          const int idx = (int)(p >> 17) * L + (int)((p >> 12) & 31u);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const int hi = approx_add(w == 0 ? S0 : S1, idx, bit[w] ? x : 0u);
            top = max(top, hi % L);
          }
        }
      }
      if (nc > 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint32_t(&S)[2 * L] = w == 0 ? S0 : S1;
          uint64_t sum = 0;
#pragma unroll
          for (int l = 0; l < L; ++l)
            if (l <= top) sum += (uint64_t)((int64_t)S[l] - (int64_t)S[L + l]) << (4 * l);
          if (sum) atomicAdd((unsigned long long *)&st.isum[(g * nc + c) * m + w * 64 + lane], (unsigned long long)sum);
        }
      }
      if (counts) {
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (cnt[w]) atomicAdd((unsigned long long *)&st.count[g * m + w * 64 + lane], (unsigned long long)cnt[w]);
        if (lane == 0) atomicAdd((unsigned long long *)&st.nrows[g], (unsigned long long)(e - s));
      }
    }
    __syncthreads();  // keys, words and vals are rewritten by the next block
  }
}

bool approx_supported(const DevInput &in, const DevState &st) {
  return in.n_fcols == 0 && !st.minmax && approx_lds_bytes(in) <= 160 * 1024;
}

size_t approx_lds_bytes(const DevInput &in) {
  const size_t R = kApproxRows;
  return R * 8 + R * 8 * in.W + R * 4 * in.n_icols + R * 4 + 8;
}

hipError_t launch_agg_approx(const LaunchEnv &env, const DevInput &in, const DevState &st) {
  if (in.n_rows <= 0) return hipSuccess;
  const size_t lds = approx_lds_bytes(in);
  const void *fn = in.W == 1 ? (const void *)agg_approx<1> : (const void *)agg_approx<2>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / lds));
  const int64_t n_blocks = (in.n_rows + kApproxRows - 1) / kApproxRows;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_blocks, (int64_t)env.n_cu * per_cu));
  if (in.W == 1)
    hipLaunchKernelGGL(agg_approx<1>, dim3(grid), dim3(64 * kApproxWaves), lds, env.stream, in, st, env.status);
  else
    hipLaunchKernelGGL(agg_approx<2>, dim3(grid), dim3(64 * kApproxWaves), lds, env.stream, in, st, env.status);
  return hipGetLastError();
}

}  // namespace pac
