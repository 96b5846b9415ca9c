// a2-a6, plain form: lane = world, rows broadcast across the wavefront.
//
// This is the paper's predicated update loop (Sec. 1 count loop, Sec. 5
// "Naive SIMD-unfriendly" / predication) mapped onto a 64-wide wavefront:
// the SIMD lanes are the worlds, each row's PU word is broadcast and lane j
// adds the row's value into world j's counter when bit j is set.  Counters
// live in a wave-private LDS region [G][A][m] (A = 1 + ints + floats, plus
// nrows), so a lane only ever touches its own world column; the adds are LDS
// atomics without a return value (no read-modify-write latency), applied in
// issue order because one wave owns the region, so FP64 sums keep a fixed order.  Workgroups flush int counters with int64 global atomics
// and float counters as per-block partials reduced in a fixed order (same
// bits on every run).  Groups whose counters do not fit in LDS, and sparse
// group keys (HBM hash table), update the global counters with atomics.
//
// Cost: about (2 + 2*ints + 2*floats) readlanes plus one LDS read-add-write
// per counter per row: VALU/LDS bound, several times the HBM time.  It is the
// baseline the ballot and matrix-core forms are measured against.
#include <algorithm>

#include "pac_internal.h"

namespace pac {

template <int W>
__global__ __launch_bounds__(256) void agg_plain_lds(DevInput in, DevState st, uint32_t *status, double *fpart,
                                                     int waves_per_block) {
  extern __shared__ uint64_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  constexpr int m = 64 * W;
  const int ni = in.n_icols, nf = in.n_fcols, A = 1 + ni + nf;
  const int64_t G = in.n_groups;
  const int64_t gstride = (int64_t)A * m + 1;  // per-group slots: A*m counters + nrows
  const int64_t region = G * gstride;
  for (int64_t i = threadIdx.x; i < region * waves_per_block; i += blockDim.x) lds[i] = 0;
  __syncthreads();
  uint64_t *my = lds + (int64_t)wave * region;
  const int64_t n_chunks = (in.n_rows + 63) >> 6;
  const int64_t total_waves = (int64_t)gridDim.x * waves_per_block;
  if (wave < waves_per_block) {
    for (int64_t chunk = (int64_t)blockIdx.x * waves_per_block + wave; chunk < n_chunks; chunk += total_waves) {
      uint64_t mk[W], iv[kMaxCols], fv[kMaxCols];
      const int64_t g = load_row<W>(in, st, chunk * 64 + lane, status, mk, iv, fv);
      uint64_t live = __ballot(g >= 0);
      while (live) {
        const int rr = __ffsll((unsigned long long)live) - 1;
        live &= live - 1;
        const int64_t gg = (int64_t)readlane_u64((uint64_t)g, rr);
        uint64_t *base = my + gg * gstride;
        if (lane == 0) __hip_atomic_fetch_add(&base[(int64_t)A * m], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        uint64_t rv[kMaxCols], rf[kMaxCols];
#pragma unroll
        for (int c = 0; c < kMaxCols; ++c) {
          if (c < ni) rv[c] = readlane_u64(iv[c], rr);
          if (c < nf) rf[c] = readlane_u64(fv[c], rr);
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint64_t word = readlane_u64(mk[w], rr);
          const int j = w * 64 + lane;
          if ((word >> lane) & 1ull) {  // no-return LDS adds: one wave's adds apply in issue order
            __hip_atomic_fetch_add(&base[j], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
            for (int c = 0; c < kMaxCols; ++c)
              if (c < ni)
                __hip_atomic_fetch_add(&base[(int64_t)(1 + c) * m + j], rv[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
            for (int c = 0; c < kMaxCols; ++c)
              if (c < nf)
                __hip_atomic_fetch_add((double *)&base[(int64_t)(1 + ni + c) * m + j],
                                       __longlong_as_double((long long)rf[c]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
    }
  }
  __syncthreads();
  // flush: sum the wave regions (fixed order), ints by atomics, floats as block partials
  for (int64_t i = threadIdx.x; i < region; i += blockDim.x) {
    const int64_t g = i / gstride, off = i % gstride;
    if (off == (int64_t)A * m) {
      uint64_t s = 0;
      for (int w = 0; w < waves_per_block; ++w) s += lds[(int64_t)w * region + i];
      if (s) atomicAdd((unsigned long long *)&st.nrows[g], (unsigned long long)s);
      continue;
    }
    const int a = (int)(off / m), j = (int)(off % m);
    if (a < 1 + ni) {
      uint64_t s = 0;
      for (int w = 0; w < waves_per_block; ++w) s += lds[(int64_t)w * region + i];
      if (s) {
        unsigned long long *dst = a == 0 ? (unsigned long long *)&st.count[g * m + j]
                                         : (unsigned long long *)&st.isum[(g * ni + (a - 1)) * m + j];
        atomicAdd(dst, (unsigned long long)s);
      }
    } else {
      double s = 0.0;
      for (int w = 0; w < waves_per_block; ++w) s += __longlong_as_double((long long)lds[(int64_t)w * region + i]);
      fpart[((int64_t)blockIdx.x * G * nf + g * nf + (a - 1 - ni)) * m + j] = s;
    }
  }
}

// Deterministic sum of the per-block float partials into the state.
__global__ __launch_bounds__(256) void reduce_fpart(const double *fpart, int nblocks, int64_t per_block,
                                                    double *fsum) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_block; i += stride) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += fpart[(int64_t)b * per_block + i];
    fsum[i] += s;
  }
}

// Global-atomic variant: large G or sparse group keys.
template <int W>
__global__ __launch_bounds__(256) void agg_plain_global(DevInput in, DevState st, uint32_t *status) {
  const int lane = threadIdx.x & 63;
  constexpr int m = 64 * W;
  const int ni = in.n_icols, nf = in.n_fcols;
  const int64_t n_chunks = (in.n_rows + 63) >> 6;
  const int64_t total_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t chunk = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); chunk < n_chunks;
       chunk += total_waves) {
    uint64_t mk[W], iv[kMaxCols], fv[kMaxCols];
    const int64_t g = load_row<W>(in, st, chunk * 64 + lane, status, mk, iv, fv);
    uint64_t live = __ballot(g >= 0);
    while (live) {
      const int rr = __ffsll((unsigned long long)live) - 1;
      live &= live - 1;
      const int64_t gg = (int64_t)readlane_u64((uint64_t)g, rr);
      if (lane == 0) atomicAdd((unsigned long long *)&st.nrows[gg], 1ull);
      uint64_t rv[kMaxCols], rf[kMaxCols];
#pragma unroll
      for (int c = 0; c < kMaxCols; ++c) {
        if (c < ni) rv[c] = readlane_u64(iv[c], rr);
        if (c < nf) rf[c] = readlane_u64(fv[c], rr);
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint64_t word = readlane_u64(mk[w], rr);
        const int j = w * 64 + lane;
        if ((word >> lane) & 1ull) {
          atomicAdd((unsigned long long *)&st.count[gg * m + j], 1ull);
#pragma unroll
          for (int c = 0; c < kMaxCols; ++c)
            if (c < ni) atomicAdd((unsigned long long *)&st.isum[(gg * ni + c) * m + j], (unsigned long long)rv[c]);
#pragma unroll
          for (int c = 0; c < kMaxCols; ++c)
            if (c < nf) atomicAdd(&st.fsum[(gg * nf + c) * m + j], __longlong_as_double((long long)rf[c]));
        }
      }
    }
  }
}

static int64_t plain_region_bytes(const DevInput &in) {
  const int64_t A = 1 + in.n_icols + in.n_fcols;
  return in.n_groups * (A * in.m + 1) * 8;
}

static constexpr int64_t kLdsBudget = 160 * 1024;

struct PlainPlan {
  bool lds;
  int wpb;     // waves per block
  int blocks;
  int64_t lds_bytes;
};

static PlainPlan plain_plan(const LaunchEnv &env, const DevInput &in) {
  PlainPlan p{};
  const int64_t region = plain_region_bytes(in);
  const int64_t n_chunks = (in.n_rows + 63) / 64;
  p.lds = !in.group_keys && region <= kLdsBudget;
  if (p.lds) {
    p.wpb = (int)std::min<int64_t>(4, kLdsBudget / region);
    p.lds_bytes = region * p.wpb;
    const int per_cu = (int)std::max<int64_t>(1, std::min<int64_t>(8, kLdsBudget / p.lds_bytes));
    int64_t want = (n_chunks + p.wpb - 1) / p.wpb;
    p.blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)env.n_cu * per_cu));
  } else {
    p.wpb = 4;
    p.lds_bytes = 0;
    int64_t want = (n_chunks + 3) / 4;
    p.blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)env.n_cu * 8));
  }
  return p;
}

bool plain_fits_lds(const DevInput &in) { return !in.group_keys && plain_region_bytes(in) <= kLdsBudget; }

// Whether four wave-private regions fit (enough waves per CU to hide latency).
bool plain_fits_lds4(const DevInput &in) { return !in.group_keys && 4 * plain_region_bytes(in) <= kLdsBudget; }

size_t plain_scratch_bytes(const LaunchEnv &env, const DevInput &in) {
  const PlainPlan p = plain_plan(env, in);
  if (!p.lds || in.n_fcols == 0) return 0;
  return (size_t)p.blocks * (size_t)in.n_groups * in.n_fcols * in.m * sizeof(double);
}

hipError_t launch_agg_plain(const LaunchEnv &env, const DevInput &in, const DevState &st, void *scratch,
                            size_t scratch_bytes) {
  if (in.n_rows <= 0) return hipSuccess;
  const PlainPlan p = plain_plan(env, in);
  if (p.lds) {
    const void *fn = in.W == 1 ? (const void *)agg_plain_lds<1> : (const void *)agg_plain_lds<2>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
    if (e != hipSuccess) return e;
    double *fpart = (double *)scratch;
    if (in.n_fcols > 0 && scratch_bytes < plain_scratch_bytes(env, in)) return hipErrorInvalidValue;
    if (in.W == 1)
      hipLaunchKernelGGL(agg_plain_lds<1>, dim3(p.blocks), dim3(64 * p.wpb), (size_t)p.lds_bytes, env.stream, in, st,
                         env.status, fpart, p.wpb);
    else
      hipLaunchKernelGGL(agg_plain_lds<2>, dim3(p.blocks), dim3(64 * p.wpb), (size_t)p.lds_bytes, env.stream, in, st,
                         env.status, fpart, p.wpb);
    e = hipGetLastError();
    if (e != hipSuccess || in.n_fcols == 0) return e;
    const int64_t per_block = in.n_groups * in.n_fcols * in.m;
    const int rb = (int)std::max<int64_t>(1, std::min<int64_t>((per_block + 255) / 256, (int64_t)env.n_cu * 4));
    hipLaunchKernelGGL(reduce_fpart, dim3(rb), dim3(256), 0, env.stream, fpart, p.blocks, per_block, st.fsum);
    return hipGetLastError();
  }
  if (in.W == 1)
    hipLaunchKernelGGL(agg_plain_global<1>, dim3(p.blocks), dim3(256), 0, env.stream, in, st, env.status);
  else
    hipLaunchKernelGGL(agg_plain_global<2>, dim3(p.blocks), dim3(256), 0, env.stream, in, st, env.status);
  return hipGetLastError();
}

}  // namespace pac
