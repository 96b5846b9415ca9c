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
//
// It is also the form of pac_min / pac_max (Sec. 4.2, agg in {min, max}):
// with a MIN/MAX state, each group's region carries per-world minimum and
// maximum words of every column after the sums, updated by LDS min/max
// atomics under the same predicate.  Min and max are exact in any order.  The
// paper's bound pruning (Sec. 5: skip values that cannot improve the worst of
// the 64 extremes) saves 64 scalar compare-and-selects per value on a CPU;
// here the 64 worlds are the lanes of one predicated LDS instruction, so there
// is nothing to prune.
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
  const bool mm = st.minmax != 0;
  // per-group slots: A*m counters + nrows, then (MIN/MAX) imin, imax [ni][m], fmin, fmax [nf][m]
  const int64_t mm_off = (int64_t)A * m + 1;
  const int64_t gstride = mm_off + (mm ? (int64_t)2 * (ni + nf) * m : 0);
  const int64_t region = G * gstride;
  for (int64_t i = threadIdx.x; i < region * waves_per_block; i += blockDim.x) {
    const int64_t off = (i % region) % gstride;
    uint64_t v = 0;
    if (off >= mm_off) {
      const int64_t sec = (off - mm_off) / m;
      v = sec < ni ? (uint64_t)INT64_MAX
                   : sec < 2 * ni ? (uint64_t)INT64_MIN
                                  : (uint64_t)__double_as_longlong(sec < 2 * ni + nf ? INFINITY : -INFINITY);
    }
    lds[i] = v;
  }
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
            if (mm) {
              long long *mi = (long long *)(base + mm_off);
#pragma unroll
              for (int c = 0; c < kMaxCols; ++c)
                if (c < ni) {
                  __hip_atomic_fetch_min(&mi[(int64_t)c * m + j], (long long)rv[c], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                  __hip_atomic_fetch_max(&mi[(int64_t)(ni + c) * m + j], (long long)rv[c], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                }
              double *mf = (double *)(base + mm_off + (int64_t)2 * ni * m);
#pragma unroll
              for (int c = 0; c < kMaxCols; ++c)
                if (c < nf) {
                  const double x = __longlong_as_double((long long)rf[c]);
                  __hip_atomic_fetch_min(&mf[(int64_t)c * m + j], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                  __hip_atomic_fetch_max(&mf[(int64_t)(nf + c) * m + j], x, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // flush: sum the wave regions (fixed order), ints by atomics, floats as block partials
  for (int64_t i = threadIdx.x; i < region; i += blockDim.x) {
    const int64_t g = i / gstride, off = i % gstride;
    if (off > (int64_t)A * m) {  // MIN / MAX: extreme over the waves, then to the state if any row came
      const int64_t sec = (off - mm_off) / m, j = (off - mm_off) % m;
      if (sec < 2 * ni) {
        const bool is_min = sec < ni;
        const int64_t c = is_min ? sec : sec - ni;
        long long x = (long long)lds[i];
        for (int w = 1; w < waves_per_block; ++w) {
          const long long y = (long long)lds[(int64_t)w * region + i];
          x = is_min ? (y < x ? y : x) : (y > x ? y : x);
        }
        long long *dst = (long long *)(is_min ? st.imin : st.imax) + (g * ni + c) * m + j;
        if (is_min && x != INT64_MAX) __hip_atomic_fetch_min(dst, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!is_min && x != INT64_MIN) __hip_atomic_fetch_max(dst, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const bool is_min = sec < 2 * ni + nf;
        const int64_t c = is_min ? sec - 2 * ni : sec - 2 * ni - nf;
        double x = __longlong_as_double((long long)lds[i]);
        for (int w = 1; w < waves_per_block; ++w) {
          const double y = __longlong_as_double((long long)lds[(int64_t)w * region + i]);
          x = is_min ? (y < x ? y : x) : (y > x ? y : x);
        }
        double *dst = (is_min ? st.fmin : st.fmax) + (g * nf + c) * m + j;
        if (is_min && x != INFINITY) __hip_atomic_fetch_min(dst, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!is_min && x != -INFINITY) __hip_atomic_fetch_max(dst, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      continue;
    }
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
          if (st.minmax) {
#pragma unroll
            for (int c = 0; c < kMaxCols; ++c)
              if (c < ni) {
                const int64_t o = (gg * ni + c) * m + j;
                __hip_atomic_fetch_min((long long *)&st.imin[o], (long long)rv[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max((long long *)&st.imax[o], (long long)rv[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
              }
#pragma unroll
            for (int c = 0; c < kMaxCols; ++c)
              if (c < nf) {
                const int64_t o = (gg * nf + c) * m + j;
                const double x = __longlong_as_double((long long)rf[c]);
                __hip_atomic_fetch_min(&st.fmin[o], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&st.fmax[o], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              }
          }
        }
      }
    }
  }
}

static int64_t plain_region_bytes(const DevInput &in, bool minmax = false) {
  const int64_t A = 1 + in.n_icols + in.n_fcols;
  const int64_t mm = minmax ? 2 * (int64_t)(in.n_icols + in.n_fcols) * in.m : 0;
  return in.n_groups * (A * in.m + 1 + mm) * 8;
}

static constexpr int64_t kLdsBudget = 160 * 1024;

struct PlainPlan {
  bool lds;
  int wpb;     // waves per block
  int blocks;
  int64_t lds_bytes;
};

static PlainPlan plain_plan(const LaunchEnv &env, const DevInput &in, bool minmax) {
  PlainPlan p{};
  const int64_t region = plain_region_bytes(in, minmax);
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

size_t plain_scratch_bytes(const LaunchEnv &env, const DevInput &in, bool minmax) {
  const PlainPlan p = plain_plan(env, in, minmax);
  if (!p.lds || in.n_fcols == 0) return 0;
  return (size_t)p.blocks * (size_t)in.n_groups * in.n_fcols * in.m * sizeof(double);
}

hipError_t launch_agg_plain(const LaunchEnv &env, const DevInput &in, const DevState &st, void *scratch,
                            size_t scratch_bytes) {
  if (in.n_rows <= 0) return hipSuccess;
  const PlainPlan p = plain_plan(env, in, st.minmax != 0);
  if (p.lds) {
    const void *fn = in.W == 1 ? (const void *)agg_plain_lds<1> : (const void *)agg_plain_lds<2>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
    if (e != hipSuccess) return e;
    double *fpart = (double *)scratch;
    if (in.n_fcols > 0 && scratch_bytes < plain_scratch_bytes(env, in, st.minmax != 0)) return hipErrorInvalidValue;
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
