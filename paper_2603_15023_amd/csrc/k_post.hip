// Post-aggregation steps (Sec. 4.2 vector-lifted expressions and PAC
// Selection; Sec. 3.2 categorical rewrites and the fused pac_select_<cmp>):
//   * world values: the m per-world results of one aggregate for every group,
//     as the j-th sampled database would compute them (SQL NULL as NaN);
//   * pac_select_cmp: the row's PU vector ANDed with the per-world truth of
//     `value op scale * world_value[g][j] + offset`, g the row's group in the
//     inner aggregate.  A following aggregation over these per-row vectors is
//     the outer query of a correlated nested query (e.g. rows below a
//     fraction of their part's average).
#include <algorithm>

#include "pac_internal.h"

namespace pac {

// out[g][j], one thread per (group, world).
__global__ __launch_bounds__(256) void world_values_kernel(DevState st, int m, int64_t G, int n_int, int n_float,
                                                           int kind, int col, double *out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= G * m) return;
  const int64_t g = t / m;
  const int j = (int)(t % m);
  const int64_t cnt = st.count[t];
  double v;
  switch (kind) {
    case PAC_CELL_COUNT: out[t] = (double)cnt; return;
    case PAC_CELL_SUM_I: v = (double)st.isum[(g * n_int + col) * m + j]; break;
    case PAC_CELL_AVG_I: v = (double)st.isum[(g * n_int + col) * m + j] / (double)(cnt > 0 ? cnt : 1); break;
    case PAC_CELL_SUM_F: v = st.fsum[(g * n_float + col) * m + j]; break;
    case PAC_CELL_AVG_F: v = st.fsum[(g * n_float + col) * m + j] / (double)(cnt > 0 ? cnt : 1); break;
    case PAC_CELL_MIN_I: v = (double)st.imin[(g * n_int + col) * m + j]; break;
    case PAC_CELL_MAX_I: v = (double)st.imax[(g * n_int + col) * m + j]; break;
    case PAC_CELL_MIN_F: v = st.fmin[(g * n_float + col) * m + j]; break;
    default: v = st.fmax[(g * n_float + col) * m + j]; break;
  }
  out[t] = cnt > 0 ? v : __longlong_as_double(0x7FF8000000000000ll);  // NULL world: NaN
}

__device__ __forceinline__ bool sel_cmp(double v, int op, double t) {
  if (t != t) return false;  // NULL (NaN) world value: the predicate is not true
  switch (op) {
    case PAC_SEL_LT: return v < t;
    case PAC_SEL_LE: return v <= t;
    case PAC_SEL_EQ: return v == t;
    case PAC_SEL_NE: return v != t;
    case PAC_SEL_GT: return v > t;
    default: return v >= t;
  }
}

// Lane = world.  Each wave takes 64-row batches; for every live row of the
// batch (broadcast by readlane) lane j reads world value [g][64 w + j] (one
// coalesced 512-byte read per row and word), compares, and the ballot ANDed
// with the row's PU word is that row's output word, kept by the row's lane.
template <int W>
__global__ __launch_bounds__(256) void select_cmp_kernel(DevInput in, DevState st, uint32_t *status, const double *wv,
                                                         int op, double scale, double offset, uint64_t *out) {
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63;
  const int64_t n_chunks = (in.n_rows + 63) >> 6;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < n_chunks; c += waves) {
    const int64_t r = c * 64 + lane;
    uint64_t mk[W], iv[kMaxCols], fv[kMaxCols];
    const int64_t g = load_row<W>(in, st, r, status, mk, iv, fv);  // -1: past the end, filtered or bad
    const double v = g < 0 ? 0.0
                     : in.n_icols > 0 ? (double)(int64_t)iv[0]
                                      : __longlong_as_double((long long)fv[0]);
    uint64_t res[W];
#pragma unroll
    for (int w = 0; w < W; ++w) res[w] = 0;
    uint64_t todo = __ballot(g >= 0);
    while (todo) {
      const int rr = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1;
      const int64_t gg = (int64_t)readlane_u64((uint64_t)g, rr);
      const double vv = __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(v), rr));
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const double t = wv[gg * m + 64 * w + lane];
        // separate roundings of the product and the sum (no fused multiply-add)
        const uint64_t bits = __ballot(sel_cmp(vv, op, __dadd_rn(__dmul_rn(scale, t), offset))) & readlane_u64(mk[w], rr);
        res[w] = lane == rr ? bits : res[w];
      }
    }
    if (r < in.n_rows) {
#pragma unroll
      for (int w = 0; w < W; ++w) out[r * W + w] = res[w];
    }
  }
}

hipError_t launch_world_values(const LaunchEnv &env, const DevState &st, int m, int64_t G, int n_int, int n_float,
                               int kind, int col, double *out) {
  const int64_t n = G * m;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(world_values_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, env.stream, st, m, G,
                     n_int, n_float, kind, col, out);
  return hipGetLastError();
}

hipError_t launch_select_cmp(const LaunchEnv &env, const DevInput &in, const double *wv, int op, double scale,
                             double offset, uint64_t *out) {
  if (in.n_rows <= 0) return hipSuccess;
  const int64_t n_chunks = (in.n_rows + 63) / 64;
  const int blocks = (int)std::min<int64_t>((n_chunks + 3) / 4, (int64_t)env.n_cu * 8);
  DevState none{};
  if (in.W == 1)
    hipLaunchKernelGGL(select_cmp_kernel<1>, dim3(blocks), dim3(256), 0, env.stream, in, none, env.status, wv, op,
                       scale, offset, out);
  else
    hipLaunchKernelGGL(select_cmp_kernel<2>, dim3(blocks), dim3(256), 0, env.stream, in, none, env.status, wv, op,
                       scale, offset, out);
  return hipGetLastError();
}

}  // namespace pac
