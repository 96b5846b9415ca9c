// Post-aggregation steps (Sec. 4.2 vector-lifted expressions and PAC
// Selection; Sec. 3.2 categorical rewrites and the fused pac_select_<cmp>):
//   * world values: the m per-world results of one aggregate for every group,
//     as the j-th sampled database would compute them (SQL NULL as NaN);
//   * pac_select_cmp: the row's PU vector ANDed with the per-world truth of
//     `value op scale * world_value[g][j] + offset`, g the row's group in the
//     inner aggregate.  A following aggregation over these per-row vectors is
//     the outer query of a correlated nested query (e.g. rows below a
//     fraction of their part's average);
//   * vector-lifted expressions: a postfix program over per-world inputs,
//     evaluated for every (group, world) -- e.g. a ratio of two sums -- whose
//     result pac_noised releases once.
#include <algorithm>

#include "pac_post.h"

namespace pac {

// out[g][j], one thread per (group, world).  kind carries the PAC_WV_* flags
// above its low byte: with PAC_WV_RELEASE the value is the release's world
// vector (the same operations as the release's phase 1) and every world
// without rows is NULL, COUNT included.
__global__ __launch_bounds__(256) void world_values_kernel(DevState st, int m, int64_t G, int n_int, int n_float,
                                                           int kind, int col, double *out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= G * m) return;
  const int64_t g = t / m;
  const int j = (int)(t % m);
  const int k = kind & 0xFF;
  const bool rel = (kind & PAC_WV_RELEASE) != 0;
  const int64_t cnt = st.count[t];
  double v;
  switch (k) {
    case PAC_CELL_COUNT: v = (double)cnt; break;
    case PAC_CELL_SUM_I:
    case PAC_CELL_AVG_I: v = (double)st.isum[(g * n_int + col) * m + j]; break;
    case PAC_CELL_SUM_F:
    case PAC_CELL_AVG_F: v = st.fsum[(g * n_float + col) * m + j]; break;
    case PAC_CELL_MIN_I: v = (double)st.imin[(g * n_int + col) * m + j]; break;
    case PAC_CELL_MAX_I: v = (double)st.imax[(g * n_int + col) * m + j]; break;
    case PAC_CELL_MIN_F: v = st.fmin[(g * n_float + col) * m + j]; break;
    default: v = st.fmax[(g * n_float + col) * m + j]; break;
  }
  if (k == PAC_CELL_AVG_I || k == PAC_CELL_AVG_F) {
    if (rel && (kind & PAC_WV_AVG_TOTALCOUNT)) {
      const double nr = (double)st.nrows[g];
      v = nr > 0.0 ? (2.0 * v) / nr : 0.0;
    } else {
      v = v / (double)(cnt > 0 ? cnt : 1);
    }
  } else if ((kind & PAC_WV_SCALE2) && (k == PAC_CELL_COUNT || k == PAC_CELL_SUM_I || k == PAC_CELL_SUM_F)) {
    v = 2.0 * v;
  }
  const bool null = cnt <= 0 && (rel || k != PAC_CELL_COUNT);
  out[t] = null ? __longlong_as_double(0x7FF8000000000000ll) : v;  // NULL world: NaN
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

// Table form for an integer compared value with a small known range
// [lo, lo + R): for every group g and value v, the m-bit word of worlds j with
// v op scale * y_j(g) + offset, one wave per group (lane = world; lane k of
// each 64-value batch keeps the ballot of value k and writes it, so the table
// rows are written contiguously).  The comparison is the one the row-wise
// form makes, on the same doubles, so a table word equals that form's result.
template <int W>
__global__ __launch_bounds__(256) void sel_table_kernel(const double *wv, int64_t G, int op, double scale,
                                                        double offset, int64_t lo, int32_t R, uint64_t *table) {
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (g >= G) return;
  double t[W];
#pragma unroll
  for (int w = 0; w < W; ++w) t[w] = __dadd_rn(__dmul_rn(scale, wv[g * m + 64 * w + lane]), offset);
  for (int v0 = 0; v0 < R; v0 += 64) {
    uint64_t mine[W];
#pragma unroll
    for (int w = 0; w < W; ++w) mine[w] = 0;
    const int nb = R - v0 < 64 ? R - v0 : 64;
    const double vb = (double)(lo + v0);  // exact: the host keeps the range within +-2^52
    for (int k = 0; k < nb; ++k) {
      const double v = vb + (double)k;  // the same double as (double)(lo + v0 + k)
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint64_t bits = __ballot(sel_cmp(v, op, t[w]));
        mine[w] = lane == k ? bits : mine[w];
      }
    }
    if (lane < nb) {
#pragma unroll
      for (int w = 0; w < W; ++w) table[((g * R) + v0 + lane) * W + w] = mine[w];
    }
  }
}

// Lane = world.  Each wave takes 64-row batches; for every live row of the
// batch (broadcast by readlane) lane j reads world value [g][64 w + j] (one
// coalesced 512-byte read per row and word), compares, and the ballot ANDed
// with the row's PU word is that row's output word, kept by the row's lane.
// With a table (TAB), a row whose integer value lies in [lo, lo + R) takes its
// word from the table instead (one 8-byte read per word); only the other rows
// go through the per-world loop.
template <int W, bool TAB>
__global__ __launch_bounds__(256) void select_cmp_kernel(DevInput in, DevState st, uint32_t *status, const double *wv,
                                                         int op, double scale, double offset, const uint64_t *table,
                                                         int64_t lo, int32_t R, uint64_t *out) {
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
    bool done = false;
    if (TAB && g >= 0) {
      const uint64_t d = (uint64_t)((int64_t)iv[0] - lo);  // wraps to a large value below lo
      if (d < (uint64_t)R) {
        done = true;
#pragma unroll
        for (int w = 0; w < W; ++w) res[w] = table[((g * R) + (int64_t)d) * W + w] & mk[w];
      }
    }
    uint64_t todo = __ballot(g >= 0 && !done);
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

// ---------------------------------------------------------------- vector-lifted expressions
// The value stack lives in registers: the stack pointer is the same in every
// lane (one program for all), and each access selects among the fixed slots.
__device__ __forceinline__ double stk_get(const double (&s)[PAC_LIFT_MAX_DEPTH], int i) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < PAC_LIFT_MAX_DEPTH; ++k) r = k == i ? s[k] : r;
  return r;
}

__device__ __forceinline__ void stk_put(double (&s)[PAC_LIFT_MAX_DEPTH], int i, double v) {
#pragma unroll
  for (int k = 0; k < PAC_LIFT_MAX_DEPTH; ++k) s[k] = k == i ? v : s[k];
}

// One thread per (group, world), grid-stride.  The host has checked the
// program: every input index exists, the stack never underflows, never holds
// more than PAC_LIFT_MAX_DEPTH values and ends with one.
__global__ __launch_bounds__(256) void lift_kernel(LiftProg p, int64_t G, int m_shift, double *out) {
  const int64_t n = G << m_shift;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int64_t g = t >> m_shift;
    double s[PAC_LIFT_MAX_DEPTH];
#pragma unroll
    for (int k = 0; k < PAC_LIFT_MAX_DEPTH; ++k) s[k] = 0.0;
    int sp = 0;
    for (int i = 0; i < p.n_ops; ++i) {
      const int op = p.op[i];
      if (op == PAC_LIFT_INPUT) {
        const int a = p.arg[i];
        const double *x = p.in[a];
        stk_put(s, sp, ((p.scalar >> a) & 1u) ? x[g] : x[t]);
        ++sp;
      } else if (op == PAC_LIFT_CONST) {
        stk_put(s, sp, p.val[i]);
        ++sp;
      } else if (op == PAC_LIFT_NEG) {
        stk_put(s, sp - 1, -stk_get(s, sp - 1));
      } else {
        const double b = stk_get(s, sp - 1), a = stk_get(s, sp - 2);
        double r;
        switch (op) {
          case PAC_LIFT_ADD: r = __dadd_rn(a, b); break;
          case PAC_LIFT_SUB: r = __dsub_rn(a, b); break;
          case PAC_LIFT_MUL: r = __dmul_rn(a, b); break;
          default: r = b == 0.0 ? __longlong_as_double(0x7FF8000000000000ll) : __ddiv_rn(a, b); break;
        }
        --sp;
        stk_put(s, sp - 1, r);
      }
    }
    out[t] = s[0];
  }
}

hipError_t launch_lift(const LaunchEnv &env, const LiftProg &prog, int64_t G, int m, double *out) {
  const int64_t n = G * m;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, (int64_t)env.n_cu * 16);
  hipLaunchKernelGGL(lift_kernel, dim3(blocks), dim3(256), 0, env.stream, prog, G, m == 64 ? 6 : 7, out);
  return hipGetLastError();
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
  return launch_select_table(env, in, wv, op, scale, offset, 0, 0, nullptr, out);
}

hipError_t launch_select_table(const LaunchEnv &env, const DevInput &in, const double *wv, int op, double scale,
                               double offset, int64_t lo, int32_t R, uint64_t *table, uint64_t *out) {
  if (in.n_rows <= 0) return hipSuccess;
  const bool tab = table != nullptr && R > 0;
  if (tab) {
    const unsigned gblocks = (unsigned)((in.n_groups + 3) / 4);
    if (in.W == 1)
      hipLaunchKernelGGL(sel_table_kernel<1>, dim3(gblocks), dim3(256), 0, env.stream, wv, in.n_groups, op, scale,
                         offset, lo, R, table);
    else
      hipLaunchKernelGGL(sel_table_kernel<2>, dim3(gblocks), dim3(256), 0, env.stream, wv, in.n_groups, op, scale,
                         offset, lo, R, table);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t n_chunks = (in.n_rows + 63) / 64;
  const int blocks = (int)std::min<int64_t>((n_chunks + 3) / 4, (int64_t)env.n_cu * 8);
  DevState none{};
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, env.stream, in, none, env.status, wv, op, scale, offset,
                       (const uint64_t *)table, lo, R, out);
  };
  if (in.W == 1) {
    if (tab) go(select_cmp_kernel<1, true>); else go(select_cmp_kernel<1, false>);
  } else {
    if (tab) go(select_cmp_kernel<2, true>); else go(select_cmp_kernel<2, false>);
  }
  return hipGetLastError();
}

}  // namespace pac
