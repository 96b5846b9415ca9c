// a7: release of the result cells (Sec. 4.1 noise function pac_noised,
// Sec. 3.2 NULLs, Sec. 5 Diversity Check, Sec. 2 adaptive composition).
//
// The posterior P over the m worlds is updated after every released cell, so
// the chain is sequential by definition: one wavefront walks the cells in
// order with lane j owning worlds j and j+64.  Each cell costs a handful of
// fp64 wave reductions (mean, variance, max, normaliser) and is latency bound.
//
// Randomness is counter based (Philox4x32-10 keyed by the query's noise
// seed, counter = (cell, purpose)), so every draw depends only on the seed
// and the cell index, never on execution order.
#include "pac_internal.h"

namespace pac {

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

enum { kDrawJStar = 0, kDrawNoise = 1, kDrawNull = 2 };

__device__ __forceinline__ void draw2(uint64_t seed, int64_t index, uint32_t purpose, uint64_t *a, uint64_t *b) {
  uint32_t c[4] = {(uint32_t)index, (uint32_t)((uint64_t)index >> 32), purpose, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  *a = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
  *b = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
}

__device__ __forceinline__ double to_unit(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

template <int W>
__global__ __launch_bounds__(64) void finalize_kernel(DevState st, const pac_cell *__restrict__ cells, FinParams fp,
                                                      double *out_val, uint8_t *out_null, uint32_t *out_flags,
                                                      double *post, double *out_y, uint32_t *status) {
  constexpr int m = 64 * W;
  const int lane = threadIdx.x;
  double P[W];
#pragma unroll
  for (int w = 0; w < W; ++w) P[w] = (fp.flags & PAC_FIN_PRIOR_IN) ? post[lane + 64 * w] : 1.0 / m;
  int jstar = fp.j_star;
  if (jstar < 0) {
    uint64_t a, b;
    draw2(fp.seed, 0, kDrawJStar, &a, &b);
    jstar = (int)(a % (uint64_t)m);
  }
  const int js_w = jstar >> 6, js_l = jstar & 63;
  const int div_max = m == 64 ? 40 : 80;
  for (int64_t c = 0; c < fp.n_cells; ++c) {
    const pac_cell cell = cells[c];
    const int64_t g = cell.group;
    const int ncol = (cell.kind == PAC_CELL_SUM_I || cell.kind == PAC_CELL_AVG_I) ? fp.n_int
                     : (cell.kind == PAC_CELL_SUM_F || cell.kind == PAC_CELL_AVG_F) ? fp.n_float : 1;
    if (g < 0 || g >= fp.n_groups || cell.kind < 0 || cell.kind > PAC_CELL_AVG_F ||
        (cell.kind != PAC_CELL_COUNT && (cell.col < 0 || cell.col >= ncol))) {
      if (lane == 0) {
        atomicOr(status, PAC_STATUS_BAD_GROUP);
        out_val[c] = 0.0;
        out_null[c] = 1;
        out_flags[c] = PAC_CELL_NULL;
      }
      continue;
    }
    double y[W];
    int pop = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int j = lane + 64 * w;
      const int64_t cnt = st.count[g * m + j];
      pop += __popcll(__ballot(cnt > 0));
      double v;
      switch (cell.kind) {
        case PAC_CELL_COUNT: v = (double)cnt; break;
        case PAC_CELL_SUM_I:
        case PAC_CELL_AVG_I: v = (double)st.isum[(g * fp.n_int + cell.col) * m + j]; break;
        default: v = st.fsum[(g * fp.n_float + cell.col) * m + j]; break;
      }
      if (cell.kind == PAC_CELL_AVG_I || cell.kind == PAC_CELL_AVG_F) {
        if (fp.flags & PAC_FIN_AVG_TOTALCOUNT) {
          const double nr = (double)st.nrows[g];
          v = nr > 0.0 ? (2.0 * v) / nr : 0.0;
        } else {
          v = cnt > 0 ? v / (double)cnt : 0.0;
        }
      } else if (fp.flags & PAC_FIN_SCALE2) {
        v = 2.0 * v;
      }
      y[w] = v;
      if (out_y) out_y[c * m + j] = v;
    }
    uint32_t flags = 0;
    if (st.nrows[g] >= 16 && pop <= div_max) {
      flags |= PAC_CELL_DIVERSITY;
      if ((fp.flags & PAC_FIN_STRICT_DIVERSITY) && lane == 0) atomicOr(status, PAC_STATUS_DIVERSITY);
    }
    uint64_t a, b;
    draw2(fp.seed, c, kDrawNull, &a, &b);
    const double p_null = (double)(m - pop) / (double)m;
    if (to_unit(a) < p_null) {
      if (lane == 0) {
        out_val[c] = 0.0;
        out_null[c] = 1;
        out_flags[c] = flags | PAC_CELL_NULL;
      }
      continue;
    }
    double part = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) part += P[w] * y[w];
    const double mu = wave_sum(part);
    part = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) part += P[w] * ((y[w] - mu) * (y[w] - mu));
    const double s2 = wave_sum(part);
    const double delta = s2 / (2.0 * fp.budget);
    const double ys = __shfl(y[js_w], js_l, 64);
    if (!(delta > 0.0)) {
      if (lane == 0) {
        out_val[c] = ys;
        out_null[c] = 0;
        out_flags[c] = flags | PAC_CELL_ZERO_VARIANCE;
      }
      continue;
    }
    draw2(fp.seed, c, kDrawNoise, &a, &b);
    const double u1 = to_unit(a), u2 = to_unit(b);
    const double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
    const double yrel = ys + sqrt(delta) * z;
    if (lane == 0) {
      out_val[c] = yrel;
      out_null[c] = 0;
      out_flags[c] = flags;
    }
    if (!(fp.flags & PAC_FIN_FIXED_PRIOR)) {
      double l[W];
      double mx = -INFINITY;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const double d = yrel - y[w];
        l[w] = log(P[w]) - (d * d) / (2.0 * delta);
        mx = fmax(mx, l[w]);
      }
      mx = wave_max(mx);
      double e[W], se = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        e[w] = exp(l[w] - mx);
        se += e[w];
      }
      se = wave_sum(se);
#pragma unroll
      for (int w = 0; w < W; ++w) P[w] = e[w] / se;
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) post[lane + 64 * w] = P[w];
}

hipError_t launch_finalize(const LaunchEnv &env, const DevState &st, const pac_cell *cells, const FinParams &fp,
                           double *out_val, uint8_t *out_is_null, uint32_t *out_flags, double *posterior,
                           double *out_y) {
  if (fp.m == 64)
    hipLaunchKernelGGL(finalize_kernel<1>, dim3(1), dim3(64), 0, env.stream, st, cells, fp, out_val, out_is_null,
                       out_flags, posterior, out_y, env.status);
  else
    hipLaunchKernelGGL(finalize_kernel<2>, dim3(1), dim3(64), 0, env.stream, st, cells, fp, out_val, out_is_null,
                       out_flags, posterior, out_y, env.status);
  return hipGetLastError();
}

}  // namespace pac
