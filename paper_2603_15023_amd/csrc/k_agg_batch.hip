// a2-a6 for several queries in one persistent launch: a shared scan.
//
// Sec. 4.2 compiles each query into one pass that fills the m per-world
// counters of its groups; Sec. 3.2 gives every query over the same sensitive
// table the same foreign-key path to the PU.  Queries that scan the same rows
// along the same links therefore share everything but their own filter,
// grouping, PU words (their own query key) and value columns.  This kernel
// walks the rows once for a batch of such queries:
//   * per 64-row step of a wavefront, the FK chain of each row is followed
//     once (the gathers through the orders table are the dominant row cost);
//   * then, query by query, each lane evaluates its row's filter and group,
//     its PU words (a gather from the query's word table, or the keyed hash of
//     the PU key) and values; the rows that reach the query's aggregate are
//     walked in order, each one broadcast to the wavefront (lane = world, the
//     paper's per-bit loop) and added into that query's counters in LDS;
//   * at the end every workgroup adds its non-zero LDS counters to the
//     queries' states with 64-bit atomics.
// The column reads of one query that repeat another's (the same filter or
// group column) hit the cache: a 64-row step touches a few hundred bytes per
// column.  Integer sums are exact (int64, modulo 2^64); float sums accumulate
// in fp64 with atomics, so their rounding depends on the order of the adds.
#include <algorithm>

#include "pac_internal.h"

namespace pac {

constexpr int kBatchI = 4;  // int columns per query
constexpr int kBatchF = 2;  // float columns per query
constexpr int kBatchG = 2;  // group columns per query
constexpr int kBatchWaves = 16;  // waves sharing a workgroup's LDS counters (latency of the gathers)
constexpr int kBatchLdsBytes = 96 * 1024;

struct BatchQuery {
  const uint64_t *masks;  // [n_idx][W] PU words, or NULL: hash pu_keys with qk
  const int64_t *pu_keys;
  uint64_t qk;
  uint32_t n_idx;
  uint32_t balanced;
  const uint32_t *filter_col;
  uint32_t filter_lt;
  int32_t n_gcols;
  const void *gcols[kBatchG];
  int32_t gcol_type[kBatchG];
  uint32_t gcards[kBatchG];
  uint32_t group_mod;
  double inv_mod;  // 1 / group_mod, for the modulus without an integer division
  uint32_t G;
  int32_t ni, nf;
  const void *icols[kBatchI];
  const void *fcols[kBatchF];
  uint8_t icol_type[kBatchI];
  uint8_t fcol_type[kBatchF];
  int64_t *count, *isum, *nrows;
  double *fsum;
  uint32_t lds_off;  // first 8-byte word of this query's LDS counters
};

struct BatchArgs {
  int64_t n_rows;
  int32_t n_links;
  const int32_t *links[kMaxLinks];
  int64_t link_len[kMaxLinks];
  int32_t nq;
  uint32_t lds_words;
  BatchQuery q[kMaxAggBatch];
};
static_assert(sizeof(BatchArgs) <= 4000, "batch arguments must fit the kernel argument segment");

// LDS layout of one query: count[G][m] | isum[G][ni][m] | fsum[G][nf][m] | nrows[G]
__host__ __device__ inline uint32_t batch_query_words(uint32_t G, int ni, int nf, int m) {
  return G * (uint32_t)((1 + ni + nf) * m + 1);
}

template <int W>
__global__ __launch_bounds__(64 * kBatchWaves) void agg_batch(BatchArgs a, uint32_t *status) {
  constexpr int m = 64 * W;
  extern __shared__ uint64_t lds[];
  for (uint32_t i = threadIdx.x; i < a.lds_words; i += blockDim.x) lds[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n_steps = (a.n_rows + 63) >> 6;
  const int64_t stride = (int64_t)gridDim.x * kBatchWaves;
  for (int64_t step = (int64_t)blockIdx.x * kBatchWaves + wave; step < n_steps; step += stride) {
    const int64_t r = step * 64 + lane;
    // the FK chain, once for every query of the batch
    bool ok = r < a.n_rows;
    int64_t idx = r;
    bool bad_link = false;
    for (int k = 0; k < a.n_links; ++k) {
      const bool in = (uint64_t)idx < (uint64_t)a.link_len[k];
      bad_link |= ok && !in;
      ok = ok && in;
      idx = ok ? (int64_t)a.links[k][idx] : 0;
    }
    if (bad_link) atomicOr(status, PAC_STATUS_BAD_LINK);
    for (int qi = 0; qi < a.nq; ++qi) {
      const BatchQuery &Q = a.q[qi];
      bool pass = ok && (!Q.filter_col || Q.filter_col[r] < Q.filter_lt);
      uint32_t g = 0;
      bool bad_group = false;
      if (pass) {
        for (int k = 0; k < Q.n_gcols; ++k) {
          const uint32_t v = load_gcol(Q.gcols[k], Q.gcol_type[k], r);
          bad_group |= v >= Q.gcards[k];
          g = g * Q.gcards[k] + v;
        }
        if (Q.group_mod) {  // g mod group_mod: a quotient from the fp64 reciprocal, corrected by one
          uint32_t q = (uint32_t)((double)g * Q.inv_mod);
          int64_t rem = (int64_t)g - (int64_t)q * Q.group_mod;
          if (rem < 0) rem += Q.group_mod;
          if (rem >= (int64_t)Q.group_mod) rem -= Q.group_mod;
          g = (uint32_t)rem;
        }
        bad_group |= g >= Q.G;
      }
      if (bad_group) atomicOr(status, PAC_STATUS_BAD_GROUP);
      pass = pass && !bad_group;
      const bool bad_pu = pass && (uint64_t)idx >= Q.n_idx;
      if (bad_pu) atomicOr(status, PAC_STATUS_BAD_LINK);
      pass = pass && !bad_pu;
      uint64_t mk[W];
      uint64_t iv[kBatchI];
      double fv[kBatchF];
#pragma unroll
      for (int w = 0; w < W; ++w)
        mk[w] = !pass ? 0ull
                : Q.masks ? Q.masks[idx * W + w]
                          : pu_word(Q.pu_keys[idx], Q.qk, w, Q.balanced != 0);
#pragma unroll
      for (int c = 0; c < kBatchI; ++c)
        iv[c] = pass && c < Q.ni ? (uint64_t)load_icol(Q.icols[c], Q.icol_type[c], r) : 0ull;
#pragma unroll
      for (int c = 0; c < kBatchF; ++c) fv[c] = pass && c < Q.nf ? load_fcol(Q.fcols[c], Q.fcol_type[c], r) : 0.0;
      uint64_t live = __ballot(pass);
      uint64_t *cnt = lds + Q.lds_off;
      uint64_t *isum = cnt + (size_t)Q.G * m;
      double *fsum = (double *)(isum + (size_t)Q.G * Q.ni * m);
      uint64_t *nrow = (uint64_t *)(fsum + (size_t)Q.G * Q.nf * m);
      while (live) {  // the query's rows of this step, in order, each broadcast to the wavefront
        const int rr = __builtin_ctzll(live);
        live &= live - 1;
        const uint32_t gg = (uint32_t)__builtin_amdgcn_readlane((int)g, rr);
        if (lane == 0) atomicAdd((unsigned long long *)&nrow[gg], 1ull);
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint64_t word = readlane_u64(mk[w], rr);
          if (!((word >> lane) & 1ull)) continue;
          const int j = 64 * w + lane;
          atomicAdd((unsigned long long *)&cnt[(size_t)gg * m + j], 1ull);
#pragma unroll
          for (int c = 0; c < kBatchI; ++c)
            if (c < Q.ni)
              atomicAdd((unsigned long long *)&isum[((size_t)gg * Q.ni + c) * m + j],
                        (unsigned long long)readlane_u64(iv[c], rr));
#pragma unroll
          for (int c = 0; c < kBatchF; ++c)
            if (c < Q.nf) {
              const uint64_t bits = readlane_u64((uint64_t)__double_as_longlong(fv[c]), rr);
              atomicAdd(&fsum[((size_t)gg * Q.nf + c) * m + j], __longlong_as_double((long long)bits));
            }
        }
      }
    }
  }
  __syncthreads();
  // the workgroup's counters into every query's state
  for (int qi = 0; qi < a.nq; ++qi) {
    const BatchQuery &Q = a.q[qi];
    const uint32_t words = batch_query_words(Q.G, Q.ni, Q.nf, m);
    const uint32_t n_cnt = Q.G * m, n_isum = Q.G * Q.ni * m, n_fsum = Q.G * Q.nf * m;
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) {
      const uint64_t v = lds[Q.lds_off + i];
      if (!v) continue;
      if (i < n_cnt) {
        atomicAdd((unsigned long long *)&Q.count[i], (unsigned long long)v);
      } else if (i < n_cnt + n_isum) {
        atomicAdd((unsigned long long *)&Q.isum[i - n_cnt], (unsigned long long)v);
      } else if (i < n_cnt + n_isum + n_fsum) {
        atomicAdd(&Q.fsum[i - n_cnt - n_isum], __longlong_as_double((long long)v));
      } else {
        atomicAdd((unsigned long long *)&Q.nrows[i - n_cnt - n_isum - n_fsum], (unsigned long long)v);
      }
    }
  }
}

// ---------------------------------------------------------------- host side
size_t batch_counter_bytes(const DevInput &in) {
  return (size_t)batch_query_words((uint32_t)std::min<int64_t>(in.n_groups, 1 << 24), in.n_icols, in.n_fcols, in.m) * 8;
}

bool batch_supported(const DevInput &in, const DevState &st) {
  if (in.group_keys || st.minmax || in.n_icols > kBatchI || in.n_fcols > kBatchF || in.n_gcols > kBatchG) return false;
  if (in.n_rows <= 0 || in.n_groups < 1 || in.n_groups > (1 << 20)) return false;
  const int64_t n_idx = in.masks ? in.n_masks : in.n_pu_keys;
  if (n_idx < 0 || n_idx >= ((int64_t)1 << 32)) return false;
  for (int k = 0; k < in.n_gcols; ++k)
    if (in.gcards[k] >= ((int64_t)1 << 32)) return false;
  if (in.group_mod >= ((int64_t)1 << 32)) return false;
  return batch_counter_bytes(in) <= (size_t)kBatchLdsBytes;
}

bool batch_same_rows(const DevInput &a, const DevInput &b) {
  if (a.n_rows != b.n_rows || a.n_links != b.n_links || a.W != b.W) return false;
  for (int k = 0; k < a.n_links; ++k)
    if (a.links[k] != b.links[k] || a.link_len[k] != b.link_len[k]) return false;
  return true;
}

size_t batch_lds_budget() { return kBatchLdsBytes; }

hipError_t launch_agg_batch(const LaunchEnv &env, const DevInput *in, const DevState *st, int n) {
  if (n <= 0) return hipSuccess;
  if (n > kMaxAggBatch) return hipErrorInvalidValue;
  BatchArgs a{};
  a.n_rows = in[0].n_rows;
  a.n_links = in[0].n_links;
  for (int k = 0; k < a.n_links; ++k) {
    a.links[k] = in[0].links[k];
    a.link_len[k] = in[0].link_len[k];
  }
  a.nq = n;
  uint32_t off = 0;
  for (int i = 0; i < n; ++i) {
    const DevInput &d = in[i];
    BatchQuery &q = a.q[i];
    q.masks = d.masks;
    q.pu_keys = d.pu_keys;
    q.qk = d.query_key;
    q.n_idx = (uint32_t)(d.masks ? d.n_masks : d.n_pu_keys);
    q.balanced = d.balanced;
    q.filter_col = d.filter_col;
    q.filter_lt = d.filter_lt;
    q.n_gcols = d.n_gcols;
    for (int k = 0; k < d.n_gcols; ++k) {
      q.gcols[k] = d.gcols[k];
      q.gcol_type[k] = d.gcol_type[k];
      q.gcards[k] = (uint32_t)d.gcards[k];
    }
    q.group_mod = (uint32_t)d.group_mod;
    q.inv_mod = d.group_mod ? 1.0 / (double)d.group_mod : 0.0;
    q.G = (uint32_t)d.n_groups;
    q.ni = d.n_icols;
    q.nf = d.n_fcols;
    for (int c = 0; c < d.n_icols; ++c) {
      q.icols[c] = d.icols[c];
      q.icol_type[c] = (uint8_t)d.icol_type[c];
    }
    for (int c = 0; c < d.n_fcols; ++c) {
      q.fcols[c] = d.fcols[c];
      q.fcol_type[c] = (uint8_t)d.fcol_type[c];
    }
    q.count = st[i].count;
    q.isum = st[i].isum;
    q.fsum = st[i].fsum;
    q.nrows = st[i].nrows;
    q.lds_off = off;
    off += batch_query_words(q.G, q.ni, q.nf, d.m);
  }
  a.lds_words = off;
  const size_t lds = (size_t)off * 8;
  if (lds > (size_t)kBatchLdsBytes) return hipErrorInvalidValue;
  const void *fn = in[0].W == 1 ? (const void *)agg_batch<1> : (const void *)agg_batch<2>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)std::max<size_t>(lds, 8));
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kBatchWaves, std::max<size_t>(lds, 8));
  if (e != hipSuccess) return e;
  per_cu = std::max(1, per_cu);
  const int64_t n_steps = (a.n_rows + 63) / 64;
  const int64_t want = (n_steps + kBatchWaves - 1) / kBatchWaves;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)env.n_cu * per_cu));
  if (in[0].W == 1)
    hipLaunchKernelGGL(agg_batch<1>, dim3(blocks), dim3(64 * kBatchWaves), std::max<size_t>(lds, 8), env.stream, a,
                       env.status);
  else
    hipLaunchKernelGGL(agg_batch<2>, dim3(blocks), dim3(64 * kBatchWaves), std::max<size_t>(lds, 8), env.stream, a,
                       env.status);
  return hipGetLastError();
}

}  // namespace pac
