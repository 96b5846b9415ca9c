// Internal definitions shared by the host dispatch and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pac.h"

namespace pac {

constexpr int kMaxLinks = PAC_MAX_LINKS;
constexpr int kMaxGcols = PAC_MAX_GCOLS;
constexpr int kMaxCols = PAC_MAX_COLS;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;  // splitmix64 increment
constexpr uint64_t kSlotSalt = 0xA24BAED4963EE407ull;  // decorrelates table slots from PU worlds

// Kernel-side view of one aggregation (a host pac_agg_input after validation,
// with int and float columns separated and the byte-digit plan of each int
// column for the matrix-core path).
struct DevInput {
  int64_t n_rows;
  const uint64_t *masks;
  int64_t n_masks;
  const int64_t *pu_keys;
  int64_t n_pu_keys;
  uint64_t query_key;
  uint32_t balanced;
  int32_t m, W;
  int32_t n_links;
  const int32_t *links[kMaxLinks];
  int64_t link_len[kMaxLinks];
  int32_t n_gcols;
  const void *gcols[kMaxGcols];
  int32_t gcol_type[kMaxGcols];
  int64_t gcards[kMaxGcols];
  int64_t group_mod;
  const int64_t *group_keys;
  int64_t n_groups;
  const uint32_t *filter_col;
  uint32_t filter_lt;
  int32_t n_icols, n_fcols;
  const void *icols[kMaxCols];
  int32_t icol_type[kMaxCols];
  int64_t icol_lo[kMaxCols];     // digits are bytes of (v - lo) as unsigned
  int32_t icol_digits[kMaxCols]; // bytes of (max - lo) that can be non-zero
  int32_t icol_bits[kMaxCols];   // bits of (max - lo) that can be non-zero
  uint64_t icol_range[kMaxCols]; // max - lo: a value v is within the statistics iff (v - lo) <= range (unsigned)
  const void *fcols[kMaxCols];
  int32_t fcol_type[kMaxCols];
};

struct DevState {
  int64_t *count;
  int64_t *isum;
  double *fsum;
  int64_t *nrows;
  int64_t *slot_keys;
  int64_t *n_used;
  int64_t *imin, *imax;  // per-world MIN / MAX (plain form only); `minmax` says whether they are wanted
  double *fmin, *fmax;
  int32_t minmax;
};

// ---------------------------------------------------------------- hashing
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Exactly 32 one-bits: rotate left by r = mix64(h) % 64, drop the highest
// surplus ones (or fill the highest surplus zeros), rotate back.
__device__ __forceinline__ uint64_t balance32(uint64_t h) {
  const unsigned r = (unsigned)(mix64(h) & 63u);
  uint64_t x = r ? ((h << r) | (h >> (64u - r))) : h;
  int pc = __popcll(x);
  while (pc > 32) {  // clear the highest set bit
    x &= ~(1ull << (63 - __clzll(x)));
    --pc;
  }
  while (pc < 32) {  // set the highest clear bit
    x |= 1ull << (63 - __clzll(~x));
    ++pc;
  }
  return r ? ((x >> r) | (x << (64u - r))) : x;
}

__device__ __forceinline__ uint64_t pu_word(int64_t key, uint64_t qk, int w, bool balanced) {
  const uint64_t h = mix64(((uint64_t)key ^ qk) + (uint64_t)(w + 1) * kGamma);
  return balanced ? balance32(h) : h;
}

// ---------------------------------------------------------------- row access
// Follows the foreign-key chain of row r; false (and a status bit) if an
// index is out of range.
__device__ __forceinline__ bool chain_index(const DevInput &in, int64_t r, int64_t *idx, uint32_t *status) {
  int64_t x = r;
  for (int k = 0; k < in.n_links; ++k) {
    if ((uint64_t)x >= (uint64_t)in.link_len[k]) {
      atomicOr(status, PAC_STATUS_BAD_LINK);
      return false;
    }
    x = in.links[k][x];
  }
  const int64_t lim = in.masks ? in.n_masks : in.n_pu_keys;
  if ((uint64_t)x >= (uint64_t)lim) {
    atomicOr(status, PAC_STATUS_BAD_LINK);
    return false;
  }
  *idx = x;
  return true;
}

__device__ __forceinline__ uint64_t pu_of_index(const DevInput &in, int64_t idx, int w) {
  if (in.masks) return in.masks[idx * in.W + w];
  return pu_word(in.pu_keys[idx], in.query_key, w, in.balanced != 0);
}

__device__ __forceinline__ uint32_t load_gcol(const void *p, int type, int64_t r) {
  switch (type) {
    case PAC_U8: return ((const uint8_t *)p)[r];
    case PAC_U16: return ((const uint16_t *)p)[r];
    default: return ((const uint32_t *)p)[r];
  }
}

__device__ __forceinline__ int64_t load_icol(const void *p, int type, int64_t r) {
  return type == PAC_I32 ? (int64_t)((const int32_t *)p)[r] : ((const int64_t *)p)[r];
}

__device__ __forceinline__ double load_fcol(const void *p, int type, int64_t r) {
  return type == PAC_F32 ? (double)((const float *)p)[r] : ((const double *)p)[r];
}

// Dense group of row r, -1 if filtered out, -2 if a group value is out of range.
__device__ __forceinline__ int64_t dense_group(const DevInput &in, int64_t r) {
  if (in.filter_col && !(in.filter_col[r] < in.filter_lt)) return -1;
  int64_t g = 0;
  for (int k = 0; k < in.n_gcols; ++k) {
    const uint32_t v = load_gcol(in.gcols[k], in.gcol_type[k], r);
    if ((int64_t)v >= in.gcards[k]) return -2;
    g = g * in.gcards[k] + (int64_t)v;
  }
  if (in.group_mod > 0) g %= in.group_mod;
  return g < in.n_groups ? g : -2;
}

// Slot of a sparse group key in the open-addressing table (linear probing,
// capacity a power of two).  Every probe sequence ends: at most `cap` probes.
// The number of occupied slots is counted after the pass (count_used), not
// here: one counter incremented by every insert serialises a million inserts
// on a single address.
__device__ __forceinline__ int64_t table_slot(int64_t key, int64_t *slot_keys, int64_t cap, uint32_t *status) {
  uint64_t h = mix64((uint64_t)key ^ kSlotSalt) & (uint64_t)(cap - 1);
  for (int64_t probe = 0; probe < cap; ++probe) {
    // A slot's key is written once (EMPTY -> key), so a cached copy that is not
    // EMPTY is current: only an EMPTY one needs the coherent re-read.
    int64_t k = slot_keys[h];
    if (k == key) return (int64_t)h;
    if (k == PAC_EMPTY_KEY) k = __hip_atomic_load(&slot_keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == key) return (int64_t)h;
    if (k == PAC_EMPTY_KEY) {
      unsigned long long expected = (unsigned long long)PAC_EMPTY_KEY;
      const unsigned long long prev =
          atomicCAS((unsigned long long *)&slot_keys[h], expected, (unsigned long long)key);
      if (prev == expected) return (int64_t)h;
      if ((int64_t)prev == key) return (int64_t)h;
    }
    h = (h + 1) & (uint64_t)(cap - 1);
  }
  atomicOr(status, PAC_STATUS_TABLE_FULL);
  return -1;
}

// Row -> group for any grouping mode; -1 = skip the row.
__device__ __forceinline__ int64_t row_group(const DevInput &in, const DevState &st, int64_t r,
                                             uint32_t *status) {
  if (in.group_keys) {
    if (in.filter_col && !(in.filter_col[r] < in.filter_lt)) return -1;
    const int64_t key = in.group_keys[r];
    if (key == PAC_EMPTY_KEY) {
      atomicOr(status, PAC_STATUS_BAD_GROUP);
      return -1;
    }
    return table_slot(key, st.slot_keys, in.n_groups, status);
  }
  const int64_t g = dense_group(in, r);
  if (g == -2) {
    atomicOr(status, PAC_STATUS_BAD_GROUP);
    return -1;
  }
  return g;
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Loads row r: group (or -1), PU words and values.
template <int W>
__device__ __forceinline__ int64_t load_row(const DevInput &in, const DevState &st, int64_t r, uint32_t *status,
                                            uint64_t (&mk)[W], uint64_t (&iv)[kMaxCols], uint64_t (&fv)[kMaxCols]) {
  int64_t g = -1;
#pragma unroll
  for (int w = 0; w < W; ++w) mk[w] = 0;
  if (r < in.n_rows) {
    g = row_group(in, st, r, status);
    int64_t idx = 0;
    if (g >= 0 && !chain_index(in, r, &idx, status)) g = -1;
    if (g >= 0) {
#pragma unroll
      for (int w = 0; w < W; ++w) mk[w] = pu_of_index(in, idx, w);
#pragma unroll
      for (int c = 0; c < kMaxCols; ++c)
        if (c < in.n_icols) iv[c] = (uint64_t)load_icol(in.icols[c], in.icol_type[c], r);
#pragma unroll
      for (int c = 0; c < kMaxCols; ++c)
        if (c < in.n_fcols) fv[c] = (uint64_t)__double_as_longlong(load_fcol(in.fcols[c], in.fcol_type[c], r));
    }
  }
  return g;
}

// PU words and values of row r after its FK chain; false (status bit set) if a link is out of range.
template <int W>
__device__ __forceinline__ bool load_payload(const DevInput &in, int64_t r, uint32_t *status, uint64_t (&mk)[W],
                                             uint64_t (&iv)[kMaxCols], uint64_t (&fv)[kMaxCols]) {
  int64_t idx = 0;
  if (!chain_index(in, r, &idx, status)) return false;
#pragma unroll
  for (int w = 0; w < W; ++w) mk[w] = pu_of_index(in, idx, w);
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c)
    if (c < in.n_icols) iv[c] = (uint64_t)load_icol(in.icols[c], in.icol_type[c], r);
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c)
    if (c < in.n_fcols) fv[c] = (uint64_t)__double_as_longlong(load_fcol(in.fcols[c], in.fcol_type[c], r));
  return true;
}

// ---------------------------------------------------------------- launch helpers (host)
struct LaunchEnv {
  hipStream_t stream;
  int n_cu;
  uint32_t *status;
  int blocks_per_cu = 0;      // matrix-core forms: workgroups per CU of the grid (0: as many as fit)
  int scatter_wg_per_cu = 0;  // partitioned form: scatter workgroups per CU (0: one)
};

hipError_t launch_hash(const LaunchEnv &env, const int64_t *keys, int64_t n, uint64_t qk, int m, bool balanced,
                       uint64_t *out);
hipError_t launch_fill_i64(const LaunchEnv &env, int64_t *p, int64_t n, int64_t v);
hipError_t launch_fill_f64(const LaunchEnv &env, double *p, int64_t n, double v);
// Up to kMaxFillSegs arrays of 64-bit words, each set to one bit pattern, in
// one launch (empty or null segments are skipped).
constexpr int kMaxFillSegs = 12;
struct FillSegs {
  int64_t *p[kMaxFillSegs];
  int64_t n[kMaxFillSegs];
  int64_t v[kMaxFillSegs];
  int count;
};
hipError_t launch_fill_multi(const LaunchEnv &env, const FillSegs &f);
// n_used = the number of occupied (non-EMPTY) slots of a sparse-key table.
hipError_t launch_count_used(const LaunchEnv &env, const int64_t *slot_keys, int64_t cap, int64_t *n_used);
hipError_t launch_agg_plain(const LaunchEnv &env, const DevInput &in, const DevState &st, void *scratch,
                            size_t scratch_bytes);
size_t plain_scratch_bytes(const LaunchEnv &env, const DevInput &in, bool minmax);
hipError_t launch_agg_ballot(const LaunchEnv &env, const DevInput &in, const DevState &st);
bool ballot_supported(const DevInput &in);
hipError_t launch_agg_mfma(const LaunchEnv &env, const DevInput &in, const DevState &st);
bool mfma_supported(const DevInput &in);
hipError_t launch_agg_star(const LaunchEnv &env, const DevInput &in, const DevState &st);
hipError_t launch_agg_part(const LaunchEnv &env, const DevInput &in, const DevState &st, void *scratch,
                           size_t scratch_bytes, bool fresh);
bool part_supported(const DevInput &in);
size_t part_scratch_bytes(const DevInput &in);
bool plain_fits_lds(const DevInput &in);
bool reg_supported(const DevInput &in, bool minmax);
hipError_t launch_filter(const LaunchEnv &env, const double *wv, int64_t G, int m, int op, double threshold,
                         uint64_t seed, uint8_t *keep, double *frac);
hipError_t launch_world_values(const LaunchEnv &env, const DevState &st, int m, int64_t G, int n_int, int n_float,
                               int kind, int col, double *out);
hipError_t launch_select_cmp(const LaunchEnv &env, const DevInput &in, const double *wv, int op, double scale,
                             double offset, uint64_t *out);
size_t reg_scratch_bytes(const DevInput &in, bool minmax, int n_cu);
hipError_t launch_agg_reg(const LaunchEnv &env, const DevInput &in, const DevState &st, void *scratch,
                          size_t scratch_bytes);
bool plain_fits_lds4(const DevInput &in);
bool star_supported(const DevInput &in);

struct FinParams {
  double budget;
  uint64_t seed;
  int32_t j_star;
  uint32_t flags;
  int32_t m, n_int, n_float;
  int64_t n_cells;
  int64_t n_groups;
};
hipError_t launch_finalize(const LaunchEnv &env, const DevState &st, const pac_cell *cells, const FinParams &fp,
                           double *out_val, uint8_t *out_is_null, uint32_t *out_flags, double *posterior,
                           double *out_y, void *scratch);
size_t finalize_scratch_bytes(int m, int64_t n_cells);

// Measurement kernels (streaming read / copy).
hipError_t launch_stream_read(const LaunchEnv &env, const void *buf, int64_t bytes, uint64_t *out);
hipError_t launch_stream_copy(const LaunchEnv &env, const void *src, void *dst, int64_t bytes);

// One float column on the bf16 matrix cores (approximate form).
bool fmma_supported(const DevInput &in, const DevState &st);
hipError_t launch_agg_fmma(const LaunchEnv &env, const DevInput &in, const DevState &st);

// Approximate two-sided integer SUM in 16-bit cascading levels.
size_t approx_lds_bytes(const DevInput &in);
bool approx_supported(const DevInput &in, const DevState &st);
hipError_t launch_agg_approx(const LaunchEnv &env, const DevInput &in, const DevState &st);

// Shared-scan aggregation of several queries in one launch (pac_group_aggregate_batch).
constexpr int kMaxAggBatch = PAC_MAX_AGG_BATCH;
bool batch_supported(const DevInput &in, const DevState &st);
bool batch_same_rows(const DevInput &a, const DevInput &b);
size_t batch_counter_bytes(const DevInput &in);
size_t batch_lds_budget();
hipError_t launch_agg_batch(const LaunchEnv &env, const DevInput *in, const DevState *st, int n);

// One query of a batched release (pac_finalize_batch).
constexpr int kMaxReleaseBatch = PAC_MAX_RELEASE_BATCH;
struct ReleaseInput {
  DevState st;
  const pac_cell *cells;
  FinParams fp;
  double *out_val;
  uint8_t *out_null;
  uint32_t *out_flags;
  double *post;
  double *out_y;
};
size_t finalize_batch_scratch_bytes(int m, const int64_t *n_cells, int n);
hipError_t launch_finalize_batch(const LaunchEnv &env, int m, const ReleaseInput *in, int n, void *scratch);

}  // namespace pac
