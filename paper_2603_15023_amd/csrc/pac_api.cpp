// Host side of the C ABI: argument checks, input planning, kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pac_internal.h"
#include "pac_join.h"
#include "pac_post.h"

struct pac_ctx {
  int device;
  int n_cu;
  uint32_t *d_status;
  void *scratch;
  size_t scratch_bytes;
  void *noalloc;  // device address of this device's copy of noalloc_scratch
  std::vector<pac_tune_entry> tuning;  // measured choices per input class (pac_set_tuning)
};

// Working memory of pac_finalize_noalloc: a fixed array in the library's code
// object, of which every device holds its own copy.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol); it passes the device address that hipGetSymbolAddress returns with
// that device current, looked up once per device.
constexpr size_t kNoAllocBytes = (size_t)PAC_NOALLOC_MAX_CELLS * (128 * sizeof(double) + 16) + 256;
static __device__ __align__(256) uint8_t noalloc_scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_addr[kMaxDevices] = {};

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(PAC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Runs the body with the context's device current, restoring the caller's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int ensure_scratch(pac_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return PAC_OK;
  if (ctx->scratch) {
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, (size_t)1 << 20);
  if (hipMalloc(&ctx->scratch, want) != hipSuccess) {
    ctx->scratch = nullptr;
    return fail(PAC_ERR_OOM, "scratch allocation of %zu bytes failed", want);
  }
  ctx->scratch_bytes = want;
  return PAC_OK;
}

// Device address of noalloc_scratch on `device`, which must be current.
int noalloc_address(int device, void **out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (device < 0 || device >= kMaxDevices) return fail(PAC_ERR_UNSUPPORTED, "device %d: above %d devices", device, kMaxDevices);
  if (!g_noalloc_addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(noalloc_scratch)");
    if (!p) return fail(PAC_ERR_HIP, "hipGetSymbolAddress(noalloc_scratch) returned null");
    g_noalloc_addr[device] = p;
  }
  *out = g_noalloc_addr[device];
  return PAC_OK;
}

bool is_int(int t) { return t == PAC_I32 || t == PAC_I64; }
bool is_float(int t) { return t == PAC_F32 || t == PAC_F64; }
bool is_gtype(int t) { return t == PAC_U8 || t == PAC_U16 || t == PAC_U32; }

// pac_select_cmp's table form: at most this many distinct compared values,
// and at most this much scratch for the [groups][values] word table.
constexpr int64_t kSelTableMaxRange = 4096;
constexpr int64_t kSelTableMaxBytes = (int64_t)1 << 30;

int bit_length(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

// Validates one input and builds the kernel view.  Returns PAC_OK or an error.
int plan_input(const pac_agg_input *in, int m, uint64_t qk, const pac_agg_state *st, pac::DevInput *d,
               pac::DevState *ds) {
  // st == nullptr: rows only (pac_select_cmp); no state checks, ds untouched
  if (!in) return fail(PAC_ERR_INVALID, "null input");
  if (m != 64 && m != 128) return fail(PAC_ERR_INVALID, "m must be 64 or 128 (got %d)", m);
  if (in->n_rows < 0) return fail(PAC_ERR_INVALID, "n_rows < 0");
  if (in->n_links < 0 || in->n_links > PAC_MAX_LINKS) return fail(PAC_ERR_INVALID, "n_links out of range");
  if (in->n_gcols < 0 || in->n_gcols > PAC_MAX_GCOLS) return fail(PAC_ERR_INVALID, "n_gcols out of range");
  if (in->n_cols < 0 || in->n_cols > PAC_MAX_COLS) return fail(PAC_ERR_INVALID, "n_cols out of range");
  if (in->n_rows > 0 && !in->masks && !in->pu_keys) return fail(PAC_ERR_INVALID, "need masks or pu_keys");
  if (in->masks && in->n_masks < 0) return fail(PAC_ERR_INVALID, "n_masks < 0");
  if (!in->masks && in->pu_keys && in->n_pu_keys < 0) return fail(PAC_ERR_INVALID, "n_pu_keys < 0");
  for (int k = 0; k < in->n_links; ++k)
    if (in->link_len[k] < 0 || (!in->links[k] && in->link_len[k] > 0))
      return fail(PAC_ERR_INVALID, "link %d missing", k);
  if (in->n_groups < 1) return fail(PAC_ERR_INVALID, "n_groups must be >= 1");
  if (in->group_keys) {
    if (in->n_gcols > 0 || in->group_mod > 0) return fail(PAC_ERR_INVALID, "sparse keys exclude group columns");
    if (in->n_groups & (in->n_groups - 1)) return fail(PAC_ERR_INVALID, "sparse capacity must be a power of two");
    if (st && (!st->slot_keys || !st->n_used)) return fail(PAC_ERR_INVALID, "sparse mode needs slot_keys and n_used");
  } else {
    if (in->n_gcols == 0 && in->group_mod == 0 && in->n_groups != 1)
      return fail(PAC_ERR_INVALID, "ungrouped aggregate needs n_groups == 1");
    if (in->group_mod < 0) return fail(PAC_ERR_INVALID, "group_mod < 0");
    double prod = 1.0;
    for (int k = 0; k < in->n_gcols; ++k) {
      if ((!in->gcols[k] && in->n_rows > 0) || !is_gtype(in->gcol_type[k]) || in->gcards[k] < 1)
        return fail(PAC_ERR_INVALID, "bad group column %d", k);
      prod *= (double)in->gcards[k];
    }
    if (prod > 4.0e9) return fail(PAC_ERR_UNSUPPORTED, "composite group key space above 2^32");
  }
  if (st && (!st->count || !st->nrows)) return fail(PAC_ERR_INVALID, "state.count and state.nrows are required");
  const int64_t G = in->n_groups;
  if ((double)G * m * (1 + in->n_cols) > 4.0e12) return fail(PAC_ERR_INVALID, "state too large");

  std::memset(d, 0, sizeof(*d));
  d->n_rows = in->n_rows;
  d->masks = in->masks;
  d->n_masks = in->n_masks;
  d->pu_keys = in->pu_keys;
  d->n_pu_keys = in->n_pu_keys;
  d->query_key = qk;
  d->balanced = (in->hash_flags & PAC_HASH_BALANCED) ? 1u : 0u;
  d->m = m;
  d->W = m / 64;
  d->n_links = in->n_links;
  for (int k = 0; k < in->n_links; ++k) {
    d->links[k] = in->links[k];
    d->link_len[k] = in->link_len[k];
  }
  d->n_gcols = in->n_gcols;
  for (int k = 0; k < in->n_gcols; ++k) {
    d->gcols[k] = in->gcols[k];
    d->gcol_type[k] = in->gcol_type[k];
    d->gcards[k] = in->gcards[k];
  }
  d->group_mod = in->group_mod;
  d->group_keys = in->group_keys;
  d->n_groups = G;
  d->filter_col = in->filter_col;
  d->filter_lt = in->filter_lt;
  for (int c = 0; c < in->n_cols; ++c) {
    const int t = in->col_type[c];
    if (!in->cols[c] && in->n_rows > 0) return fail(PAC_ERR_INVALID, "value column %d missing", c);
    if (is_int(t)) {
      const int i = d->n_icols++;
      d->icols[i] = in->cols[c];
      d->icol_type[i] = t;
      int64_t lo, hi;
      if (in->has_stats) {
        lo = in->col_min[c];
        hi = in->col_max[c];
        if (lo > hi) return fail(PAC_ERR_INVALID, "column %d: min > max", c);
        const __int128 amax = std::max<__int128>(-(__int128)lo, (__int128)hi);
        if (amax * (__int128)in->n_rows >= ((__int128)1 << 63))
          return fail(PAC_ERR_OVERFLOW, "column %d: n_rows * max|v| may exceed int64", c);
      } else if (t == PAC_I32) {
        lo = INT32_MIN;
        hi = INT32_MAX;
      } else {
        lo = INT64_MIN;
        hi = INT64_MAX;
      }
      const uint64_t range = (uint64_t)hi - (uint64_t)lo;
      d->icol_lo[i] = lo;
      d->icol_range[i] = range;
      d->icol_bits[i] = bit_length(range);
      d->icol_digits[i] = (bit_length(range) + 7) / 8;
    } else if (is_float(t)) {
      const int f = d->n_fcols++;
      d->fcols[f] = in->cols[c];
      d->fcol_type[f] = t;
    } else {
      return fail(PAC_ERR_INVALID, "value column %d: bad type %d", c, t);
    }
  }
  // the scan kernels use 16-byte vector loads of 4 consecutive rows
  auto misaligned = [](const void *p) { return ((uintptr_t)p & 15u) != 0; };
  for (int c = 0; c < in->n_cols; ++c)
    if (misaligned(in->cols[c])) return fail(PAC_ERR_INVALID, "value column %d is not 16-byte aligned", c);
  for (int k = 0; k < in->n_gcols; ++k)
    if (misaligned(in->gcols[k])) return fail(PAC_ERR_INVALID, "group column %d is not 16-byte aligned", k);
  if (misaligned(in->filter_col)) return fail(PAC_ERR_INVALID, "filter column is not 16-byte aligned");
  if (!st) return PAC_OK;
  if (d->n_icols > 0 && !st->isum) return fail(PAC_ERR_INVALID, "state.isum required for int columns");
  if (d->n_fcols > 0 && !st->fsum) return fail(PAC_ERR_INVALID, "state.fsum required for float columns");
  ds->count = st->count;
  ds->isum = st->isum;
  ds->fsum = st->fsum;
  ds->nrows = st->nrows;
  ds->slot_keys = st->slot_keys;
  ds->n_used = st->n_used;
  ds->imin = st->imin;
  ds->imax = st->imax;
  ds->fmin = st->fmin;
  ds->fmax = st->fmax;
  ds->minmax = (st->imin || st->imax || st->fmin || st->fmax) ? 1 : 0;
  if (ds->minmax && d->n_icols > 0 && !(st->imin && st->imax))
    return fail(PAC_ERR_INVALID, "state.imin and state.imax required for MIN/MAX of int columns");
  if (ds->minmax && d->n_fcols > 0 && !(st->fmin && st->fmax))
    return fail(PAC_ERR_INVALID, "state.fmin and state.fmax required for MIN/MAX of float columns");
  return PAC_OK;
}

// The input class of a tuning entry.
void tune_key(const pac::DevInput &d, const pac::DevState &ds, pac_tune_entry *k) {
  std::memset(k, 0, sizeof(*k));
  k->W = d.W;
  k->sparse = d.group_keys ? 1 : 0;
  k->gbits = bit_length((uint64_t)(d.n_groups - 1));
  k->n_int = d.n_icols;
  k->n_float = d.n_fcols;
  for (int c = 0; c < d.n_icols; ++c) k->digits = std::max(k->digits, (int32_t)d.icol_digits[c]);
  k->filter = d.filter_col ? 1 : 0;
  k->minmax = ds.minmax ? 1 : 0;
}

bool same_class(const pac_tune_entry &a, const pac_tune_entry &b) {
  return a.W == b.W && a.sparse == b.sparse && a.gbits == b.gbits && a.n_int == b.n_int && a.n_float == b.n_float &&
         a.digits == b.digits && a.filter == b.filter && a.minmax == b.minmax;
}

// Whether a form can run this input (the checks of run_one's dispatch).
bool algo_runs(uint32_t algo, const pac::DevInput &d, const pac::DevState &ds) {
  if (ds.minmax && algo != PAC_ALGO_PLAIN && algo != PAC_ALGO_REGISTER) return false;
  switch (algo) {
    case PAC_ALGO_PLAIN: return true;
    case PAC_ALGO_BALLOT: return pac::ballot_supported(d);
    case PAC_ALGO_MFMA_I8:
    case PAC_ALGO_MFMA_GENERIC: return pac::mfma_supported(d);
    case PAC_ALGO_PARTITION: return pac::part_supported(d);
    case PAC_ALGO_REGISTER: return pac::reg_supported(d, ds.minmax != 0);
    default: return false;  // the approximate bf16 form is only ever chosen explicitly
  }
}

const pac_tune_entry *find_tuning(const pac_ctx *ctx, const pac::DevInput &d, const pac::DevState &ds) {
  if (ctx->tuning.empty()) return nullptr;
  pac_tune_entry k;
  tune_key(d, ds, &k);
  for (const pac_tune_entry &e : ctx->tuning)
    if (same_class(e, k) && algo_runs(e.algo, d, ds)) return &e;
  return nullptr;
}

uint32_t choose_algo(const pac::DevInput &d, const pac::DevState &ds) {
  // float columns or per-world MIN / MAX over a few groups: counters in registers
  if ((d.n_fcols > 0 || ds.minmax) && pac::reg_supported(d, ds.minmax != 0)) return PAC_ALGO_REGISTER;
  if (ds.minmax) return PAC_ALGO_PLAIN;  // MIN / MAX otherwise: the plain form
  // counters that do not fit in LDS (many groups, sparse keys): partition the rows by group
  if (!pac::plain_fits_lds(d) && pac::part_supported(d) && d.n_rows >= 4096) return PAC_ALGO_PARTITION;
  // float columns whose wave-private regions would leave fewer than four waves per workgroup
  if (d.n_fcols > 0 && !pac::plain_fits_lds4(d) && pac::part_supported(d) && d.n_rows >= 4096)
    return PAC_ALGO_PARTITION;
  if (d.group_keys || d.n_fcols > 0) return PAC_ALGO_PLAIN;
  int64_t bits = 1;
  for (int c = 0; c < d.n_icols; ++c) bits += d.icol_bits[c];
  const int64_t ballot_cost = d.n_groups * bits;  // popcounts per 64 rows
  if (pac::ballot_supported(d) && ballot_cost <= 24) return PAC_ALGO_BALLOT;
  if (pac::mfma_supported(d)) return PAC_ALGO_MFMA_I8;
  if (pac::ballot_supported(d) && ballot_cost <= 160) return PAC_ALGO_BALLOT;
  return PAC_ALGO_PLAIN;
}

// PAC_AGG_INIT: every state array cleared (fill kernels, no memset, so the
// work can be captured in a graph); the sparse table emptied.
int init_state(const pac::LaunchEnv &env, const pac::DevInput &d, const pac::DevState &ds) {
  const int64_t G = d.n_groups, m = d.m;
  pac::FillSegs f{};
  auto add = [&](void *p, int64_t n, int64_t bits) {
    f.p[f.count] = (int64_t *)p;
    f.n[f.count] = n;
    f.v[f.count] = bits;
    ++f.count;
  };
  auto dbits = [](double x) {
    int64_t b;
    std::memcpy(&b, &x, sizeof b);
    return b;
  };
  add(ds.count, G * m, 0);
  if (ds.isum) add(ds.isum, G * d.n_icols * m, 0);
  if (ds.fsum) add(ds.fsum, G * d.n_fcols * m, dbits(0.0));
  add(ds.nrows, G, 0);
  if (d.group_keys) add(ds.slot_keys, G, PAC_EMPTY_KEY);
  if (d.group_keys) add(ds.n_used, 1, 0);
  if (ds.minmax && d.n_icols > 0) add(ds.imin, G * d.n_icols * m, INT64_MAX);
  if (ds.minmax && d.n_icols > 0) add(ds.imax, G * d.n_icols * m, INT64_MIN);
  if (ds.minmax && d.n_fcols > 0) add(ds.fmin, G * d.n_fcols * m, dbits(INFINITY));
  if (ds.minmax && d.n_fcols > 0) add(ds.fmax, G * d.n_fcols * m, dbits(-INFINITY));
  const hipError_t e = pac::launch_fill_multi(env, f);  // one launch for every array
  if (e != hipSuccess) return hip_fail(e, "state init");
  return PAC_OK;
}

int run_one(pac_ctx *ctx, hipStream_t stream, const pac_agg_input *in, int m, uint64_t qk, uint32_t algo,
            uint32_t flags, pac_agg_state *st) {
  pac::DevInput d;
  pac::DevState ds;
  int rc = plan_input(in, m, qk, st, &d, &ds);
  if (rc != PAC_OK) return rc;
  pac::LaunchEnv env{stream, ctx->n_cu, ctx->d_status};
  const int64_t G = d.n_groups;
  if (flags & PAC_AGG_INIT) {
    rc = init_state(env, d, ds);
    if (rc != PAC_OK) return rc;
  }
  if (d.n_rows == 0) return PAC_OK;
  const pac_tune_entry *tuned = find_tuning(ctx, d, ds);
  if (algo == PAC_ALGO_AUTO) algo = tuned ? tuned->algo : choose_algo(d, ds);
  if (tuned && tuned->algo == algo) {  // the launch shape measured for this class and form
    env.blocks_per_cu = tuned->blocks_per_cu;
    env.scatter_wg_per_cu = tuned->scatter_wg_per_cu;
  }
  if (ds.minmax && algo != PAC_ALGO_PLAIN && algo != PAC_ALGO_REGISTER)
    return fail(PAC_ERR_UNSUPPORTED, "MIN/MAX counters need the plain or register form");
  hipError_t e = hipSuccess;
  switch (algo) {
    case PAC_ALGO_PLAIN: {
      const size_t need = pac::plain_scratch_bytes(env, d, ds.minmax != 0);
      if (need) {
        rc = ensure_scratch(ctx, need);
        if (rc != PAC_OK) return rc;
      }
      e = pac::launch_agg_plain(env, d, ds, ctx->scratch, ctx->scratch_bytes);
      break;
    }
    case PAC_ALGO_BALLOT:
      if (!pac::ballot_supported(d))
        return fail(PAC_ERR_UNSUPPORTED, "ballot form needs int columns, dense groups and LDS-sized counters");
      e = pac::launch_agg_ballot(env, d, ds);
      break;
    case PAC_ALGO_MFMA_I8:
    case PAC_ALGO_MFMA_GENERIC:
      if (!pac::mfma_supported(d))
        return fail(PAC_ERR_UNSUPPORTED, "int8 matrix-core form needs int columns, <= 254 dense groups and "
                                         "groups x (digits+1) within the tile");
      e = algo == PAC_ALGO_MFMA_I8 && pac::star_supported(d) ? pac::launch_agg_star(env, d, ds)
                                                              : pac::launch_agg_mfma(env, d, ds);
      break;
    case PAC_ALGO_PARTITION: {
      if (!pac::part_supported(d))
        return fail(PAC_ERR_UNSUPPORTED, "partitioned form needs < 2^31 rows and one group's counters within LDS");
      rc = ensure_scratch(ctx, pac::part_scratch_bytes(d));
      if (rc != PAC_OK) return rc;
      e = pac::launch_agg_part(env, d, ds, ctx->scratch, ctx->scratch_bytes, (flags & PAC_AGG_INIT) != 0);
      break;
    }
    case PAC_ALGO_REGISTER: {
      if (!pac::reg_supported(d, ds.minmax != 0))
        return fail(PAC_ERR_UNSUPPORTED, "register form needs at most 64 (or 32) dense groups and "
                                         "1-3 value columns (1-2 with MIN/MAX)");
      rc = ensure_scratch(ctx, pac::reg_scratch_bytes(d, ds.minmax != 0, ctx->n_cu));
      if (rc != PAC_OK) return rc;
      e = pac::launch_agg_reg(env, d, ds, ctx->scratch, ctx->scratch_bytes);
      break;
    }
    case PAC_ALGO_MFMA_BF16:
      if (!pac::fmma_supported(d, ds))
        return fail(PAC_ERR_UNSUPPORTED, "bf16 matrix-core form needs one float column, no int columns, no MIN/MAX "
                                         "and at most 64 dense groups");
      e = pac::launch_agg_fmma(env, d, ds);
      break;
    case PAC_ALGO_APPROX16:
      if (!pac::approx_supported(d, ds))
        return fail(PAC_ERR_UNSUPPORTED, "approximate SUM form needs int columns only (no float columns, no MIN/MAX)");
      e = pac::launch_agg_approx(env, d, ds);
      break;
    default:
      return fail(PAC_ERR_INVALID, "unknown algorithm %u", algo);
  }
  if (e == hipSuccess && d.group_keys) e = pac::launch_count_used(env, ds.slot_keys, G, ds.n_used);
  if (e != hipSuccess) return hip_fail(e, "aggregate launch");
  return PAC_OK;
}

}  // namespace

extern "C" {

const char *pac_last_error(void) { return g_err.c_str(); }

int pac_version(void) { return 1; }

int pac_stream_read(pac_ctx *ctx, void *stream, const void *buf, int64_t bytes, uint64_t *out) {
  if (!ctx || (bytes > 0 && (!buf || !out))) return fail(PAC_ERR_INVALID, "null context, buffer or output");
  if (bytes < 0 || (bytes & 15) || ((uintptr_t)buf & 15)) return fail(PAC_ERR_INVALID, "bytes must be a multiple of 16, buffer 16-byte aligned");
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const hipError_t e = pac::launch_stream_read(env, buf, bytes, out);
  return e == hipSuccess ? PAC_OK : hip_fail(e, "stream read launch");
}

int pac_stream_copy(pac_ctx *ctx, void *stream, const void *src, void *dst, int64_t bytes) {
  if (!ctx || (bytes > 0 && (!src || !dst))) return fail(PAC_ERR_INVALID, "null context or buffer");
  if (bytes < 0 || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15))
    return fail(PAC_ERR_INVALID, "bytes must be a multiple of 16, buffers 16-byte aligned");
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const hipError_t e = pac::launch_stream_copy(env, src, dst, bytes);
  return e == hipSuccess ? PAC_OK : hip_fail(e, "stream copy launch");
}

int pac_tune_key(const pac_agg_input *in, int m, const pac_agg_state *state, pac_tune_entry *key) {
  if (!in || !key) return fail(PAC_ERR_INVALID, "null input or key");
  pac::DevInput d;
  pac::DevState ds{};
  pac_agg_state probe{};
  const pac_agg_state *st = state;
  if (!st) {  // the class does not depend on the counter arrays, only on whether MIN/MAX is wanted
    probe.count = probe.nrows = (int64_t *)16;
    probe.isum = (int64_t *)16;
    probe.fsum = (double *)16;
    probe.slot_keys = probe.n_used = (int64_t *)16;
    st = &probe;
  }
  const int rc = plan_input(in, m, 0, st, &d, &ds);
  if (rc != PAC_OK) return rc;
  tune_key(d, ds, key);
  return PAC_OK;
}

int pac_set_tuning(pac_ctx *ctx, const pac_tune_entry *entries, int n) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  if (n < 0 || (n > 0 && !entries)) return fail(PAC_ERR_INVALID, "bad tuning table");
  for (int i = 0; i < n; ++i)
    if (entries[i].algo == PAC_ALGO_AUTO || entries[i].algo > PAC_ALGO_MFMA_BF16 || entries[i].blocks_per_cu < 0 ||
        entries[i].scatter_wg_per_cu < 0 || entries[i].scatter_wg_per_cu > 8)
      return fail(PAC_ERR_INVALID, "tuning entry %d: bad algo or launch shape", i);
  ctx->tuning.assign(entries, entries + n);
  return PAC_OK;
}

int pac_ctx_create(int hip_device, pac_ctx **out) {
  if (!out) return fail(PAC_ERR_INVALID, "out is null");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= n) return fail(PAC_ERR_INVALID, "device %d out of range (%d)", hip_device, n);
  DeviceGuard guard(hip_device);
  if (!guard.ok) return fail(PAC_ERR_HIP, "hipSetDevice(%d) failed", hip_device);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, hip_device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  void *noalloc = nullptr;
  const int rc = noalloc_address(hip_device, &noalloc);
  if (rc != PAC_OK) return rc;
  pac_ctx *ctx = new pac_ctx();
  ctx->device = hip_device;
  ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  ctx->noalloc = noalloc;
  e = hipMalloc((void **)&ctx->d_status, sizeof(uint32_t));
  if (e != hipSuccess) {
    delete ctx;
    return hip_fail(e, "status word allocation");
  }
  const uint32_t zero = 0;
  e = hipMemcpy(ctx->d_status, &zero, sizeof(zero), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(ctx->d_status);
    delete ctx;
    return hip_fail(e, "status word init");
  }
  *out = ctx;
  return PAC_OK;
}

int pac_ctx_destroy(pac_ctx *ctx) {
  if (!ctx) return PAC_OK;
  DeviceGuard guard(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->d_status) (void)hipFree(ctx->d_status);
  delete ctx;
  return PAC_OK;
}

int pac_ctx_reserve(pac_ctx *ctx, size_t bytes) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  DeviceGuard guard(ctx->device);
  return ensure_scratch(ctx, bytes);
}

int pac_check(pac_ctx *ctx, void *stream, uint32_t *status) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  DeviceGuard guard(ctx->device);
  // read and clear on the caller's stream only (other streams keep running)
  const hipStream_t st = (hipStream_t)stream;
  uint32_t s = 0;
  hipError_t e = hipMemcpyAsync(&s, ctx->d_status, sizeof(s), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->d_status, 0, sizeof(uint32_t), st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "status read");
  if (status) *status = s;
  if (s) return fail(PAC_ERR_DEVICE_STATUS, "device status bits 0x%x", s);
  return PAC_OK;
}

int pac_hash_mask(pac_ctx *ctx, void *stream, const int64_t *keys, int64_t n, uint64_t query_key, int m,
                  uint32_t flags, uint64_t *out_masks) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  if (m != 64 && m != 128) return fail(PAC_ERR_INVALID, "m must be 64 or 128 (got %d)", m);
  if (n < 0) return fail(PAC_ERR_INVALID, "n < 0");
  if (n == 0) return PAC_OK;
  if (!keys || !out_masks) return fail(PAC_ERR_INVALID, "null keys or out_masks");
  if (flags & ~PAC_HASH_BALANCED) return fail(PAC_ERR_INVALID, "unknown hash flags 0x%x", flags);
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  hipError_t e = pac::launch_hash(env, keys, n, query_key, m, (flags & PAC_HASH_BALANCED) != 0, out_masks);
  if (e != hipSuccess) return hip_fail(e, "hash launch");
  return PAC_OK;
}

int pac_group_aggregate(pac_ctx *ctx, void *stream, const pac_agg_input *in, int m, uint64_t query_key,
                        uint32_t algo, uint32_t flags, pac_agg_state *inout) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  if (flags & ~PAC_AGG_INIT) return fail(PAC_ERR_INVALID, "unknown aggregate flags 0x%x", flags);
  DeviceGuard guard(ctx->device);
  return run_one(ctx, (hipStream_t)stream, in, m, query_key, algo, flags, inout);
}

int pac_group_aggregate_batch(pac_ctx *ctx, void *stream, const pac_agg_input *in, const uint64_t *query_keys,
                              int n_queries, int m, uint32_t algo, uint32_t flags, pac_agg_state *states) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  if (n_queries < 0) return fail(PAC_ERR_INVALID, "n_queries < 0");
  if (n_queries > 0 && (!in || !query_keys || !states)) return fail(PAC_ERR_INVALID, "null batch arrays");
  if (flags & ~PAC_AGG_INIT) return fail(PAC_ERR_INVALID, "unknown aggregate flags 0x%x", flags);
  DeviceGuard guard(ctx->device);
  const hipStream_t st = (hipStream_t)stream;
  std::vector<char> shared(n_queries, 0);
  if (algo == PAC_ALGO_AUTO) {
    // validate every query first: nothing is enqueued for a batch with a bad query
    std::vector<pac::DevInput> d(n_queries);
    std::vector<pac::DevState> ds(n_queries);
    for (int q = 0; q < n_queries; ++q) {
      const int rc = plan_input(&in[q], m, query_keys[q], &states[q], &d[q], &ds[q]);
      if (rc != PAC_OK) {
        std::string msg = g_err;
        return fail(rc, "query %d: %s", q, msg.c_str());
      }
    }
    // greedy packing of the queries that can share a scan: same rows as the
    // pack's first query, counters within the LDS budget, at most
    // PAC_MAX_AGG_BATCH per launch
    pac::LaunchEnv env{st, ctx->n_cu, ctx->d_status};
    std::vector<int> pending;
    for (int q = 0; q < n_queries; ++q)
      if (d[q].n_rows > 0 && pac::batch_supported(d[q], ds[q])) pending.push_back(q);
    while (pending.size() >= 2) {
      std::vector<int> pack{pending[0]}, rest;
      size_t bytes = pac::batch_counter_bytes(d[pending[0]]);
      for (size_t i = 1; i < pending.size(); ++i) {
        const int q = pending[i];
        const size_t b = pac::batch_counter_bytes(d[q]);
        if ((int)pack.size() < PAC_MAX_AGG_BATCH && pac::batch_same_rows(d[pack[0]], d[q]) &&
            bytes + b <= pac::batch_lds_budget()) {
          pack.push_back(q);
          bytes += b;
        } else {
          rest.push_back(q);
        }
      }
      pending.swap(rest);
      if (pack.size() < 2) continue;  // alone: the single-query forms below
      pac::DevInput pin[PAC_MAX_AGG_BATCH];
      pac::DevState pst[PAC_MAX_AGG_BATCH];
      for (size_t i = 0; i < pack.size(); ++i) {
        const int q = pack[i];
        pin[i] = d[q];
        pst[i] = ds[q];
        if (flags & PAC_AGG_INIT) {
          const int rc = init_state(env, d[q], ds[q]);
          if (rc != PAC_OK) return rc;
        }
        shared[q] = 1;
      }
      const hipError_t e = pac::launch_agg_batch(env, pin, pst, (int)pack.size());
      if (e != hipSuccess) return hip_fail(e, "batched aggregate launch");
    }
  }
  for (int q = 0; q < n_queries; ++q) {
    if (shared[q]) continue;
    const int rc = run_one(ctx, st, &in[q], m, query_keys[q], algo, flags, &states[q]);
    if (rc != PAC_OK) {
      std::string msg = g_err;
      return fail(rc, "query %d: %s", q, msg.c_str());
    }
  }
  return PAC_OK;
}

int pac_world_values(pac_ctx *ctx, void *stream, const pac_agg_state *state, int m, int64_t n_groups, int n_int,
                     int n_float, int32_t kind, int32_t col, double *out) {
  if (!ctx || !state || !out) return fail(PAC_ERR_INVALID, "null context, state or output");
  if (m != 64 && m != 128) return fail(PAC_ERR_INVALID, "m must be 64 or 128 (got %d)", m);
  if (n_groups < 1 || n_int < 0 || n_float < 0) return fail(PAC_ERR_INVALID, "bad sizes");
  if (!state->count) return fail(PAC_ERR_INVALID, "state.count missing");
  const int32_t wv_flags = kind & ~0xFF;
  if (wv_flags & ~(PAC_WV_RELEASE | PAC_WV_SCALE2 | PAC_WV_AVG_TOTALCOUNT))
    return fail(PAC_ERR_INVALID, "unknown world-value flags 0x%x", (unsigned)wv_flags);
  if (wv_flags && !(wv_flags & PAC_WV_RELEASE))
    return fail(PAC_ERR_INVALID, "PAC_WV_SCALE2 / PAC_WV_AVG_TOTALCOUNT need PAC_WV_RELEASE");
  if ((wv_flags & PAC_WV_AVG_TOTALCOUNT) && !state->nrows) return fail(PAC_ERR_INVALID, "state.nrows missing");
  const int32_t full_kind = kind;
  kind &= 0xFF;
  const bool on_int = kind == PAC_CELL_SUM_I || kind == PAC_CELL_AVG_I || kind == PAC_CELL_MIN_I || kind == PAC_CELL_MAX_I;
  const bool on_float = kind == PAC_CELL_SUM_F || kind == PAC_CELL_AVG_F || kind == PAC_CELL_MIN_F || kind == PAC_CELL_MAX_F;
  if (kind != PAC_CELL_COUNT && !on_int && !on_float) return fail(PAC_ERR_INVALID, "bad kind %d", kind);
  if ((on_int && (col < 0 || col >= n_int)) || (on_float && (col < 0 || col >= n_float)))
    return fail(PAC_ERR_INVALID, "column %d out of range", col);
  const void *need = kind == PAC_CELL_SUM_I || kind == PAC_CELL_AVG_I ? (const void *)state->isum
                     : kind == PAC_CELL_SUM_F || kind == PAC_CELL_AVG_F ? (const void *)state->fsum
                     : kind == PAC_CELL_MIN_I ? (const void *)state->imin
                     : kind == PAC_CELL_MAX_I ? (const void *)state->imax
                     : kind == PAC_CELL_MIN_F ? (const void *)state->fmin
                     : kind == PAC_CELL_MAX_F ? (const void *)state->fmax : (const void *)state->count;
  if (!need) return fail(PAC_ERR_INVALID, "the state has no array for kind %d", kind);
  DeviceGuard guard(ctx->device);
  pac::DevState ds{state->count, state->isum, state->fsum, state->nrows, state->slot_keys, state->n_used,
                   state->imin,  state->imax, state->fmin, state->fmax,  0};
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const hipError_t e = pac::launch_world_values(env, ds, m, n_groups, n_int, n_float, full_kind, col, out);
  if (e != hipSuccess) return hip_fail(e, "world values launch");
  return PAC_OK;
}

int pac_select_cmp(pac_ctx *ctx, void *stream, const pac_agg_input *rows, int m, uint64_t query_key,
                   const double *world_values, int64_t n_wv_groups, int32_t op, double scale, double offset,
                   uint64_t *out_masks) {
  if (!ctx || !rows) return fail(PAC_ERR_INVALID, "null context or rows");
  if (op < PAC_SEL_LT || op > PAC_SEL_GE) return fail(PAC_ERR_INVALID, "bad comparison %d", op);
  if (rows->group_keys) return fail(PAC_ERR_INVALID, "pac_select_cmp takes dense groups only");
  if (rows->n_cols < 1) return fail(PAC_ERR_INVALID, "cols[0] (the compared value) is required");
  if (n_wv_groups != rows->n_groups) return fail(PAC_ERR_INVALID, "world value table has %lld groups, rows %lld",
                                                 (long long)n_wv_groups, (long long)rows->n_groups);
  if (rows->n_rows > 0 && (!world_values || !out_masks)) return fail(PAC_ERR_INVALID, "null world values or output");
  pac::DevInput d;
  int rc = plan_input(rows, m, query_key, nullptr, &d, nullptr);
  if (rc != PAC_OK) return rc;
  if (d.n_rows == 0) return PAC_OK;
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  // Table form: an int compared value with statistics of a small range, and a
  // table (groups x values) smaller than what the row-wise form reads.
  int64_t lo = 0;
  int32_t R = 0;
  uint64_t *table = nullptr;
  const int64_t kExactLim = (int64_t)1 << 52;  // integers the table kernel forms exactly as doubles
  if (rows->has_stats && is_int(rows->col_type[0]) && rows->col_min[0] > -kExactLim && rows->col_max[0] < kExactLim) {
    const __int128 range = (__int128)rows->col_max[0] - (__int128)rows->col_min[0] + 1;
    const __int128 entries = range * (__int128)d.n_groups;
    if (range >= 1 && range <= kSelTableMaxRange && entries <= (__int128)d.n_rows * 32 &&
        entries * 8 * d.W <= (__int128)kSelTableMaxBytes) {
      lo = rows->col_min[0];
      R = (int32_t)range;
      const int rc2 = ensure_scratch(ctx, (size_t)entries * 8 * (size_t)d.W);
      if (rc2 != PAC_OK) return rc2;
      table = (uint64_t *)ctx->scratch;
    }
  }
  const hipError_t e = pac::launch_select_table(env, d, world_values, op, scale, offset, lo, R, table, out_masks);
  if (e != hipSuccess) return hip_fail(e, "select launch");
  return PAC_OK;
}

int pac_filter(pac_ctx *ctx, void *stream, const double *world_values, int64_t n_groups, int m, int32_t op,
               double threshold, uint64_t noise_seed, uint8_t *keep, double *frac) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  if (m != 64 && m != 128) return fail(PAC_ERR_INVALID, "m must be 64 or 128 (got %d)", m);
  if (n_groups < 0) return fail(PAC_ERR_INVALID, "n_groups < 0");
  if (op < PAC_SEL_LT || op > PAC_SEL_GE) return fail(PAC_ERR_INVALID, "bad comparison %d", op);
  if (n_groups > 0 && (!world_values || !keep)) return fail(PAC_ERR_INVALID, "null world values or output");
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const hipError_t e = pac::launch_filter(env, world_values, n_groups, m, op, threshold, noise_seed, keep, frac);
  if (e != hipSuccess) return hip_fail(e, "filter launch");
  return PAC_OK;
}

int pac_key_index(pac_ctx *ctx, void *stream, const int64_t *keys, int64_t n_keys, const int64_t *fk, int64_t n,
                  int32_t *out_index) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  if (n_keys < 0 || n < 0) return fail(PAC_ERR_INVALID, "negative size");
  if (n_keys >= ((int64_t)1 << 31)) return fail(PAC_ERR_UNSUPPORTED, "more than 2^31 - 1 referenced rows");
  if ((n_keys > 0 && !keys) || (n > 0 && (!fk || !out_index))) return fail(PAC_ERR_INVALID, "null array");
  DeviceGuard guard(ctx->device);
  const int rc = ensure_scratch(ctx, pac::join_scratch_bytes(n_keys));
  if (rc != PAC_OK) return rc;
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const hipError_t e = pac::launch_key_index(env, keys, n_keys, fk, n, out_index, ctx->scratch);
  if (e != hipSuccess) return hip_fail(e, "key index launch");
  return PAC_OK;
}

}  // extern "C"

namespace {

// pac_finalize's argument checks; fills the kernel-side views.
int finalize_args(pac_ctx *ctx, const pac_agg_state *state, int m, int64_t n_groups, int n_int, int n_float,
                  const pac_cell *cells, int64_t n_cells, const pac_finalize_params *params, double *out_val,
                  uint8_t *out_is_null, uint32_t *out_flags, double *posterior, pac::DevState *ds,
                  pac::FinParams *fp) {
  if (!ctx || !state || !params) return fail(PAC_ERR_INVALID, "null context, state or params");
  if (m != 64 && m != 128) return fail(PAC_ERR_INVALID, "m must be 64 or 128 (got %d)", m);
  if (n_cells < 0 || n_int < 0 || n_float < 0 || n_groups < 1) return fail(PAC_ERR_INVALID, "bad sizes");
  if (!posterior) return fail(PAC_ERR_INVALID, "posterior buffer is required");
  if (!(params->mi_budget > 0.0)) return fail(PAC_ERR_INVALID, "mi_budget must be > 0");
  if (params->j_star >= m) return fail(PAC_ERR_INVALID, "j_star out of range");
  if (params->flags & ~31u) return fail(PAC_ERR_INVALID, "unknown finalize flags 0x%x", params->flags);
  if (n_cells > 0 && (!cells || !out_val || !out_is_null || !out_flags || !state->count || !state->nrows))
    return fail(PAC_ERR_INVALID, "null cell or output arrays");
  if (n_int > 0 && !state->isum) return fail(PAC_ERR_INVALID, "state.isum missing");
  if (n_float > 0 && !state->fsum) return fail(PAC_ERR_INVALID, "state.fsum missing");
  *ds = pac::DevState{state->count, state->isum, state->fsum, state->nrows, state->slot_keys, state->n_used,
                      state->imin,  state->imax, state->fmin, state->fmax,  0};
  *fp = pac::FinParams{params->mi_budget, params->noise_seed, params->j_star, params->flags, m, n_int, n_float,
                       n_cells, n_groups};
  return PAC_OK;
}

}  // namespace

extern "C" {

int pac_finalize(pac_ctx *ctx, void *stream, const pac_agg_state *state, int m, int64_t n_groups, int n_int,
                 int n_float, const pac_cell *cells, int64_t n_cells, const pac_finalize_params *params, double *out_val,
                 uint8_t *out_is_null, uint32_t *out_flags, double *posterior, double *out_y) {
  pac::DevState ds;
  pac::FinParams fp;
  int rc = finalize_args(ctx, state, m, n_groups, n_int, n_float, cells, n_cells, params, out_val, out_is_null,
                         out_flags, posterior, &ds, &fp);
  if (rc != PAC_OK) return rc;
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  rc = ensure_scratch(ctx, pac::finalize_scratch_bytes(m, n_cells));
  if (rc != PAC_OK) return rc;
  hipError_t e =
      pac::launch_finalize(env, ds, cells, fp, out_val, out_is_null, out_flags, posterior, out_y, ctx->scratch);
  if (e != hipSuccess) return hip_fail(e, "finalize launch");
  return PAC_OK;
}

int pac_finalize_batch(pac_ctx *ctx, void *stream, int m, const pac_release_job *jobs, int n_jobs) {
  if (!ctx) return fail(PAC_ERR_INVALID, "null context");
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(PAC_ERR_INVALID, "bad job array");
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  for (int j0 = 0; j0 < n_jobs; j0 += PAC_MAX_RELEASE_BATCH) {
    const int n = std::min(PAC_MAX_RELEASE_BATCH, n_jobs - j0);
    pac::ReleaseInput in[PAC_MAX_RELEASE_BATCH];
    int64_t ncells[PAC_MAX_RELEASE_BATCH];
    for (int i = 0; i < n; ++i) {
      const pac_release_job &jb = jobs[j0 + i];
      const int rc = finalize_args(ctx, &jb.state, m, jb.n_groups, jb.n_int, jb.n_float, jb.cells, jb.n_cells,
                                   &jb.params, jb.out_val, jb.out_is_null, jb.out_flags, jb.posterior, &in[i].st,
                                   &in[i].fp);
      if (rc != PAC_OK) {
        std::string msg = g_err;
        return fail(rc, "job %d: %s", j0 + i, msg.c_str());
      }
      in[i].cells = jb.cells;
      in[i].out_val = jb.out_val;
      in[i].out_null = jb.out_is_null;
      in[i].out_flags = jb.out_flags;
      in[i].post = jb.posterior;
      in[i].out_y = jb.out_y;
      ncells[i] = jb.n_cells;
    }
    const int rc = ensure_scratch(ctx, pac::finalize_batch_scratch_bytes(m, ncells, n));
    if (rc != PAC_OK) return rc;
    const hipError_t e = pac::launch_finalize_batch(env, m, in, n, ctx->scratch);
    if (e != hipSuccess) return hip_fail(e, "batched release launch");
  }
  return PAC_OK;
}

int pac_finalize_noalloc(pac_ctx *ctx, void *stream, const pac_agg_state *state, int m, int64_t n_groups, int n_int,
                         int n_float, const pac_cell *cells, int64_t n_cells, const pac_finalize_params *params,
                         double *out_val, uint8_t *out_is_null, uint32_t *out_flags, double *posterior,
                         double *out_y) {
  pac::DevState ds;
  pac::FinParams fp;
  int rc = finalize_args(ctx, state, m, n_groups, n_int, n_float, cells, n_cells, params, out_val, out_is_null,
                         out_flags, posterior, &ds, &fp);
  if (rc != PAC_OK) return rc;
  if (n_cells > PAC_NOALLOC_MAX_CELLS)
    return fail(PAC_ERR_INVALID, "pac_finalize_noalloc releases at most %d cells per call (got %lld)",
                PAC_NOALLOC_MAX_CELLS, (long long)n_cells);
  if (pac::finalize_scratch_bytes(m, n_cells) > kNoAllocBytes)
    return fail(PAC_ERR_INVALID, "pac_finalize_noalloc: %lld cells need more than the fixed %zu bytes",
                (long long)n_cells, kNoAllocBytes);
  if (!ctx->noalloc) return fail(PAC_ERR_INVALID, "context has no fixed working memory");
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const hipError_t e =
      pac::launch_finalize(env, ds, cells, fp, out_val, out_is_null, out_flags, posterior, out_y, ctx->noalloc);
  if (e != hipSuccess) return hip_fail(e, "finalize launch");
  return PAC_OK;
}

int pac_lift(pac_ctx *ctx, void *stream, const double *const *inputs, uint32_t scalar_inputs, int n_inputs,
             int64_t n_groups, int m, const pac_lift_op *program, int n_ops, double *out) {
  if (!ctx || !program) return fail(PAC_ERR_INVALID, "null context or program");
  if (m != 64 && m != 128) return fail(PAC_ERR_INVALID, "m must be 64 or 128 (got %d)", m);
  if (n_groups < 0) return fail(PAC_ERR_INVALID, "bad sizes");
  if (n_inputs < 0 || n_inputs > PAC_LIFT_MAX_INPUTS)
    return fail(PAC_ERR_INVALID, "n_inputs must be 0..%d (got %d)", PAC_LIFT_MAX_INPUTS, n_inputs);
  if (n_inputs > 0 && !inputs) return fail(PAC_ERR_INVALID, "null inputs");
  if (n_ops < 1 || n_ops > PAC_LIFT_MAX_OPS)
    return fail(PAC_ERR_INVALID, "n_ops must be 1..%d (got %d)", PAC_LIFT_MAX_OPS, n_ops);
  if (scalar_inputs >> n_inputs) return fail(PAC_ERR_INVALID, "scalar_inputs names a missing input");
  pac::LiftProg prog{};
  prog.scalar = scalar_inputs;
  prog.n_ops = n_ops;
  int depth = 0;
  for (int i = 0; i < n_ops; ++i) {
    const pac_lift_op &o = program[i];
    switch (o.op) {
      case PAC_LIFT_INPUT:
        if (o.arg < 0 || o.arg >= n_inputs) return fail(PAC_ERR_INVALID, "op %d reads missing input %d", i, o.arg);
        ++depth;
        break;
      case PAC_LIFT_CONST: ++depth; break;
      case PAC_LIFT_NEG:
        if (depth < 1) return fail(PAC_ERR_INVALID, "op %d pops an empty stack", i);
        break;
      case PAC_LIFT_ADD:
      case PAC_LIFT_SUB:
      case PAC_LIFT_MUL:
      case PAC_LIFT_DIV:
        if (depth < 2) return fail(PAC_ERR_INVALID, "op %d needs two values", i);
        --depth;
        break;
      default: return fail(PAC_ERR_INVALID, "op %d: unknown opcode %d", i, o.op);
    }
    if (depth > PAC_LIFT_MAX_DEPTH) return fail(PAC_ERR_INVALID, "op %d: stack deeper than %d", i, PAC_LIFT_MAX_DEPTH);
    prog.op[i] = (int8_t)o.op;
    prog.arg[i] = (int8_t)(o.op == PAC_LIFT_INPUT ? o.arg : 0);
    prog.val[i] = o.value;
  }
  if (depth != 1) return fail(PAC_ERR_INVALID, "the program leaves %d values (needs 1)", depth);
  if (n_groups == 0) return PAC_OK;
  if (!out) return fail(PAC_ERR_INVALID, "null output");
  for (int k = 0; k < n_inputs; ++k) {
    if (!inputs[k]) return fail(PAC_ERR_INVALID, "input %d is null", k);
    if (inputs[k] == out) return fail(PAC_ERR_INVALID, "input %d aliases the output", k);
    prog.in[k] = inputs[k];
  }
  DeviceGuard guard(ctx->device);
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const hipError_t e = pac::launch_lift(env, prog, n_groups, m, out);
  if (e != hipSuccess) return hip_fail(e, "lift launch");
  return PAC_OK;
}

int pac_noised(pac_ctx *ctx, void *stream, const double *world_values, const int64_t *cell_rows, int64_t n_cells,
               int m, int64_t first_cell, const pac_finalize_params *params, double *out_val, uint8_t *out_is_null,
               uint32_t *out_flags, double *posterior) {
  if (!ctx || !params) return fail(PAC_ERR_INVALID, "null context or params");
  if (m != 64 && m != 128) return fail(PAC_ERR_INVALID, "m must be 64 or 128 (got %d)", m);
  if (n_cells < 0 || first_cell < 0) return fail(PAC_ERR_INVALID, "bad sizes");
  if (!posterior) return fail(PAC_ERR_INVALID, "posterior buffer is required");
  if (!(params->mi_budget > 0.0)) return fail(PAC_ERR_INVALID, "mi_budget must be > 0");
  if (params->j_star >= m) return fail(PAC_ERR_INVALID, "j_star out of range");
  if (params->flags & ~31u) return fail(PAC_ERR_INVALID, "unknown finalize flags 0x%x", params->flags);
  if (params->flags & (PAC_FIN_SCALE2 | PAC_FIN_AVG_TOTALCOUNT))
    return fail(PAC_ERR_INVALID, "PAC_FIN_SCALE2 / PAC_FIN_AVG_TOTALCOUNT apply to pac_world_values, not pac_noised");
  if (n_cells > 0 && (!world_values || !out_val || !out_is_null || !out_flags))
    return fail(PAC_ERR_INVALID, "null world value or output arrays");
  DeviceGuard guard(ctx->device);
  pac::FinParams fp{params->mi_budget, params->noise_seed, params->j_star, params->flags, m, 0, 0, n_cells, 1};
  pac::LaunchEnv env{(hipStream_t)stream, ctx->n_cu, ctx->d_status};
  const int rc = ensure_scratch(ctx, pac::finalize_scratch_bytes(m, n_cells));
  if (rc != PAC_OK) return rc;
  const hipError_t e = pac::launch_noised(env, world_values, cell_rows, first_cell, fp, out_val, out_is_null, out_flags,
                                          posterior, ctx->scratch);
  if (e != hipSuccess) return hip_fail(e, "noised launch");
  return PAC_OK;
}

}  // extern "C"
