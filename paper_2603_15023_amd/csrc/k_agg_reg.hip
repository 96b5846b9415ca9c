// a2-a6 for a few dense groups, counters in registers: the plain per-bit
// form (lane = world, rows broadcast across the wavefront, predicated
// updates; Sec. 5 predication) with every counter of the query held in the
// lanes' registers instead of LDS.
//
// Used for float columns and for pac_min / pac_max (Sec. 4.2, agg in {sum,
// count, avg, min, max}) when the groups are few: S slots (8 at m = 64, 4 at
// m = 128) of  1 + 2 (ints + floats) (x3 with MIN/MAX)  registers per world.
// Wave w takes the rows of its contiguous range in order and, per 64-row
// batch, the records of each group in row order: its sums are in row order,
// and the ranges are merged in range order by the reduction kernel, so FP64
// results are the same on every run.  MIN / MAX are exact in any order.
#include <algorithm>

#include "pac_internal.h"

namespace pac {

constexpr int kRegWaves = 2048;  // row ranges of the one-wave form
constexpr int kRegShare = 8;     // wavefronts of the shared form (a workgroup per row range)

struct RegPlan {
  int S;                 // groups per wavefront (register slots)
  int P;                 // wavefronts sharing a row range: 1, or kRegShare (groups split over them)
  int64_t n_ranges;
  int64_t slot_words;    // A*m + 1 (+ 2 (ni + nf) m with MIN/MAX)
  size_t bytes;          // partials [n_ranges][S * P][slot_words]
};

// Column mixes with a compiled loop: up to two int and two float columns,
// at most three in all (two with MIN/MAX).
static bool reg_mix(int ni, int nf, bool mm) {
  return ni <= 2 && nf <= 2 && ni + nf >= 1 && ni + nf <= (mm ? 2 : 3);
}

// Register slots per wavefront: 8, or 4 when 8 would need more than 112
// registers (S x W x (1 + 2 (ni + nf)) (x3 for the columns with MIN/MAX)).
static int reg_slots(int W, int ni, int nf, bool mm) {
  const int per = W * (1 + 2 * (ni + nf) * (mm ? 3 : 1));
  return 8 * per <= 112 ? 8 : 4;
}

static bool reg_plan(const DevInput &in, bool mm, int n_cu, RegPlan *p) {
  if (in.group_keys || !reg_mix(in.n_icols, in.n_fcols, mm) || in.n_rows <= 0) return false;
  const int S = reg_slots(in.W, in.n_icols, in.n_fcols, mm);
  // Shared ranges only at m = 64: at m = 128 every record costs two words and
  // the partitioned form was measured faster (200M rows, 64 groups: 17 vs 19 ms).
  if (in.n_groups > (in.W == 1 ? (int64_t)S * kRegShare : (int64_t)S)) return false;
  p->S = S;
  p->P = in.n_groups <= S ? 1 : kRegShare;
  const int64_t n_chunks = (in.n_rows + 63) / 64;
  p->n_ranges = p->P == 1 ? std::max<int64_t>(1, std::min<int64_t>(kRegWaves, n_chunks))
                          : std::max<int64_t>(1, std::min<int64_t>((int64_t)2 * n_cu, (n_chunks + p->P - 1) / p->P));
  const int A = 1 + in.n_icols + in.n_fcols;
  p->slot_words = (int64_t)A * in.m + 1 + (mm ? (int64_t)2 * (in.n_icols + in.n_fcols) * in.m : 0);
  p->bytes = (size_t)p->n_ranges * S * p->P * p->slot_words * 8;
  return true;
}

bool reg_supported(const DevInput &in, bool minmax) {
  RegPlan p;
  return reg_plan(in, minmax, 256, &p);
}

size_t reg_scratch_bytes(const DevInput &in, bool minmax, int n_cu) {
  RegPlan p;
  return reg_plan(in, minmax, n_cu, &p) ? p.bytes : 0;
}

// One row of a 64-row batch: group (-1: past the end or skipped), PU words, values.
template <int W, int NI, int NF>
__device__ __forceinline__ int64_t reg_row(const DevInput &in, const DevState &st, int64_t r, uint32_t *status,
                                           uint64_t (&mk)[W], uint64_t (&iv)[NI > 0 ? NI : 1],
                                           uint64_t (&fv)[NF > 0 ? NF : 1]) {
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
      for (int k = 0; k < NI; ++k) iv[k] = (uint64_t)load_icol(in.icols[k], in.icol_type[k], r);
#pragma unroll
      for (int k = 0; k < NF; ++k) fv[k] = (uint64_t)__double_as_longlong(load_fcol(in.fcols[k], in.fcol_type[k], r));
    }
  }
  return g;
}

// Counters of S groups (g0 .. g0 + S - 1) of one wavefront, lane = world.
// Partial layout of one slot: count[m], isum[NI][m], fsum[NF][m], nrows,
// then with MIN/MAX imin[NI][m], imax[NI][m], fmin[NF][m], fmax[NF][m].
template <int W, int NI, int NF, int S, bool MM>
struct RegAcc {
  static constexpr int NIa = NI > 0 ? NI : 1, NFa = NF > 0 ? NF : 1;
  uint32_t cn[S][W], nr[S];
  uint64_t is[S][W][NIa];
  double fs[S][W][NFa];
  int64_t imn[S][W][NIa], imx[S][W][NIa];
  double fmn[S][W][NFa], fmx[S][W][NFa];

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      nr[s] = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        cn[s][w] = 0;
#pragma unroll
        for (int k = 0; k < NIa; ++k) {
          is[s][w][k] = 0;
          imn[s][w][k] = INT64_MAX;
          imx[s][w][k] = INT64_MIN;
        }
#pragma unroll
        for (int k = 0; k < NFa; ++k) {
          fs[s][w][k] = 0.0;
          fmn[s][w][k] = INFINITY;
          fmx[s][w][k] = -INFINITY;
        }
      }
    }
  }

  // Row rr of a batch held in the lanes' registers (broadcast by readlane).
  struct LaneRows {
    const uint64_t (&mk)[W];
    const uint64_t (&iv)[NIa];
    const uint64_t (&fv)[NFa];
    __device__ __forceinline__ uint64_t mask(int w, int rr) const { return readlane_u64(mk[w], rr); }
    __device__ __forceinline__ uint64_t ival(int k, int rr) const { return readlane_u64(iv[k], rr); }
    __device__ __forceinline__ uint64_t fval(int k, int rr) const { return readlane_u64(fv[k], rr); }
  };
  // Row rr of a batch staged in LDS as [W][64], [NIa][64] and [NFa][64]
  // (every lane reads the same address: a broadcast, no VALU work).
  struct LdsRows {
    const uint64_t *mk, *iv, *fv;
    __device__ __forceinline__ uint64_t mask(int w, int rr) const { return mk[w * 64 + rr]; }
    __device__ __forceinline__ uint64_t ival(int k, int rr) const { return iv[k * 64 + rr]; }
    __device__ __forceinline__ uint64_t fval(int k, int rr) const { return fv[k * 64 + rr]; }
  };

  __device__ __forceinline__ void batch(int64_t g, int64_t g0, int64_t G, const uint64_t (&mk)[W],
                                        const uint64_t (&iv)[NIa], const uint64_t (&fv)[NFa], int lane) {
    batch_rows(g, g0, G, LaneRows{mk, iv, fv}, lane);
  }

  // The batch's records of each of the S groups, in lane (row) order.
  template <class Rows>
  __device__ __forceinline__ void batch_rows(int64_t g, int64_t g0, int64_t G, const Rows &rows, int lane) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (g0 + s >= G) break;
      uint64_t todo = __ballot(g == g0 + s);
      nr[s] += (uint32_t)__popcll(todo);
      while (todo) {
        const int rr = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        uint64_t u[NIa];
        double v[NFa];
#pragma unroll
        for (int k = 0; k < NI; ++k) u[k] = rows.ival(k, rr);
#pragma unroll
        for (int k = 0; k < NF; ++k) v[k] = __longlong_as_double((long long)rows.fval(k, rr));
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const bool bit = (rows.mask(w, rr) >> lane) & 1ull;
          cn[s][w] += bit ? 1u : 0u;
#pragma unroll
          for (int k = 0; k < NI; ++k) {
            is[s][w][k] += bit ? u[k] : 0ull;
            if (MM) {
              const int64_t x = (int64_t)u[k];
              imn[s][w][k] = bit && x < imn[s][w][k] ? x : imn[s][w][k];
              imx[s][w][k] = bit && x > imx[s][w][k] ? x : imx[s][w][k];
            }
          }
#pragma unroll
          for (int k = 0; k < NF; ++k) {
            fs[s][w][k] = bit ? fs[s][w][k] + v[k] : fs[s][w][k];
            if (MM) {
              fmn[s][w][k] = bit && v[k] < fmn[s][w][k] ? v[k] : fmn[s][w][k];
              fmx[s][w][k] = bit && v[k] > fmx[s][w][k] ? v[k] : fmx[s][w][k];
            }
          }
        }
      }
    }
  }

  // Slots g0 .. g0 + S - 1 (those below G) of the range's partial.
  __device__ __forceinline__ void store(uint64_t *out, int64_t slot_words, int64_t g0, int64_t G, int lane) const {
    constexpr int m = 64 * W, A = 1 + NI + NF;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (g0 + s >= G) break;
      uint64_t *b = out + (g0 + s) * slot_words;
      const int64_t mo = (int64_t)A * m + 1;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int j = w * 64 + lane;
        b[j] = cn[s][w];
#pragma unroll
        for (int k = 0; k < NI; ++k) b[(int64_t)(1 + k) * m + j] = is[s][w][k];
#pragma unroll
        for (int k = 0; k < NF; ++k) b[(int64_t)(1 + NI + k) * m + j] = (uint64_t)__double_as_longlong(fs[s][w][k]);
        if (MM) {
#pragma unroll
          for (int k = 0; k < NI; ++k) {
            b[mo + (int64_t)k * m + j] = (uint64_t)imn[s][w][k];
            b[mo + (int64_t)(NI + k) * m + j] = (uint64_t)imx[s][w][k];
          }
#pragma unroll
          for (int k = 0; k < NF; ++k) {
            b[mo + (int64_t)(2 * NI + k) * m + j] = (uint64_t)__double_as_longlong(fmn[s][w][k]);
            b[mo + (int64_t)(2 * NI + NF + k) * m + j] = (uint64_t)__double_as_longlong(fmx[s][w][k]);
          }
        }
      }
      if (lane == 0) b[(int64_t)A * m] = nr[s];
    }
  }
};

// One wavefront per row range; the wave holds every group (G <= S).
template <int W, int NI, int NF, int S, bool MM>
__global__ __launch_bounds__(256) void agg_reg(DevInput in, DevState st, uint32_t *status, int64_t n_ranges,
                                               int64_t slot_words, uint64_t *partial) {
  using Acc = RegAcc<W, NI, NF, S, MM>;
  const int lane = threadIdx.x & 63;
  const int64_t range = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (range >= n_ranges) return;  // whole wavefronts; no workgroup barrier below
  const int64_t G = in.n_groups;
  const int64_t n_chunks = (in.n_rows + 63) >> 6, cpr = (n_chunks + n_ranges - 1) / n_ranges;
  const int64_t c0 = range * cpr, c1 = min(n_chunks, c0 + cpr);
  // Each wavefront stages its batch in its own LDS slice and walks the
  // records from there (broadcast reads), so only wavefront-level ordering
  // is needed.
  __shared__ uint64_t s_mk[4][W][64], s_iv[4][Acc::NIa][64], s_fv[4][Acc::NFa][64];
  const int wv = threadIdx.x >> 6;
  Acc acc;
  acc.init();
  for (int64_t c = c0; c < c1; ++c) {
    uint64_t mk[W], iv[Acc::NIa], fv[Acc::NFa];
    const int64_t g = reg_row<W, NI, NF>(in, st, c * 64 + lane, status, mk, iv, fv);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the previous batch's reads come first
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int w = 0; w < W; ++w) s_mk[wv][w][lane] = mk[w];
#pragma unroll
    for (int k = 0; k < NI; ++k) s_iv[wv][k][lane] = iv[k];
#pragma unroll
    for (int k = 0; k < NF; ++k) s_fv[wv][k][lane] = fv[k];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    acc.batch_rows(g, 0, G, typename Acc::LdsRows{&s_mk[wv][0][0], &s_iv[wv][0][0], &s_fv[wv][0][0]}, lane);
  }
  acc.store(partial + range * (slot_words * S), slot_words, 0, G, lane);
}

// kRegShare wavefronts per row range, wave w holding groups [w S, w S + S):
// each step the waves load kRegShare consecutive 64-row batches into LDS,
// then every wave walks all of them in row order for its own groups.
template <int W, int NI, int NF, int S, bool MM>
__global__ __launch_bounds__(64 * kRegShare) void agg_reg_shared(DevInput in, DevState st, uint32_t *status,
                                                                 int64_t n_ranges, int64_t slot_words,
                                                                 uint64_t *partial) {
  using Acc = RegAcc<W, NI, NF, S, MM>;
  constexpr int P = kRegShare;
  __shared__ int32_t s_g[P][64];
  __shared__ uint64_t s_mk[P][W][64], s_iv[P][Acc::NIa][64], s_fv[P][Acc::NFa][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t range = blockIdx.x;  // n_ranges == gridDim.x
  const int64_t G = in.n_groups, g0 = (int64_t)wave * S;
  const int64_t n_chunks = (in.n_rows + 63) >> 6, cpr = (n_chunks + n_ranges - 1) / n_ranges;
  const int64_t c0 = range * cpr, c1 = min(n_chunks, c0 + cpr);
  Acc acc;
  acc.init();
  for (int64_t step = c0; step < c1; step += P) {
    {
      const int64_t c = step + wave;  // this wave's batch of the step (rows past the range read as absent)
      uint64_t mk[W], iv[Acc::NIa], fv[Acc::NFa];
      const int64_t g = c < c1 ? reg_row<W, NI, NF>(in, st, c * 64 + lane, status, mk, iv, fv) : -1;
      s_g[wave][lane] = (int32_t)g;
#pragma unroll
      for (int w = 0; w < W; ++w) s_mk[wave][w][lane] = mk[w];
#pragma unroll
      for (int k = 0; k < NI; ++k) s_iv[wave][k][lane] = iv[k];
#pragma unroll
      for (int k = 0; k < NF; ++k) s_fv[wave][k][lane] = fv[k];
    }
    __syncthreads();
    for (int sub = 0; sub < P; ++sub) {  // the step's batches in row order
      const int64_t g = s_g[sub][lane];
      if (g0 < G) acc.batch_rows(g, g0, G, typename Acc::LdsRows{&s_mk[sub][0][0], &s_iv[sub][0][0], &s_fv[sub][0][0]}, lane);
    }
    __syncthreads();
  }
  if (g0 < G) acc.store(partial + range * (slot_words * S * P), slot_words, g0, G, lane);
}

// Fixed-order merge of the range partials into the state: workgroup b takes
// the words [64 b, 64 b + 64) of the partial layout; wave q combines ranges
// q, q + 4, ... in increasing order; the four wave results are combined in
// wave order and added into (min/max-ed into) the state.
__global__ __launch_bounds__(256) void reg_reduce(DevState st, int ni, int nf, int m, int64_t G, int64_t slot_words,
                                                  int64_t words, int64_t n_ranges, int mm, const uint64_t *partial) {
  __shared__ uint64_t acc[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = i < words && i / slot_words < G;
  const int64_t o = i % slot_words;
  const int A = 1 + ni + nf;
  const int64_t mo = (int64_t)A * m + 1;
  // kind of the word: 0 int sum, 1 float sum, 2 int min, 3 int max, 4 float min, 5 float max
  int kind = 0;
  int64_t arr = 0;  // column index within its array
  if (o < (int64_t)A * m) {
    const int a = (int)(o / m);
    kind = a > ni ? 1 : 0;
    arr = a == 0 ? -1 : (a <= ni ? a - 1 : a - 1 - ni);
  } else if (o == (int64_t)A * m) {
    kind = 0;
    arr = -2;  // nrows
  } else {
    const int64_t sec = (o - mo) / m;
    kind = sec < ni ? 2 : sec < 2 * ni ? 3 : sec < 2 * ni + nf ? 4 : 5;
    arr = sec < ni ? sec : sec < 2 * ni ? sec - ni : sec < 2 * ni + nf ? sec - 2 * ni : sec - 2 * ni - nf;
  }
  uint64_t vi = kind == 2 ? (uint64_t)INT64_MAX : kind == 3 ? (uint64_t)INT64_MIN : 0;
  double vf = kind == 4 ? INFINITY : kind == 5 ? -INFINITY : 0.0;
  if (ok) {
    for (int64_t k = wave; k < n_ranges; k += 4) {
      const uint64_t x = partial[k * words + i];
      switch (kind) {
        case 0: vi += x; break;
        case 1: vf += __longlong_as_double((long long)x); break;
        case 2: vi = (int64_t)x < (int64_t)vi ? x : vi; break;
        case 3: vi = (int64_t)x > (int64_t)vi ? x : vi; break;
        case 4: { const double y = __longlong_as_double((long long)x); vf = y < vf ? y : vf; } break;
        default: { const double y = __longlong_as_double((long long)x); vf = y > vf ? y : vf; } break;
      }
    }
  }
  acc[wave][lane] = (kind == 1 || kind >= 4) ? (uint64_t)__double_as_longlong(vf) : vi;
  __syncthreads();
  if (wave != 0 || !ok) return;
  const int64_t g = i / slot_words;
  const int j = (int)(o < (int64_t)A * m ? o % m : (o - mo) % m);  // the MIN/MAX words start at A*m + 1
  if (kind == 0 || kind == 2 || kind == 3) {
    int64_t v = (int64_t)acc[0][lane];
    for (int w = 1; w < 4; ++w) {
      const int64_t y = (int64_t)acc[w][lane];
      v = kind == 0 ? (int64_t)((uint64_t)v + (uint64_t)y) : kind == 2 ? (y < v ? y : v) : (y > v ? y : v);
    }
    int64_t *dst = arr == -2  ? &st.nrows[g]
                   : arr == -1 ? &st.count[g * m + j]
                   : kind == 0 ? &st.isum[(g * ni + arr) * m + j]
                   : kind == 2 ? &st.imin[(g * ni + arr) * m + j]
                               : &st.imax[(g * ni + arr) * m + j];
    *dst = kind == 0 ? (int64_t)((uint64_t)*dst + (uint64_t)v) : kind == 2 ? (v < *dst ? v : *dst) : (v > *dst ? v : *dst);
  } else {
    double v = __longlong_as_double((long long)acc[0][lane]);
    for (int w = 1; w < 4; ++w) {
      const double y = __longlong_as_double((long long)acc[w][lane]);
      v = kind == 1 ? v + y : kind == 4 ? (y < v ? y : v) : (y > v ? y : v);
    }
    double *dst = kind == 1 ? &st.fsum[(g * nf + arr) * m + j]
                  : kind == 4 ? &st.fmin[(g * nf + arr) * m + j]
                              : &st.fmax[(g * nf + arr) * m + j];
    *dst = kind == 1 ? *dst + v : kind == 4 ? (v < *dst ? v : *dst) : (v > *dst ? v : *dst);
  }
}

using RegFn = void (*)(DevInput, DevState, uint32_t *, int64_t, int64_t, uint64_t *);

template <int W, bool MM, bool SHARED, int S>
static RegFn reg_fn_s(int ni, int nf) {
#define PAC_REG_K(NI_, NF_) (SHARED ? agg_reg_shared<W, NI_, NF_, S, MM> : agg_reg<W, NI_, NF_, S, MM>)
  if (ni == 1 && nf == 0) return PAC_REG_K(1, 0);
  if (ni == 2 && nf == 0) return PAC_REG_K(2, 0);
  if (ni == 0 && nf == 1) return PAC_REG_K(0, 1);
  if (ni == 1 && nf == 1) return PAC_REG_K(1, 1);
  if (ni == 0 && nf == 2) return PAC_REG_K(0, 2);
  if constexpr (!MM) {  // three columns: without MIN/MAX only (registers)
    if (ni == 2 && nf == 1) return PAC_REG_K(2, 1);
    if (ni == 1 && nf == 2) return PAC_REG_K(1, 2);
  }
#undef PAC_REG_K
  return nullptr;
}

template <int W, bool MM, bool SHARED>
static RegFn reg_fn(int ni, int nf, int S) {
  return S == 8 ? reg_fn_s<W, MM, SHARED, 8>(ni, nf) : reg_fn_s<W, MM, SHARED, 4>(ni, nf);
}

template <int W>
static RegFn reg_fn_w(int ni, int nf, int S, bool mm, bool shared) {
  if (mm) return shared ? reg_fn<W, true, true>(ni, nf, S) : reg_fn<W, true, false>(ni, nf, S);
  return shared ? reg_fn<W, false, true>(ni, nf, S) : reg_fn<W, false, false>(ni, nf, S);
}

hipError_t launch_agg_reg(const LaunchEnv &env, const DevInput &in, const DevState &st, void *scratch,
                          size_t scratch_bytes) {
  if (in.n_rows <= 0) return hipSuccess;
  const bool mm = st.minmax != 0;
  RegPlan p;
  if (!reg_plan(in, mm, env.n_cu, &p) || scratch_bytes < p.bytes) return hipErrorInvalidValue;
  const bool shared = p.P > 1;
  const RegFn fn = in.W == 1 ? reg_fn_w<1>(in.n_icols, in.n_fcols, p.S, mm, shared)
                             : reg_fn_w<2>(in.n_icols, in.n_fcols, p.S, mm, shared);
  if (!fn) return hipErrorInvalidValue;
  uint64_t *partial = (uint64_t *)scratch;
  if (shared)
    hipLaunchKernelGGL(fn, dim3((unsigned)p.n_ranges), dim3(64 * kRegShare), 0, env.stream, in, st, env.status,
                       p.n_ranges, p.slot_words, partial);
  else
    hipLaunchKernelGGL(fn, dim3((unsigned)((p.n_ranges + 3) / 4)), dim3(256), 0, env.stream, in, st, env.status,
                       p.n_ranges, p.slot_words, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t words = p.slot_words * p.S * p.P;
  hipLaunchKernelGGL(reg_reduce, dim3((unsigned)((words + 63) / 64)), dim3(256), 0, env.stream, st, in.n_icols,
                     in.n_fcols, in.m, in.n_groups, p.slot_words, words, p.n_ranges, mm ? 1 : 0, partial);
  return hipGetLastError();
}

}  // namespace pac
