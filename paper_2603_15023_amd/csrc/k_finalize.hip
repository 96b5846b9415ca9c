// a7: release of the result cells (Sec. 4.1 noise function pac_noised,
// Sec. 3.2 NULLs, Sec. 5 Diversity Check, Sec. 2 adaptive composition).
//
// The posterior P over the m worlds changes after every released cell, so
// the chain over cells is sequential by definition.  Everything that does not
// depend on P runs first, in parallel, one wavefront per cell (phase 1): the
// world vector y of the cell (COUNT / SUM / AVG / MIN / MAX of the per-world
// counters, doubled for COUNT/SUM, a world without rows as 0 for AVG / MIN /
// MAX), the number of worlds that received a row, the
// diversity flag and the cell's random draws.  Phase 2 is one wavefront that
// streams those vectors in cell order (several cells in flight) and applies
// the noise rule and the Bayesian update with DPP wave reductions.
//
// Randomness is counter based (Philox4x32-10 keyed by the query's noise
// seed, counter = (cell, purpose)), so every draw depends only on the seed
// and the cell index, never on execution order.
#include <algorithm>

#include "pac_post.h"

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

enum { kDrawJStar = 0, kDrawNoise = 1, kDrawNull = 2, kDrawFilter = 3 };

__device__ __forceinline__ void draw2(uint64_t seed, int64_t index, uint32_t purpose, uint64_t *a, uint64_t *b) {
  uint32_t c[4] = {(uint32_t)index, (uint32_t)((uint64_t)index >> 32), purpose, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  *a = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
  *b = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
}

__device__ __forceinline__ double to_unit(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// Per-cell record written by phase 1 (besides the world vector).
struct CellMeta {
  double z;        // standard normal draw (Box-Muller)
  uint32_t flags;  // PAC_CELL_* decided in phase 1 (NULL, DIVERSITY)
  uint32_t bad;    // cell out of range: released as NULL, no update
};

constexpr int kCellChunk = 65536;

// Phase 1 for cell c0 + ci of one query: its world vector into ybuf[ci],
// its draws and flags into meta[ci].  One wavefront.
template <int W>
__device__ __forceinline__ void cell_vector(const DevState &st, const pac_cell *__restrict__ cells,
                                            const FinParams &fp, int64_t c0, int64_t ci, double *ybuf,
                                            CellMeta *meta, double *out_y, uint32_t *status, int lane) {
  constexpr int m = 64 * W;
  const int64_t c = c0 + ci;
  const pac_cell cell = cells[c];
  const int64_t g = cell.group;
  const bool ext_i = cell.kind == PAC_CELL_MIN_I || cell.kind == PAC_CELL_MAX_I;
  const bool ext_f = cell.kind == PAC_CELL_MIN_F || cell.kind == PAC_CELL_MAX_F;
  const int ncol = (cell.kind == PAC_CELL_SUM_I || cell.kind == PAC_CELL_AVG_I || ext_i) ? fp.n_int
                   : (cell.kind == PAC_CELL_SUM_F || cell.kind == PAC_CELL_AVG_F || ext_f) ? fp.n_float : 1;
  const int64_t *ext_ip = cell.kind == PAC_CELL_MIN_I ? st.imin : st.imax;
  const double *ext_fp = cell.kind == PAC_CELL_MIN_F ? st.fmin : st.fmax;
  if (g < 0 || g >= fp.n_groups || cell.kind < 0 || cell.kind > PAC_CELL_MAX_F ||
      (cell.kind != PAC_CELL_COUNT && (cell.col < 0 || cell.col >= ncol)) || (ext_i && !ext_ip) ||
      (ext_f && !ext_fp)) {
    if (lane == 0) {
      atomicOr(status, PAC_STATUS_BAD_GROUP);
      meta[ci] = CellMeta{0.0, PAC_CELL_NULL, 1u};
    }
#pragma unroll
    for (int w = 0; w < W; ++w) ybuf[ci * m + lane + 64 * w] = 0.0;
    return;
  }
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
      case PAC_CELL_MIN_I:
      case PAC_CELL_MAX_I: v = cnt > 0 ? (double)ext_ip[(g * fp.n_int + cell.col) * m + j] : 0.0; break;
      case PAC_CELL_MIN_F:
      case PAC_CELL_MAX_F: v = cnt > 0 ? ext_fp[(g * fp.n_float + cell.col) * m + j] : 0.0; break;
      default: v = st.fsum[(g * fp.n_float + cell.col) * m + j]; break;
    }
    if (ext_i || ext_f) {
      // the world's extreme as it is: no x2 scaling
    } else if (cell.kind == PAC_CELL_AVG_I || cell.kind == PAC_CELL_AVG_F) {
      if (fp.flags & PAC_FIN_AVG_TOTALCOUNT) {
        const double nr = (double)st.nrows[g];
        v = nr > 0.0 ? (2.0 * v) / nr : 0.0;
      } else {
        v = cnt > 0 ? v / (double)cnt : 0.0;
      }
    } else if (fp.flags & PAC_FIN_SCALE2) {
      v = 2.0 * v;
    }
    ybuf[ci * m + j] = v;
    if (out_y) out_y[c * m + j] = v;
  }
  if (lane == 0) {
    uint32_t flags = 0;
    if (st.nrows[g] >= 16 && pop <= (m == 64 ? 40 : 80)) {
      flags |= PAC_CELL_DIVERSITY;
      if (fp.flags & PAC_FIN_STRICT_DIVERSITY) atomicOr(status, PAC_STATUS_DIVERSITY);
    }
    uint64_t a, b;
    draw2(fp.seed, c, kDrawNull, &a, &b);
    const double p_null = (double)(m - pop) / (double)m;
    if (to_unit(a) < p_null) flags |= PAC_CELL_NULL;
    draw2(fp.seed, c, kDrawNoise, &a, &b);
    const double u1 = to_unit(a), u2 = to_unit(b);
    const double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
    meta[ci] = CellMeta{z, flags, 0u};
  }
}

template <int W>
__global__ __launch_bounds__(256) void cell_vectors_kernel(DevState st, const pac_cell *__restrict__ cells,
                                                           FinParams fp, int64_t c0, int64_t nc, double *ybuf,
                                                           CellMeta *meta, double *out_y, uint32_t *status) {
  const int64_t ci = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (ci >= nc) return;
  cell_vector<W>(st, cells, fp, c0, ci, ybuf, meta, out_y, status, threadIdx.x & 63);
}

// Phase 1 of pac_noised over given world vectors: as cell_vectors_kernel,
// with y read from the caller's [n_cells][m] vectors (a NaN world is NULL:
// not in K, 0 in y) and the draws of cell index first + c.
template <int W>
__global__ __launch_bounds__(256) void noised_vectors_kernel(const double *__restrict__ wv,
                                                             const int64_t *__restrict__ cell_rows, FinParams fp,
                                                             int64_t first, int64_t c0, int64_t nc, double *ybuf,
                                                             CellMeta *meta, uint32_t *status) {
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63;
  const int64_t ci = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (ci >= nc) return;
  const int64_t c = c0 + ci;
  int pop = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int j = lane + 64 * w;
    const double v = wv[c * m + j];
    const bool null = v != v;
    pop += __popcll(__ballot(!null));
    ybuf[ci * m + j] = null ? 0.0 : v;
  }
  if (lane == 0) {
    uint32_t flags = 0;
    if (cell_rows && cell_rows[c] >= 16 && pop <= (m == 64 ? 40 : 80)) {
      flags |= PAC_CELL_DIVERSITY;
      if (fp.flags & PAC_FIN_STRICT_DIVERSITY) atomicOr(status, PAC_STATUS_DIVERSITY);
    }
    uint64_t a, b;
    draw2(fp.seed, first + c, kDrawNull, &a, &b);
    const double p_null = (double)(m - pop) / (double)m;
    if (to_unit(a) < p_null) flags |= PAC_CELL_NULL;
    draw2(fp.seed, first + c, kDrawNoise, &a, &b);
    const double u1 = to_unit(a), u2 = to_unit(b);
    const double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
    meta[ci] = CellMeta{z, flags, 0u};
  }
}

// ---------------------------------------------------------------- wave reductions (fp64, DPP)
__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int rlo, rhi;
  switch (ctrl_sel) {
    case 0: rlo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false); rhi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false); break;  // xor 1
    case 1: rlo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false); rhi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false); break;  // xor 2
    case 2: rlo = __builtin_amdgcn_mov_dpp(lo, 0x124, 0xF, 0xF, false); rhi = __builtin_amdgcn_mov_dpp(hi, 0x124, 0xF, 0xF, false); break;  // row_ror 4
    default: rlo = __builtin_amdgcn_mov_dpp(lo, 0x128, 0xF, 0xF, false); rhi = __builtin_amdgcn_mov_dpp(hi, 0x128, 0xF, 0xF, false); break;  // row_ror 8
  }
  return __hiloint2double(rhi, rlo);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, the same value returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  v += dpp_f64(v, 2);
  v += dpp_f64(v, 3);  // every lane: sum of its row of 16
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Orders one wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Two sums over the 64 lanes at once (each in the order of wave_sum).
__device__ __forceinline__ void wave_sum2(double &a, double &b) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a += dpp_f64(a, k);
    b += dpp_f64(b, k);
  }
  a = (readlane_f64(a, 0) + readlane_f64(a, 16)) + (readlane_f64(a, 32) + readlane_f64(a, 48));
  b = (readlane_f64(b, 0) + readlane_f64(b, 16)) + (readlane_f64(b, 32) + readlane_f64(b, 48));
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64(v, 0));
  v = fmax(v, dpp_f64(v, 1));
  v = fmax(v, dpp_f64(v, 2));
  v = fmax(v, dpp_f64(v, 3));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// The world vectors reach the sequential phase through LDS, kChainChunk cells
// at a time and double-buffered: the next chunk's vectors are loaded into
// registers while the current chunk is released, and written to the other
// buffer after it, so the wave waits for memory once per chunk instead of once
// per cell.  Each cell's outcome stays in a register of lane (cell % 64) and a
// batch of 64 outcomes is stored at once.
constexpr int kChainChunk = 16;

template <int W>
__device__ __forceinline__ void chain_load(const double *ybuf, int64_t first, int64_t nc, int lane,
                                           double (&r)[kChainChunk][W]) {
  constexpr int m = 64 * W;
#pragma unroll
  for (int i = 0; i < kChainChunk; ++i) {
    const int64_t ci = min(first + i, nc - 1);  // clamped: every chunk issues the same loads
#pragma unroll
    for (int w = 0; w < W; ++w) r[i][w] = ybuf[ci * m + lane + 64 * w];
  }
}

// Phase 2 for cells c0 .. c0 + nc - 1 of one query (one wavefront; s_y is
// its LDS staging).  The posterior enters from `post` (the prior, or the
// previous chunk's result) unless this is the first chunk without a prior.
template <int W>
__device__ __forceinline__ void release_chain(const FinParams &fp, int64_t c0, int64_t nc, const double *ybuf,
                                              const CellMeta *meta, double *out_val, uint8_t *out_null,
                                              uint32_t *out_flags, double *post, int first_chunk,
                                              double (&s_y)[2][kChainChunk][64 * W]) {
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63;
  double P[W], L[W];
  const bool prior = (fp.flags & PAC_FIN_PRIOR_IN) || !first_chunk;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    P[w] = prior ? post[lane + 64 * w] : 1.0 / m;
    L[w] = log(P[w]);
  }
  int jstar = fp.j_star;
  if (jstar < 0) {
    uint64_t a, b;
    draw2(fp.seed, 0, kDrawJStar, &a, &b);
    jstar = (int)(a % (uint64_t)m);
  }
  const int js_w = jstar >> 6, js_l = jstar & 63;
  if (nc > 0) {
    double nxt[kChainChunk][W];
    chain_load<W>(ybuf, 0, nc, lane, nxt);
#pragma unroll
    for (int i = 0; i < kChainChunk; ++i)
#pragma unroll
      for (int w = 0; w < W; ++w) s_y[0][i][lane + 64 * w] = nxt[i][w];
    wave_lds_sync();
    // After a posterior update, the next cell's weighted mean sum_j P_j y_j
    // is reduced together with the normaliser (as sum_j e_j y_j / sum_j e_j),
    // which takes one of the four dependent wave reductions off that cell.
    double mu_next = 0.0;
    bool have_mu = false;
    // lane l holds z and the phase-1 flags of cell b + l of the current batch of 64
    double zc = meta[min((int64_t)lane, nc - 1)].z;
    uint32_t fc = meta[min((int64_t)lane, nc - 1)].flags;
    for (int64_t b = 0; b < nc; b += 64) {
      // next batch's draws and flags (clamped: the same loads every batch), in flight
      const int64_t mi = min(b + 64 + lane, nc - 1);
      const double zn = meta[mi].z;
      const uint32_t fn = meta[mi].flags;
      const int nbc = nc - b < 64 ? (int)(nc - b) : 64;
      double v_keep = 0.0;
      uint32_t f_keep = 0, n_keep = 0;
      for (int64_t cs = b; cs < b + nbc; cs += kChainChunk) {
        const int buf = (int)((cs / kChainChunk) & 1);
        chain_load<W>(ybuf, cs + kChainChunk, nc, lane, nxt);  // next chunk, in flight while this one runs
        const int nk = nc - cs < kChainChunk ? (int)(nc - cs) : kChainChunk;
        for (int i = 0; i < nk; ++i) {
          const int64_t ci = cs + i;
          const int kk = (int)(ci - b);
          double y[W];
#pragma unroll
          for (int w = 0; w < W; ++w) y[w] = s_y[buf][i][lane + 64 * w];
          uint32_t cflags = (uint32_t)__builtin_amdgcn_readlane((int)fc, kk);
          double val = 0.0;
          uint32_t is_null = 0;
          if (cflags & PAC_CELL_NULL) {
            is_null = 1;
            have_mu = false;
          } else {
            double mu = mu_next;
            if (!have_mu) {
              double pm = 0.0;
#pragma unroll
              for (int w = 0; w < W; ++w) pm += P[w] * y[w];
              mu = wave_sum(pm);
            }
            have_mu = false;
            double part = 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) part += P[w] * ((y[w] - mu) * (y[w] - mu));
            const double s2 = wave_sum(part);
            const double delta = s2 / (2.0 * fp.budget);
            const double ys = readlane_f64(y[js_w], js_l);
            if (!(delta > 0.0)) {
              val = ys;
              cflags |= PAC_CELL_ZERO_VARIANCE;
            } else {
              const double yrel = ys + sqrt(delta) * readlane_f64(zc, kk);
              val = yrel;
              if (!(fp.flags & PAC_FIN_FIXED_PRIOR)) {
                const bool fuse = i + 1 < nk;  // the next cell's vector is in this chunk's buffer
                double l[W];
                double mx = -INFINITY;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                  const double d = yrel - y[w];
                  l[w] = L[w] - (d * d) / (2.0 * delta);
                  mx = fmax(mx, l[w]);
                }
                mx = wave_max(mx);
                double e[W], se = 0.0, ey = 0.0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                  e[w] = exp(l[w] - mx);
                  se += e[w];
                  ey += fuse ? e[w] * s_y[buf][i + 1][lane + 64 * w] : 0.0;
                }
                wave_sum2(se, ey);
                // L keeps the log posterior up to a constant (shifted so that its maximum is 0): the
                // constant cancels when the next cell subtracts its own maximum, so no logarithm of the
                // normaliser is needed per cell
#pragma unroll
                for (int w = 0; w < W; ++w) {
                  P[w] = e[w] / se;
                  L[w] = P[w] > 0.0 ? l[w] - mx : -INFINITY;  // an underflowed world stays at zero
                }
                mu_next = ey / se;
                have_mu = fuse;
              }
            }
          }
          v_keep = lane == kk ? val : v_keep;
          f_keep = lane == kk ? cflags : f_keep;
          n_keep = lane == kk ? is_null : n_keep;
        }
#pragma unroll
        for (int i = 0; i < kChainChunk; ++i)
#pragma unroll
          for (int w = 0; w < W; ++w) s_y[buf ^ 1][i][lane + 64 * w] = nxt[i][w];
        wave_lds_sync();
      }
      if (lane < nbc) {  // the batch's outcomes
        const int64_t c = c0 + b + lane;
        out_val[c] = v_keep;
        out_null[c] = (uint8_t)n_keep;
        out_flags[c] = f_keep;
      }
      zc = zn;
      fc = fn;
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) post[lane + 64 * w] = P[w];
}

template <int W>
__global__ __launch_bounds__(64) void release_chain_kernel(FinParams fp, int64_t c0, int64_t nc, const double *ybuf,
                                                           const CellMeta *meta, double *out_val, uint8_t *out_null,
                                                           uint32_t *out_flags, double *post, int first_chunk) {
  __shared__ double s_y[2][kChainChunk][64 * W];
  release_chain<W>(fp, c0, nc, ybuf, meta, out_val, out_null, out_flags, post, first_chunk, s_y);
}

// ---------------------------------------------------------------- batched release
// Several queries' releases in one launch per phase: phase 1 has one grid row
// per query, phase 2 one wavefront (workgroup) per query, so the sequential
// chains of the batch run side by side on different CUs.  Each query's cells
// go through the same code as a single pac_finalize, in chunks of kCellChunk
// cells (round r covers cells [r kCellChunk, (r + 1) kCellChunk) of every
// query), so the results are the same bit for bit.
struct ReleaseJob {
  DevState st;
  const pac_cell *cells;
  FinParams fp;
  double *out_val;
  uint8_t *out_null;
  uint32_t *out_flags;
  double *post;
  double *out_y;
  int64_t buf_off;  // this query's chunk of world vectors: ybuf + buf_off (doubles)
  int64_t meta_off; // and of cell records: meta + meta_off
};

struct ReleaseBatch {
  int32_t n;
  ReleaseJob job[kMaxReleaseBatch];
};

template <int W>
__global__ __launch_bounds__(256) void cell_vectors_batch(ReleaseBatch b, int64_t c0, double *ybuf, CellMeta *meta,
                                                          uint32_t *status) {
  const ReleaseJob &jb = b.job[blockIdx.y];
  const int64_t nc = min((int64_t)kCellChunk, jb.fp.n_cells - c0);
  const int64_t ci = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (ci >= nc) return;
  cell_vector<W>(jb.st, jb.cells, jb.fp, c0, ci, ybuf + jb.buf_off, meta + jb.meta_off, jb.out_y, status,
                 threadIdx.x & 63);
}

template <int W>
__global__ __launch_bounds__(64) void release_chain_batch(ReleaseBatch b, int64_t c0, const double *ybuf,
                                                          const CellMeta *meta) {
  __shared__ double s_y[2][kChainChunk][64 * W];
  const ReleaseJob &jb = b.job[blockIdx.x];
  const int64_t nc = min((int64_t)kCellChunk, jb.fp.n_cells - c0);
  if (nc < 0 || (nc == 0 && c0 > 0)) return;  // this query's cells ended in an earlier round
  release_chain<W>(jb.fp, c0, nc, ybuf + jb.buf_off, meta + jb.meta_off, jb.out_val, jb.out_null, jb.out_flags,
                   jb.post, c0 == 0 ? 1 : 0, s_y);
}

// Probabilistic filter (Sec. 3.2): one wave per group; lane j tests world j
// (NaN: not true), the popcount of the ballot over m gives p_g, and the
// group's coin (Philox at counter (g, filter)) keeps it with probability p_g.
template <int W>
__global__ __launch_bounds__(256) void filter_kernel(const double *wv, int64_t G, int op, double threshold,
                                                     uint64_t seed, uint8_t *keep, double *frac) {
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (g >= G) return;
  int n_true = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const double y = wv[g * m + 64 * w + lane];
    bool p;
    switch (op) {
      case PAC_SEL_LT: p = y < threshold; break;
      case PAC_SEL_LE: p = y <= threshold; break;
      case PAC_SEL_EQ: p = y == threshold; break;
      case PAC_SEL_NE: p = y != threshold; break;
      case PAC_SEL_GT: p = y > threshold; break;
      default: p = y >= threshold; break;
    }
    n_true += __popcll(__ballot(p && y == y));
  }
  if (lane == 0) {
    const double pg = (double)n_true / (double)m;
    uint64_t a, b;
    draw2(seed, g, kDrawFilter, &a, &b);
    keep[g] = to_unit(a) < pg ? 1 : 0;
    if (frac) frac[g] = pg;
  }
}

hipError_t launch_filter(const LaunchEnv &env, const double *wv, int64_t G, int m, int op, double threshold,
                         uint64_t seed, uint8_t *keep, double *frac) {
  if (G <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((G + 3) / 4);
  if (m == 64)
    hipLaunchKernelGGL(filter_kernel<1>, dim3(blocks), dim3(256), 0, env.stream, wv, G, op, threshold, seed, keep,
                       frac);
  else
    hipLaunchKernelGGL(filter_kernel<2>, dim3(blocks), dim3(256), 0, env.stream, wv, G, op, threshold, seed, keep,
                       frac);
  return hipGetLastError();
}

size_t finalize_scratch_bytes(int m, int64_t n_cells) {
  const int64_t chunk = n_cells < kCellChunk ? n_cells : kCellChunk;
  return (size_t)chunk * (m * sizeof(double) + sizeof(CellMeta)) + 256;
}

hipError_t launch_finalize(const LaunchEnv &env, const DevState &st, const pac_cell *cells, const FinParams &fp,
                           double *out_val, uint8_t *out_is_null, uint32_t *out_flags, double *posterior,
                           double *out_y, void *scratch) {
  const int m = fp.m;
  const int64_t chunk = fp.n_cells < kCellChunk ? fp.n_cells : kCellChunk;
  double *ybuf = (double *)scratch;
  CellMeta *meta = (CellMeta *)(((uintptr_t)(ybuf + chunk * m) + 255) & ~(uintptr_t)255);
  if (fp.n_cells == 0) {  // posterior out = prior (or uniform)
    hipLaunchKernelGGL(fp.m == 64 ? release_chain_kernel<1> : release_chain_kernel<2>, dim3(1), dim3(64), 0,
                       env.stream, fp, (int64_t)0, (int64_t)0, ybuf, meta, out_val, out_is_null, out_flags, posterior,
                       1);
    return hipGetLastError();
  }
  for (int64_t c0 = 0; c0 < fp.n_cells; c0 += chunk) {
    const int64_t nc = fp.n_cells - c0 < chunk ? fp.n_cells - c0 : chunk;
    const int blocks = (int)((nc + 3) / 4);
    if (m == 64)
      hipLaunchKernelGGL(cell_vectors_kernel<1>, dim3(blocks), dim3(256), 0, env.stream, st, cells, fp, c0, nc, ybuf,
                         meta, out_y, env.status);
    else
      hipLaunchKernelGGL(cell_vectors_kernel<2>, dim3(blocks), dim3(256), 0, env.stream, st, cells, fp, c0, nc, ybuf,
                         meta, out_y, env.status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m == 64)
      hipLaunchKernelGGL(release_chain_kernel<1>, dim3(1), dim3(64), 0, env.stream, fp, c0, nc, ybuf, meta, out_val,
                         out_is_null, out_flags, posterior, c0 == 0 ? 1 : 0);
    else
      hipLaunchKernelGGL(release_chain_kernel<2>, dim3(1), dim3(64), 0, env.stream, fp, c0, nc, ybuf, meta, out_val,
                         out_is_null, out_flags, posterior, c0 == 0 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t finalize_batch_scratch_bytes(int m, const int64_t *n_cells, int n) {
  size_t total = 0;
  for (int i = 0; i < n; ++i) total += finalize_scratch_bytes(m, n_cells[i]) + 256;
  return total;
}

hipError_t launch_finalize_batch(const LaunchEnv &env, int m, const ReleaseInput *in, int n, void *scratch) {
  if (n <= 0) return hipSuccess;
  if (n > kMaxReleaseBatch) return hipErrorInvalidValue;
  ReleaseBatch b{};
  b.n = n;
  int64_t max_cells = 0, ybuf_total = 0, meta_total = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t chunk = in[i].fp.n_cells < kCellChunk ? in[i].fp.n_cells : kCellChunk;
    b.job[i] = ReleaseJob{in[i].st,   in[i].cells,     in[i].fp,   in[i].out_val, in[i].out_null,
                          in[i].out_flags, in[i].post, in[i].out_y, ybuf_total, meta_total};
    ybuf_total += chunk * m;
    meta_total += chunk;
    max_cells = std::max(max_cells, in[i].fp.n_cells);
  }
  double *ybuf = (double *)scratch;
  CellMeta *meta = (CellMeta *)(((uintptr_t)(ybuf + ybuf_total) + 255) & ~(uintptr_t)255);
  const int64_t rounds = max_cells == 0 ? 1 : (max_cells + kCellChunk - 1) / kCellChunk;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t c0 = r * kCellChunk;
    const int64_t nc = std::min<int64_t>(kCellChunk, max_cells - c0);
    if (nc > 0) {
      const dim3 grid((unsigned)((nc + 3) / 4), (unsigned)n);
      if (m == 64)
        hipLaunchKernelGGL(cell_vectors_batch<1>, grid, dim3(256), 0, env.stream, b, c0, ybuf, meta, env.status);
      else
        hipLaunchKernelGGL(cell_vectors_batch<2>, grid, dim3(256), 0, env.stream, b, c0, ybuf, meta, env.status);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (m == 64)
      hipLaunchKernelGGL(release_chain_batch<1>, dim3((unsigned)n), dim3(64), 0, env.stream, b, c0, ybuf, meta);
    else
      hipLaunchKernelGGL(release_chain_batch<2>, dim3((unsigned)n), dim3(64), 0, env.stream, b, c0, ybuf, meta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_noised(const LaunchEnv &env, const double *wv, const int64_t *cell_rows, int64_t first_cell,
                         const FinParams &fp, double *out_val, uint8_t *out_is_null, uint32_t *out_flags,
                         double *posterior, void *scratch) {
  const int m = fp.m;
  const int64_t chunk = fp.n_cells < kCellChunk ? fp.n_cells : kCellChunk;
  double *ybuf = (double *)scratch;
  CellMeta *meta = (CellMeta *)(((uintptr_t)(ybuf + chunk * m) + 255) & ~(uintptr_t)255);
  if (fp.n_cells == 0) {  // posterior out = prior (or uniform)
    hipLaunchKernelGGL(m == 64 ? release_chain_kernel<1> : release_chain_kernel<2>, dim3(1), dim3(64), 0, env.stream,
                       fp, (int64_t)0, (int64_t)0, ybuf, meta, out_val, out_is_null, out_flags, posterior, 1);
    return hipGetLastError();
  }
  for (int64_t c0 = 0; c0 < fp.n_cells; c0 += chunk) {
    const int64_t nc = fp.n_cells - c0 < chunk ? fp.n_cells - c0 : chunk;
    const int blocks = (int)((nc + 3) / 4);
    hipLaunchKernelGGL(m == 64 ? noised_vectors_kernel<1> : noised_vectors_kernel<2>, dim3(blocks), dim3(256), 0,
                       env.stream, wv, cell_rows, fp, first_cell, c0, nc, ybuf, meta, env.status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(m == 64 ? release_chain_kernel<1> : release_chain_kernel<2>, dim3(1), dim3(64), 0, env.stream,
                       fp, c0, nc, ybuf, meta, out_val, out_is_null, out_flags, posterior, c0 == 0 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace pac
