// a6 for many groups: radix partitioning by group slot, then aggregation of
// each partition in LDS.
//
// When the per-world counters of all groups do not fit in LDS (hundreds of
// groups and up: a report grouped by a high-cardinality column, or sparse
// group keys kept in the HBM open-addressing table), updating them with
// global atomics costs one atomic per (row, world, counter).  Instead:
//   1. route:     row -> group slot (dense id, or table slot after insert),
//                 count the rows of every partition of 2^SB consecutive slots;
//   2. scan:      partition offsets and work items (a partition's rows in
//                 chunks, so a heavy group -- Zipf head -- is split over many
//                 workgroups);
//   3. scatter:   each live row's PU words and values go to its partition as
//                 a compact record (structure of arrays).  With many
//                 partitions (integer columns) this takes two passes: rows to
//                 about sqrt(partitions) coarse buckets, then each bucket's
//                 records to its fine partitions -- a workgroup then writes
//                 into few partitions at a time, so its partly written lines
//                 stay in L2 instead of going out one record at a time;
//   4. aggregate: a workgroup takes work items from a queue, accumulates the
//                 records into LDS counters [2^SB slots][A][m] (lane = world,
//                 records broadcast, LDS atomics), then adds the non-zero
//                 counters to the global state.
// Counter semantics are those of every other form (per-world COUNT, exact
// int64 SUM, FP64 SUM, row count per group).  Integer counters are exact in
// any order, so without float columns a partition is split into chunks and
// merged with atomics.  With float columns the form is deterministic: records
// reach their partition in row order (per-wave counts, no atomic cursors),
// each work item's waves sum fixed quarters of its records into private LDS
// regions combined in wave order, and the items of a partition are added in
// item order by one thread per counter word.
#include <algorithm>
#include <initializer_list>

#include "pac_internal.h"

namespace pac {

struct PartItem {
  int64_t part;
  int64_t begin;
  int64_t end;
  int64_t exclusive;  // 1: the partition's only work item (its workgroup owns the partition's counters)
};

struct PartPlan {
  bool det;             // float columns: fixed summation order
  int SB;               // log2 of the slots of a partition
  int64_t n_slots;      // dense groups, or the table capacity
  int64_t n_parts;
  int64_t cap;          // record capacity (= rows)
  int64_t slot_words;   // A * m + 1 (the last word counts rows)
  int lds_bytes;
  int64_t chunk;        // records per work item
  int64_t max_items;
  int64_t n_waves;      // deterministic routing: waves, each with a fixed contiguous row range
  size_t off_mat;       // deterministic routing: per-wave partition counts [n_waves][n_parts]
  size_t off_partial;   // deterministic: each work item's counters [max_items][2^SB * slot_words]
  size_t off_pfirst;    // deterministic: first work item and item count of each partition
  size_t off_row_slot, off_count, off_off, off_cur, off_items, off_meta, off_rec_slot, off_rec_mk, off_rec_iv,
      off_rec_fv, total;
  // two-pass scatter (S2 > 0): 2^S2 fine partitions per coarse bucket
  int S2;
  int64_t n_coarse, chunk2, max_items2;
  size_t off_ccount, off_coff, off_ccur, off_items2, off_meta2, off_tmp_slot, off_tmp_mk, off_tmp_iv;
};

// Above this many partitions the integer form scatters in two passes.
constexpr int64_t kTwoPassParts = 1024;

constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr int kPartLdsTarget = 80 * 1024;  // two workgroups per CU
// Deterministic form: four workgroups per CU (its per-record loop is latency bound).
constexpr int kPartLdsTargetDet = 40 * 1024;
constexpr int kPartWaves = 4;              // waves per workgroup of the aggregation (deterministic form)
constexpr int kPartWavesNd = 16;  // waves sharing one item's LDS counters (integer form)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Deterministic form, column mixes whose per-record loop keeps the counters in
// registers: slots per partition (0: the LDS loop).  Must agree with agg_det_fn.
static int det_reg_slots(const DevInput &in) {
  const int ni = in.n_icols, nf = in.n_fcols;
  const bool mix = (nf == 1 && ni <= 2) || (nf == 2 && ni == 0);
  return mix ? (in.W == 1 ? 8 : 4) : 0;
}

// Static LDS of the register-counter kernel beside its dynamic counters: the
// per-wave record staging s_rec[kPartWaves][W + max(CI,1) + max(CF,1)][64] and s_item.
static int64_t det_reg_static_lds(const DevInput &in) {
  return (int64_t)kPartWaves * (in.W + std::max(in.n_icols, 1) + std::max(in.n_fcols, 1)) * 64 * 8 + 8;
}

static bool part_plan(const DevInput &in, PartPlan *pl) {
  PartPlan p{};
  p.n_slots = in.n_groups;
  if (in.n_rows <= 0 || in.n_rows >= ((int64_t)1 << 31) || p.n_slots >= (int64_t)kNoSlot) return false;
  const int A = 1 + in.n_icols + in.n_fcols;
  p.slot_words = (int64_t)A * in.m + 1;
  p.det = in.n_fcols > 0;
  const int regions = p.det ? kPartWaves : 1;  // deterministic: one private region per wave
  const int64_t per_slot = p.slot_words * 8 * regions;
  const int64_t target = p.det ? kPartLdsTargetDet : kPartLdsTarget;
  if (per_slot > target) return false;
  int64_t slots = target / per_slot;
  int SB = 0;
  while (((int64_t)2 << SB) <= slots) ++SB;
  if (p.det && det_reg_slots(in)) {
    SB = det_reg_slots(in) == 8 ? 3 : 2;
    if (((int64_t)1 << SB) * per_slot + det_reg_static_lds(in) > 160 * 1024) return false;
  }
  p.SB = SB;
  p.lds_bytes = (int)(((int64_t)1 << SB) * per_slot);
  p.n_parts = (p.n_slots + ((int64_t)1 << SB) - 1) >> SB;
  p.cap = in.n_rows;
  p.chunk = p.det ? 65536 : 16384;  // deterministic: fewer items, a shorter ordered merge
  p.max_items = p.n_parts + p.cap / p.chunk + 1;
  if (p.det) {  // records land in row order: per-wave counts instead of atomic cursors
    const int64_t n_chunks = (in.n_rows + 63) / 64;
    p.n_waves = std::max<int64_t>(1, std::min<int64_t>({(int64_t)32768, n_chunks, ((int64_t)16 << 20) / p.n_parts}));
  }
  size_t o = 0;
  p.off_mat = o;
  if (p.det) o = align256(o + 4 * (size_t)p.n_waves * p.n_parts);
  p.off_partial = o;
  if (p.det) o = align256(o + 8 * (size_t)p.max_items * ((size_t)p.slot_words << p.SB));
  p.off_pfirst = o;
  if (p.det) o = align256(o + 16 * (size_t)p.n_parts);
  p.off_row_slot = o; o = align256(o + 4 * (size_t)p.cap);
  p.off_count = o;    o = align256(o + 4 * (size_t)p.n_parts);
  p.off_off = o;      o = align256(o + 8 * (size_t)(p.n_parts + 1));
  p.off_cur = o;      o = align256(o + 4 * (size_t)p.n_parts);
  p.off_items = o;    o = align256(o + sizeof(PartItem) * (size_t)p.max_items);
  p.off_meta = o;     o = align256(o + 2 * sizeof(int64_t));  // [0] items, [1] queue head
  p.off_rec_slot = o; o = align256(o + 4 * (size_t)p.cap);
  p.off_rec_mk = o;   o = align256(o + 8 * (size_t)in.W * p.cap);
  p.off_rec_iv = o;   o = align256(o + 8 * (size_t)in.n_icols * p.cap);
  p.off_rec_fv = o;   o = align256(o + 8 * (size_t)in.n_fcols * p.cap);
  if (!p.det && p.n_parts > kTwoPassParts && p.n_parts <= (int64_t)256 * 256) {
    int bits = 0;
    while (((int64_t)1 << bits) < p.n_parts) ++bits;
    p.S2 = std::min(8, (bits + 1) / 2);  // both passes write into about sqrt(n_parts) <= 256 partitions
    p.n_coarse = (p.n_parts + ((int64_t)1 << p.S2) - 1) >> p.S2;
    p.chunk2 = 65536;
    p.max_items2 = p.n_coarse + p.cap / p.chunk2 + 1;
    p.off_ccount = o;   o = align256(o + 4 * (size_t)p.n_coarse);
    p.off_coff = o;     o = align256(o + 8 * (size_t)(p.n_coarse + 1));
    p.off_ccur = o;     o = align256(o + 4 * (size_t)p.n_coarse);
    p.off_items2 = o;   o = align256(o + sizeof(PartItem) * (size_t)p.max_items2);
    p.off_meta2 = o;    o = align256(o + 2 * sizeof(int64_t));
    p.off_tmp_slot = o; o = align256(o + 4 * (size_t)p.cap);
    p.off_tmp_mk = o;   o = align256(o + 8 * (size_t)in.W * p.cap);
    p.off_tmp_iv = o;   o = align256(o + 8 * (size_t)in.n_icols * p.cap);
  }
  p.total = o;
  *pl = p;
  return true;
}

bool part_supported(const DevInput &in) {
  PartPlan p;
  return part_plan(in, &p);
}

size_t part_scratch_bytes(const DevInput &in) {
  PartPlan p;
  return part_plan(in, &p) ? p.total : 0;
}

// Each distinct key among the active lanes: leader gets the lanes sharing it.
__device__ __forceinline__ uint64_t lanes_lt(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// 1. route and count
__global__ __launch_bounds__(256) void part_route(DevInput in, DevState st, uint32_t *status, uint32_t *row_slot,
                                                  uint32_t *count, int SB) {
  const int lane = threadIdx.x & 63;
  const int64_t n_chunks = (in.n_rows + 63) >> 6;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < n_chunks; c += waves) {
    const int64_t r = c * 64 + lane;
    int64_t g = -1;
    if (r < in.n_rows) {
      g = row_group(in, st, r, status);
      int64_t idx;
      if (g >= 0 && !chain_index(in, r, &idx, status)) g = -1;
      row_slot[r] = g >= 0 ? (uint32_t)g : kNoSlot;
    }
    const uint32_t part = g >= 0 ? (uint32_t)(g >> SB) : kNoSlot;
    uint64_t todo = __ballot(g >= 0);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const uint32_t p0 = __builtin_amdgcn_readlane(part, leader);
      const uint64_t same = __ballot(part == p0) & todo;
      if (lane == leader) atomicAdd(&count[p0], (uint32_t)__popcll(same));
      todo &= ~same;
    }
  }
}

// At most 64 partitions: the lanes holding a record of this lane's partition
// (`same`), and the number of records of partition `lane` in the batch, from
// six ballots of the partition id's bits instead of a loop over the
// partitions present.
__device__ __forceinline__ void part_masks64(bool valid, uint32_t part, int lane, uint64_t *same,
                                             uint32_t *n_of_lane) {
  const uint32_t pv = valid ? part : 0u;
  const uint64_t vm = __ballot(valid);
  uint64_t sm = vm, mine = vm;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const uint64_t b = __ballot(valid && ((pv >> k) & 1u));
    sm &= ((pv >> k) & 1u) ? b : ~b;
    mine &= ((lane >> k) & 1) ? b : ~b;
  }
  *same = sm;
  *n_of_lane = (uint32_t)__popcll(mine);
}

// 1'. deterministic routing: wave w takes the contiguous chunks [w*cpw, (w+1)*cpw)
// in order and counts its rows per partition in its own entry mat[part][w].
__global__ __launch_bounds__(256) void part_route_det(DevInput in, DevState st, uint32_t *status,
                                                      uint32_t *row_slot, uint32_t *mat, int64_t n_parts, int SB,
                                                      int64_t n_waves) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= n_waves) return;
  const int64_t n_chunks = (in.n_rows + 63) >> 6, cpw = (n_chunks + n_waves - 1) / n_waves;
  const bool few = n_parts <= 64;  // lane p counts partition p in a register
  uint32_t cnt = 0;
  for (int64_t c = w * cpw; c < min(n_chunks, (w + 1) * cpw); ++c) {
    const int64_t r = c * 64 + lane;
    int64_t g = -1;
    if (r < in.n_rows) {
      g = row_group(in, st, r, status);
      int64_t idx;
      if (g >= 0 && !chain_index(in, r, &idx, status)) g = -1;
      row_slot[r] = g >= 0 ? (uint32_t)g : kNoSlot;
    }
    const uint32_t part = g >= 0 ? (uint32_t)(g >> SB) : kNoSlot;
    if (few) {
      uint64_t same;
      uint32_t n_lane;
      part_masks64(g >= 0, part, lane, &same, &n_lane);
      cnt += n_lane;
      continue;
    }
    uint64_t todo = __ballot(g >= 0);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const uint32_t p0 = __builtin_amdgcn_readlane(part, leader);
      const uint64_t same = __ballot(part == p0) & todo;
      if (lane == leader) mat[(int64_t)p0 * n_waves + w] += (uint32_t)__popcll(same);  // only this wave writes it
      todo &= ~same;
    }
  }
  if (few && lane < n_parts) mat[(int64_t)lane * n_waves + w] = cnt;
}

// Per partition (one workgroup each): exclusive prefix of the per-wave counts
// mat[part][0..n_waves) in wave order, and the partition's total.
__global__ __launch_bounds__(256) void part_colscan(uint32_t *mat, int64_t n_parts, int64_t n_waves,
                                                    uint32_t *count) {
  __shared__ uint32_t sums[256];
  const int64_t p = blockIdx.x;
  const int t = threadIdx.x;
  uint32_t *col = mat + p * n_waves;
  const int64_t per = (n_waves + 255) / 256, w0 = t * per, w1 = min(n_waves, w0 + per);
  uint32_t s = 0;
  for (int64_t w = w0; w < w1; ++w) s += col[w];
  sums[t] = s;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const uint32_t a = t >= d ? sums[t - d] : 0u;
    __syncthreads();
    sums[t] += a;
    __syncthreads();
  }
  uint32_t run = sums[t] - s;
  for (int64_t w = w0; w < w1; ++w) {
    const uint32_t c = col[w];
    col[w] = run;
    run += c;
  }
  if (t == 255) count[p] = sums[255];
}

// 1''. route with a workgroup histogram in LDS (up to kLdsParts partitions:
// the global counters then see one atomic per workgroup and partition).
constexpr int64_t kLdsParts = 32768;   // 128 KB of LDS
constexpr int64_t kLdsPartsBig = 8192; // above: 1024-thread workgroups, one per CU

__global__ __launch_bounds__(1024) void part_route_lds(DevInput in, DevState st, uint32_t *status,
                                                       uint32_t *row_slot, uint32_t *count, int SB, int64_t n_parts) {
  extern __shared__ uint32_t hist[];
  for (int64_t i = threadIdx.x; i < n_parts; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t n = in.n_rows, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    int64_t g = row_group(in, st, r, status);
    int64_t idx;
    if (g >= 0 && !chain_index(in, r, &idx, status)) g = -1;
    row_slot[r] = g >= 0 ? (uint32_t)g : kNoSlot;
    if (g >= 0) atomicAdd(&hist[g >> SB], 1u);
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n_parts; i += blockDim.x)
    if (hist[i]) atomicAdd(&count[i], hist[i]);
}

// 3''. scatter with per-workgroup range reservation: count this workgroup's
// rows per partition, reserve one range per partition, then place the rows.
template <int W>
__global__ __launch_bounds__(1024) void part_scatter_lds(DevInput in, uint32_t *status, const uint32_t *row_slot,
                                                         const int64_t *off, uint32_t *cur, int SB, int64_t n_parts,
                                                         int64_t cap, uint32_t *rec_slot, uint64_t *rec_mk,
                                                         uint64_t *rec_iv, uint64_t *rec_fv) {
  extern __shared__ uint32_t at[];
  for (int64_t i = threadIdx.x; i < n_parts; i += blockDim.x) at[i] = 0;
  __syncthreads();
  const int64_t n = in.n_rows, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = r0; r < n; r += stride) {
    const uint32_t s = row_slot[r];
    if (s != kNoSlot) atomicAdd(&at[s >> SB], 1u);
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n_parts; i += blockDim.x)
    if (at[i]) at[i] = atomicAdd(&cur[i], at[i]);  // start of this workgroup's range
  __syncthreads();
  const uint32_t lmask = (1u << SB) - 1u;
  for (int64_t r = r0; r < n; r += stride) {
    const uint32_t s = row_slot[r];
    if (s == kNoSlot) continue;
    const uint32_t p = s >> SB;
    const int64_t pos = off[p] + atomicAdd(&at[p], 1u);
    uint64_t mk[W], iv[kMaxCols], fv[kMaxCols];
    load_payload<W>(in, r, status, mk, iv, fv);
    rec_slot[pos] = s & lmask;
#pragma unroll
    for (int k = 0; k < W; ++k) rec_mk[k * cap + pos] = mk[k];
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k)
      if (k < in.n_icols) rec_iv[k * cap + pos] = iv[k];
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k)
      if (k < in.n_fcols) rec_fv[k * cap + pos] = fv[k];
  }
}

// Two-pass scatter, between the passes: rows of each coarse bucket (the sum of
// its 2^S2 fine partitions' counts), one thread per bucket.
__global__ __launch_bounds__(256) void part_coarse_count(const uint32_t *count, int64_t n_parts, int S2,
                                                         int64_t n_coarse, uint32_t *ccount) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_coarse) return;
  const int64_t p0 = c << S2, p1 = min(n_parts, (c + 1) << S2);
  uint32_t n = 0;
  for (int64_t p = p0; p < p1; ++p) n += count[p];
  ccount[c] = n;
}

// Both passes of the two-pass scatter place their records tile by tile: the
// 1024 records of a tile (one per thread) are ordered by bucket in LDS, so
// that consecutive threads write consecutive positions of a bucket's range
// instead of one record per cache line.  LDS: the buckets' cursors, the tile's
// per-bucket counts and offsets (at most kTileBuckets buckets), then the
// staged tile: slot, bucket and payload words (PU words, int and float
// values) of every record in bucket order.
constexpr int kTileBuckets = 256;
constexpr int kTileThreads = 1024;
constexpr int kPayMax = 2 + kMaxCols;

// Records per thread of a tile, and the payload words a record may carry at
// that size: narrow records (C3's PU word and value) take 4 per thread, so a
// bucket's run in a tile is 4 times longer.
__host__ __device__ constexpr int tile_rpt(int words) { return words <= 2 ? 4 : words <= 5 ? 2 : 1; }
template <int RPT>
struct TilePw {
  static constexpr int value = RPT == 4 ? 2 : RPT == 2 ? 5 : kPayMax;
};

__host__ __device__ constexpr size_t tile_lds_bytes(int words) {
  return (size_t)(3 * kTileBuckets + 2) * 4 + (size_t)tile_rpt(words) * kTileThreads * (8 + 8 * (size_t)words);
}

struct TileLds {
  uint32_t *base, *tcount, *toff, *total, *s_slot, *s_q;
  uint64_t *s_pay;
  int T;  // records per tile
  __device__ TileLds(uint8_t *raw, int recs) : T(recs) {
    base = (uint32_t *)raw;
    tcount = base + kTileBuckets;
    toff = tcount + kTileBuckets;
    total = toff + kTileBuckets;  // 2 words: keeps the payload 8-byte aligned
    s_slot = total + 2;
    s_q = s_slot + T;
    s_pay = (uint64_t *)(s_q + T);
  }
};

// Exclusive scan of tcount[0..nb) into toff, and the tile's record count
// (wave 0; nb <= 4 * 64).
__device__ __forceinline__ void tile_scan(const TileLds &L, int nb) {
  const int t = threadIdx.x;
  if (t < 64) {
    uint32_t a[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = 4 * t + k < nb ? L.tcount[4 * t + k] : 0u;
      sum += a[k];
    }
    uint32_t incl = sum;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(incl, d);
      if (t >= d) incl += v;
    }
    uint32_t ex = incl - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (4 * t + k < nb) L.toff[4 * t + k] = ex;
      ex += a[k];
    }
    if (t == 63) *L.total = incl;
  }
}

// Output pointers of the payload words: PU words, then int columns
// (structure of arrays, `cap` records each).
struct PayOut {
  uint64_t *p[kPayMax];
};

template <int W>
__device__ __forceinline__ PayOut pay_out(int ni, int64_t cap, uint64_t *mk, uint64_t *iv) {
  PayOut o{};
#pragma unroll
  for (int w = 0; w < W; ++w) o.p[w] = mk + w * cap;
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c) o.p[W + c] = c < ni ? iv + c * cap : nullptr;
  return o;
}

// One tile: each thread holds RPT records (bucket q, output slot, payload of
// `words` words); records are ranked in their bucket, staged in bucket order,
// then written from the staged order to base[q] + rank, consecutive threads
// writing consecutive records.  Every thread of the workgroup calls it
// (barriers inside).
template <int RPT, int PW>
__device__ __forceinline__ void tile_place(const TileLds &L, int nb, const bool (&live)[RPT],
                                           const uint32_t (&q)[RPT], const uint32_t (&slot_out)[RPT],
                                           const uint64_t (&pay)[RPT][PW], int words, uint32_t *out_slot,
                                           const PayOut &out) {
  const int t = threadIdx.x;
  for (int b = t; b < nb; b += blockDim.x) L.tcount[b] = 0;
  __syncthreads();
  uint32_t lr[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) lr[i] = live[i] ? atomicAdd(&L.tcount[q[i]], 1u) : 0u;
  __syncthreads();
  tile_scan(L, nb);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    if (!live[i]) continue;
    const uint32_t si = L.toff[q[i]] + lr[i];
    L.s_slot[si] = slot_out[i];
    L.s_q[si] = q[i];
#pragma unroll
    for (int k = 0; k < PW; ++k)
      if (k < words) L.s_pay[k * L.T + si] = pay[i][k];
  }
  __syncthreads();
  const uint32_t n_live = *L.total;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const uint32_t ts = (uint32_t)(i * kTileThreads + t);
    if (ts < n_live) {
      const uint32_t qq = L.s_q[ts];
      const int64_t pos = (int64_t)L.base[qq] + ((int64_t)ts - (int64_t)L.toff[qq]);
      out_slot[pos] = L.s_slot[ts];
#pragma unroll
      for (int k = 0; k < PW; ++k)
        if (k < words) out.p[k][pos] = L.s_pay[k * L.T + ts];
    }
  }
  __syncthreads();
  for (int b = t; b < nb; b += blockDim.x) L.base[b] += L.tcount[b];
  __syncthreads();
}

// Two-pass scatter (integer columns only), pass 1: rows -> coarse buckets
// (nb <= kTileBuckets buckets of 2^SBC slots).  The workgroup counts its rows
// per bucket, reserves one range per bucket, then places its rows tile by
// tile (RPT rows per thread).  Each record keeps its slot within the bucket.
// A row the route gave a slot has a valid FK chain, so every counted row is
// placed.
template <int W, int RPT>
__global__ __launch_bounds__(1024) void part_scatter_coarse(DevInput in, uint32_t *status, const uint32_t *row_slot,
                                                            const int64_t *coff, uint32_t *ccur, int SBC, int nb,
                                                            int64_t cap, uint32_t *tmp_slot, uint64_t *tmp_mk,
                                                            uint64_t *tmp_iv) {
  constexpr int PW = TilePw<RPT>::value;
  constexpr int T = RPT * kTileThreads;
  extern __shared__ uint8_t tile_raw[];
  const TileLds L(tile_raw, T);
  const int t = threadIdx.x;
  const int words = W + in.n_icols;
  const PayOut out = pay_out<W>(in.n_icols, cap, tmp_mk, tmp_iv);
  for (int b = t; b < nb; b += blockDim.x) L.base[b] = 0;
  __syncthreads();
  const int64_t n = in.n_rows, stride = (int64_t)gridDim.x * T;
  for (int64_t rt = (int64_t)blockIdx.x * T; rt < n; rt += stride) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t r = rt + i * kTileThreads + t;
      const uint32_t sl = r < n ? row_slot[r] : kNoSlot;
      if (sl != kNoSlot) atomicAdd(&L.base[sl >> SBC], 1u);
    }
  }
  __syncthreads();
  for (int b = t; b < nb; b += blockDim.x)
    if (L.base[b]) L.base[b] = (uint32_t)(coff[b] + atomicAdd(&ccur[b], L.base[b]));
  __syncthreads();
  const uint32_t lmask = (1u << SBC) - 1u;
  for (int64_t rt = (int64_t)blockIdx.x * T; rt < n; rt += stride) {
    bool live[RPT];
    uint32_t q[RPT], so[RPT];
    uint64_t pay[RPT][PW];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t r = rt + i * kTileThreads + t;
      const uint32_t sl = r < n ? row_slot[r] : kNoSlot;
      live[i] = sl != kNoSlot;
      q[i] = live[i] ? sl >> SBC : 0u;
      so[i] = sl & lmask;
#pragma unroll
      for (int k = 0; k < PW; ++k) pay[i][k] = 0;
      if (live[i]) {
        uint64_t mk[W], iv[kMaxCols], fv[kMaxCols];
        if (load_payload<W>(in, r, status, mk, iv, fv)) {
#pragma unroll
          for (int w = 0; w < W; ++w) pay[i][w] = mk[w];
#pragma unroll
          for (int c = 0; c < kMaxCols; ++c)
            if (W + c < PW && c < in.n_icols) pay[i][(W + c) < PW ? (W + c) : 0] = iv[c];
        }
      }
    }
    tile_place<RPT, PW>(L, nb, live, q, so, pay, words, tmp_slot, out);
  }
}

// Two-pass scatter, pass 2: each work item is a run of one coarse bucket's
// records; the workgroup counts them per fine partition (2^S2 of them),
// reserves one range per fine partition, then places them tile by tile.
template <int W, int RPT>
__global__ __launch_bounds__(1024) void part_scatter2(const PartItem *items2, const int64_t *meta2, int S2, int SB,
                                                      const int64_t *off, uint32_t *cur, int64_t cap, int ni,
                                                      const uint32_t *tmp_slot, const uint64_t *tmp_mk,
                                                      const uint64_t *tmp_iv, uint32_t *rec_slot, uint64_t *rec_mk,
                                                      uint64_t *rec_iv) {
  constexpr int PW = TilePw<RPT>::value;
  constexpr int T = RPT * kTileThreads;
  extern __shared__ uint8_t tile_raw[];
  const TileLds L(tile_raw, T);
  const int t = threadIdx.x;
  const int nq = 1 << S2, words = W + ni;
  const uint32_t lmask = (1u << SB) - 1u;
  const PayOut out = pay_out<W>(ni, cap, rec_mk, rec_iv);
  const int64_t n_items = meta2[0];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const PartItem item = items2[it];
    const int64_t pbase = item.part << S2;
    for (int qq = t; qq < nq; qq += blockDim.x) L.base[qq] = 0;
    __syncthreads();
    for (int64_t r = item.begin + t; r < item.end; r += blockDim.x) atomicAdd(&L.base[tmp_slot[r] >> SB], 1u);
    __syncthreads();
    for (int qq = t; qq < nq; qq += blockDim.x)
      if (L.base[qq]) L.base[qq] = (uint32_t)(off[pbase + qq] + atomicAdd(&cur[pbase + qq], L.base[qq]));
    __syncthreads();
    for (int64_t rt = item.begin; rt < item.end; rt += T) {
      bool live[RPT];
      uint32_t q[RPT], so[RPT];
      uint64_t pay[RPT][PW];
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int64_t r = rt + i * kTileThreads + t;
        live[i] = r < item.end;
        const uint32_t sc = live[i] ? tmp_slot[r] : 0u;
        q[i] = sc >> SB;
        so[i] = sc & lmask;
#pragma unroll
        for (int k = 0; k < PW; ++k) pay[i][k] = 0;
        if (live[i]) {
#pragma unroll
          for (int w = 0; w < W; ++w) pay[i][w] = tmp_mk[w * cap + r];
#pragma unroll
          for (int c = 0; c < kMaxCols; ++c)
            if (W + c < PW && c < ni) pay[i][(W + c) < PW ? (W + c) : 0] = tmp_iv[c * cap + r];
        }
      }
      tile_place<RPT, PW>(L, nq, live, q, so, pay, words, rec_slot, out);
    }
  }
}

// 2. offsets and work items (one workgroup; each thread scans a contiguous run of partitions)
__global__ __launch_bounds__(1024) void part_scan(const uint32_t *count, int64_t n_parts, int64_t chunk,
                                                  int64_t *off, uint32_t *cur, PartItem *items, int64_t *meta,
                                                  int64_t *pfirst) {
  __shared__ int64_t s_rows[1024], s_items[1024];
  const int t = threadIdx.x, T = blockDim.x;
  const int64_t per = (n_parts + T - 1) / T;
  const int64_t p0 = t * per, p1 = min(n_parts, p0 + per);
  int64_t rows = 0, nit = 0;
  for (int64_t p = p0; p < p1; ++p) {
    rows += count[p];
    nit += (count[p] + chunk - 1) / chunk;
  }
  s_rows[t] = rows;
  s_items[t] = nit;
  __syncthreads();
  for (int d = 1; d < T; d <<= 1) {  // inclusive scan over the threads
    int64_t a = 0, b = 0;
    if (t >= d) {
      a = s_rows[t - d];
      b = s_items[t - d];
    }
    __syncthreads();
    s_rows[t] += a;
    s_items[t] += b;
    __syncthreads();
  }
  int64_t r0 = s_rows[t] - rows, i0 = s_items[t] - nit;
  for (int64_t p = p0; p < p1; ++p) {
    off[p] = r0;
    cur[p] = 0;
    const int64_t n = count[p];
    if (pfirst) {
      pfirst[2 * p] = i0;
      pfirst[2 * p + 1] = (n + chunk - 1) / chunk;
    }
    for (int64_t b = 0; b < n; b += chunk) items[i0++] = PartItem{p, r0 + b, r0 + min(n, b + chunk), n <= chunk};
    r0 += n;
  }
  if (t == T - 1) {
    off[n_parts] = s_rows[t];
    meta[0] = s_items[t];
    meta[1] = 0;
  }
}

// 3. scatter the live rows into their partitions
template <int W>
__global__ __launch_bounds__(256) void part_scatter(DevInput in, uint32_t *status, const uint32_t *row_slot,
                                                    const int64_t *off, uint32_t *cur, int SB, int64_t cap,
                                                    uint32_t *rec_slot, uint64_t *rec_mk, uint64_t *rec_iv,
                                                    uint64_t *rec_fv) {
  const int lane = threadIdx.x & 63;
  const int64_t n_chunks = (in.n_rows + 63) >> 6;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const uint32_t lmask = (1u << SB) - 1u;
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < n_chunks; c += waves) {
    const int64_t r = c * 64 + lane;
    const uint32_t s = r < in.n_rows ? row_slot[r] : kNoSlot;
    const uint32_t part = s != kNoSlot ? s >> SB : kNoSlot;
    int64_t pos = -1;
    uint64_t todo = __ballot(s != kNoSlot);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const uint32_t p0 = __builtin_amdgcn_readlane(part, leader);
      const uint64_t same = __ballot(part == p0) & todo;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&cur[p0], (uint32_t)__popcll(same));
      base = __builtin_amdgcn_readlane(base, leader);
      if ((same >> lane) & 1ull) pos = off[p0] + base + __popcll(same & lanes_lt(lane));
      todo &= ~same;
    }
    if (pos >= 0) {
      uint64_t mk[W], iv[kMaxCols], fv[kMaxCols];
      load_payload<W>(in, r, status, mk, iv, fv);
      rec_slot[pos] = s & lmask;
#pragma unroll
      for (int w = 0; w < W; ++w) rec_mk[w * cap + pos] = mk[w];
#pragma unroll
      for (int k = 0; k < kMaxCols; ++k)
        if (k < in.n_icols) rec_iv[k * cap + pos] = iv[k];
#pragma unroll
      for (int k = 0; k < kMaxCols; ++k)
        if (k < in.n_fcols) rec_fv[k * cap + pos] = fv[k];
    }
  }
}

// 3'. deterministic scatter: the chunks of the routing, in the same order;
// a row's position is its partition's offset plus the rows before it.
template <int W>
__global__ __launch_bounds__(256) void part_scatter_det(DevInput in, uint32_t *status, const uint32_t *row_slot,
                                                        const int64_t *off, uint32_t *mat, int64_t n_parts, int SB,
                                                        int64_t n_waves, int64_t cap, uint32_t *rec_slot,
                                                        uint64_t *rec_mk, uint64_t *rec_iv, uint64_t *rec_fv) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= n_waves) return;
  const int64_t n_chunks = (in.n_rows + 63) >> 6, cpw = (n_chunks + n_waves - 1) / n_waves;
  const uint32_t lmask = (1u << SB) - 1u;
  // few partitions: lane p holds partition p's next position in registers
  const bool few = n_parts <= 64;
  int64_t next = few && lane < n_parts ? off[lane] + mat[(int64_t)lane * n_waves + w] : 0;
  for (int64_t c = w * cpw; c < min(n_chunks, (w + 1) * cpw); ++c) {
    const int64_t r = c * 64 + lane;
    const uint32_t s = r < in.n_rows ? row_slot[r] : kNoSlot;
    const uint32_t part = s != kNoSlot ? s >> SB : kNoSlot;
    int64_t pos = -1;
    if (few) {
      // this lane's record goes after the earlier lanes of its partition, from
      // that partition's running position (held by lane `part`)
      uint64_t same;
      uint32_t n_lane;
      const bool valid = s != kNoSlot;
      part_masks64(valid, part, lane, &same, &n_lane);
      const int src = valid ? (int)part : 0;
      const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)next, src), hi = (uint32_t)__shfl((int)(next >> 32), src);
      const int64_t start = (int64_t)(((uint64_t)hi << 32) | lo);
      if (valid) pos = start + __popcll(same & lanes_lt(lane));
      next += (int64_t)n_lane;
    }
    uint64_t todo = few ? 0ull : __ballot(s != kNoSlot);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const uint32_t p0 = __builtin_amdgcn_readlane(part, leader);
      const uint64_t same = __ballot(part == p0) & todo;
      const uint32_t n0 = (uint32_t)__popcll(same);
      uint32_t base = 0;
      if (lane == leader) {
        uint32_t *e = &mat[(int64_t)p0 * n_waves + w];
        base = *e;
        *e = base + n0;
      }
      const int64_t start = off[p0] + __builtin_amdgcn_readlane(base, leader);
      if ((same >> lane) & 1ull) pos = start + __popcll(same & lanes_lt(lane));
      todo &= ~same;
    }
    if (pos >= 0) {
      uint64_t mk[W], iv[kMaxCols], fv[kMaxCols];
      load_payload<W>(in, r, status, mk, iv, fv);
      rec_slot[pos] = s & lmask;
#pragma unroll
      for (int k = 0; k < W; ++k) rec_mk[k * cap + pos] = mk[k];
#pragma unroll
      for (int k = 0; k < kMaxCols; ++k)
        if (k < in.n_icols) rec_iv[k * cap + pos] = iv[k];
#pragma unroll
      for (int k = 0; k < kMaxCols; ++k)
        if (k < in.n_fcols) rec_fv[k * cap + pos] = fv[k];
    }
  }
}

// The records of one batch (bits of `todo`: lanes holding a live record), in
// lane order, into the counters at region + slot * slot_words (lane = world).
// Two records per iteration: the cross-lane reads of both are issued before
// the LDS adds of the first.  No-return LDS adds of one wave apply in issue
// order, so a wave-private region sums in record order.
template <int W, int CI, int CF>
__device__ __forceinline__ void part_records(uint64_t *region, int64_t slot_words, int A, int ni, int nf, uint32_t ls,
                                             const uint64_t (&mk)[W], const uint64_t (&iv)[CI > 0 ? CI : 1],
                                             const uint64_t (&fv)[CF > 0 ? CF : 1], uint64_t todo, int lane) {
  constexpr int m = 64 * W;
  struct Rec {
    uint64_t *base;
    uint64_t word[W], rv[CI > 0 ? CI : 1], rf[CF > 0 ? CF : 1];
  };
  auto fetch = [&](int rr, Rec &c) {
    c.base = region + (int64_t)__builtin_amdgcn_readlane(ls, rr) * slot_words;
#pragma unroll
    for (int k = 0; k < CI; ++k)
      if (k < ni) c.rv[k] = readlane_u64(iv[k], rr);
#pragma unroll
    for (int k = 0; k < CF; ++k)
      if (k < nf) c.rf[k] = readlane_u64(fv[k], rr);
#pragma unroll
    for (int w = 0; w < W; ++w) c.word[w] = readlane_u64(mk[w], rr);
  };
  auto apply = [&](const Rec &c) {
    if (lane == 0)
      __hip_atomic_fetch_add(&c.base[(int64_t)A * m], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int j = w * 64 + lane;
      if ((c.word[w] >> lane) & 1ull) {
        __hip_atomic_fetch_add(&c.base[j], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
        for (int k = 0; k < CI; ++k)
          if (k < ni)
            __hip_atomic_fetch_add(&c.base[(int64_t)(1 + k) * m + j], c.rv[k], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
        for (int k = 0; k < CF; ++k)
          if (k < nf)
            __hip_atomic_fetch_add((double *)&c.base[(int64_t)(1 + ni + k) * m + j],
                                   __longlong_as_double((long long)c.rf[k]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  };
  while (todo) {
    const int r0 = __ffsll((unsigned long long)todo) - 1;
    todo &= todo - 1;
    const bool two = todo != 0;
    const int r1 = two ? __ffsll((unsigned long long)todo) - 1 : r0;
    todo &= todo - 1;  // no-op when empty
    Rec c0, c1;
    fetch(r0, c0);
    fetch(r1, c1);
    apply(c0);
    if (two) apply(c1);
  }
}

// One lane's record of a batch of 64 (record r if r < end, else a dummy
// read of record `first` marked dead).
template <int W, int CI, int CF>
struct RecBatch {
  uint32_t ls;
  bool live;
  uint64_t mk[W], iv[CI > 0 ? CI : 1], fv[CF > 0 ? CF : 1];
  __device__ __forceinline__ void load(int64_t r, int64_t end, int64_t first, int64_t cap, int ni, int nf,
                                       const uint32_t *rec_slot, const uint64_t *rec_mk, const uint64_t *rec_iv,
                                       const uint64_t *rec_fv) {
    live = r < end;
    const int64_t i = live ? r : first;
    ls = rec_slot[i];
#pragma unroll
    for (int w = 0; w < W; ++w) mk[w] = rec_mk[w * cap + i];
#pragma unroll
    for (int k = 0; k < CI; ++k)
      if (k < ni) iv[k] = rec_iv[k * cap + i];
#pragma unroll
    for (int k = 0; k < CF; ++k)
      if (k < nf) fv[k] = rec_fv[k * cap + i];
  }
};

// 4. per-partition aggregation in LDS
// NI / NF >= 0: the column counts are compile-time (no per-column branches in
// the per-record loop); -1: taken from ni_rt / nf_rt.
template <int W, int NI, int NF>
__global__ __launch_bounds__(64 * kPartWavesNd) void part_aggregate(DevState st, int ni_rt, int nf_rt, int64_t n_slots,
                                                      int SB, int64_t slot_words, int64_t cap,
                                                      const uint32_t *rec_slot, const uint64_t *rec_mk,
                                                      const uint64_t *rec_iv, const uint64_t *rec_fv,
                                                      const PartItem *items, int64_t *meta, int fresh) {
  extern __shared__ uint64_t lds[];
  __shared__ int64_t s_item;
  constexpr int m = 64 * W;
  constexpr int CI = NI < 0 ? kMaxCols : NI, CF = NF < 0 ? kMaxCols : NF;
  const int ni = NI < 0 ? ni_rt : NI, nf = NF < 0 ? nf_rt : NF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int A = 1 + ni + nf;
  const int64_t words = slot_words << SB;
  const int64_t n_items = meta[0];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd((unsigned long long *)&meta[1], 1ull);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= n_items) break;  // the same value in every thread: every wave leaves
    const PartItem item = items[it];
    for (int64_t i = threadIdx.x; i < words; i += blockDim.x) lds[i] = 0;
    __syncthreads();
    for (int64_t b = item.begin + 64 * wave; b < item.end; b += 64 * waves) {
      RecBatch<W, CI, CF> c;
      c.load(b + lane, item.end, item.begin, cap, ni, nf, rec_slot, rec_mk, rec_iv, rec_fv);
      part_records<W, CI, CF>(lds, slot_words, A, ni, nf, c.ls, c.mk, c.iv, c.fv, __ballot(c.live), lane);
    }
    __syncthreads();
    // non-zero counters of this partition -> global state
    for (int64_t i = threadIdx.x; i < words; i += blockDim.x) {
      const uint64_t v = lds[i];
      if (!v) continue;
      const int64_t g = (item.part << SB) + i / slot_words, o = i % slot_words;
      if (g >= n_slots) continue;
      const int a = o == (int64_t)A * m ? -1 : (int)(o / m), j = (int)(o % m);
      // no-return atomics: measured faster than stores of the owned words
      if (a > ni) {
        atomicAdd(&st.fsum[(g * nf + (a - 1 - ni)) * m + j], __longlong_as_double((long long)v));
        continue;
      }
      unsigned long long *dst = a < 0   ? (unsigned long long *)&st.nrows[g]
                                : a == 0 ? (unsigned long long *)&st.count[g * m + j]
                                         : (unsigned long long *)&st.isum[(g * ni + (a - 1)) * m + j];
      atomicAdd(dst, (unsigned long long)v);
    }
  }
}

// 4''. integer columns, sorted runs: each chunk of kSortChunk records of a work
// item is counting-sorted by slot in LDS; then each wave walks 64 consecutive
// sorted records (read at one LDS address for all lanes), keeping the current
// slot's per-world count and sums in registers (lane = world), and adds them to
// the partition's LDS counters only when the slot changes.  The counters take
// one add per (run, counter word) instead of one per (record, counter word);
// integer sums are exact in any order, so the result equals the other forms'.
// The next chunk's records are loaded into registers while the current chunk
// is walked, and workgroups of 8 waves leave room for two per CU.
constexpr int kSortWaves = 8;
constexpr int kSortChunk = 64 * kSortWaves;
constexpr int kSortMaxSlots = 256;
constexpr int kWalkBatch = 4;  // sorted records whose LDS reads are in flight together (8 measured no faster)

static size_t sorted_stage_bytes(int W, int ni) {
  return (size_t)kSortChunk * (8 * W + 8 * ni + 4) + 4 * kSortMaxSlots;
}

__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int W, int NI>
struct SortRec {
  bool live;
  uint32_t ls;
  uint64_t mk[W], iv[NI > 0 ? NI : 1];
  __device__ __forceinline__ void load(int64_t c0, int64_t end, int t, int64_t cap, const uint32_t *rec_slot,
                                       const uint64_t *rec_mk, const uint64_t *rec_iv) {
    live = c0 + t < end;
    const int64_t i = live ? c0 + t : c0;  // a dead lane reads the chunk's first record and ignores it
    ls = rec_slot[i];
#pragma unroll
    for (int w = 0; w < W; ++w) mk[w] = rec_mk[w * cap + i];
#pragma unroll
    for (int k = 0; k < NI; ++k) iv[k] = rec_iv[k * cap + i];
  }
};

template <int W, int NI>
__global__ __launch_bounds__(64 * kSortWaves) void part_aggregate_sorted(
    DevState st, int64_t n_slots, int SB, int64_t slot_words, int64_t cap, const uint32_t *rec_slot,
    const uint64_t *rec_mk, const uint64_t *rec_iv, const PartItem *items, int64_t *meta) {
  extern __shared__ uint64_t lds[];
  __shared__ int64_t s_item;
  constexpr int m = 64 * W, CI = NI > 0 ? NI : 1, R = kSortChunk, T = 64 * kSortWaves;
  constexpr int A = 1 + NI;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
  const int64_t words = slot_words << SB;
  const int nslot = 1 << SB;
  uint64_t *s_mk = lds + words;                          // [W][R] PU words, sorted by slot
  uint64_t *s_iv = s_mk + (size_t)W * R;                 // [NI][R] values, sorted by slot
  uint32_t *s_sl = (uint32_t *)(s_iv + (size_t)NI * R);  // [R] slots, sorted
  uint32_t *hist = s_sl + R;                             // [nslot] counts, then start positions
  const int64_t n_items = meta[0];
  for (;;) {
    __syncthreads();
    if (t == 0) s_item = atomicAdd((unsigned long long *)&meta[1], 1ull);
    __syncthreads();
    // the item is the same in every thread: its fields in scalar registers, so the loops below are uniform
    const int64_t it = uniform_i64(s_item);
    if (it >= n_items) break;  // every wave leaves
    PartItem item = items[it];
    item.part = uniform_i64(item.part);
    item.begin = uniform_i64(item.begin);
    item.end = uniform_i64(item.end);
    for (int64_t i = t; i < words; i += T) lds[i] = 0;
    SortRec<W, NI> rec;
    if (item.begin < item.end) rec.load(item.begin, item.end, t, cap, rec_slot, rec_mk, rec_iv);
    for (int64_t c0 = item.begin; c0 < item.end; c0 += R) {
      const int n = (int)min<int64_t>(R, item.end - c0);
      for (int i = t; i < nslot; i += T) hist[i] = 0;
      __syncthreads();
      // rank among the chunk's records of the slot; a wave whose records share one slot takes one add
      uint32_t rank = 0;
      const uint64_t lv = __ballot(rec.live);
      if (lv) {
        const int first = __ffsll((unsigned long long)lv) - 1;
        const uint32_t s0 = __builtin_amdgcn_readlane(rec.ls, first);
        if (__ballot(rec.live && rec.ls == s0) == lv) {
          uint32_t b = 0;
          if (lane == first) b = atomicAdd(&hist[s0], (uint32_t)__popcll(lv));
          b = __builtin_amdgcn_readlane(b, first);
          rank = b + (uint32_t)__popcll(lv & ((1ull << lane) - 1ull));
        } else if (rec.live) {
          rank = atomicAdd(&hist[rec.ls], 1u);
        }
      }
      __syncthreads();
      if (wave == 0) {  // exclusive prefix sum of the counts: nslot <= 256, four per lane
        uint32_t c[4], tot = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int b = 4 * lane + i;
          c[i] = b < nslot ? hist[b] : 0u;
          tot += c[i];
        }
        uint32_t inc = tot;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t o = (uint32_t)__shfl_up((int)inc, d, 64);
          if (lane >= d) inc += o;
        }
        uint32_t run = inc - tot;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int b = 4 * lane + i;
          if (b < nslot) hist[b] = run;
          run += c[i];
        }
      }
      __syncthreads();
      if (rec.live) {
        const uint32_t pos = hist[rec.ls] + rank;
        s_sl[pos] = rec.ls;
#pragma unroll
        for (int w = 0; w < W; ++w) s_mk[w * R + pos] = rec.mk[w];
#pragma unroll
        for (int k = 0; k < NI; ++k) s_iv[k * R + pos] = rec.iv[k];
      }
      __syncthreads();
      if (c0 + R < item.end) rec.load(c0 + R, item.end, t, cap, rec_slot, rec_mk, rec_iv);  // in flight meanwhile
      // this wave's sorted records [p0, p1), read kWalkBatch at a time; runs of one slot summed in registers
      const int p0 = __builtin_amdgcn_readfirstlane(64 * wave), p1 = min(n, p0 + 64);
      if (p0 < p1) {
        uint32_t cur = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_sl[p0]);
        uint32_t cnt[W], nr = 0;
        uint64_t sum[W][CI];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          cnt[w] = 0;
#pragma unroll
          for (int k = 0; k < CI; ++k) sum[w][k] = 0;
        }
        for (int pb = p0; pb < p1; pb += kWalkBatch) {
          uint32_t sl4[kWalkBatch];
          uint64_t mk4[kWalkBatch][W], v4[kWalkBatch][CI];
#pragma unroll
          for (int i = 0; i < kWalkBatch; ++i) {
            const int p = min(pb + i, p1 - 1);  // past the end: re-read the last record, not used
            sl4[i] = s_sl[p];
#pragma unroll
            for (int w = 0; w < W; ++w) mk4[i][w] = s_mk[w * R + p];
#pragma unroll
            for (int k = 0; k < NI; ++k) v4[i][k] = s_iv[k * R + p];
          }
#pragma unroll
          for (int i = 0; i < kWalkBatch; ++i) {
            if (pb + i >= p1) break;
            const uint32_t sl = (uint32_t)__builtin_amdgcn_readfirstlane((int)sl4[i]);
            if (sl != cur) {  // the run of slot `cur` ends: its counters into LDS
              uint64_t *base = lds + (int64_t)cur * slot_words;
              if (lane == 0)
                __hip_atomic_fetch_add(&base[(int64_t)A * m], (uint64_t)nr, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
              for (int w = 0; w < W; ++w) {
                const int j = w * 64 + lane;
                if (cnt[w]) {
                  __hip_atomic_fetch_add(&base[j], (uint64_t)cnt[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
                  for (int k = 0; k < NI; ++k)
                    __hip_atomic_fetch_add(&base[(int64_t)(1 + k) * m + j], sum[w][k], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                cnt[w] = 0;
#pragma unroll
                for (int k = 0; k < CI; ++k) sum[w][k] = 0;
              }
              nr = 0;
              cur = sl;
            }
            ++nr;
#pragma unroll
            for (int w = 0; w < W; ++w) {
              const bool bit = (mk4[i][w] >> lane) & 1ull;
              cnt[w] += bit ? 1u : 0u;
#pragma unroll
              for (int k = 0; k < NI; ++k) sum[w][k] += bit ? v4[i][k] : 0ull;
            }
          }
        }
        {  // the last run
          uint64_t *base = lds + (int64_t)cur * slot_words;
          if (lane == 0)
            __hip_atomic_fetch_add(&base[(int64_t)A * m], (uint64_t)nr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const int j = w * 64 + lane;
            if (cnt[w]) {
              __hip_atomic_fetch_add(&base[j], (uint64_t)cnt[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
              for (int k = 0; k < NI; ++k)
                __hip_atomic_fetch_add(&base[(int64_t)(1 + k) * m + j], sum[w][k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
        }
      }
      __syncthreads();  // the staging is rewritten by the next chunk
    }
    __syncthreads();  // (an item without records: the counters were just cleared)
    // non-zero counters of this partition -> global state
    for (int64_t i = t; i < words; i += T) {
      const uint64_t v = lds[i];
      if (!v) continue;
      const int64_t g = (item.part << SB) + i / slot_words, o = i % slot_words;
      if (g >= n_slots) continue;
      const int a = o == (int64_t)A * m ? -1 : (int)(o / m), j = (int)(o % m);
      unsigned long long *dst = a < 0   ? (unsigned long long *)&st.nrows[g]
                                : a == 0 ? (unsigned long long *)&st.count[g * m + j]
                                         : (unsigned long long *)&st.isum[(g * NI + (a - 1)) * m + j];
      atomicAdd(dst, (unsigned long long)v);
    }
  }
}

// 4'. deterministic per-partition aggregation (float columns): wave w sums the
// w-th quarter of the partition's records, in record order, into its own LDS
// region (lane = world: no two lanes touch one word); the regions are then
// combined in wave order and the owning workgroup adds them to the state.
// S > 0 (common column mixes, S slots per partition): the quarter's counters
// are kept in registers and stored to the region once, instead of LDS adds
// per record.
template <int W, int NI, int NF, int S>
__global__ __launch_bounds__(64 * kPartWaves) void part_aggregate_det(
    DevState st, int ni_rt, int nf_rt, int64_t n_slots, int SB, int64_t slot_words, int64_t cap,
    const uint32_t *rec_slot, const uint64_t *rec_mk, const uint64_t *rec_iv, const uint64_t *rec_fv,
    const PartItem *items, int64_t *meta, uint64_t *partial) {
  extern __shared__ uint64_t lds[];
  __shared__ int64_t s_item;
  constexpr int m = 64 * W;
  constexpr int CI = NI < 0 ? kMaxCols : NI, CF = NF < 0 ? kMaxCols : NF;
  const int ni = NI < 0 ? ni_rt : NI, nf = NF < 0 ? nf_rt : NF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int A = 1 + ni + nf;
  const int64_t words = slot_words << SB;
  uint64_t *mine = lds + (int64_t)wave * words;
  const int64_t n_items = meta[0];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd((unsigned long long *)&meta[1], 1ull);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= n_items) break;
    const PartItem item = items[it];
    const int64_t n = item.end - item.begin, q = (n + kPartWaves - 1) / kPartWaves;
    const int64_t b0 = item.begin + q * wave, b1 = min(item.end, b0 + q);
    if constexpr (S > 0) {
      // S slots per partition: the wave's counters live in registers (lane =
      // world), records added slot by slot in record order -- the order of
      // the LDS form, so the sums are the same -- and are stored to the
      // wave's region (every word of it) at the end.
      uint32_t cn[S][W], nr[S];
      uint64_t is[S][W][CI > 0 ? CI : 1];
      double fs[S][W][CF > 0 ? CF : 1];
#pragma unroll
      for (int sl = 0; sl < S; ++sl) {
        nr[sl] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          cn[sl][w] = 0;
#pragma unroll
          for (int k = 0; k < CI; ++k) is[sl][w][k] = 0;
#pragma unroll
          for (int k = 0; k < CF; ++k) fs[sl][w][k] = 0.0;
        }
      }
      // The batch is staged in the wave's own LDS slice and each record read
      // from there at one address for all lanes (a broadcast).
      __shared__ uint64_t s_rec[kPartWaves][W + (CI > 0 ? CI : 1) + (CF > 0 ? CF : 1)][64];
      constexpr int kIv = W, kFv = W + (CI > 0 ? CI : 1);
      for (int64_t b = b0; b < b1; b += 64) {
        RecBatch<W, CI, CF> c;
        c.load(b + lane, b1, b0, cap, ni, nf, rec_slot, rec_mk, rec_iv, rec_fv);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the previous batch's reads come first
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int w = 0; w < W; ++w) s_rec[wave][w][lane] = c.mk[w];
#pragma unroll
        for (int k = 0; k < CI; ++k) s_rec[wave][kIv + k][lane] = c.iv[k];
#pragma unroll
        for (int k = 0; k < CF; ++k) s_rec[wave][kFv + k][lane] = c.fv[k];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
          uint64_t todo = __ballot(c.live && c.ls == (uint32_t)sl);
          nr[sl] += (uint32_t)__popcll(todo);
          while (todo) {
            const int rr = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            uint64_t u[CI > 0 ? CI : 1];
            double v[CF > 0 ? CF : 1];
#pragma unroll
            for (int k = 0; k < CI; ++k) u[k] = s_rec[wave][kIv + k][rr];
#pragma unroll
            for (int k = 0; k < CF; ++k) v[k] = __longlong_as_double((long long)s_rec[wave][kFv + k][rr]);
#pragma unroll
            for (int w = 0; w < W; ++w) {
              const bool bit = (s_rec[wave][w][rr] >> lane) & 1ull;
              cn[sl][w] += bit ? 1u : 0u;
#pragma unroll
              for (int k = 0; k < CI; ++k) is[sl][w][k] += bit ? u[k] : 0ull;
#pragma unroll
              for (int k = 0; k < CF; ++k) fs[sl][w][k] = bit ? fs[sl][w][k] + v[k] : fs[sl][w][k];
            }
          }
        }
      }
#pragma unroll
      for (int sl = 0; sl < S; ++sl) {
        uint64_t *base = mine + (int64_t)sl * slot_words;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const int j = w * 64 + lane;
          base[j] = cn[sl][w];
#pragma unroll
          for (int k = 0; k < CI; ++k) base[(int64_t)(1 + k) * m + j] = is[sl][w][k];
#pragma unroll
          for (int k = 0; k < CF; ++k)
            base[(int64_t)(1 + CI + k) * m + j] = (uint64_t)__double_as_longlong(fs[sl][w][k]);
        }
        if (lane == 0) base[(int64_t)A * m] = nr[sl];
      }
    } else {
      for (int64_t i = threadIdx.x; i < words * kPartWaves; i += blockDim.x) lds[i] = 0;
      __syncthreads();
      for (int64_t b = b0; b < b1; b += 64) {
        RecBatch<W, CI, CF> c;
        c.load(b + lane, b1, b0, cap, ni, nf, rec_slot, rec_mk, rec_iv, rec_fv);
        part_records<W, CI, CF>(mine, slot_words, A, ni, nf, c.ls, c.mk, c.iv, c.fv, __ballot(c.live), lane);
      }
    }
    __syncthreads();
    // this work item's counters, the wave regions combined in wave order
    uint64_t *out = partial + it * words;
    for (int64_t i = threadIdx.x; i < words; i += blockDim.x) {
      const int64_t o = i % slot_words;
      const int a = o == (int64_t)A * m ? -1 : (int)(o / m);
      if (a < 0 || a <= ni) {
        uint64_t v = 0;
        for (int w = 0; w < kPartWaves; ++w) v += lds[(int64_t)w * words + i];
        out[i] = v;
      } else {
        double v = 0.0;
        for (int w = 0; w < kPartWaves; ++w) v += __longlong_as_double((long long)lds[(int64_t)w * words + i]);
        out[i] = (uint64_t)__double_as_longlong(v);
      }
    }
  }
}

// Deterministic merge: each (partition, counter word) adds its work items'
// counters in item order and the thread owning the word updates the state.
__global__ __launch_bounds__(256) void part_reduce_det(DevState st, int ni, int nf, int m, int64_t n_slots, int SB,
                                                       int64_t slot_words, int64_t n_parts, const int64_t *pfirst,
                                                       const uint64_t *partial, int fresh) {
  const int64_t words = slot_words << SB;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_parts * words) return;
  const int64_t part = t / words, i = t % words;
  const int64_t first = pfirst[2 * part], n_it = pfirst[2 * part + 1];
  if (n_it == 0) return;
  const int64_t g = (part << SB) + i / slot_words, o = i % slot_words;
  if (g >= n_slots) return;
  const int A = 1 + ni + nf;
  const int a = o == (int64_t)A * m ? -1 : (int)(o / m), j = (int)(o % m);
  if (a < 0 || a <= ni) {
    uint64_t v = 0;
    for (int64_t k = 0; k < n_it; ++k) v += partial[(first + k) * words + i];
    if (!v) return;
    uint64_t *dst = a < 0 ? (uint64_t *)&st.nrows[g] : a == 0 ? (uint64_t *)&st.count[g * m + j]
                                                             : (uint64_t *)&st.isum[(g * ni + (a - 1)) * m + j];
    *dst = fresh ? v : *dst + v;
  } else {
    double v = 0.0;
    for (int64_t k = 0; k < n_it; ++k) v += __longlong_as_double((long long)partial[(first + k) * words + i]);
    double *dst = &st.fsum[(g * nf + (a - 1 - ni)) * m + j];
    *dst = fresh ? v : *dst + v;
  }
}

using AggFn = void (*)(DevState, int, int, int64_t, int, int64_t, int64_t, const uint32_t *, const uint64_t *,
                      const uint64_t *, const uint64_t *, const PartItem *, int64_t *, int);
using AggDetFn = void (*)(DevState, int, int, int64_t, int, int64_t, int64_t, const uint32_t *, const uint64_t *,
                         const uint64_t *, const uint64_t *, const PartItem *, int64_t *, uint64_t *);

// Integer columns only (the non-deterministic form): specialised loops for up to three columns.
template <int W>
static AggFn agg_fn(int ni) {
  switch (ni) {
    case 0: return part_aggregate<W, 0, 0>;
    case 1: return part_aggregate<W, 1, 0>;
    case 2: return part_aggregate<W, 2, 0>;
    case 3: return part_aggregate<W, 3, 0>;
    default: return part_aggregate<W, -1, 0>;
  }
}

using SortedFn = void (*)(DevState, int64_t, int, int64_t, int64_t, const uint32_t *, const uint64_t *,
                          const uint64_t *, const PartItem *, int64_t *);

static SortedFn sorted_fn(int W, int ni) {
  if (W == 1) {
    switch (ni) {
      case 0: return part_aggregate_sorted<1, 0>;
      case 1: return part_aggregate_sorted<1, 1>;
      case 2: return part_aggregate_sorted<1, 2>;
      default: return part_aggregate_sorted<1, 3>;
    }
  }
  switch (ni) {
    case 0: return part_aggregate_sorted<2, 0>;
    case 1: return part_aggregate_sorted<2, 1>;
    case 2: return part_aggregate_sorted<2, 2>;
    default: return part_aggregate_sorted<2, 3>;
  }
}

// Float columns present: the common small mixes keep their counters in
// registers (det_reg_slots slots per partition); others use the LDS loop.
template <int W>
static AggDetFn agg_det_fn(int ni, int nf) {
  constexpr int S = W == 1 ? 8 : 4;
  if (nf == 1 && ni == 0) return part_aggregate_det<W, 0, 1, S>;
  if (nf == 1 && ni == 1) return part_aggregate_det<W, 1, 1, S>;
  if (nf == 1 && ni == 2) return part_aggregate_det<W, 2, 1, S>;
  if (nf == 2 && ni == 0) return part_aggregate_det<W, 0, 2, S>;
  return part_aggregate_det<W, -1, -1, 0>;
}

hipError_t launch_agg_part(const LaunchEnv &env, const DevInput &in, const DevState &st, void *scratch,
                           size_t scratch_bytes, bool fresh) {
  if (in.n_rows <= 0) return hipSuccess;
  PartPlan p;
  if (!part_plan(in, &p) || scratch_bytes < p.total) return hipErrorInvalidValue;
  uint8_t *base = (uint8_t *)scratch;
  uint32_t *row_slot = (uint32_t *)(base + p.off_row_slot);
  uint32_t *count = (uint32_t *)(base + p.off_count);
  int64_t *off = (int64_t *)(base + p.off_off);
  uint32_t *cur = (uint32_t *)(base + p.off_cur);
  PartItem *items = (PartItem *)(base + p.off_items);
  int64_t *meta = (int64_t *)(base + p.off_meta);
  uint32_t *rec_slot = (uint32_t *)(base + p.off_rec_slot);
  uint64_t *rec_mk = (uint64_t *)(base + p.off_rec_mk);
  uint64_t *rec_iv = (uint64_t *)(base + p.off_rec_iv);
  uint64_t *rec_fv = (uint64_t *)(base + p.off_rec_fv);

  const int64_t n_chunks = (in.n_rows + 63) / 64;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n_chunks + 3) / 4, (int64_t)env.n_cu * 8));
  hipError_t e;
  if (p.det) {
    uint32_t *mat = (uint32_t *)(base + p.off_mat);
    const int64_t mat_words = p.n_waves * p.n_parts;
    if ((e = launch_fill_i64(env, (int64_t *)mat, (mat_words + 1) / 2, 0)) != hipSuccess) return e;
    const int wgrid = (int)((p.n_waves + 3) / 4);
    hipLaunchKernelGGL(part_route_det, dim3(wgrid), dim3(256), 0, env.stream, in, st, env.status, row_slot, mat,
                       p.n_parts, p.SB, p.n_waves);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(part_colscan, dim3((unsigned)p.n_parts), dim3(256), 0, env.stream, mat, p.n_parts, p.n_waves,
                       count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(part_scan, dim3(1), dim3(1024), 0, env.stream, count, p.n_parts, p.chunk, off, cur, items,
                       meta, (int64_t *)(base + p.off_pfirst));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (in.W == 1)
      hipLaunchKernelGGL(part_scatter_det<1>, dim3(wgrid), dim3(256), 0, env.stream, in, env.status, row_slot, off,
                         mat, p.n_parts, p.SB, p.n_waves, p.cap, rec_slot, rec_mk, rec_iv, rec_fv);
    else
      hipLaunchKernelGGL(part_scatter_det<2>, dim3(wgrid), dim3(256), 0, env.stream, in, env.status, row_slot, off,
                         mat, p.n_parts, p.SB, p.n_waves, p.cap, rec_slot, rec_mk, rec_iv, rec_fv);
  } else {
    if ((e = launch_fill_i64(env, (int64_t *)count, (p.n_parts + 1) / 2, 0)) != hipSuccess)  // u32 counts in pairs
      return e;
    const bool few = p.n_parts <= kLdsParts;  // workgroup histograms and range reservations in LDS
    // many partitions: fewer, larger workgroups, so that each sees more rows
    // per partition and the global counters fewer atomics
    const bool big = p.n_parts > kLdsPartsBig;
    const int lgrid = big ? env.n_cu : grid, lblock = big ? 1024 : 256;
    const size_t lds = (size_t)p.n_parts * 4;
    if (few) {
      if ((e = hipFuncSetAttribute((const void *)part_route_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(part_route_lds, dim3(lgrid), dim3(lblock), lds, env.stream, in, st, env.status, row_slot,
                         count, p.SB, p.n_parts);
    } else {
      hipLaunchKernelGGL(part_route, dim3(grid), dim3(256), 0, env.stream, in, st, env.status, row_slot, count,
                         p.SB);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(part_scan, dim3(1), dim3(1024), 0, env.stream, count, p.n_parts, p.chunk, off, cur, items,
                       meta, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p.S2 > 0) {
      // two passes: rows -> coarse buckets (the LDS scatter over n_coarse
      // partitions of SB + S2 bits, into the temporary records), then
      // buckets -> fine partitions
      uint32_t *ccount = (uint32_t *)(base + p.off_ccount);
      int64_t *coff = (int64_t *)(base + p.off_coff);
      uint32_t *ccur = (uint32_t *)(base + p.off_ccur);
      PartItem *items2 = (PartItem *)(base + p.off_items2);
      int64_t *meta2 = (int64_t *)(base + p.off_meta2);
      uint32_t *tmp_slot = (uint32_t *)(base + p.off_tmp_slot);
      uint64_t *tmp_mk = (uint64_t *)(base + p.off_tmp_mk);
      uint64_t *tmp_iv = (uint64_t *)(base + p.off_tmp_iv);
      hipLaunchKernelGGL(part_coarse_count, dim3((unsigned)((p.n_coarse + 255) / 256)), dim3(256), 0, env.stream,
                         count, p.n_parts, p.S2, p.n_coarse, ccount);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(part_scan, dim3(1), dim3(1024), 0, env.stream, ccount, p.n_coarse, p.chunk2, coff, ccur,
                         items2, meta2, nullptr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const int words = in.W + in.n_icols;  // the two-pass form has no float columns
      const size_t tlds = tile_lds_bytes(words);
      const int rpt = tile_rpt(words);
      // 1024-thread scatter workgroups per CU in both passes (tuned; one by default)
      const dim3 sgrid(env.n_cu * (env.scatter_wg_per_cu > 0 ? env.scatter_wg_per_cu : 1)), sblock(kTileThreads);
      auto two_pass = [&](auto cfn, auto sfn2) -> hipError_t {
        hipError_t err;
        if ((err = hipFuncSetAttribute((const void *)cfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tlds)) !=
                hipSuccess ||
            (err = hipFuncSetAttribute((const void *)sfn2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tlds)) !=
                hipSuccess)
          return err;
        hipLaunchKernelGGL(cfn, sgrid, sblock, tlds, env.stream, in, env.status, row_slot, coff, ccur, p.SB + p.S2,
                           (int)p.n_coarse, p.cap, tmp_slot, tmp_mk, tmp_iv);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        hipLaunchKernelGGL(sfn2, sgrid, sblock, tlds, env.stream, items2, meta2, p.S2, p.SB, off, cur, p.cap,
                           in.n_icols, tmp_slot, tmp_mk, tmp_iv, rec_slot, rec_mk, rec_iv);
        return hipGetLastError();
      };
      if (in.W == 1)
        e = rpt == 4 ? two_pass(part_scatter_coarse<1, 4>, part_scatter2<1, 4>)
            : rpt == 2 ? two_pass(part_scatter_coarse<1, 2>, part_scatter2<1, 2>)
                       : two_pass(part_scatter_coarse<1, 1>, part_scatter2<1, 1>);
      else
        e = rpt == 4 ? two_pass(part_scatter_coarse<2, 4>, part_scatter2<2, 4>)
            : rpt == 2 ? two_pass(part_scatter_coarse<2, 2>, part_scatter2<2, 2>)
                       : two_pass(part_scatter_coarse<2, 1>, part_scatter2<2, 1>);
      if (e != hipSuccess) return e;
    } else if (few) {
      const void *sfn = in.W == 1 ? (const void *)part_scatter_lds<1> : (const void *)part_scatter_lds<2>;
      if ((e = hipFuncSetAttribute(sfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
        return e;
      if (in.W == 1)
        hipLaunchKernelGGL(part_scatter_lds<1>, dim3(lgrid), dim3(lblock), lds, env.stream, in, env.status, row_slot,
                           off, cur, p.SB, p.n_parts, p.cap, rec_slot, rec_mk, rec_iv, rec_fv);
      else
        hipLaunchKernelGGL(part_scatter_lds<2>, dim3(lgrid), dim3(lblock), lds, env.stream, in, env.status, row_slot,
                           off, cur, p.SB, p.n_parts, p.cap, rec_slot, rec_mk, rec_iv, rec_fv);
    } else if (in.W == 1) {
      hipLaunchKernelGGL(part_scatter<1>, dim3(grid), dim3(256), 0, env.stream, in, env.status, row_slot, off, cur,
                         p.SB, p.cap, rec_slot, rec_mk, rec_iv, rec_fv);
    } else {
      hipLaunchKernelGGL(part_scatter<2>, dim3(grid), dim3(256), 0, env.stream, in, env.status, row_slot, off, cur,
                         p.SB, p.cap, rec_slot, rec_mk, rec_iv, rec_fv);
    }
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // integer columns: the sorted-runs aggregate when its staging fits beside the counters
  const size_t sorted_lds = (size_t)p.lds_bytes + sorted_stage_bytes(in.W, in.n_icols);
  if (!p.det && in.n_icols <= 3 && p.SB <= 8 && sorted_lds + 64 <= 160 * 1024) {
    const SortedFn sfn = sorted_fn(in.W, in.n_icols);
    if ((e = hipFuncSetAttribute((const void *)sfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sorted_lds)) !=
        hipSuccess)
      return e;
    int per_cu = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)sfn, 64 * kSortWaves,
                                                          sorted_lds)) != hipSuccess)
      return e;
    const int grid = std::max(1, env.n_cu * std::max(1, per_cu));
    hipLaunchKernelGGL(sfn, dim3(grid), dim3(64 * kSortWaves), sorted_lds, env.stream, st, p.n_slots, p.SB,
                       p.slot_words, p.cap, rec_slot, rec_mk, rec_iv, items, meta);
    return hipGetLastError();
  }
  const AggFn afn = p.det ? nullptr : (in.W == 1 ? agg_fn<1>(in.n_icols) : agg_fn<2>(in.n_icols));
  const AggDetFn dfn = p.det ? (in.W == 1 ? agg_det_fn<1>(in.n_icols, in.n_fcols) : agg_det_fn<2>(in.n_icols, in.n_fcols))
                             : nullptr;
  const void *fn = p.det ? (const void *)dfn : (const void *)afn;
  if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_bytes)) != hipSuccess) return e;
  int per_cu = 0;
  const int agg_block = 64 * (p.det ? kPartWaves : kPartWavesNd);
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, agg_block, p.lds_bytes)) != hipSuccess)
    return e;
  const int agg_grid = std::max(1, env.n_cu * std::max(1, per_cu));
  if (p.det) {
    uint64_t *partial = (uint64_t *)(base + p.off_partial);
    hipLaunchKernelGGL(dfn, dim3(agg_grid), dim3(64 * kPartWaves), (size_t)p.lds_bytes, env.stream, st, in.n_icols,
                       in.n_fcols, p.n_slots, p.SB, p.slot_words, p.cap, rec_slot, rec_mk, rec_iv, rec_fv, items, meta,
                       partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t threads = p.n_parts * (p.slot_words << p.SB);
    hipLaunchKernelGGL(part_reduce_det, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, env.stream, st,
                       in.n_icols, in.n_fcols, in.m, p.n_slots, p.SB, p.slot_words, p.n_parts,
                       (const int64_t *)(base + p.off_pfirst), partial, fresh ? 1 : 0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(afn, dim3(agg_grid), dim3(agg_block), (size_t)p.lds_bytes, env.stream, st, in.n_icols,
                     in.n_fcols, p.n_slots, p.SB, p.slot_words, p.cap, rec_slot, rec_mk, rec_iv, rec_fv, items, meta,
                     fresh ? 1 : 0);
  return hipGetLastError();
}

}  // namespace pac
