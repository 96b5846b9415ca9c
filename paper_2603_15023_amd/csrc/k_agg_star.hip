// a2-a6 on the int8 matrix cores, specialised for the star-schema scan of an
// aggregation-heavy report (Sec. 3.2's rewrite adds the FK joins fact ->
// orders -> PU; Sec. 4.2's per-world SUM/COUNT over the result):
//   * either two FK links into the PU-word table (the words come from
//     pac_hash_mask), or one FK link into a column that holds each order's PU
//     key (hashed here, per row: no gather into a PU table), or one FK link
//     into per-order PU words (pac_hash_mask of the orders' PU keys: the
//     clustered fact rows then read the words almost sequentially);
//   * one or two u8 group columns whose product of cardinalities is <= 8;
//   * NI int columns whose (v - lo) fits DIG <= 4 bytes (host statistics).
// The contraction is the one of the generic matrix-core kernel
// (S = sum_s 256^s (C_s + 128 CNT) + lo CNT, C_s = A x B_s in int32); what
// changes is that every shape decision is made at compile time, which keeps
// the kernel free of runtime branches and of scalar-register spills, and:
//   * the group one-hot planes are one byte lookup (v_perm) of the row's
//     group id per group, and the per-group row counts are popcounts of those
//     planes accumulated in registers;
//   * the A operand of M-tile h is (T >> k) & (0x01010101 << 4h): worlds of
//     the upper half-nibble enter as 16 instead of 1, and their accumulators
//     are divided by 16 (exactly) when flushed;
//   * the byte and half-word stages of the bit transpose are single v_perm
//     instructions.
#include "mfma_common.h"

namespace pac {

constexpr int kStarGM = 8;   // groups per scan (byte lookup into an 8-byte table)
constexpr int kStarWPB = 4;  // waves per block
constexpr int kStarTPI = 1;  // tiles per loop iteration of a wave (loads in flight)

struct StarPlan {
  int32_t kv;            // 0: two links into PU words; 1: one link into per-order PU keys, hashed in the
                         // kernel; 2: one link into per-order PU words (the keys hashed beforehand)
  int32_t G;
  uint32_t lo[kMC];      // low 32 bits of each column's offset (all digits sit in (v - lo) mod 2^32)
  int64_t lo64[kMC];     // the offset itself, for the recombination
  uint32_t range[kMC];   // max - lo of the statistics (< 2^24): a larger (v - lo) is out of range
  uint32_t card_rep[2];  // gcards[k] * 0x01010101
  uint32_t card1;        // cardinality of the second group column (1 if absent)
  int32_t n_planes;      // D + 3 + G
  int32_t wave_bytes;
  int32_t stage_off;
  int32_t blk_off;
  int32_t blk_words;
  int32_t flush_tiles;
};

// Wave-private staging of one tile, field-major ([field][lane]).  The PU
// words stay in registers (see QChain), except in the variants with six
// column tiles (MK), whose accumulators leave no room for them: there lane l
// gathers the words of rows qrow(l, 0..3) and stages them here at plane
// positions 4 l .. 4 l + 3.
template <int NGC, int NI, bool MK>
struct StarStage {
  uint32_t g[NGC][64];   // group bytes of rows qrow(lane, 0..3)
  uint32_t v[NI][4][64]; // low 32 bits of the values of row qrow(lane, i)
  uint32_t rv[64];       // non-zero: a value of one of the lane's rows lies outside the statistics
  uint64_t mk[MK ? 256 : 1];
};

// Row order inside a tile.  Lane l handles the rows 2l, 2l + 1, 128 + 2l and
// 129 + 2l of the value and group columns, so that every column load of the
// wave reads one contiguous stretch of the column; those rows sit at
// positions 4l .. 4l + 3 of the byte planes (the contraction only needs the
// two operands to agree on the order).
__device__ __forceinline__ uint32_t qrow(int lane, int j) {
  return (j < 2 ? 0u : 128u) + 2u * lane + (uint32_t)(j & 1);
}

// The row at plane position 64 u + l, whose PU word lane l holds for K-chunk
// u of the contraction: qrow(16 u + l / 4, l mod 4).
__device__ __forceinline__ uint32_t wrow(int lane, int u) {
  return ((lane & 2) ? 128u : 0u) + 32u * u + 2u * (uint32_t)(lane >> 2) + (uint32_t)(lane & 1);
}

// FK chain of the four rows of a tile that the lane gathers words for
// (wrow(lane, 0..3), or qrow(lane, 0..3) with MK): table indices and
// validity.  Every load is unconditional: an invalid row reads index 0 of the
// (non-empty) table and stays marked invalid; a foreign key outside its
// table also raises PAC_STATUS_BAD_LINK.  Without MK the words found at the
// end of the chain stay in the lane's registers, already in the order of the
// A operand (no staging through LDS).
struct QChain {
  uint32_t idx[4];
  uint32_t ok[4];
};

// First link of a full tile: each load of the wave reads two runs of 32
// consecutive foreign keys (with MK: the lane's four keys in two 8-byte loads).
template <bool MK>
__device__ __forceinline__ void qchain_first(const MfmaArgs &a, uint32_t row0, int lane, QChain &c) {
  if constexpr (MK) {
    const v2u32 f0 = __builtin_nontemporal_load((const v2u32 *)(a.links[0] + row0 + 2 * lane));
    const v2u32 f1 = __builtin_nontemporal_load((const v2u32 *)(a.links[0] + row0 + 128 + 2 * lane));
    c.idx[0] = f0[0];
    c.idx[1] = f0[1];
    c.idx[2] = f1[0];
    c.idx[3] = f1[1];
#pragma unroll
    for (int j = 0; j < 4; ++j) c.ok[j] = 1u;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c.idx[u] = (uint32_t)__builtin_nontemporal_load(a.links[0] + row0 + wrow(lane, u));
      c.ok[u] = 1u;
    }
  }
}

// First link of a partial tile (rows >= n invalid).
template <bool MK>
__device__ __forceinline__ void qchain_first_tail(const MfmaArgs &a, uint32_t row0, int lane, QChain &c) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint32_t r = row0 + (MK ? qrow(lane, u) : wrow(lane, u));
    c.ok[u] = r < a.n_rows && r < a.link_len[0];
    c.idx[u] = (uint32_t)a.links[0][c.ok[u] ? r : 0u];
  }
}

__device__ __forceinline__ void qchain_next(const MfmaArgs &a, QChain &c, uint32_t *status) {
  const int32_t *lk = a.links[1];
  const uint32_t len = a.link_len[1];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool in = c.idx[j] < len;
    bad |= c.ok[j] && !in;
    c.ok[j] = c.ok[j] && in;
    c.idx[j] = (uint32_t)lk[c.ok[j] ? c.idx[j] : 0u];
  }
  if (bad) atomicOr(status, PAC_STATUS_BAD_LINK);
}

template <int NGC, int NI>
struct StarRaw {
  uint64_t mk[4];
  uint32_t ok[4];
  uint32_t g[NGC];
  uint32_t v[NI][4];
  uint32_t rv;  // see StarStage::rv
};

// Range check of one column's four values (lo and hi words): non-zero when
// some (v - lo), taken as a 64-bit unsigned number, exceeds the range.
__device__ __forceinline__ uint32_t star_range4(const uint32_t (&vl)[4], const uint32_t (&vh)[4], int64_t lo,
                                                uint32_t range) {
  uint32_t hor = 0, lmax = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t d = (((uint64_t)vh[i] << 32) | vl[i]) - (uint64_t)lo;
    hor |= (uint32_t)(d >> 32);
    lmax = max(lmax, (uint32_t)d);
  }
  return hor | (lmax > range ? 1u : 0u);
}

// Transpose constants of one lane: the two bit stages use rotate + bitfield
// insert, the byte and half-word stages a byte permutation.
struct StarTc {
  uint32_t keep0, rot0, keep1, rot1, sel2, sel3;
};

__device__ __forceinline__ StarTc star_tc(int lane) {
  StarTc t;
  const bool lo0 = (lane & 4) == 0, lo1 = (lane & 8) == 0;
  t.keep0 = lo0 ? 0x55555555u : 0xAAAAAAAAu;
  t.rot0 = lo0 ? 31u : 1u;
  t.keep1 = lo1 ? 0x33333333u : 0xCCCCCCCCu;
  t.rot1 = lo1 ? 30u : 2u;
  // lane bit 0 <-> position bit 3: the lower lane keeps bytes 0, 2 and takes the
  // partner's bytes 0, 2 into 1, 3; the upper lane the mirror image.
  t.sel2 = (lane & 1) ? 0x03070105u : 0x06020400u;
  // lane bit 1 <-> position bit 4, on half-words.
  t.sel3 = (lane & 2) ? 0x03020706u : 0x05040100u;
  return t;
}

// Same permutation of bits as transpose_word (bit position k + 4h + 8j of
// lane i ends up holding row 4k + j of world world_of(i, h)).
__device__ __forceinline__ uint32_t star_transpose(uint32_t x, const StarTc &tc) {
  uint32_t p = dpp_xor4(x);
  x = bfi(tc.keep0, x, __builtin_amdgcn_alignbit(p, p, tc.rot0));
  p = dpp_xor8(x);
  x = bfi(tc.keep1, x, __builtin_amdgcn_alignbit(p, p, tc.rot1));
  p = dpp_xor1(x);
  x = __builtin_amdgcn_perm(p, x, tc.sel2);
  p = dpp_xor2(x);
  x = __builtin_amdgcn_perm(p, x, tc.sel3);
  return x;
}

// PU words (KV = 0, 2) or PU keys (KV = 1, hashed by star_words) of the lane's four rows.
template <int KV, int NGC, int NI>
__device__ __forceinline__ void star_issue_words(const MfmaArgs &a, const QChain &c, StarRaw<NGC, NI> &r,
                                                 uint32_t *status) {
  bool bad = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool in = c.idx[j] < a.n_idx;
    bad |= c.ok[j] && !in;
    r.ok[j] = c.ok[j] && in;
    const uint32_t i = r.ok[j] ? c.idx[j] : 0u;
    r.mk[j] = KV == 1 ? (uint64_t)a.pu_keys[i] : a.masks[i];
  }
  if (bad) atomicOr(status, PAC_STATUS_BAD_LINK);
}

// Column words of the full tile at row0 (no bounds checks).
template <int NGC, int NI>
__device__ __forceinline__ void star_issue_cols(const MfmaArgs &a, const StarPlan &pl, uint32_t row0, int lane,
                                                StarRaw<NGC, NI> &r) {
  const uint32_t ra = row0 + 2 * lane, rb = row0 + 128 + 2 * lane;
  uint32_t rv = 0;
#pragma unroll
  for (int k = 0; k < NGC; ++k) {
    const uint32_t g0 = __builtin_nontemporal_load((const uint16_t *)(a.gcols[k] + ra));
    const uint32_t g1 = __builtin_nontemporal_load((const uint16_t *)(a.gcols[k] + rb));
    r.g[k] = g0 | (g1 << 16);
  }
#pragma unroll
  for (int c = 0; c < NI; ++c) {  // low words of rows ra, ra + 1 and rb, rb + 1
    const v4u32 x = __builtin_nontemporal_load((const v4u32 *)(a.icols[c] + (size_t)ra * 8));
    const v4u32 y = __builtin_nontemporal_load((const v4u32 *)(a.icols[c] + (size_t)rb * 8));
    r.v[c][0] = x[0];
    r.v[c][1] = x[2];
    r.v[c][2] = y[0];
    r.v[c][3] = y[2];
    const uint32_t vh[4] = {x[1], x[3], y[1], y[3]};
    rv |= star_range4(r.v[c], vh, pl.lo64[c], pl.range[c]);
  }
  r.rv = rv;
}

// Column words of a partial tile (rows >= n read as zero).
template <int NGC, int NI>
__device__ __forceinline__ void star_issue_cols_tail(const MfmaArgs &a, const StarPlan &pl, uint32_t row0, int lane,
                                                     StarRaw<NGC, NI> &r) {
  const uint32_t n = a.n_rows;
#pragma unroll
  for (int k = 0; k < NGC; ++k) {
    uint32_t w = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t row = row0 + qrow(lane, j);
      w |= (row < n ? (uint32_t)a.gcols[k][row] : 0u) << (8 * j);
    }
    r.g[k] = w;
  }
  uint32_t rv = 0;
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    uint32_t vh[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // rows past the end read as lo: never out of range
      const uint32_t row = row0 + qrow(lane, j);
      const uint64_t x = row < n ? ((const uint64_t *)a.icols[c])[row] : (uint64_t)pl.lo64[c];
      r.v[c][j] = (uint32_t)x;
      vh[j] = (uint32_t)(x >> 32);
    }
    rv |= star_range4(r.v[c], vh, pl.lo64[c], pl.range[c]);
  }
  r.rv = rv;
}

// The A-operand words of a staged tile (hashed here for KV = 1), zero for an
// invalid row: word u of row wrow(lane, u) kept in wk, or (MK) the words of
// rows qrow(lane, 0..3) staged at plane positions 4 lane .. 4 lane + 3.
template <int KV, int NGC, int NI, bool MK>
__device__ __forceinline__ void star_words(const MfmaArgs &a, const StarRaw<NGC, NI> &r, StarStage<NGC, NI, MK> *sg,
                                           int lane, uint64_t (&wk)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint64_t w = KV == 1 ? pu_word((int64_t)r.mk[u], a.qk, 0, a.balanced != 0) : r.mk[u];
    if constexpr (MK)
      sg->mk[4 * lane + u] = r.ok[u] ? w : 0ull;
    else
      wk[u] = r.ok[u] ? w : 0ull;
  }
}

template <int NGC, int NI, bool MK>
__device__ __forceinline__ void star_stage_store(StarStage<NGC, NI, MK> *sg, int lane, const StarRaw<NGC, NI> &r) {
#pragma unroll
  for (int k = 0; k < NGC; ++k) sg->g[k][lane] = r.g[k];
#pragma unroll
  for (int c = 0; c < NI; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) sg->v[c][i][lane] = r.v[c][i];
  sg->rv[lane] = r.rv;
}

// Per-byte flag 0x80 where byte >= card (card <= 128), else 0.
__device__ __forceinline__ uint32_t bytes_ge(uint32_t w, uint32_t card_rep) {
  return (w | ((w | 0x80808080u) - card_rep)) & 0x80808080u;
}

// Byte planes of the staged tile: digits, then (after the ones and zeros
// planes) one 0xFF/0x00 plane per group; counts rows per group.
template <int NGC, int NI, int DIG, bool MK>
__device__ __forceinline__ void star_planes(const MfmaArgs &a, const StarPlan &pl, const StarStage<NGC, NI, MK> *sg,
                                            uint32_t row0, bool tail, uint8_t *planes, int lane,
                                            uint32_t (&gcnt)[kStarGM], uint32_t *status) {
  constexpr int D = NI * DIG;
  // group id of each of the 4 rows, one per byte; rows that update nothing get 0x0C
  uint32_t bad = 0, gid;
  {
    const uint32_t w0 = sg->g[0][lane];
    bad = bytes_ge(w0, pl.card_rep[0]);
    if (NGC == 2) {
      const uint32_t w1 = sg->g[1][lane];
      bad |= bytes_ge(w1, pl.card_rep[1]);
      const uint32_t badb = bad | (bad - (bad >> 7));
      gid = (w0 & ~badb) * pl.card1 + (w1 & ~badb);  // bytes stay < G <= 8: no carries
    } else {
      gid = w0;
    }
  }
  uint32_t off = bad;  // rows that update nothing
  if (tail) {
    uint32_t past = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) past |= (row0 + qrow(lane, i) >= a.n_rows ? 0x80u : 0u) << (8 * i);
    bad &= ~past;
    off |= past;
  }
  if (bad) atomicOr(status, PAC_STATUS_BAD_GROUP);
  if (sg->rv[lane]) {  // rare: find the lane's rows whose values lie outside the statistics; they update nothing
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t row = row0 + qrow(lane, i);
      bool out = false;
      if (row < a.n_rows)
#pragma unroll
        for (int c = 0; c < NI; ++c)
          out |= ((const uint64_t *)a.icols[c])[row] - (uint64_t)pl.lo64[c] > (uint64_t)pl.range[c];
      off |= out ? 0x80u << (8 * i) : 0u;
    }
    atomicOr(status, PAC_STATUS_OUT_OF_RANGE);
  }
  const uint32_t offb = off | (off - (off >> 7));
  gid = bfi(offb, 0x0C0C0C0Cu, gid);
#pragma unroll
  for (int g = 0; g < kStarGM; ++g) {
    const uint32_t tlo = g < 4 ? 0xFFu << (8 * g) : 0u, thi = g >= 4 ? 0xFFu << (8 * (g - 4)) : 0u;
    const uint32_t gm = __builtin_amdgcn_perm(thi, tlo, gid);
    // groups past G write to one spare plane that no column reads
    ((uint32_t *)(planes + (D + 2 + min(g, pl.G)) * kPlaneStride))[lane] = gm;
    gcnt[g] += __popc(gm);
  }
  // digit planes: byte s of (v - lo) for the 4 rows, as int8 (xor 0x80 = minus 128)
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    uint32_t x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = sg->v[c][i][lane] - pl.lo[c];
    uint32_t w[4];
    {
      const uint32_t t01 = __builtin_amdgcn_perm(x[1], x[0], 0x05010400u);
      const uint32_t t23 = __builtin_amdgcn_perm(x[3], x[2], 0x05010400u);
      w[0] = __builtin_amdgcn_perm(t23, t01, 0x05040100u);
      w[1] = __builtin_amdgcn_perm(t23, t01, 0x07060302u);
    }
    if (DIG > 2) {
      const uint32_t t01 = __builtin_amdgcn_perm(x[1], x[0], 0x07030602u);
      const uint32_t t23 = __builtin_amdgcn_perm(x[3], x[2], 0x07030602u);
      w[2] = __builtin_amdgcn_perm(t23, t01, 0x05040100u);
      w[3] = __builtin_amdgcn_perm(t23, t01, 0x07060302u);
    }
#pragma unroll
    for (int s = 0; s < DIG; ++s)
      ((uint32_t *)(planes + (c * DIG + s) * kPlaneStride))[lane] = w[s] ^ 0x80808080u;
  }
}

// A operands of K-chunk u from the lane's word of plane position 64 u + lane:
// M-tile 2 dw + h holds the worlds of word half dw whose transposed bit sits
// in nibble half h (scaled by 16^h).
__device__ __forceinline__ void star_a(uint64_t word, const StarTc &tc, v4i (&av)[4]) {
#pragma unroll
  for (int dw = 0; dw < 2; ++dw) {
    const uint32_t t0 = star_transpose((uint32_t)(word >> (32 * dw)), tc);
    const uint32_t t1 = t0 >> 1, t2 = t0 >> 2, t3 = t0 >> 3;
    av[2 * dw] = v4i{(int)(t0 & 0x01010101u), (int)(t1 & 0x01010101u), (int)(t2 & 0x01010101u),
                     (int)(t3 & 0x01010101u)};
    av[2 * dw + 1] = v4i{(int)(t0 & 0x10101010u), (int)(t1 & 0x10101010u), (int)(t2 & 0x10101010u),
                         (int)(t3 & 0x10101010u)};
  }
}

// Digit and group-mask rows of K-chunk u for this lane's columns.
template <int NT>
__device__ __forceinline__ void star_b(const uint8_t *planes, int roff, const int (&boff_d)[NT],
                                       const int (&boff_g)[NT], v4i (&d)[NT], v4i (&g)[NT]) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    d[nt] = *(const v4i *)(planes + boff_d[nt] + roff);
    g[nt] = *(const v4i *)(planes + boff_g[nt] + roff);
  }
}

// The four K-chunks of a tile, software-pipelined: the B rows of chunk u + 1
// are read and the A operands of chunk u + 1 built while the matrix cores
// work on chunk u.
template <int NGC, int NI, bool MK, int NT>
__device__ __forceinline__ void star_mfma(const uint64_t (&wk)[4], const StarStage<NGC, NI, MK> *sg, int lane,
                                          const uint8_t *planes, const int (&boff_d)[NT], const int (&boff_g)[NT],
                                          const StarTc &tc, int q, v4i (&acc)[4][NT]) {
  auto word = [&](int u) -> uint64_t {
    if constexpr (MK)
      return sg->mk[64 * u + lane];
    else
      return wk[u];
  };
  v4i av[2][4], bd[2][NT], bg[2][NT];
  star_b<NT>(planes, 16 * q, boff_d, boff_g, bd[0], bg[0]);
  star_a(word(0), tc, av[0]);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = u & 1, n = c ^ 1;
    if (u < 3) star_b<NT>(planes, 64 * (u + 1) + 16 * q, boff_d, boff_g, bd[n], bg[n]);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const v4i b = bd[c][nt] & bg[c][nt];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[c][mt], b, acc[mt][nt], 0, 0, 0);
    }
    if (u < 3) star_a(word(u + 1), tc, av[n]);
  }
}

// Accumulators -> block counters.  acc[mt][nt] register r of lane (q, p) is
// C[M row 4q + r][column 16 nt + p]; odd M-tiles carry a factor 16.
template <int NI, int DIG, int NT>
__device__ __forceinline__ void star_flush(v4i (&acc)[4][NT], uint8_t *buf, int64_t *blk, const StarPlan &pl,
                                           int lane) {
  constexpr int D = NI * DIG, A = 1 + NI, ncp = NT * 16;
  const int q = lane >> 4, p = lane & 15;
  int32_t *R = (int32_t *)buf;
  const int GA = pl.G * A;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    wave_lds_fence();
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) R[(4 * q + r) * ncp + nt * 16 + p] = acc[mt][nt][r] >> (4 * (mt & 1));
    wave_lds_fence();
    const int world = 32 * (mt >> 1) + world_of(p, mt & 1);
    for (int gc = q; gc < GA; gc += 4) {
      const int g = gc / A, c = gc - g * A;
      const int base = g * (D + 1);
      const int64_t cnt = R[p * ncp + base + D];
      int64_t val;
      if (c == NI) {
        val = cnt;
      } else {
        uint64_t s = (uint64_t)pl.lo64[c] * (uint64_t)cnt;
#pragma unroll
        for (int d = 0; d < DIG; ++d) {
          const int64_t x = (int64_t)R[p * ncp + base + c * DIG + d] + 128 * cnt;
          s += (uint64_t)x << (8 * d);
        }
        val = (int64_t)s;
      }
      if (val) atomicAdd((unsigned long long *)&blk[((int64_t)g * A + c) * 64 + world], (unsigned long long)val);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};
  }
  wave_lds_fence();
}

template <int KV, int NGC, int NI, int DIG, int NT>
__global__ __launch_bounds__(64 * kStarWPB, 2) void agg_star(MfmaArgs a, StarPlan pl, DevState st,
                                                           uint32_t *status) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  constexpr int D = NI * DIG, A = 1 + NI;
  constexpr bool MK = NT > 4;
  using Stage = StarStage<NGC, NI, MK>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, p = lane & 15;
  uint8_t *planes = smem + wave * pl.wave_bytes;
  Stage *stage = (Stage *)(planes + pl.stage_off);
  int64_t *blk = (int64_t *)(smem + pl.blk_off);
  const int G = pl.G;
  const int nrows_off = G * A * 64;

  for (int i = threadIdx.x; i < pl.blk_words; i += blockDim.x) blk[i] = 0;
  ((uint32_t *)(planes + D * kPlaneStride))[lane] = 0x01010101u;  // COUNT digit
  ((uint32_t *)(planes + (D + 1) * kPlaneStride))[lane] = 0u;     // padding columns
  __syncthreads();

  int boff_d[NT], boff_g[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = nt * 16 + p;
    if (n < G * (D + 1)) {
      const int g = n / (D + 1), t = n - g * (D + 1);
      boff_d[nt] = t * kPlaneStride;  // t == D: the ones plane
      boff_g[nt] = (D + 2 + g) * kPlaneStride;
    } else {
      boff_d[nt] = D * kPlaneStride;
      boff_g[nt] = (D + 1) * kPlaneStride;
    }
  }
  const StarTc tc = star_tc(lane);
  uint32_t gcnt[kStarGM];
#pragma unroll
  for (int g = 0; g < kStarGM; ++g) gcnt[g] = 0;
  v4i acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};

  // Tiles go to the waves in groups of kStarTPI consecutive tiles, group g to
  // wave g mod stride; the loads of the next group (kStarTPI tiles of columns
  // and PU words) are in flight while the current group is contracted, and
  // the foreign keys of the two groups after it before that, so each wave
  // keeps several tiles of HBM traffic outstanding.
  const uint32_t n_full = a.n_rows / kTileRows;
  const uint32_t n_grp = n_full / kStarTPI;
  const uint32_t stride = gridDim.x * kStarWPB;
  const uint32_t first = blockIdx.x * kStarWPB + wave;
  if (first < n_grp) {
    const uint32_t last = n_grp - 1;
    auto clampg = [&](uint32_t g) { return g < n_grp ? g : last; };
    auto row_of = [&](uint32_t g, int k) { return (g * kStarTPI + k) * kTileRows; };
    uint32_t gi = first;
    uint64_t wk[kStarTPI][4];  // A-operand words of the staged tiles (registers unless MK)
#pragma unroll
    for (int k = 0; k < kStarTPI; ++k) {  // prologue: stage group `first`
      StarRaw<NGC, NI> r;
      QChain c;
      qchain_first<MK>(a, row_of(gi, k), lane, c);
      if (KV == 0) qchain_next(a, c, status);
      star_issue_words<KV>(a, c, r, status);
      star_issue_cols(a, pl, row_of(gi, k), lane, r);
      star_stage_store(stage + k, lane, r);
      star_words<KV>(a, r, stage + k, lane, wk[k]);
    }
    QChain l1[kStarTPI], l0[kStarTPI];  // group + stride after both links, group + 2 stride after the first
#pragma unroll
    for (int k = 0; k < kStarTPI; ++k) {
      qchain_first<MK>(a, row_of(clampg(gi + stride), k), lane, l1[k]);
      if (KV == 0) qchain_next(a, l1[k], status);
      qchain_first<MK>(a, row_of(clampg(gi + 2 * stride), k), lane, l0[k]);
    }
    for (; gi < n_grp; gi += stride) {
      StarRaw<NGC, NI> r[kStarTPI];
      QChain n1[kStarTPI];
#pragma unroll
      for (int k = 0; k < kStarTPI; ++k) {
        star_issue_words<KV>(a, l1[k], r[k], status);
        star_issue_cols(a, pl, row_of(clampg(gi + stride), k), lane, r[k]);
      }
#pragma unroll
      for (int k = 0; k < kStarTPI; ++k) {
        n1[k] = l0[k];
        if (KV == 0) qchain_next(a, n1[k], status);
        qchain_first<MK>(a, row_of(clampg(gi + 3 * stride), k), lane, l0[k]);
      }
#pragma unroll
      for (int k = 0; k < kStarTPI; ++k) {
        star_planes<NGC, NI, DIG>(a, pl, stage + k, row_of(gi, k), false, planes, lane, gcnt, status);
        wave_lds_fence();
        star_mfma(wk[k], stage + k, lane, planes, boff_d, boff_g, tc, q, acc);
        wave_lds_fence();
      }
#pragma unroll
      for (int k = 0; k < kStarTPI; ++k) {
        star_stage_store(stage + k, lane, r[k]);
        star_words<KV>(a, r[k], stage + k, lane, wk[k]);
        l1[k] = n1[k];
      }
    }
  }
  // tiles after the last full group (at most kStarTPI - 1 full ones and a
  // partial one), bounds-checked, tile T by wave T mod stride
  const uint32_t n_tiles = (a.n_rows + kTileRows - 1) / kTileRows;
  for (uint32_t T = n_grp * kStarTPI; T < n_tiles; ++T) {
    if (T % stride != first) continue;
    const uint32_t row0 = T * kTileRows;
    StarRaw<NGC, NI> r;
    QChain c;
    qchain_first_tail<MK>(a, row0, lane, c);
    if (KV == 0) qchain_next(a, c, status);
    star_issue_words<KV>(a, c, r, status);
    star_issue_cols_tail(a, pl, row0, lane, r);
    star_stage_store(stage, lane, r);
    uint64_t wt[4];
    star_words<KV>(a, r, stage, lane, wt);
    star_planes<NGC, NI, DIG>(a, pl, stage, row0, true, planes, lane, gcnt, status);
    wave_lds_fence();
    star_mfma(wt, stage, lane, planes, boff_d, boff_g, tc, q, acc);
    wave_lds_fence();
  }
  star_flush<NI, DIG, NT>(acc, planes, blk, pl, lane);
  // row counts: every matching row set 8 bits of its group's plane
#pragma unroll
  for (int g = 0; g < kStarGM; ++g) {
    if (g >= G) break;
    uint32_t s = gcnt[g];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && s) atomicAdd((unsigned long long *)&blk[nrows_off + g], (unsigned long long)(s >> 3));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < pl.blk_words; i += blockDim.x) {
    const int64_t v = blk[i];
    if (!v) continue;
    if (i >= nrows_off) {
      atomicAdd((unsigned long long *)&st.nrows[i - nrows_off], (unsigned long long)v);
      continue;
    }
    const int g = i / (A * 64), rem = i - g * A * 64, c = rem / 64, j = rem - c * 64;
    unsigned long long *dst = c == NI ? (unsigned long long *)&st.count[(int64_t)g * 64 + j]
                                      : (unsigned long long *)&st.isum[((int64_t)g * NI + c) * 64 + j];
    atomicAdd(dst, (unsigned long long)v);
  }
}

// ---------------------------------------------------------------- host side
static int star_digits(const DevInput &in) {
  int dig = 0;
  for (int c = 0; c < in.n_icols; ++c) dig = std::max(dig, (int)in.icol_digits[c]);
  return dig;
}

// The shapes this kernel takes; everything else goes to the generic form.
static bool star_plan(const DevInput &in, StarPlan *pl, int *nt_out) {
  if (in.W != 1 || in.filter_col || in.group_mod || in.group_keys) return false;
  const bool kv = in.n_links == 1 && !in.masks && in.pu_keys;  // orders carry the PU key
  const bool kw = in.n_links == 1 && in.masks;                  // orders carry their PU words
  if (!kv && !kw && !(in.n_links == 2 && in.masks)) return false;
  if (in.n_fcols > 0 || in.n_icols < 1 || in.n_icols > 3 || in.n_gcols != 2) return false;
  if (star_digits(in) != 3) return false;
  const int64_t lim = (int64_t)1 << 31;
  for (int k = 0; k < in.n_links; ++k)
    if (in.link_len[k] < 1 || in.link_len[k] >= lim) return false;
  // full tiles read the first link without bounds checks
  if (in.link_len[0] < in.n_rows) return false;
  const int64_t n_idx = kv ? in.n_pu_keys : in.n_masks;
  if (n_idx < 1 || n_idx >= lim) return false;
  for (int k = 0; k < in.n_gcols; ++k)
    if (in.gcol_type[k] != PAC_U8 || in.gcards[k] < 1 || in.gcards[k] > 128) return false;
  const int64_t G = in.gcards[0] * in.gcards[1];
  if (G > kStarGM || in.n_groups != G) return false;
  for (int c = 0; c < in.n_icols; ++c)
    if (in.icol_type[c] != PAC_I64) return false;
  StarPlan p{};
  p.kv = kv ? 1 : kw ? 2 : 0;
  p.G = (int)G;
  for (int c = 0; c < in.n_icols; ++c) {
    p.lo[c] = (uint32_t)in.icol_lo[c];
    p.lo64[c] = in.icol_lo[c];
    p.range[c] = (uint32_t)in.icol_range[c];  // < 2^24: three digits
  }
  p.card_rep[0] = (uint32_t)in.gcards[0] * 0x01010101u;
  p.card_rep[1] = (uint32_t)in.gcards[1] * 0x01010101u;
  p.card1 = (uint32_t)in.gcards[1];
  const int D = in.n_icols * 3;
  int NT = ((int)G * (D + 1) + 15) / 16;
  if (NT == 5) NT = 6;
  if (NT > 6) return false;
  // six tiles: full tiles read the first link in 8-byte loads
  if (NT > 4 && ((uintptr_t)in.links[0] & 7u)) return false;
  p.n_planes = D + 3 + (int)G;  // digits, ones, zeros, G groups, one spare
  const int planes_bytes = p.n_planes * kPlaneStride;
  const int flush_bytes = 16 * NT * 16 * 4;
  p.stage_off = (std::max(planes_bytes, flush_bytes) + 15) & ~15;
  const int stage_bytes = 64 * (4 * in.n_gcols + 16 * in.n_icols + 4) + (NT > 4 ? 256 * 8 : 8);
  p.wave_bytes = (p.stage_off + kStarTPI * stage_bytes + 15) & ~15;
  p.blk_off = kStarWPB * p.wave_bytes;
  p.blk_words = (int)G * (1 + in.n_icols) * 64 + (int)G;
  p.flush_tiles = (1 << 19) / kTileRows;  // |accumulator| <= 128 * 16 * rows < 2^31
  *pl = p;
  *nt_out = NT;
  return p.blk_off + p.blk_words * 8 <= 160 * 1024;
}

bool star_supported(const DevInput &in) {
  StarPlan p;
  int nt;
  return star_plan(in, &p, &nt);
}

template <int KV, int NGC, int NI, int DIG, int NT>
static hipError_t launch_star_t(const LaunchEnv &env, const DevInput &in, const DevState &st, const StarPlan &pl) {
  static_assert(sizeof(StarStage<NGC, NI, (NT > 4)>) == 64 * (4 * NGC + 16 * NI + 4) + (NT > 4 ? 256 * 8 : 8),
                "stage");
  const int lds = pl.blk_off + pl.blk_words * 8;
  const void *fn = (const void *)agg_star<KV, NGC, NI, DIG, NT>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kStarWPB, lds);
  if (e != hipSuccess) return e;
  per_cu = std::max(1, per_cu);
  if (env.blocks_per_cu > 0) per_cu = std::min(per_cu, env.blocks_per_cu);
  const int64_t n_tiles = (in.n_rows + kTileRows - 1) / kTileRows;
  const int64_t want = (n_tiles + kStarWPB * kStarTPI - 1) / (kStarWPB * kStarTPI);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)env.n_cu * per_cu));
  const int64_t rows_per_launch =
      std::min<int64_t>((int64_t)blocks * kStarWPB * pl.flush_tiles * kTileRows, (int64_t)1 << 30);
  for (int64_t r0 = 0; r0 < in.n_rows; r0 += rows_per_launch) {
    const int64_t nr = std::min<int64_t>(in.n_rows - r0, rows_per_launch);
    hipLaunchKernelGGL((agg_star<KV, NGC, NI, DIG, NT>), dim3(blocks), dim3(64 * kStarWPB), (size_t)lds, env.stream,
                       mfma_args(in, r0, nr), pl, st, env.status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int KV, int NI>
static hipError_t launch_star_nt(const LaunchEnv &env, const DevInput &in, const DevState &st, const StarPlan &pl,
                                 int nt) {
  switch (nt) {
    case 1: return launch_star_t<KV, 2, NI, 3, 1>(env, in, st, pl);
    case 2: return launch_star_t<KV, 2, NI, 3, 2>(env, in, st, pl);
    case 3: return launch_star_t<KV, 2, NI, 3, 3>(env, in, st, pl);
    case 4: return launch_star_t<KV, 2, NI, 3, 4>(env, in, st, pl);
    default: return launch_star_t<KV, 2, NI, 3, 6>(env, in, st, pl);
  }
}

template <int KV>
static hipError_t launch_star_kv(const LaunchEnv &env, const DevInput &in, const DevState &st, const StarPlan &pl,
                                 int nt) {
  switch (in.n_icols) {
    case 1: return launch_star_nt<KV, 1>(env, in, st, pl, nt);
    case 2: return launch_star_nt<KV, 2>(env, in, st, pl, nt);
    default: return launch_star_nt<KV, 3>(env, in, st, pl, nt);
  }
}

hipError_t launch_agg_star(const LaunchEnv &env, const DevInput &in, const DevState &st) {
  if (in.n_rows <= 0) return hipSuccess;
  StarPlan pl;
  int nt;
  if (!star_plan(in, &pl, &nt)) return hipErrorInvalidValue;
  switch (pl.kv) {
    case 1: return launch_star_kv<1>(env, in, st, pl, nt);
    case 2: return launch_star_kv<2>(env, in, st, pl, nt);
    default: return launch_star_kv<0>(env, in, st, pl, nt);
  }
}

}  // namespace pac
