// a2-a6 on the int8 matrix cores (gfx950 v_mfma_i32_16x16x64_i8).
//
// For one group g, world j and int column c the stochastic SUM is the
// contraction  S[g][c][j] = sum_r bit_j(r) * [grp(r) = g] * v_c(r)  (the
// per-world sum of Sec. 4.2's pac_agg).  Writing v - lo = sum_s 256^s byte_s
// turns it into an exact int8 product of two 0/1 / byte matrices:
//   A[j][r]        = bit j of row r's PU vector          (M = worlds)
//   B[r][(g,c,s)]  = [grp(r)=g] * (byte_s(v_c(r)-lo_c) - 128)   (N = group x digit)
//   B[r][(g,cnt)]  = [grp(r)=g]                            (COUNT column)
// C = A x B accumulates in int32 (|entry| <= 128 per row; a wave flushes long
// before 2^24 rows), and the flush recombines
//   S = sum_s 256^s (C[s] + 128 * COUNT) + lo * COUNT   (mod 2^64, exact).
// This replaces the paper's CPU SWAR / cascading 8-bit lanes (Sec. 5) with
// the matrix cores: the byte lanes become the int8 operands, the cascade into
// wide counters becomes the int32 accumulator flushed to int64.
//
// Data flow per wave and 256-row tile (four K-chunks of 64 rows):
//  * lane l gathers the PU words of rows 64u+l (u = 0..3) through the
//    foreign-key chain;
//  * inside each 16-lane group the 16x16 bit blocks of those words are
//    transposed (DPP / swizzle exchanges, rotate, bitfield insert) so that
//    lane (q,p) holds world 16t+p over rows 64u+16q..+15, then expanded to
//    0/1 bytes: the A operand;
//  * lane l loads rows 4l..4l+3 of the group and value columns with vector
//    loads, and writes byte planes to LDS: one plane per value digit, one
//    0xFF/0x00 plane per group, plus constant planes of ones and zeros;
//  * lane (q,p) reads 16 bytes of its column's digit plane and of its
//    column's group plane and ANDs them: the B operand;
//  * 4W x NT mfma per K-chunk.
#include "mfma_common.h"

namespace pac {

// byte b of four 32-bit words, packed into one word (word i -> byte i)
__device__ __forceinline__ uint32_t pack_byte(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, int b) {
  const uint32_t sel = (uint32_t)b | ((uint32_t)(b + 4) << 8) | 0x0C0C0000u;
  const uint32_t p01 = __builtin_amdgcn_perm(x1, x0, sel);
  const uint32_t p23 = __builtin_amdgcn_perm(x3, x2, sel);
  return __builtin_amdgcn_perm(p23, p01, 0x05040100u);
}

// Raw words of one tile in flight: PU words of rows 64u + lane and column
// words of rows 4*lane .. 4*lane + 3, exactly as loaded.
template <int W, int NI>
struct Raw {
  uint64_t mk[4][W];
  uint32_t ok[4];
  uint32_t g[kMG][4];
  uint32_t f[4];
  uint32_t v[NI > 0 ? NI : 1][8];
};

template <int SH, int W, int NI>
__device__ __forceinline__ void issue_words(const MfmaArgs &a, Chain c, Raw<W, NI> &r) {
  for (int k = 2; k < Shape<SH>::n_links(a); ++k) chain_level(a, k, c);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const bool v = c.ok[u] && c.idx[u] < a.n_idx;
    r.ok[u] = v;
    const uint32_t si = v ? c.idx[u] : 0u;
    if (Shape<SH>::masks(a)) {
#pragma unroll
      for (int w = 0; w < W; ++w) r.mk[u][w] = a.masks[(size_t)si * W + w];
    } else {
      r.mk[u][0] = (uint64_t)a.pu_keys[si];  // hashed when staged
    }
  }
}

// Column words of the full tile starting at row0 (no bounds checks).
template <int SH, int W, int NI>
__device__ __forceinline__ void issue_cols(const MfmaArgs &a, uint32_t row0, int lane, Raw<W, NI> &r) {
  const uint32_t r4 = row0 + 4 * lane;
#pragma unroll
  for (int k = 0; k < kMG; ++k) {
    if (k < a.n_gcols) {
      const int gb = a.gcol_bytes[k];
      const uint8_t *base = a.gcols[k] + (size_t)r4 * gb;
#pragma unroll
      for (int j = 0; j < 4; ++j) r.g[k][j] = *(const uint32_t *)(base + 4 * min(j, gb - 1));
    }
  }
  if (Shape<SH>::filter(a)) {
    const v4u32 w = __builtin_nontemporal_load((const v4u32 *)(a.filter_col + r4));
    r.f[0] = w[0]; r.f[1] = w[1]; r.f[2] = w[2]; r.f[3] = w[3];
  }
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    const int eb = a.icol_bytes[c];
    const uint8_t *base = a.icols[c] + (size_t)r4 * eb;
    const v4u32 x = __builtin_nontemporal_load((const v4u32 *)base);
    const v4u32 y = __builtin_nontemporal_load((const v4u32 *)(base + (eb == 8 ? 16 : 0)));
    r.v[c][0] = x[0]; r.v[c][1] = x[1]; r.v[c][2] = x[2]; r.v[c][3] = x[3];
    r.v[c][4] = y[0]; r.v[c][5] = y[1]; r.v[c][6] = y[2]; r.v[c][7] = y[3];
  }
}

// Column words of a partial tile (bounds-checked element loads).
template <int W, int NI>
__device__ __forceinline__ void issue_cols_tail(const MfmaArgs &a, uint32_t row0, int lane, Raw<W, NI> &r) {
  const uint32_t r4 = row0 + 4 * lane, n = a.n_rows;
#pragma unroll
  for (int k = 0; k < kMG; ++k) {
    if (k < a.n_gcols) {
      const int gb = a.gcol_bytes[k];
      uint32_t v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t row = r4 + i;
        v[i] = row < n ? (gb == 1 ? a.gcols[k][row] : gb == 2 ? ((const uint16_t *)a.gcols[k])[row]
                                                              : ((const uint32_t *)a.gcols[k])[row])
                       : 0u;
      }
      if (gb == 1) {
        r.g[k][0] = v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
      } else if (gb == 2) {
        r.g[k][0] = v[0] | (v[1] << 16);
        r.g[k][1] = v[2] | (v[3] << 16);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) r.g[k][i] = v[i];
      }
    }
  }
  if (a.filter_col) {
#pragma unroll
    for (int i = 0; i < 4; ++i) r.f[i] = r4 + i < n ? a.filter_col[r4 + i] : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    const int eb = a.icol_bytes[c];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t row = r4 + i;
      if (eb == 8) {
        const uint64_t x = row < n ? ((const uint64_t *)a.icols[c])[row] : 0ull;
        r.v[c][2 * i] = (uint32_t)x;
        r.v[c][2 * i + 1] = (uint32_t)(x >> 32);
      } else {
        r.v[c][i] = row < n ? ((const uint32_t *)a.icols[c])[row] : 0u;
      }
    }
  }
}

// Wave-private LDS staging of one tile's words, field-major ([field][lane])
// so that a wave's accesses hit consecutive banks.  Lane l stores and reads
// back only its own words: no cross-lane ordering is needed.
template <int W, int NI>
struct Stage {
  uint64_t mk[4][W][64];
  uint32_t g[kMG][4][64];
  uint32_t f[4][64];
  uint32_t v[NI > 0 ? NI : 1][8][64];
};

template <int SH, int W, int NI>
__device__ __forceinline__ void stage_store(Stage<W, NI> *sg, int lane, const MfmaArgs &a, const Raw<W, NI> &r) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (Shape<SH>::masks(a)) {
#pragma unroll
      for (int w = 0; w < W; ++w) sg->mk[u][w][lane] = r.ok[u] ? r.mk[u][w] : 0ull;
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w)
        sg->mk[u][w][lane] = r.ok[u] ? pu_word((int64_t)r.mk[u][0], a.qk, w, a.balanced != 0) : 0ull;
    }
  }
#pragma unroll
  for (int k = 0; k < kMG; ++k)
    if (k < a.n_gcols)
#pragma unroll
      for (int j = 0; j < 4; ++j) sg->g[k][j][lane] = r.g[k][j];
  if (Shape<SH>::filter(a))
#pragma unroll
    for (int j = 0; j < 4; ++j) sg->f[j][lane] = r.f[j];
#pragma unroll
  for (int c = 0; c < NI; ++c)
#pragma unroll
    for (int j = 0; j < 8; ++j) sg->v[c][j][lane] = r.v[c][j];
}

// ---------------------------------------------------------------- planes (B side)
// Group byte planes, row counts and digit planes of the staged tile.
template <int SH, int W, int NI>
__device__ __forceinline__ void build_planes(const MfmaArgs &a, const MfmaPlan &pl, const Stage<W, NI> *sg,
                                             uint32_t r4, uint8_t *planes, int64_t *blk, int nrows_off, int lane,
                                             uint32_t *status) {
  const uint32_t n = a.n_rows;
  const int G = pl.G, gplane0 = pl.D + 2;
  uint32_t gv[4] = {0, 0, 0, 0};
  bool ok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) ok[i] = r4 + i < n;
#pragma unroll
  for (int k = 0; k < kMG; ++k) {
    if (k < a.n_gcols) {
      const int gb = a.gcol_bytes[k];
      uint32_t x[4];
      if (gb == 1) {
        const uint32_t w = sg->g[k][0][lane];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = (w >> (8 * i)) & 0xFFu;
      } else if (gb == 2) {
        const uint32_t w0 = sg->g[k][0][lane], w1 = sg->g[k][1][lane];
        x[0] = w0 & 0xFFFFu; x[1] = w0 >> 16; x[2] = w1 & 0xFFFFu; x[3] = w1 >> 16;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = sg->g[k][i][lane];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ok[i] = ok[i] && x[i] < a.gcards[k];
        gv[i] = __umul24(gv[i], a.gcards[k]) + x[i];
      }
    }
  }
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) bad = bad || (r4 + i < n && !ok[i]);
  if (Shape<SH>::modulo(a)) {
#pragma unroll
    for (int i = 0; i < 4; ++i) gv[i] = gv[i] % a.group_mod;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) ok[i] = ok[i] && gv[i] < (uint32_t)G;
  if (Shape<SH>::filter(a)) {
#pragma unroll
    for (int i = 0; i < 4; ++i) ok[i] = ok[i] && sg->f[i][lane] < a.filter_lt;
  }
  if (bad) atomicOr(status, PAC_STATUS_BAD_GROUP);
  {  // a value outside the stated statistics would lose digits: the row updates nothing
    bool oor = false;
#pragma unroll
    for (int c = 0; c < NI; ++c) {
      const bool wide = a.icol_bytes[c] == 8;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint64_t v = wide ? (((uint64_t)sg->v[c][2 * i + 1][lane] << 32) | sg->v[c][2 * i][lane])
                                : (uint64_t)(int64_t)(int32_t)sg->v[c][i][lane];
        const bool out = v - (uint64_t)pl.lo[c] > pl.range[c];
        oor |= ok[i] && out;
        ok[i] = ok[i] && !out;
      }
    }
    if (oor) atomicOr(status, PAC_STATUS_OUT_OF_RANGE);
  }
  uint32_t gid4 = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) gid4 |= (ok[i] ? gv[i] : 0xFFu) << (8 * i);
  for (int g = 0; g < G; ++g) {
    const uint32_t x = gid4 ^ ((uint32_t)g * 0x01010101u);
    const uint32_t nz = (x | ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu)) & 0x80808080u;
    const uint32_t z = nz ^ 0x80808080u;
    const uint32_t gm = z | (z - (z >> 7));
    ((uint32_t *)(planes + (gplane0 + g) * kPlaneStride))[lane] = gm;
    const unsigned cnt = __popcll(__ballot(gm & 0xFF)) + __popcll(__ballot(gm & 0xFF00)) +
                         __popcll(__ballot(gm & 0xFF0000)) + __popcll(__ballot(gm & 0xFF000000u));
    if (lane == 0 && cnt) atomicAdd((unsigned long long *)&blk[nrows_off + g], (unsigned long long)cnt);
  }
#pragma unroll
  for (int c = 0; c < NI; ++c) {
    const bool wide = a.icol_bytes[c] == 8;
    uint32_t lo32[4], hi32[4];
    if (pl.dig[c] <= 4) {  // (v - lo) mod 2^32 already holds every non-zero byte
#pragma unroll
      for (int i = 0; i < 4; ++i) lo32[i] = sg->v[c][wide ? 2 * i : i][lane] - (uint32_t)pl.lo[c];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uint64_t x;
        if (wide)
          x = ((uint64_t)sg->v[c][2 * i + 1][lane] << 32) | sg->v[c][2 * i][lane];
        else
          x = (uint64_t)(int64_t)(int32_t)sg->v[c][i][lane];
        x -= (uint64_t)pl.lo[c];
        lo32[i] = (uint32_t)x;
        hi32[i] = (uint32_t)(x >> 32);
      }
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (s < pl.dig[c]) {
        const uint32_t word = s < 4 ? pack_byte(lo32[0], lo32[1], lo32[2], lo32[3], s)
                                    : pack_byte(hi32[0], hi32[1], hi32[2], hi32[3], s - 4);
        ((uint32_t *)(planes + (pl.doff[c] + s) * kPlaneStride))[lane] = word ^ 0x80808080u;
      }
    }
  }
}

// ---------------------------------------------------------------- matrix work (A side + mfma)
template <int W, int NT, int NI>
__device__ __forceinline__ void mfma_tile(const Stage<W, NI> *sg, int lane, const uint8_t *planes,
                                          const int (&boff_d)[NT], const int (&boff_g)[NT],
                                          const TransposeConsts &tcs, int q, v4i (&acc)[4 * W][NT]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    v4i av[4 * W];  // M-tile 4w + 2dw + h: word w, 32-bit half dw, bit-4 value h
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t word = sg->mk[u][w][lane];
#pragma unroll
      for (int dw = 0; dw < 2; ++dw) {
        const uint32_t t = transpose_word((uint32_t)(word >> (32 * dw)), tcs);
#pragma unroll
        for (int h = 0; h < 2; ++h)
          av[4 * w + 2 * dw + h] = v4i{(int)((t >> (4 * h)) & 0x01010101u), (int)((t >> (4 * h + 1)) & 0x01010101u),
                                      (int)((t >> (4 * h + 2)) & 0x01010101u), (int)((t >> (4 * h + 3)) & 0x01010101u)};
      }
    }
    const int roff = 64 * u + 16 * q;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const v4i dgt = *(const v4i *)(planes + boff_d[nt] + roff);
      const v4i gmk = *(const v4i *)(planes + boff_g[nt] + roff);
      const v4i b = dgt & gmk;
#pragma unroll
      for (int mt = 0; mt < 4 * W; ++mt)
        acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[mt], b, acc[mt][nt], 0, 0, 0);
    }
  }
}

template <int W, int NT>
__device__ __forceinline__ void flush_acc(v4i (&acc)[4 * W][NT], uint8_t *buf, int64_t *blk, const MfmaPlan &pl,
                                          int lane) {
  constexpr int m = 64 * W;
  const int q = lane >> 4, p = lane & 15;
  const int ncp = NT * 16;  // padded columns
  int32_t *R = (int32_t *)buf;
  const int ni = pl.ni, A = 1 + ni, GA = pl.G * A;
#pragma unroll
  for (int mt = 0; mt < 4 * W; ++mt) {
    wave_lds_fence();
    // acc[mt][nt] register r of lane (q,p) = C[M row 4q+r][column 16nt+p]
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) R[(4 * q + r) * ncp + nt * 16 + p] = acc[mt][nt][r];
    wave_lds_fence();
    const int wl = p;  // M row within this tile
    const int world = 64 * (mt >> 2) + 32 * ((mt >> 1) & 1) + world_of(wl, mt & 1);
    for (int gc = q; gc < GA; gc += 4) {
      const int g = gc / A, c = gc - g * A;
      const int base = g * (pl.D + 1);
      const int64_t cnt = R[wl * ncp + base + pl.D];
      int64_t val;
      if (c == ni) {
        val = cnt;
      } else {
        uint64_t s = (uint64_t)pl.lo[c] * (uint64_t)cnt;
        for (int d = 0; d < pl.dig[c]; ++d) {
          const int64_t a = (int64_t)R[wl * ncp + base + pl.doff[c] + d] + 128 * cnt;
          s += (uint64_t)a << (8 * d);
        }
        val = (int64_t)s;
      }
      if (val) atomicAdd((unsigned long long *)&blk[((int64_t)g * A + c) * m + world], (unsigned long long)val);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};
  }
  wave_lds_fence();
}

template <int SH, int W, int NT, int NI>
__global__ __launch_bounds__(256, (16 * W * NT > 64) ? 1 : 2) void agg_mfma(MfmaArgs a, MfmaPlan pl, DevState st,
                                                                          uint32_t *status) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, p = lane & 15;
  const int waves = blockDim.x >> 6;
  uint8_t *wbase = smem + wave * pl.wave_bytes;
  uint8_t *planes = wbase;
  Stage<W, NI> *stage = (Stage<W, NI> *)(wbase + pl.stage_off);
  int64_t *blk = (int64_t *)(smem + pl.blk_off);
  const int D = pl.D, G = pl.G;
  const int ones_plane = D, zero_plane = D + 1, gplane0 = D + 2;
  const int nrows_off = G * (1 + NI) * m;

  for (int i = threadIdx.x; i < pl.blk_words; i += blockDim.x) blk[i] = 0;
  ((uint32_t *)(planes + ones_plane * kPlaneStride))[lane] = 0x01010101u;
  ((uint32_t *)(planes + zero_plane * kPlaneStride))[lane] = 0u;
  __syncthreads();

  int boff_d[NT], boff_g[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = nt * 16 + p;
    if (n < pl.ncols) {
      const int g = n / (D + 1), t = n - g * (D + 1);
      boff_d[nt] = (t < D ? t : ones_plane) * kPlaneStride;
      boff_g[nt] = (gplane0 + g) * kPlaneStride;
    } else {
      boff_d[nt] = ones_plane * kPlaneStride;
      boff_g[nt] = zero_plane * kPlaneStride;
    }
  }
  const TransposeConsts tcs = transpose_consts(lane);

  v4i acc[4 * W][NT];
#pragma unroll
  for (int mt = 0; mt < 4 * W; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};

  const uint32_t n_full = a.n_rows / kTileRows;  // full tiles: pipelined, unchecked loads
  const uint32_t stride = gridDim.x * waves;
  const uint32_t first = blockIdx.x * waves + wave;
  const int nl = Shape<SH>::n_links(a);
  const int pre = nl < 2 ? nl : 2;  // chain levels gathered ahead
  if (first < n_full) {
    const uint32_t last = n_full - 1;
    auto clampt = [&](uint32_t t) { return t < n_full ? t : last; };
    uint32_t tile = first;
    {  // prologue: stage tile `first`
      Raw<W, NI> r;
      Chain c;
      chain_rows(a, tile * kTileRows, lane, c);
      for (int k = 0; k < pre; ++k) chain_level(a, k, c);
      issue_words<SH, W, NI>(a, c, r);
      issue_cols<SH, W, NI>(a, tile * kTileRows, lane, r);
      stage_store<SH, W, NI>(stage, lane, a, r);
    }
    Chain l1, l0;  // tile + stride after `pre` links, tile + 2 stride after one link
    chain_rows(a, clampt(tile + stride) * kTileRows, lane, l1);
    for (int k = 0; k < pre; ++k) chain_level(a, k, l1);
    chain_rows(a, clampt(tile + 2 * stride) * kTileRows, lane, l0);
    if (nl > 0) chain_level(a, 0, l0);
    for (; tile < n_full; tile += stride) {
      // ---- issue the next tile's words and the chain two and three tiles ahead
      Raw<W, NI> r;
      issue_words<SH, W, NI>(a, l1, r);
      issue_cols<SH, W, NI>(a, clampt(tile + stride) * kTileRows, lane, r);
      Chain n1 = l0;
      if (nl > 1) chain_level(a, 1, n1);
      chain_rows(a, clampt(tile + 3 * stride) * kTileRows, lane, l0);
      if (nl > 0) chain_level(a, 0, l0);
      // ---- tile t from the stage (its words were loaded during the previous tile)
      build_planes<SH, W, NI>(a, pl, stage, tile * kTileRows + 4 * lane, planes, blk, nrows_off, lane, status);
      wave_lds_fence();
      mfma_tile<W, NT, NI>(stage, lane, planes, boff_d, boff_g, tcs, q, acc);
      wave_lds_fence();
      stage_store<SH, W, NI>(stage, lane, a, r);
      l1 = n1;
    }
  }
  // ---- the partial last tile, if any, goes to the wave next in the tile order
  const uint32_t n_tiles = (a.n_rows + kTileRows - 1) / kTileRows;
  if (n_full < n_tiles && n_full % stride == first) {
    const uint32_t row0 = n_full * kTileRows;
    Raw<W, NI> r;
    Chain c;
    chain_rows(a, row0, lane, c);
    for (int k = 0; k < pre; ++k) chain_level(a, k, c);
    issue_words<SH, W, NI>(a, c, r);
    issue_cols_tail<W, NI>(a, row0, lane, r);
    stage_store<SH, W, NI>(stage, lane, a, r);
    build_planes<SH, W, NI>(a, pl, stage, row0 + 4 * lane, planes, blk, nrows_off, lane, status);
    wave_lds_fence();
    mfma_tile<W, NT, NI>(stage, lane, planes, boff_d, boff_g, tcs, q, acc);
    wave_lds_fence();
  }
  flush_acc<W, NT>(acc, planes, blk, pl, lane);
  __syncthreads();
  // block counters -> global state
  const int A = 1 + NI;
  for (int i = threadIdx.x; i < pl.blk_words; i += blockDim.x) {
    const int64_t v = blk[i];
    if (!v) continue;
    if (i >= nrows_off) {
      atomicAdd((unsigned long long *)&st.nrows[i - nrows_off], (unsigned long long)v);
      continue;
    }
    const int g = i / (A * m), rem = i - g * A * m, c = rem / m, j = rem - c * m;
    unsigned long long *dst = c == NI ? (unsigned long long *)&st.count[(int64_t)g * m + j]
                                      : (unsigned long long *)&st.isum[((int64_t)g * NI + c) * m + j];
    atomicAdd(dst, (unsigned long long)v);
  }
}

static bool mfma_plan(const DevInput &in, MfmaPlan *pl, int *nt_out) {
  if (in.group_keys || in.n_fcols > 0) return false;
  if (in.n_icols > kMC || in.n_gcols > kMG || in.n_links > kMC) return false;
  // 32-bit row and table indices; every table non-empty (invalid lanes read index 0)
  const int64_t lim = (int64_t)1 << 31;
  for (int k = 0; k < in.n_links; ++k)
    if (in.link_len[k] >= lim || in.link_len[k] < 1) return false;
  const int64_t n_idx = in.masks ? in.n_masks : in.n_pu_keys;
  if (n_idx >= lim || n_idx < 1) return false;
  for (int k = 0; k < in.n_gcols; ++k)
    if (in.gcards[k] >= (1 << 24)) return false;
  int64_t G = 1;
  if (in.n_gcols > 0 || in.group_mod > 0) G = in.n_groups;
  if (G < 1 || G > 254 || in.n_groups != G) return false;
  MfmaPlan p{};
  p.G = (int)G;
  p.ni = in.n_icols;
  int D = 0;
  for (int c = 0; c < in.n_icols; ++c) {
    p.dig[c] = in.icol_digits[c];
    p.doff[c] = D;
    p.lo[c] = in.icol_lo[c];
    p.range[c] = in.icol_range[c];
    D += p.dig[c];
  }
  p.D = D;
  p.ncols = p.G * (D + 1);
  int NT = (p.ncols + 15) / 16;  // rounded up to an instantiated tile count
  if (NT == 5 || NT == 7) ++NT;
  if (in.W == 2 && NT == 3) NT = 4;
  const int max_nt = in.W == 1 ? kMaxNT : kMaxNT / 2;
  if (NT > max_nt) return false;
  const int planes_bytes = (D + 2 + p.G) * kPlaneStride;
  const int flush_bytes = 16 * NT * 16 * 4;
  p.stage_off = (std::max(planes_bytes, flush_bytes) + 15) & ~15;
  const int stage_bytes = 64 * (8 * 4 * in.W + 4 * (4 * kMG + 4 + 8 * std::max(p.ni, 1)));  // sizeof(Stage<W, NI>)
  p.wave_bytes = (p.stage_off + stage_bytes + 15) & ~15;
  p.blk_off = 4 * p.wave_bytes;
  p.blk_words = p.G * (1 + p.ni) * in.m + p.G;
  p.flush_tiles = (1 << 23) / kTileRows;  // |accumulator| <= 128 * rows < 2^31
  *pl = p;
  *nt_out = NT;
  return p.blk_off + p.blk_words * 8 <= 160 * 1024;
}

bool mfma_supported(const DevInput &in) {
  MfmaPlan p;
  int nt;
  return mfma_plan(in, &p, &nt);
}

template <int SH, int W, int NT, int NI>
static hipError_t launch_mfma_t(const LaunchEnv &env, const DevInput &in, const DevState &st, const MfmaPlan &pl) {
  static_assert(sizeof(Stage<W, NI>) == 64 * (8 * 4 * W + 4 * (4 * kMG + 4 + 8 * (NI > 0 ? NI : 1))), "stage");
  const int lds = pl.blk_off + pl.blk_words * 8;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const void *fn = (const void *)agg_mfma<SH, W, NT, NI>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds);
  if (e != hipSuccess) return e;
  per_cu = std::max(1, per_cu);
  if (env.blocks_per_cu > 0) per_cu = std::min(per_cu, env.blocks_per_cu);
  const int64_t n_tiles = (in.n_rows + kTileRows - 1) / kTileRows;
  const int64_t want = (n_tiles + 3) / 4;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)env.n_cu * per_cu));
  // each wave keeps int32 accumulators and 32-bit row indices: bound the rows of one launch
  const int64_t rows_per_launch =
      std::min<int64_t>((int64_t)blocks * 4 * pl.flush_tiles * kTileRows, (int64_t)1 << 30);
  for (int64_t r0 = 0; r0 < in.n_rows; r0 += rows_per_launch) {
    const int64_t nr = std::min<int64_t>(in.n_rows - r0, rows_per_launch);
    hipLaunchKernelGGL((agg_mfma<SH, W, NT, NI>), dim3(blocks), dim3(256), (size_t)lds, env.stream,
                       mfma_args(in, r0, nr), pl, st, env.status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The star shape: two FK links into a PU-word table, group columns only.
static bool star_shape(const DevInput &in) {
  return in.n_links == 2 && in.masks && !in.filter_col && in.group_mod == 0;
}

template <int W, int NT>
static hipError_t launch_mfma_ni(const LaunchEnv &env, const DevInput &in, const DevState &st, const MfmaPlan &pl) {
  if (W == 1 && star_shape(in) && pl.ni >= 1 && pl.ni <= 3) {
    switch (pl.ni) {
      case 1: return launch_mfma_t<1, W, NT, 1>(env, in, st, pl);
      case 2: return launch_mfma_t<1, W, NT, 2>(env, in, st, pl);
      default: return launch_mfma_t<1, W, NT, 3>(env, in, st, pl);
    }
  }
  switch (pl.ni) {
    case 0: return launch_mfma_t<0, W, NT, 0>(env, in, st, pl);
    case 1: return launch_mfma_t<0, W, NT, 1>(env, in, st, pl);
    case 2: return launch_mfma_t<0, W, NT, 2>(env, in, st, pl);
    case 3: return launch_mfma_t<0, W, NT, 3>(env, in, st, pl);
    default: return launch_mfma_t<0, W, NT, 4>(env, in, st, pl);
  }
}

hipError_t launch_agg_mfma(const LaunchEnv &env, const DevInput &in, const DevState &st) {
  if (in.n_rows <= 0) return hipSuccess;
  MfmaPlan pl;
  int nt;
  if (!mfma_plan(in, &pl, &nt)) return hipErrorInvalidValue;
  if (in.W == 1) {
    switch (nt) {
      case 1: return launch_mfma_ni<1, 1>(env, in, st, pl);
      case 2: return launch_mfma_ni<1, 2>(env, in, st, pl);
      case 3: return launch_mfma_ni<1, 3>(env, in, st, pl);
      case 4: return launch_mfma_ni<1, 4>(env, in, st, pl);
      case 6: return launch_mfma_ni<1, 6>(env, in, st, pl);
      default: return launch_mfma_ni<1, 8>(env, in, st, pl);
    }
  }
  switch (nt) {
    case 1: return launch_mfma_ni<2, 1>(env, in, st, pl);
    case 2: return launch_mfma_ni<2, 2>(env, in, st, pl);
    default: return launch_mfma_ni<2, 4>(env, in, st, pl);
  }
}

}  // namespace pac
