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
#include <algorithm>

#include "pac_internal.h"

namespace pac {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned long long v2u64 __attribute__((ext_vector_type(2)));

constexpr int kTileRows = 256;
constexpr int kMaxNT = 8;

struct MfmaPlan {
  int32_t G;            // dense groups (<= 254)
  int32_t D;            // total digit planes
  int32_t ncols;        // G * (D + 1)
  int32_t ni;
  int32_t dig[kMaxCols];
  int32_t doff[kMaxCols];
  int64_t lo[kMaxCols];
  int32_t wave_bytes;   // per-wave LDS: planes, reused as the flush buffer
  int32_t blk_off;      // block-shared int64 counters [G][1+ni][m] + nrows[G]
  int32_t blk_words;
  int32_t flush_tiles;  // tiles between accumulator flushes (int32 headroom)
};

__device__ __forceinline__ uint32_t dpp_xor1(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}
__device__ __forceinline__ uint32_t dpp_xor2(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
}
__device__ __forceinline__ uint32_t swz_xor4(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x101F);  // bit mode: lane ^ 4
}
__device__ __forceinline__ uint32_t dpp_xor8(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false);  // row_ror:8 == lane ^ 8 in a row
}

// One exchange stage of the 16x16 bit transposes held in the two 16-bit
// halves of x: swap bit b of the lane index with bit b of the bit position.
template <int B>
__device__ __forceinline__ uint32_t tstage(uint32_t x, uint32_t partner, bool lower) {
  constexpr uint32_t lo_mask = B == 8 ? 0x00FF00FFu : B == 4 ? 0x0F0F0F0Fu : B == 2 ? 0x33333333u : 0x55555555u;
  const uint32_t keep = lower ? lo_mask : ~lo_mask;
  const uint32_t rot = __builtin_amdgcn_alignbit(partner, partner, lower ? 32 - B : B);
  return (keep & x) | (~keep & rot);
}

__device__ __forceinline__ uint32_t transpose16x2(uint32_t x, int lane) {
  x = tstage<8>(x, dpp_xor8(x), (lane & 8) == 0);
  x = tstage<4>(x, swz_xor4(x), (lane & 4) == 0);
  x = tstage<2>(x, dpp_xor2(x), (lane & 2) == 0);
  x = tstage<1>(x, dpp_xor1(x), (lane & 1) == 0);
  return x;
}

// 4 bits (positions sh..sh+3 of x) -> 4 bytes of 0/1
__device__ __forceinline__ int expand_nibble(uint32_t x, int sh) {
  const uint32_t nib = (x >> sh) & 0xFu;
  return (int)((__umul24(nib, 0x204081u)) & 0x01010101u);
}

// byte b of four 32-bit words, packed into one word (word i -> byte i)
__device__ __forceinline__ uint32_t pack_byte(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, int b) {
  const uint32_t sel = (uint32_t)b | ((uint32_t)(b + 4) << 8) | 0x0C0C0000u;
  const uint32_t p01 = __builtin_amdgcn_perm(x1, x0, sel);
  const uint32_t p23 = __builtin_amdgcn_perm(x3, x2, sel);
  return __builtin_amdgcn_perm(p23, p01, 0x05040100u);
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Loads 4 consecutive unsigned group values starting at row r0 (guarded tail).
__device__ __forceinline__ void load4_gcol(const void *p, int type, int64_t r0, int64_t n, uint32_t (&v)[4]) {
  if (r0 + 3 < n) {
    if (type == PAC_U8) {
      const uint32_t w = *(const uint32_t *)((const uint8_t *)p + r0);
      v[0] = w & 0xFF; v[1] = (w >> 8) & 0xFF; v[2] = (w >> 16) & 0xFF; v[3] = w >> 24;
    } else if (type == PAC_U16) {
      const uint2 w = *(const uint2 *)((const uint16_t *)p + r0);
      v[0] = w.x & 0xFFFF; v[1] = w.x >> 16; v[2] = w.y & 0xFFFF; v[3] = w.y >> 16;
    } else {
      const uint4 w = *(const uint4 *)((const uint32_t *)p + r0);
      v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = r0 + i < n ? load_gcol(p, type, r0 + i) : 0u;
  }
}

__device__ __forceinline__ void load4_icol(const void *p, int type, int64_t r0, int64_t n, uint64_t (&v)[4]) {
  if (r0 + 3 < n) {
    if (type == PAC_I32) {
      const v4i w = __builtin_nontemporal_load((const v4i *)((const int32_t *)p + r0));
      v[0] = (uint64_t)(int64_t)w[0]; v[1] = (uint64_t)(int64_t)w[1];
      v[2] = (uint64_t)(int64_t)w[2]; v[3] = (uint64_t)(int64_t)w[3];
    } else {
      const v2u64 a = __builtin_nontemporal_load((const v2u64 *)((const int64_t *)p + r0));
      const v2u64 b = __builtin_nontemporal_load((const v2u64 *)((const int64_t *)p + r0 + 2));
      v[0] = a[0]; v[1] = a[1]; v[2] = b[0]; v[3] = b[1];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = r0 + i < n ? (uint64_t)load_icol(p, type, r0 + i) : 0ull;
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
    // acc[mt][nt] register r of lane (q,p) = C[world 16mt+4q+r][column 16nt+p]
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) R[(4 * q + r) * ncp + nt * 16 + p] = acc[mt][nt][r];
    wave_lds_fence();
    const int wl = p;                 // world within this M-tile
    const int world = 16 * mt + wl;
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
      if (val) {
        // blk layout: [g][c][m] with c = ni meaning COUNT
        atomicAdd((unsigned long long *)&blk[((int64_t)g * A + c) * m + world], (unsigned long long)val);
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};
  }
  wave_lds_fence();
}

template <int W, int NT>
__global__ __launch_bounds__(256) void agg_mfma(DevInput in, DevState st, uint32_t *status, MfmaPlan pl) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  constexpr int m = 64 * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, p = lane & 15;
  const int waves = blockDim.x >> 6;
  uint8_t *planes = smem + wave * pl.wave_bytes;
  int64_t *blk = (int64_t *)(smem + pl.blk_off);
  const int D = pl.D, G = pl.G;
  const int ones_plane = D, zero_plane = D + 1, gplane0 = D + 2;

  for (int i = threadIdx.x; i < pl.blk_words; i += blockDim.x) blk[i] = 0;
  // constant planes
  ((uint32_t *)(planes + ones_plane * 256))[lane] = 0x01010101u;
  ((uint32_t *)(planes + zero_plane * 256))[lane] = 0u;
  __syncthreads();

  int boff_d[NT], boff_g[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = nt * 16 + p;
    if (n < pl.ncols) {
      const int g = n / (D + 1), t = n - g * (D + 1);
      boff_d[nt] = (t < D ? t : ones_plane) * 256;
      boff_g[nt] = (gplane0 + g) * 256;
    } else {
      boff_d[nt] = ones_plane * 256;
      boff_g[nt] = zero_plane * 256;
    }
  }

  v4i acc[4 * W][NT];
#pragma unroll
  for (int mt = 0; mt < 4 * W; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};

  const int64_t n = in.n_rows;
  const int64_t n_tiles = (n + kTileRows - 1) / kTileRows;
  const int64_t total_waves = (int64_t)gridDim.x * waves;
  int since_flush = 0;
  for (int64_t tile = (int64_t)blockIdx.x * waves + wave; tile < n_tiles; tile += total_waves) {
    const int64_t row0 = tile * kTileRows;
    // ---- PU words of rows row0 + 64u + lane (A side)
    uint64_t mk[4][W];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = row0 + 64 * u + lane;
#pragma unroll
      for (int w = 0; w < W; ++w) mk[u][w] = 0;
      int64_t idx;
      if (r < n && chain_index(in, r, &idx, status)) {
#pragma unroll
        for (int w = 0; w < W; ++w) mk[u][w] = pu_of_index(in, idx, w);
      }
    }
    // ---- group ids of rows row0 + 4*lane + i (B side), 0xFF = no group
    const int64_t r4 = row0 + 4 * lane;
    uint32_t gv[4] = {0, 0, 0, 0};
    bool ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ok[i] = r4 + i < n;
    for (int k = 0; k < in.n_gcols; ++k) {
      uint32_t v[4];
      load4_gcol(in.gcols[k], in.gcol_type[k], r4, n, v);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ok[i] = ok[i] && (int64_t)v[i] < in.gcards[k];
        gv[i] = gv[i] * (uint32_t)in.gcards[k] + v[i];
      }
    }
    if (in.group_mod > 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) gv[i] = (uint32_t)((uint64_t)gv[i] % (uint64_t)in.group_mod);
    }
    bool bad = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool inrange = r4 + i < n;
      if (inrange && !ok[i]) bad = true;
      ok[i] = ok[i] && (int64_t)gv[i] < G;
    }
    if (in.filter_col) {
      uint32_t fv[4];
      load4_gcol(in.filter_col, PAC_U32, r4, n, fv);
#pragma unroll
      for (int i = 0; i < 4; ++i) ok[i] = ok[i] && fv[i] < in.filter_lt;
    }
    if (bad) atomicOr(status, PAC_STATUS_BAD_GROUP);
    uint32_t gid4 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) gid4 |= (ok[i] ? gv[i] : 0xFFu) << (8 * i);
    // group planes (0xFF where the row belongs to group g) and row counts
    for (int g = 0; g < G; ++g) {
      const uint32_t x = gid4 ^ ((uint32_t)g * 0x01010101u);
      const uint32_t nz = (x | ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu)) & 0x80808080u;
      const uint32_t z = nz ^ 0x80808080u;
      ((uint32_t *)(planes + (gplane0 + g) * 256))[lane] = z | (z - (z >> 7));
      unsigned cnt = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) cnt += __popcll(__ballot(ok[i] && gv[i] == (uint32_t)g));
      if (lane == 0 && cnt) atomicAdd((unsigned long long *)&blk[(int64_t)G * (1 + pl.ni) * m + g], (unsigned long long)cnt);
    }
    // digit planes: byte s of (v - lo), offset to int8 by xor 0x80
    for (int c = 0; c < pl.ni; ++c) {
      uint64_t v[4];
      load4_icol(in.icols[c], in.icol_type[c], r4, n, v);
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] -= (uint64_t)pl.lo[c];
      for (int s = 0; s < pl.dig[c]; ++s) {
        const int sh = s >= 4 ? 32 : 0;
        const uint32_t word = pack_byte((uint32_t)(v[0] >> sh), (uint32_t)(v[1] >> sh), (uint32_t)(v[2] >> sh),
                                        (uint32_t)(v[3] >> sh), s & 3);
        ((uint32_t *)(planes + (pl.doff[c] + s) * 256))[lane] = word ^ 0x80808080u;
      }
    }
    wave_lds_fence();
    // ---- four K-chunks of 64 rows
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v4i a[4 * W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint32_t lo = transpose16x2((uint32_t)mk[u][w], lane);
        const uint32_t hi = transpose16x2((uint32_t)(mk[u][w] >> 32), lane);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const uint32_t x = h < 2 ? lo : hi;
          const int sh = (h & 1) * 16;
          a[4 * w + h] = v4i{expand_nibble(x, sh), expand_nibble(x, sh + 4), expand_nibble(x, sh + 8),
                             expand_nibble(x, sh + 12)};
        }
      }
      const int roff = 64 * u + 16 * q;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const v4i dgt = *(const v4i *)(planes + boff_d[nt] + roff);
        const v4i gm = *(const v4i *)(planes + boff_g[nt] + roff);
        const v4i b = dgt & gm;
#pragma unroll
        for (int mt = 0; mt < 4 * W; ++mt)
          acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[mt], b, acc[mt][nt], 0, 0, 0);
      }
    }
    wave_lds_fence();
    if (++since_flush >= pl.flush_tiles) {
      flush_acc<W, NT>(acc, planes, blk, pl, lane);
      since_flush = 0;
    }
  }
  flush_acc<W, NT>(acc, planes, blk, pl, lane);
  __syncthreads();
  // block counters -> global state
  const int A = 1 + pl.ni;
  for (int i = threadIdx.x; i < pl.blk_words; i += blockDim.x) {
    const int64_t v = blk[i];
    if (!v) continue;
    if (i >= G * A * m) {
      atomicAdd((unsigned long long *)&st.nrows[i - G * A * m], (unsigned long long)v);
      continue;
    }
    const int g = i / (A * m), rem = i - g * A * m, c = rem / m, j = rem - c * m;
    unsigned long long *dst = c == pl.ni ? (unsigned long long *)&st.count[(int64_t)g * m + j]
                                         : (unsigned long long *)&st.isum[((int64_t)g * pl.ni + c) * m + j];
    atomicAdd(dst, (unsigned long long)v);
  }
}

static bool mfma_plan(const DevInput &in, MfmaPlan *pl, int *nt_out) {
  if (in.group_keys || in.n_fcols > 0) return false;
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
    D += p.dig[c];
  }
  p.D = D;
  p.ncols = p.G * (D + 1);
  const int NT = (p.ncols + 15) / 16;
  const int max_nt = in.W == 1 ? kMaxNT : kMaxNT / 2;
  if (NT > max_nt) return false;
  const int planes_bytes = (D + 2 + p.G) * 256;
  const int flush_bytes = 16 * NT * 16 * 4;
  p.wave_bytes = (std::max(planes_bytes, flush_bytes) + 15) & ~15;
  p.blk_off = 4 * p.wave_bytes;
  p.blk_words = p.G * (1 + p.ni) * in.m + p.G;
  // int32 headroom: each row adds at most 128 in magnitude to an accumulator
  p.flush_tiles = (1 << 24) / kTileRows;
  *pl = p;
  *nt_out = NT;
  return p.blk_off + p.blk_words * 8 <= 160 * 1024;
}

bool mfma_supported(const DevInput &in) {
  MfmaPlan p;
  int nt;
  return mfma_plan(in, &p, &nt);
}

template <int W, int NT>
static hipError_t launch_mfma_t(const LaunchEnv &env, const DevInput &in, const DevState &st, const MfmaPlan &pl) {
  const int lds = pl.blk_off + pl.blk_words * 8;
  hipError_t e = hipFuncSetAttribute((const void *)agg_mfma<W, NT>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  const int64_t n_tiles = (in.n_rows + kTileRows - 1) / kTileRows;
  const int per_cu = std::max(1, std::min(4, (160 * 1024) / lds));
  const int64_t want = (n_tiles + 3) / 4;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)env.n_cu * per_cu));
  hipLaunchKernelGGL((agg_mfma<W, NT>), dim3(blocks), dim3(256), (size_t)lds, env.stream, in, st, env.status, pl);
  return hipGetLastError();
}

hipError_t launch_agg_mfma(const LaunchEnv &env, const DevInput &in, const DevState &st) {
  if (in.n_rows <= 0) return hipSuccess;
  MfmaPlan pl;
  int nt;
  if (!mfma_plan(in, &pl, &nt)) return hipErrorInvalidValue;
  if (in.W == 1) {
    switch (nt) {
      case 1: return launch_mfma_t<1, 1>(env, in, st, pl);
      case 2: return launch_mfma_t<1, 2>(env, in, st, pl);
      case 3: return launch_mfma_t<1, 3>(env, in, st, pl);
      case 4: return launch_mfma_t<1, 4>(env, in, st, pl);
      case 5: return launch_mfma_t<1, 5>(env, in, st, pl);
      case 6: return launch_mfma_t<1, 6>(env, in, st, pl);
      case 7: return launch_mfma_t<1, 7>(env, in, st, pl);
      default: return launch_mfma_t<1, 8>(env, in, st, pl);
    }
  }
  switch (nt) {
    case 1: return launch_mfma_t<2, 1>(env, in, st, pl);
    case 2: return launch_mfma_t<2, 2>(env, in, st, pl);
    case 3: return launch_mfma_t<2, 3>(env, in, st, pl);
    default: return launch_mfma_t<2, 4>(env, in, st, pl);
  }
}

}  // namespace pac
