// Pieces shared by the int8 matrix-core aggregation kernels (generic and
// star-schema forms): tile geometry, the 16-lane bit transpose that turns PU
// words into int8 world operands, compact kernel arguments and the FK chain.
#pragma once
#include <algorithm>

#include "pac_internal.h"

namespace pac {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned long long v2u64 __attribute__((ext_vector_type(2)));
typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

constexpr int kTileRows = 256;
// Byte planes hold 256 rows; consecutive planes are 272 bytes apart so that
// the 16 lanes of a group reading 16 bytes from 16 different planes hit
// different LDS banks.
constexpr int kPlaneStride = 272;
constexpr int kMaxNT = 8;

struct MfmaPlan {
  int32_t G;            // dense groups (<= 254)
  int32_t D;            // total digit planes
  int32_t ncols;        // G * (D + 1)
  int32_t ni;
  int32_t dig[kMaxCols];
  int32_t doff[kMaxCols];
  int64_t lo[kMaxCols];
  uint64_t range[kMaxCols];  // max - lo of the statistics: (v - lo) above it is out of range
  int32_t wave_bytes;   // per-wave LDS: planes (reused as the flush buffer), then the staging area
  int32_t stage_off;
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
// lane ^ 4 inside a row of 16: banks 0 and 2 (lanes 0-3, 8-11) read lane + 4
// (row_ror:12), banks 1 and 3 read lane - 4 (row_ror:4).
__device__ __forceinline__ uint32_t dpp_xor4(uint32_t x) {
  const int t = __builtin_amdgcn_update_dpp((int)x, (int)x, 0x12C, 0xF, 0x5, false);
  return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)x, 0x124, 0xF, 0xA, false);
}
__device__ __forceinline__ uint32_t dpp_xor8(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false);  // row_ror:8 == lane ^ 8 in a row
}

// Bit transpose of the PU words inside each 16-lane group.  Lane i of group
// q holds the 64 PU bits of row 16q + i; four exchange stages each swap one
// lane-index bit with one bit-position bit of a 32-bit word:
//   lane bit 2 <-> position bit 0,  lane bit 3 <-> position bit 1,
//   lane bit 0 <-> position bit 3,  lane bit 1 <-> position bit 4.
// Afterwards bit position  k + 4h + 8j  (k, j in 0..3, h in 0..1) of lane i
// holds row 4k + j of world  world_of(i, h)  (see below) -- i.e. the rows of
// one world are spread one per byte, so the int8 A operand for rows
// 4k..4k+3 is just (T >> (k + 4h)) & 0x01010101.
// In a stage the lower lane of a pair keeps its bits whose position bit is
// clear and takes the partner's such bits rotated up; the upper lane keeps
// the others and takes the partner's bits rotated down.
struct TransposeConsts {
  uint32_t keep[4];
  uint32_t rot[4];
};

__device__ __forceinline__ TransposeConsts transpose_consts(int lane) {
  TransposeConsts t;
  const int lane_bit[4] = {4, 8, 1, 2};
  const uint32_t clear_mask[4] = {0x55555555u, 0x33333333u, 0x00FF00FFu, 0x0000FFFFu};
  const uint32_t shift[4] = {1, 2, 8, 16};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const bool lower = (lane & lane_bit[s]) == 0;
    t.keep[s] = lower ? clear_mask[s] : ~clear_mask[s];
    t.rot[s] = lower ? 32 - shift[s] : shift[s];
  }
  return t;
}

__device__ __forceinline__ uint32_t bfi(uint32_t mask, uint32_t a, uint32_t b) {
  uint32_t r;
  asm volatile("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(mask), "v"(a), "v"(b));
  return r;
}

__device__ __forceinline__ uint32_t transpose_word(uint32_t x, const TransposeConsts &tc) {
  uint32_t p = dpp_xor4(x);
  x = bfi(tc.keep[0], x, __builtin_amdgcn_alignbit(p, p, tc.rot[0]));
  p = dpp_xor8(x);
  x = bfi(tc.keep[1], x, __builtin_amdgcn_alignbit(p, p, tc.rot[1]));
  p = dpp_xor1(x);
  x = bfi(tc.keep[2], x, __builtin_amdgcn_alignbit(p, p, tc.rot[2]));
  p = dpp_xor2(x);
  x = bfi(tc.keep[3], x, __builtin_amdgcn_alignbit(p, p, tc.rot[3]));
  return x;
}

// World (0..31 within the 32-bit word) held by lane i of a group at bit-4 value h
// after transpose_word: lane bits (0,1,2,3) carry world bits (3,4,0,1), h world bit 2.
__device__ __forceinline__ int world_of(int i, int h) {
  return ((i >> 2) & 1) | (((i >> 3) & 1) << 1) | (h << 2) | ((i & 1) << 3) | (((i >> 1) & 1) << 4);
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kMC = 4;  // int columns / links handled by this path
constexpr int kMG = 2;  // group columns handled by this path

// Compact kernel arguments of the matrix-core path.  Row-indexed pointers
// (columns, first link, or the mask table when there is no link) are offset
// to the first row of the launch, so rows and table indices are 32-bit.
struct MfmaArgs {
  int32_t n_links;
  const int32_t *links[kMC];
  uint32_t link_len[kMC];
  const uint64_t *masks;
  const int64_t *pu_keys;
  uint32_t n_idx;  // rows of the mask table (or of pu_keys); >= 1
  uint64_t qk;
  uint32_t balanced;
  int32_t n_gcols;
  const uint8_t *gcols[kMG];
  int32_t gcol_bytes[kMG];  // 1, 2 or 4
  uint32_t gcards[kMG];
  uint32_t group_mod;
  const uint32_t *filter_col;
  uint32_t filter_lt;
  const uint8_t *icols[kMC];
  int32_t icol_bytes[kMC];  // 4 or 8
  uint32_t n_rows;          // rows of this launch
};

// Input shape: SH = 0 reads everything from the arguments; SH = 1 is the
// star-schema scan (two FK links into a PU-word table, up to two group
// columns, no filter, no group modulus) with those facts known at compile time.
template <int SH>
struct Shape {
  static __device__ __forceinline__ int n_links(const MfmaArgs &a) { return SH == 1 ? 2 : a.n_links; }
  static __device__ __forceinline__ bool masks(const MfmaArgs &a) { return SH == 1 ? true : a.masks != nullptr; }
  static __device__ __forceinline__ bool filter(const MfmaArgs &a) { return SH == 1 ? false : a.filter_col != nullptr; }
  static __device__ __forceinline__ bool modulo(const MfmaArgs &a) { return SH == 1 ? false : a.group_mod > 0; }
};

// ---------------------------------------------------------------- FK chain
// Indices of the four K-chunk rows (64u + lane) of a tile after some chain
// levels, with their validity.  Every load below is unconditional: invalid
// lanes read index 0 of a non-empty table and are masked when the words are
// staged, so the compiler never has to wait for a load before it is used.
struct Chain {
  uint32_t idx[4];
  uint32_t ok[4];  // 0/1, kept as integers (vector registers) rather than lane masks
};

__device__ __forceinline__ void chain_rows(const MfmaArgs &a, uint32_t row0, int lane, Chain &c) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint32_t r = row0 + 64u * u + lane;
    c.ok[u] = r < a.n_rows;
    c.idx[u] = r;
  }
}

__device__ __forceinline__ void chain_level(const MfmaArgs &a, int k, Chain &c) {
  const int32_t *lk = a.links[k];
  const uint32_t len = a.link_len[k];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const bool v = c.ok[u] && c.idx[u] < len;
    c.ok[u] = v;
    c.idx[u] = (uint32_t)lk[v ? c.idx[u] : 0u];
  }
}

// Arguments of the launch covering rows [r0, r0 + n).
static inline MfmaArgs mfma_args(const DevInput &in, int64_t r0, int64_t n) {
  MfmaArgs a{};
  a.n_rows = (uint32_t)n;
  a.n_links = in.n_links;
  for (int k = 0; k < in.n_links; ++k) {
    a.links[k] = in.links[k];
    a.link_len[k] = (uint32_t)in.link_len[k];
  }
  a.masks = in.masks;
  a.pu_keys = in.pu_keys;
  a.n_idx = (uint32_t)(in.masks ? in.n_masks : in.n_pu_keys);
  if (in.n_links > 0) {  // the first link is indexed by row
    a.links[0] = in.links[0] + r0;
    a.link_len[0] = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(in.link_len[0] - r0, n));
  } else if (in.masks) {  // the mask table is indexed by row
    a.masks = in.masks + r0 * in.W;
    a.n_idx = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(in.n_masks - r0, n));
  } else {
    a.pu_keys = in.pu_keys + r0;
    a.n_idx = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(in.n_pu_keys - r0, n));
  }
  a.qk = in.query_key;
  a.balanced = in.balanced;
  a.n_gcols = in.n_gcols;
  for (int k = 0; k < in.n_gcols; ++k) {
    const int bytes = in.gcol_type[k] == PAC_U8 ? 1 : in.gcol_type[k] == PAC_U16 ? 2 : 4;
    a.gcols[k] = (const uint8_t *)in.gcols[k] + r0 * bytes;
    a.gcol_bytes[k] = bytes;
    a.gcards[k] = (uint32_t)in.gcards[k];
  }
  a.group_mod = (uint32_t)in.group_mod;
  a.filter_col = in.filter_col ? in.filter_col + r0 : nullptr;
  a.filter_lt = in.filter_lt;
  for (int c = 0; c < in.n_icols; ++c) {
    const int bytes = in.icol_type[c] == PAC_I32 ? 4 : 8;
    a.icols[c] = (const uint8_t *)in.icols[c] + r0 * bytes;
    a.icol_bytes[c] = bytes;
  }
  return a;
}

}  // namespace pac
