// a2-a6 for one float column on the bf16 matrix cores: an approximate form.
//
// The per-world float SUM of Sec. 4.2 is the contraction
//   S[g][j] = sum_r bit_j(r) [grp(r) = g] v(r)
// of the 0/1 world-bit matrix with the value column.  Here it runs on
// v_mfma_f32_16x16x32_bf16 with fp32 accumulation:
//   * v is rounded to fp32 (the input rounding of an fp64 column) and split
//     into three bf16 terms hi + mid + lo (each the rounded remainder of the
//     previous ones), which represent the fp32 value exactly;
//   * a workgroup takes 2048 rows at a time, sorts them by group in LDS
//     (counting sort), and each wavefront owns 8 groups (4 at m = 128): the
//     B operand of one 16-column tile holds, for 4 groups, the three terms and
//     a 1.0 (COUNT) of the rows of that group and zero elsewhere, so after the
//     sort a 32-row K-chunk touches one or two column tiles instead of all 16
//     a one-hot group dimension would need;
//   * the A operand is the rows' world bits as bf16 0/1 (M = 16 worlds per tile);
//   * the fp32 accumulators are flushed every 16 super-tiles: the three term
//     sums are added in fp64 (exactly) and then into the state with fp64
//     atomics; COUNT is exact (an integer below 2^24 in fp32).
// The paper's precedent for a float state traded against precision is its
// approximate cascaded aggregate (Sec. 5, Approximation); this form is
// selected explicitly (PAC_ALGO_MFMA_BF16), never by PAC_ALGO_AUTO.
#include <algorithm>

#include "pac_internal.h"

namespace pac {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kFmRows = 2048;   // rows per super-tile
constexpr int kFmMaxG = 64;     // dense groups
constexpr int kFmFlush = 16;    // super-tiles between flushes of the fp32 accumulators

template <int W>
struct FmStage {
  uint64_t mk[W][kFmRows];  // PU words of the rows sorted by group
  uint16_t term[3][kFmRows]; // bf16 bits of hi, mid, lo
  uint8_t grp[kFmRows];
  uint32_t cnt[kFmMaxG];
  uint32_t off[kFmMaxG + 1];
  uint32_t nrows[kFmMaxG];
};

// Round-to-nearest-even fp32 -> bf16 bits (finite inputs).
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

template <int W>
__global__ __launch_bounds__(512 * W) void agg_fmma(DevInput in, DevState st, uint32_t *status) {
  constexpr int m = 64 * W;
  constexpr int MT = 4 * W;           // 16-world tiles
  constexpr int NTW = 2 / W;          // 16-column tiles (4 groups each) per wave
  constexpr int GPW = 4 * NTW;        // groups per wave
  __shared__ FmStage<W> sg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nthreads = blockDim.x;
  const int G = (int)in.n_groups;
  for (int i = tid; i < kFmMaxG; i += nthreads) sg.nrows[i] = 0;
  f32x4 acc[NTW][MT];
#pragma unroll
  for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int gw0 = wave * GPW;  // this wave's first group
  const int p = lane & 15, kq = lane >> 4;
  const int64_t n_tiles = (in.n_rows + kFmRows - 1) / kFmRows;
  int since_flush = 0;

  auto flush = [&]() {
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
      const int gi = p >> 2, c = p & 3;
      const int g = gw0 + 4 * nt + gi;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // lanes 4gi + 0, 1, 2 hold the three term sums of (g, world): added exactly in fp64
          const double x = (double)acc[nt][mt][r];
          const double s1 = __shfl_down(x, 1, 16), s2 = __shfl_down(x, 2, 16);
          const int world = 16 * mt + 4 * kq + r;
          if (g < G) {
            if (c == 0) {
              const double s = x + s1 + s2;
              if (s != 0.0) atomicAdd(&st.fsum[(int64_t)g * in.n_fcols * m + world], s);
            } else if (c == 3 && x != 0.0) {
              atomicAdd((unsigned long long *)&st.count[(int64_t)g * m + world], (unsigned long long)x);
            }
          }
        }
        acc[nt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };

  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t base = t * kFmRows;
    for (int i = tid; i < kFmMaxG; i += nthreads) sg.cnt[i] = 0;
    __syncthreads();
    // ---- load and count: each thread takes rows base + tid + k * nthreads
    constexpr int kPer = kFmRows / (512 * W);
    int32_t rg[kPer];
    uint32_t rpos[kPer];
    uint64_t rmk[kPer][W];
    float rv[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t r = base + tid + (int64_t)k * nthreads;
      rg[k] = -1;
      rv[k] = 0.f;
#pragma unroll
      for (int w = 0; w < W; ++w) rmk[k][w] = 0;
      if (r < in.n_rows) {
        const int64_t g = row_group(in, st, r, status);
        int64_t idx = 0;
        if (g >= 0 && chain_index(in, r, &idx, status)) {
          rg[k] = (int32_t)g;
#pragma unroll
          for (int w = 0; w < W; ++w) rmk[k][w] = pu_of_index(in, idx, w);
          rv[k] = (float)load_fcol(in.fcols[0], in.fcol_type[0], r);
        }
      }
      rpos[k] = rg[k] >= 0 ? atomicAdd(&sg.cnt[rg[k]], 1u) : 0u;
    }
    __syncthreads();
    if (wave == 0) {  // exclusive scan of the group counts (lane = group)
      const uint32_t c = lane < G ? sg.cnt[lane] : 0u;
      uint32_t x = c;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      sg.off[lane] = x - c;
      if (lane == 63) sg.off[64] = x;
      if (lane < G) sg.nrows[lane] += c;
    }
    __syncthreads();
    // ---- scatter into group order, splitting each value into three bf16 terms
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (rg[k] < 0) continue;
      const uint32_t s = sg.off[rg[k]] + rpos[k];
#pragma unroll
      for (int w = 0; w < W; ++w) sg.mk[w][s] = rmk[k][w];
      const float v = rv[k];
      const uint32_t h = bf16_rne(v);
      const float r1 = v - bf16_to_f32(h);
      const uint32_t md = bf16_rne(r1);
      const float r2 = r1 - bf16_to_f32(md);
      sg.term[0][s] = (uint16_t)h;
      sg.term[1][s] = (uint16_t)md;
      sg.term[2][s] = (uint16_t)bf16_rne(r2);
      sg.grp[s] = (uint8_t)rg[k];
    }
    __syncthreads();
    // ---- contraction: this wave's groups occupy the sorted rows [lo, hi)
    if (gw0 < G) {
      const uint32_t lo = sg.off[gw0], hi = sg.off[min(gw0 + GPW, 64)];
      for (uint32_t s0 = lo; s0 < hi; s0 += 32) {
        // A: world bits of rows s0 + 8 kq + i as bf16 0/1, for every 16-world tile
        uint64_t wd[8][W];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const uint32_t row = s0 + 8 * kq + i;
#pragma unroll
          for (int w = 0; w < W; ++w) wd[i][w] = row < hi ? sg.mk[w][row] : 0ull;
        }
        bf16x8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          u32x4 au;
#pragma unroll
          for (int i2 = 0; i2 < 4; ++i2) {
            const uint32_t b0 = (uint32_t)(wd[2 * i2][mt >> 2] >> (16 * (mt & 3) + p)) & 1u;
            const uint32_t b1 = (uint32_t)(wd[2 * i2 + 1][mt >> 2] >> (16 * (mt & 3) + p)) & 1u;
            au[i2] = (b0 | (b1 << 16)) * 0x3F80u;
          }
          a[mt] = __builtin_bit_cast(bf16x8, au);
        }
        // B for each column tile of the wave whose groups have rows in this chunk
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
          const int g0 = gw0 + 4 * nt;
          if (g0 >= G) continue;
          const uint32_t tlo = sg.off[g0], thi = sg.off[min(g0 + 4, 64)];
          if (thi <= s0 || tlo >= s0 + 32) continue;
          const int gi = p >> 2, c = p & 3;
          const uint32_t want = (uint32_t)(g0 + gi);
          u32x4 bu;
#pragma unroll
          for (int i2 = 0; i2 < 4; ++i2) {
            uint32_t e[2];
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
              const uint32_t row = s0 + 8 * kq + 2 * i2 + h2;
              const bool mine = row < hi && sg.grp[row] == want;
              e[h2] = !mine ? 0u : c == 3 ? 0x3F80u : (uint32_t)sg.term[c < 3 ? c : 0][row];
            }
            bu[i2] = e[0] | (e[1] << 16);
          }
          const bf16x8 b = __builtin_bit_cast(bf16x8, bu);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[nt][mt], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // the stage is rewritten by the next super-tile
    if (++since_flush == kFmFlush) {
      flush();
      since_flush = 0;
    }
  }
  flush();
  __syncthreads();
  for (int i = tid; i < G; i += nthreads)
    if (sg.nrows[i]) atomicAdd((unsigned long long *)&st.nrows[i], (unsigned long long)sg.nrows[i]);
}

// ---------------------------------------------------------------- host side
bool fmma_supported(const DevInput &in, const DevState &st) {
  if (in.group_keys || st.minmax || in.n_icols != 0 || in.n_fcols != 1) return false;
  if (in.n_groups < 1 || in.n_groups > kFmMaxG) return false;
  return in.n_gcols > 0 || in.group_mod > 0 || in.n_groups == 1;
}

hipError_t launch_agg_fmma(const LaunchEnv &env, const DevInput &in, const DevState &st) {
  if (in.n_rows <= 0) return hipSuccess;
  const void *fn = in.W == 1 ? (const void *)agg_fmma<1> : (const void *)agg_fmma<2>;
  const int threads = 512 * in.W;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0);
  if (e != hipSuccess) return e;
  per_cu = std::max(1, per_cu);
  const int64_t n_tiles = (in.n_rows + kFmRows - 1) / kFmRows;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(n_tiles, (int64_t)env.n_cu * per_cu));
  if (in.W == 1)
    hipLaunchKernelGGL(agg_fmma<1>, dim3(blocks), dim3(threads), 0, env.stream, in, st, env.status);
  else
    hipLaunchKernelGGL(agg_fmma<2>, dim3(blocks), dim3(threads), 0, env.stream, in, st, env.status);
  return hipGetLastError();
}

}  // namespace pac
