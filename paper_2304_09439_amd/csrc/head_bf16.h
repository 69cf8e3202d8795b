// The MLP head in BF16 on a 32-pair tile in LDS (appendix: MLP predictor on
// the concatenated pooled features, ReLU on the hidden layers, a linear
// output layer), shared by the BF16 kernel and the FP8 kernel whose head
// runs in BF16.
//
// Matrix cores: v_mfma_f32_32x32x16_bf16, FP32 accumulation.  Lane layouts
// (wave64): A[i][k]: i = l % 32, k = 8 (l / 32) + e; B[k][j]: j = l % 32, same
// k; D[i][j]: j = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4 for register r.
// The host packs each head matrix as B fragments: lane l of k-step s of
// column tile ct holds H[32 ct + l % 32][16 s + 8 (l / 32) + e], e = 0..7.
#pragma once

#include "geometry.h"  // wave_index

namespace locc {
namespace head_bf16 {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

__device__ __forceinline__ unsigned short bits(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);  // round to nearest even
}

// One hidden layer on the tile: dst = bf16(ReLU(src W^T + bias)), src and dst
// bf16 rows of stride SS and DS.  Wave w computes output column tiles
// [w CTH, (w+1) CTH); B fragments stream from global memory (L2) D k-steps
// ahead, in a ring of registers, so that several L2 round trips are in flight
// behind the matrix cores.
template <int KDIM, int SS, int DS, int CTH, int D>
__device__ __forceinline__ void layer(const unsigned short* __restrict__ pack, const float* __restrict__ bias,
                                      const unsigned short* src, unsigned short* dst) {
  constexpr int KS = KDIM / 16;
  static_assert(KS % D == 0, "k-steps per head layer");
  const int lane = threadIdx.x & 63, wave = wave_index(), g = lane >> 5, l32 = lane & 31;
  const u16x8* bp = reinterpret_cast<const u16x8*>(pack) + (size_t)wave * CTH * KS * 64 + lane;
  const unsigned short* arow = src + l32 * SS + 8 * g;
  f32x16 acc[CTH];
#pragma unroll
  for (int c = 0; c < CTH; ++c) acc[c] = f32x16{};
  u16x8 bq[D][CTH];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int c = 0; c < CTH; ++c) bq[d][c] = bp[((size_t)c * KS + d) * 64];
#pragma unroll 1
  for (int s0 = 0; s0 < KS; s0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int s = s0 + d;
      const u16x8 av = *reinterpret_cast<const u16x8*>(arow + 16 * s);
#pragma unroll
      for (int c = 0; c < CTH; ++c) acc[c] = mfma(av, bq[d][c], acc[c]);
      if (s + D < KS) {
#pragma unroll
        for (int c = 0; c < CTH; ++c) bq[d][c] = bp[((size_t)c * KS + s + D) * 64];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CTH; ++c) {
    const int col = (wave * CTH + c) * 32 + l32;
    const float bc = bias[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * g + (r & 3);
      dst[row * DS + col] = bits(fmaxf(acc[c][r] + bc, 0.f));
    }
  }
}

// Layers 1-3 of the head on a tile of 32 rows: z (bf16 pooled features
// [f_a, f_b], 2 H2 wide, row stride ZS) -> g (layer 1, HH wide, row stride
// GS) -> z (layer 2, overwriting the features) -> y[w][row][j], the part of
// the 8 raw outputs (without c3) that wave w's quarter of layer 3's
// reduction contributes.  The caller adds the four parts in wave order and
// c3.  Barriers: one between layers; the caller synchronises before reading
// y.
template <int H2, int HH, int ZS, int GS, int D>
__device__ __forceinline__ void layers(const unsigned short* h1p, const float* c1, const unsigned short* h2p,
                                       const float* c2, const unsigned short* h3p, unsigned short* z,
                                       unsigned short* g, float (*y)[32][8]) {
  constexpr int CTH = HH / 128, KS3 = HH / 16;
  static_assert(ZS >= 2 * H2 && ZS >= HH && GS >= HH, "head tile strides");
  const int lane = threadIdx.x & 63, wave = wave_index(), lg = lane >> 5, l32 = lane & 31;
  layer<2 * H2, ZS, GS, CTH, D>(h1p, c1, z, g);
  __syncthreads();
  layer<HH, GS, ZS, CTH, D>(h2p, c2, g, z);
  __syncthreads();
  // layer 3 (8 outputs, padded to 32 columns), reduction split over the 4 waves
  f32x16 acc = f32x16{};
  const u16x8* bp = reinterpret_cast<const u16x8*>(h3p) + lane;
  const unsigned short* arow = z + l32 * ZS + 8 * lg;
#pragma unroll
  for (int s = wave * (KS3 / 4); s < (wave + 1) * (KS3 / 4); ++s)
    acc = mfma(*reinterpret_cast<const u16x8*>(arow + 16 * s), bp[(size_t)s * 64], acc);
  if (l32 < 8)
#pragma unroll
    for (int r = 0; r < 16; ++r) y[wave][8 * (r >> 2) + 4 * lg + (r & 3)][l32] = acc[r];
}

// Layers 1-3 on two 32-row tiles at once, by eight waves: each B fragment of
// layers 1 and 2 is loaded once for both tiles (half the weight stream of
// two separate tiles), wave w (0-7) computing output column tiles
// [w CTH, (w+1) CTH) of both.  Layer 3 as in layers(): waves 0-3 on tile 0,
// waves 4-7 on tile 1, each a quarter of the reduction.  Every output sees
// the same products in the same order as layers() gives it.
template <int KDIM, int SS, int DS, int CTH, int D>
__device__ __forceinline__ void layer2t(const unsigned short* __restrict__ pack, const float* __restrict__ bias,
                                        const unsigned short* src0, const unsigned short* src1, unsigned short* dst0,
                                        unsigned short* dst1, int wave) {
  constexpr int KS = KDIM / 16;
  static_assert(KS % D == 0, "k-steps per head layer");
  const int lane = threadIdx.x & 63, g = lane >> 5, l32 = lane & 31;
  const u16x8* bp = reinterpret_cast<const u16x8*>(pack) + (size_t)wave * CTH * KS * 64 + lane;
  const unsigned short* arow0 = src0 + l32 * SS + 8 * g;
  const unsigned short* arow1 = src1 + l32 * SS + 8 * g;
  f32x16 acc0[CTH], acc1[CTH];
#pragma unroll
  for (int c = 0; c < CTH; ++c) acc0[c] = acc1[c] = f32x16{};
  u16x8 bq[D][CTH];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int c = 0; c < CTH; ++c) bq[d][c] = bp[((size_t)c * KS + d) * 64];
#pragma unroll 1
  for (int s0 = 0; s0 < KS; s0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int s = s0 + d;
      const u16x8 a0 = *reinterpret_cast<const u16x8*>(arow0 + 16 * s);
      const u16x8 a1 = *reinterpret_cast<const u16x8*>(arow1 + 16 * s);
#pragma unroll
      for (int c = 0; c < CTH; ++c) {
        acc0[c] = mfma(a0, bq[d][c], acc0[c]);
        acc1[c] = mfma(a1, bq[d][c], acc1[c]);
      }
      if (s + D < KS) {
#pragma unroll
        for (int c = 0; c < CTH; ++c) bq[d][c] = bp[((size_t)c * KS + s + D) * 64];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CTH; ++c) {
    const int col = (wave * CTH + c) * 32 + l32;
    const float bc = bias[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * g + (r & 3);
      dst0[row * DS + col] = bits(fmaxf(acc0[c][r] + bc, 0.f));
      dst1[row * DS + col] = bits(fmaxf(acc1[c][r] + bc, 0.f));
    }
  }
}

template <int H2, int HH, int ZS, int GS, int D>
__device__ __forceinline__ void layers2t(const unsigned short* h1p, const float* c1, const unsigned short* h2p,
                                         const float* c2, const unsigned short* h3p, unsigned short* z0,
                                         unsigned short* z1, unsigned short* g0, unsigned short* g1,
                                         float (*y0)[32][8], float (*y1)[32][8], int wave) {
  constexpr int CTH = HH / 256, KS3 = HH / 16;
  static_assert(HH % 256 == 0 && ZS >= 2 * H2 && ZS >= HH && GS >= HH, "head tile strides");
  const int lane = threadIdx.x & 63, lg = lane >> 5, l32 = lane & 31;
  layer2t<2 * H2, ZS, GS, CTH, D>(h1p, c1, z0, z1, g0, g1, wave);
  __syncthreads();
  layer2t<HH, GS, ZS, CTH, D>(h2p, c2, g0, g1, z0, z1, wave);
  __syncthreads();
  const int t = wave >> 2, w4 = wave & 3;
  unsigned short* z = t ? z1 : z0;
  float(*y)[32][8] = t ? y1 : y0;
  f32x16 acc = f32x16{};
  const u16x8* bp = reinterpret_cast<const u16x8*>(h3p) + lane;
  const unsigned short* arow = z + l32 * ZS + 8 * lg;
#pragma unroll
  for (int s = w4 * (KS3 / 4); s < (w4 + 1) * (KS3 / 4); ++s)
    acc = mfma(*reinterpret_cast<const u16x8*>(arow + 16 * s), bp[(size_t)s * 64], acc);
  if (l32 < 8)
#pragma unroll
    for (int r = 0; r < 16; ++r) y[w4][8 * (r >> 2) + 4 * lg + (r & 3)][l32] = acc[r];
}

}  // namespace head_bf16
}  // namespace locc
