// FP8 (OCP e4m3) encoder + head kernel of the split schedule.
//
// Same structure as the BF16 persistent kernel: workgroups claim pairs,
// stage the bf16 encoder rows the crop kernel wrote, run the per-point
// encoder with a per-object max-pool into an LDS tile, and run the head on
// every 32-pair tile.  Precision by layer (per-layer scales):
//   encoder layer 1  bf16 (inputs are coordinates and normals)  32x32x8 bf16
//   encoder layer 2  fp8 x fp8, FP32 accumulation               32x32x64 f8f6f4
//   head layers 1-2  fp8 x fp8, FP32 accumulation               32x32x64 f8f6f4
//   head layer 3     bf16                                        32x32x16 bf16
// or, with HEAD8 = false (the lower-error variant), the whole head in bf16 as
// in the BF16 kernel (head_bf16.h), encoder layer 2 the only fp8 layer.
// A weight matrix is stored as W / s_W in e4m3 with s_W = amax|W| / 448; an
// activation x enters a layer as e4m3(min(x / s_x, 448)) with a static
// s_x = amax / 448 from a calibration batch.  The product of the two scales
// is applied once per output in the epilogue (before the bias).  The
// encoder's max-pool runs on the raw sums: with a positive scale,
// fl(fl(max_r a_r s) + b) = max_r fl(fl(a_r s) + b) (rounding is monotone).
// As in the BF16 kernel, each wave computes one 32-feature tile of layer 1
// per 32-row tile and shares it through a double-buffered LDS tile; a lane's
// 16 layer-1 outputs (one point, lane group g) are 16 bytes of layer 2's A
// operand: each 64-wide k-step takes two 32-feature tiles, and W2 is packed
// so that lane group g, byte e of k-step s is feature F(2 s + e / 16, g,
// e % 16), F(ft, g, r) = 32 ft + 8 (r / 4) + 4 g + r % 4.  In the LDS tile a
// row holds, per k-step s and lane group g, those 32 bytes contiguously.
#include "fused.h"
#include "geometry.h"
#include "head_bf16.h"
#include "post.h"

#include <cmath>
#include <cstring>

namespace locc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma_k8(s16x4 a, s16x4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_k16(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}
// e4m3 x e4m3, unit block scales (E8M0 127 = 2^0)
__device__ __forceinline__ f32x16 mfma_f8(i32x8 a, i32x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}
// IEEE maximum: no canonicalisation of matrix-core results (see fused.hip)
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_elementwise_maximum(a, b); }
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}
// four floats -> four e4m3 bytes of min(ReLU(x), 448): one med3 does the
// ReLU and the clamp (layer 1 already works in units of the activation scale)
__device__ __forceinline__ float relu_clamp448(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 448.f); }
__device__ __forceinline__ int pack4_e4m3(float a, float b, float c, float d) {
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(relu_clamp448(a), relu_clamp448(b), 0, false);
  return __builtin_amdgcn_cvt_pk_fp8_f32(relu_clamp448(c), relu_clamp448(d), v, true);
}

// HEAD8: the fp8 head (z and g1 e4m3 tiles, g2 bf16); otherwise the bf16
// head of head_bf16.h (z bf16, g1 in the union, g2 over z).
template <int H1, int H2, int HH, bool HEAD8>
struct Smem8 {
  static constexpr int T = kFusedTile;
  static constexpr int ZB = 2 * H2 + 16;  // bytes per row of the fp8 z tile
  static constexpr int GB = HH + 16;      // bytes per row of the fp8 g1 tile
  static constexpr int G2 = HH + 8;       // bf16 elements per row of the g2 tile (the bf16 head's g1)
  static constexpr int HB = H1 + 16;      // bytes per row of the fp8 layer-1 tiles
  static constexpr int ZS = (2 * H2 > HH ? 2 * H2 : HH) + 8;  // bf16 elements per row of the bf16 head's z tile
  union alignas(16) {
    struct {
      alignas(16) unsigned short rows[2 * kMaxK * 8];  // encoder rows of the current pair (bf16)
      alignas(16) unsigned char h1t[2][T * HB];        // layer-1 output of a 32-row tile (e4m3)
    } e;
    unsigned short g2[T * G2];            // head layer-2 output (bf16), or the bf16 head's layer-1 output
  } u;
  alignas(16) unsigned char z[HEAD8 ? T * ZB : 2 * T * ZS];
  alignas(16) unsigned char g1[HEAD8 ? T * GB : 16];
  float y[4][T][8];
  int32_t pair[T];
  int32_t a[T];
  int32_t swapped[T];
  int32_t claim;
};

// One fp8 head layer: dst = e4m3(min(ReLU(scale * src W^T + bias) * dst_inv, 448)) or, when
// DST_BF16, bf16(ReLU(scale * src W^T + bias)).
template <int KDIM, int SB, int DS, int CTH, bool DST_BF16>
__device__ __forceinline__ void head_layer8(const unsigned char* __restrict__ pack, const float* __restrict__ bias,
                                            float scale, float dst_inv, const unsigned char* src, void* dst) {
  constexpr int KS = KDIM / 64, D = 1;  // weight fragments D k-steps ahead, in a ring of registers
  static_assert(KS % D == 0, "k-steps per head layer");
  const int lane = threadIdx.x & 63, wave = wave_index(), g = lane >> 5, l32 = lane & 31;
  const i32x8* bp = reinterpret_cast<const i32x8*>(pack) + (size_t)wave * CTH * KS * 64 + lane;
  const unsigned char* arow = src + l32 * SB + 32 * g;
  f32x16 acc[CTH];
#pragma unroll
  for (int c = 0; c < CTH; ++c) acc[c] = f32x16{};
  i32x8 bq[D][CTH];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int c = 0; c < CTH; ++c) bq[d][c] = bp[((size_t)c * KS + d) * 64];
#pragma unroll 1
  for (int s0 = 0; s0 < KS; s0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int s = s0 + d;
      const uint4 a0 = *reinterpret_cast<const uint4*>(arow + 64 * s);
      const uint4 a1 = *reinterpret_cast<const uint4*>(arow + 64 * s + 16);
      const i32x8 av = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
#pragma unroll
      for (int c = 0; c < CTH; ++c) acc[c] = mfma_f8(av, bq[d][c], acc[c]);
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
      const float v = fmaxf(acc[c][r] * scale + bc, 0.f);
      if constexpr (DST_BF16) {
        static_cast<unsigned short*>(dst)[row * DS + col] = bf16_bits(v);
      } else {
        const int q = __builtin_amdgcn_cvt_pk_fp8_f32(fminf(v * dst_inv, 448.f), 0.f, 0, false);
        static_cast<unsigned char*>(dst)[row * DS + col] = (unsigned char)(q & 0xff);
      }
    }
  }
}

// Head on the first n rows of the pooled-feature tile, then the world-frame epilogue.
template <int H1, int H2, int HH, bool HEAD8>
__device__ __forceinline__ void head_tile8(const Fp8Args& A, Smem8<H1, H2, HH, HEAD8>& S, int n) {
  using S_t = Smem8<H1, H2, HH, HEAD8>;
  constexpr int T = S_t::T, ZB = S_t::ZB, GB = S_t::GB, G2 = S_t::G2, CTH = HH / 128, KS3 = HH / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_index(), g = lane >> 5, l32 = lane & 31;
  if constexpr (HEAD8) {
    for (int e = tid; e < (T - n) * ZB; e += 256) S.z[n * ZB + e] = 0;
    __syncthreads();
    head_layer8<2 * H2, ZB, GB, CTH, false>(A.h1p, A.c1, A.s_z * A.s_h1, 1.f / A.s_g1, S.z, S.g1);
    __syncthreads();
    head_layer8<HH, GB, G2, CTH, true>(A.h2p, A.c2, A.s_g1 * A.s_h2, 0.f, S.g1, S.u.g2);
    __syncthreads();
    f32x16 acc = f32x16{};
    const u16x8* bp = reinterpret_cast<const u16x8*>(A.h3p) + lane;
    const unsigned short* arow = S.u.g2 + l32 * G2 + 8 * g;
#pragma unroll
    for (int s = wave * (KS3 / 4); s < (wave + 1) * (KS3 / 4); ++s)
      acc = mfma_k16(*reinterpret_cast<const u16x8*>(arow + 16 * s), bp[(size_t)s * 64], acc);
    if (l32 < 8)
#pragma unroll
      for (int r = 0; r < 16; ++r) S.y[wave][8 * (r >> 2) + 4 * g + (r & 3)][l32] = acc[r];
  } else {
    constexpr int ZS = S_t::ZS;
    unsigned short* z16 = reinterpret_cast<unsigned short*>(S.z);
    for (int e = tid; e < (T - n) * ZS; e += 256) z16[n * ZS + e] = 0;
    __syncthreads();
    head_bf16::layers<H2, HH, ZS, G2, 4>(reinterpret_cast<const unsigned short*>(A.h1p), A.c1,
                                         reinterpret_cast<const unsigned short*>(A.h2p), A.c2, A.h3p, z16, S.u.g2,
                                         S.y);
  }
  __syncthreads();
  for (int t = tid; t < T * 8; t += 256) {
    const int i = t >> 3, j = t & 7;
    S.y[0][i][j] = ((S.y[0][i][j] + S.y[1][i][j]) + S.y[2][i][j]) + S.y[3][i][j] + A.c3[j];
  }
  __syncthreads();
  if (tid < n) post_contact(A.objs, S.a[tid], S.swapped[tid], S.y[0][tid], A.out, A.y_dbg, S.pair[tid]);
  __syncthreads();
}

template <int H1, int H2, int HH, bool HEAD8>
__global__ __launch_bounds__(256, kFusedWgPerCu) void encoder_head_fp8_kernel(Fp8Args A) {
  using S_t = Smem8<H1, H2, HH, HEAD8>;
  constexpr int T = S_t::T, ZB = S_t::ZB;
  constexpr int FT = H1 / 32;    // layer-1 feature tiles
  constexpr int FW = (FT + 3) / 4;  // layer-1 feature tiles per wave (tiles wave, wave + 4, ...)
  constexpr int KS2 = H1 / 64;   // layer-2 fp8 k-steps (two feature tiles each)
  constexpr int HB = S_t::HB;
  constexpr int CT = H2 / 128;   // encoder column tiles per wave
  static_assert(H1 % 64 == 0 && H2 % 128 == 0 && HH % 128 == 0, "widths");
  __shared__ S_t S;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_index(), g = lane >> 5, l32 = lane & 31;
  const int K = A.K;
  const int P = pair_count(A.n_pairs, A.n_pairs_dev, A.dev_base);
  const float s_enc = A.s_h1in * A.s_w2, inv_z = 1.f / A.s_z;

  i32x8 w2f[CT][KS2];
  float bias2[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
    for (int s = 0; s < KS2; ++s)
      w2f[ct][s] = reinterpret_cast<const i32x8*>(A.w2p)[(size_t)((wave * CT + ct) * KS2 + s) * 64 + lane];
    bias2[ct] = A.b2[(wave * CT + ct) * 32 + l32];
  }
  s16x4 w1f[FW];
#pragma unroll
  for (int i = 0; i < FW; ++i)
    w1f[i] = wave + 4 * i < FT ? reinterpret_cast<const s16x4*>(A.w1p)[(size_t)(wave + 4 * i) * 64 + lane] : s16x4{};

  int slot = 0;
  for (int iter = 0;; ++iter) {
    if (tid == 0)
      S.claim = A.dynamic ? (int)atomicAdd(A.queue, (unsigned)A.claim) : (blockIdx.x + iter * gridDim.x) * A.claim;
    __syncthreads();
    const int base = S.claim;
    __syncthreads();
    if (base >= P) break;
    const int n_claim = P - base < A.claim ? P - base : A.claim;
    // the next pair's record and rows are carried in registers (two named
    // registers: an array would be moved to LDS), loaded while the current
    // pair computes
    const uint4* rows_g = reinterpret_cast<const uint4*>(A.rows_bf16);
    uint4 nxt0{}, nxt1{};
    PairMeta nmeta = A.meta[base];
    if (tid < 2 * K) nxt0 = rows_g[(size_t)base * 2 * K + tid];
    if (tid + 256 < 2 * K) nxt1 = rows_g[(size_t)base * 2 * K + tid + 256];
    for (int c = 0; c < n_claim; ++c) {
      const int p = base + c;
      const PairMeta mt = nmeta;
      const bool valid = mt.a >= 0;
      const int m_a = valid ? mt.m_a : 0, m_b = valid ? mt.m_b : 0;
      if (tid < 2 * K) reinterpret_cast<uint4*>(S.u.e.rows)[tid] = nxt0;
      if (tid + 256 < 2 * K) reinterpret_cast<uint4*>(S.u.e.rows)[tid + 256] = nxt1;
      if (c + 1 < n_claim) {
        nmeta = A.meta[p + 1];
        if (tid < 2 * K) nxt0 = rows_g[(size_t)(p + 1) * 2 * K + tid];
        if (tid + 256 < 2 * K) nxt1 = rows_g[(size_t)(p + 1) * 2 * K + tid + 256];
      }
      if (tid == 0) {
        S.pair[slot] = p;
        S.a[slot] = valid ? mt.a : -1;
        S.swapped[slot] = mt.swapped;
      }
      __syncthreads();
      // Row tiles t = 0, 1, ...: this wave's layer-1 features of tile t + 1
      // are computed while layer 2 of tile t runs, then stored to the other
      // LDS buffer; one barrier per tile publishes them (the buffer written in
      // tile t was last read in tile t - 1, before the previous barrier).
      for (int side = 0; side < 2; ++side) {
        const int m = side ? m_b : m_a;
        const int nt = (m + 31) >> 5;  // uniform over the workgroup
        const unsigned short* xrow = &S.u.e.rows[(side * K + l32) * 8 + 4 * g];
        float run[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) run[ct] = -__builtin_inff();
        f32x16 acc1[FW];
        // the input operand of the next row tile is read one tile ahead
        s16x4 xb = *reinterpret_cast<const s16x4*>(xrow);
        auto layer1_issue = [&](int t) {
#pragma unroll
          for (int i = 0; i < FW; ++i)
            if (FT % 4 == 0 || wave + 4 * i < FT) acc1[i] = mfma_k8(w1f[i], xb, f32x16{});
          if (t + 1 < nt) xb = *reinterpret_cast<const s16x4*>(xrow + (t + 1) * 32 * 8);
        };
        auto layer1_store = [&](int buf) {
#pragma unroll
          for (int i = 0; i < FW; ++i) {
            const int ft = wave + 4 * i;
            if (FT % 4 == 0 || ft < FT) {
              uint4 q;
              q.x = pack4_e4m3(acc1[i][0], acc1[i][1], acc1[i][2], acc1[i][3]);
              q.y = pack4_e4m3(acc1[i][4], acc1[i][5], acc1[i][6], acc1[i][7]);
              q.z = pack4_e4m3(acc1[i][8], acc1[i][9], acc1[i][10], acc1[i][11]);
              q.w = pack4_e4m3(acc1[i][12], acc1[i][13], acc1[i][14], acc1[i][15]);
              *reinterpret_cast<uint4*>(&S.u.e.h1t[buf][l32 * HB + 64 * (ft >> 1) + 32 * g + 16 * (ft & 1)]) = q;
            }
          }
        };
        if (nt > 0) {
          layer1_issue(0);
          layer1_store(0);
        }
        __syncthreads();
        for (int t = 0; t < nt; ++t) {
          const bool more = t + 1 < nt;
          const unsigned char* h = &S.u.e.h1t[t & 1][l32 * HB + 32 * g];
          i32x8 av[KS2];
#pragma unroll
          for (int s = 0; s < KS2; ++s) {
            const uint4 a0 = *reinterpret_cast<const uint4*>(h + 64 * s);
            const uint4 a1 = *reinterpret_cast<const uint4*>(h + 64 * s + 16);
            av[s] = i32x8{(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
          }
          if (more) layer1_issue(t + 1);
          f32x16 acc2[CT];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc2[ct] = f32x16{};
#pragma unroll
          for (int s = 0; s < KS2; ++s)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc2[ct] = mfma_f8(av[s], w2f[ct][s], acc2[ct]);
          // stored unconditionally (after the last tile into the buffer no
          // wave reads again before the next write), so that the compiler
          // keeps it behind the layer-2 products instead of merging it with
          // the conditional layer-1 issue ahead of them
          layer1_store((t + 1) & 1);
          const int r0 = 32 * t;
          if (r0 + 32 <= m) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
              for (int r = 0; r < 16; r += 2) run[ct] = vmax(vmax(run[ct], acc2[ct][r]), acc2[ct][r + 1]);
          } else {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                const int row = r0 + 8 * (r >> 2) + 4 * g + (r & 3);
                if (row < m) run[ct] = vmax(run[ct], acc2[ct][r]);
              }
          }
          __syncthreads();
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const float f = fmaxf(fmaxf(run[ct], __shfl_xor(run[ct], 32, 64)) * s_enc + bias2[ct], 0.f);
          if (lane < 32) {
            const int col = side * H2 + (wave * CT + ct) * 32 + lane;
            if constexpr (HEAD8) {
              const int q = __builtin_amdgcn_cvt_pk_fp8_f32(fminf(f * inv_z, 448.f), 0.f, 0, false);
              S.z[slot * ZB + col] = (unsigned char)(q & 0xff);
            } else {
              reinterpret_cast<unsigned short*>(S.z)[slot * S_t::ZS + col] = head_bf16::bits(f);
            }
            if (A.z_dbg) A.z_dbg[(size_t)p * 2 * H2 + col] = valid ? f : __builtin_nanf("");
          }
        }
      }
      ++slot;
      __syncthreads();
      if (slot == T) {
        head_tile8<H1, H2, HH, HEAD8>(A, S, T);
        slot = 0;
      }
    }
  }
  if (slot > 0) head_tile8<H1, H2, HH, HEAD8>(A, S, slot);
  if (A.dynamic && tid == 0) {
    __threadfence();
    if (atomicAdd(A.queue + 1, 1u) == gridDim.x - 1) {
      atomicExch(A.queue, 0u);
      atomicExch(A.queue + 1, 0u);
    }
  }
}

// One workgroup per pair (grid-stride); plain FP32 dot products, one output
// feature per thread.  Rows are the crop kernel's bf16 rows, as the FP8
// kernel consumes them.
constexpr int kCalibH1 = 128, kCalibH2 = 256, kCalibHH = 512;

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ __launch_bounds__(256) void calibrate_fp8_kernel(CalibArgs A) {
  __shared__ float x[8];
  __shared__ float h[kCalibH1];
  __shared__ float z[2 * kCalibH2];
  const int tid = threadIdx.x, h1 = A.h1, h2 = A.h2, hh = A.hh, K = A.K;
  const float* W1 = A.w;
  const float* b1 = W1 + 6 * h1;
  const float* W2 = b1 + h1;
  const float* b2 = W2 + (size_t)h2 * h1;
  const float* H1 = b2 + h2;
  const float* c1 = H1 + (size_t)hh * 2 * h2;
  float m_h = 0.f, m_z = 0.f, m_g = 0.f;
  for (int p = blockIdx.x; p < A.n_pairs; p += gridDim.x) {
    const PairMeta mt = A.meta[p];
    if (mt.a < 0) continue;  // the same for the whole workgroup
    for (int side = 0; side < 2; ++side) {
      const int m = side ? mt.m_b : mt.m_a;
      float zr = 0.f;
      for (int r = 0; r < m; ++r) {
        if (tid < 6) {
          const unsigned short bits = A.rows_bf16[((size_t)p * 2 * K + side * K + r) * 8 + tid];
          x[tid] = (float)__builtin_bit_cast(__bf16, bits);
        }
        __syncthreads();
        if (tid < h1) {
          float v = b1[tid];
          for (int c = 0; c < 6; ++c) v += W1[tid * 6 + c] * x[c];
          v = fmaxf(v, 0.f);
          h[tid] = v;
          m_h = fmaxf(m_h, v);
        }
        __syncthreads();
        if (tid < h2) {
          float v = b2[tid];
          for (int k = 0; k < h1; ++k) v += W2[(size_t)tid * h1 + k] * h[k];
          zr = fmaxf(zr, v);
        }
        __syncthreads();
      }
      if (tid < h2) {
        z[side * h2 + tid] = zr;
        m_z = fmaxf(m_z, zr);
      }
    }
    __syncthreads();
    for (int o = tid; o < hh; o += 256) {
      float v = c1[o];
      for (int k = 0; k < 2 * h2; ++k) v += H1[(size_t)o * 2 * h2 + k] * z[k];
      m_g = fmaxf(m_g, v);
    }
    __syncthreads();
  }
  m_h = wave_max(m_h);
  m_z = wave_max(m_z);
  m_g = wave_max(m_g);
  if ((tid & 63) == 0) {  // non-negative floats order as their bit patterns
    atomicMax(A.amax + 0, __float_as_uint(m_h));
    atomicMax(A.amax + 1, __float_as_uint(m_z));
    atomicMax(A.amax + 2, __float_as_uint(m_g));
  }
}

}  // namespace

void fp8_bind(Fp8Args& a, const unsigned char* base, int h1, int h2, int hh, bool head8) {
  const Fp8Layout L = fp8_layout(h1, h2, hh, head8);
  a.w1p = reinterpret_cast<const unsigned short*>(base + L.w1);
  a.w2p = base + L.w2;
  a.b2 = reinterpret_cast<const float*>(base + L.b2);
  a.h1p = base + L.h1;
  a.c1 = reinterpret_cast<const float*>(base + L.c1);
  a.h2p = base + L.h2;
  a.c2 = reinterpret_cast<const float*>(base + L.c2);
  a.h3p = reinterpret_cast<const unsigned short*>(base + L.h3);
  a.c3 = reinterpret_cast<const float*>(base + L.c3);
}

template <int H1, int H2, int HH>
void launch_fp8(const Fp8Args& a, bool head8, int grid, hipStream_t s) {
  if (head8)
    kernel_launch((encoder_head_fp8_kernel<H1, H2, HH, true>), dim3(grid), dim3(256), 0, s, a);
  else
    kernel_launch((encoder_head_fp8_kernel<H1, H2, HH, false>), dim3(grid), dim3(256), 0, s, a);
}

hipError_t launch_encoder_head_fp8(const Fp8Args& a, int h1, int h2, int hh, bool head8, int grid, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (h1 == 64 && h2 == 128 && hh == 256)
    launch_fp8<64, 128, 256>(a, head8, grid, s);
  else if (h1 == 128 && h2 == 256 && hh == 512)
    launch_fp8<128, 256, 512>(a, head8, grid, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_calibrate_fp8(const CalibArgs& a, int grid, hipStream_t s) {
  if (a.h1 > kCalibH1 || a.h2 > kCalibH2 || a.hh > kCalibHH || a.h1 > 256 || a.h2 > 256)
    return hipErrorInvalidValue;
  if (a.n_pairs <= 0) return hipSuccess;
  kernel_launch(calibrate_fp8_kernel, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace locc
