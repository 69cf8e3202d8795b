// FP32 network of the LOCC path: per-point encoder with per-object max-pool,
// then the pair head and the world-frame epilogue.
//
// Encoder (per pair, 2K rows of (x, y, z, nx, ny, nz) in a's frame):
//   h1 = ReLU(W1 r + b1), h2 = ReLU(W2 h1 + b2), f = max over the valid rows
// of each object (0 when none); the paper's shape encoder is likewise a
// per-point MLP whose features are max-pooled (Sec. III, appendix).
// Head (per pair): y = H3 ReLU(H2 ReLU(H1 [f_a, f_b] + c1) + c2) + c3, the
// paper's predictor being an MLP on the pooled crop features that ends in a
// linear layer (appendix).  Outputs: logit y0, contact point R_a y[1:4] + t_a,
// normal sgn R_a y[4:7], depth y7.
//
// MFMA v_mfma_f32_32x32x2_f32 operand layout (lane l of a wave64):
//   A[i][k]: i = l % 32, k = l / 32;   B[k][j]: j = l % 32, k = l / 32;
//   D[i][j] in 16 registers r: j = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4.
// Encoder: layer 1 is computed transposed (h1^T = [W1 | b1] [r; 1]), so each
// lane ends up holding 16 features of ONE point per 32-feature tile.  Those
// values are layer 2's A operand if layer 2's reduction index is permuted to
// F(ft, g, r) = 32 ft + 8 (r / 4) + 4 g + r % 4; the host packs W2 in that
// order.  Each wave computes its share of layer 1's feature tiles and stores
// them, in the order its lanes hold them, to an LDS tile that all four waves
// read back four reduction steps at a time.  W2's slice for the wave (h2 / 4
// output columns) is loaded once per workgroup and stays in registers for
// every pair the persistent workgroup processes.
#include "locc_internal.h"

#include <cmath>
#include <cstring>

namespace locc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// IEEE maximum (NaN-propagating, -0 < +0).  Matrix-core results are not
// known to be canonical floats, so fmaxf would canonicalise each operand
// first; maximum needs no canonicalisation and chains into v_maximum3_f32.
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_elementwise_maximum(a, b); }

// Index of the calling wave in its workgroup, wave-uniform (scalar register).
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6); }

__device__ __forceinline__ f32x16 mfma32x32x2(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__host__ __device__ constexpr int perm_feature(int ft, int g, int r) { return 32 * ft + 8 * (r / 4) + 4 * g + r % 4; }

// -------------------------------------------------------------------- encoder
// ARGMAX: also record, per object and channel, the row of the largest raw
// sum (the first such row on ties), for the pose-gradient path.
// Workgroups per compute unit: with layer 1 shared through LDS a wave needs
// at most 244 registers at widths 128 / 256 (two workgroups per CU) and 122 at
// 64 / 128 (four), so that one workgroup's matrix-core work hides another's
// waits.
template <int H1>
constexpr int encoder_wg_per_cu() { return H1 <= 64 ? 4 : 2; }

template <int H1, int H2, bool ARGMAX>
__global__ __launch_bounds__(256, encoder_wg_per_cu<H1>()) void encoder_fp32_kernel(Fp32Net W, NetArgs A) {
  constexpr int FT = H1 / 32;   // 32-feature tiles of layer 1
  constexpr int KS = H1 / 2;    // layer-2 k-steps
  constexpr int CT = H2 / 128;  // 32-column tiles per wave
  constexpr int FW = (FT + 3) / 4;  // layer-1 feature tiles per wave (tiles wave, wave + 4, ...)
  constexpr int HR = FT * 16 + 4;   // floats per (lane group, point) row of the layer-1 tile
  static_assert(H1 % 32 == 0 && H2 % 128 == 0, "widths");
  // layer-1 output of a 32-row tile, double-buffered: [g][point][ft][16] in
  // the order each lane holds it (feature perm_feature(ft, g, r) at r), rows
  // padded to 4 mod 32 floats so that float4 accesses by 8 lanes hit 32 banks
  __shared__ __align__(16) float h1s[2][64 * HR];
  const int lane = threadIdx.x & 63;
  const int wave = wave_index();
  const int g = lane >> 5;
  const int l32 = lane & 31;
  const int K = A.K;

  float w1f[FW][4];
#pragma unroll
  for (int i = 0; i < FW; ++i)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      w1f[i][s] = wave + 4 * i < FT ? W.w1pack[((wave + 4 * i) * 4 + s) * 64 + lane] : 0.f;
  float w2f[CT][KS];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int s = 0; s < KS; ++s) w2f[ct][s] = W.w2pack[((wave * CT + ct) * KS + s) * 64 + lane];
  float bias2[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) bias2[ct] = W.b2[(wave * CT + ct) * 32 + (lane & 31)];

  const int P = pair_count(A.n_pairs, A.n_pairs_dev);
  for (int p = blockIdx.x; p < P; p += gridDim.x) {
    const PairMeta mt = A.meta[p];
    float* zp = A.z + (size_t)p * 2 * H2;
    if (mt.a < 0) {
      if (lane < 32)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          zp[(wave * CT + ct) * 32 + lane] = __builtin_nanf("");
          zp[H2 + (wave * CT + ct) * 32 + lane] = __builtin_nanf("");
        }
      continue;
    }
    for (int side = 0; side < 2; ++side) {
      const int m = side ? mt.m_b : mt.m_a;
      // max-pool of the raw sums, bias and ReLU once per column afterwards
      // (exact: rounding and ReLU are monotone; an empty set gives 0)
      float run[CT];
      int arg[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        run[ct] = -__builtin_inff();
        arg[ct] = 255;
      }
      const float* rbase = A.rows + ((size_t)p * 2 * K + side * K) * kRowFloats;
      // Row tiles t = 0, 1, ...: each wave computes its layer-1 feature tiles
      // of tile t + 1 while layer 2 of tile t runs and stores them (ReLU
      // applied) to the other LDS buffer; one barrier per tile publishes them
      // (the buffer written in tile t was last read in tile t - 1, before the
      // previous barrier).
      const int nt = (m + 31) >> 5;  // uniform over the workgroup
      f32x16 acc1[FW];
      float4 xv = *reinterpret_cast<const float4*>(rbase + l32 * kRowFloats + 4 * g);
      auto layer1_issue = [&](int t) {
        const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
        for (int i = 0; i < FW; ++i)
          if (FT % 4 == 0 || wave + 4 * i < FT) {
            acc1[i] = f32x16{};
#pragma unroll
            for (int s = 0; s < 4; ++s) acc1[i] = mfma32x32x2(w1f[i][s], xs[s], acc1[i]);
          }
        if (t + 1 < nt) xv = *reinterpret_cast<const float4*>(rbase + ((t + 1) * 32 + l32) * kRowFloats + 4 * g);
      };
      auto layer1_store = [&](int buf) {
        float* dst = &h1s[buf][(g * 32 + l32) * HR];
#pragma unroll
        for (int i = 0; i < FW; ++i) {
          const int ft = wave + 4 * i;
          if (FT % 4 == 0 || ft < FT)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              *reinterpret_cast<float4*>(dst + ft * 16 + 4 * j) =
                  make_float4(vmax(acc1[i][4 * j], 0.f), vmax(acc1[i][4 * j + 1], 0.f),
                              vmax(acc1[i][4 * j + 2], 0.f), vmax(acc1[i][4 * j + 3], 0.f));
        }
      };
      if (nt > 0) {
        layer1_issue(0);
        layer1_store(0);
      }
      __syncthreads();
      for (int t = 0; t < nt; ++t) {
        const int r0 = 32 * t;
        const bool more = t + 1 < nt;
        if (more) layer1_issue(t + 1);
        const float* src = &h1s[t & 1][(g * 32 + l32) * HR];
        f32x16 acc2[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc2[ct] = f32x16{};
#pragma unroll
        for (int ft = 0; ft < FT; ++ft)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float4 a = *reinterpret_cast<const float4*>(src + ft * 16 + 4 * j);
            const float h[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) acc2[ct] = mfma32x32x2(h[e], w2f[ct][ft * 16 + 4 * j + e], acc2[ct]);
          }
        if (more) layer1_store((t + 1) & 1);
        if (ARGMAX) {
          // a lane's rows ascend with r, and blocks ascend with r0: strict > keeps the first maximum
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int row = r0 + 8 * (r >> 2) + 4 * g + (r & 3);
              if (row < m && acc2[ct][r] > run[ct]) {
                run[ct] = acc2[ct][r];
                arg[ct] = row;
              }
            }
        } else if (r0 + 32 <= m) {
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
        const float other = __shfl_xor(run[ct], 32, 64);
        const float f = fmaxf(fmaxf(run[ct], other) + bias2[ct], 0.f);
        if (lane < 32) zp[side * H2 + (wave * CT + ct) * 32 + lane] = f;
        if (ARGMAX) {
          // the two half-waves hold rows 4g + ... of every block: the larger value wins, the lower row on ties
          const int other_arg = __shfl_xor(arg[ct], 32, 64);
          const bool take = other > run[ct] || (other == run[ct] && other_arg < arg[ct]);
          if (lane < 32)
            A.amax[((size_t)p * 2 + side) * H2 + (wave * CT + ct) * 32 + lane] = (uint8_t)(take ? other_arg : arg[ct]);
        }
      }
    }
  }
}

// ----------------------------------------------------------------------- head
constexpr int kHeadPairs = 32;

template <int Z, int HH>
__global__ __launch_bounds__(256, 1) void head_fp32_kernel(Fp32Net W, NetArgs A) {
  constexpr int LZ = Z + 1;    // odd row strides: conflict-free column reads
  constexpr int LG = HH + 1;
  constexpr int CTH = HH / 128;
  extern __shared__ float smem[];
  float* zt = smem;                      // [32][LZ], later reused for g2 [32][LG]
  float* gt = smem + kHeadPairs * (LZ > LG ? LZ : LG);  // [32][LG]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_index();
  const int g = lane >> 5;
  const int p0 = blockIdx.x * kHeadPairs;
  const int P = pair_count(A.n_pairs, A.n_pairs_dev);
  if (p0 >= P) return;  // uniform

  for (int e = tid; e < kHeadPairs * Z; e += 256) {
    const int i = e / Z, k = e - i * Z;
    const int p = p0 + i;
    float v = 0.f;
    if (p < P) {
      v = A.z[(size_t)p * Z + k];
      if (v != v) v = 0.f;  // invalid pair: its outputs are NaN-ed in the epilogue
    }
    zt[i * LZ + k] = v;
  }
  __syncthreads();

  // layer 1: g1 = ReLU(zt H1^T + c1) -> gt ; layer 2: g2 = ReLU(gt H2^T + c2) -> zt
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const float* src = layer == 0 ? zt : gt;
    float* dst = layer == 0 ? gt : zt;
    const int LS = layer == 0 ? LZ : LG;
    const int LD = LG;
    const int KS = (layer == 0 ? Z : HH) / 2;
    const float* pack = layer == 0 ? W.h1pack : W.h2pack;
    const float* bias = layer == 0 ? W.c1 : W.c2;
    f32x16 acc[CTH];
#pragma unroll
    for (int ct = 0; ct < CTH; ++ct) acc[ct] = f32x16{};
    const float* arow = src + (lane & 31) * LS + g;
#pragma unroll 4
    for (int s = 0; s < KS; ++s) {
      const float av = arow[2 * s];
#pragma unroll
      for (int ct = 0; ct < CTH; ++ct)
        acc[ct] = mfma32x32x2(av, pack[((size_t)(wave * CTH + ct) * KS + s) * 64 + lane], acc[ct]);
    }
    __syncthreads();  // everyone is done reading dst's previous contents (layer 1 read zt)
#pragma unroll
    for (int ct = 0; ct < CTH; ++ct) {
      const int col = (wave * CTH + ct) * 32 + (lane & 31);
      const float bc = bias[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * g + (r & 3);
        dst[row * LD + col] = fmaxf(acc[ct][r] + bc, 0.f);
      }
    }
    __syncthreads();
  }

  // layer 3 (8 outputs per pair): one thread per (pair, output)
  __shared__ float ys[kHeadPairs][8];
  {
    const int i = tid >> 3, o = tid & 7;
    const float* h3 = W.h3 + (size_t)o * HH;
    const float* g2 = zt + i * LG;
    float acc = 0.f;
    for (int k = 0; k < HH; ++k) acc += g2[k] * h3[k];
    ys[i][o] = acc + W.c3[o];
  }
  __syncthreads();

  if (tid < kHeadPairs) {
    const int p = p0 + tid;
    if (p < P) {
      const PairMeta mt = A.meta[p];
      float out[8];
      const float* y = ys[tid];
      if (mt.a < 0) {
        for (int k = 0; k < 8; ++k) out[k] = __builtin_nanf("");
      } else {
        const locc_object o = A.objs[mt.a];
        const double w = o.q[0], x = o.q[1], yq = o.q[2], zq = o.q[3];
        const double R[9] = {1.0 - 2.0 * (yq * yq + zq * zq), 2.0 * (x * yq - w * zq), 2.0 * (x * zq + w * yq),
                             2.0 * (x * yq + w * zq), 1.0 - 2.0 * (x * x + zq * zq), 2.0 * (yq * zq - w * x),
                             2.0 * (x * zq - w * yq), 2.0 * (yq * zq + w * x), 1.0 - 2.0 * (x * x + yq * yq)};
        const double sg = mt.swapped ? -1.0 : 1.0;
        out[0] = y[0];
        for (int r = 0; r < 3; ++r) {
          out[1 + r] = (float)(R[3 * r] * y[1] + R[3 * r + 1] * y[2] + R[3 * r + 2] * y[3] + (double)o.p[r]);
          out[4 + r] = (float)(sg * (R[3 * r] * y[4] + R[3 * r + 1] * y[5] + R[3 * r + 2] * y[6]));
        }
        out[7] = y[7];
      }
      float4* dst = reinterpret_cast<float4*>(A.out + p);
      dst[0] = make_float4(out[0], out[1], out[2], out[3]);
      dst[1] = make_float4(out[4], out[5], out[6], out[7]);
      if (A.y_dbg) {
        float4* yd = reinterpret_cast<float4*>(A.y_dbg + (size_t)p * 8);
        const float nan = __builtin_nanf("");
        yd[0] = mt.a < 0 ? make_float4(nan, nan, nan, nan) : make_float4(y[0], y[1], y[2], y[3]);
        yd[1] = mt.a < 0 ? make_float4(nan, nan, nan, nan) : make_float4(y[4], y[5], y[6], y[7]);
      }
    }
  }
}

template <int Z, int HH>
size_t head_smem_bytes() {
  constexpr int LZ = Z + 1, LG = HH + 1;
  return sizeof(float) * kHeadPairs * ((LZ > LG ? LZ : LG) + LG);
}

template <int H1, int H2>
hipError_t run_encoder(const Fp32Net& w, const NetArgs& a, int n_cu, hipStream_t s) {
  const int slots = encoder_wg_per_cu<H1>() * n_cu;
  int grid = a.n_pairs < slots ? a.n_pairs : slots;
  if (a.amax)
    kernel_launch((encoder_fp32_kernel<H1, H2, true>), dim3(grid), dim3(256), 0, s, w, a);
  else
    kernel_launch((encoder_fp32_kernel<H1, H2, false>), dim3(grid), dim3(256), 0, s, w, a);
  return hipGetLastError();
}

template <int Z, int HH>
hipError_t run_head(const Fp32Net& w, const NetArgs& a, hipStream_t s) {
  const size_t smem = head_smem_bytes<Z, HH>();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&head_fp32_kernel<Z, HH>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const int grid = (a.n_pairs + kHeadPairs - 1) / kHeadPairs;
  kernel_launch((head_fp32_kernel<Z, HH>), dim3(grid), dim3(256), smem, s, w, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_encoder_fp32(const Fp32Net& w, const NetArgs& a, int n_cu, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (w.h1 == 64 && w.h2 == 128) return run_encoder<64, 128>(w, a, n_cu, s);
  if (w.h1 == 128 && w.h2 == 256) return run_encoder<128, 256>(w, a, n_cu, s);
  return hipErrorInvalidValue;
}

hipError_t launch_head_fp32(const Fp32Net& w, const NetArgs& a, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (w.h2 == 128 && w.hh == 256) return run_head<256, 256>(w, a, s);
  if (w.h2 == 256 && w.hh == 512) return run_head<512, 512>(w, a, s);
  return hipErrorInvalidValue;
}

Fp32Net fp32_view(const float* base, int h1, int h2, int hh) {
  const Fp32Layout L = fp32_layout(h1, h2, hh);
  return Fp32Net{h1, h2, hh, base + L.w1, base + L.w2, base + L.b2, base + L.h1,
                 base + L.c1, base + L.h2, base + L.c2, base + L.h3, base + L.c3};
}

}  // namespace locc
