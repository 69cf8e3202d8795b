// BF16 encoder + head kernel of the split schedule with layer 2's weights in
// LDS: one workgroup of eight waves per CU (the schedule's one workgroup per
// CU).  The crop kernel has written each pair's encoder rows (bf16) and its
// record; this kernel runs the per-point encoder with the per-object
// max-pool (Sec. III: per-point MLP features, max-pooled; appendix: ReLU on
// every layer) and the MLP head (appendix: an MLP on the concatenated pooled
// features ending in a linear layer), then the world-frame epilogue.
//
// Work: groups of 64 pairs (group k, k + grid, ...).  Inside a group the
// waves take object sides (pair, object) from an LDS counter, and each wave
// encodes a whole side by itself over all h2 output columns:
//   layer 1 (v_mfma_f32_32x32x8_bf16, computed transposed, bias on the
//     constant-1 input) for two 32-row tiles at a time; a lane's 16 features
//     of a 32-feature tile, converted to bf16, are two k-steps of its own
//     layer-2 A operand (layer 2's reduction index permuted on the host to
//     F(ft, g, r) = 32 ft + 8 (r / 4) + 4 g + r % 4), so layer 1 never leaves
//     registers;
//   layer 2 (v_mfma_f32_32x32x16_bf16) column tile by column tile, each W2
//     B fragment read once from LDS for both row tiles, and the raw sums
//     max-pooled per column as soon as a column tile is done.
// No barrier falls inside the encoder.  When the group's 128 sides are done,
// the eight waves run the head on the group's two 32-pair tiles at once, each
// head weight fragment streamed from L2 once for both (the head's first layer
// overwrites the W2 fragments in LDS, which are reloaded from L2 afterwards).
// Lane layouts (wave64): A[i][k]: i = l % 32, k = (K/2) (l / 32) + e;
// B[k][j]: j = l % 32, same k; D[i][j]: j = l % 32, i = 8 (r / 4) + 4 (l / 32)
// + r % 4 for register r.
#include "fused.h"
#include "head_bf16.h"
#include "post.h"

#include <type_traits>

namespace locc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kGroup = 2 * kFusedTile;  // pairs per group: two head tiles

// ReLU(bf16(a)), ReLU(bf16(b)) in one word (round to nearest even).
__device__ __forceinline__ unsigned bf16x2_relu(float a, float b) {
  const bf16x2 h = __builtin_convertvector((f32x2){a, b}, bf16x2);
  return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), (s16x2){0, 0}));
}

// IEEE maximum: no canonicalisation of the matrix-core results.
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_elementwise_maximum(a, b); }

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);  // round to nearest even
}

__device__ __forceinline__ f32x16 mfma_k8(s16x4 a, s16x4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_k16(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

template <int H1, int H2, int HH>
struct SmemL {
  static constexpr int T = kFusedTile;
  static constexpr int ZS = (2 * H2 > HH ? 2 * H2 : HH) + 8;  // row stride (bf16) of a z tile
  static constexpr int GS = HH + 8;                           // row stride of a g1 tile
  static constexpr int NW2 = (H2 / 32) * (H1 / 16) * 64;      // W2 B fragments (u16x8 each)
  union {
    u16x8 w2[NW2];                 // layer-2 B fragments: [column tile][k-step][lane]
    unsigned short g[2][T * GS];   // the head's layer-1 outputs of the two tiles
  } u;
  unsigned short z[2][T * ZS];     // pooled features [f_a, f_b] of the group's pairs, bf16
  float y[2][4][T][8];             // per tile: the four layer-3 waves' parts of the raw outputs
  int32_t m[kGroup][2];            // rows per object (0 for an invalid pair)
  int32_t a[kGroup];               // canonical first object, -1: invalid pair
  int32_t swapped[kGroup];
  int32_t next;                    // next unclaimed side of the group
};

template <int H1, int H2, int HH, bool ARGMAX>
__global__ __launch_bounds__(64 * kWaves, 1) void encoder_bf16_kernel(FusedArgs A) {
  using S_t = SmemL<H1, H2, HH>;
  constexpr int T = S_t::T, ZS = S_t::ZS, GS = S_t::GS;
  constexpr int FT = H1 / 32;   // layer-1 feature tiles
  constexpr int KS2 = H1 / 16;  // layer-2 k-steps
  constexpr int NCT = H2 / 32;  // layer-2 column tiles
  static_assert(H1 % 32 == 0 && H2 % 32 == 0 && HH % 128 == 0, "widths");
  __shared__ S_t S;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = wave >> 2;  // head tile whose unused rows this half of the workgroup clears
  const int g = lane >> 5;
  const int l32 = lane & 31;
  const int K = A.K;
  const int P = pair_count(A.n_pairs, A.n_pairs_dev, A.dev_base);

  s16x4 w1f[FT];
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) w1f[ft] = reinterpret_cast<const s16x4*>(A.w1p)[(size_t)ft * 64 + lane];
  float bias2[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) bias2[ct] = A.b2[ct * 32 + l32];
  auto load_w2 = [&]() {
    for (int i = tid; i < S_t::NW2; i += 64 * kWaves) S.u.w2[i] = reinterpret_cast<const u16x8*>(A.w2p)[i];
  };
  load_w2();

  // layer 1 of one or two 32-row tiles (x0, x1: this lane's four inputs of row l32 of each) into layer
  // 2's A operands; the two tiles' products of a feature tile issue back to back, so that one's
  // conversion runs behind the other's product
  auto layer1 = [&](auto two_c, s16x4 x0, s16x4 x1, u16x8 (&out0)[KS2], u16x8 (&out1)[KS2])
      __attribute__((always_inline)) {
    constexpr bool TWO = decltype(two_c)::value;
    auto cvt = [&](const f32x16& a1, int ft, u16x8 (&out)[KS2]) __attribute__((always_inline)) {
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        u32x4 w;
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = bf16x2_relu(a1[8 * hf + 2 * e], a1[8 * hf + 2 * e + 1]);
        out[2 * ft + hf] = __builtin_bit_cast(u16x8, w);
      }
    };
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      const f32x16 a0 = mfma_k8(w1f[ft], x0, f32x16{});
      f32x16 a1;
      if constexpr (TWO) a1 = mfma_k8(w1f[ft], x1, f32x16{});
      cvt(a0, ft, out0);
      if constexpr (TWO) cvt(a1, ft, out1);
    }
  };

  for (int group = blockIdx.x;; group += gridDim.x) {
    const int base = group * kGroup;
    if (base >= P) break;  // uniform
    const int n_grp = P - base < kGroup ? P - base : kGroup;
    __syncthreads();  // the previous group's records and z tiles are no longer read
    if (tid < kGroup) {
      int a = -1, sw = 0, ma = 0, mb = 0;
      if (tid < n_grp) {
        const PairMeta mt = A.meta[base + tid];
        if (mt.a >= 0) {
          a = mt.a;
          sw = mt.swapped;
          ma = mt.m_a;
          mb = mt.m_b;
        }
      }
      S.a[tid] = a;
      S.swapped[tid] = sw;
      S.m[tid][0] = ma;
      S.m[tid][1] = mb;
    }
    if (tid == 0) S.next = 0;
    __syncthreads();

    // ---------------------------------------------------------------- encoder
    // Max-pool of the raw layer-2 sums; bias and ReLU once per column
    // afterwards: fl(max_r a_r + b) = max_r fl(a_r + b) because rounding is
    // monotone, and ReLU is monotone (an empty set gives max(-inf + b, 0) = 0).
    // Each wave claims its next side as it starts one, and the rows of the
    // next tile pair (of this side, else of the next side) load while the
    // current pair of tiles computes.
    auto claim = [&]() __attribute__((always_inline)) -> int {
      int item = 0;
      if (lane == 0) item = atomicAdd(&S.next, 1);
      return __builtin_amdgcn_readfirstlane(__shfl(item, 0, 64));
    };
    auto rows_at = [&](int item) __attribute__((always_inline)) -> const unsigned short* {
      const int slot = item >> 1, sd = item & 1;
      return A.rows_bf16 + ((size_t)(base + slot) * 2 * K + (size_t)sd * K + l32) * 8 + 4 * g;
    };
    const int n_items = 2 * n_grp;
    int item = claim();
    s16x4 nx0{}, nx1{};
    if (item < n_items && S.m[item >> 1][item & 1] > 0) {
      const unsigned short* R0 = rows_at(item);
      nx0 = *reinterpret_cast<const s16x4*>(R0);
      if (S.m[item >> 1][item & 1] > 32) nx1 = *reinterpret_cast<const s16x4*>(R0 + 32 * 8);
    }
    while (item < n_items) {  // uniform over the wave
      const int nitem = claim();
      const int slot = item >> 1, sd = item & 1;
      const int p = base + slot;
      const int m = S.m[slot][sd];
      const int nt = (m + 31) >> 5;
      const unsigned short* R = rows_at(item);
      const int nm = nitem < n_items ? S.m[nitem >> 1][nitem & 1] : 0;
      const unsigned short* NR = rows_at(nitem < n_items ? nitem : item);
      // rows of tile pair t + 2 of this side, else of the next side's first pair
      auto prefetch = [&](int t) __attribute__((always_inline)) {
        if (t + 2 < nt) {
          nx0 = *reinterpret_cast<const s16x4*>(R + (size_t)(t + 2) * 32 * 8);
          if (t + 3 < nt) nx1 = *reinterpret_cast<const s16x4*>(R + (size_t)(t + 3) * 32 * 8);
        } else if (nm > 0) {
          nx0 = *reinterpret_cast<const s16x4*>(NR);
          if (nm > 32) nx1 = *reinterpret_cast<const s16x4*>(NR + 32 * 8);
        }
      };
      float run[NCT];
      int arg[NCT];  // argmax variant: the row of run (255: none yet)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        run[ct] = -__builtin_inff();
        arg[ct] = 255;
      }
      // pooling of column tile ct of the row tile that starts at r0
      auto pool = [&](const f32x16& acc, int ct, int r0) __attribute__((always_inline)) {
        if constexpr (ARGMAX) {
          // a lane's rows ascend with r, and tiles ascend with r0: strict > keeps the first maximum
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = r0 + 8 * (r >> 2) + 4 * g + (r & 3);
            if (row < m && acc[r] > run[ct]) {
              run[ct] = acc[r];
              arg[ct] = row;
            }
          }
        } else if (r0 + 32 <= m) {
#pragma unroll
          for (int r = 0; r < 16; r += 2) run[ct] = vmax(vmax(run[ct], acc[r]), acc[r + 1]);
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = r0 + 8 * (r >> 2) + 4 * g + (r & 3);
            if (row < m) run[ct] = vmax(run[ct], acc[r]);
          }
        }
      };
      // two row tiles t, t + 1 (TWO) or the last one alone
      auto tiles = [&](auto two_c, int t, s16x4 x0, s16x4 x1) __attribute__((always_inline)) {
        constexpr bool TWO = decltype(two_c)::value;
        u16x8 av0[KS2], av1[KS2];
        layer1(two_c, x0, x1, av0, av1);
        // The B fragments of column tile ct + 1 are requested while the products of tile ct run; scheduling
        // fences between column tiles keep each tile's fragments and sums within the register budget
        // (unfenced, the compiler hoists every fragment load of the fully unrolled loop).
        u16x8 bq[KS2];
#pragma unroll
        for (int s = 0; s < KS2; ++s) bq[s] = S.u.w2[s * 64 + lane];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          u16x8 bn[KS2];
          if (ct + 1 < NCT) {
#pragma unroll
            for (int s = 0; s < KS2; ++s) bn[s] = S.u.w2[((ct + 1) * KS2 + s) * 64 + lane];
          }
          f32x16 acc0 = f32x16{}, acc1 = f32x16{};
#pragma unroll
          for (int s = 0; s < KS2; ++s) {
            acc0 = mfma_k16(av0[s], bq[s], acc0);
            if constexpr (TWO) acc1 = mfma_k16(av1[s], bq[s], acc1);
          }
          pool(acc0, ct, 32 * t);
          if constexpr (TWO) pool(acc1, ct, 32 * (t + 1));
          if (ct + 1 < NCT) {
#pragma unroll
            for (int s = 0; s < KS2; ++s) bq[s] = bn[s];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      int t = 0;
      for (; t + 1 < nt; t += 2) {
        const s16x4 x0 = nx0, x1 = nx1;
        prefetch(t);
        tiles(std::true_type{}, t, x0, x1);
      }
      if (t < nt) {
        const s16x4 x0 = nx0;
        prefetch(t);
        tiles(std::false_type{}, t, x0, x0);
      }
      if (nt == 0) prefetch(0);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const float other = __shfl_xor(run[ct], 32, 64);
        const float f = fmaxf(fmaxf(run[ct], other) + bias2[ct], 0.f);
        if constexpr (ARGMAX) {
          // the two half-waves hold rows 4g + ... of every tile: the larger value wins, the lower row on ties
          const int other_arg = __shfl_xor(arg[ct], 32, 64);
          const bool take = other > run[ct] || (other == run[ct] && other_arg < arg[ct]);
          if (lane < 32) A.amax[((size_t)p * 2 + sd) * H2 + ct * 32 + lane] = (uint8_t)(take ? other_arg : arg[ct]);
        }
        if (lane < 32) {
          const int col = sd * H2 + ct * 32 + lane;
          if constexpr (!ARGMAX) S.z[slot / T][(slot % T) * ZS + col] = bf16_bits(f);
          if (A.z_dbg) A.z_dbg[(size_t)p * 2 * H2 + col] = S.a[slot] >= 0 ? f : __builtin_nanf("");
        }
      }
      item = nitem;
    }
    if constexpr (!ARGMAX) {
      // ------------------------------------------------------------------ head
      __syncthreads();  // every side's features are in z, and no wave reads W2 any more
      const int n_half = n_grp - T * half < 0 ? 0 : (n_grp - T * half < T ? n_grp - T * half : T);
      for (int e = tid - 256 * half; e < (T - n_half) * ZS; e += 256) S.z[half][n_half * ZS + e] = 0;
      __syncthreads();
      head_bf16::layers2t<H2, HH, ZS, GS, 4>(A.h1p, A.c1, A.h2p, A.c2, A.h3p, S.z[0], S.z[1], S.u.g[0], S.u.g[1],
                                             S.y[0], S.y[1], wave);
      __syncthreads();
      {
        const int i = tid >> 3, j = tid & 7;  // 512 threads: row i % 32 of tile i / 32
        const int h = i >> 5, r = i & 31;
        S.y[h][0][r][j] = ((S.y[h][0][r][j] + S.y[h][1][r][j]) + S.y[h][2][r][j]) + S.y[h][3][r][j] + A.c3[j];
      }
      __syncthreads();
      if (tid < n_grp)
        post_contact(A.objs, S.a[tid], S.swapped[tid], S.y[tid / T][0][tid % T], A.out, A.y_dbg, base + tid);
      __syncthreads();  // g (over the W2 fragments) is read no more
      if (base + (int)gridDim.x * kGroup < P) load_w2();  // uniform: this workgroup has another group
    }
  }
}

}  // namespace

hipError_t launch_encoder_head_bf16_lds(const FusedArgs& a, int h1, int h2, int hh, int grid, bool argmax,
                                        hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (!a.rows_bf16 || !a.meta || grid < 1) return hipErrorInvalidValue;
  if (argmax && (!a.z_dbg || !a.amax)) return hipErrorInvalidValue;
  const dim3 block(64 * kWaves);
#define LOCC_LDS_CASE(H1, H2, HH)                                                               \
  if (h1 == H1 && h2 == H2 && hh == HH) {                                                       \
    if (argmax)                                                                                 \
      kernel_launch((encoder_bf16_kernel<H1, H2, HH, true>), dim3(grid), block, 0, s, a);       \
    else                                                                                        \
      kernel_launch((encoder_bf16_kernel<H1, H2, HH, false>), dim3(grid), block, 0, s, a);      \
    return hipGetLastError();                                                                   \
  }
  LOCC_LDS_CASE(64, 128, 256)
  LOCC_LDS_CASE(128, 256, 512)
#undef LOCC_LDS_CASE
  return hipErrorInvalidValue;
}

}  // namespace locc
