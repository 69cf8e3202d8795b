// Fused persistent kernel of the LOCC path in BF16: crop, encoder, head and
// world mapping for all pairs in one launch.
//
// Each workgroup (4 wave64) claims pairs from a device queue (or a static
// round robin).  For every claimed pair it runs the float64 crop of
// geometry.h (scan, ordered first-K selection), gathers the encoder rows into
// LDS as bf16, and runs the per-point encoder with a per-object max-pool
// (Sec. III: per-point MLP features, max-pooled; appendix: ReLU on every
// layer).  The pooled features [f_a, f_b] go into an LDS tile; every 32
// pairs (and once at the end) the head MLP runs on the tile (appendix: MLP
// predictor ending in a linear layer) and the contacts are written.
//
// Matrix cores: v_mfma_f32_32x32x8_bf16 for encoder layer 1 (inputs x, y, z,
// nx, ny, nz, 1, 0: the bias rides in the 7th input), v_mfma_f32_32x32x16_bf16
// for encoder layer 2 and the head, FP32 accumulation.  Lane layouts (wave64):
//   A[i][k]: i = l % 32, k = (K/2) (l / 32) + e;  B[k][j]: j = l % 32, same k;
//   D[i][j]: j = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4 for register r.
// Encoder layer 1 is computed transposed (features x points), so each lane
// holds 16 features of one point per 32-feature tile; in that order they are
// 16-byte pieces of layer 2's A operand once layer 2's reduction index is
// permuted to F(ft, g, r) = 32 ft + 8 (r / 4) + 4 g + r % 4 (the host packs W2
// so).  With h1 = 128 each wave computes one feature tile of every 32-row
// tile and shares it through a double-buffered LDS tile (one barrier per row
// tile), instead of every wave computing all of layer 1.
// Wave w owns h2/4 encoder output columns; its W2 slice (64 VGPRs at h2 =
// 256) is loaded once and stays in registers for the whole kernel.
//
// The queue is self-cleaning: the last workgroup to finish resets it, so
// consecutive launches (and graph replays) need no memset.
//
// Split schedule (PRE = true): the crop runs in its own high-occupancy kernel
// (crop.hip, bf16 rows + per-pair records in HBM) and this kernel runs only
// the encoder and head; the crop's dependent loads then overlap across many
// more resident workgroups than the encoder's register budget allows.
#include "fused.h"
#include "geometry.h"
#include "head_bf16.h"
#include "post.h"

#include <cstring>

namespace locc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// ReLU(bf16(a)), ReLU(bf16(b)) packed in one word: one v_cvt_pk_bf16_f32
// (round to nearest even) and one v_pk_max_i16 for two values.
__device__ __forceinline__ unsigned bf16x2_relu(float a, float b) {
  const bf16x2 h = __builtin_convertvector((f32x2){a, b}, bf16x2);
  return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), (s16x2){0, 0}));
}

// IEEE maximum (NaN-propagating, -0 < +0).  The matrix-core results feeding
// the max-pool are not known to be canonical floats, so fmaxf would
// canonicalise each operand first; maximum needs no canonicalisation and
// chains into v_maximum3_f32.
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_elementwise_maximum(a, b); }

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  const __bf16 h = (__bf16)f;  // round to nearest even
  return __builtin_bit_cast(unsigned short, h);
}

__device__ __forceinline__ f32x16 mfma_k8(s16x4 a, s16x4 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_k16(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

template <int H1, int H2, int HH>
struct Smem {
  static constexpr int T = kFusedTile;
  static constexpr int ZS = (2 * H2 > HH ? 2 * H2 : HH) + 8;  // row stride (bf16) of the z / g2 tile
  static constexpr int GS = HH + 8;                           // row stride of the g1 tile
  static constexpr int HS = H1 + 8;                           // row stride of the layer-1 tiles
  union {
    struct {
      CropShared crop;
      alignas(16) unsigned short rows[2 * kMaxK * 8];  // encoder rows (x, y, z, nx, ny, nz, 1, 0), bf16
      alignas(16) unsigned short h1t[2][T * HS];       // layer-1 output of a 32-row tile, [row][permuted feature]
    } c;
    unsigned short g[T * GS];
  } u;
  unsigned short z[T * ZS];
  float y[4][T][8];
  int32_t pair[T];
  int32_t a[T];
  int32_t swapped[T];
  int32_t claim;
};

// Head on the first n rows of the z tile, then the world-frame epilogue.
// D: k-steps of weight fragments in flight (registers permitting)
template <int H1, int H2, int HH, int D>
__device__ __forceinline__ void head_tile(const FusedArgs& A, Smem<H1, H2, HH>& S, int n) {
  using S_t = Smem<H1, H2, HH>;
  constexpr int T = S_t::T, ZS = S_t::ZS, GS = S_t::GS;
  const int tid = threadIdx.x;
  for (int e = tid; e < (T - n) * ZS; e += 256) S.z[n * ZS + e] = 0;
  __syncthreads();
  head_bf16::layers<H2, HH, ZS, GS, D>(A.h1p, A.c1, A.h2p, A.c2, A.h3p, S.z, S.u.g, S.y);
  __syncthreads();
  for (int t = tid; t < T * 8; t += 256) {
    const int i = t >> 3, j = t & 7;
    S.y[0][i][j] = ((S.y[0][i][j] + S.y[1][i][j]) + S.y[2][i][j]) + S.y[3][i][j] + A.c3[j];
  }
  __syncthreads();
  if (tid < n) post_contact(A.objs, S.a[tid], S.swapped[tid], S.y[0][tid], A.out, A.y_dbg, S.pair[tid]);
  __syncthreads();
}

// ARGMAX (split schedule only): the encoder alone, with per channel the row of its largest raw sum; the
// pooled features and those rows go to z_dbg and amax, and no head runs.
template <int H1, int H2, int HH, bool PRE, bool ARGMAX = false>
__global__ __launch_bounds__(256, kFusedWgPerCu) void fused_bf16_kernel(FusedArgs A) {
  static_assert(PRE || !ARGMAX, "the argmax encoder reads the crop kernel's rows");
  using S_t = Smem<H1, H2, HH>;
  constexpr int T = S_t::T, ZS = S_t::ZS;
  constexpr int FT = H1 / 32;    // layer-1 feature tiles
  constexpr int FW = (FT + 3) / 4;  // layer-1 feature tiles per wave (tiles wave, wave + 4, ...)
  constexpr int HS = S_t::HS;
  constexpr int KS2 = H1 / 16;   // layer-2 k-steps
  constexpr int CT = H2 / 128;   // encoder column tiles per wave
  static_assert(H1 % 32 == 0 && H2 % 128 == 0 && HH % 128 == 0, "widths");
  __shared__ S_t S;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_index();
  const int g = lane >> 5;
  const int l32 = lane & 31;
  const int K = A.K;
  const int P = pair_count(A.n_pairs, A.n_pairs_dev, A.dev_base);

  // this wave's W2 slice, layer-1 weights and layer-2 bias stay in registers (the W2 slice is reloaded after
  // every head tile, so that its registers are free for the head's operands meanwhile)
  u16x8 w2f[CT][KS2];
  float bias2[CT];
  auto load_w2 = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int s = 0; s < KS2; ++s)
        w2f[ct][s] = reinterpret_cast<const u16x8*>(A.w2p)[(size_t)((wave * CT + ct) * KS2 + s) * 64 + lane];
  };
  load_w2();
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) bias2[ct] = A.b2[(wave * CT + ct) * 32 + l32];
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
    __syncthreads();  // S.claim is rewritten by the next claim
    if (base >= P) break;
    const int n_claim = P - base < A.claim ? P - base : A.claim;

    // split schedule: each thread carries the next pair's record and up to two
    // 16-byte encoder rows of it in registers, loaded while the current pair
    // computes
    // (two named registers rather than an array, which the compiler would
    // move to LDS)
    uint4 nxt0{}, nxt1{};
    PairMeta nmeta{};
    const uint4* rows_g = reinterpret_cast<const uint4*>(A.rows_bf16);
    if constexpr (PRE) {
      nmeta = A.meta[base];
      if (tid < 2 * K) nxt0 = rows_g[(size_t)base * 2 * K + tid];
      if (tid + 256 < 2 * K) nxt1 = rows_g[(size_t)base * 2 * K + tid + 256];
    }
    for (int c = 0; c < n_claim; ++c) {
      const int p = base + c;
      // ---------------------------------------------------------------- crop
      int a = -1, swapped = 0;
      int m_a = 0, m_b = 0;
      bool valid;
      if constexpr (PRE) {
        const PairMeta mt = nmeta;
        a = mt.a;
        swapped = mt.swapped;
        valid = a >= 0;
        m_a = valid ? mt.m_a : 0;
        m_b = valid ? mt.m_b : 0;
        if (tid < 2 * K) reinterpret_cast<uint4*>(S.u.c.rows)[tid] = nxt0;
        if (tid + 256 < 2 * K) reinterpret_cast<uint4*>(S.u.c.rows)[tid + 256] = nxt1;
        if (c + 1 < n_claim) {  // the next pair's record and rows load while this pair computes
          nmeta = A.meta[p + 1];
          if (tid < 2 * K) nxt0 = rows_g[(size_t)(p + 1) * 2 * K + tid];
          if (tid + 256 < 2 * K) nxt1 = rows_g[(size_t)(p + 1) * 2 * K + tid + 256];
        }
      } else {
      locc_object oa, ob;
      ShapeDesc da, db;
      valid = geo_fetch(A.objs, A.n_objs, A.pairs, p, A.lib, a, swapped, oa, ob, da, db);
      if (valid) {  // uniform over the workgroup
        PairGeom gm;
        geo_pair(oa, ob, da, db, A.pad, gm);
        PairScreen sc;
        geo_screen(gm, db, sc);
        geo_scan_select<4>(&gm, sc, da.off, da.n, db.off, db.n, A.lib, K, A.counts != nullptr, S.u.c.crop);
        const int n_a = S.u.c.crop.count[0], n_b = S.u.c.crop.count[1];
        m_a = n_a < K ? n_a : K;
        m_b = n_b < K ? n_b : K;
        if (tid == 0 && A.counts) {
          A.counts[2 * p + swapped] = n_a;
          A.counts[2 * p + 1 - swapped] = n_b;
        }
        // gather rows, zero-padded to the next multiple of 32 per object
        const int ra = (m_a + 31) & ~31, rb = (m_b + 31) & ~31;
        for (int e = tid; e < ra + rb; e += 256) {
          const int s = e >= ra;
          const int r = s ? e - ra : e;
          const int m = s ? m_b : m_a;
          u16x8 row = {0, 0, 0, 0, 0, 0, 0, 0};
          if (r < m) {
            float v[6];
            geo_row(gm, A.lib, (s ? db : da).off + S.u.c.crop.sel[s][r], s, v);
#pragma unroll
            for (int k = 0; k < 6; ++k) row[k] = bf16_bits(v[k]);
            row[6] = 0x3f80;  // 1.0
          }
          *reinterpret_cast<u16x8*>(&S.u.c.rows[(s * K + r) * 8]) = row;
        }
      } else if (tid == 0) {
        if (A.counts) {
          A.counts[2 * p] = -1;
          A.counts[2 * p + 1] = -1;
        }
        atomicAdd(A.err_counter, 1ull);
      }
      }
      if (tid == 0) {
        S.pair[slot] = p;
        S.a[slot] = valid ? a : -1;
        S.swapped[slot] = swapped;
      }
      __syncthreads();

      // ------------------------------------------------------------- encoder
      // max-pool of the raw layer-2 sums; bias and ReLU are applied once per
      // column afterwards: fl(max_r a_r + b) = max_r fl(a_r + b) because
      // rounding is monotone, and ReLU is monotone (an empty set gives
      // max(-inf + b, 0) = 0)
      // Row tiles t = 0, 1, ...: this wave's layer-1 features of tile t + 1
      // are computed while layer 2 of tile t runs, then stored to the other
      // LDS buffer; one barrier per tile publishes them (the buffer written in
      // tile t was last read in tile t - 1, before the previous barrier).
      for (int side = 0; side < 2; ++side) {
        const int m = side ? m_b : m_a;
        const int nt = (m + 31) >> 5;  // uniform over the workgroup
        const unsigned short* xrow = &S.u.c.rows[(side * K + l32) * 8 + 4 * g];
        float run[CT];
        int arg[CT];  // argmax variant: the row of run (255: none yet)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          run[ct] = -__builtin_inff();
          arg[ct] = 255;
        }
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
#pragma unroll
              for (int hf = 0; hf < 2; ++hf) {
                u32x4 w;
#pragma unroll
                for (int e = 0; e < 4; ++e) w[e] = bf16x2_relu(acc1[i][8 * hf + 2 * e], acc1[i][8 * hf + 2 * e + 1]);
                *reinterpret_cast<u32x4*>(&S.u.c.h1t[buf][l32 * HS + 16 * (2 * ft + hf) + 8 * g]) = w;
              }
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
          // all of this tile's layer-2 A fragments are requested before the
          // first product
          const unsigned short* h = &S.u.c.h1t[t & 1][l32 * HS + 8 * g];
          u16x8 av[KS2];
#pragma unroll
          for (int s = 0; s < KS2; ++s) av[s] = *reinterpret_cast<const u16x8*>(h + 16 * s);
          if (more) layer1_issue(t + 1);
          f32x16 acc2[CT];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc2[ct] = f32x16{};
          __builtin_amdgcn_s_setprio(1);  // issue priority while this wave feeds the matrix core
#pragma unroll
          for (int s = 0; s < KS2; ++s)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc2[ct] = mfma_k16(av[s], w2f[ct][s], acc2[ct]);
          __builtin_amdgcn_s_setprio(0);
          if (more) layer1_store((t + 1) & 1);
          const int r0 = 32 * t;
          if constexpr (ARGMAX) {
            // a lane's rows ascend with r, and tiles ascend with r0: strict > keeps the first maximum
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
          if constexpr (ARGMAX) {
            // the two half-waves hold rows 4g + ... of every tile: the larger value wins, the lower row on ties
            const int other_arg = __shfl_xor(arg[ct], 32, 64);
            const bool take = other > run[ct] || (other == run[ct] && other_arg < arg[ct]);
            if (lane < 32)
              A.amax[((size_t)p * 2 + side) * H2 + (wave * CT + ct) * 32 + lane] = (uint8_t)(take ? other_arg : arg[ct]);
          }
          if (lane < 32) {
            const int col = side * H2 + (wave * CT + ct) * 32 + lane;
            if constexpr (!ARGMAX) S.z[slot * ZS + col] = bf16_bits(f);
            if (A.z_dbg) A.z_dbg[(size_t)p * 2 * H2 + col] = valid ? f : __builtin_nanf("");
          }
        }
      }
      ++slot;
      // The crop scratch is reused by the next pair's crop.  The split schedule
      // needs no barrier here: every read of this pair's rows and layer-1 tiles
      // completed before the barrier ending its last row tile (a barrier waits
      // for the wave's LDS accesses), the next pair writes another z slot, and
      // the head begins with a barrier of its own.
      if constexpr (!PRE) __syncthreads();
      if constexpr (!ARGMAX) {
        if (slot == T) {
          head_tile<H1, H2, HH, PRE ? 4 : 2>(A, S, T);
          slot = 0;
          load_w2();
        }
      } else {
        slot = 0;
      }
    }
  }
  if constexpr (!ARGMAX)
    if (slot > 0) head_tile<H1, H2, HH, PRE ? 4 : 2>(A, S, slot);

  if (A.dynamic && tid == 0) {
    __threadfence();
    if (atomicAdd(A.queue + 1, 1u) == gridDim.x - 1) {  // last workgroup out resets the queue
      atomicExch(A.queue, 0u);
      atomicExch(A.queue + 1, 0u);
    }
  }
}

template <int H1, int H2, int HH>
hipError_t run_fused(const FusedArgs& a, int grid, bool pre, hipStream_t s) {
  if (pre)
    kernel_launch((fused_bf16_kernel<H1, H2, HH, true>), dim3(grid), dim3(256), 0, s, a);
  else
    kernel_launch((fused_bf16_kernel<H1, H2, HH, false>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

void bf16_bind(FusedArgs& a, const unsigned char* base, int h1, int h2, int hh) {
  const Bf16Layout L = bf16_layout(h1, h2, hh);
  a.w1p = reinterpret_cast<const unsigned short*>(base + L.w1);
  a.w2p = reinterpret_cast<const unsigned short*>(base + L.w2);
  a.b2 = reinterpret_cast<const float*>(base + L.b2);
  a.h1p = reinterpret_cast<const unsigned short*>(base + L.h1);
  a.c1 = reinterpret_cast<const float*>(base + L.c1);
  a.h2p = reinterpret_cast<const unsigned short*>(base + L.h2);
  a.c2 = reinterpret_cast<const float*>(base + L.c2);
  a.h3p = reinterpret_cast<const unsigned short*>(base + L.h3);
  a.c3 = reinterpret_cast<const float*>(base + L.c3);
}

hipError_t launch_encoder_bf16_argmax(const FusedArgs& a, int h1, int h2, int hh, int grid, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (!a.z_dbg || !a.amax || !a.rows_bf16 || !a.meta) return hipErrorInvalidValue;
  if (h1 == 64 && h2 == 128 && hh == 256)
    kernel_launch((fused_bf16_kernel<64, 128, 256, true, true>), dim3(grid), dim3(256), 0, s, a);
  else if (h1 == 128 && h2 == 256 && hh == 512)
    kernel_launch((fused_bf16_kernel<128, 256, 512, true, true>), dim3(grid), dim3(256), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fused_bf16(const FusedArgs& a, int h1, int h2, int hh, int grid, bool pre, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (h1 == 64 && h2 == 128 && hh == 256) return run_fused<64, 128, 256>(a, grid, pre, s);
  if (h1 == 128 && h2 == 256 && hh == 512) return run_fused<128, 256, 512>(a, grid, pre, s);
  return hipErrorInvalidValue;
}

}  // namespace locc
