// Crop step: a set-up kernel with one thread per pair validates the pair,
// puts it in canonical order and computes its float64 relative pose, crop box
// and float32 screening constants (geometry.h), so that this work is done
// once per pair instead of once per wave; then one wave per object of every
// pair runs the membership scan and the ordered first-K selection, and
// writes counts, the optional index sets, the per-pair records and the
// encoder input rows (float32 for the FP32 path, bf16 for BF16 / FP8).
#include "geometry.h"

namespace locc {
namespace {

// one thread per pair, 64 per workgroup: a batch of 16384 pairs spreads over
// 256 workgroups, one per compute unit, for this latency-bound float64 work
constexpr int kThreads = 64;
constexpr int kCropWaves = 2;  // object waves per workgroup of the crop kernel (1, 2, 4, 8 measured: 2 fastest)

__global__ __launch_bounds__(kThreads) void pair_setup_kernel(CropArgs A) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= pair_count(A.n_pairs, A.n_pairs_dev, A.dev_base)) return;
  PairSetup r{};
  locc_object oa, ob;
  ShapeDesc da, db;
  int a = -1, swapped = 0;
  r.valid = geo_fetch(A.objs, A.n_objs, A.pairs, p, A.lib, a, swapped, oa, ob, da, db);
  if (r.valid) {
    geo_pair(oa, ob, da, db, A.pad, r.g);
    geo_screen_values(r.g, db, r.sc);
    r.a = a;
    r.swapped = swapped;
    r.off_a = da.off;
    r.n_a = da.n;
    r.off_b = db.off;
    r.n_b = db.n;
  }
  *reinterpret_cast<PairSetup*>(static_cast<char*>(A.setup) + (size_t)p * kPairSetupBytes) = r;
}

// One wave per object of a pair: wave item = 2p + side scans, selects and
// gathers object `side` of pair p on its own (no barrier; the two objects of
// a pair never wait for each other), so many more pairs are in flight per
// compute unit than with a workgroup per pair.  W independent waves share a
// workgroup (each with its own LDS), so that the compute unit's limit on
// resident workgroups does not cap the resident waves.
struct ObjectShared {
  int32_t sel[kMaxK];
};

// LDS written by some lanes of a wave and then read by others of the same
// wave: the wave's LDS operations are performed in order, so it suffices that
// the compiler keeps them in order and waits for the writes (workgroup-scope
// fences); no other wave takes part.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Raw buffer view of n floats at p: a load at a byte offset >= 4n returns 0
// and reads no memory (the buffer unit's range check), so lanes past a
// shape's last point need no branch of their own.  Word 3 is the gfx9
// raw-buffer format word (32-bit data, no swizzle, no index stride).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t crop_view(const float* p, int n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, n * 4, 0x00020000);
}
__device__ __forceinline__ float crop_load(__amdgpu_buffer_rsrc_t v, int byte_offset) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(v, byte_offset, 0, 0));
}
__device__ __forceinline__ float4 crop_load4(__amdgpu_buffer_rsrc_t v, int byte_offset) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(v, byte_offset, 0, 0));
}
// A wave-uniform float copied once into a vector register, so that an fma
// taking it with a scalar coefficient needs no copy per use (one scalar
// operand per vector instruction).
__device__ __forceinline__ float crop_to_vgpr(float s) {
  float v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

// Membership scan of one object (B: the transformed object b) by one wave,
// over blocks of 256 stored points: lane l holds points 4l .. 4l + 3 of a
// block, fetched by one 16-byte load per coordinate (a quarter of the
// address-unit work of one load per point), QU blocks' loads in flight
// together.  The wave tests the blocks in stored order and keeps the number of
// members before each block (a scalar), so a member's ordered position is that
// number, plus the members of the lanes below it (one ballot per point slot),
// plus its own members before it: the first K members are placed during the
// scan.  Without `full` the scan stops at the first block after which K
// members are known.  Returns the members found (all of them when full, else
// at least min(K, members)).
template <int QU, bool B>
__device__ __forceinline__ int crop_scan(const PairSetup* __restrict__ rec, const PairScreen& sc, const float* px,
                                         const float* py, const float* pz, int n, int K, bool full, int lane,
                                         ObjectShared& S) {
  const int nblk = (n + 255) >> 8;
  int scanned = 0, found = 0;  // wave-uniform
  while (scanned < nblk && (full || found < K)) {
    const int base = scanned << 8;
    const int rem = n - base;  // > 0 points from base on
    const __amdgpu_buffer_rsrc_t vx = crop_view(px + base, rem), vy = crop_view(py + base, rem),
                                 vz = crop_view(pz + base, rem);
    float4 X[QU], Y[QU], Z[QU];
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      const int o = (256 * u + 4 * lane) * 4;
      X[u] = crop_load4(vx, o);
      Y[u] = crop_load4(vy, o);
      Z[u] = crop_load4(vz, o);
    }
#pragma unroll
    for (int u = 0; u < QU; ++u) {
      if (scanned + u < nblk && (full || found < K)) {  // uniform
        const int j0 = 256 * u + 4 * lane;  // this lane's first point: base + j0
        const int left = rem - j0;          // of its four points, those below n
        float x[4] = {X[u].x, X[u].y, X[u].z, X[u].w};
        float y[4] = {Y[u].x, Y[u].y, Y[u].z, Y[u].w};
        float z[4] = {Z[u].x, Z[u].y, Z[u].z, Z[u].w};
        if (left > 0 && left < 4) {  // the shape's last, partial four: point by point
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            x[k] = crop_load(vx, (j0 + k) * 4);
            y[k] = crop_load(vy, (j0 + k) * 4);
            z[k] = crop_load(vz, (j0 + k) * 4);
          }
        }
        bool in[4];
        unsigned long long m[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          in[k] = (B ? geo_member_b(&rec->g, sc, x[k], y[k], z[k]) : geo_member_a(sc, x[k], y[k], z[k])) & (k < left);
          m[k] = __ballot(in[k]);
        }
        unsigned pos = (unsigned)found;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          pos = __builtin_amdgcn_mbcnt_hi((unsigned)(m[k] >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m[k], pos));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (in[k] && (int)pos < K) S.sel[pos] = base + j0 + k;
          pos += in[k] ? 1u : 0u;
        }
        found += __popcll(m[0]) + __popcll(m[1]) + __popcll(m[2]) + __popcll(m[3]);
      }
    }
    scanned = scanned + QU < nblk ? scanned + QU : nblk;
  }
  return found;
}

template <int U, int W>
__global__ __launch_bounds__(64 * W) void crop_kernel(CropArgs A) {
  __shared__ ObjectShared SW[W];
  const int wave = W == 1 ? 0 : wave_index();
  ObjectShared& S = SW[wave];
  const int item = blockIdx.x * W + wave;
  const int p = item >> 1;
  const int side = item & 1;
  const int lane = threadIdx.x & 63;
  const int K = A.K;
  if (p >= pair_count(A.n_pairs, A.n_pairs_dev, A.dev_base)) return;  // uniform

  // the pair's record: the same address for the whole wave (scalar loads)
  const PairSetup* __restrict__ rec =
      reinterpret_cast<const PairSetup*>(static_cast<const char*>(A.setup) + (size_t)p * kPairSetupBytes);
  if (!rec->valid) {  // uniform; object 0's wave reports the pair
    if (side == 0) {
      if (A.idx_out)
        for (int e = lane; e < 2 * K; e += 64) A.idx_out[(size_t)p * 2 * K + e] = -1;
      if (lane == 0) {
        if (A.counts_out) {
          A.counts_out[2 * p] = -1;
          A.counts_out[2 * p + 1] = -1;
        }
        if (A.meta) A.meta[p] = PairMeta{-1, 0, 0, 0};
        atomicAdd(A.err_counter, 1ull);
      }
    }
    return;
  }
  const int swapped = rec->swapped;
  const int n = side ? rec->n_b : rec->n_a;
  const int off = side ? rec->off_b : rec->off_a;
  PairScreen sc = rec->sc;
  const bool full = A.counts_out != nullptr;  // else stop once K members are known
  const float* __restrict__ px = A.lib.px + off;
  const float* __restrict__ py = A.lib.py + off;
  const float* __restrict__ pz = A.lib.pz + off;
  int found;
  if (side) {
#pragma unroll
    for (int i = 0; i < 3; ++i) sc.t[i] = crop_to_vgpr(sc.t[i]);
    found = crop_scan<(U >= 8 ? 2 : 1), true>(rec, sc, px, py, pz, n, K, full, lane, S);
  } else {
    found = crop_scan<(U >= 8 ? 2 : 1), false>(rec, sc, px, py, pz, n, K, full, lane, S);
  }
  // found: every member when full, else at least min(K, members)
  wave_lds_sync();  // the selected indices are read by other lanes
  const int m = found < K ? found : K;
  const int caller = side ^ swapped;  // position of this object in the caller's pair
  if (lane == 0) {
    if (A.counts_out) A.counts_out[2 * p + caller] = found;
    if (A.meta) {
      if (side == 0) {
        A.meta[p].a = rec->a;
        A.meta[p].swapped = swapped;
        A.meta[p].m_a = m;
      } else {
        A.meta[p].m_b = m;
      }
    }
  }
  if (A.idx_out)
    for (int r = lane; r < K; r += 64) A.idx_out[((size_t)p * 2 + caller) * K + r] = r < m ? S.sel[r] : -1;
  if (A.rows) {
    // rows (x, y, z, nx, ny, nz, 1, 0) stored permuted as (e0, e2, e4, e6, e1, e3, e5, e7);
    // zero rows past the valid count
    const PairGeom g = rec->g;
    for (int r = lane; r < K; r += 64) {
      float4 lo4 = make_float4(0.f, 0.f, 0.f, 0.f), hi4 = lo4;
      if (r < m) {
        float v[6];
        geo_row(g, A.lib, off + S.sel[r], side, v);
        lo4 = make_float4(v[0], v[2], v[4], 1.0f);
        hi4 = make_float4(v[1], v[3], v[5], 0.0f);
      }
      float4* dst = reinterpret_cast<float4*>(A.rows + ((size_t)p * 2 * K + side * K + r) * kRowFloats);
      dst[0] = lo4;
      dst[1] = hi4;
    }
  }
  if (A.rows_bf16) {
    // bf16 rows (x, y, z, nx, ny, nz, 1, 0), zero-padded to a multiple of 32
    const PairGeom g = rec->g;
    const int rm = (m + 31) & ~31;
    for (int r = lane; r < rm; r += 64) {
      unsigned short row[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (r < m) {
        float v[6];
        geo_row(g, A.lib, off + S.sel[r], side, v);
#pragma unroll
        for (int k = 0; k < 6; ++k) row[k] = __builtin_bit_cast(unsigned short, (__bf16)v[k]);
        row[6] = 0x3f80;  // 1.0
      }
      uint4 packed;
      packed.x = row[0] | ((unsigned)row[1] << 16);
      packed.y = row[2] | ((unsigned)row[3] << 16);
      packed.z = row[4] | ((unsigned)row[5] << 16);
      packed.w = row[6] | ((unsigned)row[7] << 16);
      *reinterpret_cast<uint4*>(A.rows_bf16 + ((size_t)p * 2 * K + side * K + r) * 8) = packed;
    }
  }
}

}  // namespace

hipError_t launch_crop(const CropArgs& a, hipStream_t s, int unroll) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (!a.setup || (unroll != 2 && unroll != 4 && unroll != 8)) return hipErrorInvalidValue;
  kernel_launch(pair_setup_kernel, dim3((a.n_pairs + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
  constexpr int W = kCropWaves;
  const dim3 grid((2 * a.n_pairs + W - 1) / W), block(64 * W);
  switch (unroll) {
    case 2: kernel_launch((crop_kernel<2, W>), grid, block, 0, s, a); break;
    case 4: kernel_launch((crop_kernel<4, W>), grid, block, 0, s, a); break;
    case 8: kernel_launch((crop_kernel<8, W>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace locc
