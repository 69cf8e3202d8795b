// Crop step: a set-up kernel with one thread per pair validates the pair,
// puts it in canonical order and computes its float64 relative pose, crop box
// and float32 screening constants (geometry.h), so that this work is done
// once per pair instead of once per wave; then one workgroup (4 wave64) per
// pair runs the membership scan and the ordered first-K selection, and
// writes counts, the optional index sets, the per-pair records and the
// encoder input rows (float32 for the FP32 path, bf16 for BF16 / FP8).
#include "geometry.h"

namespace locc {
namespace {

constexpr int kThreads = 256;

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

template <int U>
__global__ __launch_bounds__(kThreads) void crop_kernel(CropArgs A) {
  __shared__ CropShared S;
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int K = A.K;
  if (p >= pair_count(A.n_pairs, A.n_pairs_dev, A.dev_base)) return;  // uniform

  // the pair's record: the same address for the whole workgroup
  const PairSetup* __restrict__ rec =
      reinterpret_cast<const PairSetup*>(static_cast<const char*>(A.setup) + (size_t)p * kPairSetupBytes);
  const int a = rec->a, swapped = rec->swapped;
  if (!rec->valid) {  // uniform
    if (A.idx_out)
      for (int e = tid; e < 2 * K; e += kThreads) A.idx_out[(size_t)p * 2 * K + e] = -1;
    if (tid == 0) {
      if (A.counts_out) {
        A.counts_out[2 * p] = -1;
        A.counts_out[2 * p + 1] = -1;
      }
      if (A.meta) A.meta[p] = PairMeta{-1, 0, 0, 0};
      atomicAdd(A.err_counter, 1ull);
    }
    return;
  }
  const PairScreen sc = rec->sc;
  const int off_a = rec->off_a, off_b = rec->off_b;
  geo_scan_select<U>(&rec->g, sc, off_a, rec->n_a, off_b, rec->n_b, A.lib, K, A.counts_out != nullptr, S);
  const PairGeom g = rec->g;

  const int n_a = S.count[0], n_b = S.count[1];
  const int m_a = n_a < K ? n_a : K;
  const int m_b = n_b < K ? n_b : K;
  if (tid == 0) {
    if (A.counts_out) {
      A.counts_out[2 * p + swapped] = n_a;
      A.counts_out[2 * p + 1 - swapped] = n_b;
    }
    if (A.meta) A.meta[p] = PairMeta{a, swapped, m_a, m_b};
  }
  if (A.idx_out) {
    for (int e = tid; e < 2 * K; e += kThreads) {
      const int s = e >= K;
      const int r = e - s * K;
      const int m = s ? m_b : m_a;
      A.idx_out[((size_t)p * 2 + (s ^ swapped)) * K + r] = r < m ? S.sel[s][r] : -1;
    }
  }
  if (A.rows) {
    // rows (x, y, z, nx, ny, nz, 1, 0) stored permuted as (e0, e2, e4, e6, e1, e3, e5, e7);
    // zero rows past the valid count
    for (int e = tid; e < 2 * K; e += kThreads) {
      const int s = e >= K;
      const int r = e - s * K;
      const int m = s ? m_b : m_a;
      float4 lo4 = make_float4(0.f, 0.f, 0.f, 0.f), hi4 = lo4;
      if (r < m) {
        float v[6];
        geo_row(g, A.lib, (s ? off_b : off_a) + S.sel[s][r], s, v);
        lo4 = make_float4(v[0], v[2], v[4], 1.0f);
        hi4 = make_float4(v[1], v[3], v[5], 0.0f);
      }
      float4* dst = reinterpret_cast<float4*>(A.rows + ((size_t)p * 2 * K + e) * kRowFloats);
      dst[0] = lo4;
      dst[1] = hi4;
    }
  }
  if (A.rows_bf16) {
    // bf16 rows (x, y, z, nx, ny, nz, 1, 0), zero-padded to a multiple of 32
    // per object; waves 0-1 write object a's rows, waves 2-3 object b's (the
    // float64 transform of b's rows then never diverges inside a wave)
    const int s = wave_index() >> 1;
    const int rm = s ? (m_b + 31) & ~31 : (m_a + 31) & ~31;
    const int m = s ? m_b : m_a;
    for (int r = tid & 127; r < rm; r += 128) {
      unsigned short row[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (r < m) {
        float v[6];
        geo_row(g, A.lib, (s ? off_b : off_a) + S.sel[s][r], s, v);
#pragma unroll
        for (int k = 0; k < 6; ++k) row[k] = __builtin_bit_cast(unsigned short, (__bf16)v[k]);
        row[6] = 0x3f80;  // 1.0
      }
      uint4 packed;
      packed.x = row[0] | ((unsigned)row[1] << 16);
      packed.y = row[2] | ((unsigned)row[3] << 16);
      packed.z = row[4] | ((unsigned)row[5] << 16);
      packed.w = row[6] | ((unsigned)row[7] << 16);
      *reinterpret_cast<uint4*>(A.rows_bf16 + ((size_t)p * 2 * K + s * K + r) * 8) = packed;
    }
  }
}

}  // namespace

hipError_t launch_crop(const CropArgs& a, hipStream_t s, int unroll) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (!a.setup || (unroll != 2 && unroll != 4 && unroll != 8)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pair_setup_kernel, dim3((a.n_pairs + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
  switch (unroll) {
    case 2: hipLaunchKernelGGL(crop_kernel<2>, dim3(a.n_pairs), dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL(crop_kernel<4>, dim3(a.n_pairs), dim3(kThreads), 0, s, a); break;
    case 8: hipLaunchKernelGGL(crop_kernel<8>, dim3(a.n_pairs), dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace locc
