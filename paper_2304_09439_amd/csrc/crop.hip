// Crop step of the LOCC path: relative pose, crop box, membership scan and
// ordered first-K selection, encoder-row gather.
//
// The paper selects the parts of each object that lie in the other object's
// box widened by a margin, so that nothing in contact is missed (Sec. III,
// appendix "Architecture Details").  Here, in the frame of a = min(i, j):
//   box = (AABB_a  intersect  axis-aligned hull of T_ab AABB_b) +- pad,
// every stored point of a and every transformed point of b is tested against
// the closed box, and the first K members of each object (stored order) are
// kept.  All geometry is float64 with no fused multiply-add, in one fixed
// order of operations, so the selected index sets are reproducible exactly:
//   R from quaternion (w,x,y,z): diag 1 - 2(s+t), off-diagonal 2(u -+ v)
//   R_ab[i][j] = (Ra[0][i] Rb[0][j] + Ra[1][i] Rb[1][j]) + Ra[2][i] Rb[2][j]
//   t_ab[i]    = (Ra[0][i] d0 + Ra[1][i] d1) + Ra[2][i] d2,  d = t_b - t_a
//   c'_i = ((R[i][0] c0 + R[i][1] c1) + R[i][2] c2) + t_i,
//   e'_i = (|R[i][0]| e0 + |R[i][1]| e1) + |R[i][2]| e2
//   lo_i = max(lo_a_i, c'_i - e'_i) - pad,  hi_i = min(hi_a_i, c'_i + e'_i) + pad
//   b point: q_i = ((R[i][0] p0 + R[i][1] p1) + R[i][2] p2) + t_i
//
// One workgroup of 256 threads (4 wave64) per pair.  Waves 0-1 scan object
// a, waves 2-3 object b, 64 consecutive points per wave step; each step's
// membership is a 64-bit ballot kept in LDS.  After one barrier, one wave per
// object turns the ballots into ordered positions (prefix sum of popcounts
// plus rank within the ballot) and writes the first K indices to LDS.
#pragma clang fp contract(off)

#include "locc_internal.h"

namespace locc {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = kMaxShapePoints / 64;

__device__ __forceinline__ double nan_max(double u, double v) {
  return (u != u || v != v) ? u + v : (u > v ? u : v);
}
__device__ __forceinline__ double nan_min(double u, double v) {
  return (u != u || v != v) ? u + v : (u < v ? u : v);
}

// Rotation matrix R[3*r + c] of a quaternion given as (w, x, y, z).
__device__ __forceinline__ void quat_to_rot(const float* qf, double* R) {
  const double w = qf[0], x = qf[1], y = qf[2], z = qf[3];
  const double xx = x * x, yy = y * y, zz = z * z;
  const double xy = x * y, xz = x * z, yz = y * z;
  const double wx = w * x, wy = w * y, wz = w * z;
  R[0] = 1.0 - 2.0 * (yy + zz);
  R[1] = 2.0 * (xy - wz);
  R[2] = 2.0 * (xz + wy);
  R[3] = 2.0 * (xy + wz);
  R[4] = 1.0 - 2.0 * (xx + zz);
  R[5] = 2.0 * (yz - wx);
  R[6] = 2.0 * (xz - wy);
  R[7] = 2.0 * (yz + wx);
  R[8] = 1.0 - 2.0 * (xx + yy);
}

__device__ __forceinline__ int wave_inclusive_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

__global__ __launch_bounds__(kThreads) void crop_kernel(CropArgs A) {
  __shared__ unsigned long long s_mask[2][kMaxBlocks];
  __shared__ int32_t s_sel[2][kMaxK];
  __shared__ int32_t s_count[2];

  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int K = A.K;

  const int i = A.pairs[2 * p];
  const int j = A.pairs[2 * p + 1];
  bool valid = i >= 0 && i < A.n_objs && j >= 0 && j < A.n_objs && i != j;
  const int a = i < j ? i : j;
  const int b = i < j ? j : i;
  int sa = -1, sb = -1;
  if (valid) {
    sa = A.objs[a].shape;
    sb = A.objs[b].shape;
    valid = sa >= 0 && sa < A.lib.n_shapes && sb >= 0 && sb < A.lib.n_shapes;
  }
  if (!valid) {  // uniform over the workgroup
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
  const int swapped = i > j;
  const locc_object oa = A.objs[a];
  const locc_object ob = A.objs[b];
  const ShapeDesc da = A.lib.shapes[sa];
  const ShapeDesc db = A.lib.shapes[sb];

  // ---- relative pose and crop box (float64, fixed order, no contraction)
  double Ra[9], Rb[9], R[9], t[3];
  quat_to_rot(oa.q, Ra);
  quat_to_rot(ob.q, Rb);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[3 * r + c] = (Ra[r] * Rb[c] + Ra[3 + r] * Rb[3 + c]) + Ra[6 + r] * Rb[6 + c];
  const double d0 = (double)ob.p[0] - (double)oa.p[0];
  const double d1 = (double)ob.p[1] - (double)oa.p[1];
  const double d2 = (double)ob.p[2] - (double)oa.p[2];
#pragma unroll
  for (int r = 0; r < 3; ++r) t[r] = (Ra[r] * d0 + Ra[3 + r] * d1) + Ra[6 + r] * d2;
  double lo[3], hi[3];
  {
    double cb[3], eb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cb[k] = 0.5 * ((double)db.lo[k] + (double)db.hi[k]);
      eb[k] = 0.5 * ((double)db.hi[k] - (double)db.lo[k]);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double c = ((R[3 * r] * cb[0] + R[3 * r + 1] * cb[1]) + R[3 * r + 2] * cb[2]) + t[r];
      const double e = (fabs(R[3 * r]) * eb[0] + fabs(R[3 * r + 1]) * eb[1]) + fabs(R[3 * r + 2]) * eb[2];
      lo[r] = nan_max((double)da.lo[r], c - e) - A.pad;
      hi[r] = nan_min((double)da.hi[r], c + e) + A.pad;
    }
  }

  // ---- membership scan: one ballot per 64 points
  const int side = wave >> 1;
  const ShapeDesc ds = side ? db : da;
  const int nblk = (ds.n + 63) >> 6;
  for (int blk = wave & 1; blk < nblk; blk += 2) {
    const int k = (blk << 6) + lane;
    bool in = false;
    if (k < ds.n) {
      const int g = ds.off + k;
      const double x = A.lib.px[g], y = A.lib.py[g], z = A.lib.pz[g];
      double q0 = x, q1 = y, q2 = z;
      if (side) {
        q0 = ((R[0] * x + R[1] * y) + R[2] * z) + t[0];
        q1 = ((R[3] * x + R[4] * y) + R[5] * z) + t[1];
        q2 = ((R[6] * x + R[7] * y) + R[8] * z) + t[2];
      }
      in = (lo[0] <= q0) & (q0 <= hi[0]) & (lo[1] <= q1) & (q1 <= hi[1]) & (lo[2] <= q2) & (q2 <= hi[2]);
    }
    const unsigned long long m = __ballot(in);
    if (lane == 0) s_mask[side][blk] = m;
  }
  __syncthreads();

  // ---- ordered first-K: prefix over ballots, one wave per object
  if ((wave & 1) == 0) {
    int carry = 0;
    for (int base = 0; base < nblk; base += 64) {
      const int blk = base + lane;
      unsigned long long m = blk < nblk ? s_mask[side][blk] : 0ull;
      const int c = __popcll(m);
      const int incl = wave_inclusive_scan(c, lane);
      int pos = carry + incl - c;
      while (m != 0ull && pos < K) {
        const int bit = __builtin_ctzll(m);
        s_sel[side][pos] = (blk << 6) + bit;
        m &= m - 1ull;
        ++pos;
      }
      carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) s_count[side] = carry;
  }
  __syncthreads();

  const int n_a = s_count[0], n_b = s_count[1];
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
      const int caller = s ^ swapped;
      A.idx_out[((size_t)p * 2 + caller) * K + r] = r < m ? s_sel[s][r] : -1;
    }
  }
  if (A.rows) {
    // encoder rows (x, y, z, nx, ny, nz, 1, 0) in a's frame, stored permuted
    // as (e0, e2, e4, e6, e1, e3, e5, e7); zero rows past the valid count
    for (int e = tid; e < 2 * K; e += kThreads) {
      const int s = e >= K;
      const int r = e - s * K;
      const int m = s ? m_b : m_a;
      float4 lo4 = make_float4(0.f, 0.f, 0.f, 0.f), hi4 = lo4;
      if (r < m) {
        const ShapeDesc d = s ? db : da;
        const int g = d.off + s_sel[s][r];
        float v[6];
        if (s) {
          const double x = A.lib.px[g], y = A.lib.py[g], z = A.lib.pz[g];
          const double u = A.lib.nx[g], w = A.lib.ny[g], h = A.lib.nz[g];
          v[0] = (float)(((R[0] * x + R[1] * y) + R[2] * z) + t[0]);
          v[1] = (float)(((R[3] * x + R[4] * y) + R[5] * z) + t[1]);
          v[2] = (float)(((R[6] * x + R[7] * y) + R[8] * z) + t[2]);
          v[3] = (float)((R[0] * u + R[1] * w) + R[2] * h);
          v[4] = (float)((R[3] * u + R[4] * w) + R[5] * h);
          v[5] = (float)((R[6] * u + R[7] * w) + R[8] * h);
        } else {
          v[0] = A.lib.px[g];
          v[1] = A.lib.py[g];
          v[2] = A.lib.pz[g];
          v[3] = A.lib.nx[g];
          v[4] = A.lib.ny[g];
          v[5] = A.lib.nz[g];
        }
        lo4 = make_float4(v[0], v[2], v[4], 1.0f);
        hi4 = make_float4(v[1], v[3], v[5], 0.0f);
      }
      float4* dst = reinterpret_cast<float4*>(A.rows + ((size_t)p * 2 * K + e) * kRowFloats);
      dst[0] = lo4;
      dst[1] = hi4;
    }
  }
}

}  // namespace

hipError_t launch_crop(const CropArgs& a, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(crop_kernel, dim3(a.n_pairs), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace locc
