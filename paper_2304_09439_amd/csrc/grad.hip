// Pose gradients of the collision logit for the FP32 crop-point path.
//
// The paper takes contact force and torque directions from the gradient of
// the collision network's output with respect to the poses (Sec. II,
// collision resolution with an object collision network).  After the crop
// (with its index sets) and the FP32 encoder (recording per object and
// channel the row of the largest raw layer-2 sum, the first on ties):
//
//   head_backward_kernel  32 pairs per workgroup: u1 = H1 f + c1, u2 = H2
//     ReLU(u1) + c2, then du2 = H3[0] (u2 > 0), du1 = (H2^T du2) (u1 > 0), and
//     for the second object's channels dm = (H1^T du1)[h2 + c] (f > 0): four
//     products on 16x16x4 FP32 matrix cores, the pairs' activations in LDS,
//     each wave owning a quarter of the output columns, the weight rows
//     (row-major [out][in]: H1, H2, H2^T, H1^T) read from L2 as float4.
//   pose_kernel  one workgroup per pair, one thread per channel c of the
//     second object: at its argmax row r the layer-1 pre-activation is
//     recomputed (W1 in LDS), dr = W1^T ((W2[c] dm[c]) (W1 r + b1 > 0)) (W2
//     read transposed, coalesced over c) gives the point
//     and normal derivatives, and with the stored point p and normal n of
//     that row dR_ab += dx p^T + dn n^T, dt_ab += dx; a block reduction, then
//     one thread applies the chain rule through R_ab = R_a^T R_b, t_ab =
//     R_a^T (p_b - p_a) and the quaternion polynomial in float64 and writes
//     the 14 derivatives in the caller's order.
#include "geometry.h"
#include "grad.h"

namespace locc {
namespace {

constexpr int kGT = 32;  // pairs per head-backward workgroup

typedef float f32x4 __attribute__((ext_vector_type(4)));

// acc[rt][ct] = In[32 rows][K] . W^T for this wave's columns c0 + 16 ct + (0..15), W row-major [out][K]
// (ldw floats per row), with v_mfma_f32_16x16x4f32: A[i][k], B[k][j] with i, j = lane % 16 and the
// reduction index permuted so that at k-step 4u + v lane group g = lane / 16 holds k = 16u + 4g + v,
// which lets A (LDS rows) and B (weight rows) be read as float4.  D[i][j]: row 4g + r, column j.
template <int CT, int K>
__device__ __forceinline__ void mfma_rows32(const float* In, int IS, const float* __restrict__ W, int ldw, int c0,
                                            int lane, f32x4 (&acc)[2][CT]) {
  const int j = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int u = 0; u < K / 16; ++u) {
    float4 b[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      b[ct] = *reinterpret_cast<const float4*>(W + (size_t)(c0 + 16 * ct + j) * ldw + 16 * u + 4 * g);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const float4 a = *reinterpret_cast<const float4*>(In + (16 * rt + j) * IS + 16 * u + 4 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[ct].x, acc[rt][ct], 0, 0, 0);
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[ct].y, acc[rt][ct], 0, 0, 0);
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b[ct].z, acc[rt][ct], 0, 0, 0);
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b[ct].w, acc[rt][ct], 0, 0, 0);
      }
    }
  }
}

template <int Z, int HH>
__global__ __launch_bounds__(256) void head_backward_kernel(GradArgs A) {
  constexpr int H2 = Z / 2;
  constexpr int CT = HH / 64;   // 16-column tiles per wave for the HH-wide products (4 waves)
  constexpr int CT2 = H2 / 64;  // ... for the H2-wide one
  constexpr int LA = (Z > HH ? Z : HH) + 4;  // +4: rows 16 B apart in the LDS banks
  constexpr int LB = HH + 4;
  extern __shared__ __align__(16) float smem[];
  float* As = smem;             // [32][LA]: f, later du2
  float* Bs = smem + kGT * LA;  // [32][LB]: ReLU(u1), later du1
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int p0 = blockIdx.x * kGT;
  const int n = A.n_pairs - p0 < kGT ? A.n_pairs - p0 : kGT;
  for (int e = t; e < kGT * Z; e += 256) {
    const int r = e / Z, k = e % Z;
    float v = r < n ? A.z[(size_t)(p0 + r) * Z + k] : 0.f;
    As[r * LA + k] = v == v ? v : 0.f;  // invalid pair: NaN features, result discarded
  }
  __syncthreads();
  const float* raw = A.raw;
  const float* H1 = raw + A.off.H1;  // [hh][2 h2]
  const float* c1 = raw + A.off.c1;
  const float* H2m = raw + A.off.H2;  // [hh][hh]
  const float* c2 = raw + A.off.c2;
  const float* h3 = raw + A.off.H3;  // row 0: the logit
  const int c0 = wave * (HH / 4);
  f32x4 acc[2][CT];
  // u1 = f H1^T + c1 -> ReLU(u1) into B
  mfma_rows32<CT, Z>(As, LA, H1, Z, c0, lane, acc);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
    const float b = c1[col];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float u = acc[rt][ct][r] + b;
        Bs[(16 * rt + 4 * g + r) * LB + col] = u > 0.f ? u : 0.f;
      }
  }
  __syncthreads();
  // u2 = ReLU(u1) H2^T + c2 -> du2 = H3[0] (u2 > 0) into A
  mfma_rows32<CT, HH>(Bs, LB, H2m, HH, c0, lane, acc);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
    const float b = c2[col], w3 = h3[col];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) As[(16 * rt + 4 * g + r) * LA + col] = acc[rt][ct][r] + b > 0.f ? w3 : 0.f;
  }
  __syncthreads();
  // du1 = (du2 H2) (u1 > 0) into B: the weight rows are H2's columns (H2^T row-major); each lane reads
  // and rewrites only its own entries of B
  mfma_rows32<CT, HH>(As, LA, A.H2t, HH, c0, lane, acc);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float* e = Bs + (16 * rt + 4 * g + r) * LB + col;
        *e = *e > 0.f ? acc[rt][ct][r] : 0.f;
      }
  }
  __syncthreads();
  // dm[c] = (du1 H1)[h2 + c] (f[h2 + c] > 0): the weight rows are H1's columns h2 + c (H1^T rows)
  f32x4 acc2[2][CT2];
  const int d0 = wave * (H2 / 4);
  mfma_rows32<CT2, HH>(Bs, LB, A.H1t + (size_t)H2 * HH, HH, d0, lane, acc2);
#pragma unroll
  for (int ct = 0; ct < CT2; ++ct) {
    const int col = d0 + 16 * ct + j;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * g + r;
        if (row < n) {
          const float f = A.z[(size_t)(p0 + row) * Z + H2 + col];
          A.dm[(size_t)(p0 + row) * H2 + col] = f > 0.f ? acc2[rt][ct][r] : 0.f;
        }
      }
  }
}

// Block-wide sum of 12 values (256 threads); the result is valid in thread 0.
__device__ __forceinline__ void block_sum12(float (&v)[12], float (*red)[12]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int q = 0; q < 12; ++q)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v[q] += __shfl_xor(v[q], d, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 12; ++q) red[wave][q] = v[q];
  __syncthreads();
  if (t == 0)
#pragma unroll
    for (int q = 0; q < 12; ++q) v[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

// d/dq of sum_ij G[i][j] R(q)[i][j] for the polynomial rotation of q = (w, x, y, z) as given.
__device__ __forceinline__ void rotation_grad(const float* qf, const double* G, double* dq) {
  const double w = qf[0], x = qf[1], y = qf[2], z = qf[3];
  dq[0] = 2.0 * (-G[1] * z + G[2] * y + G[3] * z - G[5] * x - G[6] * y + G[7] * x);
  dq[1] = 2.0 * (G[1] * y + G[2] * z + G[3] * y - 2.0 * G[4] * x - G[5] * w + G[6] * z + G[7] * w - 2.0 * G[8] * x);
  dq[2] = 2.0 * (-2.0 * G[0] * y + G[1] * x + G[2] * w + G[3] * x + G[5] * z - G[6] * w + G[7] * z - 2.0 * G[8] * y);
  dq[3] = 2.0 * (-2.0 * G[0] * z - G[1] * w + G[2] * x + G[3] * w - 2.0 * G[4] * z + G[5] * y + G[6] * x + G[7] * y);
}

template <int H1, int H2>
__global__ __launch_bounds__(256) void pose_kernel(GradArgs A) {
  __shared__ float red[4][12];
  __shared__ float w1s[H1][8];  // W1 row and bias per hidden unit
  const int p = blockIdx.x, t = threadIdx.x;
  const PairMeta mt = A.meta[p];
  for (int e = t; e < H1 * 7; e += 256) {
    const int k = e / 7, q = e % 7;
    w1s[k][q] = q < 6 ? A.raw[A.off.W1 + 6 * k + q] : A.raw[A.off.b1 + k];
  }
  __syncthreads();
  float v[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) v[q] = 0.f;
  const int b = mt.a < 0 ? -1 : (mt.swapped ? A.pairs[2 * p] : A.pairs[2 * p + 1]);
  if (A.argmax_b && t < H2)  // 255 where the second object has no rows (or the pair is invalid)
    A.argmax_b[(size_t)p * H2 + t] = mt.a >= 0 && mt.m_b > 0 ? A.amax[((size_t)p * 2 + 1) * H2 + t] : (uint8_t)255;
  if (mt.a >= 0 && mt.m_b > 0 && t < H2) {
    const float dm = A.dm[(size_t)p * H2 + t];
    if (dm != 0.f) {
      const int r = A.amax[((size_t)p * 2 + 1) * H2 + t];
      // row r of the second object, stored (x, z, ny, 1 | y, nx, nz, 0)
      const float* row = A.rows + ((size_t)p * 2 * A.K + A.K + r) * kRowFloats;
      const float4 lo = *reinterpret_cast<const float4*>(row), hi = *reinterpret_cast<const float4*>(row + 4);
      const float x[6] = {lo.x, hi.x, lo.y, hi.y, lo.z, hi.z};
      float dr[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int k = 0; k < H1; ++k) {
        const float* wk = w1s[k];
        const float pre = ((((wk[0] * x[0] + wk[1] * x[1]) + wk[2] * x[2]) + wk[3] * x[3]) + wk[4] * x[4]) +
                          wk[5] * x[5] + wk[6];
        const float d = pre > 0.f ? A.W2t[(size_t)k * H2 + t] * dm : 0.f;  // W2[c][k], coalesced over c
#pragma unroll
        for (int q = 0; q < 6; ++q) dr[q] = fmaf(wk[q], d, dr[q]);
      }
      // the stored point and normal of that row (b's own frame)
      const int cpos = 1 ^ mt.swapped;
      const int s = A.idx[((size_t)p * 2 + cpos) * A.K + r];
      const int pt = A.lib.shapes[A.objs[b].shape].off + s;
      const float ps[3] = {A.lib.px[pt], A.lib.py[pt], A.lib.pz[pt]};
      const float ns[3] = {A.lib.nx[pt], A.lib.ny[pt], A.lib.nz[pt]};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) v[3 * i + j] = dr[i] * ps[j] + dr[3 + i] * ns[j];
        v[9 + i] = dr[i];
      }
    }
  }
  block_sum12(v, red);
  if (t != 0) return;
  float* out = A.grad + (size_t)p * 14;
  if (mt.a < 0) {
    for (int q = 0; q < 14; ++q) out[q] = __builtin_nanf("");
    return;
  }
  const locc_object oa = A.objs[mt.a], ob = A.objs[b];
  double Ra[9], Rb[9], GR[9], gt[3];
  geo_quat_to_rot(oa.q, Ra);
  geo_quat_to_rot(ob.q, Rb);
  for (int q = 0; q < 9; ++q) GR[q] = v[q];
  for (int q = 0; q < 3; ++q) gt[q] = v[9 + q];
  const double d[3] = {(double)ob.p[0] - oa.p[0], (double)ob.p[1] - oa.p[1], (double)ob.p[2] - oa.p[2]};
  double dRa[9], dRb[9], dpb[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) {
      double sa = d[i] * gt[j], sb = 0.0;
      for (int k = 0; k < 3; ++k) {
        sa += Rb[3 * i + k] * GR[3 * j + k];  // R_b dR_ab^T
        sb += Ra[3 * i + k] * GR[3 * k + j];  // R_a dR_ab
      }
      dRa[3 * i + j] = sa;
      dRb[3 * i + j] = sb;
    }
    dpb[i] = Ra[3 * i] * gt[0] + Ra[3 * i + 1] * gt[1] + Ra[3 * i + 2] * gt[2];
  }
  double dqa[4], dqb[4];
  rotation_grad(oa.q, dRa, dqa);
  rotation_grad(ob.q, dRb, dqb);
  float* first = out + (mt.swapped ? 7 : 0);
  float* second = out + (mt.swapped ? 0 : 7);
  for (int i = 0; i < 3; ++i) {
    first[i] = (float)-dpb[i];
    second[i] = (float)dpb[i];
  }
  for (int i = 0; i < 4; ++i) {
    first[3 + i] = (float)dqa[i];
    second[3 + i] = (float)dqb[i];
  }
}

template <int Z, int HH>
size_t backward_smem() {
  constexpr int LA = (Z > HH ? Z : HH) + 4, LB = HH + 4;
  return sizeof(float) * kGT * (LA + LB);
}

template <int H1, int H2, int HH>
hipError_t run(const GradArgs& a, hipStream_t s) {
  const size_t smem = backward_smem<2 * H2, HH>();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&head_backward_kernel<2 * H2, HH>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((head_backward_kernel<2 * H2, HH>), dim3((a.n_pairs + kGT - 1) / kGT), dim3(256), smem, s, a);
  hipLaunchKernelGGL((pose_kernel<H1, H2>), dim3(a.n_pairs), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pose_gradients(const GradArgs& a, int h1, int h2, int hh, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (h1 == 64 && h2 == 128 && hh == 256) return run<64, 128, 256>(a, s);
  if (h1 == 128 && h2 == 256 && hh == 512) return run<128, 256, 512>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace locc
