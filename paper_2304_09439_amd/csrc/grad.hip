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

// ------------------------------------------------------------------ training
//
// One step of fitting the FP32 network to collision labels (binary
// cross-entropy of the logit plus alpha times the squared norm of the pooled
// features, Adam): head_train_kernel (32 pairs per workgroup, the head
// forward and backward on matrix cores, keeping per pair g1, g2, du2, du1,
// the pooled features' gradient dm, dx and the two loss terms);
// outer_sum_kernel reduces the head's weight and bias gradients over 16
// ranges of pairs and outer_reduce_kernel sums the ranges; enc_grad_kernel
// (one workgroup per channel and range of pairs) walks its (pair, object)
// entries in order, staging 128 argmax rows at a time in LDS, and
// enc_reduce_kernel sums the partials of dW2, db2, dW1, db1; adam_kernel updates the master weights; two gathers
// repack them into the layouts the forward and gradient kernels read.  Every
// reduction has a fixed order, so a step is reproducible bit for bit.
namespace locc {
namespace {

template <int Z, int HH>
__global__ __launch_bounds__(256) void head_train_kernel(TrainArgs A, float invB) {
  constexpr int H2 = Z / 2;
  constexpr int CT = HH / 64, CTZ = Z / 64;
  constexpr int LA = (Z > HH ? Z : HH) + 4, LB = HH + 4;
  extern __shared__ __align__(16) float smem[];
  float* As = smem;
  float* Bs = smem + kGT * LA;
  __shared__ float dxs[kGT];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int p0 = blockIdx.x * kGT;
  const int n = A.n_pairs - p0 < kGT ? A.n_pairs - p0 : kGT;
  for (int e = t; e < kGT * Z; e += 256) {
    const int r = e / Z, k = e % Z;
    const float v = r < n ? A.z[(size_t)(p0 + r) * Z + k] : 0.f;
    As[r * LA + k] = v == v ? v : 0.f;  // invalid pair: NaN features, no loss
  }
  __syncthreads();
  const float* raw = A.raw;
  const float* H1 = raw + A.off.H1;
  const float* c1 = raw + A.off.c1;
  const float* H2m = raw + A.off.H2;
  const float* c2 = raw + A.off.c2;
  const float* h3 = raw + A.off.H3;
  // squared feature norm per pair (a wave per 8 pairs)
  for (int q = 0; q < kGT / 4; ++q) {
    const int r = wave * (kGT / 4) + q;
    float s2 = 0.f;
    for (int k = lane; k < Z; k += 64) s2 = fmaf(As[r * LA + k], As[r * LA + k], s2);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s2 += __shfl_xor(s2, d, 64);
    if (lane == 0 && r < n) A.lossp[(size_t)(p0 + r) * 2 + 1] = A.meta[p0 + r].a >= 0 ? s2 : 0.f;
  }
  const int c0 = wave * (HH / 4);
  f32x4 acc[2][CT];
  // g1 = ReLU(f H1^T + c1) -> B
  mfma_rows32<CT, Z>(As, LA, H1, Z, c0, lane, acc);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
    const float b = c1[col];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * g + r;
        const float u = acc[rt][ct][r] + b;
        const float v = u > 0.f ? u : 0.f;
        Bs[row * LB + col] = v;
        if (row < n) A.g1[(size_t)(p0 + row) * HH + col] = v;
      }
  }
  __syncthreads();
  // g2 = ReLU(g1 H2^T + c2) -> A (f is no longer needed in LDS)
  mfma_rows32<CT, HH>(Bs, LB, H2m, HH, c0, lane, acc);
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
    const float b = c2[col];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * g + r;
        const float u = acc[rt][ct][r] + b;
        const float v = u > 0.f ? u : 0.f;
        As[row * LA + col] = v;
        if (row < n) A.g2[(size_t)(p0 + row) * HH + col] = v;
      }
  }
  __syncthreads();
  // logit, dx = (sigmoid(x) - y) / B and the cross-entropy (a wave per 8 pairs)
  for (int q = 0; q < kGT / 4; ++q) {
    const int r = wave * (kGT / 4) + q;
    float x = 0.f;
    for (int k = lane; k < HH; k += 64) x = fmaf(As[r * LA + k], h3[k], x);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if (lane == 0) {
      float dxv = 0.f;
      if (r < n) {
        float bce = 0.f;
        if (A.meta[p0 + r].a >= 0) {
          x += raw[A.off.c3];
          const float y = A.labels[p0 + r];
          dxv = (1.f / (1.f + expf(-x)) - y) * invB;
          bce = fmaxf(x, 0.f) - x * y + log1pf(expf(-fabsf(x)));
        }
        A.dx[p0 + r] = dxv;
        A.lossp[(size_t)(p0 + r) * 2] = bce;
      }
      dxs[r] = dxv;
    }
  }
  __syncthreads();
  // du2 = dx H3[0] (g2 > 0) -> A
  for (int e = t; e < kGT * HH; e += 256) {
    const int r = e / HH, col = e % HH;
    const float v = As[r * LA + col] > 0.f ? dxs[r] * h3[col] : 0.f;
    As[r * LA + col] = v;
    if (r < n) A.du2[(size_t)(p0 + r) * HH + col] = v;
  }
  __syncthreads();
  // du1 = (du2 H2) (g1 > 0) -> B
  mfma_rows32<CT, HH>(As, LA, A.H2t, HH, c0, lane, acc);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * g + r;
        float* e = Bs + row * LB + col;
        const float v = *e > 0.f ? acc[rt][ct][r] : 0.f;
        *e = v;
        if (row < n) A.du1[(size_t)(p0 + row) * HH + col] = v;
      }
  }
  __syncthreads();
  // dz = du1 H1 + (2 alpha / B) f; dm = dz (f > 0), both objects
  f32x4 accz[2][CTZ];
  const int d0 = wave * (Z / 4);
  mfma_rows32<CTZ, HH>(Bs, LB, A.H1t, HH, d0, lane, accz);
  const float reg = 2.f * A.alpha * invB;
#pragma unroll
  for (int ct = 0; ct < CTZ; ++ct) {
    const int col = d0 + 16 * ct + j;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * g + r;
        if (row < n) {
          const float f = A.z[(size_t)(p0 + row) * Z + col];
          A.dmv[(size_t)(p0 + row) * Z + col] = f > 0.f ? fmaf(reg, f, accz[rt][ct][r]) : 0.f;
        }
      }
  }
}

// Partial outer sums: part[z][o][k] = sum_{p in range z} X[p][o] Y[p][k] for k < NK, and column NK the
// plain sum of X[p][o] (a column of ones in Y; the bias gradient).  NaN in Y is read as 0 (an invalid
// pair's features; its X is 0).  64 x 64 outputs per workgroup, 4 x 4 per thread, 16 pairs at a time
// through LDS, pairs in ascending order within the range.
__global__ __launch_bounds__(256) void outer_sum_kernel(const float* X, int ldx, int NO, const float* Y, int ldy,
                                                        int NK, int P, float* part) {
  __shared__ float xs[16][64], ys[16][64];
  const int t = threadIdx.x, to = t >> 4, tk = t & 15;
  const int o0 = blockIdx.y * 64, k0 = blockIdx.x * 64, z = blockIdx.z;
  const int chunk = (P + kOuterSplit - 1) / kOuterSplit;
  const int pa = z * chunk, pe = pa + chunk < P ? pa + chunk : P;
  float acc[4][4] = {};
  for (int pb = pa; pb < pe; pb += 16) {
    for (int e = t; e < 16 * 64; e += 256) {
      const int pp = e >> 6, c = e & 63, p = pb + pp;
      float xv = 0.f, yv = 0.f;
      if (p < pe && o0 + c < NO) xv = X[(size_t)p * ldx + o0 + c];
      if (p < pe && k0 + c <= NK) {
        yv = k0 + c < NK ? Y[(size_t)p * ldy + k0 + c] : 1.f;
        yv = yv == yv ? yv : 0.f;
      }
      xs[pp][c] = xv;
      ys[pp][c] = yv;
    }
    __syncthreads();
#pragma unroll 4
    for (int pp = 0; pp < 16; ++pp) {
      float xv[4], yv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        xv[a] = xs[pp][4 * to + a];
        yv[a] = ys[pp][4 * tk + a];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(xv[a], yv[b], acc[a][b]);
    }
    __syncthreads();
  }
  float* dst = part + (size_t)z * NO * (NK + 1);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int o = o0 + 4 * to + a, k = k0 + 4 * tk + b;
      if (o < NO && k <= NK) dst[(size_t)o * (NK + 1) + k] = acc[a][b];
    }
}

// D[o][k] = sum_z part[z][o][k] (ranges in order); column NK goes to Dbias[o].
__global__ __launch_bounds__(256) void outer_reduce_kernel(const float* part, int NO, int NK, float* D, int ldd,
                                                           float* Dbias) {
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= NO * (NK + 1)) return;
  const int o = id / (NK + 1), k = id % (NK + 1);
  float s = 0.f;
  for (int z = 0; z < kOuterSplit; ++z) s += part[(size_t)z * NO * (NK + 1) + id];
  if (k < NK)
    D[(size_t)o * ldd + k] = s;
  else
    Dbias[o] = s;
}

// Encoder weight-gradient partials: workgroup (c, z) walks the (pair, object) entries of range z in
// order, staging 128 argmax rows at a time in LDS, for channel c's dW2 row and db2 and its partials of
// dW1, db1.
template <int H1, int H2>
__global__ __launch_bounds__(128) void enc_grad_kernel(TrainArgs A) {
  __shared__ float srow[128][6];
  __shared__ float sdm[128];
  const int c = blockIdx.x, z = blockIdx.y, t = threadIdx.x;
  float wk[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, bk = 0.f, w2ck = 0.f;
  if (t < H1) {
#pragma unroll
    for (int q = 0; q < 6; ++q) wk[q] = A.raw[A.off.W1 + 6 * t + q];
    bk = A.raw[A.off.b1 + t];
    w2ck = A.raw[A.off.W2 + (size_t)c * H1 + t];
  }
  float dw2 = 0.f, db2 = 0.f, dw1[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, db1 = 0.f;
  const int E = 2 * A.n_pairs;
  const int chunk = (E + kEncSplit - 1) / kEncSplit;
  const int ea = z * chunk, ee = ea + chunk < E ? ea + chunk : E;
  for (int base = ea; base < ee; base += 128) {
    const int e = base + t;
    float dm = 0.f, row[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (e < ee) {
      const int p = e >> 1, side = e & 1;
      const PairMeta mt = A.meta[p];
      if (mt.a >= 0 && (side ? mt.m_b : mt.m_a) > 0) {
        dm = A.dmv[(size_t)p * 2 * H2 + side * H2 + c];
        if (dm != 0.f) {
          const int r = A.amax[((size_t)p * 2 + side) * H2 + c];
          const float* rw = A.rows + ((size_t)p * 2 * A.K + side * A.K + r) * kRowFloats;
          const float4 lo = *reinterpret_cast<const float4*>(rw), hi = *reinterpret_cast<const float4*>(rw + 4);
          row[0] = lo.x;  // stored (x, z, ny, 1 | y, nx, nz, 0)
          row[1] = hi.x;
          row[2] = lo.y;
          row[3] = hi.y;
          row[4] = lo.z;
          row[5] = hi.z;
        }
      }
    }
    sdm[t] = dm;
#pragma unroll
    for (int q = 0; q < 6; ++q) srow[t][q] = row[q];
    __syncthreads();
    const int cnt = ee - base < 128 ? ee - base : 128;
    for (int i = 0; i < cnt; ++i) {
      const float d = sdm[i];
      if (d == 0.f) continue;  // uniform
      db2 += d;
      const float* rr = srow[i];
      const float pre = ((((wk[0] * rr[0] + wk[1] * rr[1]) + wk[2] * rr[2]) + wk[3] * rr[3]) + wk[4] * rr[4]) +
                        wk[5] * rr[5] + bk;
      if (pre > 0.f) {
        dw2 = fmaf(d, pre, dw2);
        const float dh = w2ck * d;
#pragma unroll
        for (int q = 0; q < 6; ++q) dw1[q] = fmaf(dh, rr[q], dw1[q]);
        db1 += dh;
      }
    }
    __syncthreads();
  }
  float* w2p = A.w2part + ((size_t)z * H2 + c) * (H1 + 1);
  if (t < H1) {
    w2p[t] = dw2;
    float* part = A.w1part + (((size_t)z * H2 + c) * H1 + t) * 7;
#pragma unroll
    for (int q = 0; q < 6; ++q) part[q] = dw1[q];
    part[6] = db1;
  }
  if (t == 0) w2p[H1] = db2;
}

// dW2, db2: ranges summed in order; dW1, db1: ranges and channels summed in order.
template <int H1, int H2>
__global__ __launch_bounds__(256) void enc_reduce_kernel(TrainArgs A) {
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id < H2 * (H1 + 1)) {
    float s = 0.f;
    for (int z = 0; z < kEncSplit; ++z) s += A.w2part[(size_t)z * H2 * (H1 + 1) + id];
    const int c = id / (H1 + 1), k = id % (H1 + 1);
    if (k < H1)
      A.grad[A.off.W2 + (size_t)c * H1 + k] = s;
    else
      A.grad[A.off.b2 + c] = s;
    return;
  }
  const int jd = id - H2 * (H1 + 1);
  if (jd >= H1 * 7) return;
  const int k = jd / 7, q = jd % 7;
  float s = 0.f;
  for (int z = 0; z < kEncSplit; ++z)
    for (int c = 0; c < H2; ++c) s += A.w1part[(((size_t)z * H2 + c) * H1 + k) * 7 + q];
  if (q < 6)
    A.grad[A.off.W1 + 6 * k + q] = s;
  else
    A.grad[A.off.b1 + k] = s;
}

// Mean loss terms, summed in a fixed order by one workgroup.
__global__ __launch_bounds__(256) void loss_kernel(TrainArgs A, float invB) {
  __shared__ float part[2][256];
  const int t = threadIdx.x;
  float s0 = 0.f, s1 = 0.f;
  for (int p = t; p < A.n_pairs; p += 256) {
    s0 += A.lossp[(size_t)p * 2];
    s1 += A.lossp[(size_t)p * 2 + 1];
  }
  part[0][t] = s0;
  part[1][t] = s1;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      part[0][t] += part[0][t + w];
      part[1][t] += part[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    A.loss[0] = part[0][0] * invB;
    A.loss[1] = A.alpha * part[1][0] * invB;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(TrainArgs A) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= A.n) return;
  const float gr = A.grad[i];
  const float m = A.beta1 * A.m[i] + (1.f - A.beta1) * gr;
  const float v = A.beta2 * A.v[i] + (1.f - A.beta2) * gr * gr;
  A.m[i] = m;
  A.v[i] = v;
  A.raw[i] -= A.lr * (m * A.corr1) / (sqrtf(v * A.corr2) + A.eps);
}

__global__ __launch_bounds__(256) void gather_kernel(float* dst, const int32_t* idx, size_t n, const float* src) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t k = idx[i];
  dst[i] = k >= 0 ? src[k] : 0.f;
}

template <int H1, int H2, int HH>
hipError_t run_train(const TrainArgs& a, hipStream_t s) {
  constexpr int Z = 2 * H2;
  const float invB = 1.f / (float)a.n_pairs;
  hipError_t e = hipMemsetAsync(a.grad, 0, a.n * sizeof(float), s);
  if (e != hipSuccess) return e;
  const size_t smem = backward_smem<Z, HH>();
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&head_train_kernel<Z, HH>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const int P = a.n_pairs;
  hipLaunchKernelGGL((head_train_kernel<Z, HH>), dim3((P + kGT - 1) / kGT), dim3(256), smem, s, a, invB);
  const GradOffsets& o = a.off;
  // dH3[0], dc3[0]; dH2, dc2; dH1, dc1: partial outer sums over pair ranges, then ordered reductions
  auto outer = [&](const float* X, int ldx, int NO, const float* Y, int ldy, int NK, float* D, float* Db) {
    hipLaunchKernelGGL(outer_sum_kernel, dim3((NK + 1 + 63) / 64, (NO + 63) / 64, kOuterSplit), dim3(256), 0, s, X,
                       ldx, NO, Y, ldy, NK, P, a.opart);
    hipLaunchKernelGGL(outer_reduce_kernel, dim3((NO * (NK + 1) + 255) / 256), dim3(256), 0, s,
                       (const float*)a.opart, NO, NK, D, NK, Db);
  };
  outer(a.dx, 1, 1, a.g2, HH, HH, a.grad + o.H3, a.grad + o.c3);
  outer(a.du2, HH, HH, a.g1, HH, HH, a.grad + o.H2, a.grad + o.c2);
  outer(a.du1, HH, HH, a.z, Z, Z, a.grad + o.H1, a.grad + o.c1);
  hipLaunchKernelGGL((enc_grad_kernel<H1, H2>), dim3(H2, kEncSplit), dim3(128), 0, s, a);
  hipLaunchKernelGGL((enc_reduce_kernel<H1, H2>), dim3((H2 * (H1 + 1) + H1 * 7 + 255) / 256), dim3(256), 0, s, a);
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, a, invB);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((a.pack_n + 255) / 256)), dim3(256), 0, s, a.pack_dst,
                     a.pack_idx, a.pack_n, (const float*)a.raw);
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((a.tr_n + 255) / 256)), dim3(256), 0, s, a.tr_dst, a.tr_idx,
                     a.tr_n, (const float*)a.raw);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_train_step(const TrainArgs& a, int h1, int h2, int hh, hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (h1 == 64 && h2 == 128 && hh == 256) return run_train<64, 128, 256>(a, s);
  if (h1 == 128 && h2 == 256 && hh == 512) return run_train<128, 256, 512>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace locc
