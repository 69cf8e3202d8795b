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
constexpr int kTT = 16;  // pairs per head-training workgroup (a 4,096-pair batch fills 256 workgroups)

typedef float f32x4 __attribute__((ext_vector_type(4)));

// acc[rt][ct] = In[16 RT rows][K] . W^T for this wave's columns c0 + 16 ct + (0..15), W row-major [out][K]
// (ldw floats per row), with v_mfma_f32_16x16x4f32: A[i][k], B[k][j] with i, j = lane % 16 and the
// reduction index permuted so that at k-step 4u + v lane group g = lane / 16 holds k = 16u + 4g + v,
// which lets A (LDS rows) and B (weight rows) be read as float4.  D[i][j]: row 4g + r, column j.
template <int CT, int K, int RT = 2>
__device__ __forceinline__ void mfma_rows32(const float* In, int IS, const float* __restrict__ W, int ldw, int c0,
                                            int lane, f32x4 (&acc)[RT][CT]) {
  const int j = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int u = 0; u < K / 16; ++u) {
    float4 b[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      b[ct] = *reinterpret_cast<const float4*>(W + (size_t)(c0 + 16 * ct + j) * ldw + 16 * u + 4 * g);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
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
size_t backward_smem(int rows = kGT) {
  constexpr int LA = (Z > HH ? Z : HH) + 4, LB = HH + 4;
  return sizeof(float) * rows * (LA + LB);
}

template <int H1, int H2, int HH>
hipError_t run(const GradArgs& a, hipStream_t s) {
  const size_t smem = backward_smem<2 * H2, HH>();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&head_backward_kernel<2 * H2, HH>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  kernel_launch((head_backward_kernel<2 * H2, HH>), dim3((a.n_pairs + kGT - 1) / kGT), dim3(256), smem, s, a);
  kernel_launch((pose_kernel<H1, H2>), dim3(a.n_pairs), dim3(256), 0, s, a);
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
// features, Adam): head_train_kernel (16 pairs per workgroup, the head
// forward and backward on matrix cores, keeping per pair g1, g2, du2, du1,
// the pooled features' gradient dm, dx and the two loss terms);
// outer_sum_kernel reduces the head's weight and bias gradients over 64
// ranges of pairs on matrix cores and outer_reduce_kernel sums the ranges;
// enc_grad_kernel (one workgroup per channel and range of pairs) walks its
// (pair, object) entries in order, staging 256 argmax rows at a time in LDS,
// and train_reduce_kernel sums the partials of dW2, db2, dW1, db1 and the
// loss terms; adam_kernel updates the master weights; two gathers
// repack them into the layouts the forward and gradient kernels read.  Every
// reduction has a fixed order, so a step is reproducible bit for bit.
namespace locc {
namespace {

template <int Z, int HH>
__global__ __launch_bounds__(256) void head_train_kernel(TrainArgs A, float invB) {
  constexpr int CT = HH / 64, CTZ = Z / 64, RT = kTT / 16;
  constexpr int LA = (Z > HH ? Z : HH) + 4, LB = HH + 4;
  extern __shared__ __align__(16) float smem[];
  float* As = smem;
  float* Bs = smem + kTT * LA;
  __shared__ float dxs[kTT];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int p0 = blockIdx.x * kTT;
  const int n = A.n_pairs - p0 < kTT ? A.n_pairs - p0 : kTT;
  for (int e = t; e < kTT * Z; e += 256) {
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
  for (int q = 0; q < kTT / 4; ++q) {
    const int r = wave * (kTT / 4) + q;
    float s2 = 0.f;
    for (int k = lane; k < Z; k += 64) s2 = fmaf(As[r * LA + k], As[r * LA + k], s2);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s2 += __shfl_xor(s2, d, 64);
    if (lane == 0 && r < n) A.lossp[(size_t)(p0 + r) * 2 + 1] = A.meta[p0 + r].a >= 0 ? s2 : 0.f;
  }
  const int c0 = wave * (HH / 4);
  f32x4 acc[RT][CT];
  // g1 = ReLU(f H1^T + c1) -> B
  mfma_rows32<CT, Z, RT>(As, LA, H1, Z, c0, lane, acc);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
    const float b = c1[col];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
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
  mfma_rows32<CT, HH, RT>(Bs, LB, H2m, HH, c0, lane, acc);
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
    const float b = c2[col];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
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
  for (int q = 0; q < kTT / 4; ++q) {
    const int r = wave * (kTT / 4) + q;
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
  for (int e = t; e < kTT * HH; e += 256) {
    const int r = e / HH, col = e % HH;
    const float v = As[r * LA + col] > 0.f ? dxs[r] * h3[col] : 0.f;
    As[r * LA + col] = v;
    if (r < n) A.du2[(size_t)(p0 + r) * HH + col] = v;
  }
  __syncthreads();
  // du1 = (du2 H2) (g1 > 0) -> B
  mfma_rows32<CT, HH, RT>(As, LA, A.H2t, HH, c0, lane, acc);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = c0 + 16 * ct + j;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
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
  f32x4 accz[RT][CTZ];
  const int d0 = wave * (Z / 4);
  mfma_rows32<CTZ, HH, RT>(Bs, LB, A.H1t, HH, d0, lane, accz);
  const float reg = 2.f * A.alpha * invB;
#pragma unroll
  for (int ct = 0; ct < CTZ; ++ct) {
    const int col = d0 + 16 * ct + j;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
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
// pair's features; its X is 0).  A 64 x 64 output tile per workgroup, one 32 x 32 quarter per wave on
// v_mfma_f32_32x32x2f32 (A[i][q] = X[p + q][o0 + i], B[q][j] = Y[p + q][k0 + j]: lanes 0-31 carry pair
// p, lanes 32-63 pair p + 1); 32 pairs at a time through LDS, in ascending order within the range.
typedef float f32x16 __attribute__((ext_vector_type(16)));
__global__ __launch_bounds__(256) void outer_sum_kernel(const float* X, int ldx, int NO, const float* Y, int ldy,
                                                        int NK, int P, float* part) {
  constexpr int PS = 32;        // pairs per stage
  constexpr int PT = PS / 4;    // stage rows loaded per thread (one column each of X and Y)
  __shared__ float xs[PS][64], ys[PS][64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wo = wave >> 1, wk = wave & 1, l32 = lane & 31, half = lane >> 5;
  const int o0 = blockIdx.y * 64, k0 = blockIdx.x * 64, z = blockIdx.z;
  const int chunk = (P + kOuterSplit - 1) / kOuterSplit;
  const int pa = z * chunk, pe = pa + chunk < P ? pa + chunk : P;
  // thread t loads rows t / 64 + 4 i (i < PT) of column t % 64 of a stage; the next stage's values are
  // loaded into registers while the current one is multiplied
  const int cc = t & 63, r0 = t >> 6;
  const bool xin = o0 + cc < NO, yin = k0 + cc <= NK, yone = k0 + cc == NK;
  float xv[PT], yv[PT];
  auto load = [&](int pb) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int p = pb + r0 + 4 * i;
      xv[i] = p < pe && xin ? X[(size_t)p * ldx + o0 + cc] : 0.f;
      float y = 0.f;
      if (p < pe && yin) y = yone ? 1.f : Y[(size_t)p * ldy + k0 + cc];
      yv[i] = y == y ? y : 0.f;
    }
  };
  f32x16 acc = f32x16{};
  if (pa < pe) load(pa);
  for (int pb = pa; pb < pe; pb += PS) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      xs[r0 + 4 * i][cc] = xv[i];
      ys[r0 + 4 * i][cc] = yv[i];
    }
    __syncthreads();
    if (pb + PS < pe) load(pb + PS);
#pragma unroll
    for (int q = 0; q < PS; q += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[q + half][32 * wo + l32], ys[q + half][32 * wk + l32], acc, 0,
                                                 0, 0);
    __syncthreads();
  }
  float* dst = part + (size_t)z * NO * (NK + 1);
  const int k = k0 + 32 * wk + l32;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int o = o0 + 32 * wo + 8 * (r >> 2) + 4 * half + (r & 3);
    if (o < NO && k <= NK) dst[(size_t)o * (NK + 1) + k] = acc[r];
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

// Encoder weight-gradient partials: workgroup (c, z) stages the (pair, object) entries of range z, 256
// at a time, in LDS (channel c's dm and argmax row); thread t handles hidden unit j = t % H1 and the
// staged entries i = t / H1 (mod 256 / H1) in ascending order, for channel c's dW2 row and db2 and its
// partials of dW1, db1; the 256 / H1 streams are then added in stream order.
template <int H1, int H2>
__global__ __launch_bounds__(256) void enc_grad_kernel(TrainArgs A) {
  constexpr int NS = 256 / H1;  // entry streams per hidden unit
  static_assert(256 % H1 == 0, "hidden width");
  __shared__ float srow[256][8];
  __shared__ float sdm[256];
  __shared__ float red[NS > 1 ? NS - 1 : 1][H1][9];
  const int c = blockIdx.x, z = blockIdx.y, t = threadIdx.x, j = t % H1, st = t / H1;
  float wk[6], bk, w2ck;
#pragma unroll
  for (int q = 0; q < 6; ++q) wk[q] = A.raw[A.off.W1 + 6 * j + q];
  bk = A.raw[A.off.b1 + j];
  w2ck = A.raw[A.off.W2 + (size_t)c * H1 + j];
  float dw2 = 0.f, db2 = 0.f, dw1[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, db1 = 0.f;
  const int E = 2 * A.n_pairs;
  const int chunk = (E + kEncSplit - 1) / kEncSplit;
  const int ea = z * chunk, ee = ea + chunk < E ? ea + chunk : E;
  for (int base = ea; base < ee; base += 256) {
    const int e = base + t;
    float dm = 0.f;
    float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
    if (e < ee) {
      const int p = e >> 1, side = e & 1;
      const PairMeta mt = A.meta[p];
      if (mt.a >= 0 && (side ? mt.m_b : mt.m_a) > 0) {
        dm = A.dmv[(size_t)p * 2 * H2 + side * H2 + c];
        if (dm != 0.f) {
          const int r = A.amax[((size_t)p * 2 + side) * H2 + c];
          const float* rw = A.rows + ((size_t)p * 2 * A.K + side * A.K + r) * kRowFloats;
          lo = *reinterpret_cast<const float4*>(rw);  // stored (x, z, ny, 1 | y, nx, nz, 0)
          hi = *reinterpret_cast<const float4*>(rw + 4);
        }
      }
    }
    sdm[t] = dm;
    *reinterpret_cast<float4*>(&srow[t][0]) = make_float4(lo.x, hi.x, lo.y, hi.y);  // x, y, z, nx
    *reinterpret_cast<float4*>(&srow[t][4]) = make_float4(lo.z, hi.z, 0.f, 0.f);    // ny, nz
    __syncthreads();
    const int cnt = ee - base < 256 ? ee - base : 256;
    for (int i = st; i < cnt; i += NS) {
      const float d = sdm[i];
      const float4 r0 = *reinterpret_cast<const float4*>(&srow[i][0]);
      const float4 r1 = *reinterpret_cast<const float4*>(&srow[i][4]);
      const float pre = ((((wk[0] * r0.x + wk[1] * r0.y) + wk[2] * r0.z) + wk[3] * r0.w) + wk[4] * r1.x) +
                        wk[5] * r1.y + bk;
      // an entry with d = 0 adds exact zeros
      const float on = pre > 0.f ? d : 0.f;
      db2 += d;
      dw2 = fmaf(on, pre, dw2);
      const float dh = w2ck * on;
      dw1[0] = fmaf(dh, r0.x, dw1[0]);
      dw1[1] = fmaf(dh, r0.y, dw1[1]);
      dw1[2] = fmaf(dh, r0.z, dw1[2]);
      dw1[3] = fmaf(dh, r0.w, dw1[3]);
      dw1[4] = fmaf(dh, r1.x, dw1[4]);
      dw1[5] = fmaf(dh, r1.y, dw1[5]);
      db1 += dh;
    }
    __syncthreads();
  }
  // streams 1.. hand their sums to stream 0, which adds them in stream order
  if (NS > 1 && st > 0) {
    float* rr = red[st - 1][j];
#pragma unroll
    for (int q = 0; q < 6; ++q) rr[q] = dw1[q];
    rr[6] = db1;
    rr[7] = dw2;
    rr[8] = db2;
  }
  __syncthreads();
  if (st == 0) {
    for (int k = 0; k + 1 < NS; ++k) {
      const float* rr = red[k][j];
#pragma unroll
      for (int q = 0; q < 6; ++q) dw1[q] += rr[q];
      db1 += rr[6];
      dw2 += rr[7];
      db2 += rr[8];
    }
    float* w2p = A.w2part + ((size_t)z * H2 + c) * (H1 + 1);
    w2p[j] = dw2;
    float* part = A.w1part + (((size_t)z * H2 + c) * H1 + j) * 7;
#pragma unroll
    for (int q = 0; q < 6; ++q) part[q] = dw1[q];
    part[6] = db1;
    if (j == 0) w2p[H1] = db2;  // every hidden unit's thread holds the same db2
  }
}

// dW2, db2: one thread per output, ranges summed in order.
template <int H1, int H2>
__device__ __forceinline__ void enc_reduce_w2(const TrainArgs& A, int block) {
  const int id = block * 256 + threadIdx.x;
  if (id >= H2 * (H1 + 1)) return;
  float s = 0.f;
  for (int z = 0; z < kEncSplit; ++z) s += A.w2part[(size_t)z * H2 * (H1 + 1) + id];
  const int c = id / (H1 + 1), k = id % (H1 + 1);
  if (k < H1)
    A.grad[A.off.W2 + (size_t)c * H1 + k] = s;
  else
    A.grad[A.off.b2 + c] = s;
}

// dW1, db1: one wave per output (hidden unit k, column q) over the kEncSplit x H2 partials: lane l adds
// partials l, l + 64, ... in order, then the lanes are combined by a fixed butterfly.
template <int H1, int H2>
__device__ __forceinline__ void enc_reduce_w1(const TrainArgs& A, int block) {
  constexpr int NP = kEncSplit * H2;
  const int jd = block * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (jd >= H1 * 7) return;  // uniform per wave
  const int k = jd / 7, q = jd % 7;
  float s = 0.f;
  for (int i = lane; i < NP; i += 64) s += A.w1part[((size_t)i * H1 + k) * 7 + q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) {
    if (q < 6)
      A.grad[A.off.W1 + 6 * k + q] = s;
    else
      A.grad[A.off.b1 + k] = s;
  }
}

// Mean loss terms, summed in a fixed order by one workgroup.
__device__ __forceinline__ void loss_sum(const TrainArgs& A, float invB) {
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

// The reductions after enc_grad_kernel in one launch: blocks [0, B2) reduce dW2 / db2, the next B1 blocks
// dW1 / db1, the last one the loss terms.
template <int H1, int H2>
__global__ __launch_bounds__(256) void train_reduce_kernel(TrainArgs A, float invB) {
  constexpr int B2 = (H2 * (H1 + 1) + 255) / 256, B1 = (H1 * 7 + 3) / 4;
  const int b = blockIdx.x;  // uniform
  if (b < B2)
    enc_reduce_w2<H1, H2>(A, b);
  else if (b < B2 + B1)
    enc_reduce_w1<H1, H2>(A, b - B2);
  else
    loss_sum(A, invB);
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
  // the gradient entries no kernel writes (the untrained outputs' rows of H3 and c3) stay zero from the
  // upload of the weights
  const size_t smem = backward_smem<Z, HH>(kTT);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&head_train_kernel<Z, HH>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const int P = a.n_pairs;
  kernel_launch((head_train_kernel<Z, HH>), dim3((P + kTT - 1) / kTT), dim3(256), smem, s, a, invB);
  const GradOffsets& o = a.off;
  // dH3[0], dc3[0]; dH2, dc2; dH1, dc1: partial outer sums over pair ranges, then ordered reductions
  auto outer = [&](const float* X, int ldx, int NO, const float* Y, int ldy, int NK, float* D, float* Db) {
    kernel_launch(outer_sum_kernel, dim3((NK + 1 + 63) / 64, (NO + 63) / 64, kOuterSplit), dim3(256), 0, s, X,
                       ldx, NO, Y, ldy, NK, P, a.opart);
    kernel_launch(outer_reduce_kernel, dim3((NO * (NK + 1) + 255) / 256), dim3(256), 0, s,
                       (const float*)a.opart, NO, NK, D, NK, Db);
  };
  outer(a.dx, 1, 1, a.g2, HH, HH, a.grad + o.H3, a.grad + o.c3);
  outer(a.du2, HH, HH, a.g1, HH, HH, a.grad + o.H2, a.grad + o.c2);
  outer(a.du1, HH, HH, a.z, Z, Z, a.grad + o.H1, a.grad + o.c1);
  kernel_launch((enc_grad_kernel<H1, H2>), dim3(H2, kEncSplit), dim3(256), 0, s, a);
  kernel_launch((train_reduce_kernel<H1, H2>), dim3((H2 * (H1 + 1) + 255) / 256 + (H1 * 7 + 3) / 4 + 1),
                     dim3(256), 0, s, a, invB);
  kernel_launch(adam_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  kernel_launch(gather_kernel, dim3((unsigned)((a.pack_n + 255) / 256)), dim3(256), 0, s, a.pack_dst,
                     a.pack_idx, a.pack_n, (const float*)a.raw);
  kernel_launch(gather_kernel, dim3((unsigned)((a.tr_n + 255) / 256)), dim3(256), 0, s, a.tr_dst, a.tr_idx,
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
