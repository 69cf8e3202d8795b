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
//     for the second object's channels dm = (H1^T du1)[h2 + c] (f > 0); the
//     pairs' activations stay in LDS, each thread owns output columns and
//     reads the weights [in][out] (coalesced) with the rows as LDS broadcasts.
//   pose_kernel  one workgroup per pair, one thread per channel c of the
//     second object: at its argmax row r the layer-1 pre-activation is
//     recomputed, dr = W1^T ((W2[c] dm[c]) (W1 r + b1 > 0)) gives the point
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

// acc[j][r] = sum_k In[r][k] Wt[k * N + col0 + 256 j + t] over K inputs (K a multiple of 4).
template <int J, int K, int IS>
__device__ __forceinline__ void rows_times(const float* In, const float* __restrict__ Wt, int N, int col0, int t,
                                           float (&acc)[J][kGT]) {
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int r = 0; r < kGT; ++r) acc[j][r] = 0.f;
  for (int k = 0; k < K; k += 4) {
    float w[J][4];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) w[j][q] = Wt[(size_t)(k + q) * N + col0 + 256 * j + t];
#pragma unroll
    for (int r = 0; r < kGT; ++r) {
      const float4 v = *reinterpret_cast<const float4*>(In + r * IS + k);
#pragma unroll
      for (int j = 0; j < J; ++j) {
        acc[j][r] = fmaf(v.x, w[j][0], acc[j][r]);
        acc[j][r] = fmaf(v.y, w[j][1], acc[j][r]);
        acc[j][r] = fmaf(v.z, w[j][2], acc[j][r]);
        acc[j][r] = fmaf(v.w, w[j][3], acc[j][r]);
      }
    }
  }
}

template <int Z, int HH>
__global__ __launch_bounds__(256) void head_backward_kernel(GradArgs A) {
  constexpr int H2 = Z / 2;
  constexpr int J = HH / 256;  // output columns per thread for the HH-wide layers
  constexpr int LA = (Z > HH ? Z : HH) + 4;
  constexpr int LB = HH + 4;
  extern __shared__ __align__(16) float smem[];
  float* As = smem;             // [32][LA]: f, later du2
  float* Bs = smem + kGT * LA;  // [32][LB]: ReLU(u1), later du1
  const int t = threadIdx.x;
  const int p0 = blockIdx.x * kGT;
  const int n = A.n_pairs - p0 < kGT ? A.n_pairs - p0 : kGT;
  for (int e = t; e < kGT * Z; e += 256) {
    const int r = e / Z, k = e % Z;
    float v = r < n ? A.z[(size_t)(p0 + r) * Z + k] : 0.f;
    As[r * LA + k] = v == v ? v : 0.f;  // invalid pair: NaN features, result discarded
  }
  __syncthreads();
  const float* raw = A.raw;
  const float* H1 = raw + A.off.H1;
  const float* c1 = raw + A.off.c1;
  const float* H2m = raw + A.off.H2;
  const float* c2 = raw + A.off.c2;
  const float* h3 = raw + A.off.H3;  // row 0: the logit
  float acc[J][kGT];
  // u1 = f H1^T + c1 -> ReLU into B
  rows_times<J, Z, LA>(As, A.H1t, HH, 0, t, acc);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int o = 256 * j + t;
    const float b = c1[o];
#pragma unroll
    for (int r = 0; r < kGT; ++r) {
      const float u = acc[j][r] + b;
      Bs[r * LB + o] = u > 0.f ? u : 0.f;
    }
  }
  __syncthreads();
  // u2 = ReLU(u1) H2^T + c2 -> du2 = H3[0] (u2 > 0) into A
  rows_times<J, HH, LB>(Bs, A.H2t, HH, 0, t, acc);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int o = 256 * j + t;
    const float b = c2[o], w3 = h3[o];
#pragma unroll
    for (int r = 0; r < kGT; ++r) As[r * LA + o] = acc[j][r] + b > 0.f ? w3 : 0.f;
  }
  __syncthreads();
  // du1 = (du2 H2) (u1 > 0) into B (each thread reads and writes only its own columns)
  rows_times<J, HH, LA>(As, H2m, HH, 0, t, acc);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int o = 256 * j + t;
#pragma unroll
    for (int r = 0; r < kGT; ++r) Bs[r * LB + o] = Bs[r * LB + o] > 0.f ? acc[j][r] : 0.f;
  }
  __syncthreads();
  // dm[c] = (du1 H1)[h2 + c] (f[h2 + c] > 0), second object's channels
  if (t < H2) {
    float a1[1][kGT];
    rows_times<1, HH, LB>(Bs, H1, Z, H2, t, a1);
    for (int r = 0; r < n; ++r) {
      const float f = A.z[(size_t)(p0 + r) * Z + H2 + t];
      A.dm[(size_t)(p0 + r) * H2 + t] = f > 0.f ? a1[0][r] : 0.f;
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
  const int p = blockIdx.x, t = threadIdx.x;
  const PairMeta mt = A.meta[p];
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
      const float* W1 = A.raw + A.off.W1;
      const float* b1 = A.raw + A.off.b1;
      const float* w2 = A.raw + A.off.W2 + (size_t)t * H1;
      float dr[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (int k = 0; k < H1; ++k) {
        const float* wk = W1 + 6 * k;
        const float pre = ((((wk[0] * x[0] + wk[1] * x[1]) + wk[2] * x[2]) + wk[3] * x[3]) + wk[4] * x[4]) +
                          wk[5] * x[5] + b1[k];
        if (pre > 0.f) {
          const float d = w2[k] * dm;
#pragma unroll
          for (int q = 0; q < 6; ++q) dr[q] = fmaf(wk[q], d, dr[q]);
        }
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
