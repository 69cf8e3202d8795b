// Broad phase over many environments: the pairs that reach the narrow phase.
//
// The paper leaves pairs that are far apart to a broad phase that runs before
// any narrow-phase test (Sec. II, footnote on the broad phase), and its
// simulations step many environments at once, an object pairing only with
// objects of its own environment.  Here, per simulation step:
//
//   world_box_kernel   one thread per object: the axis-aligned hull of its
//                      shape's box after rotation and translation, float64
//                      with contraction off, in the order
//                        c_w[i] = ((R[i][0] c0 + R[i][1] c1) + R[i][2] c2) + p_i
//                        e_w[i] = (|R[i][0]| e0 + |R[i][1]| e1) + |R[i][2]| e2
//                        lo = c_w - e_w, hi = c_w + e_w
//                      (c, e: centre and half extent of the shape box); an
//                      object whose shape id is out of range gets a NaN box,
//                      which overlaps nothing.
//   env_count_kernel   one wave per environment: every pair i < j of its
//                      objects, taken 64 at a time in (i, j) order along the
//                      flattened upper triangle; closed-interval overlap on
//                      all three axes; the wave's ballots are counted.
//   env_scan_kernel    one workgroup: exclusive prefix of the counts (first
//                      output position per environment), and the pair count.
//   env_write_kernel   the count kernel's loop again; each overlapping pair
//                      goes to its environment's start + the overlapping
//                      pairs before it (ballot rank), if below the capacity.
//
// The output is listed by environment, then i, then j, ascending, which is
// unique, so it is reproducible bit for bit.  The all-pairs test inside an
// environment costs n (n - 1) / 2 tests for n objects: it suits the many
// small environments of vectorised simulation (tens of objects each).
#include "geometry.h"

namespace locc {
namespace {

constexpr int kBoxThreads = 256;
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kBoxThreads) void world_box_kernel(BroadArgs A) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * kBoxThreads + threadIdx.x;
  if (k >= A.n_objs) return;
  const locc_object o = A.objs[k];
  double box[6];
  if (o.shape < 0 || o.shape >= A.lib.n_shapes) {
#pragma unroll
    for (int a = 0; a < 6; ++a) box[a] = __builtin_nan("");
  } else {
    const ShapeDesc d = A.lib.shapes[o.shape];
    double R[9];
    geo_quat_to_rot(o.q, R);
    double c[3], e[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = 0.5 * ((double)d.lo[a] + (double)d.hi[a]);
      e[a] = 0.5 * ((double)d.hi[a] - (double)d.lo[a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double cw = ((R[3 * a] * c[0] + R[3 * a + 1] * c[1]) + R[3 * a + 2] * c[2]) + (double)o.p[a];
      const double ew = (__builtin_fabs(R[3 * a]) * e[0] + __builtin_fabs(R[3 * a + 1]) * e[1]) +
                        __builtin_fabs(R[3 * a + 2]) * e[2];
      box[a] = cw - ew;
      box[3 + a] = cw + ew;
    }
  }
  double2* dst = reinterpret_cast<double2*>(A.boxes + (size_t)k * 6);
  dst[0] = make_double2(box[0], box[1]);
  dst[1] = make_double2(box[2], box[3]);
  dst[2] = make_double2(box[4], box[5]);
}

// Objects [a, a + n) of environment e: both bounds clamped to [0, n_objs],
// an empty or reversed range holds none.
__device__ __forceinline__ void env_range(const BroadArgs& A, int e, int& a, int& n) {
  int lo = A.env_offsets[e], hi = A.env_offsets[e + 1];
  lo = lo < 0 ? 0 : (lo > A.n_objs ? A.n_objs : lo);
  hi = hi < 0 ? 0 : (hi > A.n_objs ? A.n_objs : hi);
  a = lo;
  n = hi > lo ? hi - lo : 0;
}

// Moves (i, j) forward along the flattened upper triangle of an n-object
// environment until j is a valid partner of i (row i holds j = i+1 .. n-1);
// stops at the last row, which holds no pair, for positions past the end.
__device__ __forceinline__ void tri_normalise(int& i, int& j, int n) {
  while (j >= n && i < n - 1) {
    ++i;
    j += i + 1 - n;
  }
}

__device__ __forceinline__ bool boxes_overlap(const double* __restrict__ boxes, int i, int j) {
  const double2* bi = reinterpret_cast<const double2*>(boxes + (size_t)i * 6);
  const double2* bj = reinterpret_cast<const double2*>(boxes + (size_t)j * 6);
  const double2 i0 = bi[0], i1 = bi[1], i2 = bi[2];  // (lo x, lo y) (lo z, hi x) (hi y, hi z)
  const double2 j0 = bj[0], j1 = bj[1], j2 = bj[2];
  return (i0.x <= j1.y) & (j0.x <= i1.y) & (i0.y <= j2.x) & (j0.y <= i2.x) & (i1.x <= j2.y) & (j1.x <= i2.y);
}

// One wave per environment.  WRITE = false counts the overlapping pairs,
// WRITE = true places them.
template <bool WRITE>
__global__ __launch_bounds__(64) void env_pairs_kernel(BroadArgs A) {
  const int e = blockIdx.x;
  const int lane = threadIdx.x;
  int a, n;
  env_range(A, e, a, n);
  const long long total = (long long)n * (n - 1) / 2;
  long long pos = 0;  // write: next output position of this environment
  if (WRITE) {
    pos = A.env_start[e];
    if (pos >= A.capacity) return;  // uniform: nothing of this environment fits
  }
  int i = 0, j = 1 + lane;
  tri_normalise(i, j, n);
  long long found = 0;
  for (long long t0 = 0; t0 < total; t0 += 64) {  // uniform
    const bool hit = t0 + lane < total && boxes_overlap(A.boxes, a + i, a + j);
    const unsigned long long m = __ballot(hit);
    if (WRITE) {
      const long long p = pos + (long long)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      if (hit && p < A.capacity) *reinterpret_cast<int2*>(A.pairs + 2 * p) = make_int2(a + i, a + j);
      pos += __popcll(m);
      if (pos >= A.capacity) return;  // uniform
    } else {
      found += __popcll(m);
    }
    j += 64;
    tri_normalise(i, j, n);
  }
  if (!WRITE && lane == 0) A.env_count[e] = found;
}

// One workgroup: exclusive prefix of the per-environment counts, 1024
// environments per round; thread 0 writes the pair counts.
__global__ __launch_bounds__(kScanThreads) void env_scan_kernel(BroadArgs A) {
  __shared__ long long wave_sum[kScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  long long carry = 0;
  for (int base = 0; base < A.n_envs; base += kScanThreads) {  // uniform
    const int e = base + t;
    const long long v = e < A.n_envs ? A.env_count[e] : 0;
    long long incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const long long o = __shfl_up(incl, d, 64);
      if (lane >= d) incl += o;
    }
    if (lane == 63) wave_sum[w] = incl;
    __syncthreads();
    long long before = 0, round = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
      const long long s = wave_sum[k];
      before += k < w ? s : 0;
      round += s;
    }
    if (e < A.n_envs) A.env_start[e] = carry + before + incl - v;
    carry += round;
    __syncthreads();  // wave_sum is rewritten next round
  }
  if (t == 0) {
    A.count[0] = (int32_t)(carry < (long long)A.capacity ? carry : (long long)A.capacity);
    A.count[1] = (int32_t)(carry < 2147483647LL ? carry : 2147483647LL);
  }
}

}  // namespace

size_t broad_phase_scratch_bytes(int n_objs, int n_envs) {
  const auto a256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  return a256((size_t)n_objs * 6 * sizeof(double)) + 2 * a256((size_t)n_envs * sizeof(long long));
}

void broad_phase_carve(void* base, int n_objs, int n_envs, BroadArgs& a) {
  const auto a256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* p = static_cast<char*>(base);
  a.boxes = reinterpret_cast<double*>(p);
  p += a256((size_t)n_objs * 6 * sizeof(double));
  a.env_count = reinterpret_cast<long long*>(p);
  p += a256((size_t)n_envs * sizeof(long long));
  a.env_start = reinterpret_cast<long long*>(p);
}

hipError_t launch_broad_phase(const BroadArgs& a, hipStream_t s) {
  if (a.n_objs < 0 || a.n_envs < 0 || a.capacity < 0 || !a.count) return hipErrorInvalidValue;
  if (a.n_objs > 0) {
    if (!a.objs || !a.boxes) return hipErrorInvalidValue;
    kernel_launch(world_box_kernel, dim3((a.n_objs + kBoxThreads - 1) / kBoxThreads), dim3(kBoxThreads), 0, s,
                       a);
  }
  if (a.n_envs > 0) {
    if (!a.env_offsets || !a.env_count || !a.env_start || (a.capacity > 0 && !a.pairs)) return hipErrorInvalidValue;
    kernel_launch(env_pairs_kernel<false>, dim3(a.n_envs), dim3(64), 0, s, a);
  }
  kernel_launch(env_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a);  // also writes count when empty
  if (a.n_envs > 0 && a.capacity > 0) kernel_launch(env_pairs_kernel<true>, dim3(a.n_envs), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace locc
