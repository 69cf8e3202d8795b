// Device-side crop geometry shared by the crop kernel and the fused kernel.
//
// The paper keeps, for each object of a pair, the parts that lie in the
// other object's box widened by a margin so that nothing in contact is
// missed (Sec. III, appendix "Architecture Details").  In the frame of
// a = min(i, j) the box used here is
//   (AABB_a  intersect  axis-aligned hull of T_ab AABB_b) widened by pad,
// and the first K stored points of each object inside it are kept.
//
// Everything is float64 with contraction disabled, evaluated in exactly this
// order (so the selected index sets are reproducible bit for bit):
//   R from quaternion (w,x,y,z): diag 1 - 2(s + t), off-diagonal 2(u -+ v)
//   R_ab[i][j] = (Ra[0][i] Rb[0][j] + Ra[1][i] Rb[1][j]) + Ra[2][i] Rb[2][j]
//   t_ab[i]    = (Ra[0][i] d0 + Ra[1][i] d1) + Ra[2][i] d2,  d = t_b - t_a
//   c'_i = ((R[i][0] c0 + R[i][1] c1) + R[i][2] c2) + t_i,
//   e'_i = (|R[i][0]| e0 + |R[i][1]| e1) + |R[i][2]| e2
//   lo_i = max(lo_a_i, c'_i - e'_i) - pad,  hi_i = min(hi_a_i, c'_i + e'_i) + pad
//   b point: q_i = ((R[i][0] p0 + R[i][1] p1) + R[i][2] p2) + t_i
// max / min propagate NaN; membership is the closed box; NaN is never inside.
#pragma once

#include "locc_internal.h"

namespace locc {

constexpr int kMaxBlocks = kMaxShapePoints / 64;

struct PairGeom {
  double R[9];  // R_ab, row-major
  double t[3];  // t_ab
  double lo[3], hi[3];
};

// Shared-memory scratch of the scan / ordered selection for one pair.
struct CropShared {
  unsigned long long mask[2][kMaxBlocks];
  int32_t sel[2][kMaxK];
  int32_t count[2];
};

__device__ __forceinline__ double geo_nan_max(double u, double v) {
  return (u != u || v != v) ? u + v : (u > v ? u : v);
}
__device__ __forceinline__ double geo_nan_min(double u, double v) {
  return (u != u || v != v) ? u + v : (u < v ? u : v);
}

// Rotation matrix R[3*r + c] of a quaternion given as (w, x, y, z).
__device__ __forceinline__ void geo_quat_to_rot(const float* qf, double* R) {
#pragma clang fp contract(off)
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

// Relative pose of b in a's frame and the crop box.
__device__ __forceinline__ void geo_pair(const locc_object& oa, const locc_object& ob, const ShapeDesc& da,
                                         const ShapeDesc& db, double pad, PairGeom& g) {
#pragma clang fp contract(off)
  double Ra[9], Rb[9];
  geo_quat_to_rot(oa.q, Ra);
  geo_quat_to_rot(ob.q, Rb);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) g.R[3 * r + c] = (Ra[r] * Rb[c] + Ra[3 + r] * Rb[3 + c]) + Ra[6 + r] * Rb[6 + c];
  const double d0 = (double)ob.p[0] - (double)oa.p[0];
  const double d1 = (double)ob.p[1] - (double)oa.p[1];
  const double d2 = (double)ob.p[2] - (double)oa.p[2];
#pragma unroll
  for (int r = 0; r < 3; ++r) g.t[r] = (Ra[r] * d0 + Ra[3 + r] * d1) + Ra[6 + r] * d2;
  double cb[3], eb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    cb[k] = 0.5 * ((double)db.lo[k] + (double)db.hi[k]);
    eb[k] = 0.5 * ((double)db.hi[k] - (double)db.lo[k]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double c = ((g.R[3 * r] * cb[0] + g.R[3 * r + 1] * cb[1]) + g.R[3 * r + 2] * cb[2]) + g.t[r];
    const double e = (fabs(g.R[3 * r]) * eb[0] + fabs(g.R[3 * r + 1]) * eb[1]) + fabs(g.R[3 * r + 2]) * eb[2];
    g.lo[r] = geo_nan_max((double)da.lo[r], c - e) - pad;
    g.hi[r] = geo_nan_min((double)da.hi[r], c + e) + pad;
  }
}

// b point in a's frame.
__device__ __forceinline__ void geo_xform(const PairGeom& g, double x, double y, double z, double* q) {
#pragma clang fp contract(off)
  q[0] = ((g.R[0] * x + g.R[1] * y) + g.R[2] * z) + g.t[0];
  q[1] = ((g.R[3] * x + g.R[4] * y) + g.R[5] * z) + g.t[1];
  q[2] = ((g.R[6] * x + g.R[7] * y) + g.R[8] * z) + g.t[2];
}

// b normal in a's frame (rotation only).
__device__ __forceinline__ void geo_rotate(const PairGeom& g, double x, double y, double z, double* q) {
#pragma clang fp contract(off)
  q[0] = (g.R[0] * x + g.R[1] * y) + g.R[2] * z;
  q[1] = (g.R[3] * x + g.R[4] * y) + g.R[5] * z;
  q[2] = (g.R[6] * x + g.R[7] * y) + g.R[8] * z;
}

__device__ __forceinline__ bool geo_inside(const PairGeom& g, double q0, double q1, double q2) {
  return (g.lo[0] <= q0) & (q0 <= g.hi[0]) & (g.lo[1] <= q1) & (q1 <= g.hi[1]) & (g.lo[2] <= q2) &
         (q2 <= g.hi[2]);
}

// Index of the calling wave in its workgroup, as a wave-uniform (scalar)
// value, so that everything derived from it stays in scalar registers.
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6); }

__device__ __forceinline__ int geo_wave_inclusive_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Float32 screening of the float64 membership test (same result, fewer
// instructions).
//  * a points are float32, so p >= lo (float64) holds iff p >= the smallest
//    float >= lo, and p <= hi iff p <= the largest float <= hi: the a-side
//    test is exact in float32 with outward-rounded bounds.
//  * b points are screened in the box's normalised coordinates
//    u_i = (q_i - c_i) / h_i (c_i, h_i: centre and half-width of
//    [lo_i, hi_i]), where membership is max_i |u_i| <= 1.  The map p -> u is
//    rounded to float32 (R', t') and evaluated with fmas; u' differs from u by
//    less than 2^-21 S'_i, S'_i = sum_j |R'_ij| max|p_j| + |t'_i|.  The float64
//    q of the exact test and the float64 c, h move the boundary by less than
//    (2^-50 S_i + 2^-52 (|lo_i| + |hi_i|)) / h_i, S_i being the same sum over
//    R_ab, t_ab.  With M the largest over the axes of
//    2^-19 (S'_i + (S_i + |lo_i| + |hi_i|) / h_i), max |u'| <= 1 - M implies
//    membership and max |u'| > 1 + M non-membership; only the points in
//    between take the exact float64 test.
//  * A box with lo_i > hi_i or a NaN bound holds no point: every b point is
//    screened out.  A box too thin to normalise (h_i < 2^-960, which
//    includes lo_i == hi_i) or whose map is not finite screens nothing: every
//    b point takes the exact test.
struct PairScreen {
  float alo[3], ahi[3];           // exact a-side bounds
  float R[9], t[3];               // float32 map from a b point to u
  float thr_in, thr_out;          // max |u'| <= thr_in: member; > thr_out: not
};

// One float32 step towards +inf (up) or -inf (down) from a finite f.
__device__ __forceinline__ float geo_f32_step(float f, bool up) {
  if (f == 0.f) return up ? __int_as_float(1) : -__int_as_float(1);
  const int b = __float_as_int(f);
  return __int_as_float((f > 0.f) == up ? b + 1 : b - 1);
}
__device__ __forceinline__ float geo_f32_ceil(double v) {  // smallest float >= v
  float f = (float)v;
  if ((double)f < v) f = geo_f32_step(f, true);
  return f;
}
__device__ __forceinline__ float geo_f32_floor(double v) {  // largest float <= v
  float f = (float)v;
  if ((double)f > v) f = geo_f32_step(f, false);
  return f;
}
// Wave-uniform float, kept in a scalar register.
__device__ __forceinline__ float geo_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ void geo_screen_values(const PairGeom& g, const ShapeDesc& db, PairScreen& sc) {
#pragma clang fp contract(off)
  double P[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) P[k] = fmax(fabs((double)db.lo[k]), fabs((double)db.hi[k]));
  bool empty = false, exact_only = false;
  double M = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    sc.alo[i] = geo_f32_ceil(g.lo[i]);
    sc.ahi[i] = geo_f32_floor(g.hi[i]);
    const double lo = g.lo[i], hi = g.hi[i];
    empty |= !(lo <= hi);
    const double c = 0.5 * (lo + hi);
    const double h = 0.5 * (hi - lo);
    exact_only |= !(h >= 0x1p-960);
    const double inv = 1.0 / h;
    double S = fabs(g.t[i]), S2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float r = (float)(g.R[3 * i + j] * inv);
      sc.R[3 * i + j] = r;
      S += fabs(g.R[3 * i + j]) * P[j];
      S2 += fabs((double)r) * P[j];
    }
    const float tt = (float)((g.t[i] - c) * inv);
    sc.t[i] = tt;
    S2 += fabs((double)tt);
    const double m = 0x1p-19 * (S2 + (S + fabs(lo) + fabs(hi)) * inv);
    exact_only |= !(m <= 0x1.fffffffffffffp+1023);  // inf or NaN
    M = m > M ? m : M;
  }
  if (empty || exact_only) {
#pragma unroll
    for (int k = 0; k < 9; ++k) sc.R[k] = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) sc.t[i] = 0.f;
    sc.thr_in = -1.f;                             // u' = 0: never inside
    sc.thr_out = empty ? -1.f : __int_as_float(0x7f800000);  // always / never outside
  } else {
    sc.thr_in = geo_f32_floor(1.0 - M);
    sc.thr_out = geo_f32_ceil(1.0 + M);
  }
}

// Screening constants when every thread of the workgroup computed the same
// geometry: kept in scalar registers.
__device__ __forceinline__ void geo_screen(const PairGeom& g, const ShapeDesc& db, PairScreen& sc) {
  geo_screen_values(g, db, sc);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    sc.alo[i] = geo_uniform(sc.alo[i]);
    sc.ahi[i] = geo_uniform(sc.ahi[i]);
    sc.t[i] = geo_uniform(sc.t[i]);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) sc.R[k] = geo_uniform(sc.R[k]);
  sc.thr_in = geo_uniform(sc.thr_in);
  sc.thr_out = geo_uniform(sc.thr_out);
}

__device__ __forceinline__ bool geo_member_a(const PairScreen& sc, float x, float y, float z) {
  return (sc.alo[0] <= x) & (x <= sc.ahi[0]) & (sc.alo[1] <= y) & (y <= sc.ahi[1]) & (sc.alo[2] <= z) &
         (z <= sc.ahi[2]);
}

// The exact float64 test of a b-point, for the points the float32 screen
// cannot decide (rare): out of line, so that its float64 state does not take
// registers from the scan loop around it.
__device__ __attribute__((noinline)) bool geo_member_b_exact(const PairGeom* __restrict__ gp, float x, float y,
                                                             float z) {
  double q[3];
  geo_xform(*gp, x, y, z, q);
  return geo_inside(*gp, q[0], q[1], q[2]);
}

// gp: the pair's float64 geometry, read only for the points the screen cannot
// decide (a pointer, so that a caller holding it in memory keeps it there)
__device__ __forceinline__ bool geo_member_b(const PairGeom* __restrict__ gp, const PairScreen& sc, float x, float y,
                                             float z) {
  const float q0 = __builtin_fmaf(sc.R[2], z, __builtin_fmaf(sc.R[1], y, __builtin_fmaf(sc.R[0], x, sc.t[0])));
  const float q1 = __builtin_fmaf(sc.R[5], z, __builtin_fmaf(sc.R[4], y, __builtin_fmaf(sc.R[3], x, sc.t[1])));
  const float q2 = __builtin_fmaf(sc.R[8], z, __builtin_fmaf(sc.R[7], y, __builtin_fmaf(sc.R[6], x, sc.t[2])));
  // NaN only when a coordinate is NaN, and then on every axis: both tests fail
  const float d = fmaxf(fmaxf(fabsf(q0), fabsf(q1)), fabsf(q2));
  const bool in = d <= sc.thr_in;
  const bool out = d > sc.thr_out;
  if (in | out) return in;
  return geo_member_b_exact(gp, x, y, z);
}

// Membership scan and ordered first-K selection for one pair, by a
// workgroup of 256 threads (4 wave64) over blocks of 64 stored points.  A
// round lists the next blocks, in stored order, of each object still being
// scanned, a-blocks first; wave w tests the round's blocks w, w + 4, ...,
// kScanUnroll blocks' loads in flight at a time (so the cheap a-side and the
// transforming b-side tests spread evenly over the waves), and one 64-bit
// ballot per block goes to LDS.  With full == true one round covers every
// block and the counts are exact.  Otherwise a round holds at most
// 4 kScanUnroll blocks (half each while both objects are scanned); after its
// barrier every thread adds its popcounts to the per-object counts, and an
// object's scan ends as soon as it has K members: its first K members in
// stored order are then known, and its count is a lower bound >= K.
// Finally wave 0 (object a) and wave 2 (object b) turn the ballots into
// ordered positions (prefix of popcounts over blocks, then rank of each
// member inside its block's ballot) and store the first K indices.  Ends with a
// barrier; S.sel / S.count are then valid.
template <int kScanUnroll>
__device__ __forceinline__ void geo_scan_select(const PairGeom* __restrict__ gp, const PairScreen& sc, int off_a, int n_a,
                                                int off_b, int n_b, const DeviceLibrary& lib, int K, bool full,
                                                CropShared& S) {
  constexpr int R = 4 * kScanUnroll;  // blocks per round
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_index();
  const int nblk_a = (n_a + 63) >> 6, nblk_b = (n_b + 63) >> 6;
  int cur_a = 0, cur_b = 0, cnt_a = 0, cnt_b = 0;  // uniform
  for (;;) {
    const bool act_a = cur_a < nblk_a && (full || cnt_a < K);
    const bool act_b = cur_b < nblk_b && (full || cnt_b < K);
    if (!act_a && !act_b) break;
    // a round: all remaining blocks when every count is wanted (one barrier
    // in total), else at most R blocks, shared between the two objects
    int q_a = 0, q_b = 0;
    if (full) {
      q_a = nblk_a - cur_a;
      q_b = nblk_b - cur_b;
    } else {
      if (act_a) q_a = nblk_a - cur_a < (act_b ? R / 2 : R) ? nblk_a - cur_a : (act_b ? R / 2 : R);
      if (act_b) q_b = nblk_b - cur_b < R - q_a ? nblk_b - cur_b : R - q_a;
    }
    const int q = q_a + q_b;
    for (int i0 = wave; i0 < q; i0 += 4 * kScanUnroll) {
      float x[kScanUnroll], y[kScanUnroll], z[kScanUnroll];
#pragma unroll
      for (int u = 0; u < kScanUnroll; ++u) {
        // block, object and base pointers are wave-uniform; only the lane
        // offset lives in a vector register
        const int i = i0 + 4 * u;
        const int side = i >= q_a;
        const int off = side ? off_b : off_a;
        const unsigned k = ((unsigned)(side ? cur_b + i - q_a : cur_a + i) << 6) + (unsigned)lane;
        x[u] = y[u] = z[u] = 0.f;
        if (i < q && k < (unsigned)(side ? n_b : n_a)) {
          x[u] = (lib.px + off)[k];
          y[u] = (lib.py + off)[k];
          z[u] = (lib.pz + off)[k];
        }
      }
#pragma unroll
      for (int u = 0; u < kScanUnroll; ++u) {
        const int i = i0 + 4 * u;
        if (i < q) {  // uniform
          const int side = i >= q_a;
          const int lb = side ? cur_b + i - q_a : cur_a + i;
          const int k = (lb << 6) + lane;
          bool in = false;
          if (k < (side ? n_b : n_a))
            in = side ? geo_member_b(gp, sc, x[u], y[u], z[u]) : geo_member_a(sc, x[u], y[u], z[u]);
          const unsigned long long m = __ballot(in);
          if (lane == 0) S.mask[side][lb] = m;
        }
      }
    }
    __syncthreads();
    cur_a += q_a;
    cur_b += q_b;
    if (full) continue;  // every block is scanned in the one round
    // the round's popcounts, one block per lane, summed over the wave (every
    // wave computes the same totals)
    int ca = 0, cb = 0;
    for (int i = lane; i < q_a; i += 64) ca += __popcll(S.mask[0][cur_a - q_a + i]);
    for (int i = lane; i < q_b; i += 64) cb += __popcll(S.mask[1][cur_b - q_b + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ca += __shfl_xor(ca, o, 64);
      cb += __shfl_xor(cb, o, 64);
    }
    cnt_a += __builtin_amdgcn_readfirstlane(ca);  // the same in every lane: keep the counts scalar
    cnt_b += __builtin_amdgcn_readfirstlane(cb);
  }
  if ((wave & 1) == 0) {
    const int side = wave >> 1;
    const int nblk = side ? cur_b : cur_a;  // blocks scanned
    // block per lane (chunks of 64 blocks): the exclusive prefix of the
    // popcounts is each block's first position.  Then, block after block in
    // stored order while positions stay below K, the block's ballot and
    // start are read from its lane into scalar registers and every lane
    // places its own point at start + (members below it in the block).
    int carry = 0;
    for (int base = 0; base < nblk; base += 64) {
      const int blk = base + lane;
      const unsigned long long m = blk < nblk ? S.mask[side][blk] : 0ull;
      const int c = __popcll(m);
      const int incl = geo_wave_inclusive_scan(c, lane);
      const int start = carry + incl - c;
      const int nb = nblk - base < 64 ? nblk - base : 64;
      const unsigned m_lo = (unsigned)m, m_hi = (unsigned)(m >> 32);
      for (int j = 0; j < nb; ++j) {
        const int sj = __builtin_amdgcn_readlane(start, j);
        if (sj >= K) break;
        const unsigned lo = __builtin_amdgcn_readlane(m_lo, j), hi = __builtin_amdgcn_readlane(m_hi, j);
        const unsigned mine = lane < 32 ? (lo >> lane) & 1u : (hi >> (lane - 32)) & 1u;
        const int pos = sj + (int)__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
        if (mine && pos < K) S.sel[side][pos] = ((base + j) << 6) + lane;
      }
      carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) S.count[side] = carry;
  }
  __syncthreads();
}

// Per-pair record of the pair set-up kernel.
struct PairSetup {
  PairGeom g;
  PairScreen sc;
  int32_t valid;          // 0: invalid pair (index out of range, i == j, shape id out of range)
  int32_t a, swapped;     // canonical first object, caller order flag
  int32_t off_a, n_a, off_b, n_b;  // stored points of the two shapes
};
static_assert(sizeof(PairSetup) <= kPairSetupBytes, "pair set-up record");

// Encoder input row (x, y, z, nx, ny, nz) in a's frame of stored point gi of
// object `side` (0 = a as stored, 1 = b transformed in float64, then rounded).
__device__ __forceinline__ void geo_row(const PairGeom& g, const DeviceLibrary& lib, int gi, int side, float* v) {
  if (side) {
    double q[3], n[3];
    geo_xform(g, lib.px[gi], lib.py[gi], lib.pz[gi], q);
    geo_rotate(g, lib.nx[gi], lib.ny[gi], lib.nz[gi], n);
    v[0] = (float)q[0];
    v[1] = (float)q[1];
    v[2] = (float)q[2];
    v[3] = (float)n[0];
    v[4] = (float)n[1];
    v[5] = (float)n[2];
  } else {
    v[0] = lib.px[gi];
    v[1] = lib.py[gi];
    v[2] = lib.pz[gi];
    v[3] = lib.nx[gi];
    v[4] = lib.ny[gi];
    v[5] = lib.nz[gi];
  }
}

// Validate pair p and fetch its canonical objects and shapes.  Returns false
// for an invalid pair (index out of range, i == j, shape id out of range).
__device__ __forceinline__ bool geo_fetch(const locc_object* objs, int n_objs, const int32_t* pairs, int p,
                                          const DeviceLibrary& lib, int& a, int& swapped, locc_object& oa,
                                          locc_object& ob, ShapeDesc& da, ShapeDesc& db) {
  const int i = pairs[2 * p];
  const int j = pairs[2 * p + 1];
  if (!(i >= 0 && i < n_objs && j >= 0 && j < n_objs && i != j)) return false;
  a = i < j ? i : j;
  const int b = i < j ? j : i;
  swapped = i > j;
  oa = objs[a];
  ob = objs[b];
  if (!(oa.shape >= 0 && oa.shape < lib.n_shapes && ob.shape >= 0 && ob.shape < lib.n_shapes)) return false;
  da = lib.shapes[oa.shape];
  db = lib.shapes[ob.shape];
  return true;
}

}  // namespace locc
