// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "locc.h"
#include "pack.h"

namespace locc {

// Per-kernel timing without marker packets: while a profiled step is being
// enqueued on this host thread, its first kernel records `start` as its
// dispatch begins and every kernel records `stop` as it ends (events attached
// to the dispatches themselves, so the timing adds no work between kernels).
struct LaunchTiming {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
extern thread_local LaunchTiming g_launch_timing;

// Every kernel of the library is launched through this.
template <class F, class... Args>
inline void kernel_launch(F kernel, const dim3& grid, const dim3& block, uint32_t shmem, hipStream_t s,
                          Args... args) {
  LaunchTiming& t = g_launch_timing;
  if (!t.stop) {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0u, args...);
  t.start = nullptr;
}

// Per-shape descriptor in device memory: rows [off, off + n) of the SoA point
// arrays, and the axis-aligned box of the stored xyz (min / max).  32 bytes.
struct ShapeDesc {
  int32_t off;
  int32_t n;
  float lo[3];
  float hi[3];
};
static_assert(sizeof(ShapeDesc) == 32, "ShapeDesc layout");

// Per-pair record written by the crop step and read by the network steps.
//   a        canonical first object (min(i, j)), or -1 for an invalid pair
//   swapped  1 if the caller gave (b, a)
//   m_a, m_b number of valid encoder rows (min(count, K)) per object
struct PairMeta {
  int32_t a;
  int32_t swapped;
  int32_t m_a;
  int32_t m_b;
};
static_assert(sizeof(PairMeta) == 16, "PairMeta layout");

// Largest point count per shape (the crop step keeps one 64-bit membership
// mask per 64 points of each object in LDS).
constexpr int kMaxShapePoints = 16384;
constexpr int kMaxK = 256;
// Encoder input rows: 8 floats (x, y, z, nx, ny, nz, 1, 0) stored in the
// order (e0, e2, e4, e6, e1, e3, e5, e7) so that each half-wave of a 32x32x2
// MFMA operand load reads one float4.
constexpr int kRowFloats = 8;

struct DeviceLibrary {
  const ShapeDesc* shapes;
  int32_t n_shapes;
  const float* px;
  const float* py;
  const float* pz;
  const float* nx;
  const float* ny;
  const float* nz;
};

// Pair count of a launch: n_pairs is the capacity (grid sizing); when
// n_pairs_dev is set the kernels read the actual count from device memory
// (clamped to the capacity), so one captured graph serves steps whose pair
// counts differ.  A launch over a chunk that starts at pair `base` of the
// step sees *dev - base pairs, clamped to [0, capacity].
__device__ __forceinline__ int pair_count(int capacity, const int32_t* dev, int base = 0) {
  if (!dev) return capacity;
  const int n = *dev - base;
  return n < 0 ? 0 : (n < capacity ? n : capacity);
}

struct CropArgs {
  const locc_object* objs;
  int32_t n_objs;
  const int32_t* pairs;
  int32_t n_pairs;
  const int32_t* n_pairs_dev;  // or null
  DeviceLibrary lib;
  int32_t K;
  double pad;
  int32_t* idx_out;      // [P][2][K] caller order, may be null
  int32_t* counts_out;   // [P][2] caller order, may be null
  PairMeta* meta;        // [P], may be null
  float* rows;           // [P][2K][8], may be null
  unsigned short* rows_bf16;  // [P][2K][8] bf16 (x, y, z, nx, ny, nz, 1, 0), rows up to the next
                              // multiple of 32 of each object's count written, may be null
  unsigned long long* err_counter;
  void* setup;           // [P] records of kPairSetupBytes (library workspace), required
  int32_t dev_base;      // first pair of this launch within the step (device count mode)
};

// Bytes of the per-pair record (pose, box, screening constants, canonical
// order) the pair set-up kernel writes for the crop kernel.
constexpr size_t kPairSetupBytes = 320;

// Pair set-up (one thread per pair), then the crop (one wave per object of a
// pair, the two waves of a pair in one workgroup).  unroll (2, 4 or 8): a
// wave issues the loads of max(1, unroll / 4) blocks of 256 points together.
hipError_t launch_crop(const CropArgs& a, hipStream_t s, int unroll = 8);

// Broad phase over environments: world boxes, then every overlapping pair
// i < j of objects of the same environment (see broad_phase.hip).
struct BroadArgs {
  const locc_object* objs;
  int32_t n_objs;
  const int32_t* env_offsets;  // [n_envs + 1]
  int32_t n_envs;
  DeviceLibrary lib;
  double* boxes;               // [n_objs][6] lo xyz, hi xyz (scratch)
  long long* env_count;        // [n_envs] overlapping pairs per environment (scratch)
  long long* env_start;        // [n_envs] first output position per environment (scratch)
  int32_t* pairs;              // [capacity][2], may be null when capacity is 0
  int32_t capacity;
  int32_t* count;              // [2]: pairs written, total (saturated)
};

// Scratch bytes of a broad phase over n_objs objects and n_envs environments.
size_t broad_phase_scratch_bytes(int n_objs, int n_envs);
// Carves the scratch at `base` into a.boxes / env_count / env_start.
void broad_phase_carve(void* base, int n_objs, int n_envs, BroadArgs& a);
// Four launches on s: world boxes, per-environment counts, the scan (which
// writes count), the ordered write of the pairs.
hipError_t launch_broad_phase(const BroadArgs& a, hipStream_t s);

// FP32 network weights packed in MFMA fragment order (see net_fp32.hip).
struct Fp32Net {
  int h1, h2, hh;
  const float* w1pack;  // [h1/32][4][64]
  const float* w2pack;  // [4 waves][h2/128][h1/2][64]
  const float* b2;      // [h2]
  const float* h1pack;  // [hh/32][h2][64]   (k-steps = 2*h2 / 2)
  const float* c1;      // [hh]
  const float* h2pack;  // [hh/32][hh/2][64]
  const float* c2;      // [hh]
  const float* h3;      // [8][hh] plain row-major
  const float* c3;      // [8]
};

struct NetArgs {
  const float* rows;      // [P][2K][8]
  const PairMeta* meta;   // [P]
  const locc_object* objs;
  int32_t n_pairs;
  const int32_t* n_pairs_dev;  // or null
  int32_t K;
  float* z;               // [P][2 h2] workspace (always written)
  float* y_dbg;           // [P][8] or null
  locc_contact* out;      // [P]
  uint8_t* amax;          // [P][2][h2] row of the largest raw layer-2 sum per channel (first on ties), or null
};

hipError_t launch_encoder_fp32(const Fp32Net& w, const NetArgs& a, int n_cu, hipStream_t s);
hipError_t launch_head_fp32(const Fp32Net& w, const NetArgs& a, hipStream_t s);

// Device views of the FP32 weights packed by fp32_pack (pack.h).
Fp32Net fp32_view(const float* dev_base, int h1, int h2, int hh);

}  // namespace locc
