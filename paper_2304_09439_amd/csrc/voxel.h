// Internal declarations of the voxel-embedding variant (voxel.hip, voxel_capi.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "locc_voxel.h"

namespace locc {
namespace vox {

constexpr int kM = 6;              // grid cells per axis
constexpr int kCells = kM * kM * kM;
constexpr int kH = 256;            // point MLP width
constexpr int kC = 128;            // U-Net channels
constexpr int kB = 4 * 4 * 4;      // bottleneck cells
constexpr int kF = 16;             // embedding width
constexpr int kHP = 128;           // predictor width
constexpr int kIn = kF + 12;       // predictor input per object
constexpr int kMaxPoints = 65536;  // per shape
constexpr size_t kWeightCount = 5534609;

// Per-shape record: rows [off, off + n) of the SoA xyz, and the box of the stored xyz.
struct Shape {
  int32_t off;
  int32_t n;
  float lo[3];
  float hi[3];
};
static_assert(sizeof(Shape) == 32, "Shape layout");

// Device pointers to every weight array: the flat vector as uploaded, except
// the point MLP's layers 2-3, used transposed to [in][out] (a coalesced row
// of outputs per input), and the U-Net's weights, used transposed to
// [27 taps][in][out], both from a second, packed buffer.
struct PackedNet {
  const float *P1, *p1, *P2t, *p2, *P3t, *p3;  // point MLP
  const float *C[4], *k[4], *D[4], *e[4];      // U-Net convs, transposed convs (C, D: [27][in][128])
  const float *L, *l;                          // embedding map [16][384]
  const float *A[3], *a[3];                    // per-object MLP [128][28], [128][128] x 2 (row-major)
  const float *Bw[3], *b[4], *B4;              // pair MLP [128][128] x 3, output row [128], b[3] = its bias
};
size_t packed_floats();
// Host-side transposition of the flat weights into dst (packed_floats() floats).
void pack_transposed(const float* flat, float* dst);
PackedNet packed_view(const float* d_raw, const float* d_packed);

struct EncoderBuffers {
  int32_t* order; // [n_points]: per shape, its point indices sorted by grid cell
  uint8_t* cell;  // [n_points]: the grid cell of each entry of order
  float* grid;    // [S][256][216] (cell max of the point features, channel-major)
  float* c[4];    // [S][128][64]
  float* d[3];    // [S][128][64]
  float* d4;      // [S][128][216]
  float* glob;    // [S][256]
};
size_t encoder_scratch_floats(int n_shapes, int64_t n_points);
EncoderBuffers encoder_carve(float* base, int n_shapes, int64_t n_points);

// Shape encoder over every shape; grid must be zero (the cell max starts at 0).
hipError_t launch_encoder(const PackedNet& w, const Shape* shapes, int n_shapes, int max_points, const float* xyz,
                          int64_t n_points, const EncoderBuffers& b, float* emb, double* consts,
                          hipStream_t s);

struct PairArgs {
  const locc_object* objs;
  int32_t n_objs;
  const int32_t* pairs;
  int32_t n_pairs;
  const Shape* shapes;
  int32_t n_shapes;
  const double* consts;   // [S][4]: cell size s_0, s_1, s_2 and the margin eps (float64)
  const float* emb;       // [S][216][16]
  PackedNet w;
  float* out;             // [P][2]
  int32_t* counts;        // [P][2] or null
  float* pooled;          // [P][2][16] or null
  unsigned long long* err;
  float* z;               // workspace [P][2][28]: per-object predictor inputs (canonical order)
  int32_t* valid;         // workspace [P]
};
// Workspace bytes of a launch over n_pairs pairs.
size_t pair_workspace_bytes(int n_pairs);
// Carves the workspace at base into a.z / a.valid.
void pair_workspace_carve(void* base, int n_pairs, PairArgs& a);
// Two launches: cell selection and mean embeddings (one wave per pair), then
// the predictor MLPs (32 pairs per workgroup).
hipError_t launch_pairs(const PairArgs& a, hipStream_t s);

}  // namespace vox
}  // namespace locc
