// Internal declarations of the pose-gradient path (grad.hip).
#pragma once

#include "locc_internal.h"

namespace locc {

// Offsets (floats) of the arrays in the flat FP32 weight vector W1, b1, W2, b2, H1, c1, H2, c2, H3, c3.
struct GradOffsets {
  size_t W1, b1, W2, b2, H1, c1, H2, c2, H3, c3;
};

struct GradArgs {
  const locc_object* objs;
  int32_t n_objs;
  const int32_t* pairs;
  int32_t n_pairs;
  const PairMeta* meta;   // [P] from the crop
  const float* rows;      // [P][2K][8] FP32 encoder rows
  const int32_t* idx;     // [P][2][K] stored point indices, caller order
  const float* z;         // [P][2 h2] pooled features
  const uint8_t* amax;    // [P][2][h2] argmax rows
  float* dm;              // [P][h2] workspace: d logit / d (second object's raw maxima)
  float* grad;            // [P][14] out
  int32_t K;
  DeviceLibrary lib;
  const float* raw;       // flat FP32 weights (device)
  GradOffsets off;
  const float* H1t;       // [2 h2][hh]
  const float* H2t;       // [hh][hh]
  const float* W2t;       // [h1][h2]
  uint8_t* argmax_b;      // [P][h2] copy of the second object's argmax rows, or null
};

// Head backward (32 pairs per workgroup), then one workgroup per pair for the
// encoder backward at the argmax rows and the chain to the poses.
hipError_t launch_pose_gradients(const GradArgs& a, int h1, int h2, int hh, hipStream_t s);

// One training step of the FP32 network (crop and encoder already run, with
// argmax rows): loss terms, weight gradients, Adam, and the repacking of the
// updated weights into the layouts the kernels read.
constexpr int kEncSplit = 16;    // pair ranges of the encoder weight gradients
constexpr int kOuterSplit = 64;  // pair ranges of the head weight gradients

struct TrainArgs {
  int32_t n_pairs;
  const PairMeta* meta;   // [P]
  const float* rows;      // [P][2K][8]
  const float* z;         // [P][2 h2]
  const uint8_t* amax;    // [P][2][h2]
  const float* labels;    // [P] 0 / 1
  int32_t K;
  float alpha;            // feature-norm weight
  float* raw;             // flat FP32 master weights (updated in place)
  GradOffsets off;
  const float* H1t;       // [2 h2][hh] (of the weights before the step)
  const float* H2t;       // [hh][hh]
  // workspace
  float *g1, *g2, *du2, *du1;  // [P][hh]
  float* dmv;             // [P][2 h2]
  float* dx;              // [P]
  float* lossp;           // [P][2]: cross-entropy, squared feature norm
  float* w1part;          // [kEncSplit][h2][h1][7]: per pair-range and channel partials of dW1, db1
  float* w2part;          // [kEncSplit][h2][h1 + 1]: partials of dW2 and db2
  float* opart;           // [kOuterSplit][hh][max(hh, 2 h2) + 1]: partial outer sums
  // context state
  float* grad;            // [n] flat, same layout as the weights
  float *m, *v;           // Adam moments [n]
  size_t n;
  float lr, beta1, beta2, eps, corr1, corr2;  // corr = 1 / (1 - beta^t)
  float* loss;            // [2] out: mean cross-entropy, alpha x mean squared feature norm
  // repacking: dst[i] = src_idx[i] >= 0 ? raw[src_idx[i]] : 0
  float* pack_dst;
  const int32_t* pack_idx;
  size_t pack_n;
  float* tr_dst;          // H1^T, H2^T, W2^T
  const int32_t* tr_idx;
  size_t tr_n;
};

hipError_t launch_train_step(const TrainArgs& a, int h1, int h2, int hh, hipStream_t s);

}  // namespace locc
