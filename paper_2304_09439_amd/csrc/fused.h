// Fused persistent BF16 path: arguments, weight packing and launcher.
#pragma once

#include "locc_internal.h"
#include "pack.h"

namespace locc {

struct FusedArgs {
  const locc_object* objs;
  int32_t n_objs;
  const int32_t* pairs;
  int32_t n_pairs;              // capacity
  const int32_t* n_pairs_dev;   // actual count in device memory, or null
  DeviceLibrary lib;
  int32_t K;
  double pad;
  // packed weights (see bf16_pack)
  const unsigned short* w1p;
  const unsigned short* w2p;
  const float* b2;
  const unsigned short* h1p;
  const float* c1;
  const unsigned short* h2p;
  const float* c2;
  const unsigned short* h3p;
  const float* c3;
  // outputs
  locc_contact* out;
  int32_t* counts;   // [P][2] or null
  float* z_dbg;      // [P][2 h2] or null (the pooled features; always written by the argmax variant)
  float* y_dbg;      // [P][8] or null
  uint8_t* amax;     // argmax variant: [P][2][h2] row of the largest raw layer-2 sum per channel (first on ties)
  unsigned long long* err_counter;
  // split schedule: rows and per-pair records produced by the crop kernel
  const unsigned short* rows_bf16;  // [P][2K][8]
  const PairMeta* meta;             // [P]
  // schedule
  unsigned int* queue;  // [2]: next unclaimed pair, finished workgroups (both 0 between launches)
  int32_t claim;        // pairs claimed at once
  int32_t dynamic;      // 1: atomic queue, 0: static round robin
  int32_t dev_base;     // first pair of this launch within the step (device count mode)
};

void bf16_bind(FusedArgs& a, const unsigned char* dev_base, int h1, int h2, int hh);

// Workgroups per CU the fused kernel is compiled for.
constexpr int kFusedWgPerCu = 2;
constexpr int kFusedTile = 32;

// precropped = false: crop, encoder and head in one kernel; true: encoder and
// head only, reading rows_bf16 / meta written by the crop kernel.
hipError_t launch_fused_bf16(const FusedArgs& a, int h1, int h2, int hh, int grid, bool precropped, hipStream_t s);
// The encoder of the split schedule alone, recording the pooled features (z_dbg, float) and per channel the
// row of the largest raw layer-2 sum (amax; 255 for an object with no rows), for the pose gradients.
hipError_t launch_encoder_bf16_argmax(const FusedArgs& a, int h1, int h2, int hh, int grid, hipStream_t s);
// The split schedule's BF16 encoder + head with W2 in LDS (encoder_bf16.hip): one workgroup of eight waves
// per CU, groups of 64 pairs; argmax: the encoder alone, writing z_dbg and amax as the argmax variant above.
hipError_t launch_encoder_head_bf16_lds(const FusedArgs& a, int h1, int h2, int hh, int grid, bool argmax,
                                        hipStream_t s);

// ---------------------------------------------------------------- FP8 path
// Encoder + head on the rows the crop kernel wrote, with encoder layer 2 and
// head layers 1-2 in OCP e4m3 (per-layer scales, FP32 accumulation), or
// (head8 = false) encoder layer 2 in e4m3 and the head in bf16.
struct Fp8Args {
  const locc_object* objs;
  int32_t n_pairs;              // capacity
  const int32_t* n_pairs_dev;   // actual count in device memory, or null
  int32_t K;
  // packed weights (see fp8_pack)
  const unsigned short* w1p;    // bf16
  const unsigned char* w2p;     // e4m3, W2 / s_w2
  const float* b2;
  const unsigned char* h1p;     // e4m3, H1 / s_h1 (bf16 fragments without the fp8 head)
  const float* c1;
  const unsigned char* h2p;     // e4m3, H2 / s_h2 (bf16 fragments without the fp8 head)
  const float* c2;
  const unsigned short* h3p;    // bf16
  const float* c3;
  // scales: weights (amax / 448) and activations entering an fp8 layer
  float s_w2, s_h1, s_h2;
  float s_h1in;  // encoder layer-1 output (layer 1's weights are packed divided by it)
  float s_z;     // pooled encoder features
  float s_g1;    // head layer-1 output
  // rows and per-pair records from the crop kernel
  const unsigned short* rows_bf16;  // [P][2K][8]
  const PairMeta* meta;             // [P]
  // outputs
  locc_contact* out;
  float* z_dbg;  // [P][2 h2] or null
  float* y_dbg;  // [P][8] or null
  // schedule
  unsigned int* queue;
  int32_t claim;
  int32_t dynamic;
  int32_t dev_base;  // first pair of this launch within the step (device count mode)
};

void fp8_bind(Fp8Args& a, const unsigned char* dev_base, int h1, int h2, int hh, bool head8);
hipError_t launch_encoder_head_fp8(const Fp8Args& a, int h1, int h2, int hh, bool head8, int grid, hipStream_t s);

// Calibration: maxima over the valid pairs of the encoder layer-1 output, the
// pooled encoder features and the head layer-1 output, computed in FP32 from
// the crop kernel's rows and the unquantised weights; amax[3] (device, zeroed
// by the caller) receives them as float bits via atomicMax.
struct CalibArgs {
  const float* w;                   // weights, flat (W1, b1, W2, b2, H1, c1, ...)
  int32_t h1, h2, hh;
  int32_t n_pairs;
  int32_t K;
  const unsigned short* rows_bf16;
  const PairMeta* meta;
  unsigned int* amax;
};
hipError_t launch_calibrate_fp8(const CalibArgs& a, int grid, hipStream_t s);

}  // namespace locc
