// Fused persistent BF16 path: arguments, weight packing and launcher.
#pragma once

#include "locc_internal.h"

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
  float* z_dbg;      // [P][2 h2] or null
  float* y_dbg;      // [P][8] or null
  unsigned long long* err_counter;
  // split schedule: rows and per-pair records produced by the crop kernel
  const unsigned short* rows_bf16;  // [P][2K][8]
  const PairMeta* meta;             // [P]
  // schedule
  unsigned int* queue;  // [2]: next unclaimed pair, finished workgroups (both 0 between launches)
  int32_t claim;        // pairs claimed at once
  int32_t dynamic;      // 1: atomic queue, 0: static round robin
};

// Byte offsets of the packed BF16 weights inside one device buffer.
struct Bf16Layout {
  size_t w1, w2, b2, h1, c1, h2, c2, h3, c3, total;
};
Bf16Layout bf16_layout(int h1, int h2, int hh);
void bf16_pack(const float* W1, const float* b1, const float* W2, const float* b2, const float* H1,
               const float* c1, const float* H2, const float* c2, const float* H3, const float* c3, int h1,
               int h2, int hh, unsigned char* dst);
void bf16_bind(FusedArgs& a, const unsigned char* dev_base, int h1, int h2, int hh);

// Workgroups per CU the fused kernel is compiled for.
constexpr int kFusedWgPerCu = 2;
constexpr int kFusedTile = 32;

// precropped = false: crop, encoder and head in one kernel; true: encoder and
// head only, reading rows_bf16 / meta written by the crop kernel.
hipError_t launch_fused_bf16(const FusedArgs& a, int h1, int h2, int hh, int grid, bool precropped, hipStream_t s);

}  // namespace locc
