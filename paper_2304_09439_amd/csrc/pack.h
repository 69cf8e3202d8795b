// Host-side packing of the network weights into the fragment orders of the
// matrix-core kernels (pack.cpp).  Plain C++, no HIP.  Weights come in the
// order of locc_upload_weights (row-major W1 [h1][6], b1, W2 [h2][h1], b2,
// H1 [hh][2 h2], c1, H2 [hh][hh], c2, H3 [8][hh], c3).
#pragma once

#include <cstddef>

namespace locc {

// bf16 of f, round to nearest even (NaN stays a quiet NaN).
unsigned short host_bf16(float f);
// OCP e4m3 (E4M3FN) of x, round to nearest even, saturating at 448.
unsigned char host_e4m3(float x);

// ---------------------------------------------------------------- FP32
// Float offsets of the packed FP32 weights (net_fp32.hip reads them).
struct Fp32Layout {
  size_t w1, w2, b2, h1, c1, h2, c2, h3, c3, total;
};
Fp32Layout fp32_layout(int h1, int h2, int hh);
size_t fp32_pack_floats(int h1, int h2, int hh);
void fp32_pack(const float* W1, const float* b1, const float* W2, const float* b2, const float* H1,
               const float* c1, const float* H2, const float* c2, const float* H3, const float* c3, int h1,
               int h2, int hh, float* dst);

// ---------------------------------------------------------------- BF16
// Byte offsets of the packed BF16 weights inside one device buffer.
struct Bf16Layout {
  size_t w1, w2, b2, h1, c1, h2, c2, h3, c3, total;
};
Bf16Layout bf16_layout(int h1, int h2, int hh);
void bf16_pack(const float* W1, const float* b1, const float* W2, const float* b2, const float* H1,
               const float* c1, const float* H2, const float* c2, const float* H3, const float* c3, int h1,
               int h2, int hh, unsigned char* dst);
// A head matrix H [out][in] (row-major) as the B operand fragments of the bf16
// head (head_bf16.h); out_pad / 32 column tiles, rows past out zero.
void bf16_pack_head(const float* H, int in, int out, int out_pad, unsigned short* dst);

// ---------------------------------------------------------------- FP8
struct Fp8Layout {
  size_t w1, w2, b2, h1, c1, h2, c2, h3, c3, total;
};
// head8: head layers 1-2 in e4m3 (else their bf16 fragments)
Fp8Layout fp8_layout(int h1, int h2, int hh, bool head8);
// weight_scales receives (s_w2, s_h1, s_h2); s_h1 = s_h2 = 1 without the fp8 head.
void fp8_pack(const float* W1, const float* b1, const float* W2, const float* b2, const float* H1, const float* c1,
              const float* H2, const float* c2, const float* H3, const float* c3, int h1, int h2, int hh, bool head8,
              unsigned char* dst, float* weight_scales);
// Encoder layer-1 pack of the FP8 path, scaled by inv = 1 / s_x (h1 * 8 bf16 values).
void fp8_pack_w1(const float* W1, const float* b1, int h1, float inv, unsigned short* dst);

}  // namespace locc
