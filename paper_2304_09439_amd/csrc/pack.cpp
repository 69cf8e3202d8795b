// Host-side packing of row-major weights into the fragment orders the
// matrix-core kernels read (FP32, BF16 and FP8 paths), and the host
// conversions to bf16 and OCP e4m3 it uses.  Plain C++: no HIP, so it is
// also built and run under the address and undefined-behaviour sanitizers
// by the host tests.
#include "pack.h"

#include <cmath>
#include <cstdint>
#include <cstring>

namespace locc {
namespace {

size_t align64(size_t n) { return (n + 63) & ~size_t(63); }
size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
// Layer 1's output order: feature of lane group g, value r of 32-feature tile ft (the order in which a
// lane holds a column of a 32x32 matrix-core result); layer 2's reduction index is packed in it.
constexpr int perm_feature(int ft, int g, int r) { return 32 * ft + 8 * (r / 4) + 4 * g + r % 4; }

float amax_of(const float* w, size_t n) {
  float m = 0.f;
  for (size_t k = 0; k < n; ++k) m = std::fmax(m, std::fabs(w[k]));
  return m;
}

}  // namespace

unsigned short host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// OCP e4m3 (E4M3FN) of x with round to nearest even; magnitudes beyond 448
// saturate to 448.
unsigned char host_e4m3(float x) {
  const unsigned char s = std::signbit(x) ? 0x80 : 0;
  const double a = std::fabs((double)x);
  if (!(a == a)) return 0x7F;
  if (a >= 464.0) return s | 0x7E;
  if (a < std::ldexp(1.0, -6)) return s | (unsigned char)std::nearbyint(a / std::ldexp(1.0, -9));
  int e;
  std::frexp(a, &e);
  e -= 1;
  double q = std::nearbyint((a / std::ldexp(1.0, e) - 1.0) * 8.0);
  if (q == 8.0) {
    q = 0.0;
    e += 1;
  }
  int code = ((e + 7) << 3) | (int)q;
  if (code > 0x7E) code = 0x7E;
  return s | (unsigned char)code;
}

// ---------------------------------------------------------------- FP32
Fp32Layout fp32_layout(int h1, int h2, int hh) {
  Fp32Layout L{};
  size_t o = 0;
  L.w1 = o; o = align64(o + (size_t)8 * h1);
  L.w2 = o; o = align64(o + (size_t)h2 * h1);
  L.b2 = o; o = align64(o + h2);
  L.h1 = o; o = align64(o + (size_t)hh * 2 * h2);
  L.c1 = o; o = align64(o + hh);
  L.h2 = o; o = align64(o + (size_t)hh * hh);
  L.c2 = o; o = align64(o + hh);
  L.h3 = o; o = align64(o + (size_t)8 * hh);
  L.c3 = o; o = align64(o + 8);
  L.total = o;
  return L;
}

size_t fp32_pack_floats(int h1, int h2, int hh) { return fp32_layout(h1, h2, hh).total; }

void fp32_pack(const float* W1, const float* b1, const float* W2, const float* b2, const float* H1,
               const float* c1, const float* H2, const float* c2, const float* H3, const float* c3, int h1,
               int h2, int hh, float* dst) {
  const Fp32Layout L = fp32_layout(h1, h2, hh);
  std::memset(dst, 0, sizeof(float) * L.total);
  // layer 1 A operand: [W1 | b1 | 0][f][c], f = 32 ft + l % 32, c = 2 s + l / 32
  for (int ft = 0; ft < h1 / 32; ++ft)
    for (int s = 0; s < 4; ++s)
      for (int l = 0; l < 64; ++l) {
        const int f = 32 * ft + l % 32, c = 2 * s + l / 32;
        dst[L.w1 + (ft * 4 + s) * 64 + l] = c < 6 ? W1[f * 6 + c] : (c == 6 ? b1[f] : 0.f);
      }
  // layer 2 B operand, reduction index permuted to layer 1's output layout
  const int CT = h2 / 128, KS = h1 / 2;
  for (int w = 0; w < 4; ++w)
    for (int ct = 0; ct < CT; ++ct)
      for (int s = 0; s < KS; ++s)
        for (int l = 0; l < 64; ++l) {
          const int col = (w * CT + ct) * 32 + l % 32;
          const int f = perm_feature(s / 16, l / 32, s % 16);
          dst[L.w2 + ((size_t)(w * CT + ct) * KS + s) * 64 + l] = W2[(size_t)col * h1 + f];
        }
  std::memcpy(dst + L.b2, b2, sizeof(float) * h2);
  // head layers: B[k][j] = H[j][k]; lane l holds H[32 ct + l % 32][2 s + l / 32]
  auto pack_head = [&](const float* H, int in, int out, size_t at) {
    const int ks = in / 2;
    for (int ct = 0; ct < out / 32; ++ct)
      for (int s = 0; s < ks; ++s)
        for (int l = 0; l < 64; ++l)
          dst[at + ((size_t)ct * ks + s) * 64 + l] = H[(size_t)(32 * ct + l % 32) * in + 2 * s + l / 32];
  };
  pack_head(H1, 2 * h2, hh, L.h1);
  std::memcpy(dst + L.c1, c1, sizeof(float) * hh);
  pack_head(H2, hh, hh, L.h2);
  std::memcpy(dst + L.c2, c2, sizeof(float) * hh);
  std::memcpy(dst + L.h3, H3, sizeof(float) * 8 * hh);
  std::memcpy(dst + L.c3, c3, sizeof(float) * 8);
}


// ---------------------------------------------------------------- BF16
// B operand of 32x32x16: lane l of k-step s of column tile ct holds H[32 ct + l % 32][16 s + 8 (l / 32) + e]
// (rows from out to out_pad zero)
void bf16_pack_head(const float* H, int in, int out, int out_pad, unsigned short* dst) {
  const int ks = in / 16;
  for (int ct = 0; ct < out_pad / 32; ++ct)
    for (int s = 0; s < ks; ++s)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          const int row = 32 * ct + l % 32;
          const float v = row < out ? H[(size_t)row * in + 16 * s + 8 * (l / 32) + e] : 0.f;
          dst[(((size_t)ct * ks + s) * 64 + l) * 8 + e] = host_bf16(v);
        }
}

Bf16Layout bf16_layout(int h1, int h2, int hh) {
  Bf16Layout L{};
  size_t o = 0;
  L.w1 = o; o = align256(o + (size_t)h1 * 8 * 2);
  L.w2 = o; o = align256(o + (size_t)h2 * h1 * 2);
  L.b2 = o; o = align256(o + (size_t)h2 * 4);
  L.h1 = o; o = align256(o + (size_t)hh * 2 * h2 * 2);
  L.c1 = o; o = align256(o + (size_t)hh * 4);
  L.h2 = o; o = align256(o + (size_t)hh * hh * 2);
  L.c2 = o; o = align256(o + (size_t)hh * 4);
  L.h3 = o; o = align256(o + (size_t)32 * hh * 2);
  L.c3 = o; o = align256(o + 8 * 4);
  L.total = o;
  return L;
}

void bf16_pack(const float* W1, const float* b1, const float* W2, const float* b2, const float* H1,
               const float* c1, const float* H2, const float* c2, const float* H3, const float* c3, int h1,
               int h2, int hh, unsigned char* dst) {
  const Bf16Layout L = bf16_layout(h1, h2, hh);
  std::memset(dst, 0, L.total);
  auto u16 = [&](size_t off) { return reinterpret_cast<unsigned short*>(dst + off); };
  auto f32 = [&](size_t off) { return reinterpret_cast<float*>(dst + off); };
  // encoder layer 1, A operand of 32x32x8: [W1 | b1 | 0][32 ft + l % 32][4 (l / 32) + e]
  for (int ft = 0; ft < h1 / 32; ++ft)
    for (int l = 0; l < 64; ++l)
      for (int e = 0; e < 4; ++e) {
        const int f = 32 * ft + l % 32, c = 4 * (l / 32) + e;
        u16(L.w1)[((size_t)ft * 64 + l) * 4 + e] = host_bf16(c < 6 ? W1[f * 6 + c] : (c == 6 ? b1[f] : 0.f));
      }
  // encoder layer 2, B operand of 32x32x16, reduction index permuted to layer 1's output layout
  const int CT = h2 / 128, KS2 = h1 / 16;
  for (int w = 0; w < 4; ++w)
    for (int ct = 0; ct < CT; ++ct)
      for (int s = 0; s < KS2; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int col = (w * CT + ct) * 32 + l % 32;
            const int f = perm_feature(s / 2, l / 32, 8 * (s % 2) + e);
            u16(L.w2)[(((size_t)(w * CT + ct) * KS2 + s) * 64 + l) * 8 + e] = host_bf16(W2[(size_t)col * h1 + f]);
          }
  std::memcpy(f32(L.b2), b2, sizeof(float) * h2);
  bf16_pack_head(H1, 2 * h2, hh, hh, u16(L.h1));
  std::memcpy(f32(L.c1), c1, sizeof(float) * hh);
  bf16_pack_head(H2, hh, hh, hh, u16(L.h2));
  std::memcpy(f32(L.c2), c2, sizeof(float) * hh);
  bf16_pack_head(H3, hh, 8, 32, u16(L.h3));
  std::memcpy(f32(L.c3), c3, sizeof(float) * 8);
}


// ---------------------------------------------------------------- FP8
// Encoder layer 1 in units of the activation scale of layer 2's input:
// bf16(W1 * inv), bf16(b1 * inv) (products in float32), A operand of 32x32x8.
void fp8_pack_w1(const float* W1, const float* b1, int h1, float inv, unsigned short* dst) {
  for (int ft = 0; ft < h1 / 32; ++ft)
    for (int l = 0; l < 64; ++l)
      for (int e = 0; e < 4; ++e) {
        const int f = 32 * ft + l % 32, c = 4 * (l / 32) + e;
        const float v = c < 6 ? W1[f * 6 + c] * inv : (c == 6 ? b1[f] * inv : 0.f);
        dst[((size_t)ft * 64 + l) * 4 + e] = host_bf16(v);
      }
}

Fp8Layout fp8_layout(int h1, int h2, int hh, bool head8) {
  Fp8Layout L{};
  const size_t hb = head8 ? 1 : 2;  // bytes per head weight
  size_t o = 0;
  L.w1 = o; o = align256(o + (size_t)h1 * 8 * 2);
  L.w2 = o; o = align256(o + (size_t)h2 * h1);
  L.b2 = o; o = align256(o + (size_t)h2 * 4);
  L.h1 = o; o = align256(o + (size_t)hh * 2 * h2 * hb);
  L.c1 = o; o = align256(o + (size_t)hh * 4);
  L.h2 = o; o = align256(o + (size_t)hh * hh * hb);
  L.c2 = o; o = align256(o + (size_t)hh * 4);
  L.h3 = o; o = align256(o + (size_t)32 * hh * 2);
  L.c3 = o; o = align256(o + 8 * 4);
  L.total = o;
  return L;
}

void fp8_pack(const float* W1, const float* b1, const float* W2, const float* b2, const float* H1, const float* c1,
              const float* H2, const float* c2, const float* H3, const float* c3, int h1, int h2, int hh, bool head8,
              unsigned char* dst, float* weight_scales) {
  const Fp8Layout L = fp8_layout(h1, h2, hh, head8);
  std::memset(dst, 0, L.total);
  auto u16 = [&](size_t off) { return reinterpret_cast<unsigned short*>(dst + off); };
  auto f32 = [&](size_t off) { return reinterpret_cast<float*>(dst + off); };
  // encoder layer 1 (bf16): unscaled until the activation scale is known
  fp8_pack_w1(W1, b1, h1, 1.f, u16(L.w1));
  const float s_w2 = std::fmax(amax_of(W2, (size_t)h2 * h1), 1e-30f) / 448.f;
  const float s_h1 = head8 ? std::fmax(amax_of(H1, (size_t)hh * 2 * h2), 1e-30f) / 448.f : 1.f;
  const float s_h2 = head8 ? std::fmax(amax_of(H2, (size_t)hh * hh), 1e-30f) / 448.f : 1.f;
  weight_scales[0] = s_w2;
  weight_scales[1] = s_h1;
  weight_scales[2] = s_h2;
  // encoder layer 2 (e4m3, B operand of 32x32x64), reduction index permuted to layer 1's output
  const int CT = h2 / 128, KS2 = h1 / 64;
  for (int w = 0; w < 4; ++w)
    for (int ct = 0; ct < CT; ++ct)
      for (int s = 0; s < KS2; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 32; ++e) {
            const int col = (w * CT + ct) * 32 + l % 32;
            const int f = perm_feature(2 * s + e / 16, l / 32, e % 16);
            dst[L.w2 + (((size_t)(w * CT + ct) * KS2 + s) * 64 + l) * 32 + e] = host_e4m3(W2[(size_t)col * h1 + f] / s_w2);
          }
  std::memcpy(f32(L.b2), b2, sizeof(float) * h2);
  // head layers 1-2 (e4m3, B operand): lane l holds H[32 ct + l % 32][64 s + 32 (l / 32) + e]
  auto pack8 = [&](const float* H, int in, int out, float sc, size_t at) {
    const int ks = in / 64;
    for (int ct = 0; ct < out / 32; ++ct)
      for (int s = 0; s < ks; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 32; ++e)
            dst[at + (((size_t)ct * ks + s) * 64 + l) * 32 + e] =
                host_e4m3(H[(size_t)(32 * ct + l % 32) * in + 64 * s + 32 * (l / 32) + e] / sc);
  };
  if (head8) {
    pack8(H1, 2 * h2, hh, s_h1, L.h1);
    pack8(H2, hh, hh, s_h2, L.h2);
  } else {
    bf16_pack_head(H1, 2 * h2, hh, hh, u16(L.h1));
    bf16_pack_head(H2, hh, hh, hh, u16(L.h2));
  }
  std::memcpy(f32(L.c1), c1, sizeof(float) * hh);
  std::memcpy(f32(L.c2), c2, sizeof(float) * hh);
  bf16_pack_head(H3, hh, 8, 32, u16(L.h3));  // head layer 3 (bf16, 8 outputs padded to 32 columns)
  std::memcpy(f32(L.c3), c3, sizeof(float) * 8);
}


}  // namespace locc
