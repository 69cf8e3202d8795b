// Host-only tests of the weight packing (pack.cpp), built and run by
// tests/test_host_runtime.py under the address and undefined-behaviour
// sanitizers (which catch any write or read outside the packed buffers and
// the weight arrays):
//   * host_bf16 and host_e4m3 against brute force: the nearest representable
//     value by exact distance, ties to the even code, e4m3 saturating at 448;
//   * every packer on both compiled width sets, with distinct nonzero random
//     weights: the packed buffer holds each weight (rounded to the format it
//     is stored in) exactly once, the biases as float32, and zeros elsewhere
//     (a dropped, doubled or out-of-range entry changes the multiset).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "pack.h"

static int g_failures = 0;
#define EXPECT(cond)                                                          \
  do {                                                                        \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++g_failures;                                                           \
    }                                                                         \
  } while (0)

namespace {

float bits_to_float(uint32_t u) {
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint32_t float_to_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}
double bf16_value(unsigned short h) { return (double)bits_to_float((uint32_t)h << 16); }

// Nearest bf16 by exact distance between the two candidates around f, ties to the even code; the
// candidate past the largest finite value counts as 2^128 (where rounding overflows to infinity).
unsigned short brute_bf16(float f) {
  const uint32_t u = float_to_bits(f);
  if (std::isinf(f)) return (unsigned short)(u >> 16);
  const uint32_t sign = u & 0x80000000u, mag = u & 0x7fffffffu;
  const unsigned short lo = (unsigned short)(mag >> 16), hi = (unsigned short)(lo + 1);
  auto val = [](unsigned short h) { return h == 0x7f80 ? std::ldexp(1.0, 128) : bf16_value(h); };
  const double x = (double)bits_to_float(mag), dl = x - val(lo), dh = val(hi) - x;
  unsigned short r = (dl < dh || (dl == dh && (lo & 1) == 0)) ? lo : hi;
  return (unsigned short)(r | (sign >> 16));
}

double e4m3_value(int code) {  // code in [0, 0x7E]
  const int e = code >> 3, m = code & 7;
  return e == 0 ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, e - 7);
}

unsigned char brute_e4m3(float x) {
  if (std::isnan(x)) return 0x7F;
  const double a = std::fabs((double)x);
  int best = 0;
  double bd = INFINITY;
  for (int c = 0; c <= 0x7E; ++c) {
    const double d = std::fabs(a - e4m3_value(c));
    if (d < bd || (d == bd && (c & 1) == 0)) {
      bd = d;
      best = c;
    }
  }
  return (unsigned char)(best | (std::signbit(x) ? 0x80 : 0));
}

void test_conversions() {
  std::mt19937 rng(12345);
  int n = 0;
  auto check_bf16 = [&](float f) {
    if (std::isnan(f)) {
      EXPECT(std::isnan(bf16_value(locc::host_bf16(f))));
      return;
    }
    if (locc::host_bf16(f) != brute_bf16(f)) {
      std::fprintf(stderr, "bf16(%a): %04x, brute force %04x\n", f, locc::host_bf16(f), brute_bf16(f));
      ++g_failures;
    }
    ++n;
  };
  for (int k = 0; k < 200000; ++k) check_bf16(bits_to_float(rng()));
  for (uint32_t h = 0; h < 0x7f80; h += 7) {  // exact ties and their neighbours
    const uint32_t t = (h << 16) | 0x8000u;
    for (uint32_t d : {0u, 1u, 0xffffffffu}) check_bf16(bits_to_float(t + d));
  }
  check_bf16(INFINITY);
  check_bf16(-INFINITY);
  check_bf16(0.f);
  check_bf16(-0.f);
  check_bf16(NAN);
  EXPECT(locc::host_bf16(bits_to_float(0x7f7fffffu)) == 0x7f80);  // the largest float rounds to infinity

  auto check_e4m3 = [&](float f) {
    if (locc::host_e4m3(f) != brute_e4m3(f)) {
      std::fprintf(stderr, "e4m3(%a): %02x, brute force %02x\n", f, locc::host_e4m3(f), brute_e4m3(f));
      ++g_failures;
    }
  };
  std::uniform_real_distribution<float> mant(1.f, 2.f);
  for (int k = 0; k < 100000; ++k) check_e4m3(std::ldexp(mant(rng), (int)(rng() % 24) - 14) * (rng() & 1 ? 1 : -1));
  for (int c = 0; c < 0x7E; ++c) {  // every midpoint between neighbouring codes, and just either side of it
    const double mid = 0.5 * (e4m3_value(c) + e4m3_value(c + 1));
    for (float f : {(float)mid, std::nextafter((float)mid, 0.f), std::nextafter((float)mid, 1e9f)}) {
      check_e4m3(f);
      check_e4m3(-f);
    }
    check_e4m3((float)e4m3_value(c));
  }
  for (float f : {448.f, 449.f, 463.9f, 464.f, 500.f, 1e30f, INFINITY, -INFINITY, 0.f, -0.f, NAN}) check_e4m3(f);
  EXPECT(locc::host_e4m3(1e30f) == 0x7E && locc::host_e4m3(-INFINITY) == 0xFE);
  std::printf("conversions: %d bf16 cases against brute force\n", n);
}

struct Net {
  int h1, h2, hh;
  std::vector<float> W1, b1, W2, b2, H1, c1, H2, c2, H3, c3;
};

Net make_net(int h1, int h2, int hh, unsigned seed) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<float> mag(0.05f, 1.f);
  // distinct nonzero values: a random magnitude with a unique low-order tag in its mantissa
  uint32_t tag = 1;
  auto fill = [&](std::vector<float>& v, size_t n) {
    v.resize(n);
    for (float& x : v) {
      uint32_t u = float_to_bits(mag(rng)) & ~0x3ffffu;
      u |= (tag++ & 0x3ffffu);
      x = bits_to_float(u) * (rng() & 1 ? 1.f : -1.f);
    }
  };
  Net n{h1, h2, hh, {}, {}, {}, {}, {}, {}, {}, {}, {}, {}};
  fill(n.W1, (size_t)h1 * 6);
  fill(n.b1, h1);
  fill(n.W2, (size_t)h2 * h1);
  fill(n.b2, h2);
  fill(n.H1, (size_t)hh * 2 * h2);
  fill(n.c1, hh);
  fill(n.H2, (size_t)hh * hh);
  fill(n.c2, hh);
  fill(n.H3, (size_t)8 * hh);
  fill(n.c3, 8);
  return n;
}

template <class T>
bool same_multiset(std::vector<T> a, std::vector<T> b) {
  std::sort(a.begin(), a.end());
  std::sort(b.begin(), b.end());
  return a == b;
}

void test_fp32(const Net& n) {
  const size_t total = locc::fp32_pack_floats(n.h1, n.h2, n.hh);
  std::vector<float> dst(total, 12345.f);
  locc::fp32_pack(n.W1.data(), n.b1.data(), n.W2.data(), n.b2.data(), n.H1.data(), n.c1.data(), n.H2.data(),
                  n.c2.data(), n.H3.data(), n.c3.data(), n.h1, n.h2, n.hh, dst.data());
  std::vector<float> want, got;
  for (const auto* v : {&n.W1, &n.b1, &n.W2, &n.b2, &n.H1, &n.c1, &n.H2, &n.c2, &n.H3, &n.c3})
    want.insert(want.end(), v->begin(), v->end());
  for (float x : dst)
    if (x != 0.f) got.push_back(x);
  EXPECT(same_multiset(got, want));
}

void test_bf16(const Net& n) {
  const locc::Bf16Layout L = locc::bf16_layout(n.h1, n.h2, n.hh);
  std::vector<unsigned char> dst(L.total, 0xAB);
  locc::bf16_pack(n.W1.data(), n.b1.data(), n.W2.data(), n.b2.data(), n.H1.data(), n.c1.data(), n.H2.data(),
                  n.c2.data(), n.H3.data(), n.c3.data(), n.h1, n.h2, n.hh, dst.data());
  auto u16 = [&](size_t off, size_t count) {
    std::vector<unsigned short> v(count);
    std::memcpy(v.data(), dst.data() + off, 2 * count);
    v.erase(std::remove(v.begin(), v.end(), (unsigned short)0), v.end());
    return v;
  };
  auto f32 = [&](size_t off, size_t count) {
    std::vector<float> v(count);
    std::memcpy(v.data(), dst.data() + off, 4 * count);
    return v;
  };
  auto bf = [](const std::vector<float>& a, const std::vector<float>* b = nullptr) {
    std::vector<unsigned short> v;
    for (float x : a) v.push_back(locc::host_bf16(x));
    if (b)
      for (float x : *b) v.push_back(locc::host_bf16(x));
    return v;
  };
  EXPECT(same_multiset(u16(L.w1, (L.w2 - L.w1) / 2), bf(n.W1, &n.b1)));  // b1 rides in layer 1's 7th input
  EXPECT(same_multiset(u16(L.w2, (L.b2 - L.w2) / 2), bf(n.W2)));
  EXPECT(f32(L.b2, n.h2) == n.b2);
  EXPECT(same_multiset(u16(L.h1, (L.c1 - L.h1) / 2), bf(n.H1)));
  EXPECT(f32(L.c1, n.hh) == n.c1);
  EXPECT(same_multiset(u16(L.h2, (L.c2 - L.h2) / 2), bf(n.H2)));
  EXPECT(f32(L.c2, n.hh) == n.c2);
  EXPECT(same_multiset(u16(L.h3, (L.c3 - L.h3) / 2), bf(n.H3)));
  EXPECT(f32(L.c3, 8) == n.c3);
}

void test_fp8(const Net& n, bool head8) {
  const locc::Fp8Layout L = locc::fp8_layout(n.h1, n.h2, n.hh, head8);
  std::vector<unsigned char> dst(L.total, 0xAB);
  float sc[3] = {0, 0, 0};
  locc::fp8_pack(n.W1.data(), n.b1.data(), n.W2.data(), n.b2.data(), n.H1.data(), n.c1.data(), n.H2.data(),
                 n.c2.data(), n.H3.data(), n.c3.data(), n.h1, n.h2, n.hh, head8, dst.data(), sc);
  auto amax = [](const std::vector<float>& v) {
    float m = 0.f;
    for (float x : v) m = std::fmax(m, std::fabs(x));
    return m;
  };
  EXPECT(sc[0] == amax(n.W2) / 448.f);
  EXPECT(head8 ? sc[1] == amax(n.H1) / 448.f && sc[2] == amax(n.H2) / 448.f : sc[1] == 1.f && sc[2] == 1.f);
  auto bytes = [&](size_t off, size_t count) {
    std::vector<unsigned char> v(dst.begin() + off, dst.begin() + off + count);
    v.erase(std::remove(v.begin(), v.end(), (unsigned char)0), v.end());
    return v;
  };
  auto e4 = [](const std::vector<float>& a, float s) {
    std::vector<unsigned char> v;
    for (float x : a) {
      const unsigned char c = locc::host_e4m3(x / s);
      if (c != 0) v.push_back(c);
    }
    return v;
  };
  auto u16 = [&](size_t off, size_t count) {
    std::vector<unsigned short> v(count);
    std::memcpy(v.data(), dst.data() + off, 2 * count);
    v.erase(std::remove(v.begin(), v.end(), (unsigned short)0), v.end());
    return v;
  };
  auto bf = [](const std::vector<float>& a) {
    std::vector<unsigned short> v;
    for (float x : a) v.push_back(locc::host_bf16(x));
    return v;
  };
  EXPECT(same_multiset(bytes(L.w2, (size_t)n.h2 * n.h1), e4(n.W2, sc[0])));
  if (head8) {
    EXPECT(same_multiset(bytes(L.h1, (size_t)n.hh * 2 * n.h2), e4(n.H1, sc[1])));
    EXPECT(same_multiset(bytes(L.h2, (size_t)n.hh * n.hh), e4(n.H2, sc[2])));
  } else {
    EXPECT(same_multiset(u16(L.h1, (size_t)n.hh * 2 * n.h2), bf(n.H1)));
    EXPECT(same_multiset(u16(L.h2, (size_t)n.hh * n.hh), bf(n.H2)));
  }
  EXPECT(same_multiset(u16(L.h3, (L.c3 - L.h3) / 2), bf(n.H3)));
  std::vector<float> b2(n.h2);
  std::memcpy(b2.data(), dst.data() + L.b2, 4 * n.h2);
  EXPECT(b2 == n.b2);
  // layer 1 in units of an activation scale: bf16(W1 * inv), bf16(b1 * inv)
  const float inv = 1.f / 0.37f;
  std::vector<unsigned short> w1((size_t)n.h1 * 8, 0xABCD);
  locc::fp8_pack_w1(n.W1.data(), n.b1.data(), n.h1, inv, w1.data());
  std::vector<float> sw;
  for (float x : n.W1) sw.push_back(x * inv);
  for (float x : n.b1) sw.push_back(x * inv);
  w1.erase(std::remove(w1.begin(), w1.end(), (unsigned short)0), w1.end());
  EXPECT(same_multiset(w1, bf(sw)));
}

}  // namespace

int main() {
  test_conversions();
  const int widths[2][3] = {{64, 128, 256}, {128, 256, 512}};
  for (const auto& w : widths) {
    const Net n = make_net(w[0], w[1], w[2], 7u + (unsigned)w[0]);
    test_fp32(n);
    test_bf16(n);
    test_fp8(n, true);
    test_fp8(n, false);
  }
  if (g_failures) {
    std::fprintf(stderr, "%d failure(s)\n", g_failures);
    return 1;
  }
  std::printf("pack: all tests passed\n");
  return 0;
}
