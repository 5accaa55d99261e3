// TEST INFRASTRUCTURE: the binary16 stochastic-rounding store of the FP16 codec (common.h),
// compiled for the host against the emulated HIP headers, checked against the rounding rule
// written out directly: s = v * 2^14 is stored as its binary16 neighbour away from zero when
// (rnd >> 8) / 2^24 < frac, frac being the position of s between the neighbour toward zero and
// the one away from zero (exact in double), otherwise as the neighbour toward zero; magnitudes
// beyond the largest finite binary16 saturate to it.
#include "hip/hip_runtime.h"
#include "hip/hip_fp16.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

#include "common.h"

static unsigned short bits(__half h) {
  unsigned short u;
  std::memcpy(&u, &h, 2);
  return u;
}

static __half from_bits(unsigned short u) {
  __half h;
  std::memcpy(&h, &u, 2);
  return h;
}

// the rule, from the ordered binary16 values of the magnitude
static unsigned short reference(float v, unsigned rnd) {
  const float s = v * imb::F16_SCALE;
  const unsigned short sign = std::signbit(s) ? 0x8000 : 0;
  const double a = std::fabs((double)s);
  if (a >= 65504.0) return sign | 0x7BFF;
  // largest magnitude code whose value does not exceed a
  unsigned short lo = 0;
  for (int b = 14; b >= 0; --b) {
    const unsigned short t = lo | (unsigned short)(1u << b);
    if (t <= 0x7BFF && (double)__half2float(from_bits(t)) <= a) lo = t;
  }
  const double flo = __half2float(from_bits(lo));
  if (flo == a) return sign | lo;
  const double fhi = __half2float(from_bits((unsigned short)(lo + 1)));
  const double frac = (a - flo) / (fhi - flo);
  const double u = (double)(rnd >> 8) / 16777216.0;
  return sign | (u < frac ? (unsigned short)(lo + 1) : lo);
}

int main() {
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  long long n = 0, bad = 0;
  auto check = [&](float v, unsigned rnd) {
    __half got;
    imb::StoreF16::store_sr(&got, 0, v, rnd);
    const unsigned short want = reference(v, rnd);
    ++n;
    if (bits(got) != want && bad++ < 5)
      std::printf("v=%.9g rnd=%u got=%04x want=%04x\n", v, rnd, bits(got), want);
  };
  for (int k = 0; k < 300000; ++k) {  // magnitudes 1e-12 .. 10 (s up to 1.6e5), both signs
    const double mag = std::pow(10.0, -12.0 + 13.0 * U(g));
    check((float)(U(g) < 0.5 ? -mag : mag), (unsigned)g());
  }
  for (int k = 0; k < 100000; ++k) {  // binary16 values and their float neighbours
    const float f = __half2float(from_bits((unsigned short)(g() & 0x7BFF))) / imb::F16_SCALE;
    check(f, (unsigned)g());
    check(std::nextafter(f, 1.0f), (unsigned)g());
    check(-std::nextafter(f, 0.0f), (unsigned)g());
  }
  // the probability of rounding away equals frac for one value (exhaustive over rnd >> 19)
  const float v = 5.0e-4f;
  long long away = 0;
  for (unsigned r = 0; r < 8192; ++r) {
    __half h;
    imb::StoreF16::store_sr(&h, 0, v, r << 19);
    away += bits(h) != bits(__float2half_rz(v * imb::F16_SCALE));
  }
  const float s = v * imb::F16_SCALE;
  const double lo = __half2float(__float2half_rz(s));
  const double hi = __half2float(from_bits((unsigned short)(bits(__float2half_rz(s)) + 1)));
  const double frac = (s - lo) / (hi - lo);
  const bool prob_ok = std::fabs((double)away / 8192.0 - frac) <= 1.0 / 8192.0;
  std::printf("%lld cases, %lld differ; P(away) %.6f for frac %.6f\n", n, bad, away / 8192.0, frac);
  return bad == 0 && prob_ok ? 0 : 1;
}
