#pragma once
#include <cstdint>
#include <cstring>
#include <cmath>
struct __half { uint16_t b; };
inline float __half2float(__half h) {
  const uint32_t s = (h.b >> 15) & 1, e = (h.b >> 10) & 31, m = h.b & 1023;
  float v;
  if (e == 0) v = std::ldexp((float)m, -24);
  else if (e == 31) v = m ? NAN : INFINITY;
  else v = std::ldexp((float)(m | 1024), (int)e - 25);
  return s ? -v : v;
}
// exact conversion helpers: round to nearest even / toward zero
inline __half emu_f2h(float f, bool rz) {
  __half h;
  if (std::isnan(f)) { h.b = 0x7E00; return h; }
  const uint16_t sign = std::signbit(f) ? 0x8000 : 0;
  double a = std::fabs((double)f);
  if (a == 0.0) { h.b = sign; return h; }
  // scaled integer significand at the binary16 grid spacing of a
  int ex; std::frexp(a, &ex);            // a = m * 2^ex, m in [0.5, 1)
  int e = ex - 1;                        // a in [2^e, 2^(e+1))
  if (e < -14) e = -14;                  // subnormal spacing
  const double ulp = std::ldexp(1.0, e - 10);
  double q = a / ulp;                    // exact (power-of-two scaling)
  double qi = rz ? std::floor(q) : std::nearbyint(q);  // default mode: nearest even
  double v = qi * ulp;
  if (v >= 65536.0 - 16.0 && !rz && v > 65504.0) { h.b = sign | 0x7C00; return h; }
  if (v > 65504.0) v = 65504.0;
  // encode v
  if (v < std::ldexp(1.0, -14)) { h.b = sign | (uint16_t)(v / std::ldexp(1.0, -24)); return h; }
  int ev; double mv = std::frexp(v, &ev);  // v = mv * 2^ev
  const int E = ev - 1 + 15;
  const uint16_t M = (uint16_t)((mv * 2.0 - 1.0) * 1024.0);
  h.b = sign | (uint16_t)(E << 10) | M;
  return h;
}
inline __half __float2half_rn(float f) { return emu_f2h(f, false); }
inline __half __float2half_rz(float f) { return emu_f2h(f, true); }
inline unsigned short __half_as_ushort(__half h) { return h.b; }
inline __half __ushort_as_half(unsigned short u) { __half h; h.b = u; return h; }
