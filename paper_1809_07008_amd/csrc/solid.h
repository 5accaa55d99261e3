// solid.h -- solid ratio of a lattice cell covered by a disk (Sec. 2.2, Fig. 3a) and its
// derivative with respect to the disk centre.
//
// The paper defines eps as the covered part of the cell divided by the cell size and estimates
// it by cell decomposition; here it is the exact area of disk (radius r, centre at the origin)
// intersected with the unit cell [dx - 1/2, dx + 1/2] x [dy - 1/2, dy + 1/2].
//
// Formulation used on the GPU (well conditioned in FP32):
//   eps = I(y1) - I(y0),   I(y) = int_{x0}^{x1} clamp(y, -s(x), s(x)) dx,  s(x) = sqrt(r^2 - x^2),
// because clamp(y1, -s, s) - clamp(y0, -s, s) is the part of the vertical chord inside [y0, y1].
// For |y| < r the clamp equals y where |x| < w = s(y) and sign(y) s(x) where w <= |x| <= r, so
// I(y) is one rectangle plus at most two pieces of int s dx, each evaluated from the difference
// of the end points (no subtraction of two large primitives).
//
// Derivative (ADJOINT): moving the centre by +h shifts the cell by -h in disk coordinates, so
//   d eps / dX = L(x0) - L(x1),  d eps / dY = M(y0) - M(y1),
// with L(x) the chord length inside [y0, y1] at abscissa x and M(y) the chord length inside
// [x0, x1] at ordinate y.  eps is C1 in the centre.
#pragma once

#include <hip/hip_runtime.h>

namespace imb {

template <class T>
__host__ __device__ inline T half_chord(T r, T x) {  // sqrt(r^2 - x^2), well conditioned near |x| = r
  const T a = fabs(x);
  return a >= r ? T(0) : sqrt((r - a) * (r + a));
}

// x - sin x for 0 <= x <= pi: Taylor series below 1 (no cancellation), direct above.
template <class T>
__host__ __device__ inline T segment_excess(T x) {
  if (x < T(1)) {
    const T x2 = x * x;
    T p = T(1.0 / 51090942171709440000.0);
    p = T(1.0 / 121645100408832000.0) - x2 * p;
    p = T(1.0 / 355687428096000.0) - x2 * p;
    p = T(1.0 / 1307674368000.0) - x2 * p;
    p = T(1.0 / 6227020800.0) - x2 * p;
    p = T(1.0 / 39916800.0) - x2 * p;
    p = T(1.0 / 362880.0) - x2 * p;
    p = T(1.0 / 5040.0) - x2 * p;
    p = T(1.0 / 120.0) - x2 * p;
    p = T(1.0 / 6.0) - x2 * p;
    return x * x2 * p;
  }
  return x - sin(x);
}

// int_a^b sqrt(r^2 - x^2) dx for -r <= a <= b <= r, as the trapezoid under the chord plus the
// circular segment between chord and arc:
//   (b - a)(s_a + s_b) / 2 + r^2 (phi - sin phi) / 2,
// phi = theta(b) - theta(a) the angle the arc subtends, theta(x) = asin(x / r), from
//   r^2 sin phi = b s_a - a s_b  (= r^2 (b - a)(b + a) / (b s_a + a s_b) when a b > 0),
//   r^2 cos phi = s_a s_b + a b.
// Both terms are non-negative, so nothing cancels.
template <class T>
__host__ __device__ inline T semi_integral(T r, T a, T b) {
  if (!(b > a)) return T(0);
  const T sa = half_chord(r, a), sb = half_chord(r, b);
  T sn;
  if (a * b > T(0)) {
    sn = r * r * ((b - a) * (b + a)) / (b * sa + a * sb);
  } else {
    sn = b * sa - a * sb;
  }
  const T cs = sa * sb + a * b;
  const T phi = atan2(sn, cs);
  return T(0.5) * ((b - a) * (sa + sb) + r * r * segment_excess(phi));
}

template <class T>
__host__ __device__ inline T clamped_chord_integral(T r, T x0, T x1, T y) {
  const T xa = fmax(x0, -r), xb = fmin(x1, r);
  if (!(xb > xa)) return T(0);
  if (y >= r) return semi_integral<T>(r, xa, xb);
  if (y <= -r) return -semi_integral<T>(r, xa, xb);
  const T w = half_chord(r, y);
  const T lc = fmax(T(0), fmin(xb, w) - fmax(xa, -w));
  const T outer = semi_integral<T>(r, xa, fmin(xb, -w)) + semi_integral<T>(r, fmax(xa, w), xb);
  return y * lc + (y > T(0) ? outer : (y < T(0) ? -outer : T(0)));
}

// eps of the unit cell centred at (dx, dy) relative to the disk centre.  The exact-area branch
// is a separate (non-inlined) function: it runs only for cut cells and keeps the caller's
// register budget small.
template <class T>
__host__ __device__ __noinline__ T cut_cell_fraction(T r, T x0, T x1, T y0, T y1) {
  const T e = clamped_chord_integral(r, x0, x1, y1) - clamped_chord_integral(r, x0, x1, y0);
  return fmin(T(1), fmax(T(0), e));
}

template <class T>
__host__ __device__ inline T solid_fraction(T r, T dx, T dy) {
  const T x0 = dx - T(0.5), x1 = dx + T(0.5), y0 = dy - T(0.5), y1 = dy + T(0.5);
  // outside: the point of the cell nearest to the centre is not inside the disk
  const T nx = x0 > T(0) ? x0 : (x1 < T(0) ? x1 : T(0));
  const T ny = y0 > T(0) ? y0 : (y1 < T(0) ? y1 : T(0));
  if (nx * nx + ny * ny >= r * r) return T(0);
  // inside: the farthest corner is inside the (convex) disk
  const T fx = fabs(x0) > fabs(x1) ? fabs(x0) : fabs(x1);
  const T fy = fabs(y0) > fabs(y1) ? fabs(y0) : fabs(y1);
  if (fx * fx + fy * fy <= r * r) return T(1);
  return cut_cell_fraction(r, x0, x1, y0, y1);
}

template <class T>
__host__ __device__ inline T chord_in(T r, T c, T lo, T hi) {  // chord at coordinate c clipped to [lo, hi]
  const T s = half_chord(r, c);
  return fmax(T(0), fmin(hi, s) - fmax(lo, -s));
}

// (d eps / dX, d eps / dY) for the same cell; zero outside a partially covered cell.
template <class T>
__host__ __device__ inline void solid_fraction_grad(T r, T dx, T dy, T* gx, T* gy) {
  const T x0 = dx - T(0.5), x1 = dx + T(0.5), y0 = dy - T(0.5), y1 = dy + T(0.5);
  *gx = chord_in(r, x0, y0, y1) - chord_in(r, x1, y0, y1);
  *gy = chord_in(r, y0, x0, x1) - chord_in(r, y1, x0, x1);
}

}  // namespace imb
