// solid.h -- solid ratio of a lattice cell covered by a disk (Sec. 2.2, Fig. 3a) and its
// derivative with respect to the disk centre.
//
// The paper defines eps as the covered part of the cell divided by the cell size and estimates
// it by cell decomposition; here it is the exact area of disk (radius r, centre at the origin)
// intersected with the unit cell [dx - 1/2, dx + 1/2] x [dy - 1/2, dy + 1/2].
//
// A cut cell's area is the convex polygon of its inside corners and edge crossings plus the
// circular segments cut off by the chords (see cut_cell_fraction); cells entirely inside or
// outside are 1 or 0 exactly.
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

// ---------------------------------------------------------------- cut cells
// Area of a cut cell as the convex polygon whose vertices are the cell corners inside the disk
// and the points where the circle crosses the cell edges (walked counter-clockwise), plus one
// circular segment r^2 (phi - sin phi) / 2 for every arc between an exit and the next entry.
// Vertices are kept in cell-local coordinates (u, v) in [0, 1]^2 so the shoelace sum has no
// cancellation; a crossing is located from the nearer same-sign corner through the corner's
// power r^2 - x^2 - y^2, computed with error-free products, so crossings near a corner keep
// full relative precision.

// Power r^2 - (dx + sx/2)^2 - (dy + sy/2)^2 of the cell corner (sx, sy = -1 or +1) of the unit
// cell centred at (dx, dy): expanded as r^2 - dx^2 - dy^2 - sx dx - sy dy - 1/2, every term exact
// (error-free squares) and summed with error-free additions, so the corner is exactly
// (dx + sx/2, dy + sy/2) even where that coordinate has no representation in T, and the power
// has full relative precision near the circle.
template <class T>
__host__ __device__ inline void sum_exact(T& s, T& c, T v) {  // s + c += v (TwoSum)
  const T t = s + v, bp = t - s;
  c += (s - (t - bp)) + (v - bp);
  s = t;
}
template <class T>
__host__ __device__ inline T corner_power(T r, T dx, T dy, T sx, T sy) {
  const T hr = r * r, lr = fma(r, r, -hr);
  const T hx = dx * dx, lx = fma(dx, dx, -hx);
  const T hy = dy * dy, ly = fma(dy, dy, -hy);
  T s = hr, c = T(0);
  sum_exact(s, c, -hx);
  sum_exact(s, c, -hy);
  sum_exact(s, c, -(sx * dx));
  sum_exact(s, c, -(sy * dy));
  sum_exact(s, c, T(-0.5));
  return s + (((c + lr) - lx) - ly);
}

// Offset, from edge end e0, of the crossing at coordinate cc (cc = +-h) on an edge running from
// e0 to e0 + 1 whose end points have powers p0 and p1.  The end point with the sign of cc gives
// cc - e = (cc^2 - e^2) / (cc + e) = power(e) / (cc + e), with no cancellation.
template <class T>
__host__ __device__ inline T crossing_offset(T cc, T e0, T p0, T p1) {
  return cc > T(0) ? T(1) + p1 / (cc + (e0 + T(1))) : p0 / (cc + e0);
}

template <class T>
struct AreaWalk {
  T r;
  T u0, v0;          // first vertex
  T pu, pv;          // previous vertex
  int first_kind, prev_kind;  // 0 corner, 1 entry, 2 exit, -1 none yet
  T twice_area;      // shoelace sum
  T seg;             // circular segments
  T cx, cy;          // disk centre in cell coordinates
  __host__ __device__ void segment(T au, T av, T bu, T bv) {
    // arc counter-clockwise from exit a to entry b
    const T du = bu - au, dv = bv - av;
    const T c = sqrt(du * du + dv * dv);
    const T t = c / (T(2) * r);
    T phi;  // the smaller angle between the radii to a and b
    if (t < T(0.7)) {
      phi = T(2) * asin(t);
    } else {  // near a diameter asin loses accuracy; use the radius vectors
      const T ax = au - cx, ay = av - cy, bx = bu - cx, by = bv - cy;
      phi = atan2(fabs(ax * by - ay * bx), ax * bx + ay * by);
    }
    // minor arc when the centre lies left of the chord a -> b
    const T side = du * (cy - av) - dv * (cx - au);
    T ex = segment_excess(phi);
    if (side < T(0)) ex = T(6.283185307179586476925) - phi + sin(phi);
    seg += T(0.5) * r * r * ex;
  }
  __host__ __device__ void add(T u, T v, int kind) {
    if (prev_kind < 0) {
      u0 = u; v0 = v; first_kind = kind;
    } else {
      twice_area += pu * v - u * pv;
      if (prev_kind == 2 && kind == 1) segment(pu, pv, u, v);
    }
    pu = u; pv = v; prev_kind = kind;
  }
  __host__ __device__ T finish() {
    if (prev_kind < 0) return T(0);
    twice_area += pu * v0 - u0 * pv;
    if (prev_kind == 2 && first_kind == 1) segment(pu, pv, u0, v0);
    return T(0.5) * twice_area + seg;
  }
};

// The crossings of one edge of the walk, from the powers ps, pe of its start and end corners:
// an edge running from inside to outside holds exactly one exit, from outside to inside one
// entry, inside to inside none, outside to outside none or an entry and an exit (the circle
// dips into it).  So the walk's vertices alternate consistently even where a corner lies
// within rounding of the circle and the half-chord test alone would disagree with the corner's
// power.  cc_in, cc_out: edge coordinates of the entry and exit points of the edge's line
// (+-h); the offset of a crossing runs from the edge's lower end `low` (power plow) to its
// upper end (power phigh) and is clamped to the edge; `fixed` is the other cell coordinate.
template <class T>
__host__ __device__ inline void edge_crossings(AreaWalk<T>& w, T ps, T pe, T plow, T phigh,
                                               bool line_cut, T cc_in, T cc_out, T low, T high,
                                               T fixed, bool horizontal) {
  const bool si = ps >= T(0), ei = pe >= T(0);
  auto put = [&](T cc, int kind) {
    const T off = fmin(T(1), fmax(T(0), crossing_offset(cc, low, plow, phigh)));
    if (horizontal) w.add(off, fixed, kind);
    else w.add(fixed, off, kind);
  };
  if (!si && ei) {
    put(cc_in, 1);
  } else if (si && !ei) {
    put(cc_out, 2);
  } else if (!si && !ei && line_cut && fmin(cc_in, cc_out) > low && fmax(cc_in, cc_out) < high) {
    put(cc_in, 1);
    put(cc_out, 2);
  }
}

template <class T>
__host__ __device__ __noinline__ T cut_cell_fraction(T r, T dx, T dy) {
  // edges (rounded; they only locate the crossings, whose offsets come from the exact corner
  // powers) and corner powers, counter-clockwise from (x0, y0)
  const T x0 = dx - T(0.5), x1 = dx + T(0.5), y0 = dy - T(0.5), y1 = dy + T(0.5);
  const T p00 = corner_power(r, dx, dy, T(-1), T(-1)), p10 = corner_power(r, dx, dy, T(1), T(-1));
  const T p11 = corner_power(r, dx, dy, T(1), T(1)), p01 = corner_power(r, dx, dy, T(-1), T(1));
  AreaWalk<T> w;
  w.r = r; w.prev_kind = -1; w.first_kind = -1; w.twice_area = T(0); w.seg = T(0);
  w.u0 = w.v0 = w.pu = w.pv = T(0);
  w.cx = -x0; w.cy = -y0;
  // bottom edge: (x0, y0) -> (x1, y0), u increasing; entry at x = -h, exit at +h
  if (p00 >= T(0)) w.add(T(0), T(0), 0);
  {
    const T h = half_chord(r, y0);
    edge_crossings(w, p00, p10, p00, p10, fabs(y0) < r, -h, h, x0, x1, T(0), true);
  }
  // right edge: (x1, y0) -> (x1, y1), v increasing; entry at y = -h, exit at +h
  if (p10 >= T(0)) w.add(T(1), T(0), 0);
  {
    const T h = half_chord(r, x1);
    edge_crossings(w, p10, p11, p10, p11, fabs(x1) < r, -h, h, y0, y1, T(1), false);
  }
  // top edge: (x1, y1) -> (x0, y1), u decreasing; entry at x = +h, exit at -h
  if (p11 >= T(0)) w.add(T(1), T(1), 0);
  {
    const T h = half_chord(r, y1);
    edge_crossings(w, p11, p01, p01, p11, fabs(y1) < r, h, -h, x0, x1, T(1), true);
  }
  // left edge: (x0, y1) -> (x0, y0), v decreasing; entry at y = +h, exit at -h
  if (p01 >= T(0)) w.add(T(0), T(1), 0);
  {
    const T h = half_chord(r, x0);
    edge_crossings(w, p01, p00, p00, p01, fabs(x0) < r, h, -h, y0, y1, T(0), false);
  }
  T e;
  if (w.prev_kind < 0) {
    // no corner inside and no crossing: the disk lies inside the cell
    e = T(3.14159265358979323846) * r * r;
  } else {
    e = w.finish();
  }
  return fmin(T(1), fmax(T(0), e));
}

// Single precision, the common cut (a disk of radius >= 2 whose circle crosses the cell's
// boundary exactly twice): without branches, from the corners' sides of the circle.  The
// corners inside form one run; the entry lies on the edge that arrives at its first corner, the
// exit on the edge that leaves its last.  In cell coordinates the bottom and left edges add
// nothing to the shoelace sum, the right and top edges their inside lengths, the chord from
// exit to entry its cross product; the circular segment beyond that chord is
// r^2 (phi - sin phi) / 2 with phi - sin phi = 4 t^3 sum_k C(2k, k) 4^-k t^(2k) / (2k + 3),
// t = chord / 2r (the series of 4 int_0^t s^2 (1 - s^2)^(-1/2) ds), five terms for t <= 1/4.
// Returns false (and the caller takes the exact walk) for a corner within rounding of the
// circle, a disk reaching an edge whose both ends lie outside it, a smaller disk or a longer
// chord.
__host__ __device__ inline bool one_arc_fraction(float r, float dx, float dy, float* eps) {
  if (!(r >= 2.0f)) return false;
  const float x0 = dx - 0.5f, x1 = dx + 0.5f, y0 = dy - 0.5f, y1 = dy + 0.5f;
  const float rr = r * r;
  // corner powers, counter-clockwise from (x0, y0); their rounding stays below tau
  const float q0 = rr - (x0 * x0 + y0 * y0), q1 = rr - (x1 * x1 + y0 * y0);
  const float q2 = rr - (x1 * x1 + y1 * y1), q3 = rr - (x0 * x0 + y1 * y1);
  const float tau = 1e-6f * (r + 1.0f) * (r + 1.0f);
  if (fabsf(q0) <= tau || fabsf(q1) <= tau || fabsf(q2) <= tau || fabsf(q3) <= tau) return false;
  const bool in0 = q0 > 0.0f, in1 = q1 > 0.0f, in2 = q2 > 0.0f, in3 = q3 > 0.0f;
  // edge e runs from corner e to corner e + 1: its line coordinate l_e and the parameter
  // s = base_e - h (entry) or base_e + h (exit) of its crossings, h the half chord at l_e
  auto chord = [&](float l) {
    const float a = fabsf(l);
    return a < r ? sqrtf((r - a) * (r + a)) : -1.0f;
  };
  const float h0 = chord(y0), h1 = chord(x1), h2 = chord(y1), h3 = chord(x0);
  const float b0 = -x0, b1 = -y0, b2 = x1, b3 = y1;  // an edge's crossings: s = b -+ h
  // an edge with both ends outside must not meet the disk
  auto dips = [&](bool a, bool b, float h, float base) {
    return !a && !b && h >= 0.0f && base + h > 0.0f && base - h < 1.0f;
  };
  if (dips(in0, in1, h0, b0) || dips(in1, in2, h1, b1) || dips(in2, in3, h2, b2) ||
      dips(in3, in0, h3, b3))
    return false;
  const int nin = (!in0 && in1) + (!in1 && in2) + (!in2 && in3) + (!in3 && in0);
  if (nin != 1) return false;  // with one entry there is one exit
  // entry edge: outside start, inside end; exit edge: inside start, outside end
  const int ent = (!in0 && in1) ? 0 : ((!in1 && in2) ? 1 : ((!in2 && in3) ? 2 : 3));
  const int ext = (in0 && !in1) ? 0 : ((in1 && !in2) ? 1 : ((in2 && !in3) ? 2 : 3));
  const float he = ent == 0 ? h0 : (ent == 1 ? h1 : (ent == 2 ? h2 : h3));
  const float hx = ext == 0 ? h0 : (ext == 1 ? h1 : (ext == 2 ? h2 : h3));
  if (he < 0.0f || hx < 0.0f) return false;
  // The crossings' parameters from the exact power P of the nearer corner, which lies outside:
  // the entry edge's start corner, s = P / (c - h), and the exit edge's end corner,
  // s = 1 + P / (h + d) (c = x0, y0, -x1, -y1 and d = x1, y1, -x0, -y0 by edge), as the
  // walk's crossing offsets, so a crossing near a corner keeps full relative precision.
  // Corner k is at (x0 or x1, y0 or y1) with signs (-,-), (+,-), (+,+), (-,+).
  const int ke = ent, kx = (ext + 1) & 3;
  const float pe = corner_power(r, dx, dy, (ke == 1 || ke == 2) ? 1.0f : -1.0f,
                                ke >= 2 ? 1.0f : -1.0f);
  const float px = corner_power(r, dx, dy, (kx == 1 || kx == 2) ? 1.0f : -1.0f,
                                kx >= 2 ? 1.0f : -1.0f);
  const float ce = ent == 0 ? x0 : (ent == 1 ? y0 : (ent == 2 ? -x1 : -y1));
  const float cx = ext == 0 ? x1 : (ext == 1 ? y1 : (ext == 2 ? -x0 : -y0));
  const float se = fminf(1.0f, fmaxf(0.0f, pe / (ce - he)));
  const float sx = fminf(1.0f, fmaxf(0.0f, 1.0f + px / (hx + cx)));
  // the points in cell coordinates: edge 0 (s, 0), 1 (1, s), 2 (1 - s, 1), 3 (0, 1 - s)
  const float eu = ent == 0 ? se : (ent == 1 ? 1.0f : (ent == 2 ? 1.0f - se : 0.0f));
  const float ev = ent == 0 ? 0.0f : (ent == 1 ? se : (ent == 2 ? 1.0f : 1.0f - se));
  const float xu = ext == 0 ? sx : (ext == 1 ? 1.0f : (ext == 2 ? 1.0f - sx : 0.0f));
  const float xv = ext == 0 ? 0.0f : (ext == 1 ? sx : (ext == 2 ? 1.0f : 1.0f - sx));
  // inside lengths of the right and top edges
  const float len1 = in1 && in2 ? 1.0f : (in1 ? sx : (in2 ? 1.0f - se : 0.0f));
  const float len2 = in2 && in3 ? 1.0f : (in2 ? sx : (in3 ? 1.0f - se : 0.0f));
  const float twice = len1 + len2 + (xu * ev - eu * xv);
  const float du = eu - xu, dv = ev - xv;
  const float t2 = (du * du + dv * dv) / (4.0f * rr);
  if (t2 > 0.0625f) return false;
  const float t = sqrtf(t2);
  const float series =
      4.0f / 3.0f +
      t2 * (2.0f / 5.0f + t2 * (3.0f / 14.0f + t2 * (5.0f / 36.0f + t2 * (35.0f / 352.0f))));
  *eps = fminf(1.0f, fmaxf(0.0f, 0.5f * twice + 0.5f * rr * t * t2 * series));
  return true;
}

// eps of the unit cell centred at (dx, dy) relative to the disk centre.  The cut-cell branch is
// a separate (non-inlined) function: it runs only for cut cells and keeps the caller's register
// budget small.
// Whether the unit cell centred at (dx, dy) from the centre overlaps the disk of radius r: the
// point of the cell nearest to the centre is strictly inside.  Every kernel decides "covered"
// with exactly this test.
template <class T>
__host__ __device__ inline bool covers_cell(T r, T dx, T dy) {
  const T x0 = dx - T(0.5), x1 = dx + T(0.5), y0 = dy - T(0.5), y1 = dy + T(0.5);
  const T nx = x0 > T(0) ? x0 : (x1 < T(0) ? x1 : T(0));
  const T ny = y0 > T(0) ? y0 : (y1 < T(0) ? y1 : T(0));
  return nx * nx + ny * ny < r * r;
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
  return cut_cell_fraction(r, dx, dy);
}

// Offset of the k-th of n sub-cell centres from the cell centre along one axis, (k + 1/2)/n - 1/2
// (evaluated in FP64, then rounded to T).
template <class T>
__host__ __device__ inline T subcell_offset(int k, int n) {
  return (T)((k + 0.5) / n - 0.5);
}

// Fraction of the n x n sub-cell centres of the cell centred at (dx, dy) strictly inside the
// disk; out of line, like cut_cell_fraction, so that it does not enlarge the caller's registers.
// off: the n offsets (subcell_offset) from a table, or null to evaluate them here.
template <class T>
__host__ __device__ __noinline__ T subcell_count(T r, T dx, T dy, int n, const T* off) {
  int inside = 0;
  for (int j = 0; j < n; ++j) {
    const T yc = dy + (off ? off[j] : subcell_offset<T>(j, n));
    for (int i = 0; i < n; ++i) {
      const T xc = dx + (off ? off[i] : subcell_offset<T>(i, n));
      inside += xc * xc + yc * yc < r * r ? 1 : 0;
    }
  }
  return (T)inside / ((T)n * (T)n);
}

// A cut cell's ratio under the selected estimate (out of line: one call site in the caller).
template <class T>
__host__ __device__ __noinline__ T cut_ratio(T r, T dx, T dy, int n, const T* off) {
  if (n > 0) return subcell_count(r, dx, dy, n, off);
  return cut_cell_fraction(r, dx, dy);
}

// The solid ratio the configuration selects: the exact area (n = 0) or the paper's estimate
// (Sec. 2.2, cell decomposition), the fraction of the cell's n x n sub-cell centres strictly
// inside the disk.  Both share the test for cells wholly outside (nearest point not inside: 0)
// or inside (farthest corner inside or on the circle: 1; every sub-cell centre is then at least
// 1/(2n) further in or out), so only cut cells reach the out-of-line part.
// off: a table of the n sub-cell offsets (subcell_offset), or null.
template <class T>
__host__ __device__ inline T cell_solid_ratio(T r, T dx, T dy, int n, const T* off = nullptr) {
  const T x0 = dx - T(0.5), x1 = dx + T(0.5), y0 = dy - T(0.5), y1 = dy + T(0.5);
  const T nx = x0 > T(0) ? x0 : (x1 < T(0) ? x1 : T(0));
  const T ny = y0 > T(0) ? y0 : (y1 < T(0) ? y1 : T(0));
  if (nx * nx + ny * ny >= r * r) return T(0);
  const T fx = fabs(x0) > fabs(x1) ? fabs(x0) : fabs(x1);
  const T fy = fabs(y0) > fabs(y1) ? fabs(y0) : fabs(y1);
  if (fx * fx + fy * fy <= r * r) return T(1);
  if constexpr (sizeof(T) == 4) {  // single precision: the common cut without branches
    float e;
    if (n == 0 && one_arc_fraction(r, dx, dy, &e)) return e;
  }
  return cut_ratio(r, dx, dy, n, off);
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
