// lattice3.h -- the three-dimensional lattice step with spheres: D3Q19 velocity set, the IMB
// collision of one cell, and the sphere geometry (Yang, Jing, Kwok & Sobral, arXiv:1809.07008,
// Sec. 2: Eqs. 1-4 with the D3Q19 set of Table 1; Sec. 2.2 and Eqs. 12-16 for the spheres).
//
// Velocity order (also the order of populations exchanged through the C-ABI):
//   0: rest;  1-6: +x -x +y -y +z -z;  7-18: the face diagonals of the (x,y), (x,z) and (y,z)
//   planes, four per plane as (+,+) (-,-) (+,-) (-,+) in the plane's two axes.
// Each direction i >= 1 is followed (i odd) or preceded (i even) by its opposite.
#pragma once

#include "common.h"

namespace imb {

constexpr int NQ3 = 19;
constexpr int MAXC3 = 4;        // spheres covering one cell
constexpr int MAXCAND3 = 16;    // spheres whose boxes touch one tile
constexpr int MAXS3 = 256;      // spheres per simulation
constexpr int MAXSLOT3 = 4096;  // tiles per sphere box (force partial slots)
constexpr int NPART3 = 6;       // force (3) and torque (3) per partial

// Component a (0 = x, 1 = y, 2 = z) of velocity i.
__host__ __device__ constexpr int c3(int i, int a) {
  if (i == 0) return 0;
  if (i <= 6) return (i - 1) / 2 == a ? ((i & 1) ? 1 : -1) : 0;
  const int k = i - 7, plane = k / 4, j = k % 4;
  const int a0 = plane == 2 ? 1 : 0;       // first axis of the plane
  const int a1 = plane == 0 ? 1 : 2;       // second axis
  if (a == a0) return (j == 0 || j == 2) ? 1 : -1;
  if (a == a1) return (j == 0 || j == 3) ? 1 : -1;
  return 0;
}
__host__ __device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double w3(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
static_assert(c3(1, 0) == 1 && c3(2, 0) == -1 && c3(5, 2) == 1 && c3(6, 2) == -1, "axes");
static_assert(c3(7, 0) == 1 && c3(7, 1) == 1 && c3(8, 0) == -1 && c3(8, 1) == -1, "xy");
static_assert(c3(9, 0) == 1 && c3(9, 1) == -1 && c3(10, 0) == -1 && c3(10, 1) == 1, "xy");
static_assert(c3(13, 0) == 1 && c3(13, 2) == -1 && c3(18, 1) == -1 && c3(18, 2) == 1, "xz yz");
static_assert(c3(opp3(17), 1) == -c3(17, 1) && c3(opp3(17), 2) == -c3(17, 2), "opposites");

// One sphere as the lattice step sees it.
template <class T>
struct Sph {
  T eps, dx, dy, dz, vx, vy, vz, wx, wy, wz;
};

// The tile box of a sphere: every tile (tw x th cells in x, y; one z layer) holding a cell of
// its bounding box [floor(X - r - 1/2), ceil(X + r + 1/2)] per axis; cyclic in x and z (and y
// without walls).  When the lattice is not a whole number of tiles wide, a box that wraps can
// meet the partial last tile and the first one out of tile order; a box wider than n - tw cells
// takes the whole row of tiles instead (narrower boxes cannot meet either tile twice).  Slots are
// numbered x fastest, then y, then z.
struct Box3 {
  int tx0, ntx, ty0, nty, z0, nzz;
};

__host__ __device__ inline int wrap3i(int a, int n) {
  int m = a % n;
  return m < 0 ? m + n : m;
}

__host__ __device__ inline Box3 sphere_box3(double X, double Y, double Z, double r, int nx, int ny,
                                            int nz, int walls, int tw, int th, int tiles_x,
                                            int tiles_y) {
  Box3 b;
  const int ix0 = (int)floor(X - r - 0.5), ix1 = (int)ceil(X + r + 0.5);
  if (ix1 - ix0 + 1 > nx - tw) {
    b.tx0 = 0;
    b.ntx = tiles_x;
  } else {
    b.tx0 = wrap3i(ix0, nx) / tw;
    b.ntx = wrap3i(wrap3i(ix1, nx) / tw - b.tx0, tiles_x) + 1;
  }
  int iy0 = (int)floor(Y - r - 0.5), iy1 = (int)ceil(Y + r + 0.5);
  if (walls) {
    if (iy0 < 0) iy0 = 0;
    if (iy1 > ny - 1) iy1 = ny - 1;
    b.ty0 = iy0 / th;
    b.nty = iy1 >= iy0 ? iy1 / th - b.ty0 + 1 : 0;
  } else if (iy1 - iy0 + 1 > ny - th) {
    b.ty0 = 0;
    b.nty = tiles_y;
  } else {
    b.ty0 = wrap3i(iy0, ny) / th;
    b.nty = wrap3i(wrap3i(iy1, ny) / th - b.ty0, tiles_y) + 1;
  }
  const int iz0 = (int)floor(Z - r - 0.5), iz1 = (int)ceil(Z + r + 0.5);
  b.z0 = wrap3i(iz0, nz);
  b.nzz = iz1 - iz0 + 1;
  return b;
}

// Slot of tile (tx, ty, z) in box b, or -1 outside.
__host__ __device__ inline int box3_slot(const Box3& b, int tx, int ty, int z, int tiles_x,
                                         int tiles_y, int nz) {
  int lx = tx - b.tx0;
  if (lx < 0) lx += tiles_x;
  if (lx >= b.ntx) return -1;
  int ly = ty - b.ty0;
  if (ly < 0) ly += tiles_y;
  if (ly < 0 || ly >= b.nty) return -1;
  int lz = z - b.z0;
  if (lz < 0) lz += nz;
  if (lz >= b.nzz) return -1;
  return (lz * b.nty + ly) * b.ntx + lx;
}

// Signed offset of cell index c from centre coordinate X along an axis of n cells: the nearest
// image when the axis is periodic.
template <class T>
__device__ inline T axis_d3(int c, double X, int n, bool periodic) {
  const double fl = floor(X);
  int di = c - (int)fl;
  if (periodic) {
    const int h = n / 2;
    if (di > h) di -= n;
    else if (di < -h) di += n;
  }
  return (T)di - (T)(X - fl);
}

// The paper's solid ratio of the unit cell centred at d from the sphere centre (Sec. 2.2, cell
// decomposition): the share of its n^3 sub-cell centres strictly inside.  A cell whose nearest
// point is not inside gives 0, one whose farthest corner is inside or on the surface gives 1
// (every sub-cell centre is then strictly inside), so only cut cells count centres.
// N fixed at compile time: the offsets and each column's x term in registers and every loop
// unrolled (the general loop reads an offset from LDS per centre).  The same sums and
// comparisons as the general loop, so the same count.
template <class T, int N>
__device__ inline T sphere_subcells_n(T r, T dx, T dy, T dz, const T* off) {
  const T r2 = r * r;
  T o[N], x2[N];
#pragma unroll
  for (int i = 0; i < N; ++i) o[i] = off[i];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const T xc = dx + o[i];
    x2[i] = xc * xc;
  }
  int inside = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const T zc = dz + o[k];
    const T z2 = zc * zc;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const T yc = dy + o[j];
      const T yz2 = yc * yc + z2;
#pragma unroll
      for (int i = 0; i < N; ++i) inside += x2[i] + yz2 < r2 ? 1 : 0;
    }
  }
  return (T)inside / ((T)N * (T)N * (T)N);
}

template <class T>
__device__ __noinline__ T sphere_subcells(T r, T dx, T dy, T dz, int n, const T* off) {
  switch (n) {
    case 1: return sphere_subcells_n<T, 1>(r, dx, dy, dz, off);
    case 2: return sphere_subcells_n<T, 2>(r, dx, dy, dz, off);
    case 3: return sphere_subcells_n<T, 3>(r, dx, dy, dz, off);
    case 4: return sphere_subcells_n<T, 4>(r, dx, dy, dz, off);
    case 5: return sphere_subcells_n<T, 5>(r, dx, dy, dz, off);
    case 6: return sphere_subcells_n<T, 6>(r, dx, dy, dz, off);
    case 7: return sphere_subcells_n<T, 7>(r, dx, dy, dz, off);
    case 8: return sphere_subcells_n<T, 8>(r, dx, dy, dz, off);
    default: break;
  }
  const T r2 = r * r;
  int inside = 0;
  for (int k = 0; k < n; ++k) {
    const T zc = dz + off[k];
    const T z2 = zc * zc;
    for (int j = 0; j < n; ++j) {
      const T yc = dy + off[j];
      const T yz2 = yc * yc + z2;
      for (int i = 0; i < n; ++i) {
        const T xc = dx + off[i];
        inside += xc * xc + yz2 < r2 ? 1 : 0;
      }
    }
  }
  return (T)inside / ((T)n * (T)n * (T)n);
}

// The sub-cell centres' offsets from the cell centre along one axis, (k + 1/2)/n - 1/2 for
// k < n (evaluated in FP64, then rounded to T), for sphere_subcells; off holds n values.
template <class T>
__device__ inline void subcell_offsets(T* off, int n, int k) {
  if (k < n) off[k] = (T)((k + 0.5) / n - 0.5);
}

template <class T>
__device__ inline T cell_near2(T d) {  // squared distance to the nearest point of [d-1/2, d+1/2]
  const T lo = d - T(0.5), hi = d + T(0.5);
  const T v = lo > T(0) ? lo : (hi < T(0) ? hi : T(0));
  return v * v;
}

template <class T>
__device__ inline T sphere_ratio(T r, T dx, T dy, T dz, int n, const T* off) {
  const T r2 = r * r;
  if (cell_near2(dx) + cell_near2(dy) + cell_near2(dz) >= r2) return T(0);
  const T fx = fabs(dx) + T(0.5), fy = fabs(dy) + T(0.5), fz = fabs(dz) + T(0.5);
  if (fx * fx + fy * fy + fz * fz <= r2) return T(1);
  return sphere_subcells(r, dx, dy, dz, n, off);
}

// ---------------------------------------------------------------- collision, FP64 (plain f)
// f*_i = f_i + (1 - B_tot)(Omega^f_i + G_i) + sum_p B_p Omega^s_{p,i}, Eq. (13), with the readings
// of the two-dimensional collide_plain (several spheres per cell, forcing weighted by 1 - B_tot);
// emit(k, F, T) receives sphere k's force on the sphere B_p (m - rho u_s) and torque d x F.
__device__ inline void equilibrium3_plain(double rho, double ux, double uy, double uz,
                                          double feq[NQ3]) {
#pragma clang fp contract(off)
  const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < NQ3; ++i) {
    const double cu = (double)c3(i, 0) * ux + (double)c3(i, 1) * uy + (double)c3(i, 2) * uz;
    feq[i] = w3(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

template <class GetSph, class Emit>
__device__ inline double collide3_plain(const double f[NQ3], int nc, GetSph sph, Emit emit,
                                        double tau, double gx, double gy, double gz,
                                        double fout[NQ3]) {
#pragma clang fp contract(off)
  double rho = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
  for (int i = 0; i < NQ3; ++i) rho += f[i];
#pragma unroll
  for (int i = 0; i < NQ3; ++i) {
    mx += (double)c3(i, 0) * f[i];
    my += (double)c3(i, 1) * f[i];
    mz += (double)c3(i, 2) * f[i];
  }
  const double ux = mx / rho, uy = my / rho, uz = mz / rho;
  double feq[NQ3];
  equilibrium3_plain(rho, ux, uy, uz, feq);
  double S = 0.0;
  for (int k = 0; k < nc; ++k) S += sph(k).eps;
  const double et = S < 1.0 ? S : 1.0;
  const double a = tau - 0.5;
  const double Bt = et * a / ((1.0 - et) + a);
#pragma unroll
  for (int i = 0; i < NQ3; ++i) {
    const double G = 3.0 * w3(i) * rho *
                     ((double)c3(i, 0) * gx + (double)c3(i, 1) * gy + (double)c3(i, 2) * gz);
    const double Of = -(f[i] - feq[i]) / tau;
    fout[i] = f[i] + (1.0 - Bt) * (Of + G);
  }
  for (int k = 0; k < nc; ++k) {
    const Sph<double> s = sph(k);
    const double Bp = S > 0.0 ? Bt * (s.eps / S) : 0.0;
    const double usx = s.vx + (s.wy * s.dz - s.wz * s.dy);
    const double usy = s.vy + (s.wz * s.dx - s.wx * s.dz);
    const double usz = s.vz + (s.wx * s.dy - s.wy * s.dx);
    double feqs[NQ3];
    equilibrium3_plain(rho, usx, usy, usz, feqs);
#pragma unroll
    for (int i = 0; i < NQ3; ++i) {
      const int o = opp3(i);
      const double Os = f[o] - feq[o] + feqs[i] - f[i];
      fout[i] += Bp * Os;
    }
    const double Fx = Bp * (mx - rho * usx);
    const double Fy = Bp * (my - rho * usy);
    const double Fz = Bp * (mz - rho * usz);
    emit(k, Fx, Fy, Fz, s.dy * Fz - s.dz * Fy, s.dz * Fx - s.dx * Fz, s.dx * Fy - s.dy * Fx);
  }
  return rho;
}

// ---------------------------------------------------------- collision, FP32 (deviation form)
// h_i = f_i - w_i rho0; the equilibrium deviation is w_i (drho + rho (3 cu + 4.5 cu^2 - 1.5 uu))
// and opposite directions share its even part.
template <class GetSph, class Emit>
__device__ inline float collide3_dev(const float h[NQ3], int nc, GetSph sph, Emit emit,
                                     float rho0, float tau, float gx, float gy, float gz,
                                     float hout[NQ3]) {
#pragma clang fp contract(fast)
  float dr = h[0];
#pragma unroll
  for (int i = 1; i < NQ3; i += 2) dr += h[i] + h[i + 1];
  float mx = 0.f, my = 0.f, mz = 0.f;
#pragma unroll
  for (int i = 1; i < NQ3; i += 2) {
    const float d = h[i] - h[i + 1];  // direction i minus its opposite
    mx += (float)c3(i, 0) * d;
    my += (float)c3(i, 1) * d;
    mz += (float)c3(i, 2) * d;
  }
  const float rho = rho0 + dr;
  const float irho = 1.0f / rho;
  const float ux = mx * irho, uy = my * irho, uz = mz * irho;
  const float even0 = dr - 1.5f * rho * (ux * ux + uy * uy + uz * uz);
  const float rho45 = 4.5f * rho, rho3 = 3.f * rho;
  float neq[NQ3];
  neq[0] = h[0] - (float)w3(0) * even0;
#pragma unroll
  for (int i = 1; i < NQ3; i += 2) {
    const float cu = (float)c3(i, 0) * ux + (float)c3(i, 1) * uy + (float)c3(i, 2) * uz;
    const float ev = (rho45 * cu) * cu + even0;
    const float od = rho3 * cu;
    neq[i] = h[i] - (float)w3(i) * (ev + od);
    neq[i + 1] = h[i + 1] - (float)w3(i + 1) * (ev - od);
  }
  float S = 0.f, Bt = 0.f;
  if (nc > 0) {
    for (int k = 0; k < nc; ++k) S += sph(k).eps;
    const float et = S < 1.f ? S : 1.f;
    const float a = tau - 0.5f;
    Bt = et * a / ((1.f - et) + a);
  }
  const float fl = 1.f - Bt;
  const float k1 = fl / tau, k2 = fl * rho3;
#pragma unroll
  for (int i = 0; i < NQ3; ++i) {
    const float gw = (float)w3(i) * ((float)c3(i, 0) * gx + (float)c3(i, 1) * gy +
                                     (float)c3(i, 2) * gz);
    hout[i] = (h[i] - k1 * neq[i]) + k2 * gw;
  }
  for (int k = 0; k < nc; ++k) {
    const Sph<float> s = sph(k);
    const float Bp = S > 0.f ? Bt * (s.eps / S) : 0.f;
    const float usx = s.vx + (s.wy * s.dz - s.wz * s.dy);
    const float usy = s.vy + (s.wz * s.dx - s.wx * s.dz);
    const float usz = s.vz + (s.wx * s.dy - s.wy * s.dx);
    const float us2 = usx * usx + usy * usy + usz * usz;
#pragma unroll
    for (int i = 0; i < NQ3; ++i) {
      const float cu = (float)c3(i, 0) * usx + (float)c3(i, 1) * usy + (float)c3(i, 2) * usz;
      const float heqs = (float)w3(i) * (dr + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * us2));
      hout[i] += Bp * (neq[opp3(i)] + heqs - h[i]);
    }
    const float Fx = Bp * (mx - rho * usx);
    const float Fy = Bp * (my - rho * usy);
    const float Fz = Bp * (mz - rho * usz);
    emit(k, Fx, Fy, Fz, s.dy * Fz - s.dz * Fy, s.dz * Fx - s.dx * Fz, s.dx * Fy - s.dy * Fx);
  }
  return rho;
}

}  // namespace imb
