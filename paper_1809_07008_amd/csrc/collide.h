// collide.h -- collision of one lattice cell with the immersed-moving-boundary term.
//
//   f*_i = f_i + (1 - B_tot)(Omega^f_i + G_i) + sum_p B_p Omega^s_{p,i}          Eq. (13)
//   Omega^f_i = -(f_i - f_i^eq(rho, u)) / tau_eff                                  Eq. (1)
//   f_i^eq(rho, v) = w_i rho (1 + 3 c_i.v + 9/2 (c_i.v)^2 - 3/2 v.v)               Eq. (2)
//   Omega^s_{p,i} = f_{-i} - f_{-i}^eq(rho, u) + f_i^eq(rho, u_s,p) - f_i           Eq. (12)
//   B(eps, tau) = eps (tau - 1/2) / ((1 - eps) + (tau - 1/2))                      Eq. (14)
//   dF_p = -B_p sum_i Omega^s_{p,i} c_i = B_p (m - rho u_s,p), dT_p = d x dF_p    Eqs. (15),(16)
// with rho, m = rho u the moments of Eqs. (3), (4).  The printed force sum is the momentum the
// fluid gains; the force on the disk is its negative.  Readings where the paper is silent:
//   - several disks in one cell: eps_tot = min(1, sum eps_p), B_tot = B(eps_tot, tau_eff),
//     B_p = B_tot (eps_p / sum eps_p);
//   - body force G_i = 3 w_i rho (c_i . g) applied where the cell is fluid, weight (1 - B_tot);
//   - Smagorinsky (Sec. 3.3.2, Hou et al.):  tau_eff = (tau0 + sqrt(tau0^2 + 18 sqrt2 C_s^2 |Pi| /
//     rho)) / 2 with Pi = sum_i c_i c_i (f_i - f_i^eq) the non-equilibrium momentum flux;
//   - solid velocity at the node u_s = V + omega x d, d = node - centre (nearest image).
//
// Two forms.  collide_plain (FP64 storage) works on f and keeps the operation order of a plain
// textbook evaluation (no contraction) so that it reproduces an FP64 reference to rounding.
// collide_dev (FP32 / FP16 storage) works on deviations h_i = f_i - w_i rho0 throughout, so the
// small velocity-carrying parts never cancel against the O(1) rest populations in FP32.
//
// The covering disks are supplied by two callables so that their data can stay in LDS:
//   disk(k) -> Disk<T> for k < nc,   emit(k, fx, fy, tz) receives disk k's force / torque.
#pragma once

#include "common.h"

namespace imb {

template <class T>
struct Disk {
  T eps, dx, dy, vx, vy, om;
};

// ------------------------------------------------------------------------- FP64 (plain f)
__device__ inline void equilibrium_plain(double rho, double ux, double uy, double feq[NQ]) {
#pragma clang fp contract(off)
  const double uu = ux * ux + uy * uy;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const double cu = (double)cx_of(i) * ux + (double)cy_of(i) * uy;
    feq[i] = w_of(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

template <class GetDisk, class Emit>
__device__ inline double collide_plain(const double f[NQ], int nc, GetDisk disk, Emit emit,
                                       double tau0, double cs, double gx, double gy,
                                       double fout[NQ]) {
#pragma clang fp contract(off)
  double rho = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) rho += f[i];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    mx += (double)cx_of(i) * f[i];
    my += (double)cy_of(i) * f[i];
  }
  const double ux = mx / rho, uy = my / rho;
  double feq[NQ];
  equilibrium_plain(rho, ux, uy, feq);
  double tau = tau0;
  if (cs > 0.0) {
    double pxx = 0.0, pxy = 0.0, pyy = 0.0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const double neq = f[i] - feq[i];
      pxx += (double)(cx_of(i) * cx_of(i)) * neq;
      pxy += (double)(cx_of(i) * cy_of(i)) * neq;
      pyy += (double)(cy_of(i) * cy_of(i)) * neq;
    }
    const double pn = sqrt(pxx * pxx + 2.0 * pxy * pxy + pyy * pyy);
    tau = 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * pn / rho));
  }
  double S = 0.0;
  for (int k = 0; k < nc; ++k) S += disk(k).eps;
  const double et = S < 1.0 ? S : 1.0;
  const double a = tau - 0.5;
  const double Bt = et * a / ((1.0 - et) + a);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const double G = 3.0 * w_of(i) * rho * ((double)cx_of(i) * gx + (double)cy_of(i) * gy);
    const double Of = -(f[i] - feq[i]) / tau;
    fout[i] = f[i] + (1.0 - Bt) * (Of + G);
  }
  for (int k = 0; k < nc; ++k) {
    const Disk<double> d = disk(k);
    const double Bp = S > 0.0 ? Bt * (d.eps / S) : 0.0;
    const double usx = d.vx - d.om * d.dy;
    const double usy = d.vy + d.om * d.dx;
    double feqs[NQ];
    equilibrium_plain(rho, usx, usy, feqs);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int o = opp_of(i);
      const double Os = f[o] - feq[o] + feqs[i] - f[i];
      fout[i] += Bp * Os;
    }
    const double fx = Bp * (mx - rho * usx);
    const double fy = Bp * (my - rho * usy);
    emit(k, fx, fy, d.dx * fy - d.dy * fx);
  }
  return rho;
}

// --------------------------------------------------------------- FP32 (deviation form)
// h_i = f_i - w_i rho0; the equilibrium deviation is w_i (drho + rho (3cu + 4.5cu^2 - 1.5uu))
// with drho = rho - rho0 = sum h_i; the momentum is sum c_i h_i (the w_i rho0 parts cancel).
// Opposite directions share their even part (cu_opp = -cu_i), and with
// gw_i = w_i (c_i . g) the update of a cell is
//   h*_i = h_i - (1 - B_tot)/tau neq_i + 3 rho (1 - B_tot) gw_i + sum_p B_p Omega^s_{p,i}.
// A cell no disk covers (nc == 0) has B_tot = 0.
template <class GetDisk, class Emit>
__device__ inline float collide_dev(const float h[NQ], int nc, GetDisk disk, Emit emit,
                                    float rho0, float tau0, float cs, float gx, float gy,
                                    float hout[NQ]) {
#pragma clang fp contract(fast)
  // moments (Eqs. 3, 4); D2Q9 order: rest, E, N, W, S, NE, NW, SW, SE
  const float d57 = h[5] - h[7], d86 = h[8] - h[6];
  const float dr = ((h[0] + (h[1] + h[3])) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8]));
  const float mx = (h[1] - h[3]) + (d57 + d86);
  const float my = (h[2] - h[4]) + (d57 - d86);
  const float rho = rho0 + dr;
  const float irho = 1.0f / rho;
  const float ux = mx * irho, uy = my * irho;
  const float uu = ux * ux + uy * uy;
  const float even0 = dr - 1.5f * rho * uu;  // (drho + rho (-1.5 uu)): the part common to all i
  const float rho45 = 4.5f * rho, rho3 = 3.f * rho;
  float neq[NQ];
  neq[0] = h[0] - (float)w_of(0) * even0;
  constexpr int PAIR[4] = {1, 2, 5, 6};  // and their opposites 3, 4, 7, 8
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = PAIR[k], o = opp_of(i);
    const float cu = (float)cx_of(i) * ux + (float)cy_of(i) * uy;
    const float ev = (rho45 * cu) * cu + even0;
    const float od = rho3 * cu;
    neq[i] = h[i] - (float)w_of(i) * (ev + od);
    neq[o] = h[o] - (float)w_of(o) * (ev - od);
  }
  float tau = tau0;
  if (cs > 0.f) {
    // Pi = sum c_i c_i neq_i
    const float s57 = neq[5] + neq[7], s68 = neq[6] + neq[8];
    const float dd = s57 + s68;
    const float pxx = (neq[1] + neq[3]) + dd;
    const float pyy = (neq[2] + neq[4]) + dd;
    const float pxy = s57 - s68;
    const float pn = sqrtf(pxx * pxx + 2.f * pxy * pxy + pyy * pyy);
    tau = 0.5f * (tau0 + sqrtf(tau0 * tau0 + 25.455844122715710f * cs * cs * pn * irho));
  }
  const float itau = 1.0f / tau;
  float S = 0.f, Bt = 0.f;
  if (nc > 0) {
    for (int k = 0; k < nc; ++k) S += disk(k).eps;
    const float et = S < 1.f ? S : 1.f;
    const float a = tau - 0.5f;
    Bt = et * a / ((1.f - et) + a);
  }
  const float fl = 1.f - Bt;
  const float k1 = fl * itau, k2 = fl * rho3;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const float gw = (float)w_of(i) * ((float)cx_of(i) * gx + (float)cy_of(i) * gy);
    hout[i] = (h[i] - k1 * neq[i]) + k2 * gw;
  }
  for (int k = 0; k < nc; ++k) {
    const Disk<float> d = disk(k);
    const float Bp = S > 0.f ? Bt * (d.eps / S) : 0.f;
    const float usx = d.vx - d.om * d.dy;
    const float usy = d.vy + d.om * d.dx;
    const float us2 = usx * usx + usy * usy;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const float cu = (float)cx_of(i) * usx + (float)cy_of(i) * usy;
      const float heqs = (float)w_of(i) * (dr + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * us2));
      const float Os = neq[opp_of(i)] + heqs - h[i];
      hout[i] += Bp * Os;
    }
    const float fx = Bp * (mx - rho * usx);
    const float fy = Bp * (my - rho * usy);
    emit(k, fx, fy, d.dx * fy - d.dy * fx);
  }
  return rho;
}

}  // namespace imb
