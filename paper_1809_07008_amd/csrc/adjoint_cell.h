// adjoint_cell.h -- transposed Jacobian of the one-cell IMB collision (differentiation form).
//
// The forward cell update is the one of collide.h with a constant relaxation time (no
// Smagorinsky term), written on deviations h_i = f_i - w_i rho0:
//   drho = sum h_i, m = sum c_i h_i, rho = rho0 + drho, u = m / rho
//   heq_i(v) = w_i (drho + rho P_i(v)),  P_i(v) = 3 c_i.v + 9/2 (c_i.v)^2 - 3/2 v.v      Eq. (2)
//   neq_i = h_i - heq_i(u)
//   S = sum_k eps_k, eps_t = min(1, S), B_t = B(eps_t, tau), B_k = B_t eps_k / S         Eq. (14)
//   h*_i = h_i + (1 - B_t)(G_i - neq_i / tau) + sum_k B_k (neq_{-i} + heq_i(us_k) - h_i) Eqs. (1),(12),(13)
//   G_i = 3 w_i rho (c_i . g)
//   F_k = B_k (m - rho us_k),  T_k = d_k x F_k,  us_k = V_k + omega_k x d_k            Eqs. (15),(16)
// and the objective collects sum_k (wfx_k F_kx + wfy_k F_ky + wtz_k T_k).  Given lam_i = dJ/dh*_i
// the routine returns dJ/dh_i, dJ/dg and, per covering disk, dJ/dX, dJ/dY (through eps_k and
// through the lever arm d_k = node - X_k), dJ/dV and dJ/domega (through the solid velocity).
// The derivative of eps_k with respect to the centre is the analytic one of the exact overlap
// area (difference of the clipped chord lengths on opposite cell edges).
#pragma once

#include "common.h"

namespace imb {

template <class T>
struct DiskAdj {
  T eps, dex, dey;  // eps_k and d eps_k / d(X, Y)
  T dx, dy;         // lever arm node - centre
  T vx, vy, om;
  T wfx, wfy, wtz;  // objective weights of the disk
};

// emit(k, gX, gY, gVx, gVy, gOm) receives covering disk k's parameter gradient.
template <class T, class GetDisk, class Emit>
__device__ inline void collide_adjoint(const T h[NQ], const T lam[NQ], int nc, GetDisk disk,
                                       Emit emit, T rho0, T tau, T gx, T gy, T gh[NQ],
                                       T* ggx, T* ggy) {
  // ---- forward quantities
  T dr = T(0), mx = T(0), my = T(0);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    dr += h[i];
    mx += (T)cx_of(i) * h[i];
    my += (T)cy_of(i) * h[i];
  }
  const T rho = rho0 + dr;
  const T irho = T(1) / rho;
  const T ux = mx * irho, uy = my * irho;
  const T uu = ux * ux + uy * uy;
  T P[NQ], neq[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const T cu = (T)cx_of(i) * ux + (T)cy_of(i) * uy;
    P[i] = T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu;
    neq[i] = h[i] - (T)w_of(i) * (dr + rho * P[i]);
  }
  T S = T(0);
#pragma unroll
  for (int k = 0; k < MAXC; ++k)
    if (k < nc) S += disk(k).eps;
  const T et = S < T(1) ? S : T(1);
  const T a = tau - T(0.5);
  const T den = (T(1) - et) + a;
  const T Bt = et * a / den;
  const T fl = T(1) - Bt;
  const T itau = T(1) / tau;
  const T iS = S > T(0) ? T(1) / S : T(0);
  const T Lsum = Bt * S * iS;  // sum_k B_k

  // ---- fluid part
  T grho = T(0), gdr = T(0), gmx = T(0), gmy = T(0), gux = T(0), guy = T(0);
  T gBt = T(0), lw = T(0);
  T sgx = T(0), sgy = T(0);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const T G = T(3) * (T)w_of(i) * rho * ((T)cx_of(i) * gx + (T)cy_of(i) * gy);
    gBt -= lam[i] * (G - neq[i] * itau);
    lw += lam[i] * (T)w_of(i);
    // G_i: its rho and g derivatives
    const T lg = fl * lam[i] * T(3) * (T)w_of(i);
    grho += lg * ((T)cx_of(i) * gx + (T)cy_of(i) * gy);
    sgx += lg * (T)cx_of(i);
    sgy += lg * (T)cy_of(i);
  }
  *ggx = sgx * rho;
  *ggy = sgy * rho;
  // d/d neq_i: from the fluid relaxation of h*_i and the bounce-back term of h*_{-i}
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const T gneq = -fl * itau * lam[i] + Lsum * lam[opp_of(i)];
    gh[i] = (T(1) - Lsum) * lam[i] + gneq;
    // heq_i(u) = w_i (drho + rho P_i(u)) enters with -gneq
    const T ge = -gneq * (T)w_of(i);
    gdr += ge;
    grho += ge * P[i];
    const T cu = (T)cx_of(i) * ux + (T)cy_of(i) * uy;
    const T q = ge * rho;
    gux += q * (T(3) * (T)cx_of(i) + T(9) * cu * (T)cx_of(i) - T(3) * ux);
    guy += q * (T(3) * (T)cy_of(i) + T(9) * cu * (T)cy_of(i) - T(3) * uy);
  }

  // ---- disks, first pass: dJ/dB_k and the solid-velocity gradients
  T gB[MAXC], gusx[MAXC], gusy[MAXC], Fx[MAXC], Fy[MAXC];
  T sgB = T(0);
#pragma unroll
  for (int k = 0; k < MAXC; ++k) {
    gB[k] = gusx[k] = gusy[k] = Fx[k] = Fy[k] = T(0);
    if (k >= nc) continue;
    const DiskAdj<T> d = disk(k);
    const T Bp = Bt * d.eps * iS;
    const T usx = d.vx - d.om * d.dy, usy = d.vy + d.om * d.dx;
    const T us2 = usx * usx + usy * usy;
    T gb = T(0), lp = T(0), lgx = T(0), lgy = T(0);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const T cu = (T)cx_of(i) * usx + (T)cy_of(i) * usy;
      const T Ps = T(3) * cu + T(4.5) * cu * cu - T(1.5) * us2;
      const T heqs = (T)w_of(i) * (dr + rho * Ps);
      gb += lam[i] * (neq[opp_of(i)] + heqs - h[i]);
      const T lwi = lam[i] * (T)w_of(i);
      lp += lwi * Ps;
      lgx += lwi * (T(3) * (T)cx_of(i) + T(9) * cu * (T)cx_of(i) - T(3) * usx);
      lgy += lwi * (T(3) * (T)cy_of(i) + T(9) * cu * (T)cy_of(i) - T(3) * usy);
    }
    // objective: dJ/dF including the torque's share
    const T ax = d.wfx - d.wtz * d.dy, ay = d.wfy + d.wtz * d.dx;
    const T fmx = mx - rho * usx, fmy = my - rho * usy;
    gb += ax * fmx + ay * fmy;
    Fx[k] = Bp * fmx;
    Fy[k] = Bp * fmy;
    // heq(us_k) terms (weight B_k lam_i)
    gdr += Bp * lw;
    grho += Bp * lp;
    gusx[k] = Bp * rho * lgx - Bp * rho * ax;
    gusy[k] = Bp * rho * lgy - Bp * rho * ay;
    // force terms
    gmx += Bp * ax;
    gmy += Bp * ay;
    grho -= Bp * (ax * usx + ay * usy);
    gB[k] = gb;
    sgB += gb * d.eps;
  }
  gBt += sgB * iS;

  // ---- disks, second pass: dJ/deps_k and the parameter gradients
  const T gS = S < T(1) ? gBt * a * (T(1) + a) / (den * den) : T(0);
#pragma unroll
  for (int k = 0; k < MAXC; ++k) {
    if (k >= nc) continue;
    const DiskAdj<T> d = disk(k);
    const T geps = gS + Bt * iS * (gB[k] - sgB * iS);
    // lever arm: solid velocity and torque
    const T gdx = d.om * gusy[k] + d.wtz * Fy[k];
    const T gdy = -d.om * gusx[k] - d.wtz * Fx[k];
    const T gX = geps * d.dex - gdx;
    const T gY = geps * d.dey - gdy;
    const T gOm = -gusx[k] * d.dy + gusy[k] * d.dx;
    emit(k, gX, gY, gusx[k], gusy[k], gOm);
  }

  // ---- u = m / rho, rho = rho0 + drho, moments of h
  gmx += gux * irho;
  gmy += guy * irho;
  grho -= (gux * ux + guy * uy) * irho;
  gdr += grho;
#pragma unroll
  for (int i = 0; i < NQ; ++i) gh[i] += gdr + (T)cx_of(i) * gmx + (T)cy_of(i) * gmy;
}

}  // namespace imb
