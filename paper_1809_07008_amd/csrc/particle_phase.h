// particle_phase.h -- the particle phase of a coupled step, one workgroup:
//   1. hydrodynamic force and torque on each disk (Eqs. 15, 16), as reduced by the disk's own
//      workgroup of the lattice step;
//   2. DEM (Sec. 2.1, 2.3): N_sub velocity-Verlet (kick-drift-kick) sub-cycles of dt = 1/N_sub
//      (Eq. 17) with the hydrodynamic load held fixed; normal linear spring-dashpot contacts
//      between disks and with the walls (Eqs. 7, 8), with k_t and mu also a tangential
//      spring-dashpot with a Coulomb limit; the contact force is evaluated after each
//      drift from the new positions and half-step velocities and reused by the next kick;
//      prescribed disks move by V once per step, fixed disks stay;
//   3. the disk table (tile box, position, velocity) and the per-tile-row (band) candidate masks
//      that the next lattice step reads.
//
// Contacts are searched in a Verlet neighbour list (skin DEM_SKIN) rebuilt whenever a disk has
// moved more than DEM_SKIN/2 - MAX_MOVE since the last build; a disk moving more than MAX_MOVE in
// one step latches ERR_MOVE, so no contact can be missed silently.
// A free disk that cannot reach a neighbour or a wall during the step ("quiet", the test bounds
// each disk's displacement over the step) feels no contact force and runs its sub-cycles on its
// own, without synchronisation; the others ("active") run them together, synchronised per
// sub-step.
// Readings: damping ratio zeta with c_n = 2 zeta sqrt(k_n m_eff); m = rho_s pi r^2, I = m r^2/2;
// no gravity; a tangential force (Sec. 2.1 names it without giving a discrete form) only when k_t
// or mu is set.
#pragma once

#include "step.h"

namespace imb {

constexpr int PP_DOUBLES = 7;  // LDS doubles per disk: x, y, vx, vy, r, the step's reach, spin

// Tangential contact force (2D Cundall-Strack, with a Coulomb limit): the spring s of the contact
// grows by the slip v_t over one sub-step when `advance`; F_t = -k_t s - c_t v_t with the
// contact law's tangential stiffness k_t and damping c_t (contact_law), limited to
// mu max(F_n, 0), a sliding contact resetting the spring to -F_t / k_t.  Returns F_t (along
// t = (-n_y, n_x) of the disk's own normal n).
__device__ inline double tangential_force(const ParticleArgs& a, double* spring, double vt,
                                          double fn, double kt, double ct, bool advance) {
#pragma clang fp contract(off)
  const double dt = 1.0 / a.n_sub;
  double sp = advance ? *spring + vt * dt : *spring;
  double ft = -kt * sp - ct * vt;
  const double cap = a.mu * (fn > 0.0 ? fn : 0.0);
  if (fabs(ft) > cap) {
    ft = ft > 0.0 ? cap : -cap;
    sp = kt > 0.0 ? -ft / kt : 0.0;
  }
  *spring = sp;
  return ft;
}

// The simplified Hertz-Mindlin law (Sec. 2.1 adopts it, after Di Renzo & Di Maio) of a contact
// of overlap delta > 0, effective radius rstar and mass meff, against another disk (E* = es,
// G* = gs of the pair) or a rigid wall: returns the normal force
// 4/3 E* sqrt(R*) delta^(3/2) + 2 sqrt(5/6) zeta sqrt(S_n m*) v_n with S_n = 2 E* sqrt(R* delta),
// and the tangential stiffness S_t = 8 G* sqrt(R* delta) and damping 2 sqrt(5/6) zeta
// sqrt(S_t m*) of the Mindlin spring.
__device__ inline double hertz_law(const ParticleArgs& a, double delta, double vn, double rstar,
                                   double meff, double es, double gs, double* kt, double* ct) {
#pragma clang fp contract(off)
  const double root = sqrt(rstar * delta);
  const double Sn = 2.0 * es * root;
  const double St = 8.0 * gs * root;
  *kt = St;
  *ct = a.hm_damp * sqrt(St * meff);
  return 4.0 / 3.0 * es * root * delta + a.hm_damp * sqrt(Sn * meff) * vn;
}

__device__ inline double nearest_image(double d, int n) {
  if (d > 0.5 * n) d -= n;
  else if (d < -0.5 * n) d += n;
  return d;
}

__device__ inline double wrap_coord(double v, int n) {
  if (v >= n) v -= n;
  else if (v < 0.0) v += n;
  return v;
}

template <int NT>
__device__ inline double block_sum(double v, double* s_red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) s_red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t += s_red[w];
  __syncthreads();
  return t;
}

// Bitwise OR of v over the workgroup (one barrier); s_part holds NT / 64 ints and is free
// again once every thread has returned.
template <int NT>
__device__ inline int block_or(int v, int* s_part) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = v;
  __syncthreads();
  int r = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r |= s_part[w];
  return r;
}

// Exclusive prefix sum of cnt[0..n) in place (LDS), returns the total.
template <int NT>
__device__ inline int block_exclusive_scan(int* cnt, int n, int* s_wave) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int chunk = (n + NT - 1) / NT;
  const int lo = tid * chunk, hi = min(lo + chunk, n);
  int local = 0;
  for (int k = lo; k < hi; ++k) local += cnt[k];
  int incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  int wbase = 0, total = 0;
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wave) wbase += s_wave[w];
    total += s_wave[w];
  }
  int run = wbase + incl - local;
  for (int k = lo; k < hi; ++k) {
    const int c = cnt[k];
    cnt[k] = run;
    run += c;
  }
  __syncthreads();
  return total;
}

// Latency layout: every global load the phase needs is issued in one batch at the start and
// every global store is issued after the last barrier (band masks of more tile rows than one
// round of LDS holds aside), so barriers never wait on memory; each
// disk's state lives in its own thread's registers and only positions and velocities that other
// disks' contact tests read are mirrored in LDS.
// One disk per thread: NT >= np.  `lds` holds a.lds_doubles >= max(PP_DOUBLES np, MASK_WORDS)
// doubles.
template <int NT>
__device__ __attribute__((always_inline)) void particle_phase(const ParticleArgs& a, double* lds) {
#pragma clang fp contract(off)
  constexpr int PWAVES = NT / 64;
  __shared__ double s_red[PWAVES];
  __shared__ int s_wave[PWAVES], s_or[PWAVES], s_flag[PWAVES];
  __shared__ int s_nact, s_aid[64], s_ann[64], s_awall[64], s_anb[64][8];
  __shared__ double s_ast[64][7];
  // the tangential springs of the one-wavefront path's active disks (LDS copies of their tables)
  __shared__ int s_hid[64][HK];
  __shared__ double s_hsp[64][HK], s_hw[64][2];
  constexpr int NB_REG = 8;   // neighbour ids kept in registers; the rest are read from the list
  const int np = a.np, p = threadIdx.x;
  const bool have = p < np;
  double* sx = lds;
  double* sy = sx + np;
  double* svx = sy + np;
  double* svy = svx + np;
  double* sr = svy + np;
  const ParticleState& s = a.s;

  // ---- one batch of loads
  double x = 0, y = 0, vx = 0, vy = 0, om = 0, r = 1, fcx = 0, fcy = 0, xref = 0, yref = 0;
  double tc = 0;  // contact torque of the last evaluation
  int mode = 1, nn = 0;
  int nb[NB_REG];
#pragma unroll
  for (int u = 0; u < NB_REG; ++u) nb[u] = 0;
  if (have) {
    x = s.x[p]; y = s.y[p]; vx = s.vx[p]; vy = s.vy[p]; om = s.om[p]; r = s.r[p];
    mode = s.mode[p];
    fcx = s.fcx[p]; fcy = s.fcy[p]; xref = s.xref[p]; yref = s.yref[p];
    tc = s.tcz[p];
    nn = s.nnbr[p];
#pragma unroll
    for (int u = 0; u < NB_REG; ++u) nb[u] = s.nbr[p * NBMAX + u];
  }
  const int rebuild_flag = a.do_dem || a.init_contacts || a.build_lists ? *s.rebuild : 0;
  const double x_start = x, y_start = y;

  // ---- 1. forces of the step that just ran
  double Fx = 0.0, Fy = 0.0, Tz = 0.0;
  if (have && a.do_finalize) {
    const double4 d0 = a.direct[a.dparts * p];
    Fx = d0.x;
    Fy = d0.y;
    Tz = d0.z;
    if (a.dparts > 1) {  // the second share
      const double4 d1 = a.direct[a.dparts * p + 1];
      Fx += d1.x;
      Fy += d1.y;
      Tz += d1.z;
    }
  } else if (have) {
    Fx = s.Fx[p];
    Fy = s.Fy[p];
    Tz = s.Tz[p];
  }
  double jsum = 0.0;
  if (a.do_finalize && a.J) {
    double jl = 0.0;
    if (have) {
      if (a.wfx) jl += a.wfx[p] * Fx;
      if (a.wfy) jl += a.wfy[p] * Fy;
      if (a.wtz) jl += a.wtz[p] * Tz;
    }
    jsum = block_sum<NT>(jl, s_red);
  }

  const bool own = have && mode == 0;
  const double m_p = a.rho_s * M_PI * r * r;
  // the step's reach of each disk (the classification below), published with the mirror
  double* sB = sr + np;
  double* som = sB + np;  // spins, for the partners' slip in tangential contacts
  const bool tang = a.hertz ? a.mu > 0.0 : (a.kt > 0.0 || a.mu > 0.0);
  double Bq = 0.0;
  if (own && a.do_dem) {
    const double qax = (0.0 + Fx) / m_p, qay = (0.0 + Fy) / m_p;
    Bq = sqrt(vx * vx + vy * vy) + 0.5 * sqrt(qax * qax + qay * qay) + 1e-9;
  }
  // bit 1: some disk is free; bit 2: the neighbour list must be rebuilt (ORed over the
  // workgroup through the mirror's barrier)
  const bool lists = a.do_dem || a.init_contacts || a.build_lists;
  int mine = 0;
  if (lists) {
    mine = own ? 1 : 0;
    if (have) {
      // rebuild before any disk can have moved (by the next lattice step) far enough that a
      // pair outside the list could touch, or cover a common cell
      const double ddx = nearest_image(x - xref, a.nx);
      const double ddy = a.walls ? y - yref : nearest_image(y - yref, a.ny);
      const double lim = 0.5 * (DEM_SKIN - M_SQRT2) - MAX_MOVE;
      if (ddx * ddx + ddy * ddy > lim * lim) mine |= 2;
    }
    if (p == 0 && rebuild_flag) mine |= 2;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mine |= __shfl_xor(mine, off, 64);
    if ((threadIdx.x & 63) == 0) s_flag[threadIdx.x >> 6] = mine;
  }
  if (have) {
    sx[p] = x; sy[p] = y; svx[p] = vx; svy[p] = vy; sr[p] = r;
    som[p] = om;
    const bool touching = own && (fcx != 0.0 || fcy != 0.0 || tc != 0.0);
    sB[p] = touching ? (Bq > MAX_MOVE ? Bq : MAX_MOVE) : Bq;
  }
  __syncthreads();
  int flags = 0;
  if (lists) {
#pragma unroll
    for (int w = 0; w < PWAVES; ++w) flags |= s_flag[w];
  }

  const double kn = a.kn, zeta = a.zeta;
  // contact force on disk i (Eqs. 7, 8): neighbours in ascending id, then the walls; mi is the
  // disk's mass and cnw = 2 zeta sqrt(kn mi) its wall damping coefficient (fixed for the step).
  // cnb may be any ascending sub-list of the neighbours that holds every disk able to touch i,
  // and near_wall may be false when no wall can: the terms left out are zero, so the sum is
  // the same bit for bit.
  // Tangential springs (when k_t or mu is set): a disk's table (hid, hsp: HK entries, partner
  // id + 1 and its spring) and its two wall springs; an entry exists only while the contact
  // does, and is freed when it ends.  `advance`: the springs grow by this evaluation's slip.
  auto contact_of = [&](int i, double ri, double mi, double cnw, int cnn, const int* cnb,
                        bool near_wall, double px, double py, double pvx, double pvy, double pom,
                        int* hid, double* hsp, double* hw, bool advance, double& ox, double& oy,
                        double& otz) {
    const double r = ri;
    double fx = 0.0, fy = 0.0, tz = 0.0;
    auto find = [&](int key) {
      int k = -1;
      for (int e = 0; e < HK; ++e)
        if (hid[e] == key) k = e;
      return k;
    };
    for (int q = 0; q < cnn; ++q) {
      int j = 0;
      if (q < NB_REG) {
#pragma unroll
        for (int u = 0; u < NB_REG; ++u)
          if (u == q) j = cnb[u];
      } else {
        j = s.nbr[i * NBMAX + q];
      }
      double dx = sx[j] - px;
      double dy = sy[j] - py;
      dx = nearest_image(dx, a.nx);
      if (!a.walls) dy = nearest_image(dy, a.ny);
      const double d2 = dx * dx + dy * dy;
      const double rs = r + sr[j];
      // pairs clearly apart skip the square root (the margin keeps rounding cases exact)
      bool touch = false;
      if (d2 <= rs * rs * (1.0 + 1e-12)) {
        const double dist = sqrt(d2);
        const double delta = rs - dist;
        if (delta > 0.0 && dist > 0.0) {
          touch = true;
          const double idist = 1.0 / dist;
          const double nxu = dx * idist, nyu = dy * idist;
          const double vn = (pvx - svx[j]) * nxu + (pvy - svy[j]) * nyu;
          const double mj = a.rho_s * M_PI * sr[j] * sr[j];
          const double meff = mi * mj / (mi + mj);
          double fn, kt_c, ct_c;
          if (a.hertz) {
            const double rstar = r * sr[j] / (r + sr[j]);
            fn = hertz_law(a, delta, vn, rstar, meff, a.es_pp, a.gs_pp, &kt_c, &ct_c);
          } else {
            const double cn = 2.0 * zeta * sqrt(kn * meff);
            fn = kn * delta + cn * vn;
            kt_c = a.kt;
            ct_c = 2.0 * zeta * sqrt(a.kt * meff);
          }
          fx += -fn * nxu;
          fy += -fn * nyu;
          if (tang) {
            const double tx = -nyu, ty = nxu;
            const double li = r - 0.5 * delta, lj = sr[j] - 0.5 * delta;
            const double vt = (pvx - svx[j]) * tx + (pvy - svy[j]) * ty + pom * li + som[j] * lj;
            int k = find(j + 1);
            double sp = k >= 0 ? hsp[k] : 0.0;
            const double ft = tangential_force(a, &sp, vt, fn, kt_c, ct_c, advance);
            fx += ft * tx;
            fy += ft * ty;
            tz += li * ft;
            if (k < 0) k = find(0);
            if (k < 0) {
              // a full table can still hold a contact that has ended and whose partner comes
              // later in the list: free those entries now (the same spring, 0, they get below)
              for (int e = 0; e < HK; ++e) {
                const int o = hid[e] - 1;
                double ex = nearest_image(sx[o] - px, a.nx);
                double ey = sy[o] - py;
                if (!a.walls) ey = nearest_image(ey, a.ny);
                const double ed = sqrt(ex * ex + ey * ey);
                if (!(r + sr[o] - ed > 0.0 && ed > 0.0)) {
                  hid[e] = 0;
                  hsp[e] = 0.0;
                  if (k < 0) k = e;
                }
              }
            }
            if (k >= 0) {
              hid[k] = j + 1;
              hsp[k] = sp;
            } else {
              atomicOr(a.err, ERR_CONTACTS);
            }
          }
        }
      }
      if (tang && !touch) {
        const int k = find(j + 1);
        if (k >= 0) {
          hid[k] = 0;
          hsp[k] = 0.0;
        }
      }
    }
    if (a.walls && near_wall) {
      const double cn = cnw;
      const double db = r - (py + 0.5);  // wall at y = -1/2: n = (0, -1), t = (1, 0)
      if (db > 0.0) {
        const double vn = -pvy;
        double fn, kt_c, ct_c;
        if (a.hertz) {
          fn = hertz_law(a, db, vn, r, mi, a.es_pw, a.gs_pw, &kt_c, &ct_c);
        } else {
          fn = kn * db + cn * vn;
          kt_c = a.kt;
          ct_c = 2.0 * zeta * sqrt(a.kt * mi);
        }
        fy += fn;
        if (tang) {
          const double l = r - 0.5 * db;
          const double vt = (pvx - a.uw_bot) + pom * l;
          const double ft = tangential_force(a, &hw[0], vt, fn, kt_c, ct_c, advance);
          fx += ft;
          tz += l * ft;
        }
      } else if (tang) {
        hw[0] = 0.0;
      }
      const double dt = r - ((a.ny - 0.5) - py);  // wall at y = ny - 1/2: n = (0, 1), t = (-1, 0)
      if (dt > 0.0) {
        const double vn = pvy;
        double fn, kt_c, ct_c;
        if (a.hertz) {
          fn = hertz_law(a, dt, vn, r, mi, a.es_pw, a.gs_pw, &kt_c, &ct_c);
        } else {
          fn = kn * dt + cn * vn;
          kt_c = a.kt;
          ct_c = 2.0 * zeta * sqrt(a.kt * mi);
        }
        fy += -fn;
        if (tang) {
          const double l = r - 0.5 * dt;
          const double vt = -(pvx - a.uw_top) + pom * l;
          const double ft = tangential_force(a, &hw[1], vt, fn, kt_c, ct_c, advance);
          fx += -ft;
          tz += l * ft;
        }
      } else if (tang) {
        hw[1] = 0.0;
      }
    }
    ox = fx;
    oy = fy;
    otz = tz;
  };
  const double cnw_p = 2.0 * zeta * sqrt(kn * m_p);
  // the springs stay in global memory, each disk's read and written by its own thread only (the
  // one-wavefront path works on LDS copies)
  auto contact = [&](double px, double py, double pvx, double pvy, double pom, bool advance,
                     double& ox, double& oy, double& otz) {
    contact_of(p, r, m_p, cnw_p, nn, nb, true, px, py, pvx, pvy, pom, s.hid + p * HK,
               s.hsp + p * HK, s.hw + p * 2, advance, ox, oy, otz);
  };

  bool rebuilt = false;
  if ((flags & 1) || a.build_lists) {
    // ---- neighbour list maintenance
    if (flags & 2) {
      rebuilt = true;
      if (have) {
        int cnt = 0;
        auto consider = [&](int j, double ox, double oy, double orad) {
          if (j == p) return;
          const double dx = nearest_image(ox - x, a.nx);
          double dy = oy - y;
          if (!a.walls) dy = nearest_image(dy, a.ny);
          const double reach = r + orad + DEM_SKIN;
          if (dx * dx + dy * dy < reach * reach) {
            if (cnt < NB_REG) {
#pragma unroll
              for (int u = 0; u < NB_REG; ++u)
                if (u == cnt) nb[u] = j;
            }
            if (cnt < NBMAX) s.nbr[p * NBMAX + cnt] = j;  // read back only by this thread
            ++cnt;
          }
        };
        // candidates in ascending id, eight at a time so their loads issue together
        constexpr int RB = 8;
        int j0 = 0;
        for (; j0 + RB <= np; j0 += RB) {
          double ox[RB], oy[RB], orad[RB];
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            ox[u] = sx[j0 + u];
            oy[u] = sy[j0 + u];
            orad[u] = sr[j0 + u];
          }
#pragma unroll
          for (int u = 0; u < RB; ++u) consider(j0 + u, ox[u], oy[u], orad[u]);
        }
        for (; j0 < np; ++j0) consider(j0, sx[j0], sy[j0], sr[j0]);
        if (cnt > NBMAX) {
          atomicOr(a.err, ERR_NBR);
          cnt = NBMAX;
        }
        nn = cnt;
        xref = x;
        yref = y;
      }
    }
  }
  if ((flags & 1) && (a.do_dem || a.init_contacts)) {  // table-only calls never move a disk
    if (a.init_contacts) {
      // the force of the present overlaps; no spring stretches here
      if (own) contact(x, y, vx, vy, om, false, fcx, fcy, tc);
      else {
        fcx = 0.0;
        fcy = 0.0;
        tc = 0.0;
      }
    } else {
      // ---- classify.  During the sub-steps a disk stays within B of its start: a quiet disk
      // (no contact force all step) moves on the parabola of its fixed hydrodynamic load, so
      // B = |V| + |a| / 2 plus a rounding margin; an active disk B = MAX_MOVE (moving further
      // latches ERR_MOVE); fixed and prescribed disks keep their place until the sub-steps end,
      // B = 0.  A free disk is active when its stored contact force is not zero, when the gap
      // to a neighbour is within the sum of both reaches, or the gap to a wall within its own.
      // Starting from every free disk quiet, the test is repeated until no disk changes; then
      // no quiet disk can touch anything in any sub-step (by induction over the sub-steps).
      // An active disk searches only its "close" neighbours, those within 2 MAX_MOVE: bit u of
      // cmask marks list slot u < NB_REG, cfar a close one further down the list.
      const double dt = 1.0 / a.n_sub, h = 0.5 * dt;
      const double m = m_p;
      const double I = 0.5 * m * r * r;
      auto neighbour = [&](int q) {
        int j = 0;
        if (q < NB_REG) {
#pragma unroll
          for (int u = 0; u < NB_REG; ++u)
            if (u == q) j = nb[u];
        } else {
          j = s.nbr[p * NBMAX + q];
        }
        return j;
      };
      auto within = [&](int j, double reach) {
        const double dx = nearest_image(sx[j] - x, a.nx);
        double dy = sy[j] - y;
        if (!a.walls) dy = nearest_image(dy, a.ny);
        const double g = r + sr[j] + reach;
        return dx * dx + dy * dy <= g * g;
      };
      bool active = own && (fcx != 0.0 || fcy != 0.0 || tc != 0.0);
      bool any_active = false;
      for (;;) {
        bool turned = false;
        if (own && !active) {
          for (int q = 0; q < nn && !turned; ++q) {
            const int j = neighbour(q);
            turned = within(j, Bq + sB[j]);
          }
          if (a.walls && (y - r + 0.5 <= Bq || (a.ny - 0.5) - y - r <= Bq)) turned = true;
        }
        // the OR's barrier also ends this round's reads of the reaches
        const int ro = block_or<NT>((turned ? 1 : 0) | (active || turned ? 2 : 0), s_or);
        any_active = (ro & 2) != 0;
        if (!(ro & 1)) break;
        if (turned) {
          active = true;
          sB[p] = Bq > MAX_MOVE ? Bq : MAX_MOVE;
        }
        __syncthreads();  // the new reaches are visible to the next round
      }
      bool cfar = false, nearw = false;
      unsigned cmask = 0u;
      if (active) {
        const double reach = 2.0 * MAX_MOVE;
        for (int q = 0; q < nn; ++q) {
          if (within(neighbour(q), reach)) {
            if (q < NB_REG) cmask |= 1u << q;
            else cfar = true;
          }
        }
        nearw = a.walls && (y - r + 0.5 <= reach || (a.ny - 0.5) - y - r <= reach);
      }
      if (own && !active) {
        // quiet: no contact force during the whole step, so the accelerations are the same in
        // every sub-step (computed once; the sub-step arithmetic is otherwise unchanged)
        const double ax = (0.0 + Fx) / m;
        const double ay = (0.0 + Fy) / m;
        const double hax = h * ax, hay = h * ay, hal = h * (Tz / I);
        for (int k = 0; k < a.n_sub; ++k) {
          vx = vx + hax;
          vy = vy + hay;
          x = wrap_coord(x + dt * vx, a.nx);
          y = y + dt * vy;
          if (!a.walls) y = wrap_coord(y, a.ny);
          om = om + hal;
          vx = vx + hax;
          vy = vy + hay;
          om = om + hal;
        }
        fcx = 0.0;
        fcy = 0.0;
        tc = 0.0;
      }
      if (any_active) {
        // active disks: up to 64 are packed into the first wavefront and run their sub-steps
        // there with wavefront-level ordering only; more than 64 use every owner thread and
        // block barriers
        if (threadIdx.x == 0) s_nact = 0;
        __syncthreads();
        int idx = -1;  // this disk's slot among the active ones
        if (own && active) {
          idx = atomicAdd(&s_nact, 1);
          if (idx < 64) {
            s_aid[idx] = p;
            s_ast[idx][0] = Fx; s_ast[idx][1] = Fy; s_ast[idx][2] = Tz;
            s_ast[idx][3] = fcx; s_ast[idx][4] = fcy; s_ast[idx][5] = om;
            s_ast[idx][6] = tc;
            if (tang) {
              for (int e = 0; e < HK; ++e) {
                s_hid[idx][e] = s.hid[p * HK + e];
                s_hsp[idx][e] = s.hsp[p * HK + e];
              }
              s_hw[idx][0] = s.hw[p * 2];
              s_hw[idx][1] = s.hw[p * 2 + 1];
            }
            s_awall[idx] = nearw ? 1 : 0;
            if (cfar) {  // search the whole list
              s_ann[idx] = nn;
#pragma unroll
              for (int u = 0; u < NB_REG; ++u) s_anb[idx][u] = nb[u];
            } else {     // only the close slots, in list order
              int c = 0;
#pragma unroll
              for (int u = 0; u < NB_REG; ++u)
                if ((cmask >> u) & 1u) s_anb[idx][c++] = nb[u];
              s_ann[idx] = c;
            }
          }
        }
        __syncthreads();
        const int nact = s_nact;
        if (nact > 0 && nact <= 64) {
          // every lane of wavefront 0 runs the loop (lanes past nact on slot 0's data, storing
          // nothing), so each wavefront barrier below is reached by the whole wavefront
          const int t = threadIdx.x;
          if (t < 64) {
            const bool act = t < nact;
            const int ts = act ? t : 0;
            const int i = s_aid[ts];
            const double ri = sr[i];
            const double mi_ = a.rho_s * M_PI * ri * ri;
            const double Ii = 0.5 * mi_ * ri * ri;
            const double im = 1.0 / mi_;
            const double cnw_i = 2.0 * zeta * sqrt(kn * mi_);
            double px = sx[i], py = sy[i], pvx = svx[i], pvy = svy[i];
            const double aFx = s_ast[ts][0], aFy = s_ast[ts][1], aTz = s_ast[ts][2];
            double afx = s_ast[ts][3], afy = s_ast[ts][4], aom = s_ast[ts][5];
            double atc = s_ast[ts][6];
            const int ann = s_ann[ts];
            const bool awall = s_awall[ts] != 0;
            int anb[NB_REG];
#pragma unroll
            for (int u = 0; u < NB_REG; ++u) anb[u] = s_anb[ts][u];
            const double hal = h * (aTz / Ii);
            for (int k = 0; k < a.n_sub; ++k) {
              const double ax = (afx + aFx) * im;
              const double ay = (afy + aFy) * im;
              pvx = pvx + h * ax;
              pvy = pvy + h * ay;
              px = wrap_coord(px + dt * pvx, a.nx);
              py = py + dt * pvy;
              if (!a.walls) py = wrap_coord(py, a.ny);
              aom = aom + (tang ? h * ((aTz + atc) / Ii) : hal);
              if (act) {
                sx[i] = px; sy[i] = py; svx[i] = pvx; svy[i] = pvy;
                som[i] = aom;
              }
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              __builtin_amdgcn_wave_barrier();
              if (act)
                contact_of(i, ri, mi_, cnw_i, ann, anb, awall, px, py, pvx, pvy, aom, s_hid[t],
                           s_hsp[t], s_hw[t], true, afx, afy, atc);
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              __builtin_amdgcn_wave_barrier();
              const double bx = (afx + aFx) * im;
              const double by = (afy + aFy) * im;
              pvx = pvx + h * bx;
              pvy = pvy + h * by;
              aom = aom + (tang ? h * ((aTz + atc) / Ii) : hal);
            }
            if (act) {
              svx[i] = pvx; svy[i] = pvy;
              s_ast[t][3] = afx; s_ast[t][4] = afy; s_ast[t][5] = aom;
              s_ast[t][6] = atc;
            }
          }
          __syncthreads();
          if (own && active) {
            fcx = s_ast[idx][3]; fcy = s_ast[idx][4]; om = s_ast[idx][5];
            tc = s_ast[idx][6];
            if (tang) {
              for (int e = 0; e < HK; ++e) {
                s.hid[p * HK + e] = s_hid[idx][e];
                s.hsp[p * HK + e] = s_hsp[idx][e];
              }
              s.hw[p * 2] = s_hw[idx][0];
              s.hw[p * 2 + 1] = s_hw[idx][1];
            }
            x = sx[p]; y = sy[p]; vx = svx[p]; vy = svy[p];
          }
        } else if (nact > 64) {
          // active disks: sub-steps synchronised across the block through LDS
          const double hal = h * (Tz / I);
          const double im = 1.0 / m;
          for (int k = 0; k < a.n_sub; ++k) {
            if (own && active) {
              const double ax = (fcx + Fx) * im;
              const double ay = (fcy + Fy) * im;
              vx = vx + h * ax;
              vy = vy + h * ay;
              x = wrap_coord(x + dt * vx, a.nx);
              y = y + dt * vy;
              if (!a.walls) y = wrap_coord(y, a.ny);
              om = om + (tang ? h * ((Tz + tc) / I) : hal);
              sx[p] = x; sy[p] = y; svx[p] = vx; svy[p] = vy;
              som[p] = om;
            }
            __syncthreads();
            if (own && active) contact(x, y, vx, vy, om, true, fcx, fcy, tc);
            __syncthreads();
            if (own && active) {
              const double ax = (fcx + Fx) * im;
              const double ay = (fcy + Fy) * im;
              vx = vx + h * ax;
              vy = vy + h * ay;
              om = om + (tang ? h * ((Tz + tc) / I) : hal);
            }
          }
        }
      }
    }
  }

  double nx_ = x, ny_ = y;
  if (a.do_dem && have) {
    if (mode == 2) {
      nx_ = wrap_coord(x + vx, a.nx);
      ny_ = y + vy;
      if (!a.walls) ny_ = wrap_coord(ny_, a.ny);
    }
  }
  // ---- table: tile box of the new position
  int4 nbx = make_int4(0, 0, 0, 0);
  if (a.do_table && have) {
    if (!isfinite(nx_) || !isfinite(ny_)) {
      nbx = make_int4(0, 0, 0, 0);
    } else if (!tile_box(nx_, ny_, r, a.nx, a.ny, a.walls, a.tiles_x, a.tiles_yg, a.tw, a.th,
                         &nbx)) {
      atomicOr(a.err, ERR_SLOTS);
      nbx = make_int4(0, 0, 0, 0);
    }
  }
  // ---- band masks: bit p mod 64 of word p / 64 of tile row t is set when disk p's box touches
  // the window's tile row t (lattice tile row t + ty_off of the tiles_yg the lattice has).  Built
  // in LDS ([MASK_WORDS][R] words for R rows at a time, R from the LDS the launch gives) with one
  // atomic OR per (disk, row) of its box, then stored word-major (coalesced).
  if (a.do_table) {
    unsigned long long* sm = (unsigned long long*)lds;
    const int nbands = a.tiles_y;
    const int R = a.lds_doubles / MASK_WORDS < nbands ? a.lds_doubles / MASK_WORDS : nbands;
    const bool any = have && nbx.y > 0;
    for (int t0 = 0; t0 < nbands; t0 += R) {
      const int tn = nbands - t0 < R ? nbands - t0 : R;
      __syncthreads();  // LDS is free (the DEM's tables, or the last chunk's stores, are done)
      for (int i = threadIdx.x; i < MASK_WORDS * R; i += NT) sm[i] = 0ull;
      __syncthreads();
      if (any)
        for (int k = 0; k < nbx.w; ++k) {
          int t = nbx.z + k;
          t = t < a.tiles_yg ? t : t - a.tiles_yg;
          t -= a.ty_off + t0;
          if (t >= 0 && t < tn) atomicOr(&sm[(p >> 6) * R + t], 1ull << (p & 63));
        }
      __syncthreads();
      for (int i = threadIdx.x; i < MASK_WORDS * tn; i += NT) {
        const int w = i / tn, t = i - w * tn;
        a.band_mask[(size_t)w * nbands + t0 + t] = sm[w * R + t];
      }
    }
  }

  // ---- all remaining global stores
  if (a.do_finalize && a.J && threadIdx.x == 0) *a.J += jsum;
  if (have) {
    if (a.do_finalize) {
      s.Fx[p] = Fx;
      s.Fy[p] = Fy;
      s.Tz[p] = Tz;
    }
    if (a.do_dem) {
      const double mdx = nearest_image(nx_ - x_start, a.nx);
      const double mdy = a.walls ? ny_ - y_start : nearest_image(ny_ - y_start, a.ny);
      const bool bad = !isfinite(nx_) || !isfinite(ny_) || !isfinite(vx) || !isfinite(vy) ||
                       !isfinite(om) || (a.walls && (ny_ < -0.5 || ny_ > a.ny - 0.5));
      const bool moved_far = mdx * mdx + mdy * mdy > MAX_MOVE * MAX_MOVE;
      if (bad) atomicOr(a.err, ERR_LEFT);
      if (moved_far) atomicOr(a.err, ERR_MOVE);
      s.x[p] = nx_; s.y[p] = ny_; s.vx[p] = vx; s.vy[p] = vy; s.om[p] = om;
    }
    if (a.do_dem || a.init_contacts) {
      s.fcx[p] = fcx;
      s.fcy[p] = fcy;
      s.tcz[p] = tc;
    }
    if (rebuilt) {
      s.nnbr[p] = nn;
      s.xref[p] = xref;
      s.yref[p] = yref;
    }
    if (a.do_table) {
      a.tab.box[p] = nbx;
      a.tab.pos[p] = make_double4(nx_, ny_, r, 0.0);
      a.tab.vel[p] = make_double4(vx, vy, om, 0.0);
    }
  }
  if (rebuilt && threadIdx.x == 0) *s.rebuild = 0;
}

}  // namespace imb
