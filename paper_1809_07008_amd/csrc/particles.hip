// particles.hip -- the particle phase of a coupled step, one workgroup:
//   1. hydrodynamic force and torque on each disk: sum of the disk's per-tile partial sums
//      (Eqs. 15, 16), in slot order (deterministic);
//   2. DEM (Sec. 2.1, 2.3): N_sub velocity-Verlet (kick-drift-kick) sub-cycles of dt = 1/N_sub
//      (Eq. 17) with the hydrodynamic load held fixed; normal linear spring-dashpot contacts
//      between disks and with the walls (Eqs. 7, 8); the contact force is evaluated after each
//      drift from the new positions and half-step velocities and reused by the next kick;
//      prescribed disks move by V once per step, fixed disks stay;
//   3. the disk table (tile box, position, velocity) that the next lattice step reads.
// Contacts are searched in a Verlet neighbour list (skin DEM_SKIN) rebuilt whenever a disk has
// moved more than DEM_SKIN/2 - MAX_MOVE since the last build; a disk moving more than MAX_MOVE
// in one step latches ERR_MOVE, so no contact is ever missed silently.
// Readings: damping ratio zeta with c_n = 2 zeta sqrt(k_n m_eff); m = rho_s pi r^2, I = m r^2/2;
// no tangential force and no gravity.
#include "step.h"

namespace imb {

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

__device__ inline double block_sum(double v, double* s_red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) s_red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < PBLOCK / 64; ++w) t += s_red[w];
  __syncthreads();
  return t;
}

__device__ inline int block_or(int v, int* s_flag) {
  if (threadIdx.x == 0) *s_flag = 0;
  __syncthreads();
  if (v) atomicOr(s_flag, v);
  __syncthreads();
  const int r = *s_flag;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(PBLOCK) void k_particle_phase(ParticleArgs a) {
#pragma clang fp contract(off)
  extern __shared__ double lds[];
  __shared__ double s_red[PBLOCK / 64];
  __shared__ int s_flag;
  const int np = a.np, p = threadIdx.x;
  const bool have = p < np;
  double* sx = lds;
  double* sy = sx + np;
  double* svx = sy + np;
  double* svy = svx + np;
  double* sr = svy + np;
  int* smode = (int*)(sr + np);
  ParticleState& s = a.s;

  // 1. forces of the step that just ran
  if (a.do_finalize) {
    double jl = 0.0;
    if (have) {
      const int4 b = a.tab.box[p];
      const int ns = b.y * b.w;
      double fx = 0.0, fy = 0.0, tz = 0.0;
      for (int k = 0; k < ns; ++k) {
        const double4 v = a.partials[(long long)p * MAXSLOT + k];
        fx += v.x;
        fy += v.y;
        tz += v.z;
      }
      s.Fx[p] = fx;
      s.Fy[p] = fy;
      s.Tz[p] = tz;
      if (a.J) {
        if (a.wfx) jl += a.wfx[p] * fx;
        if (a.wfy) jl += a.wfy[p] * fy;
        if (a.wtz) jl += a.wtz[p] * tz;
      }
    }
    if (a.J) {
      const double t = block_sum(jl, s_red);
      if (threadIdx.x == 0) *a.J += t;
    }
  }

  double x = 0, y = 0, vx = 0, vy = 0, om = 0, r = 0;
  int mode = 1;
  if (have) {
    x = s.x[p]; y = s.y[p]; vx = s.vx[p]; vy = s.vy[p]; om = s.om[p]; r = s.r[p];
    mode = s.mode[p];
    sx[p] = x; sy[p] = y; svx[p] = vx; svy[p] = vy; sr[p] = r; smode[p] = mode;
  }
  __syncthreads();

  const bool need_dem = a.do_dem || a.init_contacts;
  if (need_dem) {
    const int any_free = block_or(have && mode == 0 ? 1 : 0, &s_flag);
    if (any_free) {
      // neighbour list maintenance
      int want = 0;
      if (have) {
        const double ddx = nearest_image(x - s.xref[p], a.nx);
        const double ddy = a.walls ? y - s.yref[p] : nearest_image(y - s.yref[p], a.ny);
        want = (ddx * ddx + ddy * ddy > (0.5 * DEM_SKIN - MAX_MOVE) * (0.5 * DEM_SKIN - MAX_MOVE));
      }
      if (threadIdx.x == 0 && *s.rebuild) want = 1;
      const int rebuild = block_or(want, &s_flag);
      if (rebuild) {
        if (have) {
          int cnt = 0;
          for (int j = 0; j < np; ++j) {
            if (j == p) continue;
            double dx = nearest_image(sx[j] - x, a.nx);
            double dy = sy[j] - y;
            if (!a.walls) dy = nearest_image(dy, a.ny);
            const double reach = r + sr[j] + DEM_SKIN;
            if (dx * dx + dy * dy < reach * reach) {
              if (cnt < NBMAX) s.nbr[p * NBMAX + cnt] = j;
              ++cnt;
            }
          }
          if (cnt > NBMAX) {
            atomicOr(a.err, ERR_NBR);
            cnt = NBMAX;
          }
          s.nnbr[p] = cnt;
          s.xref[p] = x;
          s.yref[p] = y;
        }
        if (threadIdx.x == 0) *s.rebuild = 0;
      }
      __syncthreads();

      const double kn = a.kn, zeta = a.zeta;
      const bool own = have && mode == 0;
      const double mi = a.rho_s * M_PI * r * r;
      const int nn = own ? s.nnbr[p] : 0;
      auto contact = [&](double& fcx, double& fcy) {
        double fx = 0.0, fy = 0.0;
        for (int q = 0; q < nn; ++q) {
          const int j = s.nbr[p * NBMAX + q];
          double dx = sx[j] - sx[p];
          double dy = sy[j] - sy[p];
          dx = nearest_image(dx, a.nx);
          if (!a.walls) dy = nearest_image(dy, a.ny);
          const double dist = sqrt(dx * dx + dy * dy);
          const double delta = r + sr[j] - dist;
          if (delta > 0.0 && dist > 0.0) {
            const double nxu = dx / dist, nyu = dy / dist;
            const double vn = (svx[p] - svx[j]) * nxu + (svy[p] - svy[j]) * nyu;
            const double mj = a.rho_s * M_PI * sr[j] * sr[j];
            const double meff = mi * mj / (mi + mj);
            const double cn = 2.0 * zeta * sqrt(kn * meff);
            const double fn = kn * delta + cn * vn;
            fx += -fn * nxu;
            fy += -fn * nyu;
          }
        }
        if (a.walls) {
          const double cn = 2.0 * zeta * sqrt(kn * mi);
          const double db = r - (sy[p] + 0.5);
          if (db > 0.0) {
            const double vn = -svy[p];
            fy += kn * db + cn * vn;
          }
          const double dt = r - ((a.ny - 0.5) - sy[p]);
          if (dt > 0.0) {
            const double vn = svy[p];
            fy += -(kn * dt + cn * vn);
          }
        }
        fcx = fx;
        fcy = fy;
      };

      if (a.init_contacts) {
        if (own) {
          double fcx, fcy;
          contact(fcx, fcy);
          s.fcx[p] = fcx;
          s.fcy[p] = fcy;
        } else if (have) {
          s.fcx[p] = 0.0;
          s.fcy[p] = 0.0;
        }
      } else {
        double fcx = own ? s.fcx[p] : 0.0, fcy = own ? s.fcy[p] : 0.0;
        const double Fx = own ? s.Fx[p] : 0.0, Fy = own ? s.Fy[p] : 0.0;
        const double Tz = own ? s.Tz[p] : 0.0;
        const double I = 0.5 * mi * r * r;
        const double dt = 1.0 / a.n_sub, h = 0.5 * dt;
        for (int k = 0; k < a.n_sub; ++k) {
          if (own) {
            const double ax = (fcx + Fx) / mi;
            const double ay = (fcy + Fy) / mi;
            vx = vx + h * ax;
            vy = vy + h * ay;
            x = wrap_coord(x + dt * vx, a.nx);
            y = y + dt * vy;
            if (!a.walls) y = wrap_coord(y, a.ny);
            om = om + h * (Tz / I);
            sx[p] = x; sy[p] = y; svx[p] = vx; svy[p] = vy;
          }
          __syncthreads();
          if (own) contact(fcx, fcy);
          __syncthreads();
          if (own) {
            const double ax = (fcx + Fx) / mi;
            const double ay = (fcy + Fy) / mi;
            vx = vx + h * ax;
            vy = vy + h * ay;
            om = om + h * (Tz / I);
          }
        }
        if (own) {
          s.fcx[p] = fcx;
          s.fcy[p] = fcy;
        }
      }
    }
  }

  if (a.do_dem && have) {
    // s.x / s.y still hold the positions at the start of this step
    if (mode == 2) {
      x = wrap_coord(x + vx, a.nx);
      y = y + vy;
      if (!a.walls) y = wrap_coord(y, a.ny);
    }
    const double mdx = nearest_image(x - s.x[p], a.nx);
    const double mdy = a.walls ? y - s.y[p] : nearest_image(y - s.y[p], a.ny);
    if (!isfinite(x) || !isfinite(y) || !isfinite(vx) || !isfinite(vy) || !isfinite(om))
      atomicOr(a.err, ERR_LEFT);
    if (mdx * mdx + mdy * mdy > MAX_MOVE * MAX_MOVE) atomicOr(a.err, ERR_MOVE);
    if (a.walls && (y < -0.5 || y > a.ny - 0.5)) atomicOr(a.err, ERR_LEFT);
    s.x[p] = x; s.y[p] = y; s.vx[p] = vx; s.vy[p] = vy; s.om[p] = om;
  }

  if (a.do_table && have) {
    int4 b;
    if (!isfinite(x) || !isfinite(y)) {  // latched above; keep the table in range
      b = make_int4(0, 0, 0, 0);
    } else if (!tile_box(x, y, r, a.nx, a.ny, a.walls, a.tiles_x, a.tiles_y, a.tw, a.th, &b)) {
      atomicOr(a.err, ERR_SLOTS);
      b = make_int4(0, 0, 0, 0);
    }
    a.tab.box[p] = b;
    a.tab.pos[p] = make_double4(x, y, r, 0.0);
    a.tab.vel[p] = make_double4(vx, vy, om, 0.0);
  }
}

void launch_particle_phase(const ParticleArgs& a, hipStream_t s) {
  const size_t lds = (size_t)a.np * (5 * sizeof(double) + sizeof(int));
  hipLaunchKernelGGL(k_particle_phase, dim3(1), dim3(PBLOCK), lds, s, a);
}

}  // namespace imb
