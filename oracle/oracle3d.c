/*
 * oracle3d.c -- plain FP64 CPU oracle of the three-dimensional lattice step of Yang, Jing, Kwok &
 * Sobral, "A comprehensive study of coupled LBM-DEM with immersed moving boundary"
 * (arXiv:1809.07008): D3Q19 BGK lattice Boltzmann with the immersed moving boundary of spheres.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite may load this code (it is compiled into the same
 * liboracle.so as oracle.c).  It shares no code, header, table or helper with the HIP
 * implementation, nor with oracle.c; it is written from the paper's equations.
 *
 * What each part follows:
 *   Sec. 2, Eqs. (1)-(4), Table 1   D3Q19 BGK equation, equilibrium, moments; weights 1/3 (rest),
 *                                   1/18 (the six axis directions), 1/36 (the twelve diagonals).
 *   Sec. 2.2                        solid ratio of a cell by the paper's cell decomposition: the
 *                                   cell is split into n^3 equal sub-cells and eps is the share of
 *                                   sub-cell centres inside the sphere (a centre on the surface
 *                                   counts as outside).
 *   Eqs. (12)-(14)                  Noble-Torczynski solid collision and its weight B(eps, tau).
 *   Eqs. (15), (16)                 force and torque vectors; the printed sum is the momentum the
 *                                   fluid gains, so the force on the sphere is its negative.
 * Readings (the same as the two-dimensional oracle): the cell of node (x, y, z) is the unit cube
 * centred on it; x and z are periodic, y has half-way bounce-back walls at -1/2 and ny - 1/2 when
 * walls are on (periodic otherwise); body force G_i = 3 w_i rho (c_i . g) weighted by (1 - B_tot);
 * several spheres in one cell: eps_tot = min(1, sum eps_p), B_tot = B(eps_tot), B_p = B_tot
 * eps_p / sum eps_p; solid velocity at the node u_s = V + omega x d, d = node - centre (nearest
 * image); spheres are fixed or move by a prescribed velocity once per step (no DEM).
 *
 * Compile with -ffp-contract=off and without -ffast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#pragma STDC FP_CONTRACT OFF

#define Q3 19
#define SLOTS3 4 /* spheres sharing one cell */

/* D3Q19 directions (Table 1): rest; the six axis directions; the twelve face diagonals.  Each
 * direction is followed by its opposite. */
static const int E3[Q3][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static int opposite3(int i) { return i == 0 ? 0 : (i % 2 ? i + 1 : i - 1); }

static double weight3(int i) {
  if (i == 0) return 1.0 / 3.0;
  if (i <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

typedef struct {
  int32_t nx, ny, nz;
  int32_t walls;        /* 1: half-way bounce-back walls in y */
  int32_t eps_subcells; /* n of the n^3 sub-cell decomposition (>= 1) */
  double tau0;
  double gx, gy, gz;
  double rho0;
} ocfg3;

typedef struct {
  ocfg3 c;
  double *f;   /* [nz][ny][nx][Q3] post-stream */
  double *fp;  /* post-collision */
  int *nslot;  /* per cell: spheres covering it */
  int *spid;   /* [cell][SLOTS3] their ids */
  double *seps, *sdx, *sdy, *sdz;             /* solid ratio, lever arm */
  double *sfx, *sfy, *sfz, *stx, *sty, *stz;  /* per-cell force and torque contributions */
  int np;
  double *x, *y, *z, *r, *vx, *vy, *vz, *wx, *wy, *wz;
  int32_t *mode; /* 1 fixed, 2 prescribed */
  double *Fx, *Fy, *Fz, *Tx, *Ty, *Tz;
  long step;
} osim3;

/* ---------------------------------------------------------------- equilibrium, Eq. (2) */
static void equilibrium3(double rho, double ux, double uy, double uz, double feq[Q3]) {
  double uu = ux * ux + uy * uy + uz * uz;
  for (int i = 0; i < Q3; ++i) {
    double cu = E3[i][0] * ux + E3[i][1] * uy + E3[i][2] * uz;
    feq[i] = weight3(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* The paper's estimate of the solid ratio (Sec. 2.2): the unit cell centred at (dx, dy, dz) from
 * the sphere centre split into n^3 sub-cells; the share of sub-cell centres strictly inside. */
double o3_subcell_fraction(double r, double dx, double dy, double dz, int n) {
  if (n < 1) return 0.0;
  long inside = 0;
  for (int k = 0; k < n; ++k) {
    double zc = dz + ((k + 0.5) / n - 0.5);
    for (int j = 0; j < n; ++j) {
      double yc = dy + ((j + 0.5) / n - 0.5);
      for (int i = 0; i < n; ++i) {
        double xc = dx + ((i + 0.5) / n - 0.5);
        if (xc * xc + yc * yc + zc * zc < r * r) ++inside;
      }
    }
  }
  return (double)inside / ((double)n * (double)n * (double)n);
}

/* Weight of Eq. (14). */
static double weight_b3(double eps, double tau) {
  double a = tau - 0.5;
  return eps * a / ((1.0 - eps) + a);
}

/* ----------------------------------------------------------- collision of one cell
 *   f*_i = f_i + (1 - B_tot)(Omega^f_i + G_i) + sum_p B_p Omega^s_{p,i}            Eq. (13)
 *   Omega^s_{p,i} = f_{-i} - f_{-i}^eq(rho, u) + f_i^eq(rho, u_s) - f_i             Eq. (12)
 *   dF_p = -B_p sum_i Omega^s_{p,i} c_i = B_p (m - rho u_s),  dT_p = d x dF_p       Eqs. (15), (16)
 * (the inner sum of Eq. 15 in closed form: sum_i c_i f_i^eq(rho, v) = rho v). */
int o3_collide_cell(const double *f, int np, const double *eps, const double *d /*[np][3]*/,
                    const double *v /*[np][3]*/, const double *w /*[np][3]*/, double tau,
                    double gx, double gy, double gz, double *fout, double *dF /*[np][3]*/,
                    double *dT /*[np][3]*/, double *Bt_out) {
  double rho = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
  for (int i = 0; i < Q3; ++i) rho += f[i];
  for (int i = 0; i < Q3; ++i) {
    mx += E3[i][0] * f[i];
    my += E3[i][1] * f[i];
    mz += E3[i][2] * f[i];
  }
  double ux = mx / rho, uy = my / rho, uz = mz / rho;
  double feq[Q3];
  equilibrium3(rho, ux, uy, uz, feq);
  double S = 0.0;
  for (int p = 0; p < np; ++p) S += eps[p];
  double et = S < 1.0 ? S : 1.0;
  double Bt = weight_b3(et, tau);
  for (int i = 0; i < Q3; ++i) {
    double G = 3.0 * weight3(i) * rho * (E3[i][0] * gx + E3[i][1] * gy + E3[i][2] * gz);
    double Of = -(f[i] - feq[i]) / tau;
    fout[i] = f[i] + (1.0 - Bt) * (Of + G);
  }
  for (int p = 0; p < np; ++p) {
    double Bp = S > 0.0 ? Bt * (eps[p] / S) : 0.0;
    const double *dp = d + 3 * p, *vp = v + 3 * p, *wp = w + 3 * p;
    /* u_s = V + omega x d */
    double usx = vp[0] + (wp[1] * dp[2] - wp[2] * dp[1]);
    double usy = vp[1] + (wp[2] * dp[0] - wp[0] * dp[2]);
    double usz = vp[2] + (wp[0] * dp[1] - wp[1] * dp[0]);
    double feqs[Q3];
    equilibrium3(rho, usx, usy, usz, feqs);
    for (int i = 0; i < Q3; ++i) {
      int o = opposite3(i);
      double Os = f[o] - feq[o] + feqs[i] - f[i];
      fout[i] += Bp * Os;
    }
    double fx = Bp * (mx - rho * usx);
    double fy = Bp * (my - rho * usy);
    double fz = Bp * (mz - rho * usz);
    dF[3 * p] = fx;
    dF[3 * p + 1] = fy;
    dF[3 * p + 2] = fz;
    dT[3 * p] = dp[1] * fz - dp[2] * fy;
    dT[3 * p + 1] = dp[2] * fx - dp[0] * fz;
    dT[3 * p + 2] = dp[0] * fy - dp[1] * fx;
  }
  if (Bt_out) *Bt_out = Bt;
  return 0;
}

/* ------------------------------------------------------------------ simulation object */
static void *zalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

void o3_destroy(osim3 *s);

osim3 *o3_create(const ocfg3 *c) {
  if (!c || c->nx < 1 || c->ny < 2 || c->nz < 1 || !(c->tau0 > 0.5) || c->eps_subcells < 1)
    return NULL;
  osim3 *s = (osim3 *)calloc(1, sizeof(osim3));
  if (!s) return NULL;
  s->c = *c;
  size_t nc = (size_t)c->nx * c->ny * c->nz;
  s->f = (double *)zalloc(nc * Q3, sizeof(double));
  s->fp = (double *)zalloc(nc * Q3, sizeof(double));
  s->nslot = (int *)zalloc(nc, sizeof(int));
  s->spid = (int *)zalloc(nc * SLOTS3, sizeof(int));
  double **arrs[10] = {&s->seps, &s->sdx, &s->sdy, &s->sdz, &s->sfx,
                       &s->sfy,  &s->sfz, &s->stx, &s->sty, &s->stz};
  int ok = s->f && s->fp && s->nslot && s->spid;
  for (int k = 0; k < 10; ++k) {
    *arrs[k] = (double *)zalloc(nc * SLOTS3, sizeof(double));
    ok = ok && *arrs[k];
  }
  if (!ok) {
    o3_destroy(s);
    return NULL;
  }
  double feq[Q3];
  equilibrium3(c->rho0, 0.0, 0.0, 0.0, feq);
  for (size_t k = 0; k < nc; ++k)
    for (int i = 0; i < Q3; ++i) s->f[k * Q3 + i] = feq[i];
  return s;
}

static void free_spheres(osim3 *s) {
  double **a[16] = {&s->x, &s->y, &s->z, &s->r, &s->vx, &s->vy, &s->vz, &s->wx,
                    &s->wy, &s->wz, &s->Fx, &s->Fy, &s->Fz, &s->Tx, &s->Ty, &s->Tz};
  for (int k = 0; k < 16; ++k) {
    free(*a[k]);
    *a[k] = NULL;
  }
  free(s->mode);
  s->mode = NULL;
  s->np = 0;
}

void o3_destroy(osim3 *s) {
  if (!s) return;
  free(s->f); free(s->fp); free(s->nslot); free(s->spid);
  free(s->seps); free(s->sdx); free(s->sdy); free(s->sdz);
  free(s->sfx); free(s->sfy); free(s->sfz); free(s->stx); free(s->sty); free(s->stz);
  free_spheres(s);
  free(s);
}

/* f = f^eq(rho, u) everywhere. */
int o3_init_equilibrium(osim3 *s, double rho, double ux, double uy, double uz) {
  double feq[Q3];
  equilibrium3(rho, ux, uy, uz, feq);
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
  for (size_t k = 0; k < nc; ++k)
    for (int i = 0; i < Q3; ++i) s->f[k * Q3 + i] = feq[i];
  return 0;
}

/* Exchange format: [q][z][y][x], post-stream. */
int o3_set_populations(osim3 *s, const double *fq) {
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
  for (int i = 0; i < Q3; ++i)
    for (size_t k = 0; k < nc; ++k) s->f[k * Q3 + i] = fq[(size_t)i * nc + k];
  return 0;
}

int o3_get_populations(const osim3 *s, double *fq) {
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
  for (int i = 0; i < Q3; ++i)
    for (size_t k = 0; k < nc; ++k) fq[(size_t)i * nc + k] = s->f[k * Q3 + i];
  return 0;
}

int o3_get_fields(const osim3 *s, double *rho, double *ux, double *uy, double *uz) {
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
  for (size_t k = 0; k < nc; ++k) {
    const double *f = s->f + k * Q3;
    double r = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (int i = 0; i < Q3; ++i) r += f[i];
    for (int i = 0; i < Q3; ++i) {
      mx += E3[i][0] * f[i];
      my += E3[i][1] * f[i];
      mz += E3[i][2] * f[i];
    }
    if (rho) rho[k] = r;
    if (ux) ux[k] = mx / r;
    if (uy) uy[k] = my / r;
    if (uz) uz[k] = mz / r;
  }
  return 0;
}

/* Spheres: centre, radius, velocity, angular velocity, mode (1 fixed, 2 prescribed). */
int o3_set_spheres(osim3 *s, int n, const double *x, const double *y, const double *z,
                   const double *r, const double *vx, const double *vy, const double *vz,
                   const double *wx, const double *wy, const double *wz, const int32_t *mode) {
  if (n < 0) return -1;
  for (int p = 0; p < n; ++p)
    if (!(r[p] > 0.0) || (mode[p] != 1 && mode[p] != 2)) return -1;
  free_spheres(s);
  double **a[16] = {&s->x, &s->y, &s->z, &s->r, &s->vx, &s->vy, &s->vz, &s->wx,
                    &s->wy, &s->wz, &s->Fx, &s->Fy, &s->Fz, &s->Tx, &s->Ty, &s->Tz};
  for (int k = 0; k < 16; ++k) {
    *a[k] = (double *)zalloc((size_t)n, sizeof(double));
    if (!*a[k]) return -2;
  }
  s->mode = (int32_t *)zalloc((size_t)n, sizeof(int32_t));
  if (!s->mode) return -2;
  const double *src[10] = {x, y, z, r, vx, vy, vz, wx, wy, wz};
  for (int k = 0; k < 10; ++k)
    for (int p = 0; p < n; ++p) (*a[k])[p] = src[k][p];
  for (int p = 0; p < n; ++p) s->mode[p] = mode[p];
  s->np = n;
  return 0;
}

/* Offset of a cell from a sphere centre along one axis: the nearest periodic image when the
 * axis is periodic, from the integer cell offset and the fractional part of the centre. */
static double axis_offset(int cell, double centre, int n, int periodic) {
  double fl = floor(centre);
  long di = (long)cell - (long)fl;
  if (periodic) {
    if (di > n / 2) di -= n;
    else if (di < -(n / 2)) di += n;
  }
  return (double)di - (centre - fl);
}

/* For every cell: the spheres covering it (ascending id), their solid ratios and lever arms.
 * Only cells within one cell of a sphere's bounding box can have eps > 0. */
static int map_spheres(osim3 *s) {
  int nx = s->c.nx, ny = s->c.ny, nz = s->c.nz, walls = s->c.walls;
  memset(s->nslot, 0, sizeof(int) * (size_t)nx * ny * nz);
  for (int p = 0; p < s->np; ++p) {
    double X = s->x[p], Y = s->y[p], Z = s->z[p], r = s->r[p];
    int ix0 = (int)floor(X - r - 0.5), ix1 = (int)ceil(X + r + 0.5);
    int iy0 = (int)floor(Y - r - 0.5), iy1 = (int)ceil(Y + r + 0.5);
    int iz0 = (int)floor(Z - r - 0.5), iz1 = (int)ceil(Z + r + 0.5);
    if (walls) {
      if (iy0 < 0) iy0 = 0;
      if (iy1 > ny - 1) iy1 = ny - 1;
    }
    for (int iz = iz0; iz <= iz1; ++iz) {
      int zw = ((iz % nz) + nz) % nz;
      double dz = axis_offset(zw, Z, nz, 1);
      for (int iy = iy0; iy <= iy1; ++iy) {
        int yw = ((iy % ny) + ny) % ny;
        double dy = axis_offset(yw, Y, ny, !walls);
        for (int ix = ix0; ix <= ix1; ++ix) {
          int xw = ((ix % nx) + nx) % nx;
          double dx = axis_offset(xw, X, nx, 1);
          double e = o3_subcell_fraction(r, dx, dy, dz, s->c.eps_subcells);
          if (e > 0.0) {
            size_t k = ((size_t)zw * ny + yw) * nx + xw;
            int ns = s->nslot[k];
            if (ns >= SLOTS3) return -3;
            /* a sphere wider than the lattice would meet a cell twice */
            for (int q = 0; q < ns; ++q)
              if (s->spid[k * SLOTS3 + q] == p) return -3;
            s->spid[k * SLOTS3 + ns] = p;
            s->seps[k * SLOTS3 + ns] = e;
            s->sdx[k * SLOTS3 + ns] = dx;
            s->sdy[k * SLOTS3 + ns] = dy;
            s->sdz[k * SLOTS3 + ns] = dz;
            s->nslot[k] = ns + 1;
          }
        }
      }
    }
  }
  return 0;
}

static void collide_all3(osim3 *s) {
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
#pragma omp parallel for schedule(static)
  for (long kk = 0; kk < (long)nc; ++kk) {
    size_t k = (size_t)kk;
    int ns = s->nslot[k];
    double eps[SLOTS3], d[3 * SLOTS3], v[3 * SLOTS3], w[3 * SLOTS3], dF[3 * SLOTS3],
        dT[3 * SLOTS3];
    for (int q = 0; q < ns; ++q) {
      int p = s->spid[k * SLOTS3 + q];
      eps[q] = s->seps[k * SLOTS3 + q];
      d[3 * q] = s->sdx[k * SLOTS3 + q];
      d[3 * q + 1] = s->sdy[k * SLOTS3 + q];
      d[3 * q + 2] = s->sdz[k * SLOTS3 + q];
      v[3 * q] = s->vx[p]; v[3 * q + 1] = s->vy[p]; v[3 * q + 2] = s->vz[p];
      w[3 * q] = s->wx[p]; w[3 * q + 1] = s->wy[p]; w[3 * q + 2] = s->wz[p];
    }
    o3_collide_cell(s->f + k * Q3, ns, eps, d, v, w, s->c.tau0, s->c.gx, s->c.gy, s->c.gz,
                    s->fp + k * Q3, dF, dT, NULL);
    for (int q = 0; q < ns; ++q) {
      s->sfx[k * SLOTS3 + q] = dF[3 * q];
      s->sfy[k * SLOTS3 + q] = dF[3 * q + 1];
      s->sfz[k * SLOTS3 + q] = dF[3 * q + 2];
      s->stx[k * SLOTS3 + q] = dT[3 * q];
      s->sty[k * SLOTS3 + q] = dT[3 * q + 1];
      s->stz[k * SLOTS3 + q] = dT[3 * q + 2];
    }
  }
}

/* Streaming (left side of Eq. 1): push f*_i to the neighbour along c_i; periodic in x and z; a
 * link leaving through a wall returns to its own node in the opposite direction. */
static void stream_all3(osim3 *s) {
  int nx = s->c.nx, ny = s->c.ny, nz = s->c.nz;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const double *fp = s->fp + (((size_t)z * ny + y) * nx + x) * Q3;
        for (int i = 0; i < Q3; ++i) {
          int xn = ((x + E3[i][0]) % nx + nx) % nx;
          int zn = ((z + E3[i][2]) % nz + nz) % nz;
          int yn = y + E3[i][1];
          if (yn < 0 || yn >= ny) {
            if (s->c.walls) {
              s->f[(((size_t)z * ny + y) * nx + x) * Q3 + opposite3(i)] = fp[i];
              continue;
            }
            yn = (yn + ny) % ny;
          }
          s->f[(((size_t)zn * ny + yn) * nx + xn) * Q3 + i] = fp[i];
        }
      }
}

static void sum_forces3(osim3 *s) {
  for (int p = 0; p < s->np; ++p) s->Fx[p] = s->Fy[p] = s->Fz[p] = s->Tx[p] = s->Ty[p] = s->Tz[p] = 0.0;
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
  for (size_t k = 0; k < nc; ++k)
    for (int q = 0; q < s->nslot[k]; ++q) {
      int p = s->spid[k * SLOTS3 + q];
      size_t j = k * SLOTS3 + q;
      s->Fx[p] += s->sfx[j]; s->Fy[p] += s->sfy[j]; s->Fz[p] += s->sfz[j];
      s->Tx[p] += s->stx[j]; s->Ty[p] += s->sty[j]; s->Tz[p] += s->stz[j];
    }
}

static double wrap3(double v, int n) {
  if (v >= n) v -= n;
  else if (v < 0.0) v += n;
  return v;
}

int o3_step(osim3 *s, int nsteps) {
  for (int n = 0; n < nsteps; ++n) {
    int rc = map_spheres(s);
    if (rc) return rc;
    collide_all3(s);
    stream_all3(s);
    sum_forces3(s);
    for (int p = 0; p < s->np; ++p) {
      if (s->mode[p] != 2) continue;
      s->x[p] = wrap3(s->x[p] + s->vx[p], s->c.nx);
      s->y[p] = s->y[p] + s->vy[p];
      if (!s->c.walls) s->y[p] = wrap3(s->y[p], s->c.ny);
      s->z[p] = wrap3(s->z[p] + s->vz[p], s->c.nz);
    }
    s->step++;
  }
  return 0;
}

/* Force and torque on each sphere of the last step (Eqs. 15, 16, on the sphere). */
int o3_get_forces(const osim3 *s, double *F /*[np][3]*/, double *T /*[np][3]*/) {
  for (int p = 0; p < s->np; ++p) {
    F[3 * p] = s->Fx[p]; F[3 * p + 1] = s->Fy[p]; F[3 * p + 2] = s->Fz[p];
    T[3 * p] = s->Tx[p]; T[3 * p + 1] = s->Ty[p]; T[3 * p + 2] = s->Tz[p];
  }
  return 0;
}

/* Conditioning scales of each sphere's force and torque of the last step (tests): the sums over
 * its covered cells of |dF| and of |d| |dF|. */
int o3_force_scales(const osim3 *s, double *sF, double *sT) {
  for (int p = 0; p < s->np; ++p) sF[p] = sT[p] = 0.0;
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
  for (size_t k = 0; k < nc; ++k)
    for (int q = 0; q < s->nslot[k]; ++q) {
      size_t j = k * SLOTS3 + q;
      int p = s->spid[j];
      double f = sqrt(s->sfx[j] * s->sfx[j] + s->sfy[j] * s->sfy[j] + s->sfz[j] * s->sfz[j]);
      sF[p] += f;
      sT[p] += sqrt(s->sdx[j] * s->sdx[j] + s->sdy[j] * s->sdy[j] + s->sdz[j] * s->sdz[j]) * f;
    }
  return 0;
}

int o3_get_spheres(const osim3 *s, double *x, double *y, double *z) {
  for (int p = 0; p < s->np; ++p) {
    x[p] = s->x[p];
    y[p] = s->y[p];
    z[p] = s->z[p];
  }
  return 0;
}

/* eps_tot of every cell ([z][y][x]) for the current sphere positions. */
int o3_solid_field(osim3 *s, double *eps) {
  int rc = map_spheres(s);
  if (rc) return rc;
  size_t nc = (size_t)s->c.nx * s->c.ny * s->c.nz;
  for (size_t k = 0; k < nc; ++k) {
    double S = 0.0;
    for (int q = 0; q < s->nslot[k]; ++q) S += s->seps[k * SLOTS3 + q];
    eps[k] = S;
  }
  return 0;
}
