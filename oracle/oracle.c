/*
 * oracle.c -- plain FP64 CPU oracle of the coupled lattice-Boltzmann / immersed-moving-boundary /
 * discrete-element time step of Yang, Jing, Kwok & Sobral, "A comprehensive study of coupled
 * LBM-DEM with immersed moving boundary" (arXiv:1809.07008).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code, header, table or helper with the HIP
 * implementation; it is written from the paper's equations so that the two can be compared.
 *
 * It is deliberately slow and literal: one cell at a time, every quantity computed the way the
 * paper defines it, arrays of structures ([y][x][q]) so that nothing resembles the GPU layout.
 * OpenMP only splits independent rows; it never changes the order of any floating-point sum.
 *
 * What each part follows (equation numbers of the paper):
 *   Sec. 2, Eqs. (1)-(4)  BGK lattice Boltzmann equation, Maxwellian equilibrium, moments.
 *                         The paper's lattice is D3Q19 (Table 1); this oracle is two-dimensional and
 *                         uses the D2Q9 set with weights 4/9, 1/9, 1/36 and c_s^2 = 1/3.
 *   Sec. 2.2             solid ratio of a cell = covered area / cell area (Fig. 3a), computed
 *                         exactly for a disk; optionally the paper's own estimate by cell
 *                         decomposition (fraction of n x n sub-cell centres inside the disk).
 *   Eq. (12)             Noble-Torczynski solid collision operator.
 *   Eq. (13), Eq. (14)   blended collision and its weight B(eps, tau).
 *   Eqs. (15), (16)      hydrodynamic force and torque; the printed sum is the momentum the fluid
 *                         gains, so the force on the particle is its negative.
 *   Eqs. (7), (8)        DEM overlap and normal spring-dashpot force; with kt, mu a tangential
 *                        spring-dashpot with a Coulomb limit (contact_forces, tangential); or the
 *                        simplified Hertz-Mindlin law Sec. 2.1 adopts (normal_law).
 *   Eqs. (10), (11), (17) Newton's equations integrated by velocity Verlet with N_sub sub-cycles per
 *                         lattice step, the hydrodynamic force and torque held fixed (Sec. 2.3).
 *   Sec. 3.3.2           Smagorinsky sub-grid model (closed form of the Hou et al. model, see
 *                         smagorinsky_tau below).
 *
 * Readings taken where the paper is silent (each one is also listed in the design notes):
 *   - node (x,y) owns the unit cell [x-1/2,x+1/2]x[y-1/2,y+1/2]; x is periodic; with walls, the
 *     walls are half-way (y = -1/2 and y = ny-1/2) and act by link-wise bounce-back (Sec. 3.1.1
 *     states no-slip walls enforced by bounce-back).
 *   - driving body force: first-order term G_i = 3 w_i rho (c_i . g), weighted by (1 - B_tot) so
 *     solid interiors are not driven; u = m / rho.
 *   - a cell covered by several disks: eps_tot = min(1, sum eps_p), B_tot = B(eps_tot),
 *     B_p = B_tot * (eps_p / sum eps_p).
 *   - cycle order: map disks -> collide -> stream -> forces -> DEM sub-cycles (Fig. 4 entered at the
 *     mapping stage).
 *   - DEM damping ratio zeta: c_n = 2 zeta sqrt(k_n m_eff); m = rho_s pi r^2, I = m r^2 / 2.
 *   - walls moving along x (plane Couette flow): bounce-back with the wall's momentum,
 *     f*_i - 6 w_i rho0 (c_i . u_w) (Ladd), the reference density taken at the wall.
 *
 * Compile with -ffp-contract=off (no fused multiply-add) and without -ffast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#pragma STDC FP_CONTRACT OFF

#define NQ 9
#define MAX_SLOTS 4 /* disks sharing one cell; three disks cannot share a unit cell unless they overlap */

/* D2Q9 directions: rest, +x, +y, -x, -y, (+1,+1), (-1,+1), (-1,-1), (+1,-1). */
static const int CX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WQ[NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

enum { O_OK = 0, O_EINVAL = -1, O_ENOMEM = -2, O_EOVERFLOW = -3 };

typedef struct {
  int32_t nx, ny;
  int32_t walls;  /* 1: half-way bounce-back walls in y; 0: periodic in y */
  int32_t n_sub;  /* DEM sub-cycles per lattice step (Eq. 17) */
  double tau0;    /* molecular relaxation time */
  double cs;      /* Smagorinsky constant (0 disables the model) */
  double gx, gy;  /* body-force acceleration on the fluid */
  double rho0;    /* reference density (initial state) */
  double kn;      /* normal contact stiffness */
  double zeta;    /* normal damping ratio */
  double rho_s;   /* particle density (mass per unit area) */
  int32_t eps_subcells; /* 0: exact solid ratio; n > 0: the n x n sub-cell estimate */
  double uw_bot, uw_top; /* x-velocity of the wall at y = -1/2 and of the wall at y = ny - 1/2 */
  double kt;      /* tangential contact stiffness (0 with mu = 0: normal force only) */
  double mu;      /* Coulomb friction coefficient of the tangential contact force */
  int32_t contact_model; /* 0: linear spring-dashpot (kn, kt); 1: Hertz-Mindlin (young, poisson) */
  double young;   /* Young's modulus of the disks (Hertz-Mindlin) */
  double poisson; /* Poisson's ratio of the disks (Hertz-Mindlin) */
} ocfg;

typedef struct {
  ocfg c;
  double *f;    /* [ny][nx][NQ] post-stream populations */
  double *fp;   /* [ny][nx][NQ] post-collision populations */
  int *nslot;   /* [ny*nx] disks covering the cell */
  int *spid;    /* [ny*nx][MAX_SLOTS] their ids, ascending */
  double *seps; /* [ny*nx][MAX_SLOTS] their solid ratios */
  double *sdx, *sdy;            /* lever arm cell - centre (nearest image) */
  double *sfx, *sfy, *stz;      /* per-cell force / torque contributions */
  int np;
  double *x, *y, *r, *vx, *vy, *om;
  int32_t *mode;                /* 0 free (DEM), 1 fixed, 2 prescribed velocity */
  double *fcx, *fcy;            /* contact force at the last DEM evaluation */
  double *tcz;                  /* contact torque at the last DEM evaluation */
  double *ht;                   /* [np][np] tangential spring of pair (i, j), seen from i */
  double *hwb, *hwt;            /* tangential spring against the bottom / top wall */
  double *Fx, *Fy, *Tz;         /* hydrodynamic force / torque of the last step */
  long step;
} osim;

/* ---------------------------------------------------------------- equilibrium, Eq. (2) */
static void equilibrium(double rho, double ux, double uy, double feq[NQ]) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < NQ; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    feq[i] = WQ[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* The paper's estimate of the solid ratio (Sec. 2.2): the unit cell centred at (dx, dy) from the
 * disk centre is split into n x n equal sub-cells, and eps is the fraction of sub-cell centres
 * lying inside the disk (strictly: a centre on the circle counts as outside). */
double o_subcell_fraction(double r, double dx, double dy, int n) {
  if (n < 1) return 0.0;
  int inside = 0;
  for (int j = 0; j < n; ++j) {
    const double yc = dy + ((j + 0.5) / n - 0.5);
    for (int i = 0; i < n; ++i) {
      const double xc = dx + ((i + 0.5) / n - 0.5);
      if (xc * xc + yc * yc < r * r) ++inside;
    }
  }
  return (double)inside / ((double)n * (double)n);
}

/* Weight of Eq. (14): B(eps, tau) = eps (tau - 1/2) / ((1 - eps) + (tau - 1/2)). */
double o_weight(double eps, double tau) {
  double a = tau - 0.5;
  return eps * a / ((1.0 - eps) + a);
}

/* Smagorinsky relaxation time (Sec. 3.3.2 cites Hou et al. 1996 without printing it).
 * With dx = dt = 1: strain rate |S| = 3 sqrt(2) |Pi| / (2 rho tau_eff) from the non-equilibrium
 * momentum flux Pi = sum_i c_i c_i (f_i - f_i^eq); eddy viscosity nu_t = C_s^2 |S|;
 * tau_eff = tau0 + 3 nu_t.  Solving the resulting quadratic for tau_eff gives the expression below. */
static double smagorinsky_tau(double tau0, double cs, double rho, const double f[NQ],
                              const double feq[NQ]) {
  if (cs <= 0.0) return tau0;
  double pxx = 0.0, pxy = 0.0, pyy = 0.0;
  for (int i = 0; i < NQ; ++i) {
    double neq = f[i] - feq[i];
    pxx += (CX[i] * CX[i]) * neq;
    pxy += (CX[i] * CY[i]) * neq;
    pyy += (CY[i] * CY[i]) * neq;
  }
  double pn = sqrt(pxx * pxx + 2.0 * pxy * pxy + pyy * pyy);
  return 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * pn / rho));
}

/* ------------------------------------------------------- solid ratio of one cell (Sec. 2.2)
 * Exact area of  disk(radius r, centre at the origin)  intersected with the unit cell
 * [dx-1/2, dx+1/2] x [dy-1/2, dy+1/2], divided by the cell area (1).
 * Written as the integral over x of the vertical chord clipped to the cell,
 *   eps = int_{x0}^{x1} max(0, min(y1, s(x)) - max(y0, -s(x))) dx,   s(x) = sqrt(r^2 - x^2),
 * split at every abscissa where the clipping changes, each piece integrated in closed form with
 * int s dx = (x s(x) + r^2 asin(x/r)) / 2.  The primitive is O(r^2) while a cell's area is O(1),
 * so the evaluation runs in long double (64-bit significand) and the result is rounded once. */
typedef long double ld;

static ld half_chord(ld r, ld x) { /* sqrt(r^2 - x^2), well conditioned near |x| = r */
  ld a = fabsl(x);
  return a >= r ? 0.0L : sqrtl((r - a) * (r + a));
}

static ld semicircle_primitive(ld r, ld x) {
  if (x > r) x = r;
  if (x < -r) x = -r;
  ld s = half_chord(r, x);
  return 0.5L * (x * s + r * r * atan2l(x, s)); /* atan2(x, s) = asin(x / r) */
}

double o_solid_fraction(double r_, double dx, double dy) {
  const ld r = r_;
  ld x0 = (ld)dx - 0.5L, x1 = (ld)dx + 0.5L, y0 = (ld)dy - 0.5L, y1 = (ld)dy + 0.5L;
  /* the cell lies outside the disk when its point nearest to the centre is not inside */
  ld nx = (x0 > 0.0L) ? x0 : ((x1 < 0.0L) ? x1 : 0.0L);
  ld ny = (y0 > 0.0L) ? y0 : ((y1 < 0.0L) ? y1 : 0.0L);
  if (nx * nx + ny * ny >= r * r) return 0.0;
  /* the cell lies inside the (convex) disk when its farthest corner does */
  ld fx = fabsl(x0) > fabsl(x1) ? fabsl(x0) : fabsl(x1);
  ld fy = fabsl(y0) > fabsl(y1) ? fabsl(y0) : fabsl(y1);
  if (fx * fx + fy * fy <= r * r) return 1.0;

  ld bp[8];
  int nb = 0;
  bp[nb++] = x0;
  bp[nb++] = x1;
  ld cand[6];
  int nc = 0;
  cand[nc++] = -r;
  cand[nc++] = r;
  /* where the circle meets the lines y = y0 and y = y1; a line tangent to the circle (|y| = r)
   * meets it at x = 0, which must split the pieces too: each piece is classified at its
   * midpoint, and a midpoint on the tangent point would take the line for the chord's end over
   * the whole piece */
  if (fabsl(y0) <= r) {
    ld w = half_chord(r, y0);
    cand[nc++] = -w;
    cand[nc++] = w;
  }
  if (fabsl(y1) <= r) {
    ld w = half_chord(r, y1);
    cand[nc++] = -w;
    cand[nc++] = w;
  }
  for (int k = 0; k < nc; ++k)
    if (cand[k] > x0 && cand[k] < x1) bp[nb++] = cand[k];
  for (int a = 1; a < nb; ++a) { /* insertion sort */
    ld v = bp[a];
    int b = a - 1;
    while (b >= 0 && bp[b] > v) {
      bp[b + 1] = bp[b];
      --b;
    }
    bp[b + 1] = v;
  }
  ld area = 0.0L;
  for (int k = 0; k + 1 < nb; ++k) {
    ld a = bp[k], b = bp[k + 1];
    if (!(b > a)) continue;
    ld m = 0.5L * (a + b);
    if (fabsl(m) >= r) continue; /* no chord on this piece */
    ld s = half_chord(r, m);
    int top_is_circle = s < y1;
    int bot_is_circle = -s > y0;
    ld top_v = top_is_circle ? s : y1;
    ld bot_v = bot_is_circle ? -s : y0;
    if (top_v <= bot_v) continue; /* chord misses the cell on this piece */
    ld semi = semicircle_primitive(r, b) - semicircle_primitive(r, a);
    ld top_int = top_is_circle ? semi : y1 * (b - a);
    ld bot_int = bot_is_circle ? -semi : y0 * (b - a);
    area += top_int - bot_int;
  }
  /* a fraction (Sec. 2.2); rounding can leave a cell that the circle only grazes a few units of
   * the last place outside [0, 1] */
  if (area < 0.0L) area = 0.0L;
  if (area > 1.0L) area = 1.0L;
  return (double)area;
}

/* ----------------------------------------------------------- collision of one cell
 * Inputs: the 9 post-stream populations of the cell; for each disk covering it (ascending id)
 * its solid ratio, the lever arm d = cell - centre, and the disk's velocity / angular velocity.
 * Outputs: post-collision populations and, per disk, the force and torque it receives from this
 * cell.  diag (optional) receives {tau_eff, B_tot}.
 *
 *   f*_i = f_i + (1 - B_tot) (Omega^f_i + G_i) + sum_p B_p Omega^s_{p,i}          Eq. (13)
 *   Omega^f_i = -(f_i - f_i^eq(rho, u)) / tau_eff                                    Eq. (1)
 *   Omega^s_{p,i} = f_{-i} - f_{-i}^eq(rho,u) + f_i^eq(rho,u_s) - f_i                Eq. (12)
 *   dF_p = -B_p sum_i Omega^s_{p,i} c_i ,  dT_p = d x dF_p                           Eqs. (15), (16)
 * The inner sum of Eq. (15) is evaluated in closed form: with Eq. (4) and the first moment of the
 * equilibrium, sum_i c_i f_i^eq(rho, v) = rho v, it is exactly rho u_s - m.  Summing the nine
 * terms literally subtracts O(0.1) populations to get an O(1e-6) result and loses about four
 * digits, more than the agreement this oracle has to certify; the literal sum is still returned
 * (lit, optional) so that the identity is checked.
 */
int o_collide_cell(const double *f, int np, const double *eps, const double *dxs,
                   const double *dys, const double *pvx, const double *pvy, const double *pom,
                   double tau0, double cs, double gx, double gy, double *fout, double *dfx,
                   double *dfy, double *dtz, double *diag, double *lit) {
  double rho = 0.0, mx = 0.0, my = 0.0;
  for (int i = 0; i < NQ; ++i) rho += f[i];
  for (int i = 0; i < NQ; ++i) {
    mx += CX[i] * f[i];
    my += CY[i] * f[i];
  }
  double ux = mx / rho, uy = my / rho;
  double feq[NQ];
  equilibrium(rho, ux, uy, feq);
  double tau = smagorinsky_tau(tau0, cs, rho, f, feq);

  double S = 0.0;
  for (int p = 0; p < np; ++p) S += eps[p];
  double et = S < 1.0 ? S : 1.0;
  double Bt = o_weight(et, tau);

  for (int i = 0; i < NQ; ++i) {
    double G = 3.0 * WQ[i] * rho * (CX[i] * gx + CY[i] * gy);
    double Of = -(f[i] - feq[i]) / tau;
    fout[i] = f[i] + (1.0 - Bt) * (Of + G);
  }
  for (int p = 0; p < np; ++p) {
    double Bp = S > 0.0 ? Bt * (eps[p] / S) : 0.0; /* no solid in the cell: no weight */
    double usx = pvx[p] - pom[p] * dys[p];
    double usy = pvy[p] + pom[p] * dxs[p];
    double feqs[NQ];
    equilibrium(rho, usx, usy, feqs);
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < NQ; ++i) {
      int o = OPP[i];
      double Os = f[o] - feq[o] + feqs[i] - f[i];
      fout[i] += Bp * Os;
      sx += CX[i] * Os;
      sy += CY[i] * Os;
    }
    dfx[p] = Bp * (mx - rho * usx);
    dfy[p] = Bp * (my - rho * usy);
    dtz[p] = dxs[p] * dfy[p] - dys[p] * dfx[p];
    if (lit) {
      lit[2 * p] = -Bp * sx;
      lit[2 * p + 1] = -Bp * sy;
    }
  }
  if (diag) {
    diag[0] = tau;
    diag[1] = Bt;
  }
  return O_OK;
}

/* ------------------------------------------------------------------ simulation object */
static void *xcalloc(size_t n, size_t sz) { return n ? calloc(n, sz) : calloc(1, sz); }

void o_destroy(osim *s);

osim *o_create(const ocfg *c) {
  if (!c || c->nx < 2 || c->ny < 2 || !(c->tau0 > 0.5) || c->cs < 0.0 || c->n_sub < 1 ||
      !(c->kt >= 0.0) || !(c->mu >= 0.0) || c->contact_model < 0 || c->contact_model > 1 ||
      (c->contact_model == 1 && (!(c->young > 0.0) || !(c->poisson >= 0.0 && c->poisson < 0.5))) ||
      c->eps_subcells < 0 || (!c->walls && (c->uw_bot != 0.0 || c->uw_top != 0.0)))
    return NULL;
  osim *s = (osim *)calloc(1, sizeof(osim));
  if (!s) return NULL;
  s->c = *c;
  size_t nc = (size_t)c->nx * c->ny;
  s->f = (double *)xcalloc(nc * NQ, sizeof(double));
  s->fp = (double *)xcalloc(nc * NQ, sizeof(double));
  s->nslot = (int *)xcalloc(nc, sizeof(int));
  s->spid = (int *)xcalloc(nc * MAX_SLOTS, sizeof(int));
  s->seps = (double *)xcalloc(nc * MAX_SLOTS, sizeof(double));
  s->sdx = (double *)xcalloc(nc * MAX_SLOTS, sizeof(double));
  s->sdy = (double *)xcalloc(nc * MAX_SLOTS, sizeof(double));
  s->sfx = (double *)xcalloc(nc * MAX_SLOTS, sizeof(double));
  s->sfy = (double *)xcalloc(nc * MAX_SLOTS, sizeof(double));
  s->stz = (double *)xcalloc(nc * MAX_SLOTS, sizeof(double));
  if (!s->f || !s->fp || !s->nslot || !s->spid || !s->seps || !s->sdx || !s->sdy || !s->sfx ||
      !s->sfy || !s->stz) {
    o_destroy(s);
    return NULL;
  }
  return s;
}

static void free_particles(osim *s) {
  free(s->x); free(s->y); free(s->r); free(s->vx); free(s->vy); free(s->om); free(s->mode);
  free(s->fcx); free(s->fcy); free(s->Fx); free(s->Fy); free(s->Tz);
  free(s->tcz); free(s->ht); free(s->hwb); free(s->hwt);
  s->x = s->y = s->r = s->vx = s->vy = s->om = s->fcx = s->fcy = s->Fx = s->Fy = s->Tz = NULL;
  s->tcz = s->ht = s->hwb = s->hwt = NULL;
  s->mode = NULL;
  s->np = 0;
}

void o_destroy(osim *s) {
  if (!s) return;
  free(s->f); free(s->fp); free(s->nslot); free(s->spid); free(s->seps); free(s->sdx);
  free(s->sdy); free(s->sfx); free(s->sfy); free(s->stz);
  free_particles(s);
  free(s);
}

void o_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int o_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* f = f^eq(rho, u) everywhere, including inside solids (initial state of every benchmark). */
int o_init_equilibrium(osim *s, double rho, double ux, double uy) {
  double feq[NQ];
  equilibrium(rho, ux, uy, feq);
  size_t nc = (size_t)s->c.nx * s->c.ny;
  for (size_t k = 0; k < nc; ++k)
    for (int i = 0; i < NQ; ++i) s->f[k * NQ + i] = feq[i];
  return O_OK;
}

/* Exchange format for populations: [q][y][x], post-stream. */
int o_set_populations(osim *s, const double *fq) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int i = 0; i < NQ; ++i)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        s->f[((size_t)y * nx + x) * NQ + i] = fq[((size_t)i * ny + y) * nx + x];
  return O_OK;
}

int o_get_populations(const osim *s, double *fq) {
  int nx = s->c.nx, ny = s->c.ny;
  for (int i = 0; i < NQ; ++i)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        fq[((size_t)i * ny + y) * nx + x] = s->f[((size_t)y * nx + x) * NQ + i];
  return O_OK;
}

/* Density and velocity u = m / rho of the post-stream populations, Eqs. (3), (4). */
int o_get_fields(const osim *s, double *rho, double *ux, double *uy) {
  size_t nc = (size_t)s->c.nx * s->c.ny;
  for (size_t k = 0; k < nc; ++k) {
    const double *f = s->f + k * NQ;
    double r = 0.0, mx = 0.0, my = 0.0;
    for (int i = 0; i < NQ; ++i) r += f[i];
    for (int i = 0; i < NQ; ++i) {
      mx += CX[i] * f[i];
      my += CY[i] * f[i];
    }
    if (rho) rho[k] = r;
    if (ux) ux[k] = mx / r;
    if (uy) uy[k] = my / r;
  }
  return O_OK;
}

/* ------------------------------------------------------------------ DEM (Sec. 2.1) */
static double disk_mass(const osim *s, int p) { return s->c.rho_s * M_PI * s->r[p] * s->r[p]; }

static double wrap_coord(double v, int n) {
  if (v >= n) v -= n;
  else if (v < 0.0) v += n;
  return v;
}

static double nearest_image(double d, int n) {
  if (d > 0.5 * n) d -= n;
  else if (d < -0.5 * n) d += n;
  return d;
}

/* Contact forces and torques (Eqs. 7, 8) on every free disk, from all other disks (ascending id)
 * and then the two walls.  Normal: -(k_n delta + c_n v_n) n, with n the unit vector from i
 * towards its partner, delta the overlap, v_n = (V_i - V_partner) . n the approach speed and
 * c_n = 2 zeta sqrt(k_n m_eff).  Tangential (only when k_t or mu is set; linear spring-dashpot
 * with a Coulomb limit): t = (-n_y, n_x); the contact point sits in the middle of the overlap,
 * at l_i = r_i - delta/2 from each centre (so l_i + l_j = |X_i - X_j| and the pair's torques
 * conserve angular momentum); the slip of i against its partner there is
 * v_t = (V_i - V_j) . t + omega_i l_i + omega_j l_j; the spring s grows by v_t dt at each
 * evaluation (`advance`); F_t = -k_t s - c_t v_t with c_t = 2 zeta sqrt(k_t m_eff), limited to
 * |F_t| <= mu max(F_n, 0), where sliding resets s = -F_t / k_t; the force F_t t acts on i with
 * torque l_i F_t.  A wall is a partner at rest in y moving along x at its wall velocity.  A
 * contact that has ended leaves s = 0. */
static double tangential(const osim *s, double *spring, double vt, double fn, double kt,
                         double ct, int advance) {
  double mu = s->c.mu;
  double dt = 1.0 / s->c.n_sub;
  double sp = advance ? *spring + vt * dt : *spring;
  double ft = -kt * sp - ct * vt;
  double cap = mu * (fn > 0.0 ? fn : 0.0);
  if (fabs(ft) > cap) {
    ft = ft > 0.0 ? cap : -cap;
    sp = kt > 0.0 ? -ft / kt : 0.0;
  }
  *spring = sp;
  return ft;
}

/* The contact law of one contact of overlap delta (> 0), effective radius rstar and mass meff,
 * with a partner that is another disk (wall = 0) or a wall (wall = 1): the normal force
 * k delta + c v_n and the tangential stiffness and damping.
 *   linear (Eq. 8 with constant coefficients): k = k_n, c = 2 zeta sqrt(k_n m_eff);
 *     tangential k_t and c_t = 2 zeta sqrt(k_t m_eff).
 *   Hertz-Mindlin, the simplified form the paper adopts (Sec. 2.1, after Di Renzo & Di Maio):
 *     normal stiffness S_n = 2 E* sqrt(R* delta), elastic force (4/3) E* sqrt(R*) delta^(3/2)
 *     (= S_n delta * 2/3), damping c_n = 2 sqrt(5/6) zeta sqrt(S_n m_eff);
 *     tangential stiffness S_t = 8 G* sqrt(R* delta), c_t = 2 sqrt(5/6) zeta sqrt(S_t m_eff);
 *     two disks of the same material: 1/E* = 2 (1 - nu^2) / E, 1/G* = 2 (2 - nu) / G with
 *     G = E / (2 (1 + nu)); against a rigid wall 1/E* = (1 - nu^2) / E, 1/G* = (2 - nu) / G.
 * Returns the normal force; *kt, *ct receive the tangential coefficients. */
static double normal_law(const osim *s, double delta, double vn, double rstar, double meff,
                         int wall, double *kt, double *ct) {
  double zeta = s->c.zeta;
  if (s->c.contact_model == 1) {
    double E = s->c.young, nu = s->c.poisson;
    double G = E / (2.0 * (1.0 + nu));
    double Es = wall ? E / (1.0 - nu * nu) : E / (2.0 * (1.0 - nu * nu));
    double Gs = wall ? G / (2.0 - nu) : G / (2.0 * (2.0 - nu));
    double root = sqrt(rstar * delta);
    double Sn = 2.0 * Es * root;
    double St = 8.0 * Gs * root;
    double damp = 2.0 * sqrt(5.0 / 6.0) * zeta;
    *kt = St;
    *ct = damp * sqrt(St * meff);
    return 4.0 / 3.0 * Es * root * delta + damp * sqrt(Sn * meff) * vn;
  }
  *kt = s->c.kt;
  *ct = 2.0 * zeta * sqrt(s->c.kt * meff);
  return s->c.kn * delta + 2.0 * zeta * sqrt(s->c.kn * meff) * vn;
}

static void contact_forces(osim *s, int advance) {
  int np = s->np;
  int tang = s->c.contact_model == 1 ? s->c.mu > 0.0 : (s->c.kt > 0.0 || s->c.mu > 0.0);
  for (int i = 0; i < np; ++i) {
    double fx = 0.0, fy = 0.0, tz = 0.0;
    if (s->mode[i] == 0) {
      double mi = disk_mass(s, i);
      for (int j = 0; j < np; ++j) {
        if (j == i) continue;
        double dx = s->x[j] - s->x[i];
        double dy = s->y[j] - s->y[i];
        dx = nearest_image(dx, s->c.nx);
        if (!s->c.walls) dy = nearest_image(dy, s->c.ny);
        double dist = sqrt(dx * dx + dy * dy);
        double delta = s->r[i] + s->r[j] - dist;
        if (delta > 0.0 && dist > 0.0) {
          double nxu = dx / dist, nyu = dy / dist;
          double vn = (s->vx[i] - s->vx[j]) * nxu + (s->vy[i] - s->vy[j]) * nyu;
          double mj = disk_mass(s, j);
          double meff = mi * mj / (mi + mj);
          double rstar = s->r[i] * s->r[j] / (s->r[i] + s->r[j]);
          double kt, ct;
          double fn = normal_law(s, delta, vn, rstar, meff, 0, &kt, &ct);
          fx += -fn * nxu;
          fy += -fn * nyu;
          if (tang) {
            double tx = -nyu, ty = nxu;
            double li = s->r[i] - 0.5 * delta, lj = s->r[j] - 0.5 * delta;
            double vt = (s->vx[i] - s->vx[j]) * tx + (s->vy[i] - s->vy[j]) * ty +
                        s->om[i] * li + s->om[j] * lj;
            double ft = tangential(s, &s->ht[(size_t)i * np + j], vt, fn, kt, ct, advance);
            fx += ft * tx;
            fy += ft * ty;
            tz += li * ft;
          }
        } else if (tang) {
          s->ht[(size_t)i * np + j] = 0.0;
        }
      }
      if (s->c.walls) {
        double db = s->r[i] - (s->y[i] + 0.5); /* wall at y = -1/2, n = (0,-1), t = (1,0) */
        if (db > 0.0) {
          double vn = -s->vy[i];
          double kt, ct;
          double fn = normal_law(s, db, vn, s->r[i], mi, 1, &kt, &ct);
          fy += fn;
          if (tang) {
            double l = s->r[i] - 0.5 * db;
            double vt = (s->vx[i] - s->c.uw_bot) + s->om[i] * l;
            double ft = tangential(s, &s->hwb[i], vt, fn, kt, ct, advance);
            fx += ft;
            tz += l * ft;
          }
        } else if (tang) {
          s->hwb[i] = 0.0;
        }
        double dt = s->r[i] - ((s->c.ny - 0.5) - s->y[i]); /* wall at y = ny-1/2, n = (0,1) */
        if (dt > 0.0) {
          double vn = s->vy[i];
          double kt, ct;
          double fn = normal_law(s, dt, vn, s->r[i], mi, 1, &kt, &ct);
          fy += -fn;
          if (tang) { /* t = (-1, 0) */
            double l = s->r[i] - 0.5 * dt;
            double vt = -(s->vx[i] - s->c.uw_top) + s->om[i] * l;
            double ft = tangential(s, &s->hwt[i], vt, fn, kt, ct, advance);
            fx += -ft;
            tz += l * ft;
          }
        } else if (tang) {
          s->hwt[i] = 0.0;
        }
      }
    }
    s->fcx[i] = fx;
    s->fcy[i] = fy;
    s->tcz[i] = tz;
  }
}

/* One lattice step of DEM: N_sub velocity-Verlet (kick-drift-kick) sub-steps of dt = 1/N_sub
 * (Eq. 17) for free disks with the hydrodynamic force and torque of this step held fixed; the
 * contact force is evaluated after each drift from the new positions and half-step velocities
 * and reused for the first kick of the next sub-step.  Prescribed disks move by V once per step;
 * fixed disks stay. */
static void dem_phase(osim *s) {
  int np = s->np;
  int any_free = 0;
  for (int i = 0; i < np; ++i) any_free |= (s->mode[i] == 0);
  if (any_free) {
    double dt = 1.0 / s->c.n_sub, h = 0.5 * dt;
    for (int k = 0; k < s->c.n_sub; ++k) {
      for (int i = 0; i < np; ++i) {
        if (s->mode[i] != 0) continue;
        double m = disk_mass(s, i);
        double I = 0.5 * m * s->r[i] * s->r[i];
        double ax = (s->fcx[i] + s->Fx[i]) / m;
        double ay = (s->fcy[i] + s->Fy[i]) / m;
        s->vx[i] = s->vx[i] + h * ax;
        s->vy[i] = s->vy[i] + h * ay;
        s->x[i] = wrap_coord(s->x[i] + dt * s->vx[i], s->c.nx);
        s->y[i] = s->y[i] + dt * s->vy[i];
        if (!s->c.walls) s->y[i] = wrap_coord(s->y[i], s->c.ny);
        s->om[i] = s->om[i] + h * ((s->Tz[i] + s->tcz[i]) / I);
      }
      contact_forces(s, 1);
      for (int i = 0; i < np; ++i) {
        if (s->mode[i] != 0) continue;
        double m = disk_mass(s, i);
        double I = 0.5 * m * s->r[i] * s->r[i];
        double ax = (s->fcx[i] + s->Fx[i]) / m;
        double ay = (s->fcy[i] + s->Fy[i]) / m;
        s->vx[i] = s->vx[i] + h * ax;
        s->vy[i] = s->vy[i] + h * ay;
        s->om[i] = s->om[i] + h * ((s->Tz[i] + s->tcz[i]) / I);
      }
    }
  }
  for (int i = 0; i < np; ++i) {
    if (s->mode[i] != 2) continue;
    s->x[i] = wrap_coord(s->x[i] + s->vx[i], s->c.nx);
    s->y[i] = s->y[i] + s->vy[i];
    if (!s->c.walls) s->y[i] = wrap_coord(s->y[i], s->c.ny);
  }
}

int o_set_particles(osim *s, int n, const double *x, const double *y, const double *r,
                    const double *vx, const double *vy, const double *om, const int32_t *mode) {
  if (n < 0) return O_EINVAL;
  for (int p = 0; p < n; ++p) {
    if (!(r[p] > 0.0) || 2.0 * (r[p] + 2.0) >= s->c.nx || 2.0 * (r[p] + 2.0) >= s->c.ny)
      return O_EINVAL;
    if (!(x[p] >= 0.0 && x[p] < s->c.nx)) return O_EINVAL;
    if (mode[p] < 0 || mode[p] > 2) return O_EINVAL;
  }
  free_particles(s);
  size_t nn = (size_t)n;
  s->x = (double *)xcalloc(nn, sizeof(double));
  s->y = (double *)xcalloc(nn, sizeof(double));
  s->r = (double *)xcalloc(nn, sizeof(double));
  s->vx = (double *)xcalloc(nn, sizeof(double));
  s->vy = (double *)xcalloc(nn, sizeof(double));
  s->om = (double *)xcalloc(nn, sizeof(double));
  s->mode = (int32_t *)xcalloc(nn, sizeof(int32_t));
  s->fcx = (double *)xcalloc(nn, sizeof(double));
  s->fcy = (double *)xcalloc(nn, sizeof(double));
  s->Fx = (double *)xcalloc(nn, sizeof(double));
  s->Fy = (double *)xcalloc(nn, sizeof(double));
  s->Tz = (double *)xcalloc(nn, sizeof(double));
  s->tcz = (double *)xcalloc(nn, sizeof(double));
  s->ht = (double *)xcalloc(nn * nn + 1, sizeof(double));
  s->hwb = (double *)xcalloc(nn + 1, sizeof(double));
  s->hwt = (double *)xcalloc(nn + 1, sizeof(double));
  if (!s->x || !s->y || !s->r || !s->vx || !s->vy || !s->om || !s->mode || !s->fcx || !s->fcy ||
      !s->Fx || !s->Fy || !s->Tz || !s->tcz || !s->ht || !s->hwb || !s->hwt)
    return O_ENOMEM;
  s->np = n;
  for (int p = 0; p < n; ++p) {
    s->x[p] = x[p]; s->y[p] = y[p]; s->r[p] = r[p];
    s->vx[p] = vx[p]; s->vy[p] = vy[p]; s->om[p] = om[p]; s->mode[p] = mode[p];
  }
  contact_forces(s, 0);  /* the force of the initial overlaps; no spring has stretched yet */
  return O_OK;
}

/* ------------------------------------------------------------ one coupled step (Sec. 2.3) */

/* Map every disk onto the lattice: for each cell its covering disks (ascending id), their solid
 * ratios and lever arms.  Only cells within one cell of a disk's bounding box can have eps > 0;
 * the lever arm uses the disk image nearest to the cell, computed from the integer cell offset
 * and the fractional part of the centre. */
static int map_particles(osim *s) {
  int nx = s->c.nx, ny = s->c.ny;
  memset(s->nslot, 0, sizeof(int) * (size_t)nx * ny);
  for (int p = 0; p < s->np; ++p) {
    double X = s->x[p], Y = s->y[p], r = s->r[p];
    double flx = floor(X), fly = floor(Y);
    double fx = X - flx, fy = Y - fly;
    int ix0 = (int)floor(X - r - 0.5), ix1 = (int)ceil(X + r + 0.5);
    int iy0 = (int)floor(Y - r - 0.5), iy1 = (int)ceil(Y + r + 0.5);
    if (s->c.walls) {
      if (iy0 < 0) iy0 = 0;
      if (iy1 > ny - 1) iy1 = ny - 1;
    }
    for (int iy = iy0; iy <= iy1; ++iy) {
      int yw = ((iy % ny) + ny) % ny;
      long dj = (long)yw - (long)fly;
      if (!s->c.walls) {
        if (dj > ny / 2) dj -= ny;
        else if (dj < -(ny / 2)) dj += ny;
      }
      double dy = (double)dj - fy;
      for (int ix = ix0; ix <= ix1; ++ix) {
        int xw = ((ix % nx) + nx) % nx;
        long di = (long)xw - (long)flx;
        if (di > nx / 2) di -= nx;
        else if (di < -(nx / 2)) di += nx;
        double dx = (double)di - fx;
        double e = s->c.eps_subcells > 0 ? o_subcell_fraction(r, dx, dy, s->c.eps_subcells)
                                         : o_solid_fraction(r, dx, dy);
        if (e > 0.0) {
          size_t k = (size_t)yw * nx + xw;
          int ns = s->nslot[k];
          if (ns >= MAX_SLOTS) return O_EOVERFLOW;
          s->spid[k * MAX_SLOTS + ns] = p;
          s->seps[k * MAX_SLOTS + ns] = e;
          s->sdx[k * MAX_SLOTS + ns] = dx;
          s->sdy[k * MAX_SLOTS + ns] = dy;
          s->nslot[k] = ns + 1;
        }
      }
    }
  }
  return O_OK;
}

static void collide_all(osim *s) {
  int nx = s->c.nx, ny = s->c.ny;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    double pvx[MAX_SLOTS], pvy[MAX_SLOTS], pom[MAX_SLOTS];
    for (int x = 0; x < nx; ++x) {
      size_t k = (size_t)y * nx + x;
      int ns = s->nslot[k];
      for (int q = 0; q < ns; ++q) {
        int p = s->spid[k * MAX_SLOTS + q];
        pvx[q] = s->vx[p];
        pvy[q] = s->vy[p];
        pom[q] = s->om[p];
      }
      o_collide_cell(s->f + k * NQ, ns, s->seps + k * MAX_SLOTS, s->sdx + k * MAX_SLOTS,
                     s->sdy + k * MAX_SLOTS, pvx, pvy, pom, s->c.tau0, s->c.cs, s->c.gx, s->c.gy,
                     s->fp + k * NQ, s->sfx + k * MAX_SLOTS, s->sfy + k * MAX_SLOTS,
                     s->stz + k * MAX_SLOTS, NULL, NULL);
    }
  }
}

/* Streaming, left-hand side of Eq. (1): f_i(x + c_i) <- f*_i(x); a link leaving through a wall
 * returns to its own node in the opposite direction (half-way bounce-back).  A wall moving with
 * velocity u_w along x hands back f*_i - 6 w_i rho0 (c_i . u_w): the momentum exchange of a
 * moving bounce-back wall (Ladd), with the reference density rho0 at the wall. */
static void stream_all(osim *s) {
  int nx = s->c.nx, ny = s->c.ny;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      const double *fp = s->fp + ((size_t)y * nx + x) * NQ;
      for (int i = 0; i < NQ; ++i) {
        int xn = (x + CX[i] + nx) % nx;
        int yn = y + CY[i];
        if (yn < 0 || yn >= ny) {
          if (s->c.walls) {
            const double uw = yn >= ny ? s->c.uw_top : s->c.uw_bot;
            const double corr = 6.0 * WQ[i] * s->c.rho0 * ((double)CX[i] * uw);
            s->f[((size_t)y * nx + x) * NQ + OPP[i]] = fp[i] - corr;
            continue;
          }
          yn = (yn + ny) % ny;
        }
        s->f[((size_t)yn * nx + xn) * NQ + i] = fp[i];
      }
    }
  }
}

/* Force and torque on each disk: sum of the per-cell contributions over the covered cells in
 * row-major cell order (Eqs. 15, 16, sign on the particle). */
static void sum_forces(osim *s) {
  for (int p = 0; p < s->np; ++p) s->Fx[p] = s->Fy[p] = s->Tz[p] = 0.0;
  size_t nc = (size_t)s->c.nx * s->c.ny;
  for (size_t k = 0; k < nc; ++k) {
    for (int q = 0; q < s->nslot[k]; ++q) {
      int p = s->spid[k * MAX_SLOTS + q];
      s->Fx[p] += s->sfx[k * MAX_SLOTS + q];
      s->Fy[p] += s->sfy[k * MAX_SLOTS + q];
      s->Tz[p] += s->stz[k * MAX_SLOTS + q];
    }
  }
}

int o_step(osim *s, int nsteps) {
  for (int n = 0; n < nsteps; ++n) {
    int rc = map_particles(s);
    if (rc) return rc;
    collide_all(s);
    stream_all(s);
    sum_forces(s);
    dem_phase(s);
    s->step++;
  }
  return O_OK;
}

/* Steps while accumulating J += sum_p (wfx_p Fx_p + wfy_p Fy_p + wt_p T_p) after every step. */
int o_step_accumulate(osim *s, int nsteps, const double *wfx, const double *wfy, const double *wt,
                      double *J) {
  double acc = *J;
  for (int n = 0; n < nsteps; ++n) {
    int rc = o_step(s, 1);
    if (rc) return rc;
    for (int p = 0; p < s->np; ++p) {
      if (wfx) acc += wfx[p] * s->Fx[p];
      if (wfy) acc += wfy[p] * s->Fy[p];
      if (wt) acc += wt[p] * s->Tz[p];
    }
  }
  *J = acc;
  return O_OK;
}

/* Conditioning scales of each disk's force and torque of the last step (tests): sF, the sum over
 * its covered cells of the magnitudes |dF| of the per-cell force contributions (Eq. 15), and sT,
 * the sum of |d| |dF| (the largest moment each contribution can exert, Eq. 16).  A sum evaluated
 * in another order, from contributions each correct to a few units in the last place of their
 * magnitude, differs from this oracle's by a small multiple of the unit roundoff times these. */
int o_force_scales(const osim *s, double *sF, double *sT) {
  for (int p = 0; p < s->np; ++p) sF[p] = sT[p] = 0.0;
  size_t nc = (size_t)s->c.nx * s->c.ny;
  for (size_t k = 0; k < nc; ++k) {
    for (int q = 0; q < s->nslot[k]; ++q) {
      size_t j = k * MAX_SLOTS + q;
      int p = s->spid[j];
      double f = sqrt(s->sfx[j] * s->sfx[j] + s->sfy[j] * s->sfy[j]);
      sF[p] += f;
      sT[p] += sqrt(s->sdx[j] * s->sdx[j] + s->sdy[j] * s->sdy[j]) * f;
    }
  }
  return O_OK;
}

/* Contact force and torque of every disk at the last DEM evaluation (tests). */
int o_get_contacts(const osim *s, double *fcx, double *fcy, double *tcz) {
  for (int p = 0; p < s->np; ++p) {
    fcx[p] = s->fcx[p];
    fcy[p] = s->fcy[p];
    tcz[p] = s->tcz[p];
  }
  return O_OK;
}

/* Sets the stored hydrodynamic force and torque that DEM-alone steps hold fixed (for tests of
 * the contact law without fluid). */
int o_set_loads(osim *s, const double *fx, const double *fy, const double *tz) {
  for (int p = 0; p < s->np; ++p) {
    s->Fx[p] = fx[p];
    s->Fy[p] = fy[p];
    s->Tz[p] = tz[p];
  }
  return O_OK;
}

/* DEM alone (no fluid): nsteps lattice steps of DEM with the stored hydrodynamic force. */
int o_dem_steps(osim *s, int nsteps) {
  for (int n = 0; n < nsteps; ++n) dem_phase(s);
  return O_OK;
}

int o_get_forces(const osim *s, double *fx, double *fy, double *tz) {
  for (int p = 0; p < s->np; ++p) {
    fx[p] = s->Fx[p];
    fy[p] = s->Fy[p];
    tz[p] = s->Tz[p];
  }
  return O_OK;
}

int o_get_particles(const osim *s, double *x, double *y, double *vx, double *vy, double *om) {
  for (int p = 0; p < s->np; ++p) {
    x[p] = s->x[p]; y[p] = s->y[p]; vx[p] = s->vx[p]; vy[p] = s->vy[p]; om[p] = s->om[p];
  }
  return O_OK;
}

/* Solid ratio field of the current particle state: eps_tot per cell ([y][x]). */
int o_solid_field(osim *s, double *eps_tot) {
  int rc = map_particles(s);
  if (rc) return rc;
  size_t nc = (size_t)s->c.nx * s->c.ny;
  for (size_t k = 0; k < nc; ++k) {
    double S = 0.0;
    for (int q = 0; q < s->nslot[k]; ++q) S += s->seps[k * MAX_SLOTS + q];
    eps_tot[k] = S;
  }
  return O_OK;
}

long o_step_count(const osim *s) { return s->step; }
