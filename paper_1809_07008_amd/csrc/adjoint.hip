// adjoint.hip -- discrete adjoint of the coupled step (differentiation form).
//
// Objective J = sum over steps n and disks p of wfx_p Fx_p^n + wfy_p Fy_p^n + wtz_p Tz_p^n, the
// hydrodynamic force and torque of Eqs. (15), (16).  The disks move by prescription
// (X^n = X^0 + n V) or are fixed, there is no DEM and no Smagorinsky term, so one step maps the
// stored post-collision state s^{n-1} to s^n = C_n(P s^{n-1}) with P the pull-streaming
// permutation (periodic x, half-way bounce-back walls) and C_n the cellwise IMB collision.  The
// reverse sweep carries lam^n = dJ/ds^n:
//     lam^{n-1} = P^T (C_n'^T lam^n + dJ_n/d(P s^{n-1}))
// cell by cell: each workgroup pulls the populations its cells saw in step n, rebuilds the
// collision's intermediates, applies the transposed cell Jacobian (adjoint_cell.h) and pushes
// the result back along the streaming links (the inverse permutation), so every adjoint value is
// written exactly once.  Parameter gradients (disk position, velocity, spin; body force) are
// reduced per tile without atomics, finalised per disk in a fixed order, and chained through the
// prescribed motion (dJ/dV += n dJ/dX^n).
//
// Memory: the forward pass keeps every k-th stored state (checkpoints) and the per-step disk
// tables (positions, tile boxes, band masks: a few KB per step); the reverse sweep recomputes
// the states of one segment from its checkpoint into a ring of k - 1 states, then walks the
// segment backwards.  Traffic per reverse step: the recomputation (9 reads + 9 writes per cell)
// and the adjoint step (9 pulled state reads, 9 adjoint reads, 9 adjoint writes).
#include <algorithm>
#include <vector>

#include "adjoint_cell.h"
#include "runtime.h"
#include "tile.h"

namespace imb {

constexpr int NG = 5;  // per-disk gradient components: X, Y, Vx, Vy, omega

struct AdjointArgs {
  LatticeArgs la;       // geometry; src = stored state before the step; table of the step
  const void* lam_in;   // dJ / d(stored state after the step)   [9][ny][pitch], type T
  void* lam_out;        // dJ / d(stored state before the step)
  const double *wfx, *wfy, *wtz;  // objective weights (null = 0)
  double* part;         // [MAXSLOT][NG][pstride] this step's per-disk partials
  double2* gg_blk;      // [tiles] dJ/dg per tile, accumulated over steps
  // finalisation of an earlier step's partials by the extra workgroup
  int fin_step;         // its step index (-1: nothing to finalise)
  const double* fin_part;
  const int4* fin_box;
  const int* mode;
  double* gacc;         // [NG][pstride] per-disk accumulated gradients
};

// Sums step `step`'s per-disk partial slots in slot order and adds them (and the prescribed
// motion's dJ/dV = step * dJ/dX^step) to the accumulators.
__device__ inline void finalise_disks(int np, int pstride, int step, const double* part,
                                      const int4* box, const int* mode, double* gacc) {
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const int4 b = box[p];
    const int ns = box_slots(b);
    double g[NG] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < ns; ++s)
#pragma unroll
      for (int c = 0; c < NG; ++c) g[c] += part[((long long)s * NG + c) * pstride + p];
    const double mult = mode[p] == IMB_MODE_PRESCRIBED ? (double)step : 0.0;
    gacc[0 * pstride + p] += g[0];
    gacc[1 * pstride + p] += g[1];
    gacc[2 * pstride + p] += g[2] + mult * g[0];
    gacc[3 * pstride + p] += g[3] + mult * g[1];
    gacc[4 * pstride + p] += g[4];
  }
}

template <class St>
__global__ __launch_bounds__(BLOCK) void k_adjoint_step(AdjointArgs A) {
  using T = typename St::T;
  using S = typename St::S;
  const LatticeArgs& a = A.la;
  __shared__ PEntry<T> s_pl[LMAX];
  __shared__ int s_cnt[2 * WAVES];
  __shared__ int s_pid[LMAX], s_slot[LMAX];
  __shared__ unsigned s_touch;
  __shared__ Acc<T> s_red[WAVES][LMAX][NG];
  __shared__ Acc<T> s_gg[WAVES][2];

  const int ntiles = a.tiles_x * a.tiles_y;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  if (b == ntiles) {  // the extra workgroup: the previous launch's per-disk partials
    if (A.fin_step >= 0)
      finalise_disks(a.np, a.pstride, A.fin_step, A.fin_part, A.fin_box, A.mode, A.gacc);
    return;
  }
  const int tid = threadIdx.x;
  const int tx = b % a.tiles_x, ty = b / a.tiles_x;
  const int tw = 1 << a.tw_log, th = BLOCK >> a.tw_log;
  const int x = tx * tw + (tid & (tw - 1));
  const int ybase = ty * th * a.rows + (tid >> a.tw_log);
  const S* src = (const S*)a.src;
  const T* lin = (const T*)A.lam_in;
  T* lout = (T*)A.lam_out;

  if (tid == 0) s_touch = 0u;
  const int n = build_tile_list<T>(a, tx, ty, s_pl, s_cnt, s_pid, s_slot);

  const T tau = (T)a.tau0, gx = (T)a.gx, gy = (T)a.gy, rho0 = (T)a.rho0;
  int aj[MAXC];
  T ag[NG][MAXC];
#pragma unroll
  for (int q = 0; q < MAXC; ++q) {
    aj[q] = -1;
#pragma unroll
    for (int c = 0; c < NG; ++c) ag[c][q] = T(0);
  }
  T ggx = T(0), ggy = T(0);

  for (int rr = 0; rr < a.rows; ++rr) {
    const int y = ybase + rr * th;
    if (x >= a.nx || y >= a.ny) continue;
    T h[NQ], lam[NQ], gh[NQ];
    pull_load<St>(a, src, x, y, h);
    if constexpr (!St::deviation) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) h[i] -= (T)w_of(i) * rho0;
    }
    const long long base = (long long)y * a.pitch + x;
#pragma unroll
    for (int i = 0; i < NQ; ++i) lam[i] = lin[(long long)i * a.plane + base];

    // covering disks of this cell (registers; slots filled in order)
    int cj[MAXC];
    T ce[MAXC], cgx[MAXC], cgy[MAXC], cdx[MAXC], cdy[MAXC];
#pragma unroll
    for (int q = 0; q < MAXC; ++q) {
      cj[q] = 0;
      ce[q] = cgx[q] = cgy[q] = cdx[q] = cdy[q] = T(0);
    }
    int nc = 0;
    for (int j = 0; j < n; ++j) {
      T dx, dy;
      lever_arm(a, s_pl[j], x, y, &dx, &dy);
      const T eps = solid_fraction<T>(s_pl[j].r, dx, dy);
      if (!(eps > T(0))) continue;
      if (nc >= MAXC) {
        atomicOr(a.err, ERR_CELL);
        continue;
      }
      T ex = T(0), ey = T(0);
      if (eps < T(1)) solid_fraction_grad<T>(s_pl[j].r, dx, dy, &ex, &ey);
#pragma unroll
      for (int q = 0; q < MAXC; ++q)
        if (q == nc) {
          cj[q] = j;
          ce[q] = eps;
          cgx[q] = ex;
          cgy[q] = ey;
          cdx[q] = dx;
          cdy[q] = dy;
        }
      ++nc;
    }
    T gk[NG][MAXC];
    auto disk = [&](int k) {
      const PEntry<T>& e = s_pl[cj[k]];
      const int p = e.pid;
      DiskAdj<T> d;
      d.eps = ce[k];
      d.dex = cgx[k];
      d.dey = cgy[k];
      d.dx = cdx[k];
      d.dy = cdy[k];
      d.vx = e.vx;
      d.vy = e.vy;
      d.om = e.om;
      d.wfx = A.wfx ? (T)A.wfx[p] : T(0);
      d.wfy = A.wfy ? (T)A.wfy[p] : T(0);
      d.wtz = A.wtz ? (T)A.wtz[p] : T(0);
      return d;
    };
    auto emit = [&](int k, T g0, T g1, T g2, T g3, T g4) {
      gk[0][k] = g0;
      gk[1][k] = g1;
      gk[2][k] = g2;
      gk[3][k] = g3;
      gk[4][k] = g4;
    };
    T cgg_x, cgg_y;
    collide_adjoint<T>(h, lam, nc, disk, emit, rho0, tau, gx, gy, gh, &cgg_x, &cgg_y);
    ggx += cgg_x;
    ggy += cgg_y;
    // per-disk accumulators of this thread (one per distinct list entry)
#pragma unroll
    for (int k = 0; k < MAXC; ++k) {
      if (k >= nc) continue;
      bool done = false;
#pragma unroll
      for (int q = 0; q < MAXC; ++q) {
        if (!done && (aj[q] == cj[k] || aj[q] < 0)) {
          aj[q] = cj[k];
#pragma unroll
          for (int c = 0; c < NG; ++c) ag[c][q] += gk[c][k];
          done = true;
        }
      }
    }
    // push along the links: the adjoint of the pull (each target is written once)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      int xs = x - cx_of(i), ys = y - cy_of(i);
      xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
      long long idx;
      if (ys < 0 || ys >= a.ny) {
        if (a.walls) {
          idx = (long long)opp_of(i) * a.plane + base;
          lout[idx] = gh[i];
          continue;
        }
        ys = ys < 0 ? ys + a.ny : ys - a.ny;
      }
      idx = (long long)i * a.plane + (long long)ys * a.pitch + xs;
      lout[idx] = gh[i];
    }
  }

  // dJ/dg: block sum in a fixed order, added to this tile's accumulator
  const int lane = tid & 63, wave = tid >> 6;
  {
    Acc<T> vx{ggx, T(0)}, vy{ggy, T(0)};
    vx = wave_sum(vx);
    vy = wave_sum(vy);
    if (lane == 0) {
      s_gg[wave][0] = vx;
      s_gg[wave][1] = vy;
    }
  }
  unsigned mine = 0u;
#pragma unroll
  for (int q = 0; q < MAXC; ++q)
    if (aj[q] >= 0) mine |= 1u << aj[q];
  if (mine) atomicOr(&s_touch, mine);
  __syncthreads();
  if (tid == 0) {
    Acc<T> vx = s_gg[0][0], vy = s_gg[0][1];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) {
      vx.add(s_gg[w][0]);
      vy.add(s_gg[w][1]);
    }
    double2 acc = A.gg_blk[b];
    acc.x += (double)vx.hi + (double)vx.lo;
    acc.y += (double)vy.hi + (double)vy.lo;
    A.gg_blk[b] = acc;
  }
  if (n == 0) return;  // block-uniform
  const unsigned touched = s_touch;
  for (int j = 0; j < n; ++j) {
    if (!((touched >> j) & 1u)) continue;
#pragma unroll
    for (int c = 0; c < NG; ++c) {
      Acc<T> v{T(0), T(0)};
#pragma unroll
      for (int q = 0; q < MAXC; ++q)
        if (aj[q] == j) v.add(ag[c][q]);
      v = wave_sum(v);
      if (lane == 0) s_red[wave][j][c] = v;
    }
  }
  __syncthreads();
  if (tid < n) {
    const int j = tid;
    const bool t = (touched >> j) & 1u;
    const long long slot = s_pl[j].slot;
#pragma unroll
    for (int c = 0; c < NG; ++c) {
      double out = 0.0;
      if (t) {
        Acc<T> v = s_red[0][j][c];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) v.add(s_red[w][j][c]);
        out = (double)v.hi + (double)v.lo;
      }
      A.part[(slot * NG + c) * a.pstride + s_pl[j].pid] = out;
    }
  }
}

// Last step's finalisation, dJ/dg summed over the tile accumulators in a fixed order.
__global__ __launch_bounds__(BLOCK) void k_adjoint_final(int np, int pstride, const double* part,
                                                         const int4* box, const int* mode,
                                                         double* gacc, const double2* gg_blk,
                                                         int ntiles, double* gg_out) {
  __shared__ double s_x[BLOCK], s_y[BLOCK];
  finalise_disks(np, pstride, 0, part, box, mode, gacc);
  double sx = 0.0, sy = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += BLOCK) {
    sx += gg_blk[t].x;
    sy += gg_blk[t].y;
  }
  s_x[threadIdx.x] = sx;
  s_y[threadIdx.x] = sy;
  __syncthreads();
  for (int w = BLOCK / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_x[threadIdx.x] += s_x[threadIdx.x + w];
      s_y[threadIdx.x] += s_y[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    gg_out[0] = s_x[0];
    gg_out[1] = s_y[0];
  }
}

// Pull of an adjoint field: dJ/d(post-stream populations) = P lam (FP64 [9][ny][nx]).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_pull_adjoint(LatticeArgs a, const T* lam, double* out) {
  const long long cell = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (cell >= (long long)a.nx * a.ny) return;
  const int x = (int)(cell % a.nx), y = (int)(cell / a.nx);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    int xs = x - cx_of(i), ys = y - cy_of(i);
    xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
    long long idx;
    if (ys < 0 || ys >= a.ny) {
      if (a.walls) {
        idx = (long long)opp_of(i) * a.plane + (long long)y * a.pitch + x;
        out[(long long)i * a.nx * a.ny + cell] = (double)lam[idx];
        continue;
      }
      ys = ys < 0 ? ys + a.ny : ys - a.ny;
    }
    idx = (long long)i * a.plane + (long long)ys * a.pitch + xs;
    out[(long long)i * a.nx * a.ny + cell] = (double)lam[idx];
  }
}

// ------------------------------------------------------------------------------ host side
struct AdjointState {
  int nseg = 0, k = 0, nsteps = 0, np_cap = 0;
  int tiles_x = 0, tiles_y = 0;  // tile grid of the per-tile buffers (band masks, gg_blk)
  size_t state_bytes = 0, lam_bytes = 0;
  std::vector<void*> ckpt;  // nseg stored states
  std::vector<void*> ring;  // k - 1 stored states
  void* lam[2] = {nullptr, nullptr};
  // per-step disk tables, slot n = the table the lattice step n uses
  int4* h_box = nullptr;
  double4* h_pos = nullptr;
  double4* h_vel = nullptr;
  unsigned long long* h_mask = nullptr;
  int* h_nbr = nullptr;     // neighbour lists of every step (the lattice step's covering tests)
  int* h_nnbr = nullptr;
  double* part = nullptr;   // 2 x [MAXSLOT][NG][pstride]
  double* gacc = nullptr;   // [NG][pstride]
  double2* gg_blk = nullptr;
  double* gg = nullptr;     // 2
  double* gf0 = nullptr;    // [9][ny][nx] FP64 staging of dJ/df0
  std::vector<void*> owned;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  float fwd_ms = 0.f, bwd_ms = 0.f;
  double adj_ms = 0.0, rec_ms = 0.0;
  int64_t adj_n = 0, rec_n = 0;
  std::vector<hipEvent_t> kev;  // per-kernel event pairs when timing
  // a forward pass whose reverse sweep has not run yet (imb_adjoint_forward)
  bool armed = false;
  int run_nsteps = 0;
  bool has_w[3] = {false, false, false};
};

static void release(AdjointState* A) {
  A->armed = false;
  for (void* p : A->owned) hipFree(p);
  A->owned.clear();
  A->ckpt.clear();
  A->ring.clear();
  A->nseg = A->k = A->nsteps = A->np_cap = A->tiles_x = A->tiles_y = 0;
}

void disarm_adjoint(imb_sim* s) {
  SimView v = sim_view(s);
  if (*v.adj) (*v.adj)->armed = false;
}

void free_adjoint(imb_sim* s) {
  SimView v = sim_view(s);
  AdjointState* A = *v.adj;
  if (!A) return;
  release(A);
  for (hipEvent_t& e : A->ev)
    if (e) hipEventDestroy(e);
  for (hipEvent_t e : A->kev) hipEventDestroy(e);
  delete A;
  *v.adj = nullptr;
}

static int take(AdjointState* A, size_t bytes, void** out) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    hipGetLastError();
    return IMB_ENOMEM;
  }
  A->owned.push_back(p);
  *out = p;
  return IMB_OK;
}

template <class P>
static int take_t(AdjointState* A, size_t n, P** out) {
  void* p = nullptr;
  const int rc = take(A, n * sizeof(P), &p);
  *out = (P*)p;
  return rc;
}

static size_t elem_bytes(int storage) { return storage == IMB_STORAGE_F64 ? 8 : 4; }

static int ensure_adjoint(SimView& v, int nsteps, int k) {
  AdjointState*& A = *v.adj;
  if (!A) {
    A = new AdjointState();
    for (hipEvent_t& e : A->ev) hipEventCreate(&e);
  }
  const int nseg = (nsteps + k - 1) / k;
  const int pstride = std::max(v.cfg->max_particles, 1);
  const size_t es = elem_bytes(v.cfg->storage);
  const size_t sb = NQ * (size_t)v.g->plane * es;
  if (A->nseg == nseg && A->k == k && A->nsteps >= nsteps && A->state_bytes == sb &&
      A->np_cap == pstride && A->tiles_x == v.g->tiles_x && A->tiles_y == v.g->tiles_y)
    return IMB_OK;
  release(A);
  int rc = IMB_OK;
  A->ckpt.resize(nseg);
  for (int i = 0; i < nseg && !rc; ++i) rc = take(A, sb, &A->ckpt[i]);
  A->ring.resize(std::max(k - 1, 0));
  for (int i = 0; i < k - 1 && !rc; ++i) rc = take(A, sb, &A->ring[i]);
  for (int i = 0; i < 2 && !rc; ++i) rc = take(A, sb, &A->lam[i]);
  const size_t slots = (size_t)nsteps + 1;
  if (!rc) rc = take_t(A, slots * pstride, &A->h_box);
  if (!rc) rc = take_t(A, slots * pstride, &A->h_pos);
  if (!rc) rc = take_t(A, slots * pstride, &A->h_vel);
  if (!rc) rc = take_t(A, slots * MASK_WORDS * v.g->tiles_y, &A->h_mask);
  if (!rc) rc = take_t(A, slots * (size_t)pstride * NBMAX, &A->h_nbr);
  if (!rc) rc = take_t(A, slots * (size_t)pstride, &A->h_nnbr);
  if (!rc) rc = take_t(A, 2 * (size_t)MAXSLOT * NG * pstride, &A->part);
  if (!rc) rc = take_t(A, (size_t)NG * pstride, &A->gacc);
  if (!rc) rc = take_t(A, (size_t)v.g->tiles_x * v.g->tiles_y, &A->gg_blk);
  if (!rc) rc = take_t(A, 2, &A->gg);
  if (rc) {
    release(A);
    *v.err = "cannot allocate adjoint checkpoints";
    return rc;
  }
  A->nseg = nseg;
  A->k = k;
  A->nsteps = nsteps;
  A->state_bytes = sb;
  A->lam_bytes = sb;
  A->np_cap = pstride;
  A->tiles_x = v.g->tiles_x;  // the tile grid the per-tile buffers are sized for
  A->tiles_y = v.g->tiles_y;
  return IMB_OK;
}

struct TableSlot {
  ParticleTable tab;
  unsigned long long* mask;
  int* nbr;
  int* nnbr;
};

static TableSlot table_slot(const SimView& v, AdjointState* A, int n) {
  const int pstride = std::max(v.cfg->max_particles, 1);
  TableSlot t;
  t.tab.box = A->h_box + (size_t)n * pstride;
  t.tab.pos = A->h_pos + (size_t)n * pstride;
  t.tab.vel = A->h_vel + (size_t)n * pstride;
  t.mask = A->h_mask + (size_t)n * MASK_WORDS * v.g->tiles_y;
  t.nbr = A->h_nbr + (size_t)n * pstride * NBMAX;
  t.nnbr = A->h_nnbr + (size_t)n * pstride;
  return t;
}

static void copy_table(const SimView& v, const ParticleTable& dt, unsigned long long* dmask,
                       const ParticleTable& st, const unsigned long long* smask,
                       hipStream_t s) {
  const int pstride = std::max(v.cfg->max_particles, 1);
  launch_copy(dt.box, st.box, sizeof(int4) * pstride, s);
  launch_copy(dt.pos, st.pos, sizeof(double4) * pstride, s);
  launch_copy(dt.vel, st.vel, sizeof(double4) * pstride, s);
  launch_copy(dmask, smask, sizeof(unsigned long long) * MASK_WORDS * v.g->tiles_y, s);
}

static void copy_lists(const SimView& v, int* dnbr, int* dnnbr, const int* snbr, const int* snnbr,
                       hipStream_t s) {
  const int pstride = std::max(v.cfg->max_particles, 1);
  launch_copy(dnbr, snbr, sizeof(int) * (size_t)pstride * NBMAX, s);
  launch_copy(dnnbr, snnbr, sizeof(int) * (size_t)pstride, s);
}

template <class St>
static void launch_adjoint_step(const AdjointArgs& A, hipStream_t s) {
  const int tiles = A.la.tiles_x * A.la.tiles_y;
  hipLaunchKernelGGL(k_adjoint_step<St>, dim3(tiles + 1), dim3(BLOCK), 0, s, A);
}

}  // namespace imb

using namespace imb;

// Forward pass of the differentiated run: nsteps coupled steps from the current state keeping a
// checkpoint every k steps and the disk tables of every step; J on the host.  Arms the reverse
// sweep (adjoint_reverse).
static int adjoint_forward(imb_sim* sim, int32_t nsteps, int32_t k, const double* wfx,
                           const double* wfy, const double* wtz, double* J) {
  if (!sim) return IMB_EINVAL;
  SimView v = sim_view(sim);
  const imb_config& cfg = *v.cfg;
  if (nsteps < 1 || k < 1) {
    *v.err = "adjoint: nsteps and k_ckpt must be positive";
    return IMB_EINVAL;
  }
  if (cfg.smag_cs != 0.0) {
    *v.err = "adjoint: the Smagorinsky term is not differentiated (smag_cs must be 0)";
    return IMB_EINVAL;
  }
  if (cfg.eps_subcells != 0) {
    *v.err = "adjoint: the sub-cell solid ratio is piecewise constant in the position and has no "
             "useful derivative (eps_subcells must be 0)";
    return IMB_EINVAL;
  }
  if (cfg.kt != 0.0 || cfg.mu != 0.0) {
    *v.err = "adjoint: the tangential contact force is not differentiated (kt and mu must be 0)";
    return IMB_EINVAL;
  }
  if (cfg.storage != IMB_STORAGE_F32 && cfg.storage != IMB_STORAGE_F64) {
    *v.err = "adjoint: needs F32 or F64 storage";
    return IMB_EUNSUPPORTED;
  }
  const int np = *v.np;
  const int pstride = std::max(cfg.max_particles, 1);
  hipStream_t st = v.stream;
  int rc = sync_and_check(sim);
  if (rc) return rc;
  if (np > 0) {
    std::vector<int> mode(np);
    if (hipMemcpy(mode.data(), v.d->ps.mode, sizeof(int) * np, hipMemcpyDeviceToHost) !=
        hipSuccess)
      return hip_fail(v.err, hipGetLastError(), "hipMemcpy(modes)");
    for (int p = 0; p < np; ++p)
      if (mode[p] != IMB_MODE_PRESCRIBED && mode[p] != IMB_MODE_FIXED) {
        *v.err = "adjoint: every disk must be prescribed or fixed (no DEM)";
        return IMB_EINVAL;
      }
  }
  rc = ensure_adjoint(v, nsteps, k);
  if (rc) return rc;
  AdjointState* A = *v.adj;
  drop_graphs(sim);
  DeviceLayout& d = *v.d;

  // weights
  const double* wd[3] = {nullptr, nullptr, nullptr};
  const double* wh[3] = {wfx, wfy, wtz};
  for (int c = 0; c < 3; ++c)
    if (wh[c] && np > 0) {
      if (hipMemcpyAsync(d.w + (size_t)c * pstride, wh[c], sizeof(double) * np,
                         hipMemcpyHostToDevice, st) != hipSuccess)
        return hip_fail(v.err, hipGetLastError(), "hipMemcpyAsync(weights)");
      wd[c] = d.w + (size_t)c * pstride;
    }
  launch_fill_zero(d.J, sizeof(double), st);
  launch_fill_zero(A->gacc, sizeof(double) * NG * pstride, st);
  launch_fill_zero(A->gg_blk, sizeof(double2) * v.g->tiles_x * v.g->tiles_y, st);
  launch_fill_zero(A->lam[0], A->lam_bytes, st);

  // ---- forward pass: checkpoints every k steps, the table of every step
  // the tables of the stored state, and those the state after the last step will use
  const int c0 = *v.cur;
  const ParticleTable live = d.tab[c0];
  unsigned long long* const live_mask = d.band_mask[c0];
  {
    TableSlot t0 = table_slot(v, A, 0);
    copy_table(v, t0.tab, t0.mask, live, live_mask, st);
    copy_lists(v, t0.nbr, t0.nnbr, d.ps.nbr, d.ps.nnbr, st);
  }
  launch_copy(A->ckpt[0], d.f[*v.cur], A->state_bytes, st);
  hipEventRecord(A->ev[0], st);
  const void* src = A->ckpt[0];
  int last = 0;
  for (int n = 0; n < nsteps; ++n) {
    void* dst;
    if ((n + 1) % k == 0 && (n + 1) / k < A->nseg) {
      dst = A->ckpt[(n + 1) / k];
    } else {
      last = (src == d.f[0]) ? 1 : 0;
      dst = d.f[last];
    }
    const TableSlot tn = table_slot(v, A, n);
    LatticeArgs la = lattice_args(sim, src, dst);
    la.tab = tn.tab;
    la.band_mask = tn.mask;
    la.nbr = tn.nbr;
    la.nnbr = tn.nnbr;
    const TableSlot tn1 = table_slot(v, A, n + 1);
    ParticleArgs pa = particle_args(sim, 0);  // writes the history slot instead
    pa.do_finalize = 1;
    pa.do_dem = 1;
    pa.do_table = 1;
    pa.tab = tn1.tab;
    pa.band_mask = tn1.mask;
    pa.wfx = wd[0];
    pa.wfy = wd[1];
    pa.wtz = wd[2];
    pa.J = d.J;
    launch_lattice_step(cfg.storage, la, st);
    if (np > 0) {
      launch_particle_phase(pa, st);
      copy_lists(v, tn1.nbr, tn1.nnbr, d.ps.nbr, d.ps.nnbr, st);
    }
    src = dst;
  }
  hipEventRecord(A->ev[1], st);
  *v.cur = last;
  *v.steps += nsteps;
  {  // the stored state's tables are the ones of the step after the last
    TableSlot tN = table_slot(v, A, nsteps);
    copy_table(v, d.tab[last], d.band_mask[last], tN.tab, tN.mask, st);
  }
  const hipError_t fe = hipGetLastError();
  if (fe != hipSuccess) return hip_fail(v.err, fe, "adjoint forward launch");
  rc = sync_and_check(sim);
  if (rc) return rc;
  hipEventElapsedTime(&A->fwd_ms, A->ev[0], A->ev[1]);
  if (J && hipMemcpy(J, d.J, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail(v.err, hipGetLastError(), "hipMemcpy(J)");
  A->armed = true;
  A->run_nsteps = nsteps;
  for (int c = 0; c < 3; ++c) A->has_w[c] = wd[c] != nullptr;
  return IMB_OK;
}

// Reverse sweep of the armed forward pass: recomputation from the checkpoints and the adjoint
// steps, then the gradients on the host.  Disarms.
static int adjoint_reverse(imb_sim* sim, double* gx0, double* gy0, double* gvx, double* gvy,
                           double* gom, double* gg, double* gf0) {
  if (!sim) return IMB_EINVAL;
  SimView v = sim_view(sim);
  AdjointState* A = *v.adj;
  if (!A || !A->armed) {
    *v.err = "adjoint: no forward pass to reverse (call imb_adjoint_forward first; "
             "imb_set_particles, imb_load_state and a second reverse sweep disarm it)";
    return IMB_EINVAL;
  }
  A->armed = false;
  const imb_config& cfg = *v.cfg;
  const int np = *v.np;
  const int pstride = std::max(cfg.max_particles, 1);
  const int nsteps = A->run_nsteps, k = A->k;
  hipStream_t st = v.stream;
  DeviceLayout& d = *v.d;
  const double* wd[3];
  for (int c = 0; c < 3; ++c) wd[c] = A->has_w[c] ? d.w + (size_t)c * pstride : nullptr;
  int rc = IMB_OK;
  drop_graphs(sim);

  // ---- reverse sweep
  const bool timing = *v.timing;
  auto timed = [&](bool adj, auto&& launch) {
    if (!timing) {
      launch();
      return;
    }
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipEventRecord(e0, st);
    launch();
    hipEventRecord(e1, st);
    A->kev.push_back(e0);
    A->kev.push_back(e1);
    (void)adj;
  };
  std::vector<char> kind;  // per timed pair: 1 adjoint, 0 recompute
  hipEventRecord(A->ev[2], st);
  int li = 0;  // lam[li] holds dJ/d(state after the step being reversed)
  const int tiles = v.g->tiles_x * v.g->tiles_y;
  for (int s = A->nseg - 1; s >= 0; --s) {
    const int n0 = s * k, n1 = std::min(n0 + k, nsteps);
    // recompute the segment's states n0 .. n1 - 2 into the ring
    const void* rs = A->ckpt[s];
    for (int n = n0; n <= n1 - 2; ++n) {
      void* dst = A->ring[n - n0];
      const TableSlot tn = table_slot(v, A, n);
      LatticeArgs la = lattice_args(sim, rs, dst);
      la.tab = tn.tab;
      la.band_mask = tn.mask;
      la.nbr = tn.nbr;
      la.nnbr = tn.nnbr;
      timed(false, [&] { launch_lattice_step(cfg.storage, la, st); });
      if (timing) kind.push_back(0);
      rs = dst;
    }
    for (int n = n1 - 1; n >= n0; --n) {
      const void* sprev = n == n0 ? A->ckpt[s] : A->ring[n - n0 - 1];
      const TableSlot tn = table_slot(v, A, n);
      AdjointArgs aa{};
      aa.la = lattice_args(sim, sprev, nullptr);
      aa.la.tab = tn.tab;
      aa.la.band_mask = tn.mask;
      aa.lam_in = A->lam[li];
      aa.lam_out = A->lam[li ^ 1];
      aa.wfx = wd[0];
      aa.wfy = wd[1];
      aa.wtz = wd[2];
      aa.part = A->part + (size_t)(n & 1) * MAXSLOT * NG * pstride;
      aa.gg_blk = A->gg_blk;
      aa.mode = d.ps.mode;
      aa.gacc = A->gacc;
      if (n + 1 < nsteps && np > 0) {
        aa.fin_step = n + 1;
        aa.fin_part = A->part + (size_t)((n + 1) & 1) * MAXSLOT * NG * pstride;
        aa.fin_box = table_slot(v, A, n + 1).tab.box;
      } else {
        aa.fin_step = -1;
      }
      if (cfg.storage == IMB_STORAGE_F64)
        timed(true, [&] { launch_adjoint_step<StoreF64>(aa, st); });
      else
        timed(true, [&] { launch_adjoint_step<StoreF32>(aa, st); });
      if (timing) kind.push_back(1);
      li ^= 1;
    }
  }
  hipLaunchKernelGGL(k_adjoint_final, dim3(1), dim3(BLOCK), 0, st, np, pstride, A->part,
                     table_slot(v, A, 0).tab.box, (const int*)d.ps.mode, A->gacc,
                     (const double2*)A->gg_blk, tiles, A->gg);
  hipEventRecord(A->ev[3], st);
  (void)tiles;
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess) return hip_fail(v.err, le, "adjoint launch");

  rc = sync_and_check(sim);
  if (rc) return rc;
  hipEventElapsedTime(&A->bwd_ms, A->ev[2], A->ev[3]);
  if (timing) {
    for (size_t i = 0; i + 1 < A->kev.size(); i += 2) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, A->kev[i], A->kev[i + 1]);
      if (kind[i / 2]) {
        A->adj_ms += ms;
        A->adj_n++;
      } else {
        A->rec_ms += ms;
        A->rec_n++;
      }
    }
    for (hipEvent_t e : A->kev) hipEventDestroy(e);
    A->kev.clear();
  }

  // ---- outputs
  double* outs[NG] = {gx0, gy0, gvx, gvy, gom};
  for (int c = 0; c < NG; ++c)
    if (outs[c] && np > 0 &&
        hipMemcpy(outs[c], A->gacc + (size_t)c * pstride, sizeof(double) * np,
                  hipMemcpyDeviceToHost) != hipSuccess)
      return hip_fail(v.err, hipGetLastError(), "hipMemcpy(gradients)");
  if (gg && hipMemcpy(gg, A->gg, 2 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail(v.err, hipGetLastError(), "hipMemcpy(dJ/dg)");
  if (gf0) {
    const size_t n = (size_t)NQ * cfg.nx * cfg.ny;
    if (!A->gf0 && take_t(A, n, &A->gf0)) {
      *v.err = "adjoint: cannot allocate dJ/df0 staging";
      return IMB_ENOMEM;
    }
    LatticeArgs la = lattice_args(sim, nullptr, nullptr);
    const int blocks = (int)((cfg.nx * (long long)cfg.ny + BLOCK - 1) / BLOCK);
    if (cfg.storage == IMB_STORAGE_F64)
      hipLaunchKernelGGL(k_pull_adjoint<double>, dim3(blocks), dim3(BLOCK), 0, st, la,
                         (const double*)A->lam[li], A->gf0);
    else
      hipLaunchKernelGGL(k_pull_adjoint<float>, dim3(blocks), dim3(BLOCK), 0, st, la,
                         (const float*)A->lam[li], A->gf0);
    if (hipMemcpyAsync(gf0, A->gf0, n * sizeof(double), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return hip_fail(v.err, hipGetLastError(), "hipMemcpy(dJ/df0)");
    rc = sync_and_check(sim);
    if (rc) return rc;
  }
  return IMB_OK;
}

extern "C" int imb_adjoint_forward(imb_sim* sim, int32_t nsteps, int32_t k_ckpt,
                                   const double* wfx, const double* wfy, const double* wtz,
                                   double* J) {
  return adjoint_forward(sim, nsteps, k_ckpt, wfx, wfy, wtz, J);
}

extern "C" int imb_adjoint_backward(imb_sim* sim, double* gx0, double* gy0, double* gvx,
                                    double* gvy, double* gom, double* gg, double* gf0) {
  return adjoint_reverse(sim, gx0, gy0, gvx, gvy, gom, gg, gf0);
}

extern "C" int imb_adjoint(imb_sim* sim, int32_t nsteps, int32_t k, const double* wfx,
                           const double* wfy, const double* wtz, double* gx0, double* gy0,
                           double* gvx, double* gvy, double* gom, double* gg, double* J,
                           double* gf0) {
  int rc = adjoint_forward(sim, nsteps, k, wfx, wfy, wtz, J);
  if (rc) return rc;
  return adjoint_reverse(sim, gx0, gy0, gvx, gvy, gom, gg, gf0);
}

extern "C" int imb_get_adjoint_timing(imb_sim* sim, double* forward_ms, double* reverse_ms,
                                      double* adjoint_kernel_ms, int64_t* adjoint_kernels,
                                      double* recompute_kernel_ms, int64_t* recompute_kernels) {
  if (!sim) return IMB_EINVAL;
  SimView v = sim_view(sim);
  AdjointState* A = *v.adj;
  if (forward_ms) *forward_ms = A ? A->fwd_ms : 0.0;
  if (reverse_ms) *reverse_ms = A ? A->bwd_ms : 0.0;
  if (adjoint_kernel_ms) *adjoint_kernel_ms = A ? A->adj_ms : 0.0;
  if (adjoint_kernels) *adjoint_kernels = A ? A->adj_n : 0;
  if (recompute_kernel_ms) *recompute_kernel_ms = A ? A->rec_ms : 0.0;
  if (recompute_kernels) *recompute_kernels = A ? A->rec_n : 0;
  if (A) {
    A->adj_ms = A->rec_ms = 0.0;
    A->adj_n = A->rec_n = 0;
  }
  return IMB_OK;
}
