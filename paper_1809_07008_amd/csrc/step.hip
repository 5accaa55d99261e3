// step.hip -- the fused lattice step: per-cell solid ratio of the disks (Sec. 2.2), IMB
// collision with Smagorinsky relaxation and body force (Eqs. 1, 2, 12-14), streaming with
// periodic x and half-way bounce-back walls (left side of Eq. 1), and per-tile partial sums of
// the hydrodynamic force and torque on each disk (Eqs. 15, 16).
//
// Layout: populations are structure-of-arrays planes f[q][y][x] with a padded row pitch; the
// kernel pulls f_i(x - c_i) from the previous step's post-collision planes (so every load and
// store of a wave is a contiguous 64-element row segment) and writes this step's post-collision
// values at x.  One 256-thread workgroup owns a tile of cells; it first finds the disks whose
// tile boxes touch the tile (an ordered compaction over all disks, so lists are sorted by id),
// evaluates eps only for those, and reduces each disk's force/torque over the tile with wave
// shuffles into one slot of the disk's partial-sum row (no atomics: the result is bit-for-bit
// reproducible).
#include "collide.h"
#include "solid.h"
#include "step.h"

namespace imb {

template <class T>
struct PEntry {
  int ix, iy, pid, slot;
  T fx, fy, r, vx, vy, om;
};

// Disks whose tile box contains tile (tx, ty), sorted by id (so every sum over them has a fixed
// order).  Candidates come from the tile row's band list written by the particle phase.  Returns
// the count (capped at LMAX; overflow latches ERR_TILE_LIST).  Block-uniform control flow.
template <class T>
__device__ int build_tile_list(const LatticeArgs& a, int tx, int ty, PEntry<T>* pl, int* s_cnt,
                               int* s_pid, int* s_slot) {
  if (a.np == 0) return 0;
  const int b0 = a.band_off[ty], b1 = a.band_off[ty + 1];
  if (b1 <= b0) return 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int base = 0;
  for (int k0 = b0; k0 < b1; k0 += BLOCK) {
    const int k = k0 + tid;
    int p = -1, slot = -1;
    if (k < b1) {
      p = a.band_ids[k];
      slot = box_slot(a.tab.box[p], tx, ty, a.tiles_x, a.tiles_y);
    }
    const bool hit = slot >= 0;
    const unsigned long long m = __ballot(hit);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_cnt[wave] = __popcll(m);
    __syncthreads();
    int off = base, total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      if (w < wave) off += s_cnt[w];
      total += s_cnt[w];
    }
    if (hit) {
      const int q = off + below;
      if (q < LMAX) {
        s_pid[q] = p;
        s_slot[q] = slot;
      } else {
        atomicOr(a.err, ERR_TILE_LIST);
      }
    }
    base += total;
    __syncthreads();
  }
  const int n = base < LMAX ? base : LMAX;
  if (tid < n) {
    const int p = s_pid[tid];
    int rank = 0;
    for (int q = 0; q < n; ++q) rank += s_pid[q] < p;
    const double4 ps = a.tab.pos[p];
    const double4 vl = a.tab.vel[p];
    const double flx = floor(ps.x), fly = floor(ps.y);
    PEntry<T> e;
    e.ix = (int)flx;
    e.iy = (int)fly;
    e.pid = p;
    e.slot = s_slot[tid];
    e.fx = (T)(ps.x - flx);
    e.fy = (T)(ps.y - fly);
    e.r = (T)ps.z;
    e.vx = (T)vl.x;
    e.vy = (T)vl.y;
    e.om = (T)vl.z;
    pl[rank] = e;
  }
  __syncthreads();
  return n;
}

// Per-thread scratch of a tile in LDS (indexed [k][thread] so a wave touches 64 distinct
// banks): the disks covering the current cell and the thread's running force sums.
template <class T>
struct CellScratch {
  int cj[MAXC][BLOCK];     // list entries of the disks covering the current cell
  T ce[MAXC][BLOCK];       // their eps
  int aj[MAXC][BLOCK];     // list entries owning the thread's accumulators (-1: free)
  T af[3][MAXC][BLOCK];    // accumulated force x, y and torque
};

template <class T>
__device__ inline void lever_arm(const LatticeArgs& a, const PEntry<T>& e, int x, int y, T* dx,
                                 T* dy) {
  int di = x - e.ix;
  const int hx = a.nx / 2, hy = a.ny / 2;
  if (di > hx) di -= a.nx;
  else if (di < -hx) di += a.nx;
  int dj = y - e.iy;
  if (!a.walls) {
    if (dj > hy) dj -= a.ny;
    else if (dj < -hy) dj += a.ny;
  }
  *dx = (T)di - e.fx;
  *dy = (T)dj - e.fy;
}

// Disks covering cell (x, y): eps > 0 with the image nearest to the cell, evaluated directly
// (used by the solid-ratio diagnostic).  Returns their count.
template <class T>
__device__ inline int covering_disks(const LatticeArgs& a, const PEntry<T>* pl, int n, int x,
                                     int y, CellScratch<T>& cs) {
  const int tid = threadIdx.x;
  int nc = 0;
  for (int j = 0; j < n; ++j) {
    T dx, dy;
    lever_arm(a, pl[j], x, y, &dx, &dy);
    const T eps = solid_fraction<T>(pl[j].r, dx, dy);
    if (eps > T(0)) {
      if (nc < MAXC) {
        cs.cj[nc][tid] = j;
        cs.ce[nc][tid] = eps;
        ++nc;
      } else {
        atomicOr(a.err, ERR_CELL);
      }
    }
  }
  return nc;
}

// Disks whose image nearest to cell (x, y) reaches the cell, classified with the cheap tests of
// solid_fraction: inside cells get eps = 1 now; cut cells are appended to the tile's queue
// (owner thread, slot, disk) and get their exact area from the whole block afterwards, so the
// expensive branch runs on densely packed lanes.  Returns the count.
template <class T>
__device__ inline int classify_cell(const LatticeArgs& a, const PEntry<T>* pl, int n, int x, int y,
                                    CellScratch<T>& cs, int* s_qn, int* s_q) {
  const int tid = threadIdx.x;
  int nc = 0;
  for (int j = 0; j < n; ++j) {
    T dx, dy;
    lever_arm(a, pl[j], x, y, &dx, &dy);
    const T r = pl[j].r;
    const T x0 = dx - T(0.5), x1 = dx + T(0.5), y0 = dy - T(0.5), y1 = dy + T(0.5);
    const T nx = x0 > T(0) ? x0 : (x1 < T(0) ? x1 : T(0));
    const T ny = y0 > T(0) ? y0 : (y1 < T(0) ? y1 : T(0));
    if (nx * nx + ny * ny >= r * r) continue;
    if (nc >= MAXC) {
      atomicOr(a.err, ERR_CELL);
      continue;
    }
    const T fx = fabs(x0) > fabs(x1) ? fabs(x0) : fabs(x1);
    const T fy = fabs(y0) > fabs(y1) ? fabs(y0) : fabs(y1);
    cs.cj[nc][tid] = j;
    if (fx * fx + fy * fy <= r * r) {
      cs.ce[nc][tid] = T(1);
    } else {
      const int q = atomicAdd(s_qn, 1);
      s_q[q] = tid | (nc << 8) | (j << 10);
    }
    ++nc;
  }
  return nc;
}

// Pull-stream load of the 9 populations arriving at (x, y).
template <class St>
__device__ inline void pull_load(const LatticeArgs& a, const typename St::S* src, int x, int y,
                                 typename St::T f[NQ]) {
  using T = typename St::T;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    int xs = x - cx_of(i), ys = y - cy_of(i);
    xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
    long long idx;
    if (ys < 0 || ys >= a.ny) {
      if (a.walls) {  // half-way bounce-back: the link left through the wall and came back
        idx = (long long)opp_of(i) * a.plane + (long long)y * a.pitch + x;
        f[i] = St::load(src, idx, T(0));
        continue;
      }
      ys = ys < 0 ? ys + a.ny : ys - a.ny;
    }
    idx = (long long)i * a.plane + (long long)ys * a.pitch + xs;
    f[i] = St::load(src, idx, T(0));
  }
}

// Compensated (hi, lo) pair used for the force sums in FP32; plain sum in FP64.
template <class T>
struct Acc {
  T hi, lo;
  __device__ void add(T v) {
    const T s = hi + v;
    const T bp = s - hi;
    lo += (hi - (s - bp)) + (v - bp);
    hi = s;
  }
  __device__ void add(const Acc& o) {
    add(o.hi);
    lo += o.lo;
  }
};

// Wave-wide sum with DPP row rotations (no LDS traffic): rotating by 8, 4, 2, 1 lanes inside each
// row of 16 leaves the row total in every lane; lanes 0, 16, 32, 48 are then added in fixed
// order, so the result is the same on every run.
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL, class T>
__device__ inline void dpp_add(Acc<T>& v) {
  Acc<T> o;
  o.hi = dpp_move<CTRL>(v.hi);
  o.lo = dpp_move<CTRL>(v.lo);
  v.add(o);
}

template <class T>
__device__ inline Acc<T> wave_sum(Acc<T> v) {
  dpp_add<0x128>(v);  // row_ror:8
  dpp_add<0x124>(v);  // row_ror:4
  dpp_add<0x122>(v);  // row_ror:2
  dpp_add<0x121>(v);  // row_ror:1
  Acc<T> t{read_lane(v.hi, 0), read_lane(v.lo, 0)};
#pragma unroll
  for (int row = 1; row < 4; ++row) t.add(Acc<T>{read_lane(v.hi, 16 * row), read_lane(v.lo, 16 * row)});
  return t;
}

template <class St>
__global__ __launch_bounds__(BLOCK) void k_lattice_step(LatticeArgs a) {
  using T = typename St::T;
  using S = typename St::S;
  __shared__ PEntry<T> s_pl[LMAX];
  __shared__ int s_cnt[WAVES];
  __shared__ int s_pid[LMAX], s_slot[LMAX];
  __shared__ unsigned s_touch;
  __shared__ int s_qn;
  __shared__ int s_q[BLOCK * MAXC];
  __shared__ Acc<T> s_red[WAVES][LMAX][3];
  __shared__ CellScratch<T> cs;

  const int tid = threadIdx.x;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tw = 1 << a.tw_log, th = BLOCK >> a.tw_log;
  const int lx = tid & (tw - 1), ly = tid >> a.tw_log;
  const int x = tx * tw + lx;
  const int ybase = ty * th * a.rows + ly;
  const S* src = (const S*)a.src;
  S* dst = (S*)a.dst;

  if (tid == 0) s_touch = 0u;
  // the first row's populations are requested before the disk list is built, so their latency
  // overlaps the list's
  T f[NQ];
  if (x < a.nx && ybase < a.ny) pull_load<St>(a, src, x, ybase, f);
  const int n = build_tile_list<T>(a, tx, ty, s_pl, s_cnt, s_pid, s_slot);
  if (n > 0) {
#pragma unroll
    for (int q = 0; q < MAXC; ++q) cs.aj[q][tid] = -1;
  }

  const T tau0 = (T)a.tau0, csm = (T)a.cs, gx = (T)a.gx, gy = (T)a.gy, rho0 = (T)a.rho0;
  for (int rr = 0; rr < a.rows; ++rr) {
    const int y = ybase + rr * th;
    const bool valid = x < a.nx && y < a.ny;
    if (rr > 0 && valid) pull_load<St>(a, src, x, y, f);
    int nc = 0;
    if (n > 0) {  // block-uniform
      if (tid == 0) s_qn = 0;
      __syncthreads();
      if (valid) nc = classify_cell<T>(a, s_pl, n, x, y, cs, &s_qn, s_q);
      __syncthreads();
      const int qn = s_qn;
      for (int q = tid; q < qn; q += BLOCK) {  // exact areas of the tile's cut cells
        const int code = s_q[q];
        const int owner = code & 255, k = (code >> 8) & 3, j = code >> 10;
        const int ox = tx * tw + (owner & (tw - 1));
        const int oy = ybase - ly + (owner >> a.tw_log) + rr * th;
        T dx, dy;
        lever_arm(a, s_pl[j], ox, oy, &dx, &dy);
        cs.ce[k][owner] = cut_cell_fraction<T>(s_pl[j].r, dx - T(0.5), dx + T(0.5),
                                               dy - T(0.5), dy + T(0.5));
      }
      __syncthreads();
    }
    if (!valid) continue;
    T fo[NQ];
    auto disk = [&](int k) {
      const int j = cs.cj[k][tid];
      Disk<T> d;
      d.eps = cs.ce[k][tid];
      lever_arm(a, s_pl[j], x, y, &d.dx, &d.dy);
      d.vx = s_pl[j].vx;
      d.vy = s_pl[j].vy;
      d.om = s_pl[j].om;
      return d;
    };
    auto emit = [&](int k, T fx, T fy, T tz) {
      const int j = cs.cj[k][tid];
      int q = 0;
      for (; q < MAXC; ++q) {
        const int o = cs.aj[q][tid];
        if (o == j) break;
        if (o < 0) {
          cs.aj[q][tid] = j;
          cs.af[0][q][tid] = T(0);
          cs.af[1][q][tid] = T(0);
          cs.af[2][q][tid] = T(0);
          break;
        }
      }
      if (q == MAXC) {
        atomicOr(a.err, ERR_CELL);
        return;
      }
      cs.af[0][q][tid] += fx;
      cs.af[1][q][tid] += fy;
      cs.af[2][q][tid] += tz;
    };
    T rho;
    if constexpr (St::deviation) {
      rho = collide_dev(f, nc, disk, emit, rho0, tau0, csm, gx, gy, fo);
    } else {
      rho = collide_plain(f, nc, disk, emit, tau0, csm, gx, gy, fo);
    }
    if (!(rho > T(0)) || !isfinite(rho)) atomicOr(a.err, ERR_RHO);
    const long long base = (long long)y * a.pitch + x;
#pragma unroll
    for (int i = 0; i < NQ; ++i) St::store(dst, (long long)i * a.plane + base, fo[i], T(0));
  }
  if (n == 0) return;  // block-uniform: no disk touches this tile

  // which list entries received a contribution in this tile
  unsigned mine = 0u;
#pragma unroll
  for (int q = 0; q < MAXC; ++q) {
    const int o = cs.aj[q][tid];
    if (o >= 0) mine |= 1u << o;
  }
  if (mine) atomicOr(&s_touch, mine);
  __syncthreads();
  const unsigned touched = s_touch;
  const int lane = tid & 63, wave = tid >> 6;

  // each wave reduces every touched disk over its cells; one barrier; then one thread per
  // disk adds the four waves in fixed order and writes the tile's slot
  for (int j = 0; j < n; ++j) {
    if (!((touched >> j) & 1u)) continue;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      Acc<T> v{T(0), T(0)};
#pragma unroll
      for (int q = 0; q < MAXC; ++q)
        if (cs.aj[q][tid] == j) v.add(cs.af[comp][q][tid]);
      v = wave_sum(v);
      if (lane == 0) s_red[wave][j][comp] = v;
    }
  }
  __syncthreads();
  if (tid < n) {
    const int j = tid;
    double out[3] = {0.0, 0.0, 0.0};
    if ((touched >> j) & 1u) {
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        Acc<T> v = s_red[0][j][comp];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) v.add(s_red[w][j][comp]);
        out[comp] = (double)v.hi + (double)v.lo;
      }
    }
    a.partials[(long long)s_pl[j].slot * a.pstride + s_pl[j].pid] =
        make_double4(out[0], out[1], out[2], 0.0);
  }
}

// eps_tot of every cell (diagnostic / parity of the solid-ratio stage alone).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_solid_field(LatticeArgs a, double* eps_out) {
  __shared__ PEntry<T> s_pl[LMAX];
  __shared__ int s_cnt[WAVES];
  __shared__ int s_pid[LMAX], s_slot[LMAX];
  __shared__ CellScratch<T> cs;
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tw = 1 << a.tw_log, th = BLOCK >> a.tw_log;
  const int x = tx * tw + (tid & (tw - 1));
  const int ybase = ty * th * a.rows + (tid >> a.tw_log);
  const int n = build_tile_list<T>(a, tx, ty, s_pl, s_cnt, s_pid, s_slot);
  for (int rr = 0; rr < a.rows; ++rr) {
    const int y = ybase + rr * th;
    if (x >= a.nx || y >= a.ny) continue;
    const int nc = covering_disks<T>(a, s_pl, n, x, y, cs);
    double s = 0.0;
    for (int k = 0; k < nc; ++k) s += (double)cs.ce[k][tid];
    eps_out[(long long)y * a.nx + x] = s;
  }
}

template <class St>
void launch_lattice_step_t(const LatticeArgs& a, hipStream_t s) {
  const int tiles = a.tiles_x * a.tiles_y;
  hipLaunchKernelGGL(k_lattice_step<St>, dim3(tiles), dim3(BLOCK), 0, s, a);
}

void launch_lattice_step(int storage, const LatticeArgs& a, hipStream_t s) {
  switch (storage) {
    case IMB_STORAGE_F64: launch_lattice_step_t<StoreF64>(a, s); break;
    case IMB_STORAGE_F32: launch_lattice_step_t<StoreF32>(a, s); break;
    default: launch_lattice_step_t<StoreF16>(a, s); break;
  }
}

void launch_solid_field(int storage, const LatticeArgs& a, double* eps_out, hipStream_t s) {
  const int tiles = a.tiles_x * a.tiles_y;
  if (storage == IMB_STORAGE_F64)
    hipLaunchKernelGGL(k_solid_field<double>, dim3(tiles), dim3(BLOCK), 0, s, a, eps_out);
  else
    hipLaunchKernelGGL(k_solid_field<float>, dim3(tiles), dim3(BLOCK), 0, s, a, eps_out);
}

}  // namespace imb
