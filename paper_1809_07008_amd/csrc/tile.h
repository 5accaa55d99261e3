// tile.h -- device helpers shared by the lattice-step and adjoint kernels: the per-tile disk
// list, the per-thread scratch of covering disks, pull-stream loads with the wall rule, and the
// deterministic compensated wave reductions used for per-disk sums.
#pragma once

#include "common.h"
#include "solid.h"

namespace imb {

template <class T>
struct PEntry {
  int ix, iy, pid, slot;
  T fx, fy, r, vx, vy, om;
};

// Disks whose tile box contains tile (tx, ty), sorted by id (so every sum over them has a fixed
// order).  The tile row's band mask (particle phase) names the disks whose box touches the row:
// wavefront w reads words w and w + WAVES of it (scalar loads) and its lanes test the boxes of
// the disks 64 w + lane and 64 (w + WAVES) + lane that are set; one barrier orders the hits by
// id.  ty counts inside the window (boxes are in lattice tile rows, ty + ty_off).  Returns the
// count (capped at LMAX; overflow latches ERR_TILE_LIST).  Block-uniform control flow.  s_cnt
// holds 2 WAVES ints.
static_assert(MASK_WORDS == 2 * WAVES, "two band-mask words per wavefront");
template <class T>
__device__ int build_tile_list(const LatticeArgs& a, int tx, int ty, PEntry<T>* pl, int* s_cnt,
                               int* s_pid, int* s_slot) {
  const int np = a.np;
  if (np == 0) return 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tyg = ty + a.ty_off;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int w1 = wave + WAVES;
  const unsigned long long c0 = 64 * wave < np ? a.band_mask[wave * a.tiles_y + ty] : 0ull;
  const unsigned long long c1 = 64 * w1 < np ? a.band_mask[w1 * a.tiles_y + ty] : 0ull;
  const int p0 = 64 * wave + lane, p1 = 64 * w1 + lane;
  int s0 = -1, s1 = -1;  // a set bit names a disk below np
  if ((c0 >> lane) & 1ull) s0 = box_slot(a.tab.box[p0], tx, tyg, a.tiles_x, a.tiles_yg);
  if ((c1 >> lane) & 1ull) s1 = box_slot(a.tab.box[p1], tx, tyg, a.tiles_x, a.tiles_yg);
  const unsigned long long m0 = __ballot(s0 >= 0), m1 = __ballot(s1 >= 0);
  if (lane == 0) {
    s_cnt[wave] = __popcll(m0);
    s_cnt[WAVES + wave] = __popcll(m1);
  }
  __syncthreads();
  int off0 = 0, off1 = 0, base = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    if (w < wave) {
      off0 += s_cnt[w];
      off1 += s_cnt[WAVES + w];
    }
    off1 += s_cnt[w];  // every hit of the first words precedes the second words'
    base += s_cnt[w] + s_cnt[WAVES + w];
  }
  const int q0 = off0 + __popcll(m0 & lt), q1 = off1 + __popcll(m1 & lt);
  if (s0 >= 0) {
    if (q0 < LMAX) {
      s_pid[q0] = p0;
      s_slot[q0] = s0;
    } else {
      atomicOr(a.err, ERR_TILE_LIST);
    }
  }
  if (s1 >= 0) {
    if (q1 < LMAX) {
      s_pid[q1] = p1;
      s_slot[q1] = s1;
    } else {
      atomicOr(a.err, ERR_TILE_LIST);
    }
  }
  __syncthreads();
  const int n = base < LMAX ? base : LMAX;
  if (tid < n) {  // s_pid is ascending: entry tid is the tid-th smallest id
    const int p = s_pid[tid];
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
    pl[tid] = e;
  }
  __syncthreads();
  return n;
}

// Per-thread scratch of a tile in LDS (indexed [k][thread] so a wave touches 64 distinct
// banks): the disks covering the current cell.
template <class T>
struct CellScratch {
  int cj[MAXC][BLOCK];     // list entries of the disks covering the current cell
  T ce[MAXC][BLOCK];       // their eps
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
                                     int y, CellScratch<T>& cs, const T* off) {
  const int tid = threadIdx.x;
  int nc = 0;
  for (int j = 0; j < n; ++j) {
    T dx, dy;
    lever_arm(a, pl[j], x, y, &dx, &dy);
    const T eps = cell_solid_ratio<T>(pl[j].r, dx, dy, a.eps_sub, off);
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

// Pull-stream load of the 9 populations arriving at (x, y) (lattice coordinates).  W: the
// lattice is a slab whose plane rows run from y0 - 1 to y0 + nyl (ghost rows included), so a
// source row beyond the window is read from a ghost row instead of wrapping around the lattice.
template <class St, bool W = false>
__device__ inline void pull_load(const LatticeArgs& a, const typename St::S* src, int x, int y,
                                 typename St::T f[NQ]) {
  using T = typename St::T;
  const int yoff = W ? a.yoff : 0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    int xs = x - cx_of(i), ys = y - cy_of(i);
    xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
    long long idx;
    if (ys < 0 || ys >= a.ny) {
      if (a.walls) {  // half-way bounce-back: the link left through the wall and came back
        idx = (long long)opp_of(i) * a.plane + (long long)(y - yoff) * a.pitch + x;
        f[i] = St::load(src, idx, T(0));
        continue;
      }
      if (!W) ys = ys < 0 ? ys + a.ny : ys - a.ny;
    }
    idx = (long long)i * a.plane + (long long)(ys - yoff) * a.pitch + xs;
    f[i] = St::load(src, idx, T(0));
  }
}

// Element at byte offset boff of p: a uniform base plus one 32-bit offset per lane, the form of
// the global memory instructions that take a scalar base.
template <class S>
__device__ __forceinline__ const S* at_bytes(const S* p, unsigned boff) {
  return (const S*)((const char*)p + boff);
}
template <class S>
__device__ __forceinline__ S* at_bytes(S* p, unsigned boff) {
  return (S*)((char*)p + boff);
}

// Pull-stream loads of a cell whose eight neighbours all lie inside the lattice (no periodic
// wrap, no wall link): population i comes from the fixed shift (-cx_i, -cy_i) of the cell, so its
// load is plane i's base moved by that shift (uniform) plus the cell's own byte offset.
template <class St>
__device__ inline void pull_load_inner(const LatticeArgs& a, const typename St::S* src,
                                       unsigned boff, typename St::T f[NQ]) {
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const typename St::S* p =
        src + ((long long)i * a.plane - (long long)cy_of(i) * a.pitch - cx_of(i));
    f[i] = St::decode(*at_bytes(p, boff));
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

}  // namespace imb
