// disk_block.h -- the lattice step split by who owns a cell.
//
// A cell that no disk covers is a fluid cell: its tile collides it with the plain BGK + body-force
// update and stores it (fluid_tile).  A cell covered by one or more disks (the covering test of
// covers_cell, the one every kernel uses) belongs to the covering disk with the lowest id; that
// disk's workgroup (disk_cells) pulls its populations, evaluates the exact solid ratio of every
// covering disk, applies the IMB collision (Eqs. 1, 2, 12-14, with the several-disk reading of
// collide.h) and stores it.  Every covering disk's workgroup also evaluates the cell to obtain
// its own share of the hydrodynamic force and torque (Eqs. 15, 16), so each workgroup reduces
// exactly its own disk's sums; there is no cross-workgroup accumulation and no atomic, and the
// results do not depend on scheduling.
//
// Disks that can cover a common cell are neighbours in the DEM neighbour list (its skin keeps
// every pair closer than r_p + r_q + sqrt 2 listed until the next rebuild), so a disk's workgroup
// finds the other covering disks among its neighbours.  Tiles still use the per-tile candidate
// lists to know which of their cells are covered.
#pragma once

#include "collide.h"
#include "tile.h"

namespace imb {

// Plain update of the uncovered cells of one tile (one BLOCK-thread workgroup): only they are
// loaded and stored.  W: the lattice is a window of rows with ghost rows (tile.h, pull_load).
template <class St, bool W = false>
__device__ void fluid_tile(const LatticeArgs& a, int tile) {
  using T = typename St::T;
  using S = typename St::S;
  __shared__ PEntry<T> s_pl[LMAX];
  __shared__ int s_cnt[2 * WAVES];
  __shared__ int s_pid[LMAX], s_slot[LMAX];

  const int tid = threadIdx.x;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tw = 1 << a.tw_log, th = BLOCK >> a.tw_log;
  const int lx = tid & (tw - 1), ly = tid >> a.tw_log;
  const int x = tx * tw + lx;
  const int y0 = W ? a.y0 : 0;           // first row of the window
  const int yend = W ? y0 + a.nyl : a.ny;
  const int nyl = W ? a.nyl : a.ny;
  const int yoff = W ? a.yoff : 0;       // plane row of lattice row y: y - yoff
  // the plane rows next to the window hold its neighbours' rows (ghost rows) or lie beyond a
  // wall
  const bool lo_ok = W && a.ghost_lo, hi_ok = W && a.ghost_hi;
  const int ybase = y0 + ty * th * a.rows + ly;
  const S* src = (const S*)a.src;
  S* dst = (S*)a.dst;

  unsigned seed = 0u;
  if constexpr (St::stochastic) seed = a.seed[a.seed_slot];
  const int n = build_tile_list<T>(a, tx, ty, s_pl, s_cnt, s_pid, s_slot);

  const T tau0 = (T)a.tau0, csm = (T)a.cs, gx = (T)a.gx, gy = (T)a.gy, rho0 = (T)a.rho0;
  // byte offsets within one plane fit 32 bits: stores (and the inner loads) take the
  // scalar-base form
  const bool off32 = (unsigned long long)a.plane * sizeof(S) <= 0xFFFFFFFFull;
  // the tile's columns have both x neighbours inside the lattice
  const bool xin = tx * tw >= 1 && tx * tw + tw <= a.nx - 1;
  // this thread's cell of pass rr exists and no disk covers it (a covered cell is loaded and
  // stored by the workgroup of its lowest-id covering disk)
  auto live = [&](int y) {
    if (x >= a.nx || y >= yend) return false;
    for (int j = 0; j < n; ++j) {
      T dx, dy;
      lever_arm(a, s_pl[j], x, y, &dx, &dy);
      if (covers_cell<T>(s_pl[j].r, dx, dy)) return false;
    }
    return true;
  };
  auto load = [&](int rr, int y, T f[NQ]) {
    // every cell of pass rr has its eight neighbours in stored rows (uniform)
    const int ylo = ybase - ly + rr * th - y0;  // window row of the pass's first row
    const bool inner = off32 && xin && (ylo >= 1 || lo_ok) && (ylo + th <= nyl - 1 || hi_ok);
    if (inner)
      pull_load_inner<St>(a, src, (unsigned)((y - yoff) * a.pitch + x) * (unsigned)sizeof(S), f);
    else pull_load<St, W>(a, src, x, y, f);
  };
  auto update = [&](int y, const T f[NQ]) {
    T fo[NQ];
    auto none = [&](int) { return Disk<T>{}; };
    auto drop = [&](int, T, T, T) {};
    T rho;
    if constexpr (St::deviation) {
      rho = collide_dev(f, 0, none, drop, rho0, tau0, csm, gx, gy, fo);
    } else {
      rho = collide_plain(f, 0, none, drop, tau0, csm, gx, gy, fo);
    }
    if (!(rho > T(0)) || !isfinite(rho)) atomicOr(a.err, ERR_RHO);
    wall_adjust<T>(a, y, fo);
    const long long base = (long long)(y - yoff) * a.pitch + x;
    S out[NQ];
    if constexpr (St::stochastic) {
      // the random words follow the lattice cell, not its place in the window
      unsigned rnd[NQ];
      sr_words(seed, (unsigned)((long long)y * a.pitch + x), rnd);
#pragma unroll
      for (int i = 0; i < NQ; ++i) out[i] = St::encode_sr(fo[i], rnd[i]);
    } else {
#pragma unroll
      for (int i = 0; i < NQ; ++i) out[i] = St::encode(fo[i]);
    }
    if (off32) {
      const unsigned boff = (unsigned)base * (unsigned)sizeof(S);
#pragma unroll
      for (int i = 0; i < NQ; ++i) *at_bytes(dst + (long long)i * a.plane, boff) = out[i];
    } else {
#pragma unroll
      for (int i = 0; i < NQ; ++i) dst[(long long)i * a.plane + base] = out[i];
    }
  };
  if constexpr (sizeof(T) == 8) {
    // FP64: one pass at a time (two passes' populations in flight cost more registers than
    // the overlap gains)
    for (int rr = 0; rr < a.rows; ++rr) {
      const int y = ybase + rr * th;
      if (!live(y)) continue;
      T f[NQ];
      load(rr, y, f);
      update(y, f);
    }
  } else {
    // passes in pairs: both passes' loads are in flight before either is updated
    for (int rr = 0; rr < a.rows; rr += 2) {
      const int ya = ybase + rr * th, yb = ya + th;
      const bool l0 = live(ya), l1 = rr + 1 < a.rows && live(yb);
      T f0[NQ], f1[NQ];
      if (l0) load(rr, ya, f0);
      if (l1) load(rr + 1, yb, f1);
      if (l0) update(ya, f0);
      if (l1) update(yb, f1);
    }
  }
  if constexpr (St::stochastic) {
    if (tile == 0 && tid == 0) a.seed[a.seed_slot ^ 1] = seed + 1u;
  }
}

// Covered cells of disk p's box, a.dparts BLOCK-thread workgroups per disk (item = dparts p +
// part; each takes a contiguous part of the disk's cell enumeration): IMB collision of the
// cells p owns, p's force and torque over the part's cells that p covers, written to
// a.force[item].  W: only the cells in the window, so the shares are the window's (zero when the
// disk's box misses the window).
template <class St, bool W = false>
__device__ void disk_cells(const LatticeArgs& a, int item) {
  const int p = item / a.dparts, part = item - p * a.dparts;
  using T = typename St::T;
  using S = typename St::S;
  __shared__ PEntry<T> s_de[NBMAX + 1];  // disk p and its neighbours, ascending id
  __shared__ int s_cj[MAXC][BLOCK];       // covering entries of each thread's current cell
  __shared__ T s_ce[MAXC][BLOCK];         //   and their solid ratios
  __shared__ Acc<T> s_fr[WAVES][3];
  __shared__ int s_rx0[64], s_rpre[65];   // row-wise cell enumeration (rows of the box <= 64)
  __shared__ unsigned long long s_rmask[64];  // per row: the entries that can reach it
  __shared__ T s_off[64];                 // sub-cell offsets when eps_sub > 0 (eps_sub <= 64)

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const S* src = (const S*)a.src;
  S* dst = (S*)a.dst;
  const int y0 = W ? a.y0 : 0;
  // a cell row (after the periodic wrap) that the stored planes hold
  auto in_window = [&](int y) { return !W || (y >= y0 && y < y0 + a.nyl); };
  const double4 pp = a.tab.pos[p];
  if constexpr (W) {
    // rows the disk can cover against the window, with its periodic images in y
    int r0 = (int)floor(pp.y - pp.z - 0.5), r1 = (int)ceil(pp.y + pp.z + 0.5);
    bool touch = false;
    if (a.walls) {
      touch = r1 >= y0 && r0 < y0 + a.nyl;
    } else {
      for (int sh = -1; sh <= 1; ++sh) {
        const int lo = y0 + sh * a.ny;
        touch = touch || (r1 >= lo && r0 < lo + a.nyl);
      }
    }
    if (!touch) {  // block-uniform
      if (tid == 0) a.force[item] = make_double4(0.0, 0.0, 0.0, 0.0);
      return;
    }
  }
  int nn = a.nnbr[p];
  if (nn > NBMAX) nn = NBMAX;
  // the sub-cell offsets of the paper's estimate, read by the cell loop after the barriers below
  if (tid < a.eps_sub) s_off[tid] = subcell_offset<T>(tid, a.eps_sub);
  const T* off = a.eps_sub > 0 ? s_off : nullptr;
  if (nn < 0) nn = 0;
  const int nd = nn + 1;
  // Entry k: p itself or neighbour k - 1, placed at its rank by id (wave 0, one lane each; the
  // neighbour list is ascending, and p's rank is the count of smaller neighbour ids)
  if (wave == 0) {
    const int q = lane == 0 ? p : (lane < nd ? a.nbr[(long long)p * NBMAX + lane - 1] : -1);
    const int nlow = (int)__popcll(__ballot(lane > 0 && lane < nd && q < p));
    if (lane < nd) {
      const int rank = lane == 0 ? nlow : (lane - 1) + (q > p ? 1 : 0);
      const double4 ps = a.tab.pos[q];
      const double4 vl = a.tab.vel[q];
      const double flx = floor(ps.x), fly = floor(ps.y);
      PEntry<T> e;
      e.ix = (int)flx;
      e.iy = (int)fly;
      e.pid = q;
      e.slot = 0;
      e.fx = (T)(ps.x - flx);
      e.fy = (T)(ps.y - fly);
      e.r = (T)ps.z;
      e.vx = (T)vl.x;
      e.vy = (T)vl.y;
      e.om = (T)vl.z;
      if (rank >= 0 && rank < nd) s_de[rank] = e;
    }
  }
  unsigned seed = 0u;
  if constexpr (St::stochastic) seed = a.seed[a.seed_slot];

  // the cells the disk can cover: [floor(X - r - 1/2), ceil(X + r + 1/2)] in x and y
  const int ix0 = (int)floor(pp.x - pp.z - 0.5), ix1 = (int)ceil(pp.x + pp.z + 0.5);
  int iy0 = (int)floor(pp.y - pp.z - 0.5), iy1 = (int)ceil(pp.y + pp.z + 0.5);
  if (a.walls) {
    if (iy0 < 0) iy0 = 0;
    if (iy1 > a.ny - 1) iy1 = a.ny - 1;
  }
  const int bw = ix1 - ix0 + 1, bh = iy1 - iy0 + 1;
  const bool boxed = bw > 0 && bh > 0 && bw <= a.nx && bh <= a.ny;
  // Row by row, only the cells whose nearest point to the centre can lie within r: in the row at
  // y-distance ny from the centre (to the row's nearest edge) those with |x - X| < s + 1/2,
  // s = sqrt(r^2 - ny^2), widened by 1e-3 so that no rounding of the exact test drops a cell.
  // Rows start at s_rx0[k]; s_rpre holds the prefix counts (wave 1, one lane per row, while
  // wave 0 fills the entries).  Boxes taller than a wavefront walk the whole box.
  const bool rowwise = boxed && bh <= 64;
  int ncell = boxed ? bw * bh : 0;
  if (rowwise && wave == 1) {
    int x0 = 0, len = 0;
    int ywin = iy0 + lane;  // the row's lattice row
    if (!a.walls) ywin = ywin < 0 ? ywin + a.ny : (ywin >= a.ny ? ywin - a.ny : ywin);
    if (lane < bh && in_window(ywin)) {
      const double dy = (double)(iy0 + lane) - pp.y;
      const double ny = dy - 0.5 > 0.0 ? dy - 0.5 : (dy + 0.5 < 0.0 ? dy + 0.5 : 0.0);
      const double q = pp.z * pp.z - ny * ny;
      if (q > 0.0) {
        const double sw = sqrt(q) + 1e-3;
        int lo = (int)floor(pp.x - sw - 0.5) + 1, hi = (int)ceil(pp.x + sw + 0.5) - 1;
        lo = lo > ix0 ? lo : ix0;
        hi = hi < ix1 ? hi : ix1;
        if (hi >= lo) {
          x0 = lo;
          len = hi - lo + 1;
        }
      }
    }
    int incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane < bh) {
      s_rx0[lane] = x0;
      s_rpre[lane + 1] = incl;
    }
    if (lane == 0) s_rpre[0] = 0;
  }
  __syncthreads();
  if (rowwise) {
    // Per row, the entries whose disk reaches it: the row's cells lie within 1/2 of its centre
    // line in y, so a disk more than r + 1/2 (+ 1e-3 against rounding) away from that line in y
    // covers none of them; the covering test below runs on the others only, in id order.
    if (wave == 0 && lane < bh) {
      unsigned long long m = 0ull;
      const int yr = iy0 + lane;
      for (int k = 0; k < nd; ++k) {
        const PEntry<T>& e = s_de[k];
        int dj = yr - e.iy;
        if (!a.walls) {
          const int hy = a.ny / 2;
          if (dj > hy) dj -= a.ny;
          else if (dj < -hy) dj += a.ny;
        }
        const double dyc = (double)dj - (double)e.fy;
        if (fabs(dyc) <= (double)e.r + 0.501) m |= 1ull << k;
      }
      s_rmask[lane] = m;
    }
    __syncthreads();
    ncell = s_rpre[bh];
  }

  const T tau0 = (T)a.tau0, csm = (T)a.cs, gx = (T)a.gx, gy = (T)a.gy, rho0 = (T)a.rho0;
  Acc<T> afx{T(0), T(0)}, afy{T(0), T(0)}, atz{T(0), T(0)};
  // this workgroup's part of the enumeration
  const int cpart = a.dparts > 1 ? (ncell + 1) / 2 : ncell;
  const int cbeg = part * cpart, cend = cbeg + cpart < ncell ? cbeg + cpart : ncell;
  for (int c = cbeg + tid; c < cend; c += BLOCK) {
    int x, y;
    unsigned long long cand = nd >= 64 ? ~0ull : (1ull << nd) - 1ull;  // entries to test
    if (rowwise) {  // the row holding cell c: s_rpre[k] <= c < s_rpre[k + 1]
      int lo = 0, hi = bh;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_rpre[mid] <= c) lo = mid;
        else hi = mid;
      }
      x = s_rx0[lo] + (c - s_rpre[lo]);
      y = iy0 + lo;
      cand = s_rmask[lo];
    } else {
      x = ix0 + c % bw;
      y = iy0 + c / bw;
    }
    x = x < 0 ? x + a.nx : (x >= a.nx ? x - a.nx : x);
    if (!a.walls) y = y < 0 ? y + a.ny : (y >= a.ny ? y - a.ny : y);
    if (!in_window(y)) continue;
    // covering disks of the cell, ascending id; the cell belongs to the first of them.  The
    // solid ratio of p itself (every cell here but a rare few) is evaluated once, after the
    // loop, so that a wavefront runs the cut-cell area once however p ranks among its lanes'
    // candidates; other covering disks (cells shared by two disks) get theirs in the loop.
    int nc = 0, own = -1;
    bool owner = true;
    T pdx = T(0), pdy = T(0);
    for (; cand; cand &= cand - 1ull) {
      const int k = (int)__builtin_ctzll(cand);
      T dx, dy;
      lever_arm(a, s_de[k], x, y, &dx, &dy);
      if (!covers_cell<T>(s_de[k].r, dx, dy)) continue;
      const bool self = s_de[k].pid == p;
      if (!self && own < 0) owner = false;  // a lower id covers the cell
      if (nc >= MAXC) {
        atomicOr(a.err, ERR_CELL);
        continue;
      }
      s_cj[nc][tid] = k;
      if (self) {
        own = nc;
        pdx = dx;
        pdy = dy;
      } else {
        s_ce[nc][tid] = cell_solid_ratio<T>(s_de[k].r, dx, dy, a.eps_sub, off);
      }
      ++nc;
    }
    if (own < 0) continue;  // p does not cover this cell
    s_ce[own][tid] = cell_solid_ratio<T>((T)pp.z, pdx, pdy, a.eps_sub, off);
    T f[NQ], fo[NQ];
    pull_load<St, W>(a, src, x, y, f);
    auto disk = [&](int k) {
      Disk<T> d;
      const PEntry<T>& e = s_de[s_cj[k][tid]];
      d.eps = s_ce[k][tid];
      lever_arm(a, e, x, y, &d.dx, &d.dy);
      d.vx = e.vx;
      d.vy = e.vy;
      d.om = e.om;
      return d;
    };
    auto emit = [&](int k, T fx, T fy, T tz) {
      if (k != own) return;
      afx.add(fx);
      afy.add(fy);
      atz.add(tz);
    };
    T rho;
    if constexpr (St::deviation) {
      rho = collide_dev(f, nc, disk, emit, rho0, tau0, csm, gx, gy, fo);
    } else {
      rho = collide_plain(f, nc, disk, emit, tau0, csm, gx, gy, fo);
    }
    if (!owner) continue;
    if (!(rho > T(0)) || !isfinite(rho)) atomicOr(a.err, ERR_RHO);
    wall_adjust<T>(a, y, fo);
    const long long off = (long long)(y - (W ? a.yoff : 0)) * a.pitch + x;
    S out[NQ];
    if constexpr (St::stochastic) {
      unsigned rnd[NQ];
      sr_words(seed, (unsigned)((long long)y * a.pitch + x), rnd);
#pragma unroll
      for (int i = 0; i < NQ; ++i) out[i] = St::encode_sr(fo[i], rnd[i]);
    } else {
#pragma unroll
      for (int i = 0; i < NQ; ++i) out[i] = St::encode(fo[i]);
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) dst[(long long)i * a.plane + off] = out[i];
  }
  // the disk's force and torque: wave sums, then the waves in a fixed order
  const Acc<T> w0 = wave_sum(afx), w1 = wave_sum(afy), w2 = wave_sum(atz);
  if (lane == 0) {
    s_fr[wave][0] = w0;
    s_fr[wave][1] = w1;
    s_fr[wave][2] = w2;
  }
  __syncthreads();
  if (tid == 0) {
    double out[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Acc<T> v = s_fr[0][c];
#pragma unroll
      for (int w = 1; w < WAVES; ++w) v.add(s_fr[w][c]);
      out[c] = (double)v.hi + (double)v.lo;
    }
    a.force[item] = make_double4(out[0], out[1], out[2], 0.0);
  }
}

}  // namespace imb
