// lattice_tile.h -- the fused lattice step: per-cell solid ratio of the disks (Sec. 2.2), IMB
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
#pragma once

#include "collide.h"
#include "tile.h"

namespace imb {

// One tile of the fused step, executed by a whole BLOCK-thread workgroup (block-uniform control
// flow; the workgroup's LDS holds the tile's disk list and per-thread scratch).
template <class St>
__device__ void lattice_tile(const LatticeArgs& a, int tile) {
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
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tw = 1 << a.tw_log, th = BLOCK >> a.tw_log;
  const int lx = tid & (tw - 1), ly = tid >> a.tw_log;
  const int x = tx * tw + lx;
  const int ybase = ty * th * a.rows + ly;
  const S* src = (const S*)a.src;
  S* dst = (S*)a.dst;

  if (tid == 0) s_touch = 0u;
  unsigned seed = 0u;
  if constexpr (St::stochastic) seed = a.seed[a.seed_slot];
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
    if constexpr (St::stochastic) {
      const unsigned r0 = pcg_hash(seed * 0x9E3779B9u + (unsigned)base);
#pragma unroll
      for (int i = 0; i < NQ; ++i)
        St::store_sr(dst, (long long)i * a.plane + base, fo[i], pcg_hash(r0 + (unsigned)i));
    } else {
#pragma unroll
      for (int i = 0; i < NQ; ++i) St::store(dst, (long long)i * a.plane + base, fo[i], T(0));
    }
  }
  if constexpr (St::stochastic) {
    if (tile == 0 && tid == 0) a.seed[a.seed_slot ^ 1] = seed + 1u;
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

}  // namespace imb
