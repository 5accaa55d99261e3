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

// Ordered list of the disks whose tile box contains tile (tx, ty).  Returns the list length
// (capped at LMAX; overflow latches ERR_TILE_LIST).
template <class T>
__device__ int build_tile_list(const LatticeArgs& a, int tx, int ty, PEntry<T>* pl,
                               int* s_cnt) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int base = 0;
  for (int p0 = 0; p0 < a.np; p0 += BLOCK) {
    const int p = p0 + tid;
    int slot = -1;
    if (p < a.np) slot = box_slot(a.tab.box[p], tx, ty, a.tiles_x, a.tiles_y);
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
      const int k = off + below;
      if (k < LMAX) {
        const double4 ps = a.tab.pos[p];
        const double4 vl = a.tab.vel[p];
        const double flx = floor(ps.x), fly = floor(ps.y);
        PEntry<T> e;
        e.ix = (int)flx;
        e.iy = (int)fly;
        e.pid = p;
        e.slot = slot;
        e.fx = (T)(ps.x - flx);
        e.fy = (T)(ps.y - fly);
        e.r = (T)ps.z;
        e.vx = (T)vl.x;
        e.vy = (T)vl.y;
        e.om = (T)vl.z;
        pl[k] = e;
      } else {
        atomicOr(a.err, ERR_TILE_LIST);
      }
    }
    base += total;
    __syncthreads();
  }
  return base < LMAX ? base : LMAX;
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

// Disks covering cell (x, y): eps > 0 with the image nearest to the cell.  Returns their count.
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

template <class T>
__device__ inline Acc<T> wave_sum(Acc<T> v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Acc<T> o;
    o.hi = __shfl_xor(v.hi, off, 64);
    o.lo = __shfl_xor(v.lo, off, 64);
    v.add(o);
  }
  return v;
}

template <class St>
__global__ __launch_bounds__(BLOCK) void k_lattice_step(LatticeArgs a) {
  using T = typename St::T;
  using S = typename St::S;
  __shared__ PEntry<T> s_pl[LMAX];
  __shared__ int s_cnt[WAVES];
  __shared__ unsigned s_touch;
  __shared__ Acc<T> s_red[WAVES][3];
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
  const int n = build_tile_list<T>(a, tx, ty, s_pl, s_cnt);
  if (n > 0) {
#pragma unroll
    for (int q = 0; q < MAXC; ++q) cs.aj[q][tid] = -1;
  }

  const T tau0 = (T)a.tau0, csm = (T)a.cs, gx = (T)a.gx, gy = (T)a.gy, rho0 = (T)a.rho0;
  for (int rr = 0; rr < a.rows; ++rr) {
    const int y = ybase + rr * th;
    if (x >= a.nx || y >= a.ny) continue;
    T f[NQ], fo[NQ];
    pull_load<St>(a, src, x, y, f);
    const int nc = n > 0 ? covering_disks<T>(a, s_pl, n, x, y, cs) : 0;
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

  for (int j = 0; j < n; ++j) {
    if (!((touched >> j) & 1u)) {
      if (tid == 0)
        a.partials[(long long)s_pl[j].pid * MAXSLOT + s_pl[j].slot] = make_double4(0, 0, 0, 0);
      continue;
    }
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      Acc<T> v{T(0), T(0)};
#pragma unroll
      for (int q = 0; q < MAXC; ++q)
        if (cs.aj[q][tid] == j) v.add(cs.af[comp][q][tid]);
      v = wave_sum(v);
      if (lane == 0) s_red[wave][comp] = v;
    }
    __syncthreads();
    if (tid == 0) {
      double out[3];
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        Acc<T> v = s_red[0][comp];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) v.add(s_red[w][comp]);
        out[comp] = (double)v.hi + (double)v.lo;
      }
      a.partials[(long long)s_pl[j].pid * MAXSLOT + s_pl[j].slot] =
          make_double4(out[0], out[1], out[2], 0.0);
    }
    __syncthreads();
  }
}

// eps_tot of every cell (diagnostic / parity of the solid-ratio stage alone).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_solid_field(LatticeArgs a, double* eps_out) {
  __shared__ PEntry<T> s_pl[LMAX];
  __shared__ int s_cnt[WAVES];
  __shared__ CellScratch<T> cs;
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tw = 1 << a.tw_log, th = BLOCK >> a.tw_log;
  const int x = tx * tw + (tid & (tw - 1));
  const int ybase = ty * th * a.rows + (tid >> a.tw_log);
  const int n = build_tile_list<T>(a, tx, ty, s_pl, s_cnt);
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
