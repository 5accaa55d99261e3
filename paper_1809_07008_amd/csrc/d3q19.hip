// d3q19.hip -- the three-dimensional lattice step with immersed spheres (D3Q19, Table 1 of the
// paper; Sec. 2.2 and Eqs. 12-16) and its C-ABI (imb3_* in include/imb.h).
//
// One step is three kernels on the simulation's stream:
//   k_plain3    one 256-thread workgroup per tile (tw x th cells of one z layer): a tile that no
//               sphere's box touches is streamed (pull: periodic x and z, half-way bounce-back
//               walls in y or periodic y) and collided (BGK with the body force); any other tile
//               is appended to the step's list of sphere tiles;
//   k_step3     one workgroup per listed tile: the same streaming, the IMB collision of every
//               cell with the spheres whose boxes touch the tile (the paper's cell-decomposition
//               solid ratio), and per sphere the tile's force and torque partial (wave sums,
//               compensated in FP32), written to the sphere's slot for the tile -- no atomics on
//               the sums;
//   k_finalize3 one workgroup: every sphere's force and torque as the fixed-order sum of its
//               slots, then prescribed spheres move by their velocity; clears the tile list.
// The sphere path holds the covering spheres' solid ratios and forces per cell; in its own
// kernel its registers do not lower the occupancy of the plain tiles, nearly all of them.
// Populations are stored as structure of arrays f[19][nz][ny][pitch], two copies (A-B); the
// step pulls from the previous step's post-collision copy.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lattice3.h"
#include "tile.h"

namespace imb {

struct Lattice3Args {
  int nx, ny, nz, pitch, walls;
  int tw_log, th, tiles_x, tiles_y;
  int nsub;                // n of the n^3 sub-cell solid ratio
  long long zstride;       // pitch * ny
  long long plane;         // elements per population: pitch * ny * nz
  double tau0, gx, gy, gz, rho0;
  const void* src;
  void* dst;
  int np;
  double4* pos;            // (X, Y, Z, r)
  const double4* vel;      // (Vx, Vy, Vz, 0)
  const double4* spin;     // (wx, wy, wz, 0)
  const int* mode;         // 1 fixed, 2 prescribed
  double* part;            // [np][MAXSLOT3][NPART3] per-tile partials of the step
  double* F;               // [np][3] force on each sphere of the last step
  double* Tq;              // [np][3] torque
  int* err;
  int* sph_tiles;          // this step's tiles that a sphere's box touches (k_plain3 appends)
  int* sph_count;          // [1] their number; k_finalize3 clears it for the next step
  int sph_grid;            // workgroups of the k_step3 launch (>= any step's sphere tiles)
};

template <class T>
__device__ inline void sphere_lever(const Lattice3Args& a, const double4& p, int x, int y, int z,
                                    T* dx, T* dy, T* dz) {
  *dx = axis_d3<T>(x, p.x, a.nx, true);
  *dy = axis_d3<T>(y, p.y, a.ny, !a.walls);
  *dz = axis_d3<T>(z, p.z, a.nz, true);
}

// Source element of population i arriving at (x, y, z) by pull streaming.
__device__ inline long long pull_index3(const Lattice3Args& a, int i, int x, int y, int z) {
  int xs = x - c3(i, 0), ys = y - c3(i, 1), zs = z - c3(i, 2);
  xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
  zs = zs < 0 ? zs + a.nz : (zs >= a.nz ? zs - a.nz : zs);
  if (ys < 0 || ys >= a.ny) {
    if (a.walls)  // the link left through the wall and came back reversed
      return (long long)opp3(i) * a.plane + (long long)z * a.zstride + (long long)y * a.pitch + x;
    ys = ys < 0 ? ys + a.ny : ys - a.ny;
  }
  return (long long)i * a.plane + (long long)zs * a.zstride + (long long)ys * a.pitch + xs;
}

// Does any sphere's box hold tile (tx, ty, z)?  Every wavefront tests every sphere, so the
// answer is uniform over the workgroup without a barrier.
__device__ __forceinline__ bool tile_touched3(const Lattice3Args& a, int tx, int ty, int z) {
  const int lane = threadIdx.x & 63, tw = 1 << a.tw_log;
  bool touched = false;
  for (int p0 = 0; p0 < a.np && !touched; p0 += 64) {
    const int p = p0 + lane;
    bool hit = false;
    if (p < a.np) {
      const double4 ps = a.pos[p];
      const Box3 bx = sphere_box3(ps.x, ps.y, ps.z, ps.w, a.nx, a.ny, a.nz, a.walls, tw, a.th,
                                  a.tiles_x, a.tiles_y);
      hit = box3_slot(bx, tx, ty, z, a.tiles_x, a.tiles_y, a.nz) >= 0;
    }
    touched = __ballot(hit) != 0ull;
  }
  return touched;
}

// The cells of a tile that no sphere's box touches: pull, BGK with the body force, store.
template <class St>
__device__ __forceinline__ void plain_cells3(const Lattice3Args& a, int tx, int ty, int z) {
  using T = typename St::T;
  using S = typename St::S;
  const int tid = threadIdx.x, tw = 1 << a.tw_log;
  const int x = tx * tw + (tid & (tw - 1)), y = ty * a.th + (tid >> a.tw_log);
  if (x >= a.nx || y >= a.ny) return;
  const S* src = (const S*)a.src;
  S* dst = (S*)a.dst;
  T f[NQ3], fo[NQ3];
#pragma unroll
  for (int i = 0; i < NQ3; ++i) f[i] = St::decode(src[pull_index3(a, i, x, y, z)]);
  auto none = [&](int) { return Sph<T>{}; };
  auto drop = [&](int, T, T, T, T, T, T) {};
  T rho;
  if constexpr (St::deviation) {
    rho = collide3_dev(f, 0, none, drop, (T)a.rho0, (T)a.tau0, (T)a.gx, (T)a.gy, (T)a.gz, fo);
  } else {
    rho = collide3_plain(f, 0, none, drop, a.tau0, a.gx, a.gy, a.gz, fo);
  }
  if (!(rho > T(0)) || !isfinite(rho)) atomicOr(a.err, ERR_RHO);
  const long long base = (long long)z * a.zstride + (long long)y * a.pitch + x;
#pragma unroll
  for (int i = 0; i < NQ3; ++i) dst[(long long)i * a.plane + base] = St::encode(fo[i]);
}

// A tile that no sphere's box touches is streamed and collided; a touched one is appended to
// the step's sphere tiles instead.
template <class St>
__global__ __launch_bounds__(BLOCK) void k_plain3(Lattice3Args a) {
  const int tiles = a.tiles_x * a.tiles_y * a.nz;
  const int b = xcd_remap(blockIdx.x, tiles);
  const int tx = b % a.tiles_x, rest = b / a.tiles_x;
  const int ty = rest % a.tiles_y, z = rest / a.tiles_y;
  if (tile_touched3(a, tx, ty, z)) {
    if (threadIdx.x == 0) {
      const int k = atomicAdd(a.sph_count, 1);  // below `tiles`: each tile once per step
      if (k < tiles) a.sph_tiles[k] = b;
    }
    return;
  }
  plain_cells3<St>(a, tx, ty, z);
}

// The cells of tile b, which some sphere's box touches: the IMB collision with the covering
// spheres and each listed sphere's force and torque partial for the tile.
template <class St>
__device__ __forceinline__ void sphere_cells3(const Lattice3Args& a, int b) {
  using T = typename St::T;
  using S = typename St::S;
  __shared__ int s_cand[MAXCAND3], s_slot[MAXCAND3];
  __shared__ int s_ncand;
  __shared__ double4 s_pos[MAXCAND3], s_vel[MAXCAND3], s_spin[MAXCAND3];
  __shared__ Acc<T> s_red[WAVES][NPART3];
  __shared__ T s_off[64];  // sub-cell offsets (a.nsub <= 64)

  subcell_offsets<T>(s_off, a.nsub, (int)threadIdx.x);  // complete at the first barrier below
  const int tx = b % a.tiles_x, rest = b / a.tiles_x;
  const int ty = rest % a.tiles_y, z = rest / a.tiles_y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tw = 1 << a.tw_log;
  const int x = tx * tw + (tid & (tw - 1)), y = ty * a.th + (tid >> a.tw_log);
  const S* src = (const S*)a.src;
  S* dst = (S*)a.dst;

  // spheres whose box holds this tile, ascending id (wavefront 0, ballot compaction), with
  // their position, velocity and spin (loaded together, kept for the listed ones)
  if (wave == 0) {
    int base = 0;
    for (int p0 = 0; p0 < a.np; p0 += 64) {
      const int p = p0 + lane;
      int slot = -1;
      double4 ps{}, vl{}, sp{};
      if (p < a.np) {
        ps = a.pos[p];
        vl = a.vel[p];
        sp = a.spin[p];
        const Box3 bx = sphere_box3(ps.x, ps.y, ps.z, ps.w, a.nx, a.ny, a.nz, a.walls, tw, a.th,
                                    a.tiles_x, a.tiles_y);
        slot = box3_slot(bx, tx, ty, z, a.tiles_x, a.tiles_y, a.nz);
      }
      const unsigned long long m = __ballot(slot >= 0);
      const int q = base + __popcll(m & ((1ull << lane) - 1ull));
      if (slot >= 0) {
        if (q < MAXCAND3) {
          s_cand[q] = p;
          s_slot[q] = slot;
          s_pos[q] = ps;
          s_vel[q] = vl;
          s_spin[q] = sp;
        } else {
          atomicOr(a.err, ERR_TILE_LIST);
        }
      }
      base += __popcll(m);
    }
    if (lane == 0) s_ncand = base < MAXCAND3 ? base : MAXCAND3;
  }
  __syncthreads();
  const int ncand = s_ncand;

  const bool live = x < a.nx && y < a.ny;
  // covering spheres of this cell: candidate index and solid ratio (ascending id)
  int cc[MAXC3];
  T ce[MAXC3];
  int nc = 0;
  T fc[MAXC3][NPART3];
#pragma unroll
  for (int k = 0; k < MAXC3; ++k) {
    cc[k] = -1;
    ce[k] = T(0);
#pragma unroll
    for (int c = 0; c < NPART3; ++c) fc[k][c] = T(0);
  }
  if (live) {
    for (int j = 0; j < ncand; ++j) {
      T dx, dy, dz;
      sphere_lever<T>(a, s_pos[j], x, y, z, &dx, &dy, &dz);
      const T e = sphere_ratio<T>((T)s_pos[j].w, dx, dy, dz, a.nsub, s_off);
      if (e > T(0)) {
        if (nc < MAXC3) {
#pragma unroll
          for (int k = 0; k < MAXC3; ++k)
            if (k == nc) {
              cc[k] = j;
              ce[k] = e;
            }
          ++nc;
        } else {
          atomicOr(a.err, ERR_CELL);
        }
      }
    }
    T f[NQ3], fo[NQ3];
#pragma unroll
    for (int i = 0; i < NQ3; ++i) f[i] = St::decode(src[pull_index3(a, i, x, y, z)]);
    auto sph = [&](int k) {
      Sph<T> s;
      int j = 0;
      T e = T(0);
#pragma unroll
      for (int q = 0; q < MAXC3; ++q)
        if (q == k) {
          j = cc[q];
          e = ce[q];
        }
      s.eps = e;
      sphere_lever<T>(a, s_pos[j], x, y, z, &s.dx, &s.dy, &s.dz);
      s.vx = (T)s_vel[j].x; s.vy = (T)s_vel[j].y; s.vz = (T)s_vel[j].z;
      s.wx = (T)s_spin[j].x; s.wy = (T)s_spin[j].y; s.wz = (T)s_spin[j].z;
      return s;
    };
    auto emit = [&](int k, T Fx, T Fy, T Fz, T Tx, T Ty, T Tz) {
#pragma unroll
      for (int q = 0; q < MAXC3; ++q)
        if (q == k) {
          fc[q][0] = Fx; fc[q][1] = Fy; fc[q][2] = Fz;
          fc[q][3] = Tx; fc[q][4] = Ty; fc[q][5] = Tz;
        }
    };
    T rho;
    if constexpr (St::deviation) {
      rho = collide3_dev(f, nc, sph, emit, (T)a.rho0, (T)a.tau0, (T)a.gx, (T)a.gy, (T)a.gz, fo);
    } else {
      rho = collide3_plain(f, nc, sph, emit, a.tau0, a.gx, a.gy, a.gz, fo);
    }
    if (!(rho > T(0)) || !isfinite(rho)) atomicOr(a.err, ERR_RHO);
    const long long base = (long long)z * a.zstride + (long long)y * a.pitch + x;
#pragma unroll
    for (int i = 0; i < NQ3; ++i) dst[(long long)i * a.plane + base] = St::encode(fo[i]);
  }

  // per candidate sphere: the tile's force and torque partial, wave sums then the waves in a
  // fixed order, into the sphere's slot for this tile
  for (int j = 0; j < ncand; ++j) {
    Acc<T> v[NPART3];
#pragma unroll
    for (int c = 0; c < NPART3; ++c) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < MAXC3; ++k) s += cc[k] == j ? fc[k][c] : T(0);
      v[c] = wave_sum(Acc<T>{s, T(0)});
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < NPART3; ++c) s_red[wave][c] = v[c];
    }
    __syncthreads();
    if (tid < NPART3) {
      Acc<T> t = s_red[0][tid];
#pragma unroll
      for (int w = 1; w < WAVES; ++w) t.add(s_red[w][tid]);
      a.part[((long long)s_cand[j] * MAXSLOT3 + s_slot[j]) * NPART3 + tid] =
          (double)t.hi + (double)t.lo;
    }
    __syncthreads();
  }
}

// One tile of the step's sphere tiles (workgroup k takes entry k of the list; the launch has
// sph_grid workgroups, at least as many as any step lists).
template <class St>
__global__ __launch_bounds__(BLOCK) void k_step3(Lattice3Args a) {
  if ((int)blockIdx.x >= *a.sph_count) return;
  sphere_cells3<St>(a, a.sph_tiles[blockIdx.x]);
}


// Every sphere's force and torque (the sum of its slots in slot order per lane, then a fixed
// butterfly across the wavefront), then the prescribed spheres move by their velocity.
__global__ __launch_bounds__(BLOCK) void k_finalize3(Lattice3Args a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tw = 1 << a.tw_log;
  // this thread's first sphere's mode, position and velocity and the list's count, loaded beside
  // the sums' loads (nothing writes them before the barrier below)
  const int p0 = threadIdx.x;
  int mode0 = IMB_MODE_FIXED;
  double4 ps0 = make_double4(0.0, 0.0, 0.0, 0.0), v0 = ps0;
  if (p0 < a.np) {
    mode0 = a.mode[p0];
    ps0 = a.pos[p0];
    v0 = a.vel[p0];
  }
  const int count0 = threadIdx.x == 0 ? *a.sph_count : 0;
  for (int p = wave; p < a.np; p += WAVES) {
    const double4 ps = a.pos[p];
    const Box3 bx = sphere_box3(ps.x, ps.y, ps.z, ps.w, a.nx, a.ny, a.nz, a.walls, tw, a.th,
                                a.tiles_x, a.tiles_y);
    int ns = bx.ntx * bx.nty * bx.nzz;
    if (ns > MAXSLOT3) ns = MAXSLOT3;
    double acc[NPART3] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = lane; s < ns; s += 64)
#pragma unroll
      for (int c = 0; c < NPART3; ++c) acc[c] += a.part[((long long)p * MAXSLOT3 + s) * NPART3 + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < NPART3; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    if (lane == 0) {
      for (int c = 0; c < 3; ++c) {
        a.F[3 * p + c] = acc[c];
        a.Tq[3 * p + c] = acc[3 + c];
      }
    }
  }
  __syncthreads();  // every box of this step is read before a sphere moves
  for (int p = threadIdx.x; p < a.np; p += blockDim.x) {
    const bool first = p == p0;
    if ((first ? mode0 : a.mode[p]) != IMB_MODE_PRESCRIBED) continue;
    double4 ps = first ? ps0 : a.pos[p];
    const double4 v = first ? v0 : a.vel[p];
    double nxp = ps.x + v.x, nyp = ps.y + v.y, nzp = ps.z + v.z;
    nxp = nxp >= a.nx ? nxp - a.nx : (nxp < 0.0 ? nxp + a.nx : nxp);
    nzp = nzp >= a.nz ? nzp - a.nz : (nzp < 0.0 ? nzp + a.nz : nzp);
    if (a.walls) {
      if (!(nyp > -0.5 && nyp < a.ny - 0.5)) atomicOr(a.err, ERR_LEFT);
    } else {
      nyp = nyp >= a.ny ? nyp - a.ny : (nyp < 0.0 ? nyp + a.ny : nyp);
    }
    ps.x = nxp;
    ps.y = nyp;
    ps.z = nzp;
    a.pos[p] = ps;
  }
  if (threadIdx.x == 0) {  // the sphere tiles of this step are done: clear the list
    if (count0 > a.sph_grid) atomicOr(a.err, ERR_TILE_LIST);
    *a.sph_count = 0;
  }
}

// Host FP64 [19][nz][ny][nx] post-stream populations (or the equilibrium of (rho, ux(y), uy, uz)
// when fq is null) into the stored representation: post-stream f_i(x) = s_i(x - c_i), or
// s_{opp i}(x) beyond a wall.
struct Init3 {
  double rho, uy, uz;
  const double* ux_of_y;  // [ny] device, or null: ux0
  double ux0;
};

template <class St>
__global__ void k_unstream3(Lattice3Args a, const double* fq, Init3 in, typename St::S* dst) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.nx || y >= a.ny || z >= a.nz) return;
  const long long cell = ((long long)z * a.ny + y) * a.nx + x;
  const long long ncell = (long long)a.nx * a.ny * a.nz;
  double feq[NQ3];
  if (!fq) {
    const double ux = in.ux_of_y ? in.ux_of_y[y] : in.ux0;
    equilibrium3_plain(in.rho, ux, in.uy, in.uz, feq);
  }
  for (int i = 0; i < NQ3; ++i) {
    const double f = fq ? fq[(long long)i * ncell + cell] : feq[i];
    int xs = x - c3(i, 0), ys = y - c3(i, 1), zs = z - c3(i, 2);
    xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
    zs = zs < 0 ? zs + a.nz : (zs >= a.nz ? zs - a.nz : zs);
    int q = i;
    if (ys < 0 || ys >= a.ny) {
      if (a.walls) {
        q = opp3(i);
        xs = x;
        ys = y;
        zs = z;
      } else {
        ys = ys < 0 ? ys + a.ny : ys - a.ny;
      }
    }
    const long long idx = (long long)q * a.plane + (long long)zs * a.zstride +
                          (long long)ys * a.pitch + xs;
    using T = typename St::T;
    if constexpr (St::deviation) dst[idx] = St::encode((T)(f - w3(q) * a.rho0));
    else dst[idx] = St::encode((T)f);
  }
}

template <class St>
__global__ void k_gather3(Lattice3Args a, const typename St::S* src, double* fq, double* rho,
                          double* ux, double* uy, double* uz) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.nx || y >= a.ny || z >= a.nz) return;
  const long long cell = ((long long)z * a.ny + y) * a.nx + x;
  const long long ncell = (long long)a.nx * a.ny * a.nz;
  double f[NQ3];
  for (int i = 0; i < NQ3; ++i) {
    const long long idx = pull_index3(a, i, x, y, z);
    const int q = (int)(idx / a.plane);
    const double v = (double)St::decode(src[idx]);
    f[i] = St::deviation ? v + w3(q) * a.rho0 : v;
  }
  if (fq)
    for (int i = 0; i < NQ3; ++i) fq[(long long)i * ncell + cell] = f[i];
  double r = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
  for (int i = 0; i < NQ3; ++i) r += f[i];
  for (int i = 0; i < NQ3; ++i) {
    mx += (double)c3(i, 0) * f[i];
    my += (double)c3(i, 1) * f[i];
    mz += (double)c3(i, 2) * f[i];
  }
  if (rho) rho[cell] = r;
  if (ux) ux[cell] = mx / r;
  if (uy) uy[cell] = my / r;
  if (uz) uz[cell] = mz / r;
}

// eps_tot of every cell for the current sphere positions (diagnostic), in the storage's
// arithmetic precision.
template <class T>
__global__ void k_solid3(Lattice3Args a, double* eps) {
  __shared__ T s_off[64];  // sub-cell offsets (a.nsub <= 64 <= blockDim.x)
  subcell_offsets<T>(s_off, a.nsub, (int)threadIdx.x);
  __syncthreads();
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= a.nx || y >= a.ny || z >= a.nz) return;
  double s = 0.0;
  for (int p = 0; p < a.np; ++p) {
    T dx, dy, dz;
    sphere_lever<T>(a, a.pos[p], x, y, z, &dx, &dy, &dz);
    s += (double)sphere_ratio<T>((T)a.pos[p].w, dx, dy, dz, a.nsub, s_off);
  }
  eps[((long long)z * a.ny + y) * a.nx + x] = s;
}

__global__ void k_zero3(double* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace imb

// ======================================================================= host runtime
using namespace imb;

struct imb3_sim {
  imb3_config cfg;
  hipStream_t stream = nullptr;
  char* mem = nullptr;
  bool owns = false;
  size_t mem_bytes = 0;
  int tw = 64, tw_log = 6, th = 4, tiles_x = 0, tiles_y = 0, pitch = 0;
  long long plane = 0;
  void* f[2] = {nullptr, nullptr};
  double4 *pos = nullptr, *vel = nullptr, *spin = nullptr;
  int* mode = nullptr;
  double *F = nullptr, *Tq = nullptr, *part = nullptr;
  int* err = nullptr;
  int* sph_tiles = nullptr;  // the step's sphere tiles and their number (k_plain3 -> k_step3)
  int* sph_count = nullptr;
  int sph_grid = 0;          // k_step3 workgroups: bounds the sphere tiles of any step
  double* stage = nullptr;  // readback staging (library-owned)
  size_t stage_bytes = 0;
  int cur = 0, np = 0;
  int64_t steps = 0;
  std::string msg;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // 32-step chains from buffer 0 / 1
  bool use_graphs = true;
  bool timing = false;
  std::vector<hipEvent_t> ev[2];  // lattice kernel, finalize: start/stop pairs
  double k_ms[2] = {0.0, 0.0};
  int64_t k_n[2] = {0, 0};
};

namespace {

constexpr int GRAPH3 = 32;
thread_local std::string g_create3_error;

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

size_t storage3_bytes(int storage) { return storage == IMB_STORAGE_F64 ? 8 : 4; }

struct Geo3 {
  int tw, tw_log, th, tiles_x, tiles_y, pitch;
  long long plane;
};

Geo3 geometry3(const imb3_config& c) {
  Geo3 g;
  int tw = c.tile_w;
  if (tw == 0) {  // the width of 16, 32, 64 with the fewest padded cells (ties: wider)
    long long best = -1;
    for (int cand : {64, 32, 16}) {
      const long long thc = 256 / cand;
      const long long cells = (long long)((c.nx + cand - 1) / cand) * cand *
                              ((c.ny + thc - 1) / thc) * thc;
      if (best < 0 || cells < best) {
        best = cells;
        tw = cand;
      }
    }
  }
  g.tw = tw;
  g.tw_log = 0;
  while ((1 << g.tw_log) < tw) ++g.tw_log;
  g.th = 256 / tw;
  g.tiles_x = (c.nx + tw - 1) / tw;
  g.tiles_y = (c.ny + g.th - 1) / g.th;
  g.pitch = (int)((c.nx + 63) / 64 * 64);
  g.plane = (long long)g.pitch * c.ny * c.nz;
  return g;
}

// Device memory of a simulation carved from one buffer: offsets when base is null.
size_t layout3(const imb3_config& c, char* base, imb3_sim* s) {
  const Geo3 g = geometry3(c);
  const size_t es = storage3_bytes(c.storage);
  const size_t mp = (size_t)std::max(c.max_spheres, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = al256(off);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  char* f0 = take(NQ3 * (size_t)g.plane * es);
  char* f1 = take(NQ3 * (size_t)g.plane * es);
  char* pos = take(mp * sizeof(double4));
  char* vel = take(mp * sizeof(double4));
  char* spin = take(mp * sizeof(double4));
  char* mode = take(mp * sizeof(int));
  char* F = take(mp * 3 * sizeof(double));
  char* Tq = take(mp * 3 * sizeof(double));
  char* part = take(mp * MAXSLOT3 * NPART3 * sizeof(double));
  char* err = take(sizeof(int));
  char* sph_tiles = take((size_t)g.tiles_x * g.tiles_y * c.nz * sizeof(int));
  char* sph_count = take(sizeof(int));
  if (s) {
    s->f[0] = f0; s->f[1] = f1;
    s->pos = (double4*)pos; s->vel = (double4*)vel; s->spin = (double4*)spin;
    s->mode = (int*)mode; s->F = (double*)F; s->Tq = (double*)Tq; s->part = (double*)part;
    s->err = (int*)err;
    s->sph_tiles = (int*)sph_tiles;
    s->sph_count = (int*)sph_count;
    s->tw = g.tw; s->tw_log = g.tw_log; s->th = g.th; s->tiles_x = g.tiles_x;
    s->tiles_y = g.tiles_y; s->pitch = g.pitch; s->plane = g.plane;
  }
  return al256(off);
}

int validate3(const imb3_config* c, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return IMB_EINVAL;
  };
  if (!c) return bad("null configuration");
  if (c->nx < 1 || c->ny < 2 || c->nz < 1) return bad("need nx >= 1, ny >= 2, nz >= 1");
  if ((long long)c->nx * c->ny * c->nz > (1ll << 31)) return bad("lattice too large");
  if (c->storage != IMB_STORAGE_F64 && c->storage != IMB_STORAGE_F32)
    return bad("storage must be F64 or F32");
  if (!(c->tau0 > 0.5) || !std::isfinite(c->tau0)) return bad("tau0 must exceed 1/2");
  if (!std::isfinite(c->gx) || !std::isfinite(c->gy) || !std::isfinite(c->gz))
    return bad("body force must be finite");
  if (!(c->rho0 > 0.0)) return bad("rho0 must be positive");
  if (c->max_spheres < 0 || c->max_spheres > MAXS3) return bad("max_spheres must be 0..256");
  if (c->eps_subcells < 1 || c->eps_subcells > 64) return bad("eps_subcells must be 1..64");
  if (c->tile_w != 0 && c->tile_w != 16 && c->tile_w != 32 && c->tile_w != 64)
    return bad("tile_w must be 0, 16, 32 or 64");
  if (c->flags & ~IMB_FLAG_WALLS) return bad("unknown flag");
  if (c->reserved != 0 || c->reserved2 != 0) return bad("reserved fields must be 0");
  return IMB_OK;
}

int fail3(imb3_sim* s, hipError_t e, const char* what) {
  s->msg = std::string(what) + ": " + hipGetErrorString(e);
  return IMB_EHIP;
}

Lattice3Args args3(imb3_sim* s, const void* src, void* dst) {
  Lattice3Args a{};
  a.nx = s->cfg.nx; a.ny = s->cfg.ny; a.nz = s->cfg.nz; a.pitch = s->pitch;
  a.walls = (s->cfg.flags & IMB_FLAG_WALLS) ? 1 : 0;
  a.tw_log = s->tw_log; a.th = s->th; a.tiles_x = s->tiles_x; a.tiles_y = s->tiles_y;
  a.nsub = s->cfg.eps_subcells;
  a.zstride = (long long)s->pitch * s->cfg.ny;
  a.plane = s->plane;
  a.tau0 = s->cfg.tau0; a.gx = s->cfg.gx; a.gy = s->cfg.gy; a.gz = s->cfg.gz;
  a.rho0 = s->cfg.rho0;
  a.src = src; a.dst = dst;
  a.np = s->np; a.pos = s->pos; a.vel = s->vel; a.spin = s->spin; a.mode = s->mode;
  a.part = s->part; a.F = s->F; a.Tq = s->Tq; a.err = s->err;
  a.sph_tiles = s->sph_tiles; a.sph_count = s->sph_count; a.sph_grid = s->sph_grid;
  return a;
}

hipEvent_t new_event() {
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

void enqueue_step3(imb3_sim* s) {
  const int c = s->cur;
  Lattice3Args a = args3(s, s->f[c], s->f[c ^ 1]);
  const dim3 grid((unsigned)(s->tiles_x * s->tiles_y * s->cfg.nz));
  const bool spheres = s->np > 0;
  // timing: e0 at the plain kernel's start, e1 at the end of the last lattice kernel
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (s->timing) {
    e0 = new_event();
    e1 = new_event();
  }
  auto go = [&](auto kernel, dim3 g, hipEvent_t start, hipEvent_t stop) {
    if (start || stop)
      hipExtLaunchKernelGGL(kernel, g, dim3(BLOCK), 0, s->stream, start, stop, 0, a);
    else
      hipLaunchKernelGGL(kernel, g, dim3(BLOCK), 0, s->stream, a);
  };
  const dim3 sgrid((unsigned)std::max(s->sph_grid, 1));
  if (s->cfg.storage == IMB_STORAGE_F64) {
    go(k_plain3<StoreF64>, grid, e0, spheres ? nullptr : e1);
    if (spheres) go(k_step3<StoreF64>, sgrid, nullptr, e1);
  } else {
    go(k_plain3<StoreF32>, grid, e0, spheres ? nullptr : e1);
    if (spheres) go(k_step3<StoreF32>, sgrid, nullptr, e1);
  }
  if (e0) {
    s->ev[0].push_back(e0);
    s->ev[0].push_back(e1);
  }
  if (spheres) {
    hipEvent_t g0 = nullptr, g1 = nullptr;
    if (s->timing) {
      g0 = new_event();
      g1 = new_event();
      hipExtLaunchKernelGGL(k_finalize3, dim3(1), dim3(BLOCK), 0, s->stream, g0, g1, 0, a);
      s->ev[1].push_back(g0);
      s->ev[1].push_back(g1);
    } else {
      hipLaunchKernelGGL(k_finalize3, dim3(1), dim3(BLOCK), 0, s->stream, a);
    }
  }
  s->cur ^= 1;
  s->steps++;
}

void drop_graphs3(imb3_sim* s) {
  for (auto& g : s->graph)
    if (g) {
      hipGraphExecDestroy(g);
      g = nullptr;
    }
}

hipGraphExec_t capture3(imb3_sim* s, int start) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
  const hipStream_t saved = s->stream;
  const int saved_cur = s->cur;
  const int64_t saved_steps = s->steps;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    s->stream = cs;
    s->cur = start;
    for (int k = 0; k < GRAPH3; ++k) enqueue_step3(s);
    s->stream = saved;
    if (hipStreamEndCapture(cs, &g) == hipSuccess && g) {
      if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) ge = nullptr;
      hipGraphDestroy(g);
    }
  }
  s->stream = saved;
  s->cur = saved_cur;
  s->steps = saved_steps;
  hipStreamDestroy(cs);
  hipGetLastError();
  return ge;
}

int check3(imb3_sim* s) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail3(s, e, "hipStreamSynchronize");
  int bits = 0;
  e = hipMemcpy(&bits, s->err, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail3(s, e, "hipMemcpy(error flags)");
  if (bits & ERR_RHO) {
    s->msg = "device reported a non-finite or non-positive density";
    return IMB_EUNSTABLE;
  }
  if (bits & ERR_LEFT) {
    s->msg = "device reported a sphere leaving the channel";
    return IMB_EDEM;
  }
  if (bits) {
    s->msg = "device reported a list overflow (more than 16 sphere boxes on one tile or more "
             "than 4 spheres covering one cell)";
    return IMB_EOVERFLOW;
  }
  return IMB_OK;
}

int launched(imb3_sim* s, const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? IMB_OK : fail3(s, e, what);
}

int stage3(imb3_sim* s, size_t bytes) {
  if (s->stage_bytes >= bytes) return IMB_OK;
  if (s->stage) hipFree(s->stage);
  s->stage = nullptr;
  s->stage_bytes = 0;
  if (hipMalloc((void**)&s->stage, bytes) != hipSuccess) {
    hipGetLastError();
    s->stage = nullptr;
    s->msg = "cannot allocate readback staging";
    return IMB_ENOMEM;
  }
  s->stage_bytes = bytes;
  return IMB_OK;
}

void zero_dev(imb3_sim* s, void* p, size_t bytes) {
  const long long n = (long long)(bytes / sizeof(double));
  if (n > 0) hipLaunchKernelGGL(k_zero3, dim3(256), dim3(256), 0, s->stream, (double*)p, n);
}

int init_state3(imb3_sim* s, const double* fq, const Init3& in) {
  Lattice3Args a = args3(s, nullptr, nullptr);
  const dim3 grid((unsigned)((s->cfg.nx + 127) / 128), (unsigned)s->cfg.ny, (unsigned)s->cfg.nz);
  if (s->cfg.storage == IMB_STORAGE_F64)
    hipLaunchKernelGGL(k_unstream3<StoreF64>, grid, dim3(128), 0, s->stream, a, fq, in,
                       (double*)s->f[s->cur]);
  else
    hipLaunchKernelGGL(k_unstream3<StoreF32>, grid, dim3(128), 0, s->stream, a, fq, in,
                       (float*)s->f[s->cur]);
  return launched(s, "unstream3");
}

}  // namespace

extern "C" {

void imb3_config_default(imb3_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->nx = 32; c->ny = 32; c->nz = 32; c->storage = IMB_STORAGE_F64; c->tau0 = 0.6;
  c->rho0 = 1.0; c->max_spheres = 8; c->eps_subcells = 5; c->flags = IMB_FLAG_WALLS;
}

int imb3_required_bytes(const imb3_config* c, size_t* bytes) {
  if (!bytes) return IMB_EINVAL;
  const int rc = validate3(c, nullptr);
  if (rc) return rc;
  *bytes = layout3(*c, nullptr, nullptr);
  return IMB_OK;
}

int imb3_create(const imb3_config* c, void* stream, void* dev_buf, size_t dev_bytes,
                imb3_sim** out) {
  if (!out) return IMB_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = validate3(c, &why);
  if (rc) {
    g_create3_error = why;
    return rc;
  }
  imb3_sim* s = new (std::nothrow) imb3_sim();
  if (!s) return IMB_ENOMEM;
  s->cfg = *c;
  s->stream = (hipStream_t)stream;
  const size_t need = layout3(*c, nullptr, nullptr);
  if (dev_buf) {
    if (dev_bytes < need || ((uintptr_t)dev_buf & 255)) {
      g_create3_error = "bound device buffer too small or not 256-byte aligned";
      delete s;
      return IMB_ENOMEM;
    }
    s->mem = (char*)dev_buf;
  } else {
    if (hipMalloc((void**)&s->mem, need) != hipSuccess) {
      hipGetLastError();
      g_create3_error = "hipMalloc failed";
      delete s;
      return IMB_ENOMEM;
    }
    s->owns = true;
  }
  s->mem_bytes = need;
  layout3(*c, s->mem, s);
  zero_dev(s, s->mem, need);
  Init3 in{c->rho0, 0.0, 0.0, nullptr, 0.0};
  rc = init_state3(s, nullptr, in);
  if (!rc) rc = check3(s);
  if (rc) {
    g_create3_error = s->msg;
    imb3_destroy(s);
    return rc;
  }
  *out = s;
  return IMB_OK;
}

void imb3_destroy(imb3_sim* s) {
  if (!s) return;
  hipStreamSynchronize(s->stream);
  drop_graphs3(s);
  for (auto& v : s->ev)
    for (auto e : v) hipEventDestroy(e);
  if (s->stage) hipFree(s->stage);
  if (s->owns && s->mem) hipFree(s->mem);
  delete s;
}

int imb3_init_equilibrium(imb3_sim* s, double rho, double ux, double uy, double uz) {
  if (!s) return IMB_EINVAL;
  if (!(rho > 0.0) || !std::isfinite(ux) || !std::isfinite(uy) || !std::isfinite(uz)) {
    s->msg = "invalid equilibrium state";
    return IMB_EINVAL;
  }
  Init3 in{rho, uy, uz, nullptr, ux};
  return init_state3(s, nullptr, in);
}

int imb3_init_shear(imb3_sim* s, double rho, const double* ux_of_y) {
  if (!s || !ux_of_y || !(rho > 0.0)) return IMB_EINVAL;
  for (int y = 0; y < s->cfg.ny; ++y)
    if (!std::isfinite(ux_of_y[y])) {
      s->msg = "non-finite velocity";
      return IMB_EINVAL;
    }
  int rc = stage3(s, sizeof(double) * s->cfg.ny);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(s->stage, ux_of_y, sizeof(double) * s->cfg.ny,
                                hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  Init3 in{rho, 0.0, 0.0, s->stage, 0.0};
  rc = init_state3(s, nullptr, in);
  if (rc) return rc;
  return check3(s);
}

int imb3_set_populations(imb3_sim* s, const double* host_f) {
  if (!s || !host_f) return IMB_EINVAL;
  const size_t n = (size_t)NQ3 * s->cfg.nx * s->cfg.ny * s->cfg.nz;
  int rc = stage3(s, n * sizeof(double));
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(s->stage, host_f, n * sizeof(double), hipMemcpyHostToDevice,
                                s->stream);
  if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  Init3 in{1.0, 0.0, 0.0, nullptr, 0.0};
  rc = init_state3(s, s->stage, in);
  if (rc) return rc;
  return check3(s);
}

static int gather3(imb3_sim* s, double* fq, double* r, double* ux, double* uy, double* uz) {
  Lattice3Args a = args3(s, nullptr, nullptr);
  const dim3 grid((unsigned)((s->cfg.nx + 127) / 128), (unsigned)s->cfg.ny, (unsigned)s->cfg.nz);
  if (s->cfg.storage == IMB_STORAGE_F64)
    hipLaunchKernelGGL(k_gather3<StoreF64>, grid, dim3(128), 0, s->stream, a,
                       (const double*)s->f[s->cur], fq, r, ux, uy, uz);
  else
    hipLaunchKernelGGL(k_gather3<StoreF32>, grid, dim3(128), 0, s->stream, a,
                       (const float*)s->f[s->cur], fq, r, ux, uy, uz);
  return launched(s, "gather3");
}

int imb3_get_populations(imb3_sim* s, double* host_f) {
  if (!s || !host_f) return IMB_EINVAL;
  const size_t n = (size_t)NQ3 * s->cfg.nx * s->cfg.ny * s->cfg.nz;
  int rc = stage3(s, n * sizeof(double));
  if (!rc) rc = gather3(s, s->stage, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(host_f, s->stage, n * sizeof(double), hipMemcpyDeviceToHost,
                                s->stream);
  if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  return check3(s);
}

int imb3_get_fields(imb3_sim* s, double* rho, double* ux, double* uy, double* uz) {
  if (!s) return IMB_EINVAL;
  const size_t n = (size_t)s->cfg.nx * s->cfg.ny * s->cfg.nz;
  int rc = stage3(s, 4 * n * sizeof(double));
  if (!rc) rc = gather3(s, nullptr, s->stage, s->stage + n, s->stage + 2 * n, s->stage + 3 * n);
  if (rc) return rc;
  double* outs[4] = {rho, ux, uy, uz};
  for (int k = 0; k < 4; ++k) {
    if (!outs[k]) continue;
    hipError_t e = hipMemcpyAsync(outs[k], s->stage + k * n, n * sizeof(double),
                                  hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  }
  return check3(s);
}

int imb3_get_solid_field(imb3_sim* s, double* host_eps) {
  if (!s || !host_eps) return IMB_EINVAL;
  const size_t n = (size_t)s->cfg.nx * s->cfg.ny * s->cfg.nz;
  int rc = stage3(s, n * sizeof(double));
  if (rc) return rc;
  Lattice3Args a = args3(s, nullptr, nullptr);
  const dim3 grid((unsigned)((s->cfg.nx + 127) / 128), (unsigned)s->cfg.ny, (unsigned)s->cfg.nz);
  if (s->cfg.storage == IMB_STORAGE_F64)
    hipLaunchKernelGGL(k_solid3<double>, grid, dim3(128), 0, s->stream, a, s->stage);
  else
    hipLaunchKernelGGL(k_solid3<float>, grid, dim3(128), 0, s->stream, a, s->stage);
  rc = launched(s, "solid3");
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(host_eps, s->stage, n * sizeof(double), hipMemcpyDeviceToHost,
                                s->stream);
  if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  return check3(s);
}

int imb3_set_spheres(imb3_sim* s, int32_t n, const double* x, const double* y, const double* z,
                     const double* r, const double* vx, const double* vy, const double* vz,
                     const double* wx, const double* wy, const double* wz, const int32_t* mode) {
  if (!s) return IMB_EINVAL;
  if (n < 0 || n > s->cfg.max_spheres) {
    s->msg = "sphere count exceeds max_spheres";
    return IMB_EINVAL;
  }
  const double* arrs[11] = {x, y, z, r, vx, vy, vz, wx, wy, wz, nullptr};
  if (n > 0) {
    for (int k = 0; k < 10; ++k)
      if (!arrs[k]) {
        s->msg = "null sphere array";
        return IMB_EINVAL;
      }
    if (!mode) return IMB_EINVAL;
  }
  const imb3_config& c = s->cfg;
  const bool walls = c.flags & IMB_FLAG_WALLS;
  std::vector<double4> hp(n), hv(n), hw(n);
  for (int p = 0; p < n; ++p) {
    bool ok = r[p] > 0.0 && 2.0 * (r[p] + 2.0) < c.nx && 2.0 * (r[p] + 2.0) < c.nz &&
              2.0 * (r[p] + 2.0) < c.ny && x[p] >= 0.0 && x[p] < c.nx && z[p] >= 0.0 &&
              z[p] < c.nz && (mode[p] == IMB_MODE_FIXED || mode[p] == IMB_MODE_PRESCRIBED);
    for (int k = 0; k < 10 && ok; ++k) ok = std::isfinite(arrs[k][p]);
    if (ok) ok = walls ? (y[p] > -0.5 && y[p] < c.ny - 0.5) : (y[p] >= 0.0 && y[p] < c.ny);
    if (ok) {
      const Box3 b = sphere_box3(x[p], y[p], z[p], r[p], c.nx, c.ny, c.nz, walls ? 1 : 0, s->tw,
                                 s->th, s->tiles_x, s->tiles_y);
      ok = (long long)b.ntx * b.nty * b.nzz <= MAXSLOT3;
    }
    if (!ok) {
      char buf[200];
      snprintf(buf, sizeof buf, "sphere %d out of range (need r > 0, 2 (r + 2) < nx, ny, nz, "
               "the centre inside the lattice, mode fixed or prescribed, at most %d tiles)", p,
               MAXSLOT3);
      s->msg = buf;
      return IMB_EINVAL;
    }
    hp[p] = make_double4(x[p], y[p], z[p], r[p]);
    hv[p] = make_double4(vx[p], vy[p], vz[p], 0.0);
    hw[p] = make_double4(wx[p], wy[p], wz[p], 0.0);
  }
  // workgroups of the sphere-tile launch: the sum over spheres of the most tiles a box of the
  // sphere's radius can span anywhere (a run of m cells spans at most m / w + 2 tiles of width w)
  long long grid = 0;
  for (int p = 0; p < n; ++p) {
    const long long m = (long long)std::floor(2.0 * r[p] + 4.0);
    grid += std::min<long long>(s->tiles_x, m / s->tw + 2) *
            std::min<long long>(s->tiles_y, m / s->th + 2) * std::min<long long>(c.nz, m);
  }
  hipStreamSynchronize(s->stream);
  drop_graphs3(s);
  s->np = n;
  s->sph_grid = (int)std::min<long long>(grid, (long long)s->tiles_x * s->tiles_y * c.nz);
  hipError_t e = hipSuccess;
  if (n > 0) {
    e = hipMemcpy(s->pos, hp.data(), n * sizeof(double4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->vel, hv.data(), n * sizeof(double4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->spin, hw.data(), n * sizeof(double4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->mode, mode, n * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return fail3(s, e, "hipMemcpy(spheres)");
  zero_dev(s, s->F, (size_t)std::max(c.max_spheres, 1) * 3 * sizeof(double));
  zero_dev(s, s->Tq, (size_t)std::max(c.max_spheres, 1) * 3 * sizeof(double));
  int zero = 0;
  e = hipMemcpyAsync(s->err, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return fail3(s, e, "reset error flags");
  return check3(s);
}

int imb3_step(imb3_sim* s, int32_t nsteps) {
  if (!s || nsteps < 0) return IMB_EINVAL;
  if (!s->use_graphs || s->timing) {
    for (int k = 0; k < nsteps; ++k) enqueue_step3(s);
    return launched(s, "step3");
  }
  while (nsteps >= GRAPH3) {
    hipGraphExec_t& ge = s->graph[s->cur];
    if (!ge) ge = capture3(s, s->cur);
    if (!ge) {
      s->use_graphs = false;
      break;
    }
    hipError_t e = hipGraphLaunch(ge, s->stream);
    if (e != hipSuccess) return fail3(s, e, "hipGraphLaunch");
    s->steps += GRAPH3;  // an even number of steps keeps the buffer parity
    nsteps -= GRAPH3;
  }
  for (int k = 0; k < nsteps; ++k) enqueue_step3(s);
  return launched(s, "step3");
}

int imb3_get_forces(imb3_sim* s, double* F, double* T) {
  if (!s) return IMB_EINVAL;
  const size_t n = (size_t)s->np * 3;
  if (n && F) {
    hipError_t e = hipMemcpyAsync(F, s->F, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  }
  if (n && T) {
    hipError_t e = hipMemcpyAsync(T, s->Tq, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  }
  return check3(s);
}

int imb3_get_spheres(imb3_sim* s, double* xyzr) {
  if (!s) return IMB_EINVAL;
  if (s->np && xyzr) {
    hipError_t e = hipMemcpyAsync(xyzr, s->pos, s->np * sizeof(double4), hipMemcpyDeviceToHost,
                                  s->stream);
    if (e != hipSuccess) return fail3(s, e, "hipMemcpyAsync");
  }
  return check3(s);
}

int imb3_sync(imb3_sim* s) { return s ? check3(s) : IMB_EINVAL; }

int imb3_set_kernel_timing(imb3_sim* s, int enable) {
  if (!s) return IMB_EINVAL;
  hipStreamSynchronize(s->stream);
  for (auto& v : s->ev) {
    for (auto e : v) hipEventDestroy(e);
    v.clear();
  }
  s->k_ms[0] = s->k_ms[1] = 0.0;
  s->k_n[0] = s->k_n[1] = 0;
  s->timing = enable != 0;
  return IMB_OK;
}

int imb3_get_kernel_timing(imb3_sim* s, double* lattice_ms, int64_t* lattice_n,
                           double* finalize_ms, int64_t* finalize_n) {
  if (!s) return IMB_EINVAL;
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail3(s, e, "hipStreamSynchronize");
  for (int k = 0; k < 2; ++k) {
    for (size_t i = 0; i + 1 < s->ev[k].size(); i += 2) {
      float t = 0.f;
      hipEventElapsedTime(&t, s->ev[k][i], s->ev[k][i + 1]);
      s->k_ms[k] += t;
      s->k_n[k] += 1;
      hipEventDestroy(s->ev[k][i]);
      hipEventDestroy(s->ev[k][i + 1]);
    }
    s->ev[k].clear();
  }
  if (lattice_ms) *lattice_ms = s->k_ms[0];
  if (lattice_n) *lattice_n = s->k_n[0];
  if (finalize_ms) *finalize_ms = s->k_ms[1];
  if (finalize_n) *finalize_n = s->k_n[1];
  return IMB_OK;
}

const char* imb3_last_error(const imb3_sim* s) { return s ? s->msg.c_str() : g_create3_error.c_str(); }

}  // extern "C"
