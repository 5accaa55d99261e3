// common.h -- internal definitions shared by the HIP kernels and the host runtime of libimb.
//
// Method: Yang, Jing, Kwok & Sobral, "A comprehensive study of coupled LBM-DEM with immersed
// moving boundary" (arXiv:1809.07008), Sec. 2 (LBM, DEM, IMB, coupling), in two dimensions (D2Q9).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "imb.h"

namespace imb {

constexpr int NQ = 9;              // D2Q9
constexpr int BLOCK = 256;         // threads of a lattice-step workgroup (4 wave64)
constexpr int WAVES = BLOCK / 64;
constexpr int LMAX = 32;           // disks whose boxes may touch one tile
constexpr int MAXC = 4;            // disks covering one cell (three cannot unless they overlap)
constexpr int MAXSLOT = 64;        // tiles per disk box (partial-sum slots per disk)
constexpr int NBMAX = 32;          // DEM neighbour-list capacity per disk
constexpr int MAX_PARTICLES = 512;
constexpr int MASK_WORDS = MAX_PARTICLES / 64;  // 64-bit words of a tile row's disk mask
// Most workgroups of the lattice step per disk (a simulation's `dparts`, 1 or 2): each takes a
// contiguous part of the disk's cells and writes its own share of the disk's force and torque,
// force[dparts p + part].  Two halve a disk's latency where few disks run beside few tiles (a
// slab); on a whole lattice the tiles hide it and one per disk is faster.
constexpr int DISK_PARTS = 2;
constexpr int PBLOCK = 512;        // threads of the particle-phase workgroup (one per disk)
constexpr int HK = 8;         // tangential springs per disk (disks touching it at once)
constexpr double DEM_SKIN = 5.0;   // neighbour-list skin (lattice units)
constexpr double MAX_MOVE = 1.0;   // largest displacement of a disk in one lattice step
constexpr float F16_SCALE = 16384.0f;  // power-of-two scale of FP16 deviations

// Device error bits, latched in one int by the kernels and mapped to IMB_E* by the host.
enum : int {
  ERR_TILE_LIST = 1,   // more than LMAX disk boxes touch a tile
  ERR_SLOTS = 2,       // a disk box spans more than MAXSLOT tiles
  ERR_CELL = 4,        // more than MAXC disks cover one cell / one thread column
  ERR_RHO = 8,         // non-finite or non-positive density
  ERR_NBR = 16,        // DEM neighbour list full
  ERR_MOVE = 32,       // a disk moved more than MAX_MOVE in one step
  ERR_LEFT = 64,       // a disk centre left the channel between the walls
  ERR_CONTACTS = 256,  // a disk touches more than HK other disks at once (tangential springs)
};

// D2Q9 velocity set (the paper's Table 1 gives the 3D D3Q19 set; its 2D analogue here).
__host__ __device__ constexpr int cx_of(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp_of(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
}
__host__ __device__ constexpr double w_of(int i) {
  return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
static_assert(opp_of(1) == 3 && opp_of(2) == 4 && opp_of(3) == 1 && opp_of(4) == 2, "opp");
static_assert(opp_of(5) == 7 && opp_of(6) == 8 && opp_of(7) == 5 && opp_of(8) == 6, "opp");

// Disk data for the lattice step, rewritten by the particle phase after every DEM update.
struct ParticleTable {
  int4* box;      // tile box: (tx0, ntx, ty0, nty); ntx * nty partial-sum slots
  double4* pos;   // (X, Y, r, 0)
  double4* vel;   // (Vx, Vy, omega, 0)
};

// Everything one lattice step of one channel needs.
struct LatticeArgs {
  int nx, ny, pitch, walls;
  int tiles_x, tiles_y;  // tile grid
  int tw_log, rows;      // tile = (1 << tw_log) x ((BLOCK >> tw_log) * rows) cells
  int eps_sub;           // 0: exact solid ratio; n > 0: fraction of n x n sub-cell centres
  // moving walls: 6 w_j rho0 (c_j . u_w) for a population j sent into a wall moving along x
  // at u_w; it comes back as opp(j) lowered by it.  Only the diagonal directions carry it:
  // [0], [1] for j = 7, 8 into the wall at y = -1/2, [2], [3] for j = 5, 6 into y = ny - 1/2
  int walls_move;
  double wall_c[4];
  float wall_cf[4];  // the same rounded to FP32 (the FP32 arithmetic forms)
  long long plane;       // elements per population plane (pitch * ny)
  double tau0, cs, gx, gy, rho0;
  const void* src;       // stored post-collision populations of the previous step
  void* dst;             // post-collision populations of this step
  int np;
  ParticleTable tab;
  // [MASK_WORDS][tiles_y]: bit l of word w of tile row ty is set when disk 64 w + l's box
  // touches the row
  const unsigned long long* band_mask;
  int pstride;           // per-disk array stride (max_particles)
  int* err;
  unsigned* seed;        // [2] step counters of the stochastic rounding: this step reads
  int seed_slot;         //   seed[seed_slot], tile 0 writes seed[seed_slot ^ 1] = it + 1
  const int* nbr;        // [np][NBMAX] neighbour lists (ascending ids) and their lengths
  const int* nnbr;
  double4* force;        // [np][dparts] shares of each disk's force and torque (Fx, Fy, Tz, 0)
  int dparts;            // workgroups (and shares) per disk, 1 or 2
  // The rows [y0, y0 + nyl) of the lattice that this step updates (a slab of a lattice split in
  // y; the whole lattice: y0 = 0, nyl = ny).  Lattice row y is stored in plane row y - yoff: a
  // slab's planes hold a ghost row on each side (yoff = y0 - 1), where its neighbours' crossing
  // populations are copied between steps (ghost_lo, ghost_hi: that neighbour exists; a wall
  // otherwise).  Tile rows count inside the window: tile row ty is lattice tile row ty + ty_off
  // of the tiles_yg that the lattice has.
  int y0, nyl, yoff, ty_off, tiles_yg;
  int ghost_lo, ghost_hi;
};

// The momentum a moving wall takes from population j sent into it (through y = -1/2 when
// `bottom`): the returning opp(j) is lowered by this.

// A population that a wall-row cell sends into a moving wall is read back only by that cell's
// own bounce-back pull, so it is stored already lowered by the wall's momentum: the pull then
// returns f*_j - 6 w_j rho0 (c_j . u_w) unchanged.  No-op unless a wall moves (uniform).
template <class T>
__device__ inline void wall_adjust(const LatticeArgs& a, int y, T fo[NQ]) {
  if (!a.walls_move) return;
  static_assert(cy_of(7) < 0 && cy_of(8) < 0 && cy_of(5) > 0 && cy_of(6) > 0, "diagonals");
  if (y == 0) {
    if constexpr (sizeof(T) == 4) {
      fo[7] = fo[7] - a.wall_cf[0];
      fo[8] = fo[8] - a.wall_cf[1];
    } else {
      fo[7] = fo[7] - a.wall_c[0];
      fo[8] = fo[8] - a.wall_c[1];
    }
  }
  if (y == a.ny - 1) {
    if constexpr (sizeof(T) == 4) {
      fo[5] = fo[5] - a.wall_cf[2];
      fo[6] = fo[6] - a.wall_cf[3];
    } else {
      fo[5] = fo[5] - a.wall_c[2];
      fo[6] = fo[6] - a.wall_c[3];
    }
  }
}

// Particle state on the device (structure of arrays, FP64).
struct ParticleState {
  double *x, *y, *r, *vx, *vy, *om;
  int* mode;
  double *fcx, *fcy;      // contact force of the last DEM evaluation
  double* tcz;            // contact torque of the last DEM evaluation
  int* hid;               // [np][HK] partners with a tangential spring, id + 1 (0: free entry)
  double* hsp;            // [np][HK] their springs (tangential displacement, from this disk)
  double* hw;             // [np][2] springs against the bottom and the top wall
  double *Fx, *Fy, *Tz;   // hydrodynamic force / torque of the last step
  double *xref, *yref;    // positions at the last neighbour-list build
  int* nbr;               // [np][NBMAX] neighbour ids, ascending
  int* nnbr;              // neighbours per disk
  int* rebuild;           // 1: rebuild the neighbour list before the next DEM phase
};

struct ParticleArgs {
  int np, nx, ny, walls, n_sub;
  double kn, zeta, rho_s;
  double kt, mu;          // tangential stiffness and friction (both 0: normal force only)
  int hertz;              // 1: Hertz-Mindlin law (kn, kt unused), 0: linear spring-dashpot
  double es_pp, es_pw;    // Hertz-Mindlin E* of a disk pair and of a disk against a wall
  double gs_pp, gs_pw;    //   and G*
  double hm_damp;         //   2 sqrt(5/6) zeta
  double uw_bot, uw_top;  // wall velocities along x (the walls' tangential slip)
  int tiles_x, tiles_y, tw, th;
  int tiles_yg, ty_off;   // the lattice's tile rows; band masks cover rows [ty_off, +tiles_y)
  ParticleState s;
  ParticleTable tab;
  const double4* direct;  // [np][dparts] shares of the step's force and torque, added in order
  int dparts;
  int build_lists;        // maintain the neighbour lists even when no disk is free
  unsigned long long* band_mask;  // written with the table: per tile row, the disks whose box
                                  // touches it ([MASK_WORDS][tiles_y], as LatticeArgs reads it)
  int lds_doubles;                // the LDS the phase's launch gives it (set by the launch)
  int do_finalize, do_dem, do_table, init_contacts;
  const double *wfx, *wfy, *wtz;  // objective weights (adjoint forward); may be null
  double* J;                      // objective accumulator; null = not accumulated
  int* err;
};

// Storage codecs: how a population is kept in memory and what precision the step computes in.
struct StoreF64 {
  using T = double;
  using S = double;
  static constexpr bool deviation = false;
  static constexpr bool stochastic = false;
  __device__ static T decode(S s) { return s; }
  __device__ static S encode(T v) { return v; }
  __device__ static T load(const S* p, long long i, T) { return p[i]; }
  __device__ static void store(S* p, long long i, T v, T) { p[i] = v; }
};
struct StoreF32 {
  using T = float;
  using S = float;
  static constexpr bool deviation = true;
  static constexpr bool stochastic = false;
  __device__ static T decode(S s) { return s; }
  __device__ static S encode(T v) { return v; }
  __device__ static T load(const S* p, long long i, T) { return p[i]; }
  __device__ static void store(S* p, long long i, T v, T) { p[i] = v; }
};
// FP16: h * 2^14 in binary16.  store() rounds to nearest even (used for set-up); store_sr()
// rounds stochastically: away from zero with probability equal to the fractional position
// between the two neighbouring binary16 values, from a counter-based random word, so the
// rounding error of the step-to-step updates has zero mean instead of the systematic bias of
// round-to-nearest on increments of about one unit in the last place.
struct StoreF16 {
  using T = float;
  using S = __half;
  static constexpr bool deviation = true;
  static constexpr bool stochastic = true;
  __device__ static T decode(S s) { return __half2float(s) * (1.0f / F16_SCALE); }
  __device__ static S encode(T v) { return __float2half_rn(v * F16_SCALE); }
  __device__ static T load(const S* p, long long i, T) { return decode(p[i]); }
  __device__ static void store(S* p, long long i, T v, T) { p[i] = encode(v); }
  // The value rounds away from zero when u < frac, u = (rnd >> 8) / 2^24 and frac the fractional
  // position of s between its neighbours toward and away from zero.
  __device__ static S encode_sr(T v, unsigned rnd) {
    const float s = v * F16_SCALE;
    const float a = fabsf(s);
    if (a >= 6.103515625e-05f && a < 65504.0f) {
      // binary16 normal range: a half ulp is 2^13 float ulps, so frac = low / 2^13 with low the
      // 13 float mantissa bits below the half mantissa, and u < frac exactly when
      // (rnd >> 19) < low, i.e. when adding (~rnd >> 19) = 8191 - (rnd >> 19) to the float's bits
      // carries into the half mantissa; the truncated value converts to binary16 exactly
      const unsigned b = (__float_as_uint(s) + (~rnd >> 19)) & ~0x1FFFu;
      return __float2half_rn(__uint_as_float(b));
    }
    if (!(a < 6.103515625e-05f)) return __float2half_rz(s);  // beyond the range (saturates)
    // subnormal binary16 values (spacing 2^-24)
    const __half lo = __float2half_rz(s);  // neighbour toward zero
    const float flo = __half2float(lo);
    if (flo == s) return lo;
    const __half hi = __ushort_as_half((unsigned short)(__half_as_ushort(lo) + 1u));  // away
    const float fhi = __half2float(hi);
    const float frac = (s - flo) / (fhi - flo);
    const float u = (float)(rnd >> 8) * (1.0f / 16777216.0f);
    return u < frac ? hi : lo;
  }
  __device__ static void store_sr(S* p, long long i, T v, unsigned rnd) { p[i] = encode_sr(v, rnd); }
};

// 32-bit integer hash "pcg_hash" (Jarzynski & Olano, Hash Functions for GPU Rendering, JCGT 9(3),
// 2020): one PCG step followed by the RXS-M-XS output permutation.
__host__ __device__ inline unsigned pcg_hash(unsigned v) {
  const unsigned state = v * 747796405u + 2891336453u;
  const unsigned word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

// The random words of one cell's stochastic-rounding stores: w0 = pcg_hash of (step counter,
// lattice cell), then four xorshift32 steps (Marsaglia, Xorshift RNGs, J. Stat. Softw. 8(14),
// 2003; shifts 13, 17, 5), so a cell costs one hash instead of one per population.  The normal
// binary16 range uses the top 13 bits of a word (encode_sr), so each word serves two
// populations: population 2k takes word k, population 2k + 1 word k shifted left by 13 (its
// bits 6..18 on top).
__device__ inline void sr_words(unsigned seed, unsigned cell, unsigned rnd[NQ]) {
  unsigned w = pcg_hash(seed * 0x9E3779B9u + cell);
#pragma unroll
  for (int k = 0; k < (NQ + 1) / 2; ++k) {
    if (k > 0) {
      w ^= w << 13;
      w ^= w >> 17;
      w ^= w << 5;
    }
    rnd[2 * k] = w;
    if (2 * k + 1 < NQ) rnd[2 * k + 1] = w << 13;
  }
}

// Block index -> tile index so that consecutive tiles run on the same XCD (workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2).
__device__ inline int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int xcd = b & 7, j = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + j;
}

__host__ __device__ inline int wrap_int(int a, int n) { int m = a % n; return m < 0 ? m + n : m; }
// wrap_int for a within one period of [0, n) without a division (the general form otherwise)
__host__ __device__ inline int wrap_near(int a, int n) {
  if (a >= 0 && a < n) return a;
  if (a < 0 && a >= -n) return a + n;
  if (a >= n && a < 2 * n) return a - n;
  return wrap_int(a, n);
}
// a / d for a >= 0; a shift when d is a power of two (tile widths and heights are)
__host__ __device__ inline int div_tile(int a, int d) {
  return (d & (d - 1)) == 0 ? a >> __builtin_ctz((unsigned)d) : a / d;
}

// Tile box of a disk: the cyclic range of tiles that contain a cell of its bounding box
// [floor(X - r - 1/2), ceil(X + r + 1/2)] (only those cells can be covered).  Returns false if
// the box needs more than MAXSLOT slots.
__host__ __device__ inline bool tile_box(double X, double Y, double r, int nx, int ny, int walls,
                                         int tiles_x, int tiles_y, int tw, int th, int4* out) {
  const int ix0 = (int)floor(X - r - 0.5), ix1 = (int)ceil(X + r + 0.5);
  int tx0, ntx;
  if (ix1 - ix0 + 1 > nx - tw) {
    tx0 = 0;
    ntx = tiles_x;
  } else {
    tx0 = div_tile(wrap_near(ix0, nx), tw);
    const int txe = div_tile(wrap_near(ix1, nx), tw);
    ntx = wrap_near(txe - tx0, tiles_x) + 1;
  }
  int iy0 = (int)floor(Y - r - 0.5), iy1 = (int)ceil(Y + r + 0.5);
  int ty0, nty;
  if (walls) {
    if (iy0 < 0) iy0 = 0;
    if (iy1 > ny - 1) iy1 = ny - 1;
    if (iy0 > iy1) {
      ty0 = 0;
      nty = 0;
    } else {
      ty0 = div_tile(iy0, th);
      nty = div_tile(iy1, th) - ty0 + 1;
    }
  } else if (iy1 - iy0 + 1 > ny - th) {
    ty0 = 0;
    nty = tiles_y;
  } else {
    ty0 = div_tile(wrap_near(iy0, ny), th);
    const int tye = div_tile(wrap_near(iy1, ny), th);
    nty = wrap_near(tye - ty0, tiles_y) + 1;
  }
  *out = make_int4(tx0, ntx, ty0, nty);
  return ntx * nty <= MAXSLOT;
}

// Slot of tile (tx, ty) in a disk's box, or -1 if the tile is outside it.  The result is always
// -1 or in [0, MAXSLOT), whatever the box holds (a box is only meaningful for the tile grid it
// was built for).
__device__ inline int box_slot(int4 b, int tx, int ty, int tiles_x, int tiles_y) {
  int lx = tx - b.x;
  if (lx < 0) lx += tiles_x;
  if (lx < 0 || lx >= b.y) return -1;
  int ly = ty - b.z;
  if (ly < 0) ly += tiles_y;
  if (ly < 0 || ly >= b.w) return -1;
  const int slot = ly * b.y + lx;
  return slot < MAXSLOT ? slot : -1;
}

// Number of partial-sum slots of a box, bounded by MAXSLOT.
__host__ __device__ inline int box_slots(int4 b) {
  const int n = b.y * b.w;
  return n < 0 ? 0 : (n > MAXSLOT ? MAXSLOT : n);
}

}  // namespace imb
