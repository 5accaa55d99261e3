// convert.hip -- moving populations between the caller's FP64 [q][y][x] post-stream format and
// the stored representation (post-collision planes of the previous step, in storage precision),
// the moments of Eqs. (3), (4), and plain streaming copy / fill kernels.
//
// The stored planes s are what the pull step reads: post-stream f_i(x) = s_i(x - c_i), or
// s_{-i}(x) when x - c_i lies beyond a wall.  This map is one-to-one, so "unstream" computes each
// s entry once, from the one population that it becomes.
#include "step.h"

namespace imb {

struct Feq9 {
  double v[NQ];
};

template <class St>
__device__ inline void encode_store(typename St::S* dst, long long idx, double f, int q,
                                    double rho0) {
  using T = typename St::T;
  if constexpr (St::deviation) St::store(dst, idx, (T)(f - w_of(q) * rho0), T(0));
  else St::store(dst, idx, (T)f, T(0));
}

template <class St>
__device__ inline double decode_load(const typename St::S* src, long long idx, int q, double rho0) {
  using T = typename St::T;
  const T v = St::load(src, idx, T(0));
  if constexpr (St::deviation) return (double)v + w_of(q) * rho0;
  else return (double)v;
}

// Stored entry i of cell (x, y) (lattice coordinates): the population that the pull of the next
// step delivers to (x + c_i), or, where that lies beyond a wall, the one that the bounce-back
// returns to (x, y) itself as population -i.  A slab also fills its ghost rows y0 - 1 and
// y0 + nyl (where it has a neighbour there) with the populations that cross into it.
template <class St>
__global__ void k_unstream(LatticeArgs a, const double* fq, Feq9 feq, typename St::S* dst) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = a.y0 - 1 + (int)blockIdx.y;  // grid rows: the window and the rows next to it
  if (x >= a.nx) return;
  const bool lo = y == a.y0 - 1, hi = y == a.y0 + a.nyl;
  if ((lo && !a.ghost_lo) || (hi && !a.ghost_hi)) return;
  int yc = y;  // the cell's lattice row (a ghost row wraps in a periodic lattice)
  if (yc < 0) yc += a.ny;
  if (yc >= a.ny) yc -= a.ny;
  for (int i = 0; i < NQ; ++i) {
    if ((lo && cy_of(i) <= 0) || (hi && cy_of(i) >= 0)) continue;  // not crossing into the slab
    int xa = x + cx_of(i), ya = yc + cy_of(i);
    int qa = i;
    if (ya < 0 || ya >= a.ny) {
      if (a.walls) {
        xa = x;
        ya = yc;
        qa = opp_of(i);
      } else {
        ya = ya < 0 ? ya + a.ny : ya - a.ny;
      }
    }
    xa = xa < 0 ? xa + a.nx : (xa >= a.nx ? xa - a.nx : xa);
    const double f = fq ? fq[((long long)qa * a.ny + ya) * a.nx + xa] : feq.v[qa];
    encode_store<St>(dst, (long long)i * a.plane + (long long)(y - a.yoff) * a.pitch + x, f, i,
                     a.rho0);
  }
}

// Post-stream populations, density and velocity of the window's cells (pull_load's rule, in
// FP64), written at their lattice rows of [q][ny][nx] outputs.
template <class St>
__global__ void k_gather(LatticeArgs a, const typename St::S* src, double* fq, double* rho,
                         double* ux, double* uy) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = a.y0 + (int)blockIdx.y;
  if (x >= a.nx || y >= a.y0 + a.nyl) return;
  const bool slab = a.nyl != a.ny;
  double f[NQ];
  for (int i = 0; i < NQ; ++i) {
    int xs = x - cx_of(i), ys = y - cy_of(i);
    xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
    long long idx;
    int q = i;
    if (ys < 0 || ys >= a.ny) {
      if (a.walls) {
        q = opp_of(i);
        idx = (long long)q * a.plane + (long long)(y - a.yoff) * a.pitch + x;
        f[i] = decode_load<St>(src, idx, q, a.rho0);
        continue;
      }
      if (!slab) ys = ys < 0 ? ys + a.ny : ys - a.ny;  // a slab reads its ghost row
    }
    idx = (long long)i * a.plane + (long long)(ys - a.yoff) * a.pitch + xs;
    f[i] = decode_load<St>(src, idx, q, a.rho0);
  }
  const long long c = (long long)y * a.nx + x;
  if (fq)
    for (int i = 0; i < NQ; ++i) fq[(long long)i * a.nx * a.ny + c] = f[i];
  double r = 0.0, mx = 0.0, my = 0.0;
  for (int i = 0; i < NQ; ++i) r += f[i];
  for (int i = 0; i < NQ; ++i) {
    mx += (double)cx_of(i) * f[i];
    my += (double)cy_of(i) * f[i];
  }
  if (rho) rho[c] = r;
  if (ux) ux[c] = mx / r;
  if (uy) uy[c] = my / r;
}

template <class St>
void unstream_t(const LatticeArgs& a, const double* fq, const double* feq9, void* dst,
                hipStream_t s) {
  Feq9 fe{};
  if (feq9)
    for (int i = 0; i < NQ; ++i) fe.v[i] = feq9[i];
  dim3 grid((a.nx + 255) / 256, a.nyl + 2);
  hipLaunchKernelGGL(k_unstream<St>, grid, dim3(256), 0, s, a, fq, fe, (typename St::S*)dst);
}

void launch_unstream(int storage, const LatticeArgs& a, const double* fq, const double* feq9,
                     void* dst, hipStream_t s) {
  if (storage == IMB_STORAGE_F64) unstream_t<StoreF64>(a, fq, feq9, dst, s);
  else if (storage == IMB_STORAGE_F32) unstream_t<StoreF32>(a, fq, feq9, dst, s);
  else unstream_t<StoreF16>(a, fq, feq9, dst, s);
}

template <class St>
void gather_t(const LatticeArgs& a, const void* src, double* fq, double* rho, double* ux,
              double* uy, hipStream_t s) {
  dim3 grid((a.nx + 255) / 256, a.nyl);
  hipLaunchKernelGGL(k_gather<St>, grid, dim3(256), 0, s, a, (const typename St::S*)src, fq, rho,
                     ux, uy);
}

void launch_gather(int storage, const LatticeArgs& a, const void* src, double* fq, double* rho,
                   double* ux, double* uy, hipStream_t s) {
  if (storage == IMB_STORAGE_F64) gather_t<StoreF64>(a, src, fq, rho, ux, uy, s);
  else if (storage == IMB_STORAGE_F32) gather_t<StoreF32>(a, src, fq, rho, ux, uy, s);
  else gather_t<StoreF16>(a, src, fq, rho, ux, uy, s);
}

// Streaming copy: each thread moves COPY_UNROLL 16-byte vectors per trip, every load of the trip
// issued before its stores, with non-temporal loads and stores (nothing is reused); the byte
// tail is copied per byte.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int COPY_UNROLL = 4;
__global__ __launch_bounds__(256) void k_copy(u32x4* __restrict__ dst,
                                              const u32x4* __restrict__ src, size_t n16,
                                              unsigned char* dtail, const unsigned char* stail,
                                              int ntail) {
  const size_t chunk = (size_t)256 * COPY_UNROLL;
  for (size_t base = (size_t)blockIdx.x * chunk; base < n16; base += (size_t)gridDim.x * chunk) {
    u32x4 v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
      const size_t i = base + (size_t)u * 256 + threadIdx.x;
      if (i < n16) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
      const size_t i = base + (size_t)u * 256 + threadIdx.x;
      if (i < n16) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) dtail[threadIdx.x] = stail[threadIdx.x];
}

__global__ void k_fill_zero(uint4* dst, size_t n16, unsigned char* dtail, int ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) dtail[threadIdx.x] = 0;
}

static int copy_grid(size_t n16) {
  size_t g = (n16 + 255) / 256;
  if (g > 256 * 16) g = 256 * 16;
  return g < 1 ? 1 : (int)g;
}

void launch_copy(void* dst, const void* src, size_t n_bytes, hipStream_t s) {
  const size_t n16 = n_bytes / 16;
  const int ntail = (int)(n_bytes - n16 * 16);
  // one trip per workgroup up to 2^20 workgroups (16 GiB), grid-stride beyond
  size_t g = (n16 + 256 * COPY_UNROLL - 1) / (256 * COPY_UNROLL);
  if (g > (1u << 20)) g = 1u << 20;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)g), dim3(256), 0, s, (u32x4*)dst,
                     (const u32x4*)src, n16, (unsigned char*)dst + n16 * 16,
                     (const unsigned char*)src + n16 * 16, ntail);
}

void launch_fill_zero(void* dst, size_t n_bytes, hipStream_t s) {
  const size_t n16 = n_bytes / 16;
  const int ntail = (int)(n_bytes - n16 * 16);
  hipLaunchKernelGGL(k_fill_zero, dim3(copy_grid(n16)), dim3(256), 0, s, (uint4*)dst, n16,
                     (unsigned char*)dst + n16 * 16, ntail);
}

}  // namespace imb
