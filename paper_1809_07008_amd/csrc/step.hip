// step.hip -- the lattice part of a coupled step as one kernel: workgroups [0, dparts np) are
// the disks' (disk_cells: covered cells, each disk's force and torque, one or two workgroups per
// disk), the rest the tiles' (fluid_tile: the cells no disk covers).  A second instantiation
// runs a window of rows of a lattice split in y (one slab, with ghost rows).  The disks' longer,
// latency-bound work is dispatched first and overlaps the tiles' streaming.  The particle phase
// follows as its own one-workgroup kernel (particles.hip) on the same stream.
#include <hip/hip_ext.h>

#include "disk_block.h"
#include "step.h"

namespace imb {

// W: the lattice is a window of rows of a larger one (a slab), with ghost rows.
template <class St, bool W>
__device__ __forceinline__ void lattice_roles(const LatticeArgs& a) {
  const int b = blockIdx.x;
  const int nd = a.np * a.dparts;  // disk items: dparts per disk
  if (b < nd) {
    disk_cells<St, W>(a, b);
    return;
  }
  fluid_tile<St, W>(a, xcd_remap(b - nd, a.tiles_x * a.tiles_y));
}

// FP32 arithmetic (FP32 or FP16 storage): held to 80 VGPRs, six wavefronts per SIMD.
template <class St, bool W>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_step(
    LatticeArgs a) {
  lattice_roles<St, W>(a);
}

// FP64 arithmetic needs more registers than that budget (it would spill).
template <bool W>
__global__ __launch_bounds__(BLOCK) void k_step_f64(LatticeArgs a) {
  lattice_roles<StoreF64, W>(a);
}

// eps_tot of every cell (diagnostic / parity of the solid-ratio stage alone).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_solid_field(LatticeArgs a, double* eps_out) {
  __shared__ PEntry<T> s_pl[LMAX];
  __shared__ int s_cnt[2 * WAVES];
  __shared__ int s_pid[LMAX], s_slot[LMAX];
  __shared__ CellScratch<T> cs;
  __shared__ T s_off[64];  // sub-cell offsets when eps_sub > 0 (eps_sub <= 64)
  const int tid = threadIdx.x;
  // the sub-cell offsets of the paper's estimate, read after the tile list's barriers
  if (tid < a.eps_sub) s_off[tid] = subcell_offset<T>(tid, a.eps_sub);
  const T* off = a.eps_sub > 0 ? s_off : nullptr;
  const int tile = blockIdx.x;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tw = 1 << a.tw_log, th = BLOCK >> a.tw_log;
  const int x = tx * tw + (tid & (tw - 1));
  const int ybase = ty * th * a.rows + (tid >> a.tw_log);
  const int n = build_tile_list<T>(a, tx, ty, s_pl, s_cnt, s_pid, s_slot);
  for (int rr = 0; rr < a.rows; ++rr) {
    const int y = ybase + rr * th;
    if (x >= a.nx || y >= a.ny) continue;
    const int nc = covering_disks<T>(a, s_pl, n, x, y, cs, off);
    double s = 0.0;
    for (int k = 0; k < nc; ++k) s += (double)cs.ce[k][tid];
    eps_out[(long long)y * a.nx + x] = s;
  }
}

void launch_lattice_step(int storage, const LatticeArgs& a, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  const dim3 grid(a.np * a.dparts + a.tiles_x * a.tiles_y);
  auto go = [&](auto kernel) {
    if (e0 || e1) hipExtLaunchKernelGGL(kernel, grid, dim3(BLOCK), 0, s, e0, e1, 0, a);
    else hipLaunchKernelGGL(kernel, grid, dim3(BLOCK), 0, s, a);
  };
  if (a.nyl != a.ny) {  // a slab
    switch (storage) {
      case IMB_STORAGE_F64: go(k_step_f64<true>); break;
      case IMB_STORAGE_F32: go(k_step<StoreF32, true>); break;
      default: go(k_step<StoreF16, true>); break;
    }
    return;
  }
  switch (storage) {
    case IMB_STORAGE_F64: go(k_step_f64<false>); break;
    case IMB_STORAGE_F32: go(k_step<StoreF32, false>); break;
    default: go(k_step<StoreF16, false>); break;
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
