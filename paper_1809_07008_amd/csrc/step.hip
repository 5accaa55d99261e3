// step.hip -- the lattice step as two kernels (disk_block.h): the covered cells and each disk's
// force by the disks' workgroups, the uncovered cells by the tiles.  They write disjoint cells and
// read only the source populations and the step's disk tables, so they may run concurrently.
#include "disk_block.h"
#include "step.h"

namespace imb {

// One workgroup per disk: its covered cells and its own force and torque.
template <class St>
__global__ __launch_bounds__(BLOCK) void k_disk_step(LatticeArgs a) {
  disk_cells<St>(a, blockIdx.x / DISK_PARTS, blockIdx.x % DISK_PARTS);
}

// One workgroup per tile: the cells no disk covers.
template <class St>
__global__ __launch_bounds__(BLOCK) void k_fluid_step(LatticeArgs a) {
  fluid_tile<St>(a, xcd_remap(blockIdx.x, a.tiles_x * a.tiles_y));
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
void launch_disk_step_t(const LatticeArgs& a, hipStream_t s) {
  if (a.np > 0) hipLaunchKernelGGL(k_disk_step<St>, dim3(a.np * DISK_PARTS), dim3(BLOCK), 0, s, a);
}

template <class St>
void launch_fluid_step_t(const LatticeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_fluid_step<St>, dim3(a.tiles_x * a.tiles_y), dim3(BLOCK), 0, s, a);
}

void launch_disk_step(int storage, const LatticeArgs& a, hipStream_t s) {
  switch (storage) {
    case IMB_STORAGE_F64: launch_disk_step_t<StoreF64>(a, s); break;
    case IMB_STORAGE_F32: launch_disk_step_t<StoreF32>(a, s); break;
    default: launch_disk_step_t<StoreF16>(a, s); break;
  }
}

void launch_fluid_step(int storage, const LatticeArgs& a, hipStream_t s) {
  switch (storage) {
    case IMB_STORAGE_F64: launch_fluid_step_t<StoreF64>(a, s); break;
    case IMB_STORAGE_F32: launch_fluid_step_t<StoreF32>(a, s); break;
    default: launch_fluid_step_t<StoreF16>(a, s); break;
  }
}

void launch_lattice_step(int storage, const LatticeArgs& a, hipStream_t s) {
  launch_disk_step(storage, a, s);
  launch_fluid_step(storage, a, s);
}

void launch_solid_field(int storage, const LatticeArgs& a, double* eps_out, hipStream_t s) {
  const int tiles = a.tiles_x * a.tiles_y;
  if (storage == IMB_STORAGE_F64)
    hipLaunchKernelGGL(k_solid_field<double>, dim3(tiles), dim3(BLOCK), 0, s, a, eps_out);
  else
    hipLaunchKernelGGL(k_solid_field<float>, dim3(tiles), dim3(BLOCK), 0, s, a, eps_out);
}

}  // namespace imb
