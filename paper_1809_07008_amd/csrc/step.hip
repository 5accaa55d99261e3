// step.hip -- the coupled step as one kernel.  Workgroups [0, np) are the disks' (disk_cells:
// covered cells, each disk's force and torque), the rest the tiles' (fluid_tile: the cells no disk
// covers); the disks' workgroups are dispatched first.  The last disk workgroup to finish runs
// the particle phase (particle_phase.h: DEM and the next step's disk tables) while the tiles
// still stream, so the one-workgroup DEM costs no extra launch and mostly no extra time.  The
// particle phase writes the other copy of the disk tables, never the one the tiles read.
#include "disk_block.h"
#include "particle_phase.h"
#include "step.h"

namespace imb {

// Register budget: 80 VGPRs (6 waves per SIMD), what the lattice roles need; the particle phase,
// run by one workgroup per launch, spills its excess.
template <class St>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_step(
    LatticeArgs a, ParticleArgs pa, int with_dem) {
  extern __shared__ double lds[];
  __shared__ int s_last;
  const int b = blockIdx.x;
  if (b >= a.np) {
    fluid_tile<St>(a, xcd_remap(b - a.np, a.tiles_x * a.tiles_y));
    return;
  }
  disk_cells<St>(a, b);
  if (!with_dem) return;
  // count this workgroup as finished once its force store is visible device-wide
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(a.done, 1u) == (unsigned)a.np - 1u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();  // every disk's force is visible to this workgroup
  if (threadIdx.x == 0) __hip_atomic_store(a.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  particle_phase<BLOCK>(pa, lds);
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
void launch_step_t(const LatticeArgs& a, const ParticleArgs& pa, bool with_dem, hipStream_t s) {
  const bool dem = with_dem && a.np > 0;
  const size_t lds = dem ? particle_phase_lds(pa.np, pa.tiles_y) : 0;
  hipLaunchKernelGGL(k_step<St>, dim3(a.np + a.tiles_x * a.tiles_y), dim3(BLOCK), lds, s, a, pa,
                     dem ? 1 : 0);
}

void launch_step(int storage, const LatticeArgs& a, const ParticleArgs& pa, bool with_dem,
                 hipStream_t s) {
  switch (storage) {
    case IMB_STORAGE_F64: launch_step_t<StoreF64>(a, pa, with_dem, s); break;
    case IMB_STORAGE_F32: launch_step_t<StoreF32>(a, pa, with_dem, s); break;
    default: launch_step_t<StoreF16>(a, pa, with_dem, s); break;
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
