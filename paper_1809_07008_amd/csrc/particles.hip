// particles.hip -- the particle phase as its own one-workgroup kernel (particle_phase.h).
#include <hip/hip_ext.h>

#include "particle_phase.h"

namespace imb {

__global__ __launch_bounds__(PBLOCK) void k_particle_phase(ParticleArgs a) {
  extern __shared__ double lds[];
  particle_phase<PBLOCK>(a, lds);
}

// LDS of the phase: the DEM's per-disk tables, or the band masks of up to 512 tile rows at a
// time (more rows take several rounds).
size_t particle_phase_lds(int np, int tiles_y) {
  const size_t dem = (size_t)np * PP_DOUBLES * sizeof(double);
  const size_t band = (size_t)(tiles_y < 512 ? tiles_y : 512) * MASK_WORDS * sizeof(double);
  return dem > band ? dem : band;
}

void launch_particle_phase(const ParticleArgs& args, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  const size_t lds = particle_phase_lds(args.np, args.tiles_y);
  ParticleArgs a = args;
  a.lds_doubles = (int)(lds / sizeof(double));
  if (e0 || e1)
    hipExtLaunchKernelGGL(k_particle_phase, dim3(1), dim3(PBLOCK), (uint32_t)lds, s, e0, e1, 0, a);
  else
    hipLaunchKernelGGL(k_particle_phase, dim3(1), dim3(PBLOCK), lds, s, a);
}

}  // namespace imb
