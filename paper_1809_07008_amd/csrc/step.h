// step.h -- host-side launchers of the kernels (one translation unit each).
#pragma once

#include "common.h"

namespace imb {

// lattice step (step.hip): the disks' covered cells and forces, the tiles' uncovered cells, and
// both in that order on one stream
void launch_disk_step(int storage, const LatticeArgs& a, hipStream_t s);
void launch_fluid_step(int storage, const LatticeArgs& a, hipStream_t s);
void launch_lattice_step(int storage, const LatticeArgs& a, hipStream_t s);
void launch_solid_field(int storage, const LatticeArgs& a, double* eps_out, hipStream_t s);

// particle phase (particles.hip): force finalisation, DEM, tile boxes for the next step
void launch_particle_phase(const ParticleArgs& a, hipStream_t s);

// population format conversion and moments (convert.hip)
void launch_unstream(int storage, const LatticeArgs& a, const double* fq, const double* feq9,
                     void* dst, hipStream_t s);
void launch_gather(int storage, const LatticeArgs& a, const void* src, double* fq, double* rho,
                   double* ux, double* uy, hipStream_t s);
void launch_copy(void* dst, const void* src, size_t n_bytes, hipStream_t s);
void launch_fill_zero(void* dst, size_t n_bytes, hipStream_t s);

}  // namespace imb
