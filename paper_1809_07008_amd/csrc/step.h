// step.h -- host-side launchers of the kernels (one translation unit each).
#pragma once

#include "common.h"

namespace imb {

// lattice part of the coupled step (step.hip): every cell's update, each disk's force and torque
// With e0/e1 given, the events are recorded at the kernel's own start and end (timing).
void launch_lattice_step(int storage, const LatticeArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
void launch_solid_field(int storage, const LatticeArgs& a, double* eps_out, hipStream_t s);

// particle phase alone (particles.hip): DEM and/or the disk tables, one workgroup
void launch_particle_phase(const ParticleArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
size_t particle_phase_lds(int np, int tiles_y);  // dynamic LDS bytes of the particle phase

// population format conversion and moments (convert.hip)
void launch_unstream(int storage, const LatticeArgs& a, const double* fq, const double* feq9,
                     void* dst, hipStream_t s);
void launch_gather(int storage, const LatticeArgs& a, const void* src, double* fq, double* rho,
                   double* ux, double* uy, hipStream_t s);
void launch_copy(void* dst, const void* src, size_t n_bytes, hipStream_t s);
void launch_fill_zero(void* dst, size_t n_bytes, hipStream_t s);

}  // namespace imb
