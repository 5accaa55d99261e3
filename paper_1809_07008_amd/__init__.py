"""MI355X (gfx950) implementation of the coupled D2Q9 lattice-Boltzmann / immersed-moving-boundary
/ DEM time step of Yang, Jing, Kwok & Sobral (arXiv:1809.07008).

The compute path is a C-ABI library of hand-written HIP kernels (``libimb.so``, declared in
``include/imb.h``); :mod:`paper_1809_07008_amd.imb` is its thin ctypes binding.  Importing this
package does not load the library; the binding does, and fails loudly if it is missing.
"""

__all__ = ["imb", "workloads", "adjoint"]
