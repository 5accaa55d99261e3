"""FP64 CPU oracle of the coupled D2Q9 LBM-IMB-DEM step and of the D3Q19 lattice step with
spheres.

Test infrastructure only: used by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the product package.
"""
from .oracle import (OracleConfig, OracleConfig3, OracleSim, OracleSim3, build, collide_cell,
                     collide_cell3, get_threads, set_threads, solid_fraction, subcell_fraction,
                     subcell_fraction3, weight)

__all__ = ["OracleConfig", "OracleConfig3", "OracleSim", "OracleSim3", "build", "collide_cell",
           "collide_cell3", "get_threads", "set_threads", "solid_fraction", "subcell_fraction",
           "subcell_fraction3", "weight"]
