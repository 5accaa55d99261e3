"""FP64 CPU oracle of the coupled D2Q9 LBM-IMB-DEM step.

Test infrastructure only: used by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the product package.
"""
from .oracle import (OracleConfig, OracleSim, build, collide_cell, get_threads, set_threads,
                     solid_fraction, subcell_fraction, weight)

__all__ = ["OracleConfig", "OracleSim", "build", "collide_cell", "get_threads", "set_threads",
           "solid_fraction", "subcell_fraction", "weight"]
