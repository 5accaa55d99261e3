"""Writes adjoint_512x256_n20.json: the FP64 oracle's objective and its central-difference
gradient for the adjoint workload (512x256 channel, walls in y, 20 disks of diameter 20 at
seeded positions, at rest in prescribed motion, tau 0.6, g_x = 1e-6, 200 steps), with
J = sum over the 200 steps and the 20 disks of the x-force on the disk (Eq. 15).

Calls only the oracle (through tests/adjoint_fd.py) and the seeded input generator.  Derivatives
are Richardson-extrapolated central differences with h = 1e-4 lattice units (positions),
1e-4 per step (velocities, spin) and 1e-4 * g_x (body force).  Run from the repository root:
    python tests/golden/make_adjoint_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

import numpy as np  # noqa: E402

from adjoint_fd import fd_gradient  # noqa: E402
from paper_1809_07008_amd import workloads as W  # noqa: E402

SEED = 0


def main():
    case = W.adjoint_channel(seed=SEED)
    n = case.particles.n
    t0 = time.time()
    g = fd_gradient(case, case.steps, wfx=np.ones(n))
    out = {
        "what": "J = sum over steps and disks of Fx (force on the disk); FP64 oracle; gradient by "
                "Richardson-extrapolated central differences",
        "workload": case.name, "seed": SEED, "steps": case.steps, "tau0": case.tau0,
        "gx": case.gx, "h_position": 1e-4, "h_velocity": 1e-4, "h_g_relative": 1e-4,
        "J": g["J"],
        "gradient": {k: np.asarray(v).tolist() for k, v in g.items() if k != "J"},
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "adjoint_512x256_n20.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote adjoint_512x256_n20.json in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
