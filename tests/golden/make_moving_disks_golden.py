"""Writes moving_disks_2048x1024_n500_fp64.npz: the FP64 oracle's state after 1000 coupled steps
of the moving-disk channel (2048x1024, walls in y, 500 free disks of diameter U[16, 24] seeded
with seed 0, velocities N(0, 0.01), tau 0.55, Smagorinsky C_s = 0.1, g_x = 1e-6, linear
spring-dashpot DEM with 10 sub-cycles).

Stored (all from the oracle; nothing here runs the HIP path):
  fx, fy, tz           force and torque on every disk in step 1000 (Eqs. 15, 16)
  sF, sT               their conditioning scales: per disk the sum over its covered cells of
                       |dF| and of |d| |dF| (dF the per-cell force contribution, d its lever arm)
  x, y, vx, vy, om     disk state after the DEM of step 1000
  ux_s, uy_s, rho_s    the velocity and density fields after step 1000 on the sub-grid
                       rows 3::8, columns 3::8 (128 x 256 nodes)
  umax                 max over the whole field of max(|u_x|, |u_y|)
  fx10, fy10, tz10, sF10, sT10   the same forces and scales after step 10
  fx_r1, fy_r1, tz_r1  the forces after step 1000 of a second oracle run whose radii are all
                       larger by one unit in the last place (r (1 + 2^-52)): how far the result
                       moves under a change of the input below any rounding of the solid ratio
                       (the conditioning of the 1000-step forces)

Takes a few minutes on 8 cores.  Run from the repository root:
    python tests/golden/make_moving_disks_golden.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT]

import numpy as np  # noqa: E402

from oracle import OracleConfig, OracleSim  # noqa: E402
from paper_1809_07008_amd import workloads as W  # noqa: E402

SEED = 0
STEPS = 1000
OUT = os.path.join(HERE, "moving_disks_2048x1024_n500_fp64.npz")
SUB = (slice(3, None, 8), slice(3, None, 8))


def oracle_run(case, rfac=1.0):
    ref = OracleSim(OracleConfig(nx=case.nx, ny=case.ny, tau0=case.tau0, walls=case.walls,
                                 cs=case.cs, gx=case.gx, gy=case.gy, rho0=case.rho0,
                                 n_sub=case.n_sub, kn=case.kn, zeta=case.zeta, rho_s=case.rho_s))
    p = case.particles
    ref.set_particles(p.x, p.y, p.r * rfac, p.vx, p.vy, p.om, p.mode)
    return ref


def main():
    case = W.moving_disks(seed=SEED, storage="f64")
    ref = oracle_run(case)
    t0 = time.time()
    out = {}
    done = 0
    for chunk in (10, 90, 300, 300, 300):
        ref.step(chunk)
        done += chunk
        print("oracle: %d steps, %.0f s" % (done, time.time() - t0), flush=True)
        if done == 10:
            for k, v in zip(("fx10", "fy10", "tz10"), ref.forces()):
                out[k] = v
            for k, v in zip(("sF10", "sT10"), ref.force_scales()):
                out[k] = v
    assert done == STEPS
    for k, v in zip(("fx", "fy", "tz"), ref.forces()):
        out[k] = v
    for k, v in zip(("sF", "sT"), ref.force_scales()):
        out[k] = v
    for k, v in zip(("x", "y", "vx", "vy", "om"), ref.particles()):
        out[k] = v
    rho, ux, uy = ref.fields()
    out["ux_s"] = ux[SUB]
    out["uy_s"] = uy[SUB]
    out["rho_s"] = rho[SUB]
    out["umax"] = np.array(max(np.abs(ux).max(), np.abs(uy).max()))
    out["meta"] = np.array([SEED, STEPS, case.nx, case.ny, case.particles.n], np.int64)
    pert = oracle_run(case, 1.0 + 2.0 ** -52)
    pert.step(STEPS)
    print("oracle (radii + 1 ulp): %d steps, %.0f s" % (STEPS, time.time() - t0), flush=True)
    for k, v in zip(("fx_r1", "fy_r1", "tz_r1"), pert.forces()):
        out[k] = v
    np.savez_compressed(OUT, **out)
    print("wrote %s in %.0f s" % (os.path.basename(OUT), time.time() - t0))


if __name__ == "__main__":
    main()
