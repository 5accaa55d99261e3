"""Central finite differences of the FP64 oracle's objective: the reference the discrete adjoint
is checked against.

J = sum over steps n and disks p of wfx_p Fx_p^n + wfy_p Fy_p^n + wtz_p Tz_p^n, evaluated by the
oracle (plain FP64 CPU implementation of the coupled step) with the disks in prescribed motion.
Each derivative is the Richardson combination (4 D(h/2) - D(h)) / 3 of two central differences
D(h) = (J(p + h) - J(p - h)) / 2h, which removes the O(h^2) term.  Steps: h = 1e-4 lattice units
for positions, 1e-4 per step for velocities and spin, 1e-4 * |g_x| for both body-force
components.  Test infrastructure only (calls the oracle, nothing of the HIP path).
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import OracleConfig, OracleSim

PARAMS = ("x", "y", "vx", "vy", "om")


def objective(case, state, gx, gy, steps, wfx=None, wfy=None, wtz=None, f0=None) -> float:
    """J of the oracle for disk state ``state`` (dict of x, y, vx, vy, om arrays)."""
    ref = OracleSim(OracleConfig(nx=case.nx, ny=case.ny, tau0=case.tau0, walls=case.walls,
                                 cs=case.cs, gx=gx, gy=gy, rho0=case.rho0, n_sub=case.n_sub,
                                 kn=case.kn, zeta=case.zeta, rho_s=case.rho_s))
    if f0 is not None:
        ref.set_populations(f0)
    p = case.particles
    ref.set_particles(state["x"], state["y"], p.r, state["vx"], state["vy"], state["om"], p.mode)
    return ref.step_accumulate(steps, wfx, wfy, wtz)


def base_state(case) -> dict:
    p = case.particles
    return {"x": p.x.copy(), "y": p.y.copy(), "vx": p.vx.copy(), "vy": p.vy.copy(),
            "om": p.om.copy()}


def fd_gradient(case, steps, wfx=None, wfy=None, wtz=None, h=1e-4, hg_rel=1e-4,
                params=PARAMS + ("g",), disks=None, richardson=True) -> dict:
    """Finite-difference gradient of J.  Returns {name: array} for the disk parameters (length
    n, or the selected ``disks``) and "g" (2 values), plus "J"."""
    s0 = base_state(case)
    gx0, gy0 = case.gx, case.gy
    n = case.particles.n
    idx = list(range(n)) if disks is None else list(disks)

    def central(fn, step):
        return (fn(step) - fn(-step)) / (2.0 * step)

    def derivative(fn, step):
        d1 = central(fn, step)
        if not richardson:
            return d1
        d2 = central(fn, step / 2.0)
        return (4.0 * d2 - d1) / 3.0

    out = {"J": objective(case, s0, gx0, gy0, steps, wfx, wfy, wtz)}
    for name in params:
        if name == "g":
            hg = hg_rel * abs(gx0) if gx0 != 0.0 else 1e-10
            gxd = derivative(lambda e: objective(case, s0, gx0 + e, gy0, steps, wfx, wfy, wtz), hg)
            gyd = derivative(lambda e: objective(case, s0, gx0, gy0 + e, steps, wfx, wfy, wtz), hg)
            out["g"] = np.array([gxd, gyd])
            continue
        g = np.zeros(len(idx))
        for k, p in enumerate(idx):
            def fn(e, name=name, p=p):
                s = {key: v.copy() for key, v in s0.items()}
                s[name][p] += e
                return objective(case, s, gx0, gy0, steps, wfx, wfy, wtz)
            g[k] = derivative(fn, h)
        out[name] = g
    return out


def block_errors(adj: dict, fd: dict, names=PARAMS + ("g",)) -> dict:
    """Norm-wise relative error per gradient block: ||a - f|| / ||f||."""
    errs = {}
    for name in names:
        if name not in fd:
            continue
        a = np.asarray(adj[name] if name in adj else adj[name + "0"], float)
        f = np.asarray(fd[name], float)
        nf = np.linalg.norm(f)
        errs[name] = float(np.linalg.norm(a - f) / nf) if nf > 0 else float(np.linalg.norm(a))
    return errs


def elementwise_errors(adj: dict, fd: dict, names=PARAMS + ("g",)) -> dict:
    """Per gradient block, the element-wise relative errors |a_i - f_i| / |f_i| (array)."""
    errs = {}
    for name in names:
        if name not in fd:
            continue
        a = np.asarray(adj[name] if name in adj else adj[name + "0"], float)
        f = np.asarray(fd[name], float)
        errs[name] = np.abs(a - f) / np.where(f != 0.0, np.abs(f), 1.0)
    return errs
