"""torch.autograd.Function over the library's discrete adjoint (imb_adjoint).

``drag_objective(x, y, vx, vy, om, g, setup)`` returns the scalar
    J = sum over the unrolled steps n and disks p of wfx_p Fx_p^n + wfy_p Fy_p^n + wtz_p Tz_p^n
(hydrodynamic force and torque on the disks, Eqs. 15-16) of a channel whose disks move with
prescribed constant velocity (X^n = X^0 + n V, spin omega), and differentiates it with respect to
the disk positions, velocities, spins and the body force g.  forward runs the forward pass with
its checkpoints (imb_adjoint_forward) and keeps the simulation; backward runs the recomputation
and the adjoint sweep (imb_adjoint_backward), releases the simulation and scales the gradients by
the incoming gradient.  All arithmetic runs in the HIP kernels; the tensors here are FP64 host
tensors that carry the inputs and results across the C-ABI.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import imb


@dataclass
class AdjointSetup:
    """The fixed part of the differentiated problem (lattice units)."""
    nx: int
    ny: int
    radii: np.ndarray
    tau0: float
    steps: int
    k_ckpt: int = 20
    storage: str = "f32"
    walls: bool = True
    rho0: float = 1.0
    wfx: Optional[np.ndarray] = None   # default: ones (summed x-drag)
    wfy: Optional[np.ndarray] = None
    wtz: Optional[np.ndarray] = None
    fixed: bool = False                # disks stay in place (V enters only the solid velocity)
    tile: tuple = (32, 2)
    stream: object = None
    last: dict = field(default_factory=dict)  # timings of the last call


def _np(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu", torch.float64).numpy()


class DragObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, vx, vy, om, g, setup: AdjointSetup):
        n = len(setup.radii)
        gx, gy = (float(v) for v in _np(g).reshape(2))
        cfg = imb.make_config(setup.nx, setup.ny, setup.tau0, storage=setup.storage,
                              walls=setup.walls, gx=gx, gy=gy, rho0=setup.rho0,
                              max_particles=max(n, 1), tile_w=setup.tile[0],
                              tile_rows=setup.tile[1])
        sim = imb.Simulation(cfg, setup.stream)
        try:
            mode = np.full(n, imb.MODE_FIXED if setup.fixed else imb.MODE_PRESCRIBED, np.int32)
            sim.set_particles(_np(x), _np(y), np.asarray(setup.radii, float), _np(vx), _np(vy),
                              _np(om), mode)
            wfx = np.ones(n) if setup.wfx is None else setup.wfx
            J = sim.adjoint_forward(setup.steps, setup.k_ckpt, wfx=wfx, wfy=setup.wfy,
                                    wtz=setup.wtz)
        except BaseException:
            sim.close()
            raise
        ctx.sim = sim  # holds the checkpoints until backward
        ctx.setup = setup
        ctx.meta = (x.dtype, x.device, g.dtype, g.device, g.shape)
        return torch.tensor(J, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, gJ):
        # the reverse sweep runs once; a second backward through the same graph
        # (retain_graph) reuses its gradients
        res = getattr(ctx, "grads", None)
        if res is None:
            sim = ctx.sim
            try:
                res = sim.adjoint_backward()
                ctx.setup.last = sim.adjoint_timing()
            finally:
                sim.close()
                ctx.sim = None
            ctx.grads = res
        xd, xdev, gd, gdev, gshape = ctx.meta
        grads = [torch.as_tensor(res[k], dtype=xd, device=xdev)
                 for k in ("x0", "y0", "vx", "vy", "om")]
        grads.append(torch.as_tensor(res["g"], dtype=gd, device=gdev).reshape(gshape))
        return tuple(gJ.to(t.dtype) * t for t in grads) + (None,)


def drag_objective(x, y, vx, vy, om, g, setup: AdjointSetup) -> torch.Tensor:
    """Differentiable summed (weighted) drag; see the module docstring."""
    return DragObjective.apply(x, y, vx, vy, om, g, setup)
