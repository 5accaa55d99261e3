"""Seeded synthetic inputs for the D2Q9 LBM-IMB-DEM step.

This module only draws random numbers and places disks; it contains none of the method's
arithmetic, so that the HIP path and the CPU oracle can both be fed from it without sharing code.

Parameters follow the paper's ranges: about 20 lattice cells per particle diameter (Sec. 3.1.2
and Sec. 4 recommend N = 20), relaxation times between 0.5 and 1 (Sec. 3.1.3), dilute to moderately
dense disk fractions, a linear spring-dashpot DEM (Eq. 8) and a small driving body force
(Sec. 3.1.1).  The paper measures on no public dataset; these generators stand in for its
benchmark set-ups in two dimensions.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

MODE_FREE, MODE_FIXED, MODE_PRESCRIBED = 0, 1, 2


@dataclass
class Particles:
    x: np.ndarray
    y: np.ndarray
    r: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    om: np.ndarray
    mode: np.ndarray

    @property
    def n(self) -> int:
        return int(len(self.x))

    @staticmethod
    def empty() -> "Particles":
        z = np.zeros(0)
        return Particles(z, z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), np.zeros(0, np.int32))

    def copy(self) -> "Particles":
        return Particles(*(np.array(a, copy=True) for a in
                           (self.x, self.y, self.r, self.vx, self.vy, self.om, self.mode)))


@dataclass
class Case:
    """One simulation set-up in lattice units (dx = dt = 1)."""
    name: str
    nx: int
    ny: int
    tau0: float
    steps: int
    storage: str = "f64"        # population storage: f64, f32 (deviations) or f16 (deviations)
    walls: bool = True          # half-way bounce-back walls in y (x always periodic)
    cs: float = 0.0             # Smagorinsky constant
    gx: float = 1.0e-6
    gy: float = 0.0
    rho0: float = 1.0
    n_sub: int = 10
    kn: float = 1.0e3
    zeta: float = 0.1
    rho_s: float = 1.0
    eps_subcells: int = 0       # solid ratio: 0 exact area, n > 0 the n x n sub-cell estimate
    uw_bot: float = 0.0         # x-velocity of the bottom wall (walls only)
    uw_top: float = 0.0         # x-velocity of the top wall (walls only)
    kt: float = 0.0             # tangential contact stiffness (with mu: the tangential force)
    mu: float = 0.0             # Coulomb friction coefficient of the tangential contact force
    contact_model: int = 0      # 0 linear spring-dashpot (kn, kt), 1 Hertz-Mindlin
    young: float = 0.0          # Young's modulus (Hertz-Mindlin)
    poisson: float = 0.0        # Poisson's ratio (Hertz-Mindlin)
    particles: Particles = field(default_factory=Particles.empty)

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def with_(self, **kw) -> "Case":
        return replace(self, **kw)


def place_disks(rng: np.random.Generator, nx: int, ny: int, n: int, dmin: float, dmax: float,
                gap: float, wall_gap: float, walls: bool = True, max_tries: int = 200000):
    """Random sequential addition of n disks with diameters U[dmin, dmax]: surface gap >= gap to
    every other disk (nearest periodic image in x, and in y without walls) and >= wall_gap to the
    walls at y = -1/2 and y = ny - 1/2.  Returns (x, y, r) as float64 arrays."""
    xs, ys, rs = [], [], []
    tries = 0
    while len(xs) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d disks in %dx%d" % (n, nx, ny))
        r = 0.5 * rng.uniform(dmin, dmax)
        x = rng.uniform(0.0, nx)
        if walls:
            lo, hi = -0.5 + r + wall_gap, ny - 0.5 - r - wall_gap
            if hi <= lo:
                continue
            y = rng.uniform(lo, hi)
        else:
            y = rng.uniform(0.0, ny)
        if xs:
            ax, ay, ar = np.asarray(xs), np.asarray(ys), np.asarray(rs)
            ddx = ax - x
            ddx -= nx * np.round(ddx / nx)
            ddy = ay - y
            if not walls:
                ddy -= ny * np.round(ddy / ny)
            if np.any(np.hypot(ddx, ddy) < ar + r + gap):
                continue
        xs.append(x); ys.append(y); rs.append(r)
    return np.asarray(xs), np.asarray(ys), np.asarray(rs)


def _particles(x, y, r, vx=None, vy=None, om=None, mode=MODE_FREE) -> Particles:
    n = len(x)
    z = np.zeros(n)
    return Particles(np.asarray(x, float), np.asarray(y, float), np.asarray(r, float),
                     z.copy() if vx is None else np.asarray(vx, float),
                     z.copy() if vy is None else np.asarray(vy, float),
                     z.copy() if om is None else np.asarray(om, float),
                     np.full(n, mode, np.int32))


def single_disk_channel(storage: str = "f64") -> Case:
    """200x100 channel, one fixed disk of diameter 20 at (60, 50), tau = 0.6, g_x = 1e-6,
    periodic x, walls in y, rest state, 1000 steps (drag and velocity field)."""
    p = _particles([60.0], [50.0], [10.0], mode=MODE_FIXED)
    return Case("single_disk_200x100", 200, 100, tau0=0.6, steps=1000, storage=storage, gx=1.0e-6,
                particles=p)


def moving_disks(seed: int = 0, nx: int = 2048, ny: int = 1024, n: int = 500,
                 storage: str = "f32", steps: int = 1000) -> Case:
    """2048x1024 channel with 500 free disks, diameters U[16, 24], surface gap >= 1 and wall gap
    >= 1, velocities N(0, 0.01), no spin; tau = 0.55, Smagorinsky C_s = 0.1, k_n = 1e3,
    damping ratio 0.1, 10 DEM sub-cycles, g_x = 1e-6."""
    rng = np.random.default_rng(seed)
    x, y, r = place_disks(rng, nx, ny, n, 16.0, 24.0, gap=1.0, wall_gap=1.0)
    vx = rng.normal(0.0, 0.01, n)
    vy = rng.normal(0.0, 0.01, n)
    p = _particles(x, y, r, vx, vy, mode=MODE_FREE)
    return Case("moving_disks_%dx%d_n%d" % (nx, ny, n), nx, ny, tau0=0.55, steps=steps,
                storage=storage, cs=0.1, gx=1.0e-6, kn=1.0e3, zeta=0.1, n_sub=10, particles=p)


def touching_disks(rows: int = 6, walls: bool = True, steps: int = 4, seed: int = 0) -> Case:
    """Free disks of radius U[2.9, 3.01] on a triangular lattice of spacing 6 (ten per row,
    positions jittered by 0.05), so each touches or nearly touches its six nearest neighbours and
    has twelve within the DEM list reach; velocities N(0, 0.02).  60x48 with walls, 60x42
    periodic; k_n = 20 keeps the overlaps' accelerations small."""
    rng = np.random.default_rng(11 + rows + 100 * seed)
    xs, ys = [], []
    for k in range(rows):
        for c in range(10):
            xs.append((6.0 * c + 3.0 * (k % 2) + rng.uniform(-0.05, 0.05)) % 60.0)
            ys.append(4.0 + 5.196 * k + rng.uniform(-0.05, 0.05))
    n = len(xs)
    r = rng.uniform(2.9, 3.01, n)
    p = _particles(xs, ys, r, rng.normal(0.0, 0.02, n), rng.normal(0.0, 0.02, n))
    return Case("touching_disks_%d" % n, 60, 48 if walls else 42, tau0=0.7, steps=steps,
                walls=walls, gx=1.0e-5, kn=20.0, particles=p)


def frictional_disks(rows: int = 6, walls: bool = True, steps: int = 4, kt: float = 10.0,
                     mu: float = 0.3, seed: int = 0) -> Case:
    """The packing of :func:`touching_disks` with the tangential contact force (k_t, mu) and
    spins N(0, 0.005).  With walls the packing sits 1.6 cells lower, so its bottom row presses
    on the bottom wall, and the walls move along x at +0.01 (bottom) and -0.01 (top)."""
    base = touching_disks(rows, walls, steps, seed)
    p = base.particles.copy()
    rng = np.random.default_rng(31 + rows + 100 * seed)
    p.om[:] = rng.normal(0.0, 0.005, p.n)
    if walls:
        p.y[:] -= 1.6
    return base.with_(name="frictional_disks_%d" % p.n, particles=p, kt=kt, mu=mu,
                      uw_bot=0.01 if walls else 0.0, uw_top=-0.01 if walls else 0.0)


def crowded_disk(n_small: int = 7, kt: float = 10.0, mu: float = 0.3) -> Case:
    """64x48 channel with walls: a free disk of radius 6 at (32, 24) and n_small free disks of
    radius 2 around it, centres 7.95 away at equal angles, each overlapping it by 0.05 (and
    apart from one another, up to nine); with nine the large disk has more simultaneous contacts
    than its tangential spring table holds."""
    a = 2.0 * np.pi * np.arange(n_small) / n_small
    x = [32.0] + list(32.0 + 7.95 * np.cos(a))
    y = [24.0] + list(24.0 + 7.95 * np.sin(a))
    p = _particles(x, y, [6.0] + [2.0] * n_small)
    return Case("crowded_disk_%d" % n_small, 64, 48, tau0=0.7, steps=2, gx=1.0e-5, kn=20.0,
                kt=kt, mu=mu, particles=p)


def approaching_disks(steps: int = 300) -> Case:
    """128x48 channel with walls, free disks of radius 5 on the line y = 24: a touching pair, then
    disks at gaps 0.9 and 0.95 (each within one cell of the previous) drifting towards it, a
    disk 3 cells further on, and a pair 3 cells apart closing at 0.4 cells per step; k_n = 50."""
    x = [20.0, 29.99, 40.89, 51.84, 64.84, 90.0, 103.0]
    vx = [0.005, 0.0, -0.004, -0.003, -0.01, 0.2, -0.2]
    n = len(x)
    p = _particles(x, [24.0] * n, [5.0] * n, vx, [0.0] * n)
    return Case("approaching_disks", 128, 48, tau0=0.7, steps=steps, gx=1.0e-5, kn=50.0,
                particles=p)


def couette_channel(storage: str = "f64", disk: bool = True, steps: int = 400) -> Case:
    """128x48 channel between walls moving along x at -0.02 (bottom) and +0.03 (top), tau 0.8,
    no body force; optionally a fixed disk of radius 6 at (52.3, 23.6) in the shear flow."""
    p = (_particles([52.3], [23.6], [6.0], mode=MODE_FIXED) if disk else Particles.empty())
    return Case("couette_128x48", 128, 48, tau0=0.8, steps=steps, storage=storage, gx=0.0,
                uw_bot=-0.02, uw_top=0.03, particles=p)


def adjoint_channel(seed: int = 0, storage: str = "f32", v_std: float = 0.0) -> Case:
    """512x256 channel, 20 disks of diameter 20 at seeded positions (gap >= 2), tau = 0.6,
    g_x = 1e-6, 200 steps; disks move with prescribed constant velocity (zero by default)."""
    rng = np.random.default_rng(seed)
    x, y, r = place_disks(rng, 512, 256, 20, 20.0, 20.0, gap=2.0, wall_gap=2.0)
    vx = rng.normal(0.0, v_std, 20) if v_std > 0 else None
    vy = rng.normal(0.0, v_std, 20) if v_std > 0 else None
    p = _particles(x, y, r, vx, vy, mode=MODE_PRESCRIBED)
    return Case("adjoint_512x256_n20", 512, 256, tau0=0.6, steps=200, storage=storage, gx=1.0e-6,
                particles=p)


def batch_channels(seed: int = 0, count: int = 64, steps: int = 500) -> list:
    """Independent channels: width U{128, 144, ..., 1024}, height = width / 2, 1-200 disks of
    diameter U[12, 24] (count clipped so the disk area fraction stays <= 0.3), tau U[0.52, 0.8],
    FP32 storage, periodic x with walls in y, g_x = 1e-6, DEM as in the moving-disk case, no
    Smagorinsky, velocities N(0, 0.01)."""
    rng = np.random.default_rng(seed)
    cases = []
    for c in range(count):
        w = int(rng.integers(0, (1024 - 128) // 16 + 1)) * 16 + 128
        h = w // 2
        tau = float(rng.uniform(0.52, 0.8))
        n = int(rng.integers(1, 201))
        mean_area = np.pi * (6.0 ** 2 + 6.0 * 12.0 + 12.0 ** 2) / 3.0
        n = max(1, min(n, int(0.3 * w * h / mean_area)))
        x, y, r = place_disks(rng, w, h, n, 12.0, 24.0, gap=1.0, wall_gap=1.0)
        vx = rng.normal(0.0, 0.01, n)
        vy = rng.normal(0.0, 0.01, n)
        p = _particles(x, y, r, vx, vy, mode=MODE_FREE)
        cases.append(Case("channel%02d_%dx%d_n%d" % (c, w, h, n), w, h, tau0=tau, steps=steps,
                          storage="f32", gx=1.0e-6, particles=p))
    return cases


def random_populations(rng: np.random.Generator, nx: int, ny: int, base: float = 1.0 / 9.0,
                       amplitude: float = 0.05) -> np.ndarray:
    """Positive random populations [9][ny][nx] around ``base`` (relative amplitude ``amplitude``):
    a far-from-equilibrium but valid state used to exercise every term of a step."""
    return base * (1.0 + amplitude * rng.uniform(-1.0, 1.0, size=(9, ny, nx)))


def random_disks(rng: np.random.Generator, nx: int, ny: int, n: int, rmin: float, rmax: float,
                 walls: bool = True, modes=(MODE_FREE, MODE_FIXED, MODE_PRESCRIBED),
                 v_std: float = 0.01, om_std: float = 0.002, gap: float = 0.5,
                 wall_gap: float = 0.5) -> Particles:
    """n disks of random radius U[rmin, rmax] with random modes, velocities and spins."""
    x, y, r = place_disks(rng, nx, ny, n, 2 * rmin, 2 * rmax, gap=gap, wall_gap=wall_gap,
                          walls=walls)
    mode = rng.choice(np.asarray(modes, np.int32), size=n).astype(np.int32)
    return Particles(x, y, r, rng.normal(0, v_std, n), rng.normal(0, v_std, n),
                     rng.normal(0, om_std, n), mode)
