"""ctypes wrapper of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this module; the product package never does.  It imports nothing from the product
package either.  The library is compiled with gcc (``-ffp-contract=off``, OpenMP) on first use if
it is missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC3 = os.path.join(_HERE, "oracle3d.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off",
             "-fno-fast-math", "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]


def build(force: bool = False) -> str:
    """Compile liboracle.so (always when ``force``)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC3))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, _SRC3, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("walls", C.c_int32),
                ("n_sub", C.c_int32), ("tau0", C.c_double), ("cs", C.c_double),
                ("gx", C.c_double), ("gy", C.c_double), ("rho0", C.c_double),
                ("kn", C.c_double), ("zeta", C.c_double), ("rho_s", C.c_double),
                ("eps_subcells", C.c_int32), ("uw_bot", C.c_double), ("uw_top", C.c_double),
                ("kt", C.c_double), ("mu", C.c_double), ("contact_model", C.c_int32),
                ("young", C.c_double), ("poisson", C.c_double)]


class _Cfg3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls", C.c_int32),
                ("eps_subcells", C.c_int32), ("tau0", C.c_double), ("gx", C.c_double),
                ("gy", C.c_double), ("gz", C.c_double), ("rho0", C.c_double)]


_lib = None
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build())
        lib.o_create.restype = C.c_void_p
        lib.o_create.argtypes = [C.POINTER(_Cfg)]
        lib.o_destroy.argtypes = [C.c_void_p]
        lib.o_set_threads.argtypes = [C.c_int]
        lib.o_get_threads.restype = C.c_int
        lib.o_init_equilibrium.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        lib.o_set_populations.argtypes = [C.c_void_p, _D]
        lib.o_get_populations.argtypes = [C.c_void_p, _D]
        lib.o_get_fields.argtypes = [C.c_void_p, _D, _D, _D]
        lib.o_set_particles.argtypes = [C.c_void_p, C.c_int, _D, _D, _D, _D, _D, _D, _I]
        lib.o_step.argtypes = [C.c_void_p, C.c_int]
        lib.o_step_accumulate.argtypes = [C.c_void_p, C.c_int, _D, _D, _D, _D]
        lib.o_dem_steps.argtypes = [C.c_void_p, C.c_int]
        lib.o_set_loads.argtypes = [C.c_void_p, _D, _D, _D]
        lib.o_get_contacts.argtypes = [C.c_void_p, _D, _D, _D]
        lib.o_get_forces.argtypes = [C.c_void_p, _D, _D, _D]
        lib.o_force_scales.argtypes = [C.c_void_p, _D, _D]
        lib.o_get_particles.argtypes = [C.c_void_p, _D, _D, _D, _D, _D]
        lib.o_solid_field.argtypes = [C.c_void_p, _D]
        lib.o_solid_fraction.restype = C.c_double
        lib.o_solid_fraction.argtypes = [C.c_double, C.c_double, C.c_double]
        lib.o_subcell_fraction.restype = C.c_double
        lib.o_subcell_fraction.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
        lib.o_weight.restype = C.c_double
        lib.o_weight.argtypes = [C.c_double, C.c_double]
        lib.o_collide_cell.argtypes = [_D, C.c_int, _D, _D, _D, _D, _D, _D, C.c_double,
                                       C.c_double, C.c_double, C.c_double, _D, _D, _D, _D, _D,
                                       _D]
        lib.o_step_count.restype = C.c_long
        lib.o_step_count.argtypes = [C.c_void_p]
        # three-dimensional oracle (oracle3d.c)
        lib.o3_create.restype = C.c_void_p
        lib.o3_create.argtypes = [C.POINTER(_Cfg3)]
        lib.o3_destroy.argtypes = [C.c_void_p]
        lib.o3_init_equilibrium.argtypes = [C.c_void_p] + [C.c_double] * 4
        lib.o3_set_populations.argtypes = [C.c_void_p, _D]
        lib.o3_get_populations.argtypes = [C.c_void_p, _D]
        lib.o3_get_fields.argtypes = [C.c_void_p, _D, _D, _D, _D]
        lib.o3_set_spheres.argtypes = [C.c_void_p, C.c_int] + [_D] * 10 + [_I]
        lib.o3_step.argtypes = [C.c_void_p, C.c_int]
        lib.o3_get_forces.argtypes = [C.c_void_p, _D, _D]
        lib.o3_force_scales.argtypes = [C.c_void_p, _D, _D]
        lib.o3_get_spheres.argtypes = [C.c_void_p, _D, _D, _D]
        lib.o3_solid_field.argtypes = [C.c_void_p, _D]
        lib.o3_subcell_fraction.restype = C.c_double
        lib.o3_subcell_fraction.argtypes = [C.c_double] * 4 + [C.c_int]
        lib.o3_collide_cell.argtypes = [_D, C.c_int, _D, _D, _D, _D, C.c_double, C.c_double,
                                        C.c_double, C.c_double, _D, _D, _D, _D]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().o_set_threads(int(n))


def get_threads() -> int:
    return int(_load().o_get_threads())


def solid_fraction(r: float, dx: float, dy: float) -> float:
    """Exact covered fraction of the unit cell centred at (dx, dy) relative to a disk of radius r
    centred at the origin."""
    return float(_load().o_solid_fraction(r, dx, dy))


def subcell_fraction(r: float, dx: float, dy: float, n: int) -> float:
    """The paper's sub-cell estimate of the same fraction: the share of the n x n sub-cell centres
    of the unit cell centred at (dx, dy) that lie strictly inside the disk."""
    return float(_load().o_subcell_fraction(r, dx, dy, n))


def weight(eps: float, tau: float) -> float:
    """Noble-Torczynski weight B(eps, tau), Eq. (14)."""
    return float(_load().o_weight(eps, tau))


def collide_cell(f, eps=(), dx=(), dy=(), vx=(), vy=(), om=(), tau0=0.6, cs=0.0, gx=0.0, gy=0.0,
                 literal=False):
    """One-cell collision (Eqs. 1, 12-16).  Returns (f_out[9], dF[n,2], dT[n], tau_eff, B_tot),
    plus the literal nine-term force sums [n,2] when ``literal``."""
    lib = _load()
    f = _f64(f)
    n = len(eps)
    eps, dx, dy, vx, vy, om = (_f64(a) if n else np.zeros(1) for a in (eps, dx, dy, vx, vy, om))
    fout = np.zeros(9)
    dfx = np.zeros(max(n, 1)); dfy = np.zeros(max(n, 1)); dtz = np.zeros(max(n, 1))
    diag = np.zeros(2)
    lit = np.zeros(2 * max(n, 1))
    lib.o_collide_cell(_dp(f), n, _dp(eps), _dp(dx), _dp(dy), _dp(vx), _dp(vy), _dp(om),
                       tau0, cs, gx, gy, _dp(fout), _dp(dfx), _dp(dfy), _dp(dtz), _dp(diag),
                       _dp(lit))
    out = (fout, np.stack([dfx[:n], dfy[:n]], axis=1), dtz[:n].copy(), diag[0], diag[1])
    if literal:
        return out + (lit[: 2 * n].reshape(n, 2),)
    return out


@dataclass
class OracleConfig:
    nx: int
    ny: int
    tau0: float
    walls: bool = True
    cs: float = 0.0
    gx: float = 0.0
    gy: float = 0.0
    rho0: float = 1.0
    n_sub: int = 10
    kn: float = 1.0e3
    zeta: float = 0.1
    rho_s: float = 1.0
    eps_subcells: int = 0       # 0: exact solid ratio; n > 0: the paper's n x n sub-cell estimate
    uw_bot: float = 0.0         # x-velocity of the bottom wall (y = -1/2), walls only
    uw_top: float = 0.0         # x-velocity of the top wall (y = ny - 1/2), walls only
    kt: float = 0.0             # tangential contact stiffness
    mu: float = 0.0             # Coulomb friction coefficient
    contact_model: int = 0      # 0 linear spring-dashpot, 1 Hertz-Mindlin
    young: float = 0.0          # Young's modulus (Hertz-Mindlin)
    poisson: float = 0.0        # Poisson's ratio (Hertz-Mindlin)


class OracleSim:
    """One oracle simulation (FP64, CPU)."""

    def __init__(self, cfg: OracleConfig):
        lib = _load()
        self.cfg = cfg
        c = _Cfg(cfg.nx, cfg.ny, 1 if cfg.walls else 0, cfg.n_sub, cfg.tau0, cfg.cs, cfg.gx,
                 cfg.gy, cfg.rho0, cfg.kn, cfg.zeta, cfg.rho_s, cfg.eps_subcells,
                 cfg.uw_bot, cfg.uw_top, cfg.kt, cfg.mu, cfg.contact_model, cfg.young,
                 cfg.poisson)
        self._h = lib.o_create(C.byref(c))
        if not self._h:
            raise ValueError("oracle: invalid configuration %r" % (cfg,))
        self.np = 0
        lib.o_init_equilibrium(self._h, cfg.rho0, 0.0, 0.0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.o_destroy(h)
            self._h = None

    def init_equilibrium(self, rho=1.0, ux=0.0, uy=0.0):
        _load().o_init_equilibrium(self._h, rho, ux, uy)

    def set_populations(self, f):
        f = _f64(f)
        assert f.shape == (9, self.cfg.ny, self.cfg.nx)
        _load().o_set_populations(self._h, _dp(f))

    def populations(self) -> np.ndarray:
        f = np.zeros((9, self.cfg.ny, self.cfg.nx))
        _load().o_get_populations(self._h, _dp(f))
        return f

    def fields(self):
        shp = (self.cfg.ny, self.cfg.nx)
        rho, ux, uy = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        _load().o_get_fields(self._h, _dp(rho), _dp(ux), _dp(uy))
        return rho, ux, uy

    def set_particles(self, x, y, r, vx=None, vy=None, om=None, mode=None):
        n = len(x)
        z = np.zeros(n)
        x, y, r = _f64(x), _f64(y), _f64(r)
        vx = _f64(z if vx is None else vx)
        vy = _f64(z if vy is None else vy)
        om = _f64(z if om is None else om)
        mode = np.ascontiguousarray(np.zeros(n, np.int32) if mode is None else mode, np.int32)
        if n == 0:
            x = y = r = vx = vy = om = np.zeros(1)
            mode = np.zeros(1, np.int32)
        rc = _load().o_set_particles(self._h, n, _dp(x), _dp(y), _dp(r), _dp(vx), _dp(vy),
                                     _dp(om), mode.ctypes.data_as(_I))
        if rc:
            raise ValueError("oracle: invalid particles (code %d)" % rc)
        self.np = n

    def step(self, n: int = 1):
        rc = _load().o_step(self._h, int(n))
        if rc:
            raise RuntimeError("oracle: step failed (code %d)" % rc)

    def step_accumulate(self, n, wfx=None, wfy=None, wt=None, J=0.0) -> float:
        def opt(w):
            return None if w is None else _dp(_f64(w))
        keep = [None if w is None else _f64(w) for w in (wfx, wfy, wt)]
        Jc = C.c_double(J)
        rc = _load().o_step_accumulate(self._h, int(n), *(None if k is None else _dp(k) for k in keep),
                                       C.byref(Jc))
        if rc:
            raise RuntimeError("oracle: step failed (code %d)" % rc)
        return Jc.value

    def set_loads(self, fx, fy, tz):
        """Hydrodynamic force and torque held fixed by dem_steps (tests of the contact law)."""
        fx, fy, tz = _f64(fx), _f64(fy), _f64(tz)
        _load().o_set_loads(self._h, _dp(fx), _dp(fy), _dp(tz))

    def contacts(self):
        """Contact force (x, y) and torque of every disk at the last DEM evaluation."""
        n = max(self.np, 1)
        a = [np.zeros(n) for _ in range(3)]
        _load().o_get_contacts(self._h, *(_dp(v) for v in a))
        return tuple(v[: self.np] for v in a)

    def dem_steps(self, n: int = 1):
        _load().o_dem_steps(self._h, int(n))

    def forces(self):
        n = max(self.np, 1)
        fx, fy, tz = np.zeros(n), np.zeros(n), np.zeros(n)
        _load().o_get_forces(self._h, _dp(fx), _dp(fy), _dp(tz))
        return fx[: self.np], fy[: self.np], tz[: self.np]

    def force_scales(self):
        """Per disk, the conditioning scales of its force and torque sums in the last step:
        (sum over covered cells of |dF|, sum of |d| |dF|), dF the per-cell force contribution
        and d its lever arm."""
        n = max(self.np, 1)
        a = [np.zeros(n) for _ in range(2)]
        _load().o_force_scales(self._h, *(_dp(v) for v in a))
        return tuple(v[: self.np] for v in a)

    def particles(self):
        n = max(self.np, 1)
        a = [np.zeros(n) for _ in range(5)]
        _load().o_get_particles(self._h, *(_dp(v) for v in a))
        return tuple(v[: self.np] for v in a)

    def solid_field(self) -> np.ndarray:
        e = np.zeros((self.cfg.ny, self.cfg.nx))
        rc = _load().o_solid_field(self._h, _dp(e))
        if rc:
            raise RuntimeError("oracle: mapping failed (code %d)" % rc)
        return e

    @property
    def step_count(self) -> int:
        return int(_load().o_step_count(self._h))


# ----------------------------------------------------------------- D3Q19 spheres (oracle3d.c)
def subcell_fraction3(r: float, dx: float, dy: float, dz: float, n: int) -> float:
    """The paper's cell-decomposition solid ratio in 3D: the share of the n^3 sub-cell centres of
    the unit cell centred at (dx, dy, dz) strictly inside the sphere of radius r at the origin."""
    return float(_load().o3_subcell_fraction(r, dx, dy, dz, n))


def collide_cell3(f, eps=(), d=(), v=(), w=(), tau=0.6, g=(0.0, 0.0, 0.0)):
    """One D3Q19 cell (Eqs. 1, 12-16).  Returns (f_out[19], dF[n,3], dT[n,3], B_tot)."""
    lib = _load()
    f = _f64(f)
    n = len(eps)
    eps = _f64(eps) if n else np.zeros(1)
    d, v, w = ((_f64(a).reshape(-1) if n else np.zeros(3)) for a in (d, v, w))
    fout = np.zeros(19)
    dF = np.zeros(3 * max(n, 1))
    dT = np.zeros(3 * max(n, 1))
    bt = np.zeros(1)
    lib.o3_collide_cell(_dp(f), n, _dp(eps), _dp(d), _dp(v), _dp(w), tau, g[0], g[1], g[2],
                        _dp(fout), _dp(dF), _dp(dT), _dp(bt))
    return fout, dF[: 3 * n].reshape(n, 3), dT[: 3 * n].reshape(n, 3), float(bt[0])


@dataclass
class OracleConfig3:
    nx: int
    ny: int
    nz: int
    tau0: float
    walls: bool = True
    eps_subcells: int = 5       # n of the paper's n^3 sub-cell decomposition
    gx: float = 0.0
    gy: float = 0.0
    gz: float = 0.0
    rho0: float = 1.0


class OracleSim3:
    """One three-dimensional oracle simulation (D3Q19, spheres, FP64, CPU)."""

    def __init__(self, cfg: OracleConfig3):
        lib = _load()
        self.cfg = cfg
        c = _Cfg3(cfg.nx, cfg.ny, cfg.nz, 1 if cfg.walls else 0, cfg.eps_subcells, cfg.tau0,
                  cfg.gx, cfg.gy, cfg.gz, cfg.rho0)
        self._h = lib.o3_create(C.byref(c))
        if not self._h:
            raise ValueError("oracle3: invalid configuration %r" % (cfg,))
        self.np = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.o3_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (self.cfg.nz, self.cfg.ny, self.cfg.nx)

    def init_equilibrium(self, rho=1.0, ux=0.0, uy=0.0, uz=0.0):
        _load().o3_init_equilibrium(self._h, rho, ux, uy, uz)

    def set_populations(self, f):
        f = _f64(f)
        assert f.shape == (19,) + self.shape
        _load().o3_set_populations(self._h, _dp(f))

    def populations(self) -> np.ndarray:
        f = np.zeros((19,) + self.shape)
        _load().o3_get_populations(self._h, _dp(f))
        return f

    def fields(self):
        a = [np.zeros(self.shape) for _ in range(4)]
        _load().o3_get_fields(self._h, *(_dp(v) for v in a))
        return tuple(a)

    def set_spheres(self, x, y, z, r, v=None, w=None, mode=None):
        n = len(x)
        v = np.zeros((n, 3)) if v is None else np.asarray(v, float).reshape(n, 3)
        w = np.zeros((n, 3)) if w is None else np.asarray(w, float).reshape(n, 3)
        mode = np.ascontiguousarray(np.ones(n, np.int32) if mode is None else mode, np.int32)
        cols = [_f64(x), _f64(y), _f64(z), _f64(r)] + [_f64(v[:, k]) for k in range(3)] + \
               [_f64(w[:, k]) for k in range(3)]
        if n == 0:
            cols = [np.zeros(1) for _ in range(10)]
            mode = np.ones(1, np.int32)
        rc = _load().o3_set_spheres(self._h, n, *(_dp(c) for c in cols),
                                    mode.ctypes.data_as(_I))
        if rc:
            raise ValueError("oracle3: invalid spheres (code %d)" % rc)
        self.np = n

    def step(self, n: int = 1):
        rc = _load().o3_step(self._h, int(n))
        if rc:
            raise RuntimeError("oracle3: step failed (code %d)" % rc)

    def forces(self):
        """(F[n,3], T[n,3]) on each sphere in the last step."""
        m = max(self.np, 1)
        F, T = np.zeros(3 * m), np.zeros(3 * m)
        _load().o3_get_forces(self._h, _dp(F), _dp(T))
        return F[: 3 * self.np].reshape(-1, 3), T[: 3 * self.np].reshape(-1, 3)

    def force_scales(self):
        """Per sphere: (sum over covered cells of |dF|, sum of |d| |dF|) of the last step."""
        m = max(self.np, 1)
        a, b = np.zeros(m), np.zeros(m)
        _load().o3_force_scales(self._h, _dp(a), _dp(b))
        return a[: self.np], b[: self.np]

    def spheres(self):
        m = max(self.np, 1)
        a = [np.zeros(m) for _ in range(3)]
        _load().o3_get_spheres(self._h, *(_dp(v) for v in a))
        return tuple(v[: self.np] for v in a)

    def solid_field(self) -> np.ndarray:
        e = np.zeros(self.shape)
        rc = _load().o3_solid_field(self._h, _dp(e))
        if rc:
            raise RuntimeError("oracle3: mapping failed (code %d)" % rc)
        return e
