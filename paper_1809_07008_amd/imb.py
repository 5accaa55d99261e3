"""Thin ctypes binding of libimb.so (C-ABI declared in include/imb.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.  PyTorch
supplies the device memory (one uint8 workspace tensor per simulation, bound with
``imb_create``) and the stream (the current torch stream).  If the library is missing this
module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimb.so")
_HIP_LIB = LIB_PATH


def _device_buffer(nbytes: int, device):
    """The workspace tensor the library carves; the HIP library needs GPU memory (only a test
    build of the library for the host may be given host memory)."""
    import torch
    dev = torch.device(device)
    if dev.type != "cuda" and os.path.abspath(LIB_PATH) == os.path.abspath(_HIP_LIB):
        raise ValueError("libimb.so runs on the GPU: its workspace must be a cuda device tensor")
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)

STORAGE = {"f64": 0, "f32": 1, "f16": 2}
FLAG_WALLS = 1
MODE_FREE, MODE_FIXED, MODE_PRESCRIBED = 0, 1, 2
CONTACT_LINEAR, CONTACT_HERTZ_MINDLIN = 0, 1

IMB_OK = 0
IMB_BATCH_PERSISTENT = 0  # one persistent kernel per imb_batch_step call
IMB_BATCH_PER_STEP = 1    # two launches per step (lattice of all channels, particle phases)
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EOVERFLOW", -5: "EUNSTABLE", -6: "EDEM",
          -7: "EUNSUPPORTED"}

# every symbol include/imb.h declares
EXPORTED = [
    "imb_config_default", "imb_required_bytes", "imb_create", "imb_destroy",
    "imb_init_equilibrium", "imb_set_populations", "imb_get_populations", "imb_get_fields",
    "imb_set_particles", "imb_step", "imb_get_forces", "imb_get_particles", "imb_get_counts",
    "imb_sync", "imb_state_bytes", "imb_save_state", "imb_load_state", "imb_set_kernel_timing",
    "imb_get_kernel_timing", "imb_copy_kernel", "imb_adjoint", "imb_batch_required_bytes",
    "imb_batch_create", "imb_batch_destroy", "imb_batch_set_particles", "imb_batch_step",
    "imb_batch_get_forces", "imb_batch_get_particles", "imb_batch_get_fields", "imb_batch_sync",
    "imb_batch_set_launch", "imb_strerror", "imb_last_error", "imb_version",
    "imb_get_solid_field", "imb_set_graphs", "imb_get_adjoint_timing",
    "imb_batch_get_populations", "imb_batch_get_launch", "imb_batch_autotune",
    "imb_batch_get_timing", "imb_batch_last_error", "imb_batch_set_schedule",
    "imb_batch_get_schedule", "imb_prepare_graphs", "imb_adjoint_forward",
    "imb_adjoint_backward", "imb_step_noalloc",
    "imb3_config_default", "imb3_required_bytes", "imb3_create", "imb3_destroy",
    "imb3_init_equilibrium", "imb3_init_shear", "imb3_set_populations", "imb3_get_populations",
    "imb3_get_fields", "imb3_get_solid_field", "imb3_set_spheres", "imb3_step",
    "imb3_get_forces", "imb3_get_spheres", "imb3_sync", "imb3_set_kernel_timing",
    "imb3_get_kernel_timing", "imb3_last_error",
    "imb_slab_create", "imb_slab_destroy", "imb_slab_layout", "imb_slab_init_equilibrium",
    "imb_slab_set_populations", "imb_slab_get_populations", "imb_slab_get_fields",
    "imb_slab_set_particles", "imb_slab_step", "imb_slab_get_forces",
    "imb_slab_get_partial_forces", "imb_slab_get_particles", "imb_slab_set_kernel_timing",
    "imb_slab_get_kernel_timing", "imb_slab_sync", "imb_slab_last_error",
]


class ImbError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__("%s failed: %s (%d)%s" % (what, ERRORS.get(code, "?"), code,
                                                   (": " + detail) if detail else ""))


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("storage", C.c_int32),
                ("n_sub", C.c_int32), ("tau0", C.c_double), ("smag_cs", C.c_double),
                ("gx", C.c_double), ("gy", C.c_double), ("rho0", C.c_double),
                ("kn", C.c_double), ("damping_ratio", C.c_double), ("rho_solid", C.c_double),
                ("max_particles", C.c_int32), ("flags", C.c_uint32), ("tile_w", C.c_int32),
                ("tile_rows", C.c_int32), ("eps_subcells", C.c_int32), ("reserved", C.c_int32),
                ("wall_ux_bottom", C.c_double), ("wall_ux_top", C.c_double),
                ("kt", C.c_double), ("mu", C.c_double), ("contact_model", C.c_int32),
                ("reserved2", C.c_int32), ("young", C.c_double), ("poisson", C.c_double)]


class Config3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("storage", C.c_int32),
                ("tau0", C.c_double), ("gx", C.c_double), ("gy", C.c_double),
                ("gz", C.c_double), ("rho0", C.c_double), ("max_spheres", C.c_int32),
                ("eps_subcells", C.c_int32), ("flags", C.c_uint32), ("tile_w", C.c_int32),
                ("reserved", C.c_int32), ("reserved2", C.c_int32)]


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_VP = C.c_void_p


def load_library():
    """Load libimb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch must be imported first: libimb.so then binds to the HIP runtime torch already
    # loaded (same SONAME) instead of bringing a second runtime into the process
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libimb.so not found at %s: build it with "
                           "`python -m paper_1809_07008_amd.build`" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "imb_config_default": (None, [P(Config)]),
        "imb_required_bytes": (C.c_int, [P(Config), P(C.c_size_t)]),
        "imb_create": (C.c_int, [P(Config), _VP, _VP, C.c_size_t, P(_VP)]),
        "imb_destroy": (None, [_VP]),
        "imb_init_equilibrium": (C.c_int, [_VP, C.c_double, C.c_double, C.c_double]),
        "imb_set_populations": (C.c_int, [_VP, _D]),
        "imb_get_populations": (C.c_int, [_VP, _D]),
        "imb_get_fields": (C.c_int, [_VP, _D, _D, _D]),
        "imb_get_solid_field": (C.c_int, [_VP, _D]),
        "imb_set_particles": (C.c_int, [_VP, C.c_int32, _D, _D, _D, _D, _D, _D, _I32]),
        "imb_step": (C.c_int, [_VP, C.c_int32]),
        "imb_step_noalloc": (C.c_int, [_VP, C.c_int32]),
        "imb_set_graphs": (C.c_int, [_VP, C.c_int]),
        "imb_prepare_graphs": (C.c_int, [_VP]),
        "imb_get_forces": (C.c_int, [_VP, _D, _D, _D]),
        "imb_get_particles": (C.c_int, [_VP, _D, _D, _D, _D, _D]),
        "imb_get_counts": (C.c_int, [_VP, _I32, P(C.c_int64)]),
        "imb_sync": (C.c_int, [_VP]),
        "imb_state_bytes": (C.c_int, [_VP, P(C.c_size_t)]),
        "imb_save_state": (C.c_int, [_VP, _VP, C.c_size_t]),
        "imb_load_state": (C.c_int, [_VP, _VP, C.c_size_t]),
        "imb_set_kernel_timing": (C.c_int, [_VP, C.c_int]),
        "imb_get_kernel_timing": (C.c_int, [_VP, _D, P(C.c_int64), _D, P(C.c_int64)]),
        "imb_copy_kernel": (C.c_int, [_VP, _VP, C.c_size_t, _VP]),
        "imb_adjoint": (C.c_int, [_VP, C.c_int32, C.c_int32, _D, _D, _D, _D, _D, _D, _D, _D,
                                  _D, _D, _D]),
        "imb_adjoint_forward": (C.c_int, [_VP, C.c_int32, C.c_int32, _D, _D, _D, _D]),
        "imb_adjoint_backward": (C.c_int, [_VP, _D, _D, _D, _D, _D, _D, _D]),
        "imb_get_adjoint_timing": (C.c_int, [_VP, _D, _D, _D, P(C.c_int64), _D,
                                             P(C.c_int64)]),
        "imb_batch_required_bytes": (C.c_int, [C.c_int32, P(Config), P(C.c_size_t)]),
        "imb_batch_create": (C.c_int, [C.c_int32, P(Config), _VP, _VP, C.c_size_t, P(_VP)]),
        "imb_batch_destroy": (None, [_VP]),
        "imb_batch_set_particles": (C.c_int, [_VP, C.c_int32, C.c_int32, _D, _D, _D, _D, _D, _D,
                                              _I32]),
        "imb_batch_step": (C.c_int, [_VP, C.c_int32]),
        "imb_batch_get_forces": (C.c_int, [_VP, C.c_int32, _D, _D, _D]),
        "imb_batch_get_particles": (C.c_int, [_VP, C.c_int32, _D, _D, _D, _D, _D]),
        "imb_batch_get_fields": (C.c_int, [_VP, C.c_int32, _D, _D, _D]),
        "imb_batch_sync": (C.c_int, [_VP]),
        "imb_batch_set_launch": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32]),
        "imb_batch_get_populations": (C.c_int, [_VP, C.c_int32, _D]),
        "imb_batch_get_launch": (C.c_int, [_VP, _I32, _I32, _I32, _I32]),
        "imb_batch_autotune": (C.c_int, [_VP, C.c_int32, _D, C.c_int32]),
        "imb_batch_get_timing": (C.c_int, [_VP, C.c_int32, _D]),
        "imb_batch_last_error": (C.c_char_p, [_VP]),
        "imb_batch_set_schedule": (C.c_int, [_VP, C.c_int32]),
        "imb_batch_get_schedule": (C.c_int, [_VP, _I32]),
        "imb3_config_default": (None, [P(Config3)]),
        "imb3_required_bytes": (C.c_int, [P(Config3), P(C.c_size_t)]),
        "imb3_create": (C.c_int, [P(Config3), _VP, _VP, C.c_size_t, P(_VP)]),
        "imb3_destroy": (None, [_VP]),
        "imb3_init_equilibrium": (C.c_int, [_VP, C.c_double, C.c_double, C.c_double,
                                            C.c_double]),
        "imb3_init_shear": (C.c_int, [_VP, C.c_double, _D]),
        "imb3_set_populations": (C.c_int, [_VP, _D]),
        "imb3_get_populations": (C.c_int, [_VP, _D]),
        "imb3_get_fields": (C.c_int, [_VP, _D, _D, _D, _D]),
        "imb3_get_solid_field": (C.c_int, [_VP, _D]),
        "imb3_set_spheres": (C.c_int, [_VP, C.c_int32] + [_D] * 10 + [_I32]),
        "imb3_step": (C.c_int, [_VP, C.c_int32]),
        "imb3_get_forces": (C.c_int, [_VP, _D, _D]),
        "imb3_get_spheres": (C.c_int, [_VP, _D]),
        "imb3_sync": (C.c_int, [_VP]),
        "imb3_set_kernel_timing": (C.c_int, [_VP, C.c_int]),
        "imb3_get_kernel_timing": (C.c_int, [_VP, _D, P(C.c_int64), _D, P(C.c_int64)]),
        "imb3_last_error": (C.c_char_p, [_VP]),
        "imb_slab_create": (C.c_int, [P(Config), C.c_int32, _VP, P(_VP)]),
        "imb_slab_destroy": (None, [_VP]),
        "imb_slab_layout": (C.c_int, [_VP, _I32, _I32]),
        "imb_slab_init_equilibrium": (C.c_int, [_VP, C.c_double, C.c_double, C.c_double]),
        "imb_slab_set_populations": (C.c_int, [_VP, _D]),
        "imb_slab_get_populations": (C.c_int, [_VP, _D]),
        "imb_slab_get_fields": (C.c_int, [_VP, _D, _D, _D]),
        "imb_slab_set_particles": (C.c_int, [_VP, C.c_int32, _D, _D, _D, _D, _D, _D, _I32]),
        "imb_slab_step": (C.c_int, [_VP, C.c_int32]),
        "imb_slab_get_forces": (C.c_int, [_VP, _D, _D, _D]),
        "imb_slab_get_partial_forces": (C.c_int, [_VP, C.c_int32, _D, _D, _D]),
        "imb_slab_get_particles": (C.c_int, [_VP, C.c_int32, _D, _D, _D, _D, _D]),
        "imb_slab_set_kernel_timing": (C.c_int, [_VP, C.c_int]),
        "imb_slab_get_kernel_timing": (C.c_int, [_VP, _D, _D, _D, P(C.c_int64)]),
        "imb_slab_sync": (C.c_int, [_VP]),
        "imb_slab_last_error": (C.c_char_p, [_VP]),
        "imb_strerror": (C.c_char_p, [C.c_int]),
        "imb_last_error": (C.c_char_p, [_VP]),
        "imb_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a, n=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape != (n,):
        raise ValueError("expected %d values, got shape %s" % (n, a.shape))
    return a


def make_config(nx, ny, tau0, storage="f64", walls=True, cs=0.0, gx=0.0, gy=0.0, rho0=1.0,
                n_sub=10, kn=1.0e3, zeta=0.1, rho_s=1.0, max_particles=64, tile_w=64,
                tile_rows=1, eps_subcells=0, uw_bot=0.0, uw_top=0.0, kt=0.0, mu=0.0,
                contact_model=0, young=0.0, poisson=0.0) -> Config:
    c = Config()
    load_library().imb_config_default(C.byref(c))
    c.nx, c.ny, c.tau0 = int(nx), int(ny), float(tau0)
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.smag_cs, c.gx, c.gy, c.rho0 = float(cs), float(gx), float(gy), float(rho0)
    c.n_sub, c.kn, c.damping_ratio, c.rho_solid = int(n_sub), float(kn), float(zeta), float(rho_s)
    c.max_particles = int(max_particles)
    c.flags = FLAG_WALLS if walls else 0
    c.tile_w, c.tile_rows = int(tile_w), int(tile_rows)
    c.eps_subcells = int(eps_subcells)
    c.wall_ux_bottom, c.wall_ux_top = float(uw_bot), float(uw_top)
    c.kt, c.mu = float(kt), float(mu)
    c.contact_model = int(contact_model)
    c.young, c.poisson = float(young), float(poisson)
    return c


def config_from_case(case, max_particles=None, tile_w=64, tile_rows=1, storage=None) -> Config:
    """Config of a :class:`paper_1809_07008_amd.workloads.Case`."""
    n = case.particles.n
    return make_config(case.nx, case.ny, case.tau0, storage or case.storage, case.walls, case.cs,
                       case.gx, case.gy, case.rho0, case.n_sub, case.kn, case.zeta, case.rho_s,
                       max(n, 1) if max_particles is None else max_particles, tile_w, tile_rows,
                       case.eps_subcells, case.uw_bot, case.uw_top, case.kt, case.mu,
                       case.contact_model, case.young, case.poisson)


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Simulation:
    """One simulation; device memory is a torch uint8 tensor owned by this object."""

    def __init__(self, cfg: Config, stream=None, device="cuda"):
        import torch
        lib = load_library()
        self.cfg = cfg
        nbytes = C.c_size_t()
        self._check(lib.imb_required_bytes(C.byref(cfg), C.byref(nbytes)), "imb_required_bytes",
                    handle=False)
        self._buf = _device_buffer(nbytes.value + 256, device)
        ptr = self._buf.data_ptr()
        off = (-ptr) % 256
        self._stream = stream
        h = C.c_void_p()
        self._check(lib.imb_create(C.byref(cfg), _stream_handle(stream), C.c_void_p(ptr + off),
                                   nbytes.value, C.byref(h)), "imb_create", handle=False)
        self._h = h
        self.n = 0

    def _check(self, rc, what, handle=True):
        if rc != IMB_OK:
            lib = load_library()
            msg = lib.imb_last_error(self._h if handle else None)
            raise ImbError(rc, what, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            load_library().imb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.cfg.ny, self.cfg.nx)

    def init_equilibrium(self, rho=1.0, ux=0.0, uy=0.0):
        self._check(load_library().imb_init_equilibrium(self._h, rho, ux, uy),
                    "imb_init_equilibrium")

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (9, self.cfg.ny, self.cfg.nx):
            raise ValueError("populations must have shape (9, ny, nx)")
        self._check(load_library().imb_set_populations(self._h, _dp(f)), "imb_set_populations")

    def populations(self) -> np.ndarray:
        f = np.empty((9, self.cfg.ny, self.cfg.nx))
        self._check(load_library().imb_get_populations(self._h, _dp(f)), "imb_get_populations")
        return f

    def fields(self):
        rho, ux, uy = (np.empty(self.shape) for _ in range(3))
        self._check(load_library().imb_get_fields(self._h, _dp(rho), _dp(ux), _dp(uy)),
                    "imb_get_fields")
        return rho, ux, uy

    def solid_field(self) -> np.ndarray:
        e = np.empty(self.shape)
        self._check(load_library().imb_get_solid_field(self._h, _dp(e)), "imb_get_solid_field")
        return e

    def set_particles(self, x, y, r, vx=None, vy=None, om=None, mode=None):
        n = len(x)
        z = np.zeros(n)
        arrs = [_f64(a, n) for a in (x, y, r, z if vx is None else vx, z if vy is None else vy,
                                      z if om is None else om)]
        md = np.ascontiguousarray(np.zeros(n, np.int32) if mode is None else mode, np.int32)
        if n == 0:
            arrs = [np.zeros(1) for _ in range(6)]
            md = np.zeros(1, np.int32)
        self._check(load_library().imb_set_particles(self._h, n, *(_dp(a) for a in arrs),
                                                     md.ctypes.data_as(_I32)),
                    "imb_set_particles")
        self.n = n

    def set_case_particles(self, p):
        self.set_particles(p.x, p.y, p.r, p.vx, p.vy, p.om, p.mode)

    def step(self, n: int = 1):
        self._check(load_library().imb_step(self._h, int(n)), "imb_step")

    def step_noalloc(self, n: int = 1):
        """imb_step_noalloc: the same steps, launched directly, with no allocation."""
        self._check(load_library().imb_step_noalloc(self._h, int(n)), "imb_step_noalloc")

    def forces(self):
        m = max(self.n, 1)
        fx, fy, tz = np.zeros(m), np.zeros(m), np.zeros(m)
        self._check(load_library().imb_get_forces(self._h, _dp(fx), _dp(fy), _dp(tz)),
                    "imb_get_forces")
        return fx[: self.n], fy[: self.n], tz[: self.n]

    def particles(self):
        m = max(self.n, 1)
        a = [np.zeros(m) for _ in range(5)]
        self._check(load_library().imb_get_particles(self._h, *(_dp(v) for v in a)),
                    "imb_get_particles")
        return tuple(v[: self.n] for v in a)

    def counts(self):
        n = C.c_int32()
        s = C.c_int64()
        self._check(load_library().imb_get_counts(self._h, C.byref(n), C.byref(s)),
                    "imb_get_counts")
        return n.value, s.value

    def sync(self):
        self._check(load_library().imb_sync(self._h), "imb_sync")

    def save_state(self) -> bytes:
        lib = load_library()
        nb = C.c_size_t()
        self._check(lib.imb_state_bytes(self._h, C.byref(nb)), "imb_state_bytes")
        buf = C.create_string_buffer(nb.value)
        self._check(lib.imb_save_state(self._h, buf, nb.value), "imb_save_state")
        return buf.raw

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(load_library().imb_load_state(self._h, buf, len(data)), "imb_load_state")
        n = C.c_int32()
        load_library().imb_get_counts(self._h, C.byref(n), None)
        self.n = n.value

    def set_graphs(self, on: bool):
        self._check(load_library().imb_set_graphs(self._h, 1 if on else 0), "imb_set_graphs")

    def prepare_graphs(self):
        """Captures and uploads every step graph imb_step may replay (imb_prepare_graphs)."""
        self._check(load_library().imb_prepare_graphs(self._h), "imb_prepare_graphs")

    def set_kernel_timing(self, on: bool):
        self._check(load_library().imb_set_kernel_timing(self._h, 1 if on else 0),
                    "imb_set_kernel_timing")

    def kernel_timing(self):
        """Summed milliseconds and launch counts of the lattice kernel and the particle phase
        since set_kernel_timing(True) (HIP events around every launch on the simulation's
        stream)."""
        lm, pm = C.c_double(), C.c_double()
        ln, pn = C.c_int64(), C.c_int64()
        self._check(load_library().imb_get_kernel_timing(self._h, C.byref(lm), C.byref(ln),
                                                         C.byref(pm), C.byref(pn)),
                    "imb_get_kernel_timing")
        return {"lattice_ms": lm.value, "lattice_launches": ln.value,
                "particle_ms": pm.value, "particle_launches": pn.value}

    def adjoint(self, nsteps: int, k_ckpt: int, wfx=None, wfy=None, wtz=None,
                populations: bool = False):
        """Discrete adjoint of ``nsteps`` coupled steps from the current state (imb_adjoint).

        J = sum over steps and disks of wfx Fx + wfy Fy + wtz Tz.  Returns a dict with J and the
        gradients x0, y0, vx, vy, om (per disk), g (dJ/dg_x, dJ/dg_y) and, when ``populations``,
        f0 = dJ/d(post-stream populations at the start) as [9, ny, nx].  The simulation advances
        by nsteps."""
        n = self.n
        m = max(n, 1)
        w = [None if a is None else _f64(a, n) for a in (wfx, wfy, wtz)]
        outs = [np.zeros(m) for _ in range(5)]
        gg = np.zeros(2)
        J = np.zeros(1)
        gf0 = np.zeros((9, self.cfg.ny, self.cfg.nx)) if populations else None
        self._check(load_library().imb_adjoint(self._h, int(nsteps), int(k_ckpt),
                                               *(_dp(a) for a in w), *(_dp(o) for o in outs),
                                               _dp(gg), _dp(J), _dp(gf0)), "imb_adjoint")
        names = ["x0", "y0", "vx", "vy", "om"]
        res = {k: v[:n] for k, v in zip(names, outs)}
        res["g"] = gg
        res["J"] = float(J[0])
        if populations:
            res["f0"] = gf0
        return res

    def adjoint_forward(self, nsteps: int, k_ckpt: int, wfx=None, wfy=None, wtz=None) -> float:
        """Forward pass of a differentiated run (imb_adjoint_forward): advances nsteps keeping
        the checkpoints, returns J and arms one reverse sweep."""
        n = self.n
        w = [None if a is None else _f64(a, n) for a in (wfx, wfy, wtz)]
        J = np.zeros(1)
        self._check(load_library().imb_adjoint_forward(self._h, int(nsteps), int(k_ckpt),
                                                       *(_dp(a) for a in w), _dp(J)),
                    "imb_adjoint_forward")
        return float(J[0])

    def adjoint_backward(self, populations: bool = False):
        """Reverse sweep of the armed forward pass (imb_adjoint_backward): the gradients as
        :meth:`adjoint` returns them, without J."""
        m = max(self.n, 1)
        outs = [np.zeros(m) for _ in range(5)]
        gg = np.zeros(2)
        gf0 = np.zeros((9, self.cfg.ny, self.cfg.nx)) if populations else None
        self._check(load_library().imb_adjoint_backward(self._h, *(_dp(o) for o in outs),
                                                        _dp(gg), _dp(gf0)),
                    "imb_adjoint_backward")
        res = {k: v[: self.n] for k, v in zip(["x0", "y0", "vx", "vy", "om"], outs)}
        res["g"] = gg
        if populations:
            res["f0"] = gf0
        return res

    def adjoint_timing(self):
        """GPU milliseconds of the last adjoint call (forward pass, reverse sweep) and, with
        kernel timing on, the summed adjoint-step and recompute kernel times and counts."""
        f, r, a, rc = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        an, rn = C.c_int64(), C.c_int64()
        self._check(load_library().imb_get_adjoint_timing(self._h, C.byref(f), C.byref(r),
                                                          C.byref(a), C.byref(an),
                                                          C.byref(rc), C.byref(rn)),
                    "imb_get_adjoint_timing")
        return {"forward_ms": f.value, "reverse_ms": r.value, "adjoint_kernel_ms": a.value,
                "adjoint_kernels": an.value, "recompute_kernel_ms": rc.value,
                "recompute_kernels": rn.value}


def copy_kernel(dst_ptr: int, src_ptr: int, nbytes: int, stream=None) -> None:
    rc = load_library().imb_copy_kernel(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), int(nbytes),
                                        _stream_handle(stream))
    if rc != IMB_OK:
        raise ImbError(rc, "imb_copy_kernel")


def simulation_from_case(case, storage=None, tile_w=64, tile_rows=1, max_particles=None,
                         stream=None) -> Simulation:
    """Simulation of a workload case, particles uploaded, fluid at rest."""
    sim = Simulation(config_from_case(case, max_particles, tile_w, tile_rows, storage), stream)
    sim.set_case_particles(case.particles)
    return sim


class Batch:
    """Independent channels advanced together (imb_batch_*): one persistent kernel per step
    call, or two launches per step (the per-step schedule, the only one for a batch holding a
    channel of more than 256 disks).  Device memory is a torch uint8 tensor owned by this
    object."""

    def __init__(self, cfgs, stream=None, device="cuda"):
        import torch
        lib = load_library()
        self.cfgs = list(cfgs)
        arr = (Config * len(self.cfgs))(*self.cfgs)
        self._arr = arr
        nbytes = C.c_size_t()
        self._h = None
        self._check(lib.imb_batch_required_bytes(len(self.cfgs), arr, C.byref(nbytes)),
                    "imb_batch_required_bytes", handle=False)
        self._buf = _device_buffer(nbytes.value + 256, device)
        ptr = self._buf.data_ptr()
        off = (-ptr) % 256
        h = C.c_void_p()
        self._check(lib.imb_batch_create(len(self.cfgs), arr, _stream_handle(stream),
                                         C.c_void_p(ptr + off), nbytes.value, C.byref(h)),
                    "imb_batch_create", handle=False)
        self._h = h
        self.n = [0] * len(self.cfgs)

    def _check(self, rc, what, handle=True):
        if rc != IMB_OK:
            msg = load_library().imb_batch_last_error(self._h if handle else None)
            raise ImbError(rc, what, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            load_library().imb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.cfgs)

    def set_particles(self, sim, x, y, r, vx=None, vy=None, om=None, mode=None):
        n = len(x)
        z = np.zeros(n)
        arrs = [_f64(a, n) for a in (x, y, r, z if vx is None else vx, z if vy is None else vy,
                                      z if om is None else om)]
        md = np.ascontiguousarray(np.zeros(n, np.int32) if mode is None else mode, np.int32)
        if n == 0:
            arrs = [np.zeros(1) for _ in range(6)]
            md = np.zeros(1, np.int32)
        self._check(load_library().imb_batch_set_particles(
            self._h, int(sim), n, *(_dp(a) for a in arrs), md.ctypes.data_as(_I32)),
            "imb_batch_set_particles")
        self.n[sim] = n

    def set_case_particles(self, sim, p):
        self.set_particles(sim, p.x, p.y, p.r, p.vx, p.vy, p.om, p.mode)

    def step(self, n: int = 1):
        self._check(load_library().imb_batch_step(self._h, int(n)), "imb_batch_step")

    def sync(self):
        self._check(load_library().imb_batch_sync(self._h), "imb_batch_sync")

    def forces(self, sim):
        m = max(self.n[sim], 1)
        a = [np.zeros(m) for _ in range(3)]
        self._check(load_library().imb_batch_get_forces(self._h, int(sim), *(_dp(v) for v in a)),
                    "imb_batch_get_forces")
        return tuple(v[: self.n[sim]] for v in a)

    def particles(self, sim):
        m = max(self.n[sim], 1)
        a = [np.zeros(m) for _ in range(5)]
        self._check(load_library().imb_batch_get_particles(self._h, int(sim),
                                                           *(_dp(v) for v in a)),
                    "imb_batch_get_particles")
        return tuple(v[: self.n[sim]] for v in a)

    def fields(self, sim):
        c = self.cfgs[sim]
        a = [np.zeros((c.ny, c.nx)) for _ in range(3)]
        self._check(load_library().imb_batch_get_fields(self._h, int(sim), *(_dp(v) for v in a)),
                    "imb_batch_get_fields")
        return tuple(a)

    def populations(self, sim):
        c = self.cfgs[sim]
        f = np.zeros((9, c.ny, c.nx))
        self._check(load_library().imb_batch_get_populations(self._h, int(sim), _dp(f)),
                    "imb_batch_get_populations")
        return f

    def set_launch(self, grid=0, tile_w=0, tile_rows=0):
        self._check(load_library().imb_batch_set_launch(self._h, int(grid), int(tile_w),
                                                        int(tile_rows)), "imb_batch_set_launch")

    def set_schedule(self, schedule: int):
        self._check(load_library().imb_batch_set_schedule(self._h, int(schedule)),
                    "imb_batch_set_schedule")

    def launch(self):
        v = [C.c_int32() for _ in range(5)]
        lib = load_library()
        self._check(lib.imb_batch_get_launch(self._h, *(C.byref(x) for x in v[:4])),
                    "imb_batch_get_launch")
        self._check(lib.imb_batch_get_schedule(self._h, C.byref(v[4])), "imb_batch_get_schedule")
        return {"grid": v[0].value, "tile_w": v[1].value, "tile_rows": v[2].value,
                "max_grid": v[3].value,
                "schedule": "per_step" if v[4].value == IMB_BATCH_PER_STEP else "persistent"}

    def autotune(self, trial_steps: int = 5, max_trials: int = 0) -> float:
        """Runs the library's autotuner; returns the best time per step (ms)."""
        ms = C.c_double()
        self._check(load_library().imb_batch_autotune(self._h, int(trial_steps), C.byref(ms),
                                                      int(max_trials)), "imb_batch_autotune")
        return ms.value

    def timed_steps(self, n: int) -> float:
        """Runs n steps as one graph replay; returns the GPU milliseconds (HIP events)."""
        ms = C.c_double()
        self._check(load_library().imb_batch_get_timing(self._h, int(n), C.byref(ms)),
                    "imb_batch_get_timing")
        return ms.value


def batch_from_cases(cases, tile_w=32, tile_rows=2, stream=None) -> Batch:
    """Batch of workload cases (F32 storage), particles uploaded, fluid at rest."""
    cfgs = [config_from_case(c, None, tile_w, tile_rows, "f32") for c in cases]
    b = Batch(cfgs, stream)
    for k, c in enumerate(cases):
        b.set_case_particles(k, c.particles)
    return b


# ------------------------------------------------------- one GPU's share of a split lattice
class Slabs:
    """The lattice of ``cfg`` split in y into ``nslabs`` slabs (imb_slab_*): each slab stores its
    rows and exchanges its faces with its neighbours; the library allocates the memory on the
    current device."""

    def __init__(self, cfg: Config, nslabs: int, stream=None):
        lib = load_library()
        self.cfg = cfg
        self.nslabs = int(nslabs)
        self._h = None
        h = C.c_void_p()
        self._check(lib.imb_slab_create(C.byref(cfg), self.nslabs, _stream_handle(stream),
                                        C.byref(h)), "imb_slab_create", handle=False)
        self._h = h
        self.n = 0

    def _check(self, rc, what, handle=True):
        if rc != IMB_OK:
            msg = load_library().imb_slab_last_error(self._h if handle else None)
            raise ImbError(rc, what, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            load_library().imb_slab_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.cfg.ny, self.cfg.nx)

    def layout(self):
        """(first row, row count) of each slab."""
        y0 = np.zeros(self.nslabs, np.int32)
        rows = np.zeros(self.nslabs, np.int32)
        self._check(load_library().imb_slab_layout(self._h, y0.ctypes.data_as(_I32),
                                                   rows.ctypes.data_as(_I32)), "imb_slab_layout")
        return y0, rows

    def init_equilibrium(self, rho=1.0, ux=0.0, uy=0.0):
        self._check(load_library().imb_slab_init_equilibrium(self._h, rho, ux, uy),
                    "imb_slab_init_equilibrium")

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (9, self.cfg.ny, self.cfg.nx):
            raise ValueError("populations must have shape (9, ny, nx)")
        self._check(load_library().imb_slab_set_populations(self._h, _dp(f)),
                    "imb_slab_set_populations")

    def populations(self) -> np.ndarray:
        f = np.empty((9, self.cfg.ny, self.cfg.nx))
        self._check(load_library().imb_slab_get_populations(self._h, _dp(f)),
                    "imb_slab_get_populations")
        return f

    def fields(self):
        rho, ux, uy = (np.empty(self.shape) for _ in range(3))
        self._check(load_library().imb_slab_get_fields(self._h, _dp(rho), _dp(ux), _dp(uy)),
                    "imb_slab_get_fields")
        return rho, ux, uy

    def set_particles(self, x, y, r, vx=None, vy=None, om=None, mode=None):
        n = len(x)
        z = np.zeros(n)
        arrs = [_f64(a, n) for a in (x, y, r, z if vx is None else vx, z if vy is None else vy,
                                      z if om is None else om)]
        md = np.ascontiguousarray(np.zeros(n, np.int32) if mode is None else mode, np.int32)
        if n == 0:
            arrs = [np.zeros(1) for _ in range(6)]
            md = np.zeros(1, np.int32)
        self._check(load_library().imb_slab_set_particles(self._h, n, *(_dp(a) for a in arrs),
                                                          md.ctypes.data_as(_I32)),
                    "imb_slab_set_particles")
        self.n = n

    def set_case_particles(self, p):
        self.set_particles(p.x, p.y, p.r, p.vx, p.vy, p.om, p.mode)

    def step(self, n: int = 1):
        self._check(load_library().imb_slab_step(self._h, int(n)), "imb_slab_step")

    def forces(self):
        m = max(self.n, 1)
        fx, fy, tz = np.zeros(m), np.zeros(m), np.zeros(m)
        self._check(load_library().imb_slab_get_forces(self._h, _dp(fx), _dp(fy), _dp(tz)),
                    "imb_slab_get_forces")
        return fx[:self.n], fy[:self.n], tz[:self.n]

    def partial_forces(self, slab: int):
        m = max(self.n, 1)
        fx, fy, tz = np.zeros(m), np.zeros(m), np.zeros(m)
        self._check(load_library().imb_slab_get_partial_forces(self._h, int(slab), _dp(fx),
                                                               _dp(fy), _dp(tz)),
                    "imb_slab_get_partial_forces")
        return fx[:self.n], fy[:self.n], tz[:self.n]

    def particles(self, slab: int = 0):
        m = max(self.n, 1)
        a = [np.zeros(m) for _ in range(5)]
        self._check(load_library().imb_slab_get_particles(self._h, int(slab),
                                                          *(_dp(v) for v in a)),
                    "imb_slab_get_particles")
        return tuple(v[:self.n] for v in a)

    def set_kernel_timing(self, enable: bool):
        self._check(load_library().imb_slab_set_kernel_timing(self._h, int(bool(enable))),
                    "imb_slab_set_kernel_timing")

    def kernel_timing(self):
        """(lattice ms per slab, exchange ms, particle-phase ms per slab, timed steps)."""
        lat = np.zeros(self.nslabs)
        par = np.zeros(self.nslabs)
        xch = C.c_double()
        n = C.c_int64()
        self._check(load_library().imb_slab_get_kernel_timing(self._h, _dp(lat), C.byref(xch),
                                                              _dp(par), C.byref(n)),
                    "imb_slab_get_kernel_timing")
        return lat, xch.value, par, n.value

    def sync(self):
        self._check(load_library().imb_slab_sync(self._h), "imb_slab_sync")


def slabs_from_case(case, nslabs, storage=None, tile_w=64, tile_rows=1, stream=None) -> Slabs:
    """Slabs of a workload case, particles uploaded, fluid at rest."""
    s = Slabs(config_from_case(case, None, tile_w, tile_rows, storage), nslabs, stream)
    s.set_case_particles(case.particles)
    return s


# ------------------------------------------------------- three dimensions: D3Q19 with spheres
def make_config3(nx, ny, nz, tau0, storage="f64", walls=True, g=(0.0, 0.0, 0.0), rho0=1.0,
                 max_spheres=8, eps_subcells=5, tile_w=0) -> Config3:
    c = Config3()
    load_library().imb3_config_default(C.byref(c))
    c.nx, c.ny, c.nz, c.tau0 = int(nx), int(ny), int(nz), float(tau0)
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.gx, c.gy, c.gz = (float(v) for v in g)
    c.rho0 = float(rho0)
    c.max_spheres = int(max_spheres)
    c.eps_subcells = int(eps_subcells)
    c.flags = FLAG_WALLS if walls else 0
    c.tile_w = int(tile_w)
    return c


class Simulation3:
    """One D3Q19 simulation with spheres (imb3_*); device memory is a torch uint8 tensor."""

    def __init__(self, cfg: Config3, stream=None, device="cuda"):
        lib = load_library()
        self.cfg = cfg
        self._h = None
        nbytes = C.c_size_t()
        self._check(lib.imb3_required_bytes(C.byref(cfg), C.byref(nbytes)),
                    "imb3_required_bytes", handle=False)
        self._buf = _device_buffer(nbytes.value + 256, device)
        ptr = self._buf.data_ptr()
        off = (-ptr) % 256
        h = C.c_void_p()
        self._check(lib.imb3_create(C.byref(cfg), _stream_handle(stream), C.c_void_p(ptr + off),
                                    nbytes.value, C.byref(h)), "imb3_create", handle=False)
        self._h = h
        self.n = 0

    def _check(self, rc, what, handle=True):
        if rc != IMB_OK:
            msg = load_library().imb3_last_error(self._h if handle else None)
            raise ImbError(rc, what, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            load_library().imb3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.cfg.nz, self.cfg.ny, self.cfg.nx)

    def init_equilibrium(self, rho=1.0, ux=0.0, uy=0.0, uz=0.0):
        self._check(load_library().imb3_init_equilibrium(self._h, rho, ux, uy, uz),
                    "imb3_init_equilibrium")

    def init_shear(self, ux_of_y, rho=1.0):
        u = _f64(ux_of_y, self.cfg.ny)
        self._check(load_library().imb3_init_shear(self._h, rho, _dp(u)), "imb3_init_shear")

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (19,) + self.shape:
            raise ValueError("populations must have shape (19, nz, ny, nx)")
        self._check(load_library().imb3_set_populations(self._h, _dp(f)), "imb3_set_populations")

    def populations(self) -> np.ndarray:
        f = np.empty((19,) + self.shape)
        self._check(load_library().imb3_get_populations(self._h, _dp(f)), "imb3_get_populations")
        return f

    def fields(self):
        a = [np.empty(self.shape) for _ in range(4)]
        self._check(load_library().imb3_get_fields(self._h, *(_dp(v) for v in a)),
                    "imb3_get_fields")
        return tuple(a)

    def solid_field(self) -> np.ndarray:
        e = np.empty(self.shape)
        self._check(load_library().imb3_get_solid_field(self._h, _dp(e)), "imb3_get_solid_field")
        return e

    def set_spheres(self, x, y, z, r, v=None, w=None, mode=None):
        n = len(x)
        v = np.zeros((n, 3)) if v is None else np.asarray(v, float).reshape(n, 3)
        w = np.zeros((n, 3)) if w is None else np.asarray(w, float).reshape(n, 3)
        cols = [_f64(x, n), _f64(y, n), _f64(z, n), _f64(r, n)] + \
               [_f64(v[:, k], n) for k in range(3)] + [_f64(w[:, k], n) for k in range(3)]
        md = np.ascontiguousarray(np.full(n, MODE_FIXED, np.int32) if mode is None else mode,
                                  np.int32)
        if n == 0:
            cols = [np.zeros(1) for _ in range(10)]
            md = np.ones(1, np.int32)
        self._check(load_library().imb3_set_spheres(self._h, n, *(_dp(c) for c in cols),
                                                    md.ctypes.data_as(_I32)), "imb3_set_spheres")
        self.n = n

    def step(self, n: int = 1):
        self._check(load_library().imb3_step(self._h, int(n)), "imb3_step")

    def sync(self):
        self._check(load_library().imb3_sync(self._h), "imb3_sync")

    def forces(self):
        """(F[n,3], T[n,3]) on each sphere in the last step."""
        m = max(self.n, 1)
        F, T = np.zeros(3 * m), np.zeros(3 * m)
        self._check(load_library().imb3_get_forces(self._h, _dp(F), _dp(T)), "imb3_get_forces")
        return F[: 3 * self.n].reshape(-1, 3), T[: 3 * self.n].reshape(-1, 3)

    def spheres(self) -> np.ndarray:
        a = np.zeros(4 * max(self.n, 1))
        self._check(load_library().imb3_get_spheres(self._h, _dp(a)), "imb3_get_spheres")
        return a[: 4 * self.n].reshape(-1, 4)

    def set_kernel_timing(self, on: bool):
        self._check(load_library().imb3_set_kernel_timing(self._h, 1 if on else 0),
                    "imb3_set_kernel_timing")

    def kernel_timing(self):
        lm, fm = C.c_double(), C.c_double()
        ln, fn = C.c_int64(), C.c_int64()
        self._check(load_library().imb3_get_kernel_timing(self._h, C.byref(lm), C.byref(ln),
                                                          C.byref(fm), C.byref(fn)),
                    "imb3_get_kernel_timing")
        return {"lattice_ms": lm.value, "lattice_launches": ln.value,
                "finalize_ms": fm.value, "finalize_launches": fn.value}
