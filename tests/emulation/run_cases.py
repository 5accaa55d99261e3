"""Cases run against the CPU emulation of libimb (test infrastructure; run by
tests/test_cpu_emulation.py in a subprocess with AddressSanitizer preloaded).  Each case compares
the emulated kernels with the FP64 oracle or with another path of the library and exits non-zero
on a mismatch; AddressSanitizer aborts the process on any out-of-bounds access."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

import numpy as np  # noqa: E402

from adjoint_fd import block_errors, fd_gradient  # noqa: E402
from oracle import OracleConfig, OracleSim  # noqa: E402
from paper_1809_07008_amd import imb  # noqa: E402
from paper_1809_07008_amd import workloads as W  # noqa: E402

imb.LIB_PATH = os.environ["EMU_LIB"]


class HostStream:  # the emulated library ignores streams
    cuda_stream = 0


S = HostStream()


def sim_of(case, storage, tile=(32, 2)):
    s = imb.Simulation(imb.config_from_case(case, None, tile[0], tile[1], storage), S, device="cpu")
    s.set_case_particles(case.particles)
    return s


def oracle_of(case):
    r = OracleSim(OracleConfig(nx=case.nx, ny=case.ny, tau0=case.tau0, walls=case.walls, cs=case.cs,
                               gx=case.gx, gy=case.gy, rho0=case.rho0, n_sub=case.n_sub,
                               kn=case.kn, zeta=case.zeta, rho_s=case.rho_s,
                               eps_subcells=case.eps_subcells, uw_bot=case.uw_bot,
                               uw_top=case.uw_top, kt=case.kt, mu=case.mu,
                               contact_model=case.contact_model, young=case.young,
                               poisson=case.poisson))
    p = case.particles
    r.set_particles(p.x, p.y, p.r, p.vx, p.vy, p.om, p.mode)
    return r


def check(name, ok, detail):
    print("%-48s %s  %s" % (name, "ok" if ok else "FAIL", detail), flush=True)
    if not ok:
        sys.exit(1)


def moving_case():
    rng = np.random.default_rng(5)
    x, y, r = W.place_disks(rng, 64, 40, 3, 8.0, 11.0, gap=1.0, wall_gap=1.0)
    p = W.Particles(x, y, r, rng.normal(0, 0.01, 3), rng.normal(0, 0.01, 3), np.zeros(3),
                    np.zeros(3, np.int32))
    return W.Case("emu_moving", 64, 40, tau0=0.6, steps=4, gx=1e-5, cs=0.1, particles=p)


def overlap_case(walls):
    p = W.Particles(np.array([20.2, 31.0, 25.6, 54.3]), np.array([16.1, 17.3, 25.4, 9.7]),
                    np.array([6.2, 5.1, 5.4, 4.0]), np.array([0.01, -0.01, 0.0, 0.002]),
                    np.zeros(4), np.array([0.0, 0.001, 0.0, 0.0]), np.array([1, 2, 1, 0], np.int32))
    return W.Case("emu_overlap", 64, 36, tau0=0.7, steps=3, walls=walls, gx=1e-5, particles=p)


def fp64_parity(part=(0, 1)):
    """FP64 parity with the oracle; part = (k, n) runs the cases whose index is k mod n."""
    for i, case in enumerate((moving_case(), overlap_case(True), overlap_case(False),
                 W.touching_disks(6, True, steps=2), W.touching_disks(8, False, steps=2),
                 W.approaching_disks(steps=12), moving_case().with_(eps_subcells=4),
                 overlap_case(True).with_(eps_subcells=5), W.couette_channel("f64", steps=6),
                 moving_case().with_(uw_bot=0.02, uw_top=-0.01),
                 W.frictional_disks(6, True, steps=3), W.frictional_disks(8, False, steps=3),
                 W.frictional_disks(6, True, steps=3, mu=0.05),
                 W.frictional_disks(6, True, steps=3).with_(contact_model=1, young=100.0,
                                                            poisson=0.3),
                 W.touching_disks(8, False, steps=2).with_(contact_model=1, young=100.0,
                                                           poisson=0.3))):
        if i % part[1] != part[0]:
            continue
        s = sim_of(case, "f64")
        s.step(case.steps)
        ref = oracle_of(case)
        ref.step(case.steps)
        fg, fo = np.array(s.forces()), np.array(ref.forces())
        ferr = np.abs(fg - fo).max() / np.abs(fo).max()
        perr = np.abs(s.populations() - ref.populations()).max()
        kerr = 0.0
        if case.particles.n:
            kg, ko = np.array(s.particles()), np.array(ref.particles())
            d = kg - ko
            d[0] -= case.nx * np.round(d[0] / case.nx)
            if not case.walls:
                d[1] -= case.ny * np.round(d[1] / case.ny)
            kerr = np.abs(d).max()
        check("fp64 parity %s walls=%s eps_subcells=%d mu=%g law=%d" % (
                  case.name, case.walls, case.eps_subcells, case.mu, case.contact_model),
              ferr < 1e-12 and perr < 1e-13 and kerr < 1e-12,
              "force %.2e populations %.2e disks %.2e" % (ferr, perr, kerr))


def spring_table_limit():
    """Eight simultaneous tangential contacts fit a disk's spring table; a ninth latches the
    device error."""
    case = W.crowded_disk(8)
    s = sim_of(case, "f64")
    s.step(case.steps)
    ref = oracle_of(case)
    ref.step(case.steps)
    kerr = np.abs(np.array(s.particles()) - np.array(ref.particles())).max()
    check("eight tangential contacts on one disk", kerr < 1e-12, "disks %.2e" % kerr)
    nine = W.crowded_disk(9)
    try:
        s = sim_of(nine, "f64")
        s.step(1)
        s.sync()
        msg = None
    except imb.ImbError as e:
        msg = "%d %s" % (e.code, e)
    check("a ninth latches the device error", msg is not None and "more than 8" in msg,
          str(msg))


def wide_tiles():
    """Tiles 128 and 256 wide on ragged widths (odd, not a multiple of the tile), walls and
    periodic y, random initial populations: FP64 parity, and FP16 equal bit for bit to 32x2.
    The 200x72 grids also hold tile passes away from every edge, which load through the
    shifted-plane form; 32x2 tiles cut the grid differently, so the FP16 comparison sets that
    form against the general one."""
    for nx, ny, tile, walls in ((131, 40, (128, 2), True), (259, 24, (256, 2), False),
                                (130, 37, (128, 4), False), (97, 30, (128, 2), True),
                                (200, 72, (64, 2), True), (200, 72, (16, 4), False)):
        base = moving_case()
        case = base.with_(nx=nx, ny=ny, walls=walls, particles=W.Particles(
            np.array([20.3, 60.8, nx - 0.4]), np.array([12.2, ny / 2, ny - 9.7]),
            np.array([5.5, 4.2, 3.9]), np.array([0.01, -0.01, 0.0]), np.zeros(3),
            np.array([0.0, 0.001, 0.0]), np.array([0, 2, 1], np.int32)))
        f0 = W.random_populations(np.random.default_rng(nx), nx, ny, amplitude=0.03)
        s = sim_of(case, "f64", tile)
        s.set_populations(f0)
        s.step(case.steps)
        ref = oracle_of(case)
        ref.set_populations(f0)
        ref.step(case.steps)
        fg, fo = np.array(s.forces()), np.array(ref.forces())
        ferr = np.abs(fg - fo).max() / np.abs(fo).max()
        perr = np.abs(s.populations() - ref.populations()).max()
        check("fp64 parity %dx%d tile %dx%d walls=%s" % (nx, ny, tile[0], tile[1], walls),
              ferr < 1e-12 and perr < 1e-13, "force %.2e populations %.2e" % (ferr, perr))
        a, b = sim_of(case, "f16", tile), sim_of(case, "f16", (32, 2))
        a.set_populations(f0)
        b.set_populations(f0)
        a.step(case.steps)
        b.step(case.steps)
        check("f16 tile %dx%d equals tile 32x2 bit for bit" % tile,
              np.array_equal(a.populations(), b.populations()), "")


def reduced_precision():
    case = moving_case()
    ref = oracle_of(case)
    ref.step(case.steps)
    fo = np.array(ref.forces())
    for st, tol in (("f32", 1e-4), ("f16", 5e-2)):
        s = sim_of(case, st)
        s.step(case.steps)
        err = np.abs(np.array(s.forces()) - fo).max() / np.abs(fo).max()
        check("%s storage against the oracle" % st, err < tol, "force %.2e" % err)


def roundtrip():
    case = moving_case().with_(storage="f32")
    a = sim_of(case, "f32")
    a.step(2)
    blob = a.save_state()
    a.step(3)
    b = sim_of(case, "f32")
    b.load_state(blob)
    b.step(3)
    same = np.array_equal(a.populations(), b.populations()) and all(
        np.array_equal(u, v) for u, v in zip(a.forces() + a.particles(), b.forces() + b.particles()))
    check("checkpoint round trip continues bit for bit", same, "")


def adjoint():
    p = overlap_case(True).particles.copy()
    p.mode[:] = 2
    case = W.Case("emu_adjoint", 64, 36, tau0=0.7, steps=3, gx=1e-5, gy=2e-6,
                  particles=W.Particles(p.x[[0, 3]], p.y[[0, 3]], p.r[[0, 3]], p.vx[[0, 3]],
                                        p.vy[[0, 3]], p.om[[0, 3]], p.mode[[0, 3]]))
    w = dict(wfx=np.array([1.0, 0.7]), wfy=np.array([0.3, -0.5]), wtz=np.array([0.05, 0.02]))
    res = sim_of(case, "f64").adjoint(case.steps, 2, **w)
    fd = fd_gradient(case, case.steps, **w)
    errs = block_errors(res, fd)
    check("fp64 adjoint against finite differences", max(errs.values()) < 1e-5,
          " ".join("%s %.1e" % kv for kv in errs.items()))


def batch():
    cases = [moving_case(), overlap_case(False).with_(nx=48, ny=32,
                                                      particles=W.Particles.empty())]
    b = imb.Batch([imb.config_from_case(c, None, 32, 2, "f32") for c in cases], S, device="cpu")
    for k, c in enumerate(cases):
        b.set_case_particles(k, c.particles)
    b.step(3)
    b.set_schedule(imb.IMB_BATCH_PER_STEP)
    b.step(2)
    b.sync()
    for k, c in enumerate(cases):
        s = sim_of(c, "f32")
        s.step(5)
        check("batch channel %d equals the channel alone" % k,
              np.array_equal(b.populations(k), s.populations()), "both schedules")
    b.autotune(trial_steps=1, max_trials=3)
    b.step(1)
    b.sync()
    check("batch autotune", True, str(b.launch()))
    # a channel of 300 small disks, more than the persistent kernel takes: per-step schedule
    # with the 512-thread particle phase
    rng = np.random.default_rng(17)
    x, y, r = W.place_disks(rng, 160, 120, 300, 2.0, 3.0, gap=1.0, wall_gap=1.0)
    p = W.Particles(x, y, r, rng.normal(0, 0.01, 300), rng.normal(0, 0.01, 300), np.zeros(300),
                    np.zeros(300, np.int32))
    cases = [moving_case().with_(nx=160, ny=120, particles=p), moving_case()]
    b = imb.Batch([imb.config_from_case(c, None, 32, 2, "f32") for c in cases], S, device="cpu")
    for k, c in enumerate(cases):
        b.set_case_particles(k, c.particles)
    refused = False
    try:
        b.set_schedule(imb.IMB_BATCH_PERSISTENT)
    except imb.ImbError:
        refused = True
    check("wide batch refuses the persistent schedule", refused and
          b.launch()["schedule"] == "per_step", "")
    b.step(2)
    b.sync()
    for k, c in enumerate(cases):
        s = sim_of(c, "f32")
        s.step(2)
        same = np.array_equal(b.populations(k), s.populations()) and all(
            np.array_equal(u, v) for u, v in zip(b.forces(k) + b.particles(k),
                                                  s.forces() + s.particles()))
        check("wide batch channel %d equals the channel alone" % k, same, "%d disks" % c.particles.n)


def no_allocation_step():
    """imb_step_noalloc (per-disk forces in the library-wide array) equals imb_step, twice in a
    row, the second on a smaller simulation."""
    for case, steps in ((moving_case(), 3), (overlap_case(True), 2)):
        a, b = sim_of(case, "f32"), sim_of(case, "f32")
        a.step(steps)
        b.step_noalloc(steps)
        same = np.array_equal(a.populations(), b.populations()) and all(
            np.array_equal(u, v) for u, v in zip(a.forces() + a.particles(),
                                                  b.forces() + b.particles()))
        check("step_noalloc equals step (%s)" % case.name, same, "")


def mask_rounds():
    """600 tile rows of 256x1 tiles on a 20-wide lattice, more than the 512 rows one round of the
    particle phase's LDS holds, so the band masks are built in two rounds: disks astride the
    rounds' boundary (tile row 512) and near both walls, FP64 parity for 3 coupled steps."""
    xs = np.array([6.0, 15.0, 10.0, 8.0, 12.0])
    ys = np.array([506.0, 514.5, 521.0, 4.5, 594.0])
    rs = np.array([4.5, 3.5, 2.5, 3.0, 4.0])
    p = W.Particles(xs, ys, rs, np.array([0.01, -0.01, 0.0, 0.0, 0.0]),
                    np.array([0.0, 0.02, -0.01, 0.0, 0.0]), np.zeros(5),
                    np.array([0, 0, 2, 0, 1], np.int32))
    case = W.Case("emu_rounds", 20, 600, tau0=0.6, steps=3, gx=1e-5, cs=0.1, particles=p)
    s = sim_of(case, "f64", (256, 1))
    s.step(case.steps)
    ref = oracle_of(case)
    ref.step(case.steps)
    fg, fo = np.array(s.forces()), np.array(ref.forces())
    ferr = np.abs(fg - fo).max() / np.abs(fo).max()
    perr = np.abs(s.populations() - ref.populations()).max()
    xerr = max(np.abs(a - b).max() for a, b in zip(s.particles(), ref.particles()))
    check("fp64 parity, band masks in two rounds", ferr < 1e-12 and perr < 1e-13 and xerr < 1e-12,
          "force %.2e populations %.2e disks %.2e" % (ferr, perr, xerr))


def slab_cases():
    """A lattice split in y: the slabs' composition against the FP64 oracle (free disks, walls
    and periodic, disks spanning up to four slabs and the periodic seam), and bit for bit
    against the whole lattice where forces do not feed back (fixed and prescribed disks, FP32
    and FP16)."""
    seam = overlap_case(False)
    p = seam.particles.copy()
    p.y[3] = 1.2  # across the periodic boundary in y
    seam = seam.with_(particles=p)
    for case, tile, nslab in ((moving_case(), (32, 2), 2), (moving_case(), (64, 1), 10),
                              (seam, (32, 2), 3), (seam, (64, 1), 4),
                              (moving_case().with_(uw_bot=0.02, uw_top=-0.01), (64, 1), 3)):
        ref = oracle_of(case)
        ref.step(case.steps)
        sl = imb.Slabs(imb.config_from_case(case, None, tile[0], tile[1], "f64"), nslab, S)
        sl.set_case_particles(case.particles)
        sl.step(case.steps)
        fx, fy, tz = sl.forces()
        Fx, Fy, Tz = ref.forces()
        scale = max(np.abs(Fx).max(), np.abs(Fy).max(), 1e-300)
        ferr = max(np.abs(fx - Fx).max(), np.abs(fy - Fy).max(), np.abs(tz - Tz).max() / 10) / scale
        perr = np.abs(sl.populations() - ref.populations()).max()
        same = all(np.array_equal(a, b) for k in range(1, nslab)
                   for a, b in zip(sl.particles(0), sl.particles(k)))
        check("slabs fp64 %s x%d tile %dx%d" % (case.name, nslab, *tile),
              ferr < 1e-12 and perr < 1e-14 and same,
              "force %.2e populations %.2e replicas equal %s" % (ferr, perr, same))
    fixed = seam.particles.copy()
    fixed.mode[:] = np.array([1, 2, 2, 1], np.int32)
    for storage in ("f32", "f16"):
        case = seam.with_(particles=fixed, storage=storage)
        whole = sim_of(case, storage, (64, 1))
        whole.step(3)
        sl = imb.Slabs(imb.config_from_case(case, None, 64, 1, storage), 3, S)
        sl.set_case_particles(case.particles)
        sl.step(3)
        fw, fs = whole.forces(), sl.forces()
        ferr = max(np.abs(a - b).max() for a, b in zip(fw, fs)) / np.abs(fw[0]).max()
        parts = [sl.partial_forces(k) for k in range(3)]
        psum = [sum(pk[c] for pk in parts) for c in range(3)]
        check("slabs %s equal the whole lattice (fixed disks)" % storage,
              np.array_equal(whole.populations(), sl.populations()) and ferr < 1e-5 and
              all(np.array_equal(a, b) for a, b in zip(psum, fs)),
              "force %.1e" % ferr)


def three_d():
    """D3Q19 with spheres against the 3D oracle: fixed and prescribed spheres across the periodic
    seams, two spheres sharing cells, walls and periodic y, random populations, every tile width."""
    from oracle import OracleConfig3, OracleSim3
    rng = np.random.default_rng(7)
    cases = [  # nx, ny, nz, walls, tile_w, spheres (x, y, z, r, v, w, mode)
        (19, 13, 11, True, 16, [(0.4, 6.3, 5.2, 3.1, (0.0, 0.0, 0.0), (0.0, 0.002, 0.0), 1),
                                (8.7, 6.9, 10.6, 2.6, (0.02, -0.01, 0.005), (0.0, 0.0, 0.0), 2)]),
        (22, 16, 12, False, 32, [(11.2, 0.5, 4.4, 3.3, (0.01, 0.0, 0.0), (0.001, 0.0, -0.002), 2),
                                (14.6, 3.8, 4.9, 2.4, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 1)]),
        (70, 12, 11, True, 64, [(35.5, 4.0, 3.5, 2.9, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 1)]),
    ]
    for nx, ny, nz, walls, tw, sph in cases:
        f0 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None, None, None] * (
            1.0 + 0.03 * rng.uniform(-1, 1, (19, nz, ny, nx)))
        x, y, z, r = (np.array([t[k] for t in sph]) for k in range(4))
        v = np.array([t[4] for t in sph])
        w = np.array([t[5] for t in sph])
        mode = np.array([t[6] for t in sph], np.int32)
        ref = OracleSim3(OracleConfig3(nx=nx, ny=ny, nz=nz, tau0=0.7, walls=walls, gx=2e-5,
                                       gy=-1e-5, gz=5e-6, eps_subcells=4))
        ref.set_populations(f0)
        ref.set_spheres(x, y, z, r, v, w, mode)
        ref.step(3)
        for storage, tol in (("f64", 1e-12), ("f32", 1e-4)):
            cfg = imb.make_config3(nx, ny, nz, 0.7, storage, walls, (2e-5, -1e-5, 5e-6),
                                   max_spheres=4, eps_subcells=4, tile_w=tw)
            s = imb.Simulation3(cfg, S, device="cpu")
            s.set_populations(f0)
            s.set_spheres(x, y, z, r, v, w, mode)
            s.step(3)
            Fg, Tg = s.forces()
            Fo, To = ref.forces()
            ferr = max(np.abs(Fg - Fo).max() / np.abs(Fo).max(),
                       np.abs(Tg - To).max() / np.abs(To).max())
            perr = np.abs(s.populations() - ref.populations()).max()
            check("3d %s %dx%dx%d walls=%s tile %d" % (storage, nx, ny, nz, walls, tw),
                  ferr < tol and perr < (1e-14 if storage == "f64" else 1e-6),
                  "force %.2e populations %.2e" % (ferr, perr))
            ok = np.abs(s.spheres()[:, :3] - np.stack(ref.spheres(), 1)).max() < 1e-12
            check("3d spheres move as prescribed", ok, "")


ALL = (slab_cases, three_d, no_allocation_step, spring_table_limit, fp64_parity, wide_tiles,
       reduced_precision, roundtrip, adjoint, batch, mask_rounds)


if __name__ == "__main__":
    # arguments: case functions to run (all without any); "fp64_parity:k/n" runs part k of n
    for spec in sys.argv[1:] or [fn.__name__ for fn in ALL]:
        name, _, part = spec.partition(":")
        fn = {f.__name__: f for f in ALL}[name]
        if part:
            k, n = part.split("/")
            fn(part=(int(k), int(n)))
        else:
            fn()
    print("all emulated cases passed", flush=True)
