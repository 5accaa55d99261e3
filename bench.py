"""Benchmark of the coupled D2Q9 IMB-DEM step on one MI355X.

Workload: 2048x1024 channel, 500 moving disks (diameters U[16, 24]), Smagorinsky C_s = 0.1,
tau 0.55, linear spring-dashpot DEM, FP32 deviation storage, seeded synthetic input (seed 0).
One "step" is one full coupled step: solid ratio, IMB collision + streaming, force/torque sums,
DEM update (two kernels: the lattice kernel, then the particle phase).  Prints one JSON line
(throughput in MLUPS, HBM roofline of the lattice kernel, the adjoint/forward time ratio, the CPU
oracle's throughput on the same workload).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
CSRC = os.path.join(ROOT, "paper_1809_07008_amd", "csrc")
LATTICE_SOURCES = ("step.hip", "disk_block.h", "tile.h", "collide.h", "solid.h", "common.h")
COUNTERS = os.path.join(ROOT, "profiles", "k_step_2048x1024_n500_counters.txt")


def lattice_source_hash() -> str:
    """sha256 over the sources the lattice kernel (k_step) is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in LATTICE_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, tile, disks: int = 500) -> float | None:
    """HBM-side bytes per lattice-kernel launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by what the counter reads for a copy kernel of known
    size), or None when the summary is missing, was taken for another storage format, tile or
    disk count, or the kernel's sources have changed since."""
    try:
        with open(COUNTERS) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    try:
        if (kv["kernel_source_sha256"] != lattice_source_hash() or kv["storage"] != storage
                or kv["tile"] != "%dx%d" % tuple(tile) or int(kv["disks"]) != disks):
            return None
        fetch_scale = float(kv["copy_bytes"]) / (float(kv["copy_fetch_kib"]) * 1024.0)
        write_scale = float(kv["copy_bytes"]) / (float(kv["copy_write_kib"]) * 1024.0)
        return (float(kv["fetch_kib"]) * 1024.0 * fetch_scale
                + float(kv["write_kib"]) * 1024.0 * write_scale)
    except (KeyError, ValueError, ZeroDivisionError):
        return None


# Tile of the differentiation leg: the adjoint kernel holds 252 VGPRs (two wavefronts per
# SIMD), so on the 512x256 channel one-row tiles (512 workgroups instead of 256 for 32x2) give
# it twice the workgroups in flight; the forward step is within 2% of its 32x2 time there.
ADJOINT_TILE = (64, 1)


def adjoint_ratio(tile=ADJOINT_TILE, reps: int = 3):
    """Differentiation form on the 512x256 / 20-disk channel (FP32, 200 steps, checkpoint every
    20): GPU time per reverse step (recomputation + adjoint step) over the forward step time,
    both with the same tile shape."""
    import numpy as np
    from paper_1809_07008_amd import imb, workloads
    case = workloads.adjoint_channel(seed=0, storage="f32")
    n = case.particles.n
    fwd = imb.simulation_from_case(case, storage="f32", tile_w=tile[0], tile_rows=tile[1])
    fwd.step(20)
    warm_graphs(fwd)
    t0 = time.perf_counter()
    fwd.step(case.steps)
    fwd.sync()
    fwd_us = (time.perf_counter() - t0) / case.steps * 1e6
    fwd.set_kernel_timing(True)
    fwd.step(case.steps)
    kt = fwd.kernel_timing()
    fwd.close()
    sim = imb.simulation_from_case(case, storage="f32", tile_w=tile[0], tile_rows=tile[1])
    sim.adjoint(case.steps, 20, wfx=np.ones(n))  # allocation and warm-up
    best = None
    for _ in range(reps):
        sim.adjoint(case.steps, 20, wfx=np.ones(n))
        t = sim.adjoint_timing()
        if best is None or t["reverse_ms"] < best["reverse_ms"]:
            best = t
    sim.set_kernel_timing(True)
    sim.adjoint(case.steps, 20, wfx=np.ones(n))
    kk = sim.adjoint_timing()
    sim.close()
    rev_us = best["reverse_ms"] * 1e3 / case.steps
    whole_us = (best["forward_ms"] + best["reverse_ms"]) * 1e3 / case.steps
    return {"workload": "adjoint_512x256_n20", "storage": "f32", "steps": case.steps,
            "k_ckpt": 20, "tile": list(tile), "forward_step_us": round(fwd_us, 2),
            "forward_pass_in_adjoint_us_per_step": round(best["forward_ms"] * 1e3 / case.steps, 2),
            "reverse_step_us": round(rev_us, 2),
            # reverse sweep (recomputation + adjoint step) per step over a forward step
            "ratio": round(rev_us / fwd_us, 3),
            # the whole differentiated run (checkpointed forward pass + reverse sweep) per step
            # over a forward step
            "ratio_whole_call": round(whole_us / fwd_us, 3),
            "adjoint_kernel_us": round(kk["adjoint_kernel_ms"] * 1e3 /
                                       max(kk["adjoint_kernels"], 1), 2),
            "recompute_kernel_us": round(kk["recompute_kernel_ms"] * 1e3 /
                                         max(kk["recompute_kernels"], 1), 2),
            "forward_lattice_kernel_us": round(kt["lattice_ms"] * 1e3 /
                                               max(kt["lattice_launches"], 1), 2),
            "forward_particle_kernel_us": round(kt["particle_ms"] * 1e3 /
                                                max(kt["particle_launches"], 1), 2)}


def batch_throughput(steps: int = 100):
    """Batched form on the 64-channel workload (11.1 M cells, 4489 disks, FP32): GPU time per
    step (HIP events around one graph replay) under each schedule at the default tile shape, then
    after the autotuner."""
    from paper_1809_07008_amd import imb, workloads
    cases = workloads.batch_channels(seed=0)
    cells = sum(c.cells for c in cases)
    b = imb.batch_from_cases(cases)
    out = {"workload": "batch_channels_n64", "channels": len(cases), "cells": cells,
           "disks": int(sum(c.particles.n for c in cases)), "steps": steps}
    for name, sched in (("persistent", imb.IMB_BATCH_PERSISTENT),
                        ("per_step", imb.IMB_BATCH_PER_STEP)):
        b.set_schedule(sched)
        b.step(4)
        ms = b.timed_steps(steps) / steps
        out[name + "_ms_per_step"] = round(ms, 4)
    b.autotune(trial_steps=10)
    ms = b.timed_steps(steps) / steps
    out["tuned"] = b.launch()
    out["tuned_ms_per_step"] = round(ms, 4)
    out["tuned_mlups"] = round(cells / (ms * 1e-3) / 1e6, 1)
    b.close()
    return out


def subcell_estimate(storage: str, tile, n: int = 5, steps: int = 300):
    """The same workload with the paper's n x n sub-cell solid ratio instead of the exact one:
    whole-step time (graph replay) and lattice-kernel time (HIP events)."""
    from paper_1809_07008_amd import imb, workloads
    case = workloads.moving_disks(seed=0, storage=storage).with_(eps_subcells=n)
    sim = imb.simulation_from_case(case, storage=storage, tile_w=tile[0], tile_rows=tile[1])
    sim.step(20)
    warm_graphs(sim)
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    step_us = (time.perf_counter() - t0) * 1e6 / steps
    sim.set_kernel_timing(True)
    sim.step(steps)
    kt = sim.kernel_timing()
    sim.close()
    return {"eps_subcells": n, "ms_per_step": round(step_us * 1e-3, 5),
            "mlups": round(case.cells / step_us, 1),
            "lattice_kernel_us": round(kt["lattice_ms"] * 1e3 / max(kt["lattice_launches"], 1), 2)}


def warm_graphs(sim) -> None:
    """Captures every step graph imb_step may replay and replays the two of the current buffer
    parity once (34 steps, the parity unchanged), so a timed region replays warm graphs only."""
    sim.prepare_graphs()
    sim.step(32)
    sim.step(2)
    sim.sync()


def hbm_control(tile, steps: int = 100, n: int = 512):
    """The moving-disk workload at 8192x4096 (1.2 GB per FP32 population copy, far beyond the
    256 MB Infinity Cache, so every byte comes from HBM): whole-step time (graph replay) and the
    lattice kernel's time (HIP events), with n disks."""
    from paper_1809_07008_amd import imb, workloads
    case = workloads.moving_disks(seed=0, nx=8192, ny=4096, n=n, storage="f32")
    sim = imb.simulation_from_case(case, storage="f32", tile_w=tile[0], tile_rows=tile[1])
    sim.step(4)
    warm_graphs(sim)
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    step_s = (time.perf_counter() - t0) / steps
    sim.set_kernel_timing(True)
    sim.step(steps // 2)
    kt = sim.kernel_timing()
    sim.close()
    lat_s = kt["lattice_ms"] * 1e-3 / max(kt["lattice_launches"], 1)
    byts = case.cells * bytes_per_lup("f32")
    return {"workload": "moving_disks_8192x4096_n%d" % n, "disks": n,
            "ms_per_step": round(step_s * 1e3, 4), "mlups": round(case.cells / step_s / 1e6, 1),
            "lattice_kernel_us": round(lat_s * 1e6, 2),
            "lattice_kernel_GBps": round(byts / lat_s / 1e9, 1),
            "lattice_kernel_frac_of_8TBps": round(byts / lat_s / 8e12, 4),
            "particle_phase_us": round(kt["particle_ms"] * 1e3 / max(kt["particle_launches"], 1),
                                       2)}


def slab_share(storage: str, tile, nslabs: int = 8, steps: int = 200):
    """One device's share of the 2048x1024 channel split in y into eight 2048x128 slabs, the
    shape each of eight GPUs would hold: every slab's lattice kernel (HIP events at each
    launch), the kernel that stands in for the face transfers and the force all-reduce, and the
    particle phase that every slab replicates; also the whole eight-slab step run on this one
    device (graph replay)."""
    from paper_1809_07008_amd import imb, workloads
    case = workloads.moving_disks(seed=0, storage=storage)
    sl = imb.slabs_from_case(case, nslabs, storage=storage, tile_w=tile[0], tile_rows=tile[1])
    y0, rows = sl.layout()
    sl.step(34)  # captures and replays the 2- and 32-step graphs
    sl.sync()
    t0 = time.perf_counter()
    sl.step(steps)
    sl.sync()
    all_s = (time.perf_counter() - t0) / steps
    sl.set_kernel_timing(True)
    sl.step(steps)
    lat, xch, par, n = sl.kernel_timing()
    sl.close()
    lat_us = lat * 1e3 / n
    bpl = bytes_per_lup(storage)
    cells = case.nx * rows
    gbps = cells * bpl / (lat_us * 1e-6) / 1e9
    es = {"f64": 8, "f32": 4, "f16": 2}[storage]
    return {"workload": "moving_disks_2048x1024_n500 as %d slabs" % nslabs,
            "slab_rows": rows.tolist(),
            "lattice_kernel_us": [round(v, 2) for v in lat_us],
            "lattice_kernel_us_max": round(float(lat_us.max()), 2),
            "lattice_kernel_GBps_min": round(float(gbps.min()), 1),
            "lattice_kernel_frac_of_8TBps_min": round(float(gbps.min()) / HBM_PEAK_GBS, 4),
            "exchange_us_all_slabs": round(xch * 1e3 / n, 2),
            "particle_phase_us": round(float(par.mean()) * 1e3 / n, 2),
            "face_bytes_per_slab_per_step": 2 * 3 * case.nx * es,
            "force_share_bytes_per_step": case.particles.n * 24,
            "share_compute_us_per_step": round(float(lat_us.max() + par.mean() * 1e3 / n), 2),
            "all_slabs_one_device_ms_per_step": round(all_s * 1e3, 4)}


def hbm_control_density(tile, steps: int = 50, nch: int = 16):
    """The headline's disk density at the HBM-resident size: 16 independent 2048x1024 channels
    of the moving-disk workload with 500 disks each, seeds 0-15 (33.5 M cells and 8000 disks, as
    many cells as the 8192x4096 control; 2.4 GB per population copy), advanced by the batched
    form's per-step schedule.  Whole-step time per step (HIP events around one graph replay)."""
    from paper_1809_07008_amd import imb, workloads
    cases = [workloads.moving_disks(seed=k, nx=2048, ny=1024, n=500, storage="f32")
             for k in range(nch)]
    cells = sum(c.cells for c in cases)
    b = imb.batch_from_cases(cases, tile_w=tile[0], tile_rows=tile[1])
    b.set_schedule(imb.IMB_BATCH_PER_STEP)
    b.step(4)
    ms = b.timed_steps(steps) / steps
    b.close()
    return {"workload": "%d channels of moving_disks_2048x1024_n500" % nch, "cells": cells,
            "disks": int(sum(c.particles.n for c in cases)), "ms_per_step": round(ms, 4),
            "mlups": round(cells / (ms * 1e-3) / 1e6, 1),
            "whole_step_GBps": round(cells * bytes_per_lup("f32") / (ms * 1e-3) / 1e9, 1),
            "whole_step_frac_of_8TBps": round(cells * bytes_per_lup("f32") / (ms * 1e-3) / 8e12,
                                              4)}


def memory_calibration(sizes=(158 * 2 ** 20, 2400 * 2 ** 20), reps: int = 20):
    """Attainable bandwidth of plain device copies (two bytes moved per byte copied), HIP events
    on the current stream: the library's copy kernel (several 16-byte loads in flight per lane,
    non-temporal loads and stores) and torch's device copy, at a size the Infinity Cache holds
    and at one it does not."""
    import torch
    from paper_1809_07008_amd import imb
    out = {}
    for nbytes in sizes:
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for name, fn in (("copy_kernel", lambda: imb.copy_kernel(b.data_ptr(), a.data_ptr(),
                                                                 nbytes)),
                         ("torch_copy", lambda: b.copy_(a))):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            dt = e0.elapsed_time(e1) * 1e-3 / reps
            out["%s_%dMiB_GBps" % (name, nbytes >> 20)] = round(2 * nbytes / dt / 1e9, 1)
        del a, b
    return out


def copy_calibration(nbytes: int, reps: int = 10) -> int:
    """Runs only the plain copy kernel over nbytes (the counter calibration of the traffic
    figure) and prints its bandwidth."""
    import torch
    from paper_1809_07008_amd import imb
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    imb.copy_kernel(b.data_ptr(), a.data_ptr(), nbytes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        imb.copy_kernel(b.data_ptr(), a.data_ptr(), nbytes)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"mode": "copy_calibration", "bytes_read": nbytes, "bytes_written": nbytes,
                      "reps": reps, "us_per_copy": round(dt * 1e6, 2),
                      "GBps": round(2 * nbytes / dt / 1e9, 1)}), flush=True)
    return 0


def bytes_per_lup(storage: str) -> int:
    """Algorithmic bytes per lattice update: 9 populations read + 9 written."""
    return 2 * 9 * {"f64": 8, "f32": 4, "f16": 2}[storage]


def cpu_baseline(case, target_s: float = 15.0):
    """The FP64 CPU oracle on the same workload, a bounded number of steps, on the host's cores
    and (as `single_core`) on one core."""
    import oracle
    ref = oracle.OracleSim(oracle.OracleConfig(nx=case.nx, ny=case.ny, tau0=case.tau0,
                                               walls=case.walls, cs=case.cs, gx=case.gx,
                                               gy=case.gy, rho0=case.rho0, n_sub=case.n_sub,
                                               kn=case.kn, zeta=case.zeta, rho_s=case.rho_s))
    p = case.particles
    ref.set_particles(p.x, p.y, p.r, p.vx, p.vy, p.om, p.mode)
    t0 = time.perf_counter()
    ref.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, min(1000, int(target_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    ref.step(n)
    dt = time.perf_counter() - t0
    out = {"value": round(case.cells * n / dt / 1e6, 3), "unit": "MLUPS",
           "cores": oracle.get_threads(), "kind": "oracle",
           "sample": "%d coupled steps of the %dx%d / %d-disk workload in FP64 (after 1 warm-up "
                     "step), %.1f s" % (n, case.nx, case.ny, p.n, dt)}
    # the same on one core (a few steps, about 5 s)
    threads = oracle.get_threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        ref.step(1)
        t1 = time.perf_counter() - t0
        n1 = max(1, min(100, int(5.0 / max(t1, 1e-6))))
        t0 = time.perf_counter()
        ref.step(n1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    out["single_core"] = {"value": round(case.cells * n1 / dt1 / 1e6, 3), "unit": "MLUPS",
                          "cores": 1, "sample": "%d coupled steps, %.1f s" % (n1, dt1)}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16"])
    ap.add_argument("--tile-w", type=int, default=32)
    ap.add_argument("--tile-rows", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward ratio and the batched form (profiling the "
                         "forward step alone)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--disks", type=int, default=500,
                    help="disks of the 2048x1024 channel (500: the headline workload; 0: the "
                         "lattice alone, a control)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch kernels directly instead of replaying captured graphs")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run the copy kernel over this many bytes (counter calibration)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the batched form (64 channels) and print its JSON")
    ap.add_argument("--slab-only", action="store_true",
                    help="only run the eight-slab share of the lattice and print its JSON")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (got --gpus %d); one GPU's share of "
              "a lattice split in y slabs is measured by --slab-only (and in the default run), "
              "but no run spans several GPUs." % args.gpus, file=sys.stderr)
        return 2

    import torch
    from paper_1809_07008_amd import imb, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.copy_bytes:
        return copy_calibration(args.copy_bytes)
    if args.batch_only:
        print(json.dumps({"mode": "batch_only", "batch": batch_throughput()}), flush=True)
        return 0
    if args.slab_only:
        print(json.dumps({"mode": "slab_only",
                          "slab_share": slab_share(args.storage, (args.tile_w, args.tile_rows))}),
              flush=True)
        return 0
    case = workloads.moving_disks(seed=args.seed, storage=args.storage, n=args.disks)
    sim = imb.simulation_from_case(case, storage=args.storage, tile_w=args.tile_w,
                                   tile_rows=args.tile_rows)
    if args.no_graphs:
        sim.set_graphs(False)
    sim.step(args.warmup)
    if not args.no_graphs:
        warm_graphs(sim)  # the timed call replays only captured, already replayed graphs
    sim.sync()
    print("bench: warmup done", file=sys.stderr, flush=True)

    # timed region: K coupled steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    mlups = case.cells * args.steps / wall / 1e6
    print("bench: %d steps %.3f ms/step %.1f MLUPS" % (args.steps, ms_per_step, mlups),
          file=sys.stderr, flush=True)

    # per-kernel durations with HIP events on the simulation's stream (same K steps again)
    sim.set_kernel_timing(True)
    sim.step(args.steps)
    kt = sim.kernel_timing()
    sim.set_kernel_timing(False)
    lat_ms = kt["lattice_ms"] / max(kt["lattice_launches"], 1)
    par_ms = kt["particle_ms"] / max(kt["particle_launches"], 1)
    bpl = bytes_per_lup(args.storage)
    step_bytes = case.cells * bpl
    achieved = step_bytes / (lat_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.storage, (args.tile_w, args.tile_rows),
                                            args.disks),
                "kernel_source_sha256": lattice_source_hash(),
                "kernel": "k_step<%s>" % {"f64": "StoreF64", "f32": "StoreF32",
                                          "f16": "StoreF16"}[args.storage],
                "kernel_avg_us": round(lat_ms * 1e3, 2),
                "bytes_per_launch": step_bytes,
                "particle_phase_avg_us": round(par_ms * 1e3, 2)}

    out = {
        "metric": "MLUPS & % of HBM roofline, D2Q9 IMB 2048x1024; adjoint/forward time ratio",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "graph_warm_steps": 0 if args.no_graphs else 34,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic (seeded disks, fluid at rest)",
        "config": {"workload": case.name, "nx": case.nx, "ny": case.ny,
                   "disks": case.particles.n, "tau0": case.tau0, "smagorinsky_cs": case.cs,
                   "storage": args.storage, "tile": [args.tile_w, args.tile_rows],
                   "parallelism": "single GPU"},
        "hbm_frac_whole_step": round(mlups * 1e6 * bpl / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roofline,
    }
    if not args.no_adjoint:
        out["memory_calibration"] = memory_calibration()
        print("bench: calibration %s" % out["memory_calibration"], file=sys.stderr, flush=True)
        out["hbm_control"] = hbm_control((args.tile_w, args.tile_rows))
        print("bench: hbm control %s" % out["hbm_control"], file=sys.stderr, flush=True)
        out["hbm_control_density"] = hbm_control_density((args.tile_w, args.tile_rows))
        print("bench: hbm control at the headline density %s" % out["hbm_control_density"],
              file=sys.stderr, flush=True)
        out["subcell"] = subcell_estimate(args.storage, (args.tile_w, args.tile_rows))
        out["adjoint"] = adjoint_ratio()
        print("bench: adjoint ratio %.3f" % out["adjoint"]["ratio"], file=sys.stderr, flush=True)
        out["batch"] = batch_throughput()
        print("bench: batch %.3f ms per step" % out["batch"]["tuned_ms_per_step"],
              file=sys.stderr, flush=True)
        out["slab_share"] = slab_share(args.storage, (args.tile_w, args.tile_rows))
        print("bench: slab share %s" % out["slab_share"], file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
