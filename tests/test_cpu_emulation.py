"""The library's kernels compiled for the host against an emulation of the HIP execution model
(tests/emulation), run under AddressSanitizer: every kernel index is bounds-checked on the CPU,
and the emulated kernels are compared with the FP64 oracle (parity to 1e-12), with finite
differences (adjoint) and with each other (batch vs single, checkpoint round trip)."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emulation"))


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


# The emulated cases in four processes that run at once (each workgroup's threads are operating
# system threads, so one process keeps only a few cores busy), of about equal length.
GROUPS = (["fp64_parity:0/2", "slab_cases"],
          ["fp64_parity:1/2", "batch", "roundtrip", "reduced_precision"],
          ["three_d", "adjoint", "spring_table_limit"],
          ["wide_tiles", "no_allocation_step", "mask_rounds"])


@pytest.mark.skipif(_asan_runtime() is None, reason="g++ with AddressSanitizer not available")
def test_kernels_under_cpu_emulation_with_address_sanitizer(tmp_path):
    import build_emu
    lib = build_emu.build()
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
               EMU_LIB=lib, OMP_NUM_THREADS="2")
    procs = []
    for k, group in enumerate(GROUPS):
        out = open(tmp_path / ("group%d.out" % k), "w+")
        procs.append((group, out, subprocess.Popen(
            [sys.executable, os.path.join(HERE, "emulation", "run_cases.py"), *group],
            env=env, stdout=out, stderr=subprocess.STDOUT, text=True)))
    failures = []
    for group, out, p in procs:
        try:
            rc = p.wait(timeout=1200)
        except subprocess.TimeoutExpired:
            p.kill()
            rc = "timeout"
        out.seek(0)
        text = out.read()
        out.close()
        print(text)
        if "AddressSanitizer" in text or rc != 0 or "all emulated cases passed" not in text:
            failures.append("%s: exit %s\n%s" % (" ".join(group), rc, text[-4000:]))
    assert not failures, "\n".join(failures)


def test_fp16_stochastic_rounding_matches_its_rule(tmp_path):
    """The FP16 codec's stochastic-rounding store, compiled for the host, against the rounding
    rule written out (tests/emulation/sr_check.cpp)."""
    root = os.path.dirname(HERE)
    exe = str(tmp_path / "sr_check")
    subprocess.check_call(["g++", "-std=c++20", "-O1", "-ffp-contract=off", "-pthread",
                           "-I" + os.path.join(HERE, "emulation"),
                           "-I" + os.path.join(root, "paper_1809_07008_amd", "csrc"),
                           "-I" + os.path.join(root, "include"),
                           os.path.join(HERE, "emulation", "sr_check.cpp"),
                           os.path.join(HERE, "emulation", "emu.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr


def test_solid_ratio_of_cut_cells_against_the_oracle(tmp_path):
    """The kernels' solid ratio (solid.h, compiled for the host) on cut cells near circles of
    radius 0.3 to 32, against the oracle's exact area (a chord integral in long double): the
    double-precision walk within 1e-13, the single-precision forms (a branch-free evaluation of
    the common one-arc cut, else the walk) within 1e-6.  The cells include four where an earlier
    single-precision walk, deciding a crossing from the rounded half chord while a corner's
    exact power put that corner on the other side of the circle, paired the arcs wrongly
    (errors up to 0.5)."""
    import numpy as np
    from oracle import solid_fraction
    root = os.path.dirname(HERE)
    exe = str(tmp_path / "solid_check")
    subprocess.check_call(["g++", "-std=c++20", "-O1", "-ffp-contract=off",
                           "-I" + os.path.join(HERE, "emulation"),
                           "-I" + os.path.join(root, "paper_1809_07008_amd", "csrc"),
                           "-I" + os.path.join(root, "include"),
                           os.path.join(HERE, "emulation", "solid_check.cpp"), "-o", exe])
    rng = np.random.default_rng(77)
    n = 60000
    r = np.where(np.arange(n) % 3 == 0, rng.uniform(0.3, 2.0, n), rng.uniform(2.0, 32.0, n))
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    d = r + rng.uniform(-0.8, 0.8, n)
    cells = np.stack([r, d * np.cos(th), d * np.sin(th)], 1).astype(np.float32).astype(np.float64)
    regress = np.array([[21.7573776, -3.55847311, 21.041338], [10.2143087, -9.15695381, 4.92118549],
                        [29.3627167, -9.1782999, 27.5509586], [29.8560715, -22.8762226, 19.265871]],
                       np.float32).astype(np.float64)
    cells = np.concatenate([regress, cells])
    inp = "\n".join("%.17g %.17g %.17g" % tuple(c) for c in cells) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([[float(v) for v in line.split()] for line in out.splitlines()])
    exact = np.array([solid_fraction(*c) for c in cells])
    cut = (exact > 0.0) & (exact < 1.0)
    assert cut.sum() > 20000 and cut[:4].all()
    e32 = np.abs(got[:, 0] - exact)[cut].max()
    e64 = np.abs(got[:, 1] - exact)[cut].max()
    print("cut cells %d: single %.2e, double %.2e; the four former failures %s"
          % (cut.sum(), e32, e64, np.abs(got[:4, 0] - exact[:4])))
    assert e32 <= 1e-6 and e64 <= 1e-13
