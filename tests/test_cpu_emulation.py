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


@pytest.mark.skipif(_asan_runtime() is None, reason="g++ with AddressSanitizer not available")
def test_kernels_under_cpu_emulation_with_address_sanitizer():
    import build_emu
    lib = build_emu.build()
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
               EMU_LIB=lib, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, os.path.join(HERE, "emulation", "run_cases.py")],
                       env=env, capture_output=True, text=True, timeout=1200)
    print(r.stdout)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "all emulated cases passed" in r.stdout


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
