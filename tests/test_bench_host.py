"""CPU: the host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic bytes per
lattice update, and the lookup of the committed counter summary (it answers only for the storage
format, tile shape and disk count it was taken with)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bytes_per_lattice_update():
    assert bench.bytes_per_lup("f64") == 144
    assert bench.bytes_per_lup("f32") == 72
    assert bench.bytes_per_lup("f16") == 36


def test_counter_summary_answers_only_for_its_own_workload():
    for storage, tile, disks in (("f16", (32, 2), 500), ("f32", (64, 1), 500),
                                 ("f32", (32, 2), 7)):
        assert bench.measured_traffic(storage, tile, disks) is None
    t = bench.measured_traffic("f32", (32, 2), 500)
    # either the summary matches the kernel's sources (bytes at least the algorithmic 151 MB) or
    # the sources changed since it was taken (no figure)
    assert t is None or t >= 72 * 2048 * 1024
