"""Host logic of bench.py (CPU): the one-GPU guard, the algorithmic bytes of the
electron push, and the HBM traffic taken from the committed counter summary
only while the kernel source is the one it was measured on."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_push_bytes_are_the_per_unit_figures():
    from paper_0705_0497_amd import binding as B
    dc = np.zeros(B.NCOUNT, np.int64)
    dc[B.C_PUSH] = 1000
    dc[B.C_CAND] = 383
    dc[B.C_PUSH + 1] = 50                     # ion pushes do not count for the electron kernel
    assert bench.push_alg_bytes(dc) == 24 * 1000 + 20 * 383


def test_traffic_only_for_the_measured_kernel_source(tmp_path, monkeypatch):
    text = open(bench.TRAFFIC_SUMMARY).read()
    assert "kernels.hip sha256[:16]" in text and "HBM bytes per electron push" in text
    per_push = float(text.split("HBM bytes per electron push:")[1].split()[0])
    got = bench.measured_traffic(1e6)
    assert got is None or abs(got - per_push * 1e6) < 1e-6 * per_push * 1e6
    changed = tmp_path / "kernels.hip"
    changed.write_bytes(open(bench.KERNEL_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(changed))
    assert bench.measured_traffic(1e6) is None
