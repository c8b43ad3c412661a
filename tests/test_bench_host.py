"""Host checks of the benchmark's own arithmetic and contract (no GPU): the
evaluated voxel-pair count against the oracle's count of valid
displacements, the per-axis count against brute force, the one-GPU exit,
and the committed traffic records."""

import json
import os
import subprocess
import sys

import numpy as np

import bench
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_evaluated_pairs_equal_the_oracles_valid_displacements():
    rng = np.random.default_rng(3)
    dims = (40, 33, 27)
    for b, w in [(3, 2), (7, 5), (9, 12)]:
        h = (b - 1) // 2
        c = np.stack([rng.integers(h, d - h, 60) for d in dims], axis=1).astype(np.int32)
        c[:5, 0] = h       # on the low x face
        c[5:10, 2] = 26 - h  # on the high z face
        want = int(oracle.valid_shifts(dims, c, b, w).sum()) * b ** 3
        assert bench.evaluated_pairs(c, dims, b, w) == want


def test_evaluated_pairs_per_axis_by_brute_force():
    dims = np.array([20, 17, 12])
    b, w = np.array([5, 3, 7]), np.array([3, 1, 4])
    h = (b - 1) // 2
    c = np.array([[2, 1, 3], [10, 8, 6], [17, 15, 8], [5, 9, 4]], np.int32)
    total = 0
    for cc in c:
        for dz in range(-w[2], w[2] + 1):
            for dy in range(-w[1], w[1] + 1):
                for dx in range(-w[0], w[0] + 1):
                    lo = cc + np.array([dx, dy, dz]) - h
                    if np.all(lo >= 0) and np.all(lo + b <= dims):
                        total += int(np.prod(b))
    assert bench.evaluated_pairs(c, tuple(dims), tuple(b), tuple(w)) == total


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_records_are_well_formed():
    for (wl, arith), (name, sources) in bench.TRAFFIC_FILES.items():
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
        assert t["workload"] == wl and t["sources"] == sources
        scaled = (t["fetch_kib_per_dispatch"] * 1024 * t["fetch_scale"]
                  + t["write_kib_per_dispatch"] * 1024 * t["write_scale"])
        assert abs(t["traffic_bytes"] - scaled) <= 1e-4 * scaled
        # the scales come from the 256 MiB copy calibration
        assert abs(t["fetch_scale"] - 262144.0 / t["copy_256mib_fetch_kib"]) < 1e-3
        got = bench.measured_traffic(wl, arith)
        assert got is None or got == t["traffic_bytes"]
    assert bench.measured_traffic("no_such_workload", "dot2") is None
