"""Host-side checks of bench.py's bookkeeping (no GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_peak_in_flight():
    assert bench.peak_in_flight([]) == 0
    assert bench.peak_in_flight([(0, 1), (1, 2), (2, 3)]) == 1  # back to back: one at a time
    assert bench.peak_in_flight([(0, 10), (1, 2), (1.5, 3), (5, 6)]) == 3


def test_measured_traffic_follows_the_kernel_source():
    path = os.path.join(ROOT, "profiles", "si512_mixed_hbm_traffic.json")
    with open(path) as f:
        d = json.load(f)
    t = bench.measured_traffic("si512", d["mixed_flags"], "nl")
    k = d["kernels"]["nl"]
    want = 1024.0 * (k["FETCH_SIZE_KiB"] * d["scale"]["FETCH_SIZE"] + k["WRITE_SIZE_KiB"] * d["scale"]["WRITE_SIZE"])
    import hashlib
    with open(os.path.join(ROOT, d["source"]), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == d["source_sha256"]
    assert (t == want) if current else (t is None)
    assert bench.measured_traffic("si512", d["mixed_flags"] ^ 1, "nl") is None
    assert bench.measured_traffic("si4096", d["mixed_flags"], "nl") is None
