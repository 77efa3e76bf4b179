"""Host-side checks of bench.py's helpers (no GPU): the learned closure's scaling ranges, the
--gpus guard, and the traffic lookup keyed by kernel source hash."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_feature_range_pads_spans_and_constant_inputs():
    import torch
    import bench
    x = torch.tensor([[1.0, 0.0078125, 3.0], [2.0, 0.0078125, 5.0]], dtype=torch.float32)
    lo, hi = bench.feature_range(torch, x)
    # a quarter of the span on each side, plus at least 1e-5 of the value's size
    assert np.allclose(lo, [1.0 - 0.25 - 1e-5 * 2.0, 0.0078125 - 1e-5, 3.0 - 0.5 - 1e-5 * 5.0])
    assert np.allclose(hi, [2.0 + 0.25 + 1e-5 * 2.0, 0.0078125 + 1e-5, 5.0 + 0.5 + 1e-5 * 5.0])
    # a constant input's float32 rounding (relative 6e-8) stays well inside its range
    d64 = np.float64(0.0078125) * (1 + 6e-8)
    assert lo[1] < d64 < hi[1] and (d64 - lo[1]) / (hi[1] - lo[1]) < 0.6


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_traffic_entries_match_their_sources():
    """Every counter-derived traffic entry names a kernel source file of the package and the
    workload it was measured on; the lookup returns it only while the hash matches."""
    import bench
    data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert data
    for key, ent in data.items():
        src = os.path.join(ROOT, "paper_2411_09364_amd", "csrc", ent["source"])
        assert os.path.exists(src), key
        assert ent["bytes_per_launch"] > 0 and ent["workload"]
    names = {c["name"] for c in bench.CONFIGS.values()}
    assert all(ent["workload"] in names for ent in data.values())
