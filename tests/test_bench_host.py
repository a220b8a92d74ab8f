"""Host-side pieces of bench.py (CPU): the one-GPU guard, the committed HBM-traffic figure and the
CPU baseline's record."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2112_04556_amd import inputs
from paper_2112_04556_amd.profiling import stencil_source_hash

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_stencil_traffic_record():
    """The committed counter summary parses, and bench reports its figure only while the stencil
    sources hash to the value stamped in it."""
    path = os.path.join(ROOT, "profiles", "stencil_traffic_16x16x16x16.json")
    with open(path) as fh:
        t = json.load(fh)
    assert t["traffic_bytes_per_launch"] > 0
    val, src = bench.stencil_traffic("stencil")
    if t["stencil_source_sha256"] == stencil_source_hash():
        assert val == round(float(t["traffic_bytes_per_launch"])) and src.startswith("profiles")
    else:
        assert val is None and "stale" in src
    assert bench.stencil_traffic("force") == (None, None)


def test_cpu_baseline_record():
    """The baseline leg times the oracle's stencil on one core and reports Gsite/s."""
    L = (4, 4, 4, 4)
    U = inputs.random_links(L, "eps", 0.5, seed=2)
    P = inputs.gaussian_fields(L, 1, seed=2)[0]
    rec = bench.cpu_baseline(U, P, L, budget_s=0.05)
    assert rec["unit"] == "Gsite/s" and rec["cores"] == 1 and rec["kind"] == "oracle"
    assert np.isfinite(rec["value"]) and rec["value"] > 0
