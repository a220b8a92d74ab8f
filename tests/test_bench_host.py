"""Host-side pieces of bench.py (CPU): the one-GPU guard, the committed HBM-traffic figure and the
CPU baseline's record."""
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2112_04556_amd.profiling import stencil_source_hash

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_stencil_traffic_record():
    """The committed counter summaries of the headline kernel parse, and bench reports a figure only
    for a profiled launch configuration while the stencil sources hash to the value stamped in it."""
    assert bench.stencil_traffic("stencil", "no_such_record.json") == (None, None)
    recs = bench.traffic_records()
    assert recs and all(r["traffic_bytes_per_launch"] > 0 and len(r["launch_config"]) == 8 for r in recs)
    assert bench.stencil_traffic("force") == (None, None)
    for t in recs:
        val, src = bench.stencil_traffic("stencil", cfg=t["launch_config"])
        if t["stencil_source_sha256"] == stencil_source_hash():
            assert val == round(float(t["traffic_bytes_per_launch"])) and src.startswith("profiles")
        else:
            assert val is None and "stale" in src
    other = list(recs[0]["launch_config"])
    other[1] = 64 if other[1] != 64 else 128
    v2, s2 = bench.stencil_traffic("stencil", cfg=other)
    assert v2 is None and "launch configuration" in s2


def test_cpu_baseline_record():
    """The baseline leg times the oracle's Laplacian on one core and on the host cores (forked
    workers) and the oracle's per-shift CG, and reports Gsite/s with the core count (tiny lattices
    here; the bench runs it on the 32^3 x 64 workload)."""
    rec = bench.cpu_baseline(budget_s=0.05, Lb=(4, 4, 4, 8), L16=(2, 2, 2, 4), chunk=64)
    assert rec["unit"] == "Gsite/s" and rec["kind"] == "oracle"
    assert 1 <= rec["cores"] <= 16
    assert np.isfinite(rec["value"]) and rec["value"] > 0
    one = rec["single_core"]
    assert one["cores"] == 1 and one["value"] > 0
    cg = rec["cg_iteration"]
    assert cg["one_shift_one_core_ms"] > 0 and cg["twelve_shifts_all_cores_ms"] > 0
