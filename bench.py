#!/usr/bin/env python3
"""Benchmark of the adjoint-Laplacian hot path on one MI355X.

One step is one RMHMC kinetic-force evaluation on the 16^4 lattice with eps = 0.5 links
(the lattice, link ensemble and 12-pole (1 - kappa + kappa Delta)^-1-type rational of
the rational-solve workload, kappa = 0.9), through every stage of the path:

  1. ingest: pack the links into the SoA layout (FP64) and, inside the solver, FP32;
  2. forward: multi-shift CG for R(Delta) P to FP64 true residual 1e-10 on every shift,
     FP32 stencil and vectors with FP64 reliable updates, Y = R(Delta) P, K = 1/2 <Y, Y>;
  3. backward: second multi-shift solve z_j = (Delta + sigma_j)^-1 Y and the link
     derivative dK/d omega (the mass-term force, section 3);
  4. the Chebyshev power spectrum of the force (degree 64, 16 windows, FP64 moments);
  5. a Chebyshev vector filter of the momentum onto 4 windows (degree 32).

`value` is the Laplacian throughput of the whole step: lattice sites times link fields
passed through Delta, divided by the step time (every other kernel of the step counts
against it).  Extra fields report the time to 1e-10 of the rational solve alone, FP64
against mixed precision, for one and eight momentum fields, and the stencil on the
32^3 x 64 lattice, where the working set exceeds every cache.
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

HBM_PEAK_GBS = 8000.0
METRIC = "Laplacian Gsite/s & %HBM peak; rational-solve time to 1e-10, mixed vs FP64"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed force steps")
    ap.add_argument("--kappa", type=float, default=0.9)
    return ap.parse_args()


def cpu_baseline(U, P, L, budget_s=12.0):
    """The oracle's stencil on the same 16^4 field, repeated for about budget_s seconds."""
    from oracle import laplacian as olap
    U = U.numpy()
    P = P.numpy()
    olap.laplacian(U, P, L)             # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        olap.laplacian(U, P, L)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    V = L[0] * L[1] * L[2] * L[3]
    return {"value": V * n / dt / 1e9, "unit": "Gsite/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} applications of the oracle's Laplacian (numpy FP64, literal 3x3 products, "
                      f"single thread) to the 16^4 momentum field in {dt:.1f} s; stencil only, so it "
                      f"overstates the oracle's rate for the whole step"}


def stencil_traffic(kernel_class):
    """HBM bytes per stencil launch of this step from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a calibration copy), or None when the summary is
    missing or the stencil sources have changed since it was taken."""
    if kernel_class != "stencil":
        return None, None
    path = os.path.join(ROOT, "profiles", "stencil_traffic_16x16x16x16.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    from paper_2112_04556_amd.profiling import stencil_source_hash
    rel = os.path.relpath(path, ROOT)
    if t.get("stencil_source_sha256") != stencil_source_hash():
        return None, rel + " (stale: stencil sources changed)"
    return round(float(t["traffic_bytes_per_launch"])), rel


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(sharding across GPUs is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2112_04556_amd import api, inputs

    dev = torch.device("cuda:0")
    L = (16, 16, 16, 16)
    V = api.volume(L)
    log("generating inputs")
    U = inputs.random_links(L, "eps", 0.5, seed=2)
    P = inputs.gaussian_fields(L, 1, seed=2)
    U_aos = U.to(dev)
    Pd = P.to(dev)
    rat = api.rational_kappa(args.kappa, 12)
    solver = api.Solver(tol=1e-10, mode=1)

    # stencil launch configurations for the shapes of the step (outside the timed region)
    Ud = api.pack_links(L, U_aos)
    U32 = api.pack_links(L, U_aos, torch.float32)
    api.autotune_laplacian(L, Ud, Pd, reps=3)
    api.autotune_laplacian(L, U32, Pd.float(), reps=3)
    ws = torch.empty(api.workspace_bytes(6, L, 0, 1, 12, 0, 1), dtype=torch.uint8, device=dev)

    def step():
        Uw = api.pack_links(L, U_aos)
        out = api.kinetic_force(L, Uw, Pd, rat, solver, ws=ws)
        api.power_spectrum(L, Uw, out["dK"], 64, 16)
        api.cheb_filter(L, Uw, Pd, 32, 4)
        return out

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        last = step()
    torch.cuda.synchronize()
    api.profile_enable(True)
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        last = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {c: api.profile_read(c) for c in api.PROF_CLASSES}
    api.profile_enable(False)
    ms_step = (t1 - t0) / args.steps * 1e3
    fields_per_step = prof["stencil"]["items"] / args.steps
    value = V * fields_per_step / (ms_step * 1e-3) / 1e9
    log(f"{ms_step:.2f} ms/step, {fields_per_step:.0f} link-field stencil applications per step")

    # dominant kernel class of the step by event time
    dom = max(prof, key=lambda c: prof[c]["ms"])
    d = prof[dom]
    traffic, traffic_src = stencil_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": traffic_src,
                "avg_launch_ms": d["avg_ms"], "bytes_per_launch": d["bytes"] / max(d["launches"], 1),
                "launches": d["launches"]}
    shares = {c: round(prof[c]["ms"] / max(sum(p["ms"] for p in prof.values()), 1e-12), 4) for c in prof}

    extras = {}
    if not args.no_extras:
        extras = run_extras(api, inputs, torch, np, dev, L, U_aos, Ud, Pd)

    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gsite/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "RMHMC kinetic-force evaluation, 16^4 lattice, eps=0.5 links (seed 2), "
                               f"one Gaussian momentum field, 12-pole kappa={args.kappa} rational to FP64 true "
                               "residual 1e-10 (FP32 + FP64 reliable updates), force, degree-64/16-window power "
                               "spectrum, degree-32/4-window filter",
                   "lattice": list(L), "n_rhs": 1, "poles": 12, "kappa": args.kappa,
                   "value_definition": "sites x link fields through Delta per second, whole step"},
        "roofline": roofline,
        "kernel_time_share": shares,
        "stats_last_step": last["stats"],
        **extras,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(U, P, L)
    print(json.dumps(result), flush=True)


def run_extras(api, inputs, torch, np, dev, L, U_aos, Ud, Pd):
    out = {}
    # rational solve alone: time to 1e-10, FP64 against mixed, 1 and 8 momentum fields
    solves = {}
    P8 = inputs.gaussian_fields(L, 8, seed=22).to(dev)
    for kappa in (0.9, 0.5):
        rat = api.rational_kappa(kappa, 12)
        for n, src in ((1, Pd), (8, P8)):
            row = {}
            for mode, name in ((0, "fp64"), (1, "mixed")):
                sv = api.Solver(tol=1e-10, mode=mode)
                api.rational_apply(L, Ud, src, rat, sv)          # warm-up (workspace, tuner)
                torch.cuda.synchronize()
                reps = 3
                t0 = time.perf_counter()
                for _ in range(reps):
                    o = api.rational_apply(L, Ud, src, rat, sv)
                torch.cuda.synchronize()
                row[f"{name}_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
                st = o["stats"]
                row[f"{name}_iters"] = st["iters"]
                row[f"{name}_refine_iters"] = st["refine_iters"]
                row[f"{name}_true_relres_max"] = st["true_relres_max"]
                if mode == 1:
                    row["mixed_reliable_updates"] = st["reliable_updates"]
            row["mixed_speedup"] = round(row["fp64_ms"] / row["mixed_ms"], 3)
            solves[f"kappa{kappa}_nrhs{n}"] = row
            log(f"solve kappa={kappa} n={n}: {row}")
    out["rational_solve_time_to_1e-10"] = solves
    del P8

    # the stencil where nothing is cache resident: 32^3 x 64, FP64 and FP32
    Lb = (32, 32, 32, 64)
    Vb = api.volume(Lb)
    log("generating 32^3x64 inputs")
    Ub = inputs.random_links(Lb, "haar", seed=5).to(dev)
    Fb = inputs.gaussian_fields(Lb, 1, seed=5).to(dev)
    sten = {}
    for dt, name, ts in ((torch.float64, "fp64", 8), (torch.float32, "fp32", 4)):
        Ubd = api.pack_links(Lb, Ub, dt)
        Fbd = Fb.to(dt)
        cfg, _ = api.autotune_laplacian(Lb, Ubd, Fbd, reps=3)
        y = torch.empty_like(Fbd)
        for _ in range(3):
            api.laplacian_apply(Lb, Ubd, Fbd, out=y)
        torch.cuda.synchronize()
        api.profile_enable(True)
        reps = 20
        for _ in range(reps):
            api.laplacian_apply(Lb, Ubd, Fbd, out=y)
        torch.cuda.synchronize()
        p = api.profile_read("stencil")
        api.profile_enable(False)
        gsite = Vb / (p["avg_ms"] * 1e-3) / 1e9
        sten[name] = {"gsite_s": round(gsite, 3), "avg_ms": round(p["avg_ms"], 4),
                      "achieved_GBs": round(p["gbs"], 1), "hbm_frac": round(p["gbs"] / HBM_PEAK_GBS, 4),
                      "bytes_per_site": 136 * ts,
                      "config": {"form": cfg[0], "block": cfg[1], "xcd_remap": cfg[2], "nv": cfg[3],
                                 "order": cfg[4], "walk": cfg[5]}}
        log(f"stencil 32^3x64 {name}: {sten[name]}")
        del Ubd, Fbd, y
    out["laplacian_32x32x32x64"] = sten

    # the rational solve where nothing is cache resident: 16 poles, one momentum field
    rat16 = api.rational_kappa(0.9, 16)
    Ubd = api.pack_links(Lb, inputs.random_links(Lb, "eps", 0.4, seed=2).to(dev))
    Pb = inputs.gaussian_fields(Lb, 1, seed=2).to(dev)
    row = {}
    for mode, name in ((0, "fp64"), (1, "mixed")):
        sv = api.Solver(tol=1e-10, mode=mode)
        api.rational_apply(Lb, Ubd, Pb, rat16, sv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = api.rational_apply(Lb, Ubd, Pb, rat16, sv)
        torch.cuda.synchronize()
        row[f"{name}_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        st = o["stats"]
        row[f"{name}_iters"] = st["iters"]
        row[f"{name}_refine_iters"] = st["refine_iters"]
        row[f"{name}_true_relres_max"] = st["true_relres_max"]
    row["mixed_speedup"] = round(row["fp64_ms"] / row["mixed_ms"], 3)
    out["rational_solve_32x32x32x64_kappa0.9_16poles"] = row
    log(f"solve 32^3x64: {row}")
    return out


if __name__ == "__main__":
    main()
