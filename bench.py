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
  4. the Chebyshev power spectrum of the force (degree 64, 16 windows): FP32 stencil sweeps
     with the moments summed in FP64, as for the batched spectra;
  5. a Chebyshev vector filter of the momentum onto 4 windows (degree 32), on a second
     stream beside stages 2-4 (it depends only on the momentum and the links).

`value` is the Laplacian throughput of the whole step: lattice sites times link fields
passed through Delta, divided by the step time (every other kernel of the step counts
against it).  The step time comes from a pass without instrumentation; `roofline` and
`kernel_time_share` from a second pass of the same steps on one stream (the filter after the
spectrum, so no launch shares the chip) with HIP events around every launch.

Extra fields (skipped with --no-extras):
  D1  the Laplacian alone at 16^4, 24^4 and 32^3 x 64, FP64 and FP32 (working sets under the
      256 MB Infinity Cache timed over rotating buffer sets of >= 1 GiB), against 8 TB/s and
      against a measured 1 GiB copy;
  D2  the rational solve alone, time to FP64 true residual 1e-10, FP64 against mixed precision,
      12 poles, kappa 0.9 and 0.5, one and eight momentum fields (median of 5);
  D3  the batched power spectrum at 24^4 (32 sources, degree 256, 64 windows), Haar and U = 1;
  D4  the 8-pole kinetic force at 16^4;
  D5  the full force step at 32^3 x 64: 16-pole kinetic force of 8 momentum fields, then the
      128-window degree-256 power spectrum of the 8 forces, FP64 against mixed precision;
  D6  the backward of the degree-64, 16-window power spectrum at 16^4 (link derivative and source
      gradient) beside its forward;
  D7  the Wilson gauge force and its degree-128, 32-window power spectrum (the gauge-force spectra
      of section 2) at 16^4 and 32^3 x 64;
  D8  one implicit leapfrog step of the non-separable Hamiltonian (kinetic term with the 12-pole
      kappa = 0.9 mass term plus the Wilson action, beta = 5.5, eps = 0.02) at 16^4: time,
      fixed-point iterations, solver iterations, the energy change of the step and the stencil
      launches inside it;
  D9  RMHMC heat-bath momenta P = R(Delta)^-1 xi (12-pole kappa = 0.9 set) at 16^4 and their
      projection onto 4 spectral windows (degree-32 filter), the input of the section-3 momentum
      injection.
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
    from threadpoolctl import threadpool_limits

    from oracle import laplacian as olap
    U = U.numpy()
    P = P.numpy()
    with threadpool_limits(limits=1):   # the one core the figure is quoted for
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
    api.autotune_laplacian(L, Ud, Pd, reps=10)
    api.autotune_laplacian(L, U32, Pd.float(), reps=10)
    # the solver's FP64 true-residual check applies Delta to all 12 shift solutions in one launch
    api.autotune_laplacian(L, Ud, Pd.expand(12, -1, -1, -1).contiguous(), reps=5)
    ws = torch.empty(api.workspace_bytes(6, L, 0, 1, 12, 0, 1), dtype=torch.uint8, device=dev)

    # the momentum filter needs only P and the links: it runs on a second stream (default
    # priority) beside the force and its spectrum, whose short CG kernels leave the GPU room
    side = torch.cuda.Stream(device=dev)

    def step(overlap=True):
        main = torch.cuda.current_stream(dev)
        Uw = api.pack_links(L, U_aos)
        if overlap:
            side.wait_stream(main)
            Uw.record_stream(side)
            with torch.cuda.stream(side):
                api.cheb_filter(L, Uw, Pd, 32, 4)
        out = api.kinetic_force(L, Uw, Pd, rat, solver, ws=ws)
        # spectrum: FP32 stencil sweeps, FP64 moment sums (as the batched spectra)
        api.power_spectrum(L, api.convert_f64_f32(Uw), api.convert_f64_f32(out["dK"]), 64, 16)
        if overlap:
            main.wait_stream(side)
        else:
            api.cheb_filter(L, Uw, Pd, 32, 4)
        return out

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        last = step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        last = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    # the same steps again with HIP events around every launch of the instrumented kernel classes
    # (the events add launch gaps, so the step time above is taken without them), on one stream,
    # so that every launch's duration is its own and not shared with the overlapped filter
    api.profile_enable(True)
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        step(overlap=False)
    torch.cuda.synchronize()
    ms_step_profiled = (time.perf_counter() - tp0) / args.steps * 1e3
    prof = {c: api.profile_read(c) for c in api.PROF_CLASSES}
    api.profile_enable(False)
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
                "launches": d["launches"],
                "measured_over": f"a second pass of the {args.steps} timed steps on one stream with HIP "
                                 f"events ({ms_step_profiled:.3f} ms/step with the events)"}
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
                               "spectrum (FP32 sweeps, FP64 moments), degree-32/4-window FP64 filter of the "
                               "momentum on a second stream",
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


def _median_ms(fn, torch, reps=5):
    """Median wall time of reps calls after one warm-up (each call synchronized)."""
    fn()
    torch.cuda.synchronize()
    ts = []
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return ts[len(ts) // 2], out


def copy_bandwidth(torch, dev):
    """Plain 1 GiB device copy: the bandwidth the memory system delivers to a streaming kernel."""
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    ms, _ = _median_ms(lambda: b.copy_(a), torch, reps=5)
    del a, b
    return {"bytes": 2 * (1 << 30), "ms": round(ms, 4), "GBs": round(2 * (1 << 30) / (ms * 1e-3) / 1e9, 1)}


def d1_laplacian(api, inputs, torch, dev, copy_gbs):
    """Laplacian on one link field: 16^4, 24^4, 32^3x64, FP64 and FP32, eps=0.4 links.  A working
    set under 256 MB (the Infinity Cache) is timed over rotating buffer sets of >= 1 GiB."""
    out = {}
    for L in ((16, 16, 16, 16), (24, 24, 24, 24), (32, 32, 32, 64)):
        V = api.volume(L)
        U = inputs.random_links(L, "eps", 0.4, seed=1).to(dev)
        F = inputs.gaussian_fields(L, 1, seed=1).to(dev)
        for dt, name, ts in ((torch.float64, "fp64", 8), (torch.float32, "fp32", 4)):
            Ud = api.pack_links(L, U, dt)
            Fd = F.to(dt)
            cfg, _ = api.autotune_laplacian(L, Ud, Fd, reps=3)
            set_bytes = 136 * ts * V   # buffers of one set: links (18 reals), input and output
            nset = 1 if set_bytes >= (256 << 20) else -(-(1 << 30) // set_bytes)
            sets = [(Ud, Fd, torch.empty_like(Fd))]
            for _ in range(nset - 1):
                sets.append((Ud.clone(), Fd.clone(), torch.empty_like(Fd)))
            reps = max(20, 2 * nset)
            for k in range(nset):
                api.laplacian_apply(L, sets[k][0], sets[k][1], out=sets[k][2])
            torch.cuda.synchronize()
            api.profile_enable(True)
            for r in range(reps):
                u, x, y = sets[r % nset]
                api.laplacian_apply(L, u, x, out=y)
            torch.cuda.synchronize()
            p = api.profile_read("stencil")
            api.profile_enable(False)
            gsite = V / (p["avg_ms"] * 1e-3) / 1e9
            key = "x".join(map(str, L))
            out.setdefault(key, {})[name] = {
                "gsite_s": round(gsite, 3), "avg_ms": round(p["avg_ms"], 4), "achieved_GBs": round(p["gbs"], 1),
                "hbm_frac": round(p["gbs"] / HBM_PEAK_GBS, 4), "copy_frac": round(p["gbs"] / copy_gbs, 4),
                "bytes_per_site": 112 * ts, "rotating_sets": nset,
                "config": dict(zip(("form", "block", "xcd_remap", "nv", "order", "walk"), cfg))}
            log(f"D-1 {key} {name}: {out[key][name]}")
            del sets, Ud, Fd
        del U, F
    return out


def d2_solves(api, inputs, torch, dev, L, Ud, Pd):
    """Rational solve alone, time to FP64 true residual 1e-10: FP64 against mixed precision."""
    solves = {}
    P8 = inputs.gaussian_fields(L, 8, seed=22).to(dev)
    for kappa in (0.9, 0.5):
        rat = api.rational_kappa(kappa, 12)
        for n, src in ((1, Pd), (8, P8)):
            row = {}
            for mode, name in ((0, "fp64"), (1, "mixed")):
                sv = api.Solver(tol=1e-10, mode=mode)
                ms, o = _median_ms(lambda: api.rational_apply(L, Ud, src, rat, sv), torch)
                st = o["stats"]
                row[f"{name}_ms"] = round(ms, 3)
                row[f"{name}_iters"] = st["iters"]
                row[f"{name}_fp64_iters"] = st["fp64_iters"]
                row[f"{name}_refine_iters"] = st["refine_iters"]
                row[f"{name}_true_relres_max"] = st["true_relres_max"]
                if mode == 1:
                    row["mixed_reliable_updates"] = st["reliable_updates"]
            row["mixed_speedup"] = round(row["fp64_ms"] / row["mixed_ms"], 3)
            solves[f"kappa{kappa}_nrhs{n}"] = row
            log(f"D-2 solve kappa={kappa} n={n}: {row}")
    return solves


def d3_spectrum(api, inputs, torch, dev):
    """Batched power spectrum at 24^4: 32 Gaussian sources, degree 256, 64 windows, FP32 stencil
    with FP64 moments; Haar links and the U = 1 control."""
    L = (24, 24, 24, 24)
    out = {}
    F = inputs.gaussian_fields(L, 32, seed=3).to(dev).float()
    for kind in ("haar", "unit"):
        U32 = api.pack_links(L, inputs.random_links(L, kind, seed=3).to(dev), torch.float32)
        api.autotune_laplacian(L, U32, F, reps=2)
        api.power_spectrum(L, U32, F, 256, 64)
        torch.cuda.synchronize()
        api.profile_enable(True)
        t0 = time.perf_counter()
        api.power_spectrum(L, U32, F, 256, 64)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        p = api.profile_read("stencil")
        api.profile_enable(False)
        out[kind] = {"ms": round(ms, 3), "sweeps": p["launches"], "stencil_ms": round(p["ms"], 3),
                     "stencil_GBs": round(p["gbs"], 1), "hbm_frac": round(p["gbs"] / HBM_PEAK_GBS, 4),
                     "gsite_rhs_s": round(api.volume(L) * p["items"] / (ms * 1e-3) / 1e9, 3)}
        log(f"D-3 spectrum 24^4 {kind}: {out[kind]}")
        del U32
    return out


def d4_force(api, inputs, torch, dev):
    """Kinetic force at 16^4, eps=0.4: 8 poles kappa=0.9, both solves to 1e-10, link derivative."""
    L = (16, 16, 16, 16)
    Ud = api.pack_links(L, inputs.random_links(L, "eps", 0.4, seed=4).to(dev))
    P = inputs.gaussian_fields(L, 1, seed=4).to(dev)
    rat = api.rational_kappa(0.9, 8)
    row = {}
    for mode, name in ((0, "fp64"), (1, "mixed")):
        sv = api.Solver(tol=1e-10, mode=mode)
        ms, o = _median_ms(lambda: api.kinetic_force(L, Ud, P, rat, sv), torch)
        row[f"{name}_ms"] = round(ms, 3)
        row[f"{name}_iters"] = o["stats"]["iters"]
    row["mixed_speedup"] = round(row["fp64_ms"] / row["mixed_ms"], 3)
    log(f"D-4 force 16^4: {row}")
    return row


def d5_force_step(api, inputs, torch, dev):
    """Full force step at 32^3 x 64, eps=0.4: for 8 momentum fields (two per call), the 16-pole
    kappa=0.9 kinetic force (two multi-shift solves to 1e-10 and the link derivative), then the
    128-window degree-256 power spectrum of the 8 forces (FP32 stencil, FP64 moments)."""
    L = (32, 32, 32, 64)
    V = api.volume(L)
    U = inputs.random_links(L, "eps", 0.4, seed=5).to(dev)
    Ud = api.pack_links(L, U)
    U32 = api.pack_links(L, U, torch.float32)
    del U
    P = inputs.gaussian_fields(L, 8, seed=5).to(dev)
    rat = api.rational_kappa(0.9, 16)
    need = max(api.workspace_bytes(6, L, 0, 2, 16, 0, m) for m in (0, 1))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    row = {"workspace_GiB": round(need / 2**30, 1)}
    for mode, name in ((0, "fp64"), (1, "mixed")):
        sv = api.Solver(tol=1e-10, mode=mode)
        forces = torch.empty((8, 4, 8, V), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        api.profile_enable(True)
        t0 = time.perf_counter()
        iters = 0
        for c in range(4):
            o = api.kinetic_force(L, Ud, P[2 * c:2 * c + 2], rat, sv, per_rhs=True, ws=ws)
            forces[2 * c:2 * c + 2] = o["dK"].float()
            iters += o["stats"]["iters"]
            del o
        t1 = time.perf_counter()
        api.power_spectrum(L, U32, forces, 256, 128)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        prof = {c: api.profile_read(c) for c in api.PROF_CLASSES}
        api.profile_enable(False)
        row[name] = {"ms_per_force": round((t1 - t0) * 1e3 / 8, 3), "spectrum_ms": round((t2 - t1) * 1e3, 3),
                     "total_ms": round((t2 - t0) * 1e3, 3), "solver_iters": iters,
                     "stencil_GBs": round(prof["stencil"]["gbs"], 1),
                     "stencil_hbm_frac": round(prof["stencil"]["gbs"] / HBM_PEAK_GBS, 4),
                     "kernel_ms": {c: round(prof[c]["ms"], 2) for c in prof}}
        log(f"D-5 force step 32^3x64 {name}: {row[name]}")
        del forces
    row["mixed_speedup"] = round(row["fp64"]["total_ms"] / row["mixed"]["total_ms"], 3)
    del ws
    return row


def d6_spectrum_bwd(api, inputs, torch, np, dev):
    """Backward of the power spectrum (link derivative and source gradient) at 16^4, eps=0.5,
    degree 64, 16 windows: the reverse Chebyshev sweep (3 x 64 stencil sweeps, 64 derivative passes)."""
    L = (16, 16, 16, 16)
    Ud = api.pack_links(L, inputs.random_links(L, "eps", 0.5, seed=6).to(dev))
    F = inputs.gaussian_fields(L, 1, seed=6).to(dev)
    gamma = np.ones((1, 16))
    fwd_ms, _ = _median_ms(lambda: api.power_spectrum(L, Ud, F, 64, 16), torch)
    bwd_ms, _ = _median_ms(lambda: api.power_spectrum_bwd(L, Ud, F, gamma, 64, 16), torch)
    api.profile_enable(True)
    api.power_spectrum_bwd(L, Ud, F, gamma, 64, 16)
    torch.cuda.synchronize()
    prof = {c: api.profile_read(c) for c in ("stencil", "force")}
    api.profile_enable(False)
    row = {"forward_ms": round(fwd_ms, 3), "backward_ms": round(bwd_ms, 3),
           "stencil": {"launches": prof["stencil"]["launches"], "GBs": round(prof["stencil"]["gbs"], 1)},
           "force": {"launches": prof["force"]["launches"], "GBs": round(prof["force"]["gbs"], 1)}}
    log(f"D6 power spectrum backward 16^4: {row}")
    return row


def d7_gauge_force_spectrum(api, inputs, torch, dev):
    """The gauge-force spectra of section 2 (Fig. 1 workload) on synthetic links: Wilson force
    (beta = 6.4) and its power spectrum, degree 128 and 32 windows, at 16^4 and 32^3 x 64."""
    out = {}
    for L in ((16, 16, 16, 16), (32, 32, 32, 64)):
        V = api.volume(L)
        Ud = api.pack_links(L, inputs.random_links(L, "eps", 0.4, seed=7).to(dev))
        f_ms, (F, _) = _median_ms(lambda: api.wilson_gauge_force(L, Ud, 6.4, want_action=False), torch)
        Fb = F[None].contiguous()
        s_ms, _ = _median_ms(lambda: api.power_spectrum(L, Ud, Fb, 128, 32), torch, reps=3)
        key = "x".join(map(str, L))
        out[key] = {"force_ms": round(f_ms, 4), "force_GBs": round(V * 104 * 8 / (f_ms * 1e-3) / 1e9, 1),
                    "spectrum_ms": round(s_ms, 3)}
        log(f"D7 gauge force + spectrum {key}: {out[key]}")
        del Ud, F, Fb
    return out


def d8_leapfrog(api, inputs, torch, dev):
    """One implicit leapfrog step at 16^4 (eps-links 0.5, one Gaussian momentum field)."""
    L = (16, 16, 16, 16)
    Ud = api.pack_links(L, inputs.random_links(L, "eps", 0.5, seed=8).to(dev))
    Pd = inputs.gaussian_fields(L, 1, seed=8)[0].to(dev)
    rat = api.rational_kappa(0.9, 12)
    sv = api.Solver(tol=1e-10)
    beta, eps = 5.5, 0.02
    ws = torch.empty(api.workspace_bytes(api.L_.OP_LEAPFROG, L, api.RMH_F64, 1, 12), dtype=torch.uint8, device=dev)
    ms, (U1, P1, st) = _median_ms(lambda: api.leapfrog_step(L, Ud, Pd, rat, eps, beta, sv, fp_tol=1e-10, ws=ws),
                                  torch, reps=3)
    api.profile_enable(True)
    api.leapfrog_step(L, Ud, Pd, rat, eps, beta, sv, fp_tol=1e-10, ws=ws)
    torch.cuda.synchronize()
    p = api.profile_read("stencil")
    api.profile_enable(False)

    def ham(U, P):
        K = api.rational_apply(L, U, P[None], rat, api.Solver(tol=1e-12))["K"][0]
        return float(K) + api.wilson_gauge_force(L, U, beta)[1]

    out = {"ms_per_step": round(ms, 2), "p_iters": st["p_iters"], "u_iters": st["u_iters"],
           "solver_iters": st["solver"]["iters"], "true_relres_max": st["solver"]["true_relres_max"],
           "dH": ham(U1, P1) - ham(Ud, Pd), "stencil": {"launches": p["launches"], "ms": round(p["ms"], 2),
                                                        "GBs": round(p["gbs"], 1)}}
    log(f"D8 leapfrog step 16^4: {out}")
    return out


def d9_heatbath(api, inputs, torch, dev):
    """Heat-bath momenta and their window projection at 16^4 (one Gaussian field)."""
    L = (16, 16, 16, 16)
    Ud = api.pack_links(L, inputs.random_links(L, "eps", 0.5, seed=9).to(dev))
    xi = inputs.gaussian_fields(L, 1, seed=9).to(dev)
    rat = api.rational_kappa(0.9, 12)
    sv = api.Solver(tol=1e-10)
    hb_ms, out = _median_ms(lambda: api.heatbath_momenta(L, Ud, xi, 0.9, rat, sv), torch)
    P = out["P"]
    f_ms, _ = _median_ms(lambda: api.cheb_filter(L, Ud, P, 32, 4), torch)
    res = {"heatbath_ms": round(hb_ms, 3), "solver_iters": out["stats"]["iters"],
           "true_relres_max": out["stats"]["true_relres_max"], "filter_ms": round(f_ms, 3)}
    log(f"D9 heat-bath momenta + window projection 16^4: {res}")
    return res


def run_extras(api, inputs, torch, np, dev, L, U_aos, Ud, Pd):
    out = {}
    cp = copy_bandwidth(torch, dev)
    out["copy_1GiB"] = cp
    log(f"copy: {cp}")
    out["D1_laplacian"] = d1_laplacian(api, inputs, torch, dev, cp["GBs"])
    out["D2_rational_solve_time_to_1e-10"] = d2_solves(api, inputs, torch, dev, L, Ud, Pd)
    out["D3_power_spectrum_24x24x24x24"] = d3_spectrum(api, inputs, torch, dev)
    out["D4_kinetic_force_16x16x16x16"] = d4_force(api, inputs, torch, dev)
    out["D5_force_step_32x32x32x64"] = d5_force_step(api, inputs, torch, dev)
    out["D6_power_spectrum_bwd_16x16x16x16"] = d6_spectrum_bwd(api, inputs, torch, np, dev)
    out["D7_gauge_force_spectrum"] = d7_gauge_force_spectrum(api, inputs, torch, dev)
    out["D8_leapfrog_step_16x16x16x16"] = d8_leapfrog(api, inputs, torch, dev)
    out["D9_heatbath_projection_16x16x16x16"] = d9_heatbath(api, inputs, torch, dev)
    return out


if __name__ == "__main__":
    main()
