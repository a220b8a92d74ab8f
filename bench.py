#!/usr/bin/env python3
"""Benchmark of the adjoint-Laplacian hot path on one MI355X.

The metric has two halves: the Laplacian's throughput (Gsite/s and its fraction of the HBM peak)
and the rational solve's time to an FP64 true residual of 1e-10, mixed precision against FP64.

Timed step (the JSON line's `value`, `ms_per_step`, `roofline`): one application of Delta to one
su(3) link field on the largest single-GPU lattice of the workloads, 32^3 x 64 (2.1M sites,
eps = 0.4 links, FP64, launch configuration autotuned beforehand); inputs resident in HBM, W
untimed and K timed applications.  `value` = sites x applications / wall time (Gsite/s);
`roofline` = the kernel's algorithmic bytes (links once, 12 reals per link; input and output once:
896 B per site) over its HIP-event average launch time, against 8 TB/s, with the HBM traffic the
committed rocprofv3 counters show for that kernel while its sources are unchanged.

Second half (`rational_solve`): the 16^4 rational-solve workload (eps = 0.5 links, 12-pole
(1 - kappa + kappa Delta)^-1-type rational, kappa 0.9 and 0.5, one and eight Gaussian fields),
time from the call to every shift's FP64 true residual <= 1e-10, FP64 against mixed precision
(FP32 stencil and vectors with FP64 reliable updates), median of 5.

`hot_path_step`: one pass of every stage of the path on the 16^4 workload: pack the links, the
12-pole kappa = 0.9 kinetic force (both multi-shift solves to 1e-10 in mixed precision and the link
derivative), the degree-64/16-window power spectrum of the force (FP32 sweeps, FP64 moments) and a
degree-32/4-window filter of the momentum on a second stream.

Extra fields (skipped with --no-extras):
  D1  the Laplacian alone at 16^4, 24^4 and 32^3 x 64, FP64 and FP32 (working sets under the
      256 MB Infinity Cache timed over rotating buffer sets of >= 1 GiB), against 8 TB/s and
      against a measured 1 GiB copy;
  D3  the batched power spectrum at 24^4 (32 sources, degree 256, 64 windows), Haar and U = 1;
  D4  the 8-pole kinetic force at 16^4;
  D5  the full force step at 32^3 x 64: 16-pole kinetic force of 8 momentum fields, then the
      128-window degree-256 power spectrum of the 8 forces, FP64 against mixed precision;
  D6  the backward of the degree-64, 16-window power spectrum at 16^4 (link derivative and source
      gradient) beside its forward;
  D7  the Wilson gauge force and its degree-128, 32-window power spectrum (the gauge-force spectra
      of section 2) at 16^4 and 32^3 x 64;
  D8  one implicit leapfrog step of the non-separable Hamiltonian (kinetic term with the 12-pole
      kappa = 0.9 mass term plus the Wilson action, beta = 5.5, eps = 0.02) at 16^4;
  D9  RMHMC heat-bath momenta P = R(Delta)^-1 xi (12-pole kappa = 0.9 set) at 16^4, as
      (1 - kappa + kappa Delta) R(Delta) xi and exactly through the partial fractions of 1/R, and
      their projection onto 4 spectral windows (degree-32 filter).
`cpu_baseline`: the oracle timed on the host cores (see cpu_baseline).
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
    ap.add_argument("--steps", type=int, default=100, help="timed Laplacian applications")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--steps-hot", type=int, default=10, help="timed passes of the whole hot path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the per-component figures")
    ap.add_argument("--headline-config", type=int, nargs=8, default=None,
                    metavar=("FORM", "BLOCK", "XCD", "NV", "ORDER", "WALK", "NS", "TILE2"),
                    help="launch the headline stencil with this configuration instead of the autotuner's")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed Laplacian applications (the profiled command of the headline kernel)")
    ap.add_argument("--kappa", type=float, default=0.9)
    return ap.parse_args()


# ---- the CPU-baseline leg: the only code of this file that runs the oracle ----

_CPU = {}   # inputs of the oracle timing, shared with forked workers (copy-on-write)


def _host_cores():
    """The host cores this process may use (the machine's CPU share), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_lap_chunk(bounds):
    """Worker: the oracle's site-by-site Laplacian on sites [lo, hi), one thread."""
    from threadpoolctl import threadpool_limits

    import numpy as np
    from oracle import laplacian as olap
    lo, hi = bounds
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        olap.laplacian_at(_CPU["U"], _CPU["P"], _CPU["L"], np.arange(lo, hi))
        return hi - lo, time.perf_counter() - t0


def _oracle_cg_iters(args):
    """Worker: k iterations of the oracle's per-shift CG on the 16^4 field for one shift, one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import rational as orat
    sigma, k = args
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        orat.cg_solve(_CPU["U16"], _CPU["P16"][0], _CPU["L16"], sigma, tol=1e-30, maxiter=k)
        return k, time.perf_counter() - t0


def cpu_baseline(budget_s=6.0, Lb=(32, 32, 32, 64), L16=(16, 16, 16, 16), chunk=16384):
    """The oracle (numpy FP64, as it stands) on the host cores, before the GPU is touched:

    * the Laplacian of the headline workload (one link field, 32^3 x 64, eps = 0.4 links), the
      site-by-site form laplacian_at over chunks of 16384 sites: one core, then every core of the
      box's share in a pool of forked single-threaded workers;
    * per-shift CG iterations (the oracle's solver: one Delta and the vector updates per iteration) on
      the 16^4 field of the rational-solve workload: one core, then the 12 shifts of the 12-pole set
      in parallel."""
    import multiprocessing as mp

    from oracle import rational as orat
    from paper_2112_04556_amd import inputs
    Vb = Lb[0] * Lb[1] * Lb[2] * Lb[3]
    _CPU.update(L=Lb, U=inputs.random_links(Lb, "eps", 0.4, seed=1).numpy(),
                P=inputs.gaussian_fields(Lb, 1, seed=1).numpy())
    _CPU.update(L16=L16, U16=inputs.random_links(L16, "eps", 0.5, seed=2).numpy(),
                P16=inputs.gaussian_fields(L16, 1, seed=2).numpy())
    cores = _host_cores()
    # one core
    sites, t_one, lo = 0, 0.0, 0
    while t_one < budget_s and lo + chunk <= Vb:
        n, dt = _oracle_lap_chunk((lo, lo + chunk))
        sites += n
        t_one += dt
        lo += chunk
    lap_one = sites / t_one / 1e9
    # every core: a fixed set of chunks sized to about budget_s of wall time
    per_core = max(1, int(round(budget_s * lap_one * 1e9 / chunk)))
    nchunk = min(cores * per_core, Vb // chunk)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        done = pool.map(_oracle_lap_chunk, [(i * chunk, (i + 1) * chunk) for i in range(nchunk)], chunksize=1)
        t_all = time.perf_counter() - t0
    lap_all = sum(n for n, _ in done) / t_all / 1e9
    # per-shift CG
    _, _, sigma = orat.kappa_poles(0.9, 12)
    k = 2
    n1, t1 = _oracle_cg_iters((float(sigma[0]), k))
    with ctx.Pool(min(cores, 12)) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_cg_iters, [(float(s), k) for s in sigma], chunksize=1)
        t12 = time.perf_counter() - t0
    return {
        "value": round(lap_all, 7), "unit": "Gsite/s", "cores": cores, "kind": "oracle",
        "sample": f"{nchunk} chunks of {chunk} sites of the {'x'.join(map(str, Lb))} eps=0.4 link field, the oracle's "
                  f"site-by-site Laplacian (numpy FP64, literal 3x3 products) in {cores} forked "
                  f"single-threaded workers: {t_all:.1f} s wall",
        "single_core": {"value": round(lap_one, 7), "unit": "Gsite/s", "cores": 1,
                        "sample": f"{sites} sites of the same field on one thread in {t_one:.1f} s"},
        "cg_iteration": {"lattice": list(L16),
            "one_shift_one_core_ms": round(t1 / n1 * 1e3, 1),
            "twelve_shifts_all_cores_ms": round(t12 / k * 1e3, 1), "cores": min(cores, 12),
            "sample": f"{k} iterations of the oracle's per-shift CG (one Delta, vector updates) on the {'x'.join(map(str, L16))} "
                      f"eps=0.5 field, one shift on one thread, then the 12 shifts of the 12-pole kappa=0.9 "
                      f"set on {min(cores, 12)} forked workers"},
    }


# ---- end of the CPU-baseline leg ----

TRAFFIC_RECORD = "stencil_traffic_32x32x32x64_f64.json"


def traffic_records(record=TRAFFIC_RECORD):
    """The committed rocprofv3 counter summaries of the headline stencil (one per profiled launch
    configuration), or []."""
    try:
        with open(os.path.join(ROOT, "profiles", record)) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        return []
    if "records" in doc:
        return list(doc["records"])
    return [doc] if "traffic_bytes_per_launch" in doc else []


def stencil_traffic(kernel_class, record=TRAFFIC_RECORD, cfg=None):
    """HBM bytes per launch of the headline stencil from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a calibration copy) of launch configuration cfg, or None
    when there is none, or the stencil sources have changed since it was taken."""
    if kernel_class != "stencil":
        return None, None
    recs = traffic_records(record)
    if not recs:
        return None, None
    from paper_2112_04556_amd.profiling import stencil_source_hash
    rel = os.path.join("profiles", record)
    if cfg is not None:
        match = [r for r in recs if r.get("launch_config") is not None and list(r["launch_config"]) == list(cfg)]
        if not match:
            have = [r.get("launch_config") for r in recs]
            return None, rel + f" (taken with launch configurations {have})"
        t = match[0]
    else:
        t = recs[0]
    if t.get("stencil_source_sha256") != stencil_source_hash():
        return None, rel + " (stale: stencil sources changed)"
    return round(float(t["traffic_bytes_per_launch"])), rel


def prefer_profiled_config(api, torch, L, U, F, cfg, best_ms, slack=1.03):
    """A launch configuration whose HBM traffic the committed counter summary holds, when the fastest
    of them runs within `slack` of the autotuner's pick (several shapes tie within the timing noise,
    which differs from box to box); else the pick."""
    profiled = [tuple(r["launch_config"]) for r in traffic_records() if r.get("launch_config") is not None]
    if not profiled or tuple(cfg) in profiled:
        return cfg
    y = torch.empty_like(F)
    best = None
    for rec in profiled:
        set_config(api, torch, L, rec)
        for _ in range(3):
            api.laplacian_apply(L, U, F, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            api.laplacian_apply(L, U, F, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        if best is None or ms < best[0]:
            best = (ms, rec)
    if best[0] <= slack * best_ms:
        set_config(api, torch, L, best[1])
        return best[1]
    set_config(api, torch, L, cfg)
    return cfg


def set_config(api, torch, L, cfg):
    """Store an 8-field launch configuration for the one-field FP64 Laplacian of lattice L."""
    kw = dict(zip(("form", "block", "xcd_remap", "nv", "order", "walk", "ns", "tile2"), cfg))
    form = kw.pop("form")
    api.tune_set(L, torch.float64, 1, form, purpose="apply", **kw)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(sharding across GPUs is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    # the oracle on the host cores first: its workers are forked before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the host cores)")
        cpu = cpu_baseline()
        _CPU.clear()
        log(f"cpu baseline: {cpu}")

    import numpy as np
    import torch

    from paper_2112_04556_amd import api, inputs

    dev = torch.device("cuda:0")

    # ---- timed step: Delta on one FP64 link field at 32^3 x 64 ----
    Lb = (32, 32, 32, 64)
    Vb = api.volume(Lb)
    log("generating the 32^3x64 inputs")
    Ub = api.pack_links(Lb, inputs.random_links(Lb, "eps", 0.4, seed=1).to(dev))
    Fb = inputs.gaussian_fields(Lb, 1, seed=1).to(dev)
    Yb = torch.empty_like(Fb)
    if args.headline_config:
        cfg = tuple(args.headline_config)
        set_config(api, torch, Lb, cfg)
    else:
        cfg, best_ms = api.autotune_laplacian(Lb, Ub, Fb, reps=3, purpose="apply")
        cfg = prefer_profiled_config(api, torch, Lb, Ub, Fb, cfg, best_ms)
    log(f"launch configuration {cfg}")
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        api.laplacian_apply(Lb, Ub, Fb, out=Yb)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        api.laplacian_apply(Lb, Ub, Fb, out=Yb)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / args.steps * 1e3
    value = Vb / (ms_step * 1e-3) / 1e9
    # the same launches again with HIP events around each (on the launch stream)
    api.profile_enable(True)
    for _ in range(args.steps):
        api.laplacian_apply(Lb, Ub, Fb, out=Yb)
    torch.cuda.synchronize()
    p = api.profile_read("stencil")
    api.profile_enable(False)
    traffic, traffic_src = stencil_traffic("stencil", cfg=cfg)
    bytes_launch = p["bytes"] / max(p["launches"], 1)
    roofline = {"bound": "hbm", "kernel": "stencil", "achieved": round(p["gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(p["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": traffic_src, "avg_launch_ms": round(p["avg_ms"], 5),
                "bytes_per_launch": bytes_launch, "bytes_per_site": round(bytes_launch / Vb, 1),
                "launches": p["launches"], "working_set": "1.9 GB, HBM (larger than the 256 MB Infinity Cache)",
                "measured_over": f"the {args.steps} timed applications repeated with HIP events on the launch stream"}
    log(f"{ms_step:.4f} ms per application, {value:.3f} Gsite/s, {p['gbs']:.1f} GB/s algorithmic")
    del Ub, Fb, Yb
    torch.cuda.empty_cache()
    solves, hot, extras = None, None, {}
    if not args.headline_only:
        solves, hot, extras = second_half(args, api, inputs, torch, np, dev)

    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gsite/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Delta on one su(3) link field (4 x 8 reals per site), 32^3x64 lattice, eps=0.4 "
                               "links (seed 1), Gaussian field, FP64, periodic",
                   "lattice": list(Lb), "n_rhs": 1, "launch_config": dict(zip(
                       ("form", "block", "xcd_remap", "nv", "order", "walk", "ns", "tile2"), cfg)),
                   "value_definition": "lattice sites through Delta per second (one link field per application)"},
        "roofline": roofline,
        **({} if solves is None else {"rational_solve": solves, "hot_path_step": hot}),
        **extras,
    }
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def second_half(args, api, inputs, torch, np, dev):
    """The rational solves to 1e-10 (FP64 against mixed precision), one pass of the whole hot path and
    the per-component figures, all on the 16^4 workload."""
    L = (16, 16, 16, 16)
    U = inputs.random_links(L, "eps", 0.5, seed=2)
    P = inputs.gaussian_fields(L, 1, seed=2)
    U_aos = U.to(dev)
    Pd = P.to(dev)
    Ud = api.pack_links(L, U_aos)
    U32 = api.pack_links(L, U_aos, torch.float32)
    solves = d2_solves(api, inputs, torch, dev, L, Ud, Pd)
    hot = hot_path_step(api, torch, dev, L, U_aos, Ud, U32, Pd, args.kappa, args.steps_hot)
    extras = {}
    if not args.no_extras:
        extras = run_extras(api, inputs, torch, np, dev, L, U_aos, Ud, Pd)
    return solves, hot, extras


def hot_path_step(api, torch, dev, L, U_aos, Ud, U32, Pd, kappa, steps):
    """Every stage of the path on the 16^4 workload (one Gaussian momentum field): pack the links,
    the 12-pole kinetic force in mixed precision (both solves to 1e-10, the link derivative), the
    degree-64/16-window FP32 power spectrum of the force, the degree-32/4-window filter of the momentum
    on a second stream; timed over `steps` passes, then the same passes on one stream with HIP events
    around every launch for the kernel-class shares."""
    V = api.volume(L)
    rat = api.rational_kappa(kappa, 12)
    solver = api.Solver(tol=1e-10, mode=1)
    api.autotune_laplacian(L, Ud, Pd, reps=10)
    api.autotune_laplacian(L, U32, Pd.float(), reps=10)
    api.autotune_laplacian(L, Ud, Pd.expand(12, -1, -1, -1).contiguous(), reps=5, purpose="cg64")
    ws = torch.empty(api.workspace_bytes(6, L, 0, 1, 12, 0, 1), dtype=torch.uint8, device=dev)
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
        api.power_spectrum(L, api.convert_f64_f32(Uw), api.convert_f64_f32(out["dK"]), 64, 16)
        if overlap:
            main.wait_stream(side)
        else:
            api.cheb_filter(L, Uw, Pd, 32, 4)
        return out

    for _ in range(2):
        last = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        last = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    api.profile_enable(True)
    for _ in range(steps):
        step(overlap=False)
    torch.cuda.synchronize()
    prof = {c: api.profile_read(c) for c in api.PROF_CLASSES}
    api.profile_enable(False)
    tot = max(sum(p["ms"] for p in prof.values()), 1e-12)
    st = prof["stencil"]
    out = {"ms": round(ms, 3), "steps": steps, "lattice": list(L), "poles": 12, "kappa": kappa,
           "stencil_applications": st["items"] / steps,
           "gsite_s_through_delta": round(V * st["items"] / steps / (ms * 1e-3) / 1e9, 3),
           "stencil": {"avg_launch_ms": round(st["avg_ms"], 5), "GBs": round(st["gbs"], 1),
                       "hbm_frac": round(st["gbs"] / HBM_PEAK_GBS, 4),
                       "working_set": "71 MB, resident in the 256 MB Infinity Cache"},
           "kernel_time_share": {c: round(prof[c]["ms"] / tot, 4) for c in prof},
           "stats_last_step": last["stats"]}
    log(f"hot path step 16^4: {out}")
    return out


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
                "config": dict(zip(("form", "block", "xcd_remap", "nv", "order", "walk", "ns", "tile2"), cfg))}
            log(f"D-1 {key} {name}: {out[key][name]}")
            del sets, Ud, Fd
        del U, F
    return out


def d2_solves(api, inputs, torch, dev, L, Ud, Pd):
    """Rational solve alone, time to FP64 true residual 1e-10: FP64 against mixed precision."""
    solves = {}
    P8 = inputs.gaussian_fields(L, 8, seed=22).to(dev)
    # launch configurations of the solves' stencils (outside the timed calls): the CG iterations in
    # each precision and the FP64 residuals (reliable updates, the true residuals of all 12 shifts)
    U32 = api.convert_f64_f32(Ud)
    for n, src in ((1, Pd), (8, P8)):
        api.autotune_laplacian(L, Ud, src, reps=5, purpose="cg")
        api.autotune_laplacian(L, U32, src.float(), reps=5, purpose="cg")
        api.autotune_laplacian(L, Ud, src, reps=5, purpose="cg64")
        api.autotune_laplacian(L, Ud, src.repeat(12, 1, 1, 1), reps=3, purpose="cg64")
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
        api.autotune_laplacian(L, U32, F, reps=5, purpose="moments")
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
    # launch configurations of the solves' stencils at this size (outside the timed calls): the CG
    # iterations in each precision, the FP64 reliable updates (2 fields) and the true residuals of
    # all 16 shifts (32 fields), and the FP32 recursion of the 8-force spectrum
    api.autotune_laplacian(L, Ud, P[:2], reps=2, purpose="cg")
    api.autotune_laplacian(L, U32, P[:2].float(), reps=2, purpose="cg")
    api.autotune_laplacian(L, Ud, P[:2], reps=2, purpose="cg64")
    P32 = P[:2].repeat(16, 1, 1, 1)
    api.autotune_laplacian(L, Ud, P32, reps=1, purpose="cg64")
    del P32
    api.autotune_laplacian(L, U32, P.float(), reps=1, purpose="moments")
    torch.cuda.empty_cache()
    need = max(api.workspace_bytes(6, L, 0, 2, 16, 0, m) for m in (0, 1))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    row = {"workspace_GiB": round(need / 2**30, 1)}

    def force_step(sv, forces):
        iters = 0
        t0 = time.perf_counter()
        for c in range(4):
            o = api.kinetic_force(L, Ud, P[2 * c:2 * c + 2], rat, sv, per_rhs=True, ws=ws)
            forces[2 * c:2 * c + 2] = o["dK"].float()
            iters += o["stats"]["iters"]
            del o
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        api.power_spectrum(L, U32, forces, 256, 128)
        torch.cuda.synchronize()
        return iters, t1 - t0, time.perf_counter() - t1

    for mode, name in ((0, "fp64"), (1, "mixed")):
        sv = api.Solver(tol=1e-10, mode=mode)
        forces = torch.empty((8, 4, 8, V), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        iters, t_force, t_spec = force_step(sv, forces)
        # the same step again with HIP events around every launch, for the kernel-class figures
        api.profile_enable(True)
        force_step(sv, forces)
        prof = {c: api.profile_read(c) for c in api.PROF_CLASSES}
        api.profile_enable(False)
        row[name] = {"ms_per_force": round(t_force * 1e3 / 8, 3), "spectrum_ms": round(t_spec * 1e3, 3),
                     "total_ms": round((t_force + t_spec) * 1e3, 3), "solver_iters": iters,
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
    degree 64, 16 windows: the forward sweep to t_64, then the reverse sweep (per degree one stencil
    launch over the adjoint and the recomputed forward vectors, and one derivative pass)."""
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
        # links as two rows of 12 reals (the third is rebuilt) and the 32-real force: 80 reals per site
        out[key] = {"force_ms": round(f_ms, 4), "force_GBs": round(V * 80 * 8 / (f_ms * 1e-3) / 1e9, 1),
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
    # the exact inverse R(Delta)^-1 xi through the partial fractions of 1/R (kappa = 0 in the call)
    ex_ms, ex = _median_ms(lambda: api.heatbath_momenta(L, Ud, xi, 0.0, rat, sv), torch)
    res = {"heatbath_ms": round(hb_ms, 3), "solver_iters": out["stats"]["iters"],
           "true_relres_max": out["stats"]["true_relres_max"], "filter_ms": round(f_ms, 3),
           "exact_inverse_ms": round(ex_ms, 3), "exact_inverse_iters": ex["stats"]["iters"],
           "exact_inverse_true_relres_max": ex["stats"]["true_relres_max"]}
    log(f"D9 heat-bath momenta + window projection 16^4: {res}")
    return res


def run_extras(api, inputs, torch, np, dev, L, U_aos, Ud, Pd):
    out = {}
    cp = copy_bandwidth(torch, dev)
    out["copy_1GiB"] = cp
    log(f"copy: {cp}")
    out["D1_laplacian"] = d1_laplacian(api, inputs, torch, dev, cp["GBs"])
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
