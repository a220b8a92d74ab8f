"""Helpers around rocprofv3 for the stencil: workloads to profile and summaries of the CSVs.

Workloads (run under ``rocprofv3``; each prints what it launched):

    python -m paper_2112_04556_amd.profiling copy
        a 1 GiB device-to-device copy (calibration: read and written bytes are known)
    python -m paper_2112_04556_amd.profiling stencil --L 32 32 32 64 --dtype f64 --reps 3
        the Laplacian on one link field, autotuned first, then ``reps`` timed launches
    python -m paper_2112_04556_amd.profiling kinetic --L 32 32 32 64 --n 2 --poles 16 --mode 1 --reps 1
        kinetic-force evaluations (kappa = 0.9 pole set, solves to 1e-10) of n momentum fields,
        after one warm-up evaluation
    python -m paper_2112_04556_amd.profiling spectrum --L 24 24 24 24 --n 32 --degree 16 --windows 64 --dtype f32
        batched power spectra of n Gaussian sources on Haar links (autotuned first, then one call)
    python -m paper_2112_04556_amd.profiling solve --L 16 16 16 16 --n 8 --poles 12 --kappa 0.9 --mode 1 --reps 2
        rational solves (eps = 0.5 links, tol 1e-10) of n Gaussian fields, after one warm-up solve
    python -m paper_2112_04556_amd.profiling leapfrog --L 16 16 16 16 --reps 2
        implicit leapfrog steps (12-pole kappa = 0.9 mass term, beta = 5.5, eps = 0.02) on one
        momentum field, after one warm-up step

Summaries (run on the host, over the CSV files rocprofv3 wrote):

    python -m paper_2112_04556_amd.profiling summarize-trace DIR --prefix rmh::k_hop --last N
    python -m paper_2112_04556_amd.profiling traffic --fetch DIR1 --write DIR2 --prefix rmh::k_hop \
        --last N --fetch-scale 2.0 --write-scale 1.0 --out FILE.json --command-fetch ... --command-write ... \
        [--launch-config FORM BLOCK XCD NV ORDER WALK NS TILE2] [--append]

``traffic`` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) over the last N dispatches
whose kernel name starts with the prefix, scales each by the factor the same counter shows for
the calibration copy, and stamps the result with the hash of the stencil sources, so a reader
can tell whether the kernel has changed since.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
STENCIL_SOURCES = ("csrc/rmh_stencil.hip", "csrc/rmh_device.h")


def stencil_source_hash() -> str:
    h = hashlib.sha256()
    for rel in STENCIL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _csv(dirname: str, suffix: str):
    files = sorted(glob.glob(os.path.join(dirname, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {dirname}")
    with open(files[0], newline="") as fh:
        return list(csv.DictReader(fh))


def trace_dispatches(dirname: str, prefix: str):
    rows = _csv(dirname, "kernel_trace.csv")
    rows = [r for r in rows if r["Kernel_Name"].replace("void ", "").startswith(prefix)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    return [(r["Kernel_Name"], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9) for r in rows]


def counter_dispatches(dirname: str, counter: str, prefix: str):
    rows = _csv(dirname, "counter_collection.csv")
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        if not r["Kernel_Name"].replace("void ", "").startswith(prefix):
            continue
        d = int(r["Dispatch_Id"])
        name, v = per.get(d, (r["Kernel_Name"], 0.0))
        per[d] = (name, v + float(r["Counter_Value"]))
    return [per[d] for d in sorted(per)]


def summarize_trace(dirname: str, prefix: str, last: int) -> dict:
    disp = trace_dispatches(dirname, prefix)[-last:]
    by = {}
    for name, t in disp:
        short = name.replace("void ", "").split("(")[0]
        c, s = by.get(short, (0, 0.0))
        by[short] = (c + 1, s + t)
    total = sum(t for _, t in disp)
    return {"dispatches": len(disp), "avg_ms": total / max(len(disp), 1) * 1e3, "total_ms": total * 1e3,
            "kernels": {k: {"calls": c, "avg_ms": s / c * 1e3} for k, (c, s) in sorted(by.items())}}


def traffic(fetch_dir: str, write_dir: str, prefix: str, last: int, fetch_scale: float, write_scale: float) -> dict:
    f = counter_dispatches(fetch_dir, "FETCH_SIZE", prefix)[-last:]
    w = counter_dispatches(write_dir, "WRITE_SIZE", prefix)[-last:]
    if not f or not w:
        raise ValueError("no matching dispatches")
    fk = sum(v for _, v in f) / len(f)
    wk = sum(v for _, v in w) / len(w)
    names = sorted({n.replace("void ", "").split("(")[0] for n, _ in f + w})
    return {"dispatches": min(len(f), len(w)), "kernels": names,
            "fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
            "fetch_scale": fetch_scale, "write_scale": write_scale,
            "traffic_bytes_per_launch": (fk * fetch_scale + wk * write_scale) * 1024.0,
            "stencil_source_sha256": stencil_source_hash()}


def run_copy():
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy: 3 x {a.numel() * 8} bytes read and written", flush=True)


def run_stencil(L, dtype_name: str, reps: int):
    import torch
    from . import api, inputs
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    U = inputs.random_links(L, "haar", seed=5).to("cuda")
    F = inputs.gaussian_fields(L, 1, seed=5).to("cuda").to(dt)
    Ud = api.pack_links(L, U, dt)
    cfg, ms = api.autotune_laplacian(L, Ud, F, reps=2)
    y = torch.empty_like(F)
    for _ in range(reps):
        api.laplacian_apply(L, Ud, F, out=y)
    torch.cuda.synchronize()
    print(f"stencil {L} {dtype_name}: config {cfg} (autotune {ms:.4f} ms), {reps} launches", flush=True)


def run_kinetic(L, n: int, poles: int, mode: int, reps: int):
    import torch
    from . import api, inputs
    U = api.pack_links(L, inputs.random_links(L, "eps", 0.4, seed=5).to("cuda"))
    P = inputs.gaussian_fields(L, n, seed=5).to("cuda")
    rat = api.rational_kappa(0.9, poles)
    sv = api.Solver(tol=1e-10, mode=mode)
    ws = torch.empty(api.workspace_bytes(api.L_.OP_KINETIC_FORCE, L, api.RMH_F64, n, poles, 0, mode),
                     dtype=torch.uint8, device="cuda")
    out = None
    for _ in range(reps + 1):
        out = api.kinetic_force(L, U, P, rat, sv, per_rhs=True, ws=ws)
    torch.cuda.synchronize()
    print(f"kinetic {L} n={n} poles={poles} mode={mode}: {reps + 1} evaluations, "
          f"{out['stats']['iters']} solver iterations", flush=True)


def run_spectrum(L, n: int, degree: int, windows: int, dtype_name: str, kind: str, config=None):
    import torch
    from . import api, inputs
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    U = api.pack_links(L, inputs.random_links(L, kind, seed=3).to("cuda"), dt)
    F = inputs.gaussian_fields(L, n, seed=3).to("cuda").to(dt)
    if config:
        # a pinned launch configuration, so that separate counter runs count the same kernel
        cfg = tuple(config)
        form, block, xcd, nv, order, walk, ns, tile2 = cfg
        api.tune_set(L, dt, n, form, block, xcd, nv, order, walk, ns=ns, tile2=tile2)
    else:
        cfg, ms = api.autotune_laplacian(L, U, F, reps=2)
    api.power_spectrum(L, U, F, degree, windows)
    torch.cuda.synchronize()
    print(f"spectrum {L} n={n} degree={degree} {dtype_name} {kind}: config {cfg}, one call "
          f"({(degree + 1) // 2} sweeps)", flush=True)


def run_solve(L, n: int, poles: int, kappa: float, mode: int, reps: int):
    import torch
    from . import api, inputs
    U = api.pack_links(L, inputs.random_links(L, "eps", 0.5, seed=2).to("cuda"))
    P = inputs.gaussian_fields(L, n, seed=22).to("cuda")
    rat = api.rational_kappa(kappa, poles)
    sv = api.Solver(tol=1e-10, mode=mode)
    out = None
    for _ in range(reps + 1):
        out = api.rational_apply(L, U, P, rat, sv)
    torch.cuda.synchronize()
    print(f"solve {L} n={n} poles={poles} kappa={kappa} mode={mode}: {reps + 1} solves, stats {out['stats']}",
          flush=True)


def run_leapfrog(L, reps: int):
    import torch
    from . import api, inputs
    U = api.pack_links(L, inputs.random_links(L, "eps", 0.5, seed=8).to("cuda"))
    P = inputs.gaussian_fields(L, 1, seed=8)[0].to("cuda")
    rat = api.rational_kappa(0.9, 12)
    sv = api.Solver(tol=1e-10)
    ws = torch.empty(api.workspace_bytes(api.L_.OP_LEAPFROG, L, api.RMH_F64, 1, 12), dtype=torch.uint8,
                     device="cuda")
    st = None
    for _ in range(reps + 1):
        _, _, st = api.leapfrog_step(L, U, P, rat, 0.02, 5.5, sv, fp_tol=1e-10, ws=ws)
    torch.cuda.synchronize()
    print(f"leapfrog {L}: {reps + 1} steps, last {st['p_iters']} + {st['u_iters']} fixed-point iterations, "
          f"{st['solver']['iters']} solver iterations", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    p = sub.add_parser("stencil")
    p.add_argument("--L", type=int, nargs=4, default=[32, 32, 32, 64])
    p.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    p.add_argument("--reps", type=int, default=3)
    p = sub.add_parser("kinetic")
    p.add_argument("--L", type=int, nargs=4, default=[32, 32, 32, 64])
    p.add_argument("--n", type=int, default=2)
    p.add_argument("--poles", type=int, default=16)
    p.add_argument("--mode", type=int, default=1)
    p.add_argument("--reps", type=int, default=1)
    p = sub.add_parser("spectrum")
    p.add_argument("--L", type=int, nargs=4, default=[24, 24, 24, 24])
    p.add_argument("--n", type=int, default=32)
    p.add_argument("--degree", type=int, default=16)
    p.add_argument("--windows", type=int, default=64)
    p.add_argument("--dtype", choices=["f64", "f32"], default="f32")
    p.add_argument("--kind", choices=["haar", "unit", "eps"], default="haar")
    p.add_argument("--config", type=int, nargs=8, default=None,
                   help="pin the stencil launch configuration (form block xcd_remap nv order walk ns tile2) "
                        "instead of autotuning")
    p = sub.add_parser("solve")
    p.add_argument("--L", type=int, nargs=4, default=[16, 16, 16, 16])
    p.add_argument("--n", type=int, default=8)
    p.add_argument("--poles", type=int, default=12)
    p.add_argument("--kappa", type=float, default=0.9)
    p.add_argument("--mode", type=int, default=1)
    p.add_argument("--reps", type=int, default=2)
    p = sub.add_parser("leapfrog")
    p.add_argument("--L", type=int, nargs=4, default=[16, 16, 16, 16])
    p.add_argument("--reps", type=int, default=2)
    p = sub.add_parser("summarize-trace")
    p.add_argument("dir")
    p.add_argument("--prefix", default="rmh::k_hop")
    p.add_argument("--last", type=int, default=0)
    p = sub.add_parser("traffic")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--prefix", default="rmh::k_hop")
    p.add_argument("--last", type=int, default=0)
    p.add_argument("--fetch-scale", type=float, required=True)
    p.add_argument("--write-scale", type=float, required=True)
    p.add_argument("--out")
    p.add_argument("--command-fetch", default="")
    p.add_argument("--command-write", default="")
    p.add_argument("--workload", default="")
    p.add_argument("--launch-config", type=int, nargs=8, default=None,
                   help="the stencil launch configuration of the counted dispatches (form block xcd_remap nv "
                        "order walk ns tile2)")
    p.add_argument("--append", action="store_true",
                   help="add the record to the file's list of records (one per launch configuration)")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        run_copy()
    elif a.cmd == "kinetic":
        run_kinetic(tuple(a.L), a.n, a.poles, a.mode, a.reps)
    elif a.cmd == "leapfrog":
        run_leapfrog(tuple(a.L), a.reps)
    elif a.cmd == "stencil":
        run_stencil(tuple(a.L), a.dtype, a.reps)
    elif a.cmd == "solve":
        run_solve(tuple(a.L), a.n, a.poles, a.kappa, a.mode, a.reps)
    elif a.cmd == "spectrum":
        run_spectrum(tuple(a.L), a.n, a.degree, a.windows, a.dtype, a.kind, a.config)
    elif a.cmd == "summarize-trace":
        print(json.dumps(summarize_trace(a.dir, a.prefix, a.last or 10**9), indent=1))
    else:
        t = traffic(a.fetch, a.write, a.prefix, a.last or 10**9, a.fetch_scale, a.write_scale)
        t.update({"workload": a.workload, "command_fetch": a.command_fetch, "command_write": a.command_write,
                  "prefix": a.prefix})
        if a.launch_config:
            t["launch_config"] = list(a.launch_config)
        doc = t
        if a.append and a.out and os.path.exists(a.out):
            with open(a.out) as fh:
                old = json.load(fh)
            recs = old.get("records", [old] if "traffic_bytes_per_launch" in old else [])
            recs = [r for r in recs if r.get("launch_config") != t.get("launch_config")] + [t]
            doc = {"records": recs}
        elif a.append:
            doc = {"records": [t]}
        text = json.dumps(doc, indent=1)
        if a.out:
            with open(a.out, "w") as fh:
                fh.write(text + "\n")
        print(text)


if __name__ == "__main__":
    sys.exit(main())
