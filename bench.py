"""Benchmark of the HEVI dynamical-core step on one GPU.

Default workload: the 1024x1024x64 warm-bubble domain (16 seeded bubbles of
radius 2-8 km, Gaussian velocity noise of 0.1 m/s in a 10 m/s wind,
isothermal reference, dx = dy = 2 km, stretched levels to 20 km), RK3 long
steps of dt = 10 s with 6 HEVI short steps per stage, periodic in x and y.
One "step" is one long step of the whole path: 3 slow sweeps, 18 short steps
and the float64 mass sum.  The primary number is the float32 path; the mixed
(float32 sweeps, float64 column solve) and float64 paths are timed on the same
state for the speedup over the plain float64 step.

Other workloads (--workload): terrain (1600x1280x64 over Gaussian hills with
wind shear, mixed precision primary, error of each path against the float64
GPU run), xl (2048x2048x64 over hills, for --layout kij / ijk), ensemble
(48 members of uneven sizes), diffusion (the seven-point stencil of the
paper's reduced weather application on 1024x1024x64, timed against its
no-cache and perfect-cache bandwidth models).  With the CPU baseline (the
oracle timed on the host cores) comes the per-field error of every path
against the oracle on the oracle-sized sub-run of the workload.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s + achieved HBM GB/s (% peak), FP32/mixed vs FP64 step, 1 GPU"
HBM_PEAK_GBS = 8000.0
BYTES = {"fp32": 4, "mixed": 4, "fp64": 8}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def model_bytes_per_cell(b: int, n_short: int, terrain: bool = False) -> int:
    """Compulsory bytes per cell per long step: 3 slow sweeps (read 5 state,
    write 7; over terrain also read the 3 per-cell reference fields),
    3*n short steps (read 5 state + 4 tendencies + 3 stage coefficients,
    write 5), one mass sum (read rho')."""
    return b * (3 * (15 if terrain else 12) + 3 * n_short * 17 + 1)


def short_step_bytes(b: int, cells: int) -> int:
    return 17 * b * cells


def kernel_digest() -> str:
    """Digest of the sources the column-fastest kernels are built from, with
    comments and blank lines removed, so that a comment edit does not
    invalidate the recorded counters."""
    code = []
    for name in ("hevi_kernels.hip", "hevi_device.h"):
        src = os.path.join(ROOT, "paper_1710_08616_amd", "csrc", name)
        for line in open(src, encoding="utf-8"):
            line = line.split("//", 1)[0].rstrip()
            if line:
                code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


def read_traffic(prec: str):
    """The committed rocprofv3 counter record of the short step (HBM bytes per
    launch and the launch configuration it was taken in), if it was taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "short_step_large_traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic:"):
            try:
                rec = json.loads(line[len("traffic:"):])
            except ValueError:
                continue
            if rec.get("kernel_sha") == kernel_digest() and rec.get("precision") == prec:
                return rec
    return None


def time_precision(hevi, s, prec, steps, warmup, layout="kij", keep=False, short="fb", tune=True):
    import torch
    log(f"[bench] {prec}: init {s.nx}x{s.ny}x{s.nz}")
    d = hevi.Domain(s, precision=prec, layout=layout, short=short)
    tiles = None
    if tune:
        # the autotuner times each launch configuration per kernel kind on this state
        # (results are bitwise independent of the shape; the state is left
        # unchanged)
        tiles, lanes = d.tune()
        tiles = {"tile_x": tiles, "lanes_per_column": lanes}
        log(f"[bench] {prec}: tiles (x-extent per kind) {tiles['tile_x']}, lanes per column "
            f"{lanes}")
    if warmup:
        d.step(s.dt, warmup, s.n_short)
    m0 = d.mass()
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record(d.stream)
    d.step(s.dt, steps, s.n_short)     # graph replay, no per-kernel events
    g1.record(d.stream)
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1)
    d.trace(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(d.stream)
    d.step(s.dt, steps, s.n_short)
    e1.record(d.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kern = d.trace_read()
    d.trace(False)
    m1 = d.mass()
    final = d.read_all() if keep else None
    d.close()
    del d
    torch.cuda.empty_cache()
    cells = s.cells
    res = {
        "ms_per_step": ms / steps,
        "graph_ms_per_step": graph_ms / steps,
        "cell_updates_per_s": cells * steps / (ms * 1e-3),
        "model_gbps": model_bytes_per_cell(BYTES[prec], s.n_short, s.terrain is not None)
        * cells * steps / (ms * 1e-3) / 1e9,
        "mass_drift_rel": abs(m1 - m0) / m0,
        "kernels_ms_avg": {k: (v[0] / v[1] if v[1] else None) for k, v in kern.items()},
        "kernels_launches": {k: v[1] for k, v in kern.items()},
        "kernels_ms_total": {k: v[0] for k, v in kern.items()},
        "launch_config": tiles,
    }
    log(f"[bench] {prec}: {res['ms_per_step']:.3f} ms/step (graph replay {res['graph_ms_per_step']:.3f}), "
        f"{res['cell_updates_per_s']:.3e} cell-updates/s, model {res['model_gbps']:.0f} GB/s")
    return (res, final) if keep else res


def field_errors(got, ref):
    """Per field: max and RMS of (got - ref), each divided by the range of ref."""
    from paper_1710_08616_amd import inputs
    out = {}
    for name, a, b in zip(inputs.FIELD_NAMES, got, ref):
        rng = float(np.ptp(b)) or 1.0
        d = a - b
        out[name] = {"max_rel": float(np.abs(d).max()) / rng,
                     "rms_rel": float(np.sqrt(np.mean(d * d))) / rng}
    return out


def twin_tolerances(case: str):
    """The frozen per-field bars of the reduced-precision paths for a sub-run
    (10x the binary32-storage twin of the oracle), or None."""
    path = os.path.join(ROOT, "tests", "golden", "twin_tolerances.json")
    try:
        return json.load(open(path))["cases"][case]["tolerance"]
    except (OSError, KeyError, ValueError):
        return None


def accuracy_vs_oracle(hevi, sub, ref, precs, case):
    """Every path against the float64 oracle's result `ref` on an oracle-sized
    sub-run of the workload (same generator), after its full number of long
    steps; reduced-precision paths against their frozen per-field bars."""
    tol = twin_tolerances(case)
    out = {}
    for p in precs:
        d = hevi.Domain(sub, precision=p)
        m0 = d.mass()
        d.step(sub.dt, sub.n_long, sub.n_short)
        got = d.read_all()
        m1 = d.mass()
        d.close()
        fe = field_errors(got, ref)
        rec = {"fields": fe, "mass_drift_rel": abs(m1 - m0) / m0}
        if p != "fp64" and tol is not None:
            rec["within_tolerance"] = all(fe[f]["max_rel"] <= tol[f]["max_rel"] and
                                          fe[f]["rms_rel"] <= tol[f]["rms_rel"] for f in fe)
        elif p == "fp64":
            rec["within_tolerance"] = all(fe[f]["max_rel"] <= 1e-11 for f in fe)
        out[p] = rec
        log(f"[bench] accuracy {p}: worst max {max(v['max_rel'] for v in fe.values()):.2e} of "
            f"the range, within tolerance: {rec.get('within_tolerance')}")
    return {"sub_run": f"{sub.nx}x{sub.ny}x{sub.nz}, {sub.n_long} long steps, n={sub.n_short}",
            "tolerance": tol, "per_precision": out}


def time_ensemble(hevi, members, prec, steps, warmup, layout="kij", tune=True):
    """The batched ensemble: autotune launch configurations, warm up, then time `steps`
    long steps of all members (each with its own dt) with per-kernel events."""
    import torch
    n_short = members[0].n_short
    cells = sum(m.cells for m in members)
    log(f"[bench] ensemble {prec}: init {len(members)} members, {cells / 1e6:.1f} M cells")
    e = hevi.Ensemble(members, precision=prec, layout=layout)
    shapes = e.tune() if tune else None
    if warmup:
        e.step(warmup, n_short)
    m0 = [e.mass(q) for q in range(e.n)]
    torch.cuda.synchronize()
    # graph replay (production path), then the same length with kernel events
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record(e.stream)
    e.step(steps, n_short)
    g1.record(e.stream)
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1)
    e.trace(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(e.stream)
    e.step(steps, n_short)
    e1.record(e.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kern = e.trace_read()
    e.trace(False)
    drift = max(abs(e.mass(q) - m0[q]) / m0[q] for q in range(e.n))
    e.close()
    del e
    torch.cuda.empty_cache()
    b = BYTES[prec]
    res = {
        "members": len(members), "cells": cells, "tile_x": shapes,
        "ms_per_step": ms / steps, "graph_ms_per_step": graph_ms / steps,
        "cell_updates_per_s": cells * steps / (ms * 1e-3),
        "graph_cell_updates_per_s": cells * steps / (graph_ms * 1e-3),
        "model_gbps": model_bytes_per_cell(b, n_short) * cells * steps / (ms * 1e-3) / 1e9,
        "mass_drift_rel_max": drift,
        "kernels_ms_avg": {k: (v[0] / v[1] if v[1] else None) for k, v in kern.items()},
        "kernels_launches": {k: v[1] for k, v in kern.items()},
    }
    log(f"[bench] ensemble {prec}: graph {res['graph_ms_per_step']:.3f} ms/step "
        f"({res['graph_cell_updates_per_s']:.3e} cell-updates/s, model {res['model_gbps']:.0f} GB/s), "
        f"traced {res['ms_per_step']:.3f} ms/step, tiles {shapes}")
    return res


def time_diffusion(hevi, prec, steps, warmup, layout="kij", n=1024, nz=64):
    """hv_diffuse on an n x n x nz field, each tile shape; the fastest is kept.
    Bytes per cell and step: perfect cache 2b (one read, one write), no
    cache 8b (7 reads, 1 write)."""
    import torch
    dt = torch.float32 if prec == "fp32" else torch.float64
    b = 4 if prec == "fp32" else 8
    shape = (n, n, nz) if layout == "kij" else (nz, n, n)
    g = torch.Generator(device="cuda").manual_seed(1716)
    x = torch.rand(shape, generator=g, device="cuda", dtype=dt) + 1.0
    y = torch.empty_like(x)
    k = (0.1, 0.1, 0.2)
    best = None
    for tile in (16, 8, 4):
        for _ in range(warmup):
            hevi.diffuse(x, y, *k, layout=layout, tile_x=tile)
            x, y = y, x
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            hevi.diffuse(x, y, *k, layout=layout, tile_x=tile)
            x, y = y, x
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        log(f"[bench] diffusion {prec} {layout} tile {tile}: {ms:.4f} ms/step")
        if best is None or ms < best[1]:
            best = (tile, ms)
    cells = n * n * nz
    tile, ms = best
    t_perfect = 2 * b * cells / (HBM_PEAK_GBS * 1e9) * 1e3
    t_nocache = 8 * b * cells / (HBM_PEAK_GBS * 1e9) * 1e3
    return {"ms_per_step": ms, "tile_x": tile, "cells": cells,
            "cell_updates_per_s": cells / (ms * 1e-3),
            "perfect_cache_gbps": 2 * b * cells / (ms * 1e-3) / 1e9,
            "frac_of_perfect_cache_limit": t_perfect / ms,
            "speedup_vs_no_cache_model": t_nocache / ms}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, sub):
    """The FP64 oracle on the host cores, as a baseline: one long step of the
    workload at its full shape on all cores, one long step of the
    oracle-sized sub-run on one thread, and the whole sub-run on all cores
    (cell-updates/s each).  Also returns the sub-run's final fields, the
    reference of the accuracy check."""
    from oracle import oracle
    oracle.lib()
    cores = oracle.threads()
    t0 = time.perf_counter()
    oracle.step(s, n_long=1)
    sec = time.perf_counter() - t0
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.step(sub, n_long=1)
        sec1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    log(f"[bench] oracle: {sub.nx}x{sub.ny}x{sub.nz}, {sub.n_long} long steps")
    t2 = time.perf_counter()
    ref = oracle.step(sub)
    sec2 = time.perf_counter() - t2
    rec = {"value": s.cells / sec, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"one long step (n={s.n_short}) of the {s.nx}x{s.ny}x{s.nz} workload itself, "
                     f"{sec:.1f} s on {cores} threads",
           "single_thread": {"value": sub.cells / sec1, "unit": "cell-updates/s", "cores": 1,
                             "sample": f"one long step of the {sub.nx}x{sub.ny}x{sub.nz} sub-run, "
                                       f"{sec1:.2f} s"},
           "sub_run": {"value": sub.cells * sub.n_long / sec2, "unit": "cell-updates/s",
                       "cores": cores, "sample": f"{sub.n_long} long steps of the sub-run, "
                                                 f"{sec2:.1f} s"},
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    return rec, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precisions", default=None,
                    help="default: fp32,mixed,fp64 (terrain: mixed,fp64; xl: fp32,mixed)")
    ap.add_argument("--layout", default="kij")
    ap.add_argument("--workload", default="large")
    ap.add_argument("--short", default="fb", choices=["fb", "rk2"],
                    help="short-step integrator: forward-backward or two-stage Runge-Kutta")
    ap.add_argument("--damping", action="store_true",
                    help="lateral (8-cell) and upper (above 15 km) damping toward synthetic "
                         "boundary data after every short step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner: keep the launch configurations of the tune "
                         "cache ($HV_TUNE_CACHE) or the defaults (the counter runs use this so "
                         "that their passes measure one configuration)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the per-field error of every path against the float64 oracle "
                         "on the oracle-sized sub-run (run by default with the CPU baseline, "
                         "whose sub-run it compares with)")
    args = ap.parse_args()
    if args.precisions is None:
        args.precisions = {"terrain": "mixed,fp64", "xl": "fp32,mixed", "ensemble": "fp32,mixed",
                           "diffusion": "fp32,fp64"}.get(args.workload, "fp32,mixed,fp64")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the step is built and measured on a single "
              "MI355X (multi-GPU decomposition is design-only); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1710_08616_amd import hevi, inputs
    hevi.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.workload == "diffusion":
        precs = [p for p in args.precisions.split(",") if p and p != "mixed"] or ["fp32"]
        res = {p: time_diffusion(hevi, p, args.steps, args.warmup, args.layout) for p in precs}
        r = res[precs[0]]
        b = 4 if precs[0] == "fp32" else 8
        cpu = None
        if not args.no_cpu_baseline:
            from oracle import oracle
            q = np.random.default_rng(1716).random((64, 512, 512)) + 1.0
            oracle.lib()
            t0 = time.perf_counter()
            oracle.diffuse(q, 0.1, 0.1, 0.2, steps=20)
            sec = time.perf_counter() - t0
            cpu = {"value": q.size * 20 / sec, "unit": "cell-updates/s", "cores": oracle.threads(),
                   "kind": "oracle", "sample": f"512x512x64, 20 steps, {sec:.1f} s"}
        out = {
            "metric": METRIC, "value": r["cell_updates_per_s"], "unit": "cell-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" if precs[0] == "fp32" else "f64",
            "data": "synthetic",
            "config": {"workload": "seven-point diffusion 1024x1024x64 (bandwidth-model stencil)",
                       "precision": precs[0], "layout": args.layout, "tile_x": r["tile_x"],
                       "parallelism": "1 GPU"},
            "roofline": {"bound": "hbm", "achieved": round(r["perfect_cache_gbps"], 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(r["perfect_cache_gbps"] / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "diffuse", "bytes_per_launch": 2 * b * r["cells"],
                         "launch_ms_avg": round(r["ms_per_step"], 4)},
            "cpu_baseline": cpu,
            "per_precision": res,
        }
        print(json.dumps(out), flush=True)
        return

    if args.workload == "ensemble":
        t0 = time.time()
        members = inputs.ensemble()
        log(f"[bench] {len(members)} members generated in {time.time() - t0:.1f} s")
        precs = [p for p in args.precisions.split(",") if p and p != "fp64"] or ["fp32"]
        res = {p: time_ensemble(hevi, members, p, args.steps, args.warmup, args.layout)
               for p in precs}
        r = res[precs[0]]
        out = {
            "metric": METRIC, "value": r["cell_updates_per_s"], "unit": "cell-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" if precs[0] == "fp32" else "f32+f64",
            "data": "synthetic",
            "config": {"workload": f"ensemble of {len(members)} domains, nx, ny in 128..512, "
                                   f"nz in 32/64, per-member dt, n=6", "members": len(members),
                       "cells": r["cells"], "precision": precs[0], "layout": args.layout,
                       "parallelism": "1 GPU"},
            "model_gbps": r["model_gbps"], "model_frac_of_peak": r["model_gbps"] / HBM_PEAK_GBS,
            "per_precision": res,
        }
        print(json.dumps(out), flush=True)
        return

    t0 = time.time()
    s = inputs.workload(args.workload)
    if args.damping:
        s.damping = inputs.damping(s)
    log(f"[bench] state {s.nx}x{s.ny}x{s.nz} generated in {time.time() - t0:.1f} s")
    precs = [p for p in args.precisions.split(",") if p]
    terrain = s.terrain is not None
    # over terrain, every path is also compared with the float64 GPU run
    # (all paths take the same number of long steps from the same state)
    keep = terrain and "fp64" in precs and len(precs) > 1
    res, finals = {}, {}
    for p in precs:
        r = time_precision(hevi, s, p, args.steps, args.warmup, args.layout, keep=keep,
                           short=args.short, tune=not args.no_tune)
        if keep:
            r, finals[p] = r
        res[p] = r
    errors_vs_fp64 = None
    if keep:
        errors_vs_fp64 = {p: field_errors(finals[p], finals["fp64"]) for p in precs if p != "fp64"}
        finals.clear()
    primary = "fp32" if "fp32" in res else precs[0]
    r = res[primary]
    b = BYTES[primary]
    # one launch of the short-step kernel (the Runge-Kutta form launches it
    # twice per short step, the second reading 3 more fields)
    short_ms = r["kernels_ms_avg"]["short_step"]
    ach = short_step_bytes(b, s.cells) / (short_ms * 1e-3) / 1e9
    rec = read_traffic(primary) if args.workload == "large" and args.short == "fb" and \
        not args.damping and args.layout == "kij" else None
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": rec.get("bytes_per_launch") if rec else None,
                "kernel": "short_step", "bytes_per_launch": short_step_bytes(b, s.cells),
                "launch_ms_avg": round(short_ms, 4)}
    if rec:
        # the counters were taken with this tile x-extent (negative: XCD-chunked)
        roofline["traffic_tile_x"] = rec.get("tile_x")
    case = {"large": "large_sub", "terrain": "terrain_sub"}.get(args.workload, "small")
    sub = inputs.workload(case)
    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle baseline")
        cpu, sub_ref = cpu_baseline(s, sub)
        log(f"[bench] oracle: {cpu['value']:.3e} cell-updates/s on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']:.3e} on one")
        if not args.no_accuracy and args.short == "fb" and not args.damping:
            accuracy = accuracy_vs_oracle(hevi, sub, sub_ref, precs, case)
    out = {
        "metric": METRIC,
        "value": r["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if primary == "fp32" else ("f32+f64" if primary == "mixed" else "f64"),
        "data": "synthetic",
        "config": {"workload": f"{s.nx}x{s.ny}x{s.nz} warm bubbles + noise"
                               f"{' over Gaussian hills (max 2 km), shear 0-30 m/s' if terrain else ''}"
                               f", dt=10 s, {s.n_short} short steps/stage",
                   "nx": s.nx, "ny": s.ny, "nz": s.nz, "n_short": s.n_short, "dt": s.dt,
                   "precision": primary, "layout": args.layout, "short_step": args.short,
                   "damping": bool(args.damping), "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "model_gbps": r["model_gbps"],
        "model_frac_of_peak": r["model_gbps"] / HBM_PEAK_GBS,
        "per_precision": res,
    }
    if errors_vs_fp64 is not None:
        out["errors_vs_fp64_gpu"] = errors_vs_fp64
    if accuracy is not None:
        out["accuracy_vs_oracle"] = accuracy
    if "fp64" in res:
        for p in res:
            if p != "fp64":
                out[f"speedup_{p}_vs_fp64"] = res["fp64"]["ms_per_step"] / res[p]["ms_per_step"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
