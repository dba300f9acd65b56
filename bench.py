#!/usr/bin/env python3
"""Throughput of the particle-mesh-particle hot path on one MI355X.

One step = Step 1 (zero the buffer, CIC and supernova deposits with atomic
adds), Step 2 (ghost fold), Steps 3 + 5 (limiter + apply), run through the
C-ABI of libpmp.so on the 256^3 periodic workload: log-normal gas in FP32,
1e6 uniform CIC particles, 1e5 uniform supernovae of radius 4 cells, ghost
width 4.  Inputs are resident in HBM before timing starts.  Prints one JSON
line.

  python bench.py [--steps K] [--warmup W] [--acc f32|f64|fix64]
                  [--workload c2|c3|c3bh|c4|c5|c5s] [--no-cpu] [--no-modes]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published
PHASE_ORDER = ["bin", "tile", "zero", "cic", "sn", "sink_deposit", "fold", "sink_update",
               "apply"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def acc_bytes(acc):
    return 4 if acc == "f32" else 8


def algorithmic_bytes(w, acc, counts, F, fused=False):
    """Bytes per launch each phase must move at minimum (no scratch, no
    re-reads): buffer writes for the zero fill, particle records plus a
    read-modify-write of every touched (cell, field) for deposits, the owned
    shell and its ghost images for the fold, and for apply the buffer in, the
    five state fields in and rho and E out (the momentum is written back only
    where a sink removes mass: no kind deposits momentum).  F = buffer
    channels of the timed layout.  fused: the step applies the interior cells
    (owned, at least g from every face) in the tile pass, which stores the
    buffer only for the other cells, and the shell cells are folded and
    applied in one pass."""
    import numpy as np
    ba = acc_bytes(acc)
    bs = np.dtype(w.state.dtype).itemsize
    n = w.n.astype(np.int64)
    g = w.ghost
    owned = int(np.prod(n, axis=1).sum())
    padded = int(np.prod(n + 2 * g, axis=1).sum())
    ghost_cells = padded - owned
    inner = np.maximum(n - 2 * g, 0)
    shell = owned - int(np.prod(inner, axis=1).sum())
    parts = 0
    if w.cic is not None:
        parts += w.cic.n * 32
    if w.sn is not None:
        parts += w.sn.n * 48
    interior = int(np.prod(np.maximum(n - 2 * g, 0), axis=1).sum())
    st = 7 * bs  # per applied cell: 5 fields in, rho and E out
    removed = counts.get("sink", 0) if w.sinks is not None else 0  # cells with a removal
    out = {
        "zero": padded * F * ba,
        # binned path: every buffer cell stored once plus the particle records
        "tile": padded * F * ba + parts,
        "bin": 0,
        "fold": F * ba * (2 * shell + ghost_cells),
        "apply": owned * (st + F * ba) + 3 * bs * removed,
    }
    if fused:
        # tile: buffer for the non-interior cells, records, interior state in/out
        out["tile"] = (padded - interior) * F * ba + parts + interior * st
        # fold: shell values and their ghost images in, shell state in/out
        out["fold"] = F * ba * (shell + ghost_cells) + shell * st
        out["apply"] = 0
    if w.cic is not None and w.cic.n:
        out["cic"] = w.cic.n * 32 + 2 * ba * counts["cic"]
    if w.sn is not None and w.sn.n:
        out["sn"] = w.sn.n * 48 + 2 * ba * counts["sn"]
    if w.sinks is not None and w.sinks.n:
        out["sink_deposit"] = w.sinks.n * 32 + 2 * ba * counts["sink"] + bs * counts["sink"]
        out["sink_update"] = w.sinks.n * 64 + counts["sink"] * (4 * bs + ba)
    return out


def nominal_step_bytes(w, acc, counts):
    """The method's nominal bytes per step, counted as if every phase ran
    separately with the full channel set (5 fields, 6 with sinks): zero fill,
    particle records, a read-modify-write of every touched (cell, field), the
    sinks' state reads, three accesses per ghost cell and field for the fold,
    and state in/out plus buffer in for the apply.  A yardstick for the whole
    step; the fused path moves far fewer bytes than this."""
    import numpy as np
    ba = acc_bytes(acc)
    bs = np.dtype(w.state.dtype).itemsize
    n = w.n.astype(np.int64)
    g = w.ghost
    owned = int(np.prod(n, axis=1).sum())
    padded = int(np.prod(n + 2 * g, axis=1).sum())
    F = 6 if (w.sinks is not None and w.sinks.n) else 5
    parts = (w.cic.n * 32 if w.cic is not None else 0) + (w.sn.n * 48 if w.sn is not None else 0) + \
        (w.sinks.n * 32 if w.sinks is not None else 0)
    touched = counts.get("cic", 0) + counts.get("sn", 0) + counts.get("sink", 0)
    return (padded * F * ba + parts + 2 * ba * touched + 5 * bs * counts.get("sink", 0)
            + 3 * ba * F * (padded - owned) + owned * F * (2 * bs + ba))


def touched_counts(B, w, acc):
    """Unique (cell, field) pairs each particle kind writes, counted as the
    nonzero buffer entries after depositing that kind alone (all
    contributions are positive)."""
    import dataclasses
    import torch
    counts = {}
    for kind in ("cic", "sn", "sinks"):
        P = getattr(w, kind)
        if P is None or P.n == 0:
            continue
        kw = {"cic": None, "sn": None, "sinks": None}
        kw[kind] = P
        wk = dataclasses.replace(w, **kw)
        if kind != "sinks" and w.sinks is not None:
            wk = dataclasses.replace(wk, sinks=None)
        ctx = B.Context(wk, acc)
        ctx.deposit()
        torch.cuda.synchronize()
        counts["sink" if kind == "sinks" else kind] = int(torch.count_nonzero(ctx.buf).item())
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    return counts


def run_steps(ctx, steps, warmup, profile=True):
    import torch
    for _ in range(warmup):
        ctx.step()
    torch.cuda.synchronize()
    if profile:
        ctx.profile_begin(steps)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        ctx.step()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    phases = ctx.profile_end() if profile else {}
    return ms, phases


def run_graph(ctx, steps, warmup, spread=None):
    """ms per step of a captured one-step HIP graph, replayed `steps` times
    after `warmup` untimed replays, with one event on each side of the timed
    replays.  `spread`, a dict, receives the median, min and max of a second
    pass of as many replays with an event between every two."""
    import statistics
    import torch
    ctx.graph_build(1)
    for _ in range(warmup):
        ctx.graph_launch()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        ctx.graph_launch()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    if spread is not None:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for i in range(steps):
            ctx.graph_launch()
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        spread.update({"median": statistics.median(per), "min": min(per), "max": max(per)})
    return ms


def sink_create_rate(B, w, acc, channels, reps=10):
    """Sink creation (Sec. 3.1.2) after one step: rho_Tr = e^3 (about one cell
    in 700 of the log-normal gas lies above it), r_K the workload's.  Each
    timed call starts from the same post-step state (restored outside the
    timed region).  Algorithmic bytes: rho and K of every cell."""
    import math

    import numpy as np
    import torch
    ctx = B.Context(w, acc, channels=channels)
    ctx.step()
    torch.cuda.synchronize()
    base = ctx.state.clone()
    rho_tr, max_new = math.exp(3.0), 65536
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    total, n = 0.0, 0
    for r in range(reps + 1):
        ctx.state.copy_(base)
        torch.cuda.synchronize()
        t0.record()
        out, work = ctx.sink_create(w.r_k, rho_tr, max_new)
        t1.record()
        torch.cuda.synchronize()
        if r:  # the first call warms up
            total += t0.elapsed_time(t1)
        n = int(work[0].item())
    ctx.close()
    ms = total / reps
    bs = np.dtype(w.state.dtype).itemsize
    ba = {"f32": 4, "f64": 8, "fix64": 8}[acc]
    nbytes = w.owned_cells * (bs + ba)
    return {"ms_per_call": round(ms, 4), "new_sinks": n, "rho_tr": rho_tr, "r_k": w.r_k,
            "algo_GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "kernels": "k_create_find+k_create_rank+k_create_apply"}


def stream_copy_gbps(B, nbytes=1 << 30, reps=10):
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    B.stream_copy(b, a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        B.stream_copy(b, a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


def traffic_for(workload, kernel):
    """Measured HBM bytes per launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if kernel not in rec.get("kernels", {}):
        return None
    src = os.path.join(ROOT, "paper_2509_18261_amd", "csrc", "pmp_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("kernel_source_sha256_16") != h:
        return None
    return rec["kernels"][kernel]["hbm_bytes_per_launch"]


def batched_comparison(ctx, args, eager_ms):
    """Multi-box layouts: the batched step (one launch per kernel over every
    box), the same steps captured in one HIP graph, and the per-box launch
    baseline (every kernel launched once per box)."""
    import torch
    n = args.graph_steps
    ctx.graph_build(n)
    ctx.graph_launch()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    t0.record()
    for _ in range(reps):
        ctx.graph_launch()
    t1.record()
    torch.cuda.synchronize()
    graph_ms = t0.elapsed_time(t1) / (reps * n)
    log(f"graph: {graph_ms:.4f} ms/step ({n} steps per graph)")
    tun = ctx.tuning()
    pb_steps = 3
    ctx.step_per_box()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(pb_steps):
        ctx.step_per_box()
    t1.record()
    torch.cuda.synchronize()
    per_box_ms = t0.elapsed_time(t1) / pb_steps
    log(f"per-box launches: {per_box_ms:.3f} ms/step")
    return {"boxes": ctx.w.nbox, "eager_batched_ms_per_step": eager_ms,
            "graph_ms_per_step": graph_ms, "graph_steps": n,
            "per_box_launch_ms_per_step": per_box_ms,
            "per_box_launches_per_step": 5 * ctx.w.nbox,
            "speedup_graph_vs_per_box": per_box_ms / graph_ms,
            "tuning": tun.as_dict()}


def repro_rates(B, w, channels):
    """Fraction of the deposited buffer's nonzero elements that are bit-identical
    between two deposits of the same inputs: the same launch again, and tiles
    of another shape (another summation order), for FP64 sums, the
    reproducibility mode (App. A.1 error bound and truncation) and int64
    fixed point."""
    import numpy as np
    import torch
    out = {}
    shapes = ({}, {}, {"tile_x": 32, "tile_yz": 4, "tile_block": 128})
    for acc in ("f64", "f64r", "fix64"):
        bufs = []
        for tun in shapes:
            ctx = B.Context(w, acc, channels=channels)
            ctx.set_tuning(deposit_path=1, **tun)
            ctx.deposit()
            torch.cuda.synchronize()
            bufs.append(ctx.buf.cpu().numpy().copy())
            ctx.close()
            del ctx
            torch.cuda.empty_cache()
        nz = bufs[0] != 0
        out[acc] = {"elements": int(nz.sum()),
                    "same_launch": float(np.mean(bufs[0][nz] == bufs[1][nz])),
                    "other_tiles": float(np.mean(bufs[0][nz] == bufs[2][nz]))}
    return out


def cpu_baseline(w, n_particles, target_s=10.0):
    import oracle
    ncores = 1
    times = []
    t_start = time.perf_counter()
    while True:
        times.append(oracle.timed_step(w, "f64"))
        if time.perf_counter() - t_start >= target_s or len(times) >= 5:
            break
    t = min(times)
    cpu = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": n_particles / t, "unit": "particles/s", "cores": ncores, "kind": "oracle",
            "host_cpu": cpu, "host_cpus_visible": os.cpu_count(),
            "sample": f"{len(times)} full serial FP64 oracle steps of the same workload "
                      f"(deposit, fold, apply; {t:.2f} s each, best taken)",
            "cells_per_s": w.owned_cells / t, "s_per_step": t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--acc", default="f32", choices=["f32", "f64", "fix64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--no-calib", action="store_true")
    ap.add_argument("--set", default="", help="tuning overrides, e.g. deposit_path=0,tile_x=32")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the library's autotuner (default: tune, cached per shape)")
    ap.add_argument("--channels", default="auto",
                    help='buffer channels: "auto" (only those deposited into) or "all"')
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="steps per captured graph in the batched comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: bench.py measures one MI355X only; "
                                   f"--gpus {args.gpus} is not supported"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_18261_amd import binding as B
    from paper_2509_18261_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"bench: workload {args.workload}, acc {args.acc}, steps {args.steps}")
    w = W.CONFIGS[args.workload]()
    nparts = sum(P.n for P in (w.cic, w.sn, w.sinks) if P is not None)
    counts = touched_counts(B, w, args.acc)
    log("touched (cell, field) pairs:", counts)
    overrides = {}
    for kv in filter(None, args.set.split(",")):
        k, v = kv.split("=")
        overrides[k.strip()] = int(v)
    ctx = B.Context(w, args.acc, channels=args.channels)
    nchan = len(ctx.fields)
    log(f"buffer channels {ctx.fields}")
    tuned = None
    if not args.no_autotune and not overrides:
        from paper_2509_18261_amd import autotune
        cache = os.path.join(ROOT, "gpurun_out", "autotune_cache.json")
        tuned = autotune.tune(ctx, cache_path=cache)
        log(f"autotune: {tuned}")
    if overrides:
        ctx.set_tuning(**overrides)
    # headline: the step replayed from a captured HIP graph; eager launches
    # and the per-phase profile (events between phases) in runs of their own
    eager_ms, _ = run_steps(ctx, args.steps, args.warmup, profile=False)
    spread = {}
    ms = run_graph(ctx, args.steps, args.warmup, spread)
    _, phases = run_steps(ctx, args.steps, 2, profile=True)
    st = ctx.status()
    log(f"step {ms:.4f} ms (graph), {eager_ms:.4f} ms (eager); status {st}")
    tun = ctx.tuning().as_dict()
    batched = None
    if w.nbox > 1 and (w.sinks is None or w.sinks.n == 0):
        # the per-box launch form has no sinks, so it is compared only without them
        batched = batched_comparison(ctx, args, eager_ms)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    fused = bool(tun.get("fuse_apply", 0)) and tun.get("deposit_path", 0) == 1 and \
        (w.sinks is None or w.sinks.n == 0) and nparts > 0
    algo = algorithmic_bytes(w, args.acc, counts, nchan, fused)
    per_phase = {}
    for name in PHASE_ORDER:
        if name not in phases:
            continue
        tot_ms, nl = phases[name]
        avg = tot_ms / nl
        b = algo.get(name, 0)
        per_phase[name] = {"avg_ms": round(avg, 5), "launches": nl,
                           "algo_bytes": int(b),
                           "GBps": round(b / (avg * 1e-3) / 1e9, 1) if avg > 0 else None}
    # dominant kernel: the longest single kernel that moves algorithmic bytes
    # (the binning phase is several small launches of scratch traffic)
    dom = max((k for k in per_phase if per_phase[k]["algo_bytes"] > 0),
              key=lambda k: per_phase[k]["avg_ms"])
    kernel_names = {"bin": "k_sn_count+k_l1_*+k_scan_*+k_l2_*+k_units", "tile": "k_tile_deposit",
                    "zero": "k_zero", "cic": "k_cic_direct", "sn": "k_sn_direct",
                    "sink_deposit": "k_sink_deposit", "fold": "k_fold_apply" if fused else "k_fold",
                    "sink_update": "k_sink_update", "apply": "k_apply"}
    d = per_phase[dom]
    achieved = d["algo_bytes"] / (d["avg_ms"] * 1e-3) / 1e9
    step_bytes = sum(algo.get(k, 0) for k in per_phase)
    out = {
        "metric": "particle-deposits/s and mesh cells applied/s; % HBM roofline vs plain FP64",
        "value": nparts / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_spread": {k: round(v, 5) for k, v in spread.items()},
        "eager_ms_per_step": eager_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.acc,
        "data": "synthetic (seeded; stands in for the paper's AGORA galaxy run)",
        "config": {"workload": w.name, "cells": w.owned_cells,
                   "cic": w.cic.n if w.cic else 0, "sn": w.sn.n if w.sn else 0,
                   "sinks": w.sinks.n if w.sinks else 0, "ghost": w.ghost,
                   "state": str(np.dtype(w.state.dtype)), "acc": args.acc,
                   "limiter": "f64", "boxes": w.nbox, "buffer_channels": nchan,
                   "fused_apply": fused},
        "cells_per_s": w.owned_cells / (ms * 1e-3),
        "step_algo_bytes": int(step_bytes),
        "step_hbm_frac": step_bytes / (ms * 1e-3) / (HBM_PEAK_GBPS * 1e9),
        # the unfused, full-channel count of the same step (a yardstick, not traffic)
        "step_nominal_bytes": int(nominal_step_bytes(w, args.acc, counts)),
        "step_nominal_frac": nominal_step_bytes(w, args.acc, counts) / (ms * 1e-3) /
                             (HBM_PEAK_GBPS * 1e9),
        "roofline": {"bound": "hbm", "kernel": kernel_names[dom], "phase": dom,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_for(args.workload, kernel_names[dom]),
                     "algo_bytes_per_launch": d["algo_bytes"],
                     "avg_launch_ms": d["avg_ms"]},
        "phases": per_phase,
        "tuning": tun,
        "autotune": tuned,
        "status_flags": st["flag_names"],
    }
    if batched is not None:
        out["batched"] = batched
    if w.sinks is not None and w.sinks.n and w.nbox == 1:
        out["sink_create"] = sink_create_rate(B, w, args.acc, args.channels)
        log(f"sink creation: {out['sink_create']}")
    if not args.no_calib:
        gbps, cms = stream_copy_gbps(B)
        out["stream_copy_GBps"] = round(gbps, 1)
        log(f"stream copy {gbps:.0f} GB/s")
    if not args.no_modes:
        modes = {}
        for acc, dt in (("fix64", None), ("f64r", None), ("f64", np.float64)):
            if acc == "f64r" and (overrides or {}).get("deposit_path", 1) != 1:
                continue  # the reproducibility mode runs on the binned path only
            wm = w.with_state(w.state.astype(dt)) if dt is not None else w
            c2 = B.Context(wm, acc, channels=args.channels)
            if overrides:
                c2.set_tuning(**overrides)
            mms = run_graph(c2, max(5, args.steps // 2), 2)
            c2.close()
            del c2
            torch.cuda.empty_cache()
            modes[acc if dt is None else "f64_plain"] = {
                "ms_per_step": mms, "particles_per_s": nparts / (mms * 1e-3),
                "cells_per_s": w.owned_cells / (mms * 1e-3),
                "state": "f64" if dt is not None else str(np.dtype(w.state.dtype))}
            log(f"mode {acc}: {mms:.4f} ms/step")
        out["modes"] = modes
        out["speedup_vs_plain_f64"] = modes["f64_plain"]["ms_per_step"] / ms
        out["reproducibility"] = repro_rates(B, w, args.channels)
        log(f"reproducibility: {out['reproducibility']}")
    if not args.no_cpu:
        log("cpu baseline (serial oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, nparts)
        log(f"oracle {out['cpu_baseline']['s_per_step']:.2f} s/step")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
