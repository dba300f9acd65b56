#!/usr/bin/env python3
"""Throughput of the particle-mesh-particle hot path on one MI355X.

One step = Step 1 (CIC and supernova deposits into a zeroed, ghost-zoned
buffer), Step 2 (ghost fold), Steps 3 + 5 (limiter + apply), run through the
C-ABI of libpmp.so.  Default workload: the 512^3 periodic box (log-normal
gas, 4e6 particles, half uniform and half in 32 Plummer clumps, CIC:SN 10:1,
supernova radius 3, ghost width 4) with FP64 state and FP64 buffer; inputs
are resident in HBM before timing starts.  Also reported: the FP32 and
fixed-point modes, the plain FP64 path (direct atomics, nothing fused), the
atomic and copy peaks, the 4096-box batched level against per-box launches,
and the serial oracle on the host.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--acc f32|f64|fix64] [--state f32|f64]
                  [--workload c2|c3|c3bh|c4|c5|c5s] [--no-cpu] [--no-modes]
                  [--no-calib] [--no-c5]
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


def _shape(w):
    import numpy as np
    n = w.n.astype(np.int64)
    g = w.ghost
    owned = int(np.prod(n, axis=1).sum())
    padded = int(np.prod(n + 2 * g, axis=1).sum())
    interior = int(np.prod(np.maximum(n - 2 * g, 0), axis=1).sum())
    return owned, padded, interior


def record_bytes(w):
    """Particle records read: CIC x, y, z, m (32 B); supernova x, y, z, m, e,
    r (48 B); sink x, y, z, a (32 B)."""
    return sum(P.n * nb for P, nb in ((w.cic, 32), (w.sn, 48), (w.sinks, 32)) if P is not None)


def method_bytes(w, acc, counts, F, applied=None):
    """The method's own HBM bytes per step (Sec. 2.2 Steps 1-5 as written,
    every phase separate, only the F buffer channels the particle kinds
    deposit into; no binning or scratch traffic, nothing fused):
      zero      F b_acc per padded cell;
      records   per particle (record_bytes);
      deposit   2 b_acc per unique touched (cell, channel) (read-modify-write);
      sinks     5 b_state per sink-kernel cell (the state the request reads);
      fold      3 b_acc per ghost cell and channel (ghost in, owner in/out);
      apply     per owned cell the F channels in; per updated cell (some
                channel nonzero, counted by applied_cells; a cell without an
                update keeps its state) 5 b_state in (the energy limiter
                needs |p|^2) and rho and E out (2 b_state); the momentum out
                (3 b_state) only in cells a sink removes from (no kind
                deposits momentum, so elsewhere it does not change);
      sink update: 64 B per sink (record, gains out) and per kernel cell
                4 b_state (rho, p) + b_acc (K).
    """
    import numpy as np
    ba = acc_bytes(acc)
    bs = np.dtype(w.state.dtype).itemsize
    owned, padded, _ = _shape(w)
    ks = counts.get("sink", 0)
    touched = counts.get("cic", 0) + counts.get("sn", 0) + ks
    out = {
        "zero": padded * F * ba,
        "records": record_bytes(w),
        "deposit": 2 * ba * touched + 5 * bs * ks,
        "fold": 3 * ba * F * (padded - owned),
        "apply": owned * F * ba + 7 * bs * (owned if applied is None else applied["total"]) +
                 3 * bs * ks,
        "sink_update": (w.sinks.n * 64 + ks * (4 * bs + ba)) if w.sinks is not None else 0,
    }
    out["total"] = sum(out.values())
    return out


def kernel_method_bytes(w, acc, counts, F, fused, applied=None, owner=False):
    """The method's bytes that each kernel of the timed step carries (the
    terms of method_bytes assigned to the kernel that does that work).
    Binned path: the tile pass does the zero fill, reads the records and
    performs every deposit read-modify-write (in LDS; counted as the method's
    HBM bytes all the same); fused (no sinks), it also applies the interior
    cells (owned, at least g from every face), and the shell kernel folds and
    applies the rest.  On owner tiles (fuse_apply 2: no ghost zone, no fold)
    the tile pass processes every owned cell as the fused pass processes the
    interior ones: records, deposits, each owned cell's buffer value and the
    updated cells' state; the zero fill and the fold, which it never
    performs, stay out of its bytes (they remain in the step's).  Direct
    path: zero fill, CIC and supernova atomics, fold, apply, one kernel
    each."""
    import numpy as np
    ba = acc_bytes(acc)
    bs = np.dtype(w.state.dtype).itemsize
    owned, padded, interior = _shape(w)
    if applied is None:
        applied = {"interior": interior, "shell": owned - interior, "total": owned}
    dep = 2 * ba * (counts.get("cic", 0) + counts.get("sn", 0))
    out = {
        "tile": padded * F * ba + record_bytes(w) - (w.sinks.n * 32 if w.sinks else 0) + dep,
        "zero": padded * F * ba,
        "fold": 3 * ba * F * (padded - owned),
        "apply": owned * F * ba + 7 * bs * applied["total"] + 3 * bs * counts.get("sink", 0),
        "bin": 0,
    }
    if fused:
        out["tile"] = (padded - interior) * F * ba + record_bytes(w) + dep + \
            interior * F * ba + 7 * bs * applied["interior"]
        out["fold"] = 3 * ba * F * (padded - owned) + (owned - interior) * F * ba + \
            7 * bs * applied["shell"]
        out["apply"] = 0
    if owner:
        out["tile"] = record_bytes(w) + dep + owned * F * ba + 7 * bs * applied["total"]
        out["fold"] = 0
    if w.cic is not None and w.cic.n:
        out["cic"] = w.cic.n * 32 + 2 * ba * counts["cic"]
    if w.sn is not None and w.sn.n:
        out["sn"] = w.sn.n * 48 + 2 * ba * counts["sn"]
    if w.sinks is not None and w.sinks.n:
        ks = counts["sink"]
        out["sink_deposit"] = w.sinks.n * 32 + 2 * ba * ks + 5 * bs * ks
        out["sink_update"] = w.sinks.n * 64 + ks * (4 * bs + ba)
    return out


def touched_counts(B, w, acc):
    """Unique (cell, field) pairs each particle kind writes, counted as the
    nonzero buffer entries after depositing that kind alone (all
    contributions are positive), on the direct path so that the timed
    kernels' profile holds only the timed launches."""
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
        ctx.set_tuning(deposit_path=0)
        ctx.deposit()
        torch.cuda.synchronize()
        counts["sink" if kind == "sinks" else kind] = int(torch.count_nonzero(ctx.buf).item())
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    return counts


def applied_cells(B, w, acc):
    """Owned cells whose folded buffer is nonzero in some channel: the cells
    Steps 3 + 5 update (a cell without an update keeps its state), split into
    those at least g from every face of their box (the fused tile pass
    applies them) and the rest.  Counted after a deposit and fold on the
    direct path."""
    import numpy as np
    import torch
    ctx = B.Context(w, acc, channels="all")
    ctx.set_tuning(deposit_path=0)
    ctx.deposit()
    ctx.ghost_fold()
    torch.cuda.synchronize()
    g = w.ghost
    F = len(ctx.fields)
    inner = shell = 0
    off = 0
    for n in w.n.astype(np.int64):
        p = n + 2 * g
        npad = int(np.prod(p))
        blk = ctx.buf[off: off + F * npad].view(F, int(p[2]), int(p[1]), int(p[0]))
        own = (blk[:, g:g + n[2], g:g + n[1], g:g + n[0]] != 0).any(dim=0)
        tot = int(own.sum().item())
        if (n > 2 * g).all():
            core = own[g:n[2] - g, g:n[1] - g, g:n[0] - g]
            ci = int(core.sum().item())
        else:
            ci = 0
        inner += ci
        shell += tot - ci
        off += F * npad
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return {"interior": inner, "shell": shell, "total": inner + shell}


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
        out, work = ctx.sink_create(w.r_k, rho_tr, max_new, existing="workload")
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


def snr_rate(B, reps=10):
    """Supernova remnants (TIGRESS variant, pmp_deposit_snr) on a 256^3 slab
    box (mean densities 0.05, 1 and 30: all three regimes), FP64 state and
    buffer, 20000 remnants, r_K = 3, 4^3 sample points per cell: the call
    alone, after a deposit, averaged over `reps` calls."""
    import numpy as np
    import torch
    from paper_2509_18261_amd import workloads as W
    w = W.snr_box(nx=256, n_snr=20000, seed=31, dtype=np.float64)
    ctx = B.Context(w, "f64", channels="all")
    ctx.deposit()
    info = torch.zeros(4 * w.snr.n, dtype=torch.float64, device="cuda")
    ctx.deposit_snr(info)
    torch.cuda.synchronize()
    ctx.profile_begin(reps)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        ctx.deposit_snr(info)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    ph = ctx.profile_end()
    inf = info.cpu().numpy().reshape(4, -1)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    rm = inf[1] / (1679.0 * inf[2] ** -0.26)
    kern_ms = ph["snr"][0] / ph["snr"][1] if "snr" in ph else None
    return {"workload": w.name, "ms_per_call": round(ms, 4), "kernel_ms": kern_ms,
            "remnants_per_s": w.snr.n / (ms * 1e-3), "sub": w.snr_params.sub,
            "r_k": w.snr_params.r_k,
            "regimes": {"MC": int((rm > 1).sum()), "ST": int(((rm > 0.027) & (rm <= 1)).sum()),
                        "EJ": int((rm <= 0.027).sum())},
            "kernel": "k_snr_deposit (one workgroup per remnant: 9^3 candidate cells x 4^3 "
                      "sample points, twice; bound by the sample tests, not by memory)"}


def copy_gbps(B, nbytes=1 << 30, reps=10):
    """Device copy bandwidth (bytes read + written per second) of the
    library's two copy kernels and the runtime's hipMemcpyAsync."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    out = {}
    for variant, name in ((0, "k_copy"), (1, "k_copy4"), (2, "hipMemcpyAsync")):
        B.copy_bench(b, a, variant)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            B.copy_bench(b, a, variant)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def atomic_rates(B, slots_log2=26, reps=3):
    """Global-atomic throughput (adds per second) measured by the library's
    microbenchmark: int64, f32 and f64 adds on coalesced and scattered
    distinct addresses (2^26 elements) and on one contended address."""
    import torch
    out = {}
    dt = {"int64": torch.int64, "f32": torch.float32, "f64": torch.float64}
    for tname, tdt in dt.items():
        buf = torch.zeros(1 << slots_log2, dtype=tdt, device="cuda")
        out[tname] = {}
        for pat, n_ops in (("coalesced", 1 << 28), ("scattered", 1 << 28),
                           ("same_address", 1 << 22)):
            B.atomic_bench(buf, tname, pat, n_ops)
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(reps):
                B.atomic_bench(buf, tname, pat, n_ops)
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / reps
            out[tname][pat] = n_ops / (ms * 1e-3)
        del buf
        torch.cuda.empty_cache()
    return out


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
    # the per-box baseline runs the direct path (zero fill, global atomics,
    # fold, apply); the same path batched (one launch per kernel over every
    # box, eager) separates the gain of batching from that of the binned path
    d = tun.as_dict()
    ctx.set_tuning(**{**d, "deposit_path": 0, "fuse_apply": 0})
    ctx.step()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(pb_steps):
        ctx.step()
    t1.record()
    torch.cuda.synchronize()
    direct_ms = t0.elapsed_time(t1) / pb_steps
    ctx.set_tuning(**d)
    log(f"batched direct path: {direct_ms:.3f} ms/step")
    return {"boxes": ctx.w.nbox, "eager_batched_ms_per_step": eager_ms,
            "graph_ms_per_step": graph_ms, "graph_steps": n,
            "per_box_launch_ms_per_step": per_box_ms,
            "per_box_launches_per_step": 5 * ctx.w.nbox,
            "speedup_graph_vs_per_box": per_box_ms / graph_ms,
            "batched_direct_path_ms_per_step": direct_ms,
            "speedup_batching_direct_path": per_box_ms / direct_ms,
            "speedup_binned_vs_direct_batched": direct_ms / eager_ms,
            "tuning": d}


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


def cpu_baseline(w, n_particles):
    """One full serial FP64 step of the oracle on the headline workload (the
    oracle as it stands, single-threaded: deposit, fold, limiter + apply)."""
    import oracle
    t = oracle.timed_step(w, "f64")
    cpu = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": n_particles / t, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "host_cpu": cpu, "host_cpus_visible": os.cpu_count(),
            "sample": f"one full serial FP64 oracle step of the same workload ({w.name}: "
                      f"deposit, fold, limiter + apply; {t:.2f} s)",
            "cells_per_s": w.owned_cells / t, "s_per_step": t}


def sn_contributions(w):
    """Supernova (cell, channel) contributions of one step, counted on the
    host from the sphere membership test (cell centre within r, inclusive):
    two channels (rho, E) per member cell."""
    import numpy as np
    if w.sn is None or w.sn.n == 0:
        return 0
    total = 0
    f = w.sn.fields
    for s0 in range(0, w.sn.n, 1 << 16):
        x, y, z, r = (f[k][s0:s0 + (1 << 16)] for k in ("x", "y", "z", "r"))
        r2 = r * r
        span = int(np.ceil(r.max())) * 2 + 2
        cnt = np.zeros(x.size, dtype=np.int64)
        lo = [np.ceil(p - r - 0.5 - 1e-6).astype(np.int64) for p in (x, y, z)]
        for dk in range(span):
            ddz = (lo[2] + dk + 0.5) - z
            for dj in range(span):
                ddy = (lo[1] + dj + 0.5) - y
                for di in range(span):
                    ddx = (lo[0] + di + 0.5) - x
                    cnt += ((ddx * ddx + ddy * ddy) + ddz * ddz) <= r2
        total += int(cnt.sum())
    return 2 * total


def tuned_context(B, w, acc, channels, overrides=None, autotune_on=True):
    ctx = B.Context(w, acc, channels=channels)
    tuned = None
    if autotune_on and not overrides:
        from paper_2509_18261_amd import autotune
        cache = os.path.join(ROOT, "gpurun_out", "autotune_cache.json")
        tuned = autotune.tune(ctx, cache_path=cache)
    if overrides:
        ctx.set_tuning(**overrides)
    return ctx, tuned


def measure(ctx, steps, warmup):
    """Headline timing: the step replayed from a captured one-step HIP graph;
    eager launches and the per-kernel profile (HIP events around every
    kernel, on the stream it runs on) in passes of their own."""
    eager_ms, _ = run_steps(ctx, steps, warmup, profile=False)
    spread = {}
    ms = run_graph(ctx, steps, warmup, spread)
    _, phases = run_steps(ctx, steps, 2, profile=True)
    return ms, eager_ms, spread, phases, ctx.status()


KERNELS = {"bin": "k_sn_count+k_l1_*+k_scan_*+k_l2_*+k_units", "tile": "k_tile_deposit",
           "zero": "k_zero", "cic": "k_cic_direct", "sn": "k_sn_direct",
           "sink_deposit": "k_sink_deposit", "fold": "k_fold", "sink_update": "k_sink_update",
           "apply": "k_apply"}


def phase_table(phases, kbytes):
    out = {}
    for name in PHASE_ORDER:
        if name not in phases:
            continue
        tot_ms, nl = phases[name]
        avg = tot_ms / nl
        b = kbytes.get(name, 0)
        out[name] = {"avg_ms": round(avg, 5), "launches": nl, "method_bytes": int(b),
                     "GBps": round(b / (avg * 1e-3) / 1e9, 1) if avg > 0 else None}
    return out


def is_fused(tun, w, nparts):
    return bool(tun.get("fuse_apply", 0)) and tun.get("deposit_path", 0) == 1 and \
        (w.sinks is None or w.sinks.n == 0) and nparts > 0


def run_mode(B, w, acc, counts_acc, args, overrides=None, autotune_on=True, steps=None,
             applied=None):
    """A timed run of one (state, accumulator) mode: ms per step (graph),
    the per-kernel table and the step's method bytes."""
    import torch
    nparts = sum(P.n for P in (w.cic, w.sn, w.sinks) if P is not None)
    ctx, tuned = tuned_context(B, w, acc, args.channels, overrides, autotune_on)
    nchan = len(ctx.fields)
    ms, eager_ms, spread, phases, st = measure(ctx, steps or args.steps, args.warmup)
    tun = ctx.tuning().as_dict()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    fused = is_fused(tun, w, nparts)
    # owner tiles: the library ran the fold-free step (no fold launch)
    owner = fused and tun.get("fuse_apply") == 2 and "fold" not in phases
    mb = method_bytes(w, acc, counts_acc, nchan, applied)
    table = phase_table(phases, kernel_method_bytes(w, acc, counts_acc, nchan, fused, applied,
                                                    owner))
    return {"ms_per_step": ms, "eager_ms_per_step": eager_ms, "spread": spread,
            "particles_per_s": nparts / (ms * 1e-3), "cells_per_s": w.owned_cells / (ms * 1e-3),
            "state": str(w.state.dtype), "acc": acc, "tuning": tun, "autotune": tuned,
            "fused_apply": 2 if owner else int(fused), "buffer_channels": nchan,
            "phases": table,
            "step_method_bytes": mb["total"],
            "step_method_frac": mb["total"] / (ms * 1e-3) / (HBM_PEAK_GBPS * 1e9),
            "status_flags": st["flag_names"]}


def c5_batched(B, args):
    """The batched AMR level (4096 uneven boxes, FP32): the step replayed
    from a graph of 10 steps, autotuned, against the per-box launch form."""
    import torch
    from paper_2509_18261_amd import workloads as W
    w = W.c5()
    ctx, tuned = tuned_context(B, w, "f32", args.channels)
    eager_ms, _ = run_steps(ctx, 5, 2, profile=False)
    res = batched_comparison(ctx, args, eager_ms)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    nparts = w.cic.n + w.sn.n
    res.update({"workload": w.name, "acc": "f32", "state": "float32", "particles": nparts,
                "particles_per_s_graph": nparts / (res["graph_ms_per_step"] * 1e-3),
                "autotune": tuned})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--acc", default="f64", choices=["f32", "f64", "fix64"])
    ap.add_argument("--state", default="f64", choices=["f32", "f64"],
                    help="gas state type (the workload's FP32 draw, promoted for f64)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--no-calib", action="store_true", help="skip the copy and atomic peaks")
    ap.add_argument("--no-atomics", action="store_true", help="skip the atomic peaks")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 path")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the supernova-remnant and sink-creation legs")
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
    log(f"bench: workload {args.workload}, state {args.state}, acc {args.acc}, "
        f"steps {args.steps}")
    w32 = W.CONFIGS[args.workload]()
    w = w32.with_state(w32.state.astype(np.float64)) if args.state == "f64" else w32
    nparts = sum(P.n for P in (w.cic, w.sn, w.sinks) if P is not None)
    counts = touched_counts(B, w, args.acc)
    log("touched (cell, channel) pairs:", counts)
    applied = applied_cells(B, w, args.acc)
    log("updated cells:", applied)
    overrides = {}
    for kv in filter(None, args.set.split(",")):
        k, v = kv.split("=")
        overrides[k.strip()] = int(v)

    head = run_mode(B, w, args.acc, counts, args, overrides, not args.no_autotune,
                    applied=applied)
    ms = head["ms_per_step"]
    log(f"step {ms:.4f} ms (graph), {head['eager_ms_per_step']:.4f} ms (eager); "
        f"flags {head['status_flags']}")
    batched = None
    if w.nbox > 1 and (w.sinks is None or w.sinks.n == 0):
        ctx, _ = tuned_context(B, w, args.acc, args.channels, overrides, not args.no_autotune)
        batched = batched_comparison(ctx, args, head["eager_ms_per_step"])
        ctx.close()
        del ctx
        torch.cuda.empty_cache()

    per_phase = head["phases"]
    # dominant kernel: the longest single kernel that carries method bytes
    # (binning is several small launches of scratch traffic)
    dom = max((k for k in per_phase if per_phase[k]["method_bytes"] > 0),
              key=lambda k: per_phase[k]["avg_ms"])
    d = per_phase[dom]
    achieved = d["method_bytes"] / (d["avg_ms"] * 1e-3) / 1e9
    kname = KERNELS[dom]
    if dom == "fold" and head["fused_apply"]:
        kname = "k_fold_apply"
    mb = method_bytes(w, args.acc, counts, head["buffer_channels"], applied)
    step_gbps = mb["total"] / (ms * 1e-3) / 1e9
    out = {
        "metric": "particle-deposits/s and mesh cells applied/s; % HBM roofline vs plain FP64",
        "value": nparts / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_spread": {k: round(v, 5) for k, v in head["spread"].items()},
        "eager_ms_per_step": head["eager_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.acc,
        "data": "synthetic (seeded; stands in for the paper's AGORA galaxy run)",
        "config": {"workload": w.name, "cells": w.owned_cells,
                   "cic": w.cic.n if w.cic else 0, "sn": w.sn.n if w.sn else 0,
                   "sinks": w.sinks.n if w.sinks else 0, "ghost": w.ghost,
                   "state": str(np.dtype(w.state.dtype)), "acc": args.acc,
                   "limiter": "f64", "boxes": w.nbox,
                   "buffer_channels": head["buffer_channels"],
                   "fused_apply": head["fused_apply"]},
        "cells_per_s": w.owned_cells / (ms * 1e-3),
        "roofline": {"bound": "hbm", "kernel": kname, "phase": dom,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_for(args.workload, kname),
                     "method_bytes_per_launch": d["method_bytes"],
                     "avg_launch_ms": d["avg_ms"]},
        # the whole step: the method's own bytes (every phase separate, the
        # deposited channels only) over the step time
        "updated_cells": applied,
        "step_roofline": {"bound": "hbm", "achieved": round(step_gbps, 1),
                          "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                          "frac": round(step_gbps / HBM_PEAK_GBPS, 4),
                          "method_bytes": mb},
        "phases": per_phase,
        "tuning": head["tuning"],
        "autotune": head["autotune"],
        "status_flags": head["status_flags"],
    }
    if batched is not None:
        out["batched"] = batched
    if w.sinks is not None and w.sinks.n and w.nbox == 1:
        out["sink_create"] = sink_create_rate(B, w, args.acc, args.channels)
        log(f"sink creation: {out['sink_create']}")
    if not args.no_modes:
        modes = {}
        for acc, wm in (("f32", w32), ("fix64", w32)):
            if acc == args.acc and wm is w:
                continue
            # the same particles touch the same (cell, channel) pairs in every mode
            modes[f"{acc}_state_{wm.state.dtype}"] = run_mode(B, wm, acc, counts, args, None,
                                                              True, max(5, args.steps // 2),
                                                              applied)
            log(f"mode {acc}: {modes[f'{acc}_state_{wm.state.dtype}']['ms_per_step']:.4f} ms")
        if w.sinks is None or w.sinks.n == 0:
            modes["f64r_state_" + str(w.state.dtype)] = run_mode(
                B, w, "f64r", counts, args, {"deposit_path": 1}, False, max(5, args.steps // 2),
                applied)
        out["modes"] = modes
        out["reproducibility"] = repro_rates(B, w, args.channels)
        log(f"reproducibility: {out['reproducibility']}")
    if not args.no_plain:
        # the plain FP64 path: zero fill, direct global atomics, separate
        # fold and apply, no binning or fusion
        wp = w if args.state == "f64" else w32.with_state(w32.state.astype(np.float64))
        plain = run_mode(B, wp, "f64", counts, args, {"deposit_path": 0, "fuse_apply": 0},
                         False, max(5, args.steps // 2), applied)
        out["plain_f64"] = plain
        out["speedup_vs_plain_f64"] = plain["ms_per_step"] / ms
        log(f"plain f64: {plain['ms_per_step']:.4f} ms")
    if not args.no_calib:
        out["copy_GBps"] = copy_gbps(B)
        log(f"copy: {out['copy_GBps']}")
    if not args.no_calib and not args.no_atomics:
        rates = atomic_rates(B)
        out["atomics_per_s"] = rates
        log(f"atomics: {rates}")
        if "plain_f64" in out:
            ph = out["plain_f64"]["phases"]
            ach = {}
            if "cic" in ph and w.cic is not None:
                n_at = 8 * w.cic.n
                ach["k_cic_direct"] = {"atomics": n_at,
                                       "per_s": n_at / (ph["cic"]["avg_ms"] * 1e-3)}
            if "sn" in ph and w.sn is not None:
                n_at = sn_contributions(w)
                ach["k_sn_direct"] = {"atomics": n_at,
                                      "per_s": n_at / (ph["sn"]["avg_ms"] * 1e-3)}
            # CIC atomics hit 8 cells in pairs along x (nearly scattered);
            # supernova atomics run along x rows of the sphere (coalesced runs)
            for v in ach.values():
                v["frac_of_scattered_f64_peak"] = v["per_s"] / rates["f64"]["scattered"]
                v["frac_of_coalesced_f64_peak"] = v["per_s"] / rates["f64"]["coalesced"]
            out["atomic_roofline"] = {
                "peaks": "f64 adds measured by pmp_atomic_bench: scattered distinct addresses "
                         "and wavefront-coalesced consecutive addresses",
                "scattered_per_s": rates["f64"]["scattered"],
                "coalesced_per_s": rates["f64"]["coalesced"], "kernels": ach}
    if not args.no_c5 and args.workload != "c5":
        out["c5_batched"] = c5_batched(B, args)
        log(f"c5 batched: graph {out['c5_batched']['graph_ms_per_step']:.3f} ms, per-box "
            f"{out['c5_batched']['per_box_launch_ms_per_step']:.3f} ms")
    if not args.no_next:
        out["snr_deposit"] = snr_rate(B)
        log(f"supernova remnants: {out['snr_deposit']}")
        if not (w.sinks is not None and w.sinks.n and w.nbox == 1):
            wc = W.c3()
            out["sink_create"] = {"workload": wc.name,
                                  **sink_create_rate(B, wc, "f32", args.channels)}
            log(f"sink creation: {out['sink_create']}")
    if not args.no_cpu:
        log("cpu baseline (serial oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, nparts)
        log(f"oracle {out['cpu_baseline']['s_per_step']:.2f} s/step")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
