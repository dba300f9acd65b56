"""Autotuning driver: runs the library's own tuner (pmp_autotune) once per
workload shape and GPU architecture and caches the winning tuning in a JSON
file, so later runs start from it."""
from __future__ import annotations

import hashlib
import json
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pmp_autotune.json")


def shape_key(ctx) -> str:
    """What the best tuning depends on: mesh shape, particle counts and radii,
    accumulator and state types, and the GPU architecture."""
    import numpy as np
    import torch
    w = ctx.w
    arch = torch.cuda.get_device_properties(ctx.state.device).gcnArchName
    desc = {
        "arch": arch, "acc": ctx.acc, "state": str(np.dtype(w.state.dtype)),
        "domain": list(w.domain), "nbox": w.nbox, "ghost": w.ghost, "fields": list(ctx.fields),
        "box_cells": int(w.owned_cells),
        "cic": w.cic.n if w.cic else 0, "sn": w.sn.n if w.sn else 0,
        "sink": w.sinks.n if w.sinks else 0,
        "sn_r": float(np.max(w.sn.fields["r"])) if w.sn is not None and w.sn.n else 0.0,
        # a cached tuning is only reused for the tuning struct it was made with
        "tuning_fields": [k for k, _ in type(ctx.tuning())._fields_],
    }
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:20]


def tune(ctx, cache_path: str | None = DEFAULT_CACHE, force: bool = False) -> dict:
    """Apply the cached tuning for this shape, or run the tuner and cache it.
    Returns {"tuning": ..., "best_ms": ..., "cached": bool}."""
    key = shape_key(ctx)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        ctx.set_tuning(**cache[key]["tuning"])
        return {**cache[key], "cached": True}
    best = ctx.autotune()
    rec = {"tuning": ctx.tuning().as_dict(), "best_ms": best}
    if cache_path:
        cache[key] = rec
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        tmp = cache_path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return {**rec, "cached": False}
