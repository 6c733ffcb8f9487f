"""Autotuner for the launch knobs of the counting kernels.

Every knob (threads per workgroup, points per thread, LDS pre-aggregation
slots, table load factor, counting path) changes speed only, never the
result.  The tuner times a caller-supplied workload under a sweep of knob
values, one knob at a time starting from the defaults (coordinate descent),
keeps the fastest setting of each knob, and caches the winner in a JSON file
keyed by GPU architecture and a size bucket of the workload.

    from paper_1907_03620_amd import autotune
    best = autotune.tune("batch", lambda: raster.cluster_batch(jobs), points=total_points)
    raster.set_tuning(best)
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict

from . import Tuning, get_tuning, set_tuning

SWEEPS = {
    "mode": [0, 1],
    "block": [128, 256, 512],
    "items": [2, 4, 8],
    "preagg_slots": [0, 1024, 4096],
    "load_factor": [0.4, 0.6, 0.8],
}
STREAM_SWEEPS = {"mode": [0, 1], "load_factor": [0.5, 0.6, 0.75]}


def cache_path() -> str:
    return os.environ.get("RASTER_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "raster_mi355x", "autotune.json"))


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def bucket(points: int) -> str:
    """Size bucket: powers of 4 of the point count."""
    return f"4^{int(math.log(max(points, 1), 4))}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(data: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached(kind: str, points: int) -> Tuning | None:
    entry = _load().get(_arch(), {}).get(kind, {}).get(bucket(points))
    return Tuning(**entry["tuning"]) if entry else None


def _time(run, reps: int) -> float:
    import torch
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        del out
    return best


def tune(kind: str, run, points: int, reps: int = 3, use_cache: bool = True, sweeps: dict | None = None,
         log=None) -> Tuning:
    """Coordinate-descent search; returns the fastest Tuning and caches it.
    ``run`` executes the workload once under the current tuning."""
    if use_cache:
        hit = cached(kind, points)
        if hit is not None:
            return hit
    sweeps = sweeps or (STREAM_SWEEPS if kind == "stream" else SWEEPS)
    saved = get_tuning()
    best = Tuning()
    trials = []
    try:
        set_tuning(best)
        run()  # warm-up: buffers, graph capture
        best_t = _time(run, reps)
        trials.append((asdict(best), best_t))
        for knob, values in sweeps.items():
            for v in values:
                if getattr(best, knob) == v:
                    continue
                cand = Tuning(**{**asdict(best), knob: v})
                set_tuning(cand)
                run()
                t = _time(run, reps)
                trials.append((asdict(cand), t))
                if log:
                    log(f"autotune {kind}: {knob}={v} {t * 1e3:.2f} ms (best {best_t * 1e3:.2f})")
                if t < best_t:
                    best, best_t = cand, t
    finally:
        set_tuning(saved)
    data = _load()
    data.setdefault(_arch(), {}).setdefault(kind, {})[bucket(points)] = {
        "tuning": asdict(best), "seconds": best_t, "trials": len(trials)}
    _store(data)
    return best
