"""Autotuner for the persistent mixed-batch launch.

Candidate shapes (persistent workgroups per compute unit, one-vertex instances
per work item, queue order) are timed with device events on the live workload;
the fastest is cached in a JSON file keyed by the device name and a workload
signature, so later runs reuse it without timing.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import spoly

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "spoly_autotune.json")
CANDIDATES = {"workgroups_per_cu": (1, 2, 4, 8), "r_tile": (64, 256, 1024), "order": (0, 1, 2)}


def signature(n1: int, n2: int, event: str, precision: int) -> str:
    """Workload key: sizes rounded to powers of two, event and precision."""
    b = lambda n: max(0, int(n).bit_length() - 1)  # noqa: E731
    return f"mixed:n1=2^{b(n1)}:n2=2^{b(n2)}:{event}:p{precision}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(run, key: str, cache_path: str = DEFAULT_CACHE, reps: int = 2, candidates: dict | None = None,
         force: bool = False):
    """run(shape) enqueues one solve with the given spoly.MixedShape.
    Returns (best shape, timings in ms per shape, whether it came from the cache)."""
    dev = torch.cuda.get_device_name(0)
    full = f"{dev}|{key}"
    cache = _load(cache_path)
    if not force and full in cache:
        c = cache[full]
        return spoly.MixedShape(c["workgroups_per_cu"], c["r_tile"], c["order"], 0), c.get("timings", {}), True
    cand = candidates or CANDIDATES
    timings = {}
    best, best_ms = None, float("inf")
    for wg, rt, order in itertools.product(cand["workgroups_per_cu"], cand["r_tile"], cand["order"]):
        shape = spoly.MixedShape(wg, rt, order, 0)
        run(shape)  # warm-up
        ms = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            run(shape)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        t = min(ms)
        timings[f"{wg}/{rt}/{order}"] = t
        if t < best_ms:
            best, best_ms = shape, t
    cache[full] = {"workgroups_per_cu": best.workgroups_per_cu, "r_tile": best.r_tile, "order": best.order,
                   "ms": best_ms, "timings": timings}
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    with open(cache_path, "w") as f:
        json.dump(cache, f, indent=1)
    return best, timings, False
