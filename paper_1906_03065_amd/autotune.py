"""Launch-shape autotuner for batched D2Q9 simulations.

For every size class present in a batch (lattice width <= 128, <= 256,
wider) it times candidate shapes of the batched lattice kernel -- lanes per
workgroup, rows per work item, register ring depth -- for about twenty steps
on a throwaway batch of the same workloads, one class at a time with the
other classes fixed, and keeps the fastest.  Results are cached as JSON keyed
by GPU architecture, lattice, storage and size class, so a later batch on the
same hardware reuses them without timing.
"""
from __future__ import annotations

import json
import os
import time

from . import lbib

CANDIDATES = [(bx, seg, ring) for bx in (64, 128, 192, 256) for ring in (3, 4) for seg in (-1, 16, 48)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lbib", "autotune.json")


def size_class(nx: int) -> int:
    return 0 if nx <= 128 else (1 if nx <= 256 else 2)


def arch(device="cuda:0") -> str:
    import torch

    return torch.cuda.get_device_properties(torch.device(device)).gcnArchName


def key(arch_name: str, cls: int, lattice="D2Q9", storage="fp32") -> str:
    return f"{arch_name}|{lattice}|{storage}|class{cls}"


def load(path=DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(cache: dict, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_steps(b: lbib.Batch, steps: int) -> float:
    b.step(2)  # rebuilds the tables and graphs for the new shape
    b.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.synchronize()
    return (time.perf_counter() - t0) / steps


def tune(workloads: list, steps: int = 20, cache_path=DEFAULT_CACHE, device="cuda:0",
         force: bool = False, candidates=CANDIDATES) -> dict:
    """Best shape per size class present in the workloads: {class: {block_x,
    seg, ring, ms_per_step}} (from the cache when it holds the class)."""
    a = arch(device)
    cache = load(cache_path)
    classes = sorted({size_class(w["params"]["nx"]) for w in workloads})
    todo = [c for c in classes if force or key(a, c) not in cache]
    if todo:
        b = lbib.Batch.from_workloads(workloads, device=device)
        for c in classes:  # start from the cached or default shapes
            if key(a, c) in cache:
                v = cache[key(a, c)]
                b.set_launch(c, v["block_x"], v["seg"], v["ring"])
        for c in todo:
            timings = {}
            for bx, seg, ring in candidates:
                b.set_launch(c, bx, seg, ring)
                timings[f"{bx},{seg},{ring}"] = _time_steps(b, steps) * 1e3
            best = min(timings, key=timings.get)
            bx, seg, ring = (int(v) for v in best.split(","))
            b.set_launch(c, bx, seg, ring)
            cache[key(a, c)] = {"block_x": bx, "seg": seg, "ring": ring, "ms_per_step": timings[best],
                                "timed_ms_per_step": timings, "steps": steps}
        b.close()
        save(cache, cache_path)
    return {c: cache[key(a, c)] for c in classes}


def apply(batch: lbib.Batch, tuned: dict):
    """Set the tuned shape of every class on a batch."""
    for c, v in tuned.items():
        batch.set_launch(int(c), v["block_x"], v["seg"], v["ring"])
