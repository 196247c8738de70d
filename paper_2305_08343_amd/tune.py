"""Launch-shape autotuner for the traversal (successive halving, JSON cache).

The traversal's results never depend on its launch shape (threads per block,
LDS stack depth, rays per queue fetch, XCD ray partitions, cap on resident
waves per SIMD, Morton ray sorting, leaf and refill gathering, and for LUT-compressed
masks whether the codebook is copied to LDS or read through the caches), so
the tuner only
measures time: every candidate is timed once, the faster half is kept and
timed again with twice the repetitions, until one remains. Results are
cached per (workload signature, GPU) in a JSON file so later runs reuse
them.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

# (block, stack) pairs with compiled kernels; chunk = rays per fetch / 64; parts = ray partitions
PAIRS = [(256, 8), (128, 8), (256, 12), (256, 4), (128, 16)]
CHUNKS = [1, 2]
PARTS = [8, 1]
WAVES = [0, 6]  # occupancy limit, or at most 6 waves per SIMD
SORT = [0, 1]   # rays in input order, or in the Morton order of their origins
CODEBOOK = [0, 1]  # LUT mode: codebook in LDS when it fits, or read from global memory
GATHER = [0, 12, 20]  # leaf lanes wait for this many of their wave (0 = never)
REFILL = [1, 12, 24]  # idle lanes take new rays once this many are idle (1 = at once)


def candidates(lut: bool = False):
    """Every launch shape (block, stack, chunk, parts, waves, sort, codebook, gather,
    refill); the codebook choice only for LUT-mode scenes (it changes nothing elsewhere)."""
    cbs = CODEBOOK if lut else [0]
    return [(b, s, c, p, w, o, q, g, f) for (b, s) in PAIRS for c in CHUNKS for p in PARTS for w in WAVES
            for o in SORT for q in cbs for g in GATHER for f in REFILL]


def _gpu_name():
    import torch
    return torch.cuda.get_device_name(0)


def successive_halving(ctx, run, cands=None, reps0: int = 1, log=None):
    """run() launches the workload once (asynchronously on the current stream).
    Returns (best config, {config: median ms of its last round})."""
    import torch
    cands = list(cands or candidates())
    reps = reps0
    last = {}
    while True:
        times = {}
        for cfg in cands:
            ctx.set_tune(*cfg)
            run()  # warm-up with this shape
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(reps)]
            for a, b in evs:
                a.record()
                run()
                b.record()
            torch.cuda.synchronize()
            times[cfg] = float(np.median([a.elapsed_time(b) for a, b in evs]))
        last.update(times)
        if log:
            log(f"tune round: {len(cands)} shapes x {reps} reps, best {min(times, key=times.get)} "
                f"{min(times.values()):.3f} ms")
        if len(cands) == 1:
            break
        cands = sorted(cands, key=times.get)[:max(1, len(cands) // 2)]
        reps *= 2
    best = cands[0]
    ctx.set_tune(*best)
    return best, last


def tuned(ctx, key: str, run, cache_path: str | None = None, log=None, cands=None):
    """Look up (or measure and store) the best launch shape for `key` among `cands`
    (default: every candidate)."""
    cache_path = cache_path or os.path.join(os.path.expanduser("~"), ".cache", "subcull_tune.json")
    full_key = f"{key}|{_gpu_name()}"
    cache = {}
    if os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if full_key in cache:
        cfg = tuple(cache[full_key]["config"])
        ctx.set_tune(*cfg)
        return cfg, cache[full_key]
    t0 = time.perf_counter()
    best, times = successive_halving(ctx, run, cands=cands, log=log)
    entry = {"config": list(best), "ms": times[best], "seconds": time.perf_counter() - t0,
             "tried": {",".join(map(str, k)): v for k, v in times.items()}}
    cache[full_key] = entry
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return best, entry
