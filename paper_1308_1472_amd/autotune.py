"""Autotuner of the batched launch.

Measures every combination of the batch tunables -- tile of forests with
m >= 16 (8 or 16), threads per 8 x 8 and 16 x 16 tile, a workgroup per tile
or persistent workgroups -- on a scratch copy of the state, through captured
graphs, and keeps the fastest.  Results are cached per device and batch composition in
`_build/autotune.json` next to the library.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "_build", "autotune.json")

SPACE = {
    "tile_big": (8, 16),
    "threads8": (64, 128),
    "threads16": (256, 512),
    "persistent": (0, 1),
}


def signature(batch) -> str:
    import torch
    # the tunables' names are part of the key: a change of the space voids
    # cached choices
    parts = [torch.cuda.get_device_name(0), str(batch.precision), ",".join(SPACE)]
    for c in batch.contexts:
        parts.append(f"{c.cfg.m}:{c.cfg.physics}:{c.num_patches()}")
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:20]


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, CACHE)


def tune(batch, q, steps=4, reps=3, use_cache=True, log=None):
    """Pick the fastest tunables for `batch` (state `q` is not modified);
    returns (best config, {config: ms per step})."""
    import torch
    sig = signature(batch)
    cache = _load() if use_cache else {}
    if sig in cache:
        best = cache[sig]["best"]
        batch.set_tuning(**best)
        return best, cache[sig]["timings"]
    n = batch.n
    qa = q.clone()
    qb = torch.empty_like(q)
    dt = torch.full((n,), 1e-6, dtype=torch.float64, device="cuda")
    nu = torch.zeros(n, dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    timings = {}
    for vals in itertools.product(*SPACE.values()):
        cfg = dict(zip(SPACE.keys(), vals))
        # the threads of a class that no forest uses do not matter
        batch.set_tuning(**cfg)
        batch.capture(steps, qa, qb, dt, nu, st)
        batch.replay()
        torch.cuda.synchronize()
        best_ms = None
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            batch.replay()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / steps
            best_ms = ms if best_ms is None else min(best_ms, ms)
        key = json.dumps(cfg, sort_keys=True)
        timings[key] = best_ms
        if log:
            log(f"autotune {key}: {best_ms:.3f} ms/step")
    best = json.loads(min(timings, key=timings.get))
    batch.set_tuning(**best)
    cache[sig] = {"best": best, "timings": timings}
    _store(cache)
    return best, timings
