"""Autotuner for the batched circuit executor.

It times candidate settings of the library's tuning knobs (ciphertexts per
blind-rotation launch, MFMA row tiles per pass) on the caller's own workload
and keeps the fastest.  No knob changes an output bit, so the choice only
affects time.  Results are cached per (GPU, parameter set, workload key) in a
JSON file so a serving process tunes once.
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fhesql_autotune.json")

ROW_PASS = {(32, 256): [4, 2], (32, 512): [8, 4], (32, 1024): [16, 8], (64, 2048): [8, 4]}


def candidates(p, batches=(16384, 32768, 65536, 131072, 262144)):
    """Grid of settings for parameter set p."""
    rps = ROW_PASS.get((p.q, p.N), [0])
    return [{"max_batch": b, "row_pass": rp} for b in batches for rp in rps]


def _gpu_name():
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def tune(ctx, key, run, cands=None, reps=1, cache_path=DEFAULT_CACHE, log=None):
    """Time `run()` (which must synchronize the device) under each candidate
    setting; apply and return the fastest.  Cached results are reused."""
    full_key = f"{_gpu_name()}|{ctx.p.name}|{key}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if full_key in cache:
        best = cache[full_key]["best"]
        ctx.set_tuning(**best)
        return best, cache[full_key]["times"]
    cands = cands or candidates(ctx.p)
    times = []
    for cand in cands:
        ctx.set_tuning(**cand)
        run()  # warm (workspace growth, code load)
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        dt = (time.perf_counter() - t0) / reps
        times.append({"setting": cand, "seconds": dt})
        if log:
            log(f"autotune {key}: {cand} -> {dt:.4f} s")
    best = min(times, key=lambda t: t["seconds"])["setting"]
    ctx.set_tuning(**best)
    if cache_path:
        cache[full_key] = {"best": best, "times": times}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, times
