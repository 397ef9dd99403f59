"""Autotuner for the batched circuit executor.

It times candidate settings of the library's tuning knobs on the caller's
own workload and keeps the fastest: ciphertexts per blind-rotation launch
(how a level's gates are cut into launches), MFMA row tiles per pass (the
Toeplitz tile height a workgroup covers per pass) and, for rings of 512
coefficients or more, the batch size below which a blind rotation spreads
each 16-ciphertext group over many workgroups.  No knob changes an output
bit, so the choice only affects time.  The tile width -- ciphertexts per
tile -- is the MFMA operand's 16 columns and is not a knob (32 ciphertexts
per workgroup, two tiles sharing each key fragment, measured no faster at
the toy size).  Results are cached per (GPU, parameter values, workload key)
in a JSON file so a serving process tunes once.
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
    splits = [-1, 0] if p.N >= 512 else [-1]
    return [{"max_batch": b, "row_pass": rp, "split_groups": sg} for b in batches for rp in rps for sg in splits]


def _gpu_name():
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def cache_key(p, key):
    """Cache entry name: the GPU, the parameter values and the workload key."""
    return f"{_gpu_name()}|q{p.q} n{p.n} N{p.N} l{p.l} bg{p.bg_bits} ks{p.ks_bits}x{p.ks_t}|{key}"


def tune(ctx, key, run, cands=None, reps=1, cache_path=DEFAULT_CACHE, log=None):
    """Time `run()` (which must synchronize the device) under each candidate
    setting; apply and return (best setting, timings).  A cached result for
    the same GPU, parameters and key is applied without running anything."""
    full_key = cache_key(ctx.p, key)
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
        d = os.path.dirname(cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, times
