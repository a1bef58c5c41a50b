"""Autotuner for libhfx plans.

Times every compiled kernel configuration for a system's grid size
(``hfx.variants``) crossed with a few orbital-tile batch sizes and rows per
tile pair (those that fit the orbital count), on the caller's orbitals, with HIP events around ``apply_exchange``; the fastest
candidate wins, and among candidates within ``tie`` of the fastest the first
in a fixed candidate order is taken, so re-runs agree.  Results are cached in
a JSON file keyed by GPU architecture, grid, orbital count, precision and a
hash of the library binary.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import hfx

TILE_CHOICES = (4, 8, 16)
ROW_CHOICES = (8, 16, 32)


def _build_id():
    h = hashlib.sha1()
    with open(hfx.LIB_PATH, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def cache_key(spec, precision):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return (f"{arch}|n={spec.n}|n_orb={spec.n_orb}|kernel={spec.kernel}|"
            f"prec={precision}|build={_build_id()}")


def candidates(spec, precision):
    # rows beyond the orbital count (rounded up to a column tile) repeat the
    # schedule of the largest row count that fits
    rows = [r for r in ROW_CHOICES if r == ROW_CHOICES[0] or r <= -(-spec.n_orb // 8) * 8]
    out = []
    for v in hfx.variants(spec.n, precision):
        for t in TILE_CHOICES:
            for r in rows:
                out.append(f"variant={v};tiles={t};rows={r}")
    return out


def time_candidate(spec, precision, psi, options, reps=2):
    plan = hfx.Plan(spec, precision, options=options, device=psi.device)
    kpsi = torch.empty(psi.shape, dtype=plan.kpsi_dtype, device=psi.device)
    ex = torch.empty(1, dtype=torch.float64, device=psi.device)
    plan.apply_exchange(psi, kpsi=kpsi, ex=ex)      # warm-up
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        plan.apply_exchange(psi, kpsi=kpsi, ex=ex)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    plan.close()
    return ms


def tune(spec, precision, psi, cache_path=None, reps=2, tie=0.02, log=None):
    """Return the best options string for this system (and store it in the cache)."""
    key = cache_key(spec, precision)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["options"]
    timings = {}
    for opt in candidates(spec, precision):
        timings[opt] = time_candidate(spec, precision, psi, opt, reps)
        if log:
            log(f"{opt}: {timings[opt]:.2f} ms")
    best_ms = min(timings.values())
    best = next(o for o in timings if timings[o] <= best_ms * (1 + tie))
    if cache_path:
        cache[key] = {"options": best, "ms": timings[best], "timings": timings}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best


def cached_options(spec, precision, cache_path):
    """Options stored for this system, or None."""
    if not cache_path or not os.path.exists(cache_path):
        return None
    with open(cache_path) as f:
        cache = json.load(f)
    rec = cache.get(cache_key(spec, precision))
    return rec["options"] if rec else None
