"""Autotuner binding: argument marshalling for the library's hfx_autotune.

The tuner itself is native (``csrc/autotune.cpp``): for each system it times
the compiled kernel configurations of the system's grid crossed with batch
sizes and rows per tile pair on the caller's orbitals, keeps the fastest
(ties within 5 % go to the earliest candidate, the plan defaults first), and
records the choice in a text cache keyed by device architecture, grid,
orbital count, precision, kz band and the identity of the kernel sources.
Plans created with ``tune_cache=<path>`` pick the cached choices up.
"""
from __future__ import annotations

import ctypes

import torch

from . import hfx


def tune(specs, precision, psi, cache_path=None, reps=2, options=None):
    """Per-system plan options chosen by the tuner, e.g.
    ``"variant=f32-n96;tiles=0;rows=32"`` (lists for several systems).

    ``psi``: the systems' float64 orbitals concatenated on the GPU; ``options``:
    options every trial plan gets (e.g. ``"ecut=20"``); ``cache_path``: the
    text cache to read and extend."""
    lib = hfx.load_library()
    if isinstance(specs, hfx.SystemSpec):
        specs = [specs]
    specs = list(specs)
    if psi.dtype != torch.float64 or not psi.is_cuda or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous float64 CUDA tensor")
    if psi.numel() != sum(s.n_orb * s.nr for s in specs):
        raise ValueError("psi does not hold the systems' orbitals")
    arr = (hfx.System * len(specs))(*[s.to_c() for s in specs])
    out = ctypes.create_string_buffer(64 * len(specs) + 64)
    with torch.cuda.device(psi.device):
        hfx._check(lib.hfx_autotune(arr, len(specs), int(precision),
                                    options.encode() if options else None,
                                    ctypes.c_void_p(psi.data_ptr()), int(reps),
                                    cache_path.encode() if cache_path else None, out,
                                    len(out), hfx._stream()))
    return out.value.decode()


def cached_lines(cache_path):
    """The cache's choices as (key, options, ms) tuples."""
    return [r for r in _records(cache_path) if "#" not in r[0]]


def candidate_table(cache_path, key):
    """{options: ms} of every candidate timed for key."""
    return {o: ms for k, o, ms in _records(cache_path) if k == key + "#candidate"}


def _records(cache_path):
    out = []
    with open(cache_path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 3:
                out.append((parts[0], parts[1], float(parts[2])))
    return out
