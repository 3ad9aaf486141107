"""Tile autotuner of the batched path.

Two parameters of the contraction are tuned: the tiling target (workgroups
per instance the node chunks are split for: fewer, longer chunks mean fewer
partial sums to reduce, more chunks fill the chip) and, for FP64, the tile
edge (64 x 64 tiles with four 16 x 16 MFMA blocks per wave, or 32 x 32 tiles:
4x more, smaller workgroups over the same chunks).  For a given batch every
candidate pair is timed on the device with HIP events around the contraction
launch and the fastest is kept in a JSON cache keyed by the batch's shape
and precision.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import tl

CANDIDATES = (128, 256, 512, 1024, 2048, 4096)
TILE_EDGES = (64, 32)   # FP64 only; the split kernels have one tile shape
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "tl_tuning.json")


def batch_key(systems, precision: str, n_slices: int) -> str:
    shape = [(int(s.L[0]), int(s.m0), int(s.n[0]), int(s.n[1]), int(s.n[2]), int(s.R))
             for s in systems]
    h = hashlib.sha1(json.dumps([shape, precision, n_slices]).encode()).hexdigest()[:16]
    return f"batch-{len(systems)}-{h}"


def _time_contraction(bp, reps: int) -> float:
    import torch
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        b.record(stream)
    bp.run()
    torch.cuda.synchronize()
    for a, b in evs:
        tl.tl_set_contraction_events(a.cuda_event, b.cuda_event)
        bp.run()
    torch.cuda.synchronize()
    tl.tl_set_contraction_events(None, None)
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def tune_batch(systems, precision: str = "fp64", n_slices: int = 0, candidates=CANDIDATES,
               reps: int = 3, cache_path: str | None = DEFAULT_CACHE, tile_edges=TILE_EDGES):
    """Return ((best want_blocks, best tile edge), {"edge x want": contraction ms})."""
    from .pipeline import BatchPipeline
    key = batch_key(systems, precision, n_slices)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache and "tile_edge" in cache[key]:
        c = cache[key]
        return (int(c["want_blocks"]), int(c["tile_edge"])), dict(c["ms"])
    edges = tile_edges if precision == "fp64" else (64,)
    times = {}
    for e in edges:
        for c in candidates:
            bp = BatchPipeline(systems, precision=precision, n_slices=n_slices, want_blocks=c,
                               tile_edge=e)
            times[f"{e}x{int(c)}"] = _time_contraction(bp, reps)
            del bp
    best = min(times, key=times.get)
    be, bw = (int(v) for v in best.split("x"))
    if cache_path:
        cache[key] = {"want_blocks": bw, "tile_edge": be, "ms": times}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return (bw, be), times
