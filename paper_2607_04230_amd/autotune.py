"""Autotuner for the raster launch shape (tile edge, work-item size, workgroup
size, tiles per segment before the direct path, or the direct algorithm).

Every candidate produces a bit-identical visibility buffer (min is
order-independent), so the tuner only measures: it times the whole
hm_raster_vis call with HIP events on the current stream, keeps the median of
a few repetitions, and caches the winner per (GPU architecture, scenes,
resolution, capacity bucket, r_min) in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
from typing import Iterable, Optional, Tuple

from . import hm

Candidate = Tuple[int, int, int, int, int]   # algo, tile, chunk, block, max_tiles_per_seg

DEFAULT_CANDIDATES: Tuple[Candidate, ...] = tuple(
    [(hm.RASTER_TILED, t, c, b, k)
     for t in (16, 32) for c in (256, 512, 1024, 2048, 1 << 20) for b in (128, 256)
     for k in (4, 8, 16)]
    + [(hm.RASTER_TILED_ROWS, t, 512, 512, 4) for t in (16, 32)]
    + [(hm.RASTER_TILED, 8, 1 << 20, 256, 16), (hm.RASTER_DIRECT, 32, 256, 256, 4)])

QUICK_CANDIDATES: Tuple[Candidate, ...] = (
    (hm.RASTER_TILED, 32, 512, 256, 8), (hm.RASTER_TILED, 32, 512, 256, 4),
    (hm.RASTER_TILED, 32, 1024, 256, 8), (hm.RASTER_TILED, 32, 2048, 256, 8),
    (hm.RASTER_TILED, 32, 512, 256, 16), (hm.RASTER_TILED, 32, 1024, 256, 16),
    (hm.RASTER_TILED, 32, 2048, 256, 16), (hm.RASTER_TILED, 16, 2048, 256, 8),
    (hm.RASTER_TILED_ROWS, 32, 512, 256, 8))


def cache_path() -> str:
    p = os.environ.get("HM_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "hm_autotune.json")


def _key(ds) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cap_bucket = 2 ** int(math.ceil(math.log2(max(ds.cap, 2))))
    return f"{arch}|S{ds.S}|{ds.W}x{ds.H}|cap{cap_bucket}|rmin{ds.sc.r_min:g}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(tab: dict):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(tab, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def params_of(c: Candidate, r_min: float) -> hm.RasterParams:
    algo, tile, chunk, block, k = c
    return hm.RasterParams(r_min, algo, tile, chunk, k, block, 0)


def time_raster(ds, reps: int = 5) -> float:
    """Median ms of hm_raster_vis on the current stream."""
    import torch
    ds.raster()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ds.raster()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune(ds, candidates: Optional[Iterable[Candidate]] = None, reps: int = 5,
         use_cache: bool = True, verbose: bool = False) -> Tuple[hm.RasterParams, dict]:
    """Pick the fastest raster launch shape for DeviceScene `ds` and install it.
    Returns (params, {candidate: ms})."""
    key = _key(ds)
    tab = _load() if use_cache else {}
    if use_cache and key in tab:
        c = tuple(tab[key]["candidate"])
        p = params_of(c, ds.sc.r_min)
        ds.set_raster_params(p)
        return p, {c: tab[key]["ms"]}
    # the raster is timed on the frame's own strand stream
    ds.lod()
    ds.generate()
    results = {}
    for c in (candidates or DEFAULT_CANDIDATES):
        ds.set_raster_params(params_of(c, ds.sc.r_min))
        results[tuple(c)] = time_raster(ds, reps)
        if verbose:
            print(f"[autotune] {c}: {results[tuple(c)]:.4f} ms", flush=True)
    best = min(results, key=results.get)
    p = params_of(best, ds.sc.r_min)
    ds.set_raster_params(p)
    tab = _load()
    tab[key] = {"candidate": list(best), "ms": results[best]}
    _store(tab)
    return p, results
