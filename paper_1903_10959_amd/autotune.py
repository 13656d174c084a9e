"""Autotuner for the filter: vector-block width, cell-kernel tile and cells per tile.

The paper picks its filtering block size B^f by experiment (Sec. 3.3: too small
wastes memory bandwidth and latency, too large costs memory and batched-GEMM
efficiency).  Here the same trade-off is measured on the device: for a live
problem, a short filter (a few Chebyshev steps) is timed at each candidate
width and the fastest is cached per (architecture, degree p, block size N_b,
precision).  The cell kernel's work-group tile (four waves with two column
blocks each, or eight waves with one) is chosen the same way, per
(architecture, degree p, precision), and so is the number of cells a
work-group holds (1, 2 or 4, the tile's 64 columns split over them), per
(architecture, degree p, column count, precision): few columns per block
waste fewer MFMA columns with more cells per tile.  Timing is wall time
around the filter call, which returns synchronised.
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "chfsi_autotune.json")


def _key(arch: str, p: int, nblock: int, prec: str) -> str:
    return f"{arch}|p{p}|nb{nblock}|{prec}"


def _tile_key(arch: str, p: int, prec: str) -> str:
    return f"tile|{arch}|p{p}|{prec}"


TILE_VARIANTS = (0, 1)
CELLS_PER_TILE = (1, 2, 4)


def _cpt_key(arch: str, p: int, ncols: int, prec: str) -> str:
    return f"cpt|{arch}|p{p}|nc{ncols}|{prec}"


def candidates(nblock: int):
    c = [w for w in (64, 128, 192, 256, 384, 512) if w < nblock]
    c.append(nblock)
    return sorted(set(c))


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(timings: dict) -> int:
    """Fastest width (ties: the smaller one, which needs less memory)."""
    return min(timings, key=lambda w: (timings[w], w))


def tune_block_width(ctx, X, bounds, prec: str = "fp64", steps: int = 3, arch: str = None,
                     cache_path: str = DEFAULT_CACHE, refresh: bool = False, timer=None):
    """Best filter block width for ctx's problem and X's column count.

    bounds = (a, b, a0) of the filter.  X is filtered in place by each trial,
    so pass a scratch copy.  `timer(width) -> seconds` replaces the device
    measurement (used by the tests)."""
    if arch is None:
        import torch

        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if timer is None else "test"
    nb = int(X.shape[1]) if timer is None else int(X)
    key = _key(arch, int(getattr(ctx, "p", 0)), nb, prec)
    cache = load_cache(cache_path)
    if not refresh and key in cache:
        return int(cache[key]["width"])
    timings = {}
    for w in candidates(nb):
        if timer is not None:
            timings[w] = float(timer(w))
            continue
        a, b, a0 = bounds
        ctx.chebyshev_filter(X, 1, a, b, a0, prec=prec, block_width=w)   # warm the workspaces
        t0 = time.perf_counter()
        ctx.chebyshev_filter(X, steps, a, b, a0, prec=prec, block_width=w)
        timings[w] = time.perf_counter() - t0
    best = pick(timings)
    cache[key] = {"width": best, "timings_s": {str(k): v for k, v in timings.items()}}
    save_cache(cache, cache_path)
    return best


def tune_tile_variant(ctx, X, bounds, prec: str = "fp32", steps: int = 4, arch: str = None,
                      cache_path: str = DEFAULT_CACHE, refresh: bool = False, timer=None, apply: bool = True):
    """Fastest cell-kernel tile variant for ctx's degree and precision; sets it
    on ctx when apply is true.  X (device, DoF-major) is filtered in place by
    each trial, so pass a scratch copy.  `timer(variant) -> seconds` replaces
    the device measurement (used by the tests)."""
    if arch is None:
        import torch

        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if timer is None else "test"
    key = _tile_key(arch, int(getattr(ctx, "p", 0)), prec)
    cache = load_cache(cache_path)
    if not refresh and key in cache:
        best = int(cache[key]["variant"])
    else:
        timings = {}
        for v in TILE_VARIANTS:
            if timer is not None:
                timings[v] = float(timer(v))
                continue
            a, b, a0 = bounds
            ctx.set_tile_variant(v)
            ctx.chebyshev_filter(X, 1, a, b, a0, prec=prec)            # warm-up
            t0 = time.perf_counter()
            ctx.chebyshev_filter(X, steps, a, b, a0, prec=prec)
            timings[v] = time.perf_counter() - t0
        best = pick(timings)
        cache[key] = {"variant": best, "timings_s": {str(k): v for k, v in timings.items()}}
        save_cache(cache, cache_path)
    if apply and timer is None:
        ctx.set_tile_variant(best)
    return best


def tune_cells_per_tile(ctx, X, bounds, prec: str = "fp32", steps: int = 4, arch: str = None,
                        cache_path: str = DEFAULT_CACHE, refresh: bool = False, timer=None, apply: bool = True):
    """Fastest number of cells per work-group for ctx's degree, X's column
    count (filtered as one block) and precision; sets it on ctx when apply is
    true.  X is filtered in place by each trial, so pass a scratch copy.
    `timer(cpt) -> seconds` replaces the device measurement (tests)."""
    if arch is None:
        import torch

        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if timer is None else "test"
    nc = int(X.shape[1]) if timer is None else int(X)
    p = int(getattr(ctx, "p", 0))
    key = _cpt_key(arch, p, nc, prec)
    cache = load_cache(cache_path)
    cands = CELLS_PER_TILE if p <= 6 else (1,)
    if not refresh and key in cache:
        best = int(cache[key]["cpt"])
    else:
        timings = {}
        for cpt in cands:
            if timer is not None:
                timings[cpt] = float(timer(cpt))
                continue
            a, b, a0 = bounds
            ctx.set_cells_per_tile(cpt)
            ctx.chebyshev_filter(X, 1, a, b, a0, prec=prec, block_width=nc)            # warm-up
            t0 = time.perf_counter()
            ctx.chebyshev_filter(X, steps, a, b, a0, prec=prec, block_width=nc)
            timings[cpt] = time.perf_counter() - t0
        best = pick(timings)
        cache[key] = {"cpt": best, "timings_s": {str(k): v for k, v in timings.items()}}
        save_cache(cache, cache_path)
    if apply and timer is None:
        ctx.set_cells_per_tile(best)
    return best
