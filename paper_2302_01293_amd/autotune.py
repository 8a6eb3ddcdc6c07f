"""Autotuner for the search's work-item size.

The plan cuts every star's frequency grid into work items of about ``tile_cells``
points x frequencies; the persistent search kernel pulls them in cost order.  Small
items balance the tail of a launch, large ones amortise each item's set-up (grid
descriptors, point loads per frequency group).  The best size depends on the
device and on the batch shape, so it is measured: each candidate is timed on a
sample of the batch's stars (device time of ``bls_search_batch``, median of a few
launches) and the winner is cached per device and batch shape in a JSON file.
The tile size never changes results, only speed.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

CANDIDATES = (1 << 20, 3 << 19, 3 << 20, 6 << 20, 12 << 20, 24 << 20)


def default_cache_path() -> str:
    return os.environ.get("MI355BLS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mi355bls", "tune.json"))


def shape_key(device_name: str, points: np.ndarray) -> str:
    """Device plus the batch's size class: log2 buckets of the median and largest
    point count per star."""
    med = int(np.median(points)) if len(points) else 0
    mx = int(points.max()) if len(points) else 0
    return "%s|med2^%d|max2^%d" % (device_name, int(math.log2(max(med, 1))), int(math.log2(max(mx, 1))))


def load_cache(path: str) -> dict:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def sample_stars(points: np.ndarray, n: int, seed: int = 0) -> np.ndarray:
    """Up to n stars spread over the batch's cost range (stratified by points)."""
    S = len(points)
    if S <= n:
        return np.arange(S)
    order = np.argsort(points, kind="stable")
    picks = order[np.linspace(0, S - 1, n).round().astype(np.int64)]
    return np.unique(picks)


def tune(batch, params=None, candidates=CANDIDATES, n_sample: int = 256, reps: int = 3,
         cache_path: str | None = None, use_cache: bool = True) -> dict:
    """Pick ``tile_cells`` for a batch; returns {"tile_cells", "times_ms", "key", "cached"}."""
    import torch
    from . import _lib
    from .device import DeviceSearch

    points = np.diff(np.asarray(batch.offsets))
    key = shape_key(torch.cuda.get_device_name(), points)
    path = cache_path or default_cache_path()
    cache = load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        return dict(tile_cells=int(cache[key]["tile_cells"]), times_ms=cache[key].get("times_ms", {}),
                    key=key, cached=True)
    sub = batch.subset(sample_stars(points, n_sample))
    times = {}
    for c in candidates:
        p = params if params is not None else _lib.default_params()
        p = _lib.default_params(**{f: getattr(p, f) for f, _ in _lib.BlsParams._fields_})
        p.tile_cells = int(c)
        ds = DeviceSearch.from_batch(sub, p, want_snr=False, want_best=False)
        ds.run_prepare()
        ds.run_search()  # warm-up
        stream = torch.cuda.current_stream()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ds.run_search()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        times[str(c)] = float(np.median(ms))
        del ds
    best = int(min(times, key=lambda k: times[k]))
    if use_cache:
        cache[key] = dict(tile_cells=best, times_ms=times)
        save_cache(path, cache)
    return dict(tile_cells=best, times_ms=times, key=key, cached=False)
