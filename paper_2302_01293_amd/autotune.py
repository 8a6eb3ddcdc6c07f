"""Autotuner of the search's schedule.

Three run-time choices of the plan change only speed, never results:
  * ``tile_cells``: points x frequencies per work item.  The persistent search
    kernel pulls items in cost order; small items balance the tail of a launch,
    large ones amortise each item's set-up (grid descriptors, point loads per
    frequency group);
  * ``item_freqs``: the most frequencies per item (short stars spread over more
    items, and the groups of an XCD share fewer stars' points in its L2);
  * ``big_points``: stars with more points take the large workgroup shape (72 KB
    accumulator window, two groups per CU) for every frequency instead of the common
    one (48 KB, three per CU): fewer point re-reads per frequency against less
    latency hiding.
The best values depend on the device and on the batch shape, so they are measured:
coordinate descent over the three axes, each candidate timed on the batch or a
stratified sample of its stars (device time of ``bls_search_batch``, median of a few
launches), the winners cached per device and batch shape in a JSON file.  Each axis
also times the current pick (the library default at first), so the result is never
slower than the default on what was timed; a small sample can still mislead (a few
dozen stars do not fill 256 CUs the way a full batch does), so callers that care
time the batch itself.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

CANDIDATES = (1 << 20, 3 << 19, 3 << 20, 6 << 20, 12 << 20, 24 << 20)
ITEM_FREQS = (64, 128, 256, 1024)
BIG_POINTS = (50_000, 100_000, 200_000, 1 << 40)


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


def _time_search(sub, params, reps: int, warmup: bool = True) -> float:
    import torch
    from .device import DeviceSearch
    ds = DeviceSearch.from_batch(sub, params, want_snr=False, want_best=False)
    ds.run_prepare()
    if warmup:
        ds.run_search()
    stream = torch.cuda.current_stream()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ds.run_search()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del ds
    return float(np.median(ms))


def tune(batch, params=None, candidates=CANDIDATES, n_sample: int = 256, reps: int = 3,
         cache_path: str | None = None, use_cache: bool = True, axes=("tile_cells",),
         item_freqs=ITEM_FREQS, big_points=BIG_POINTS, log=None, include_current: bool = True,
         warmup: bool = True) -> dict:
    """Pick the schedule for a batch by coordinate descent over ``axes`` (any of
    "tile_cells", "item_freqs", "big_points", tuned in that order, each with the
    others at their current picks; with ``include_current`` the current pick is one
    of each axis's candidates, a schedule is timed once); returns {"tile_cells",
    "item_freqs", "big_points", "times_ms", "key", "cached", and when timed here
    "default_ms" and "best_ms"} (0 = library default)."""
    import torch
    from . import _lib

    points = np.diff(np.asarray(batch.offsets))
    key = shape_key(torch.cuda.get_device_name(), points) + "|" + ",".join(axes)
    path = cache_path or default_cache_path()
    cache = load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        c = cache[key]
        return dict(tile_cells=int(c["tile_cells"]), item_freqs=int(c.get("item_freqs", 0)),
                    big_points=int(c.get("big_points", 0)), times_ms=c.get("times_ms", {}), key=key,
                    cached=True)
    sub = batch.subset(sample_stars(points, n_sample))
    base = params if params is not None else _lib.default_params()
    pick = dict(tile_cells=int(base.tile_cells), item_freqs=int(base.item_freqs), big_points=int(base.big_points))
    grid = dict(tile_cells=candidates, item_freqs=item_freqs, big_points=big_points)
    times = {}
    seen = {}
    for ax in ("tile_cells", "item_freqs", "big_points"):
        if ax not in axes:
            continue
        cands = [int(c) for c in grid[ax]]
        if include_current and pick[ax] not in cands:
            cands = [pick[ax]] + cands
        res = {}
        for c in cands:
            sched = dict(pick, **{ax: c})
            tag = (sched["tile_cells"], sched["item_freqs"], sched["big_points"])
            if tag not in seen:
                p = _lib.default_params(**{f: getattr(base, f) for f, _ in _lib.BlsParams._fields_})
                for k, v in sched.items():
                    setattr(p, k, int(v))
                seen[tag] = _time_search(sub, p, reps, warmup)
            res[str(c)] = seen[tag]
            if log:
                log("autotune %s = %d: %.2f ms" % (ax, c, res[str(c)]))
        pick[ax] = int(min(res, key=lambda k: res[k]))
        times[ax] = res
    base_tag = (int(base.tile_cells), int(base.item_freqs), int(base.big_points))
    best_tag = (pick["tile_cells"], pick["item_freqs"], pick["big_points"])
    out = dict(pick, times_ms=times, key=key, cached=False, default_ms=seen.get(base_tag),
               best_ms=seen.get(best_tag))
    if use_cache:
        cache[key] = dict(pick, times_ms=times)
        save_cache(path, cache)
    return out
