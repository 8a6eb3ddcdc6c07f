"""Streamed search over many batches with the host-to-device copy of the next batch
overlapping the search of the current one (double buffering).

For every batch: the host builds the plan (C++), the light curve is copied from
pinned host memory on a copy stream, and prepare -> search -> S/N run on the
compute stream once the copy's event has fired; the 88-byte results come back on
the copy stream.  Two batches are in flight at a time, so at steady state the
copy of batch b + 1 hides under the search of batch b.  Wall-clock stars/hour
covers plan, copies, search, S/N and the results' return.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib
from .device import DeviceSearch


class _Slot:
    def __init__(self):
        self.ds = None
        self.done = None
        self.result_host = None
        self.index = -1


def _pinned(a: np.ndarray) -> torch.Tensor:
    t = torch.empty(a.shape, dtype=torch.float64, pin_memory=True)
    t.numpy()[...] = a
    return t


def run_stream(batches, params=None, log=None, autotune_first: bool = False):
    """Search an iterable of ``synth.Batch``; returns (list of result arrays, stats).
    ``autotune_first``: tune the schedule (``autotune.tune``, all three axes) on the
    first batch and use it for every batch; the picks are in stats["schedule"]."""
    dev = torch.device("cuda")
    copy_stream = torch.cuda.Stream()
    compute = torch.cuda.current_stream()
    slots = [_Slot(), _Slot()]
    results = {}
    n_stars = 0
    cells = 0.0
    t0 = time.perf_counter()
    pending = []
    schedule = None
    for bi, b in enumerate(batches):
        if bi == 0 and autotune_first:
            from . import autotune
            base = params if params is not None else _lib.default_params()
            schedule = autotune.tune(b, base, n_sample=b.n_stars, reps=1, use_cache=False,
                                     axes=("tile_cells", "item_freqs", "big_points"),
                                     candidates=(3 << 20, 12 << 20), item_freqs=(64, 256),
                                     big_points=(50_000, 200_000), warmup=False)
            params = _lib.default_params(**{f: getattr(base, f) for f, _ in _lib.BlsParams._fields_})
            for k in ("tile_cells", "item_freqs", "big_points"):
                setattr(params, k, int(schedule[k]))
            t0 = time.perf_counter()       # the clock starts after tuning
        slot = slots[bi % 2]
        if slot.done is not None:          # the slot's previous batch must be finished
            slot.done.synchronize()
            results[slot.index] = slot.result_host.numpy().view(_lib.RESULT_DTYPE).copy()
            slot.done = None
        ht, hy, hw = _pinned(b.t), _pinned(b.y), _pinned(b.w)
        with torch.cuda.stream(copy_stream):
            dt_ = ht.to(dev, non_blocking=True)
            dy_ = hy.to(dev, non_blocking=True)
            dw_ = hw.to(dev, non_blocking=True)
            copied = torch.cuda.Event()
            copied.record(copy_stream)
        ds = DeviceSearch(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax, params, want_snr=False,
                          inputs=(dt_, dy_, dw_))
        compute.wait_event(copied)
        for tsr in (dt_, dy_, dw_):
            tsr.record_stream(compute)
        ds.run(compute)
        finished = torch.cuda.Event()
        finished.record(compute)
        copy_stream.wait_event(finished)
        res_host = torch.empty(ds.result.shape, dtype=torch.uint8, pin_memory=True)
        with torch.cuda.stream(copy_stream):
            res_host.copy_(ds.result, non_blocking=True)
            done = torch.cuda.Event()
            done.record(copy_stream)
        slot.ds, slot.done, slot.result_host, slot.index = ds, done, res_host, bi
        n_stars += b.n_stars
        cells += float(np.sum(np.diff(ds.plan.freq_offsets).astype(np.float64) * np.diff(b.offsets)))
        pending.append((ht, hy, hw))
        if len(pending) > 2:
            pending.pop(0)
        if log:
            log("batch %d queued: %d stars" % (bi, b.n_stars))
    for slot in slots:
        if slot.done is not None:
            slot.done.synchronize()
            results[slot.index] = slot.result_host.numpy().view(_lib.RESULT_DTYPE).copy()
    wall = time.perf_counter() - t0
    return [results[i] for i in sorted(results)], dict(stars=n_stars, cells=cells, wall_s=wall,
                                                       stars_per_hour=n_stars / wall * 3600.0,
                                                       cells_per_s=cells / wall, schedule=schedule)
