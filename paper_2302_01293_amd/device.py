"""Device-side driver: PyTorch tensors for HBM buffers and streams, the C ABI for work.

``DeviceSearch`` owns the device copies of one packed batch, the plan's workspace
and the output buffers, and enqueues ``bls_search_batch`` + ``bls_snr`` on the
current PyTorch stream.  Nothing here computes any part of the search.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import BEST_DTYPE, RESULT_DTYPE, Plan


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class DeviceSearch:
    """Plain BLS + S/N over a packed batch resident in HBM."""

    def __init__(self, t, y, w, offsets, rho=None, pmin=None, pmax=None, params=None,
                 device: str = "cuda", want_snr: bool = True, want_best: bool = True, inputs=None):
        """``inputs`` (optional): device tensors (t, y, w) already holding the same
        packed arrays, shared instead of copied (e.g. by a second plan of the same
        batch)."""
        if not torch.cuda.is_available():
            raise RuntimeError("DeviceSearch needs a GPU (HIP device)")
        self.plan = Plan(t, y, w, offsets, rho, pmin, pmax, params)
        dev = torch.device(device)
        self.device = dev
        if inputs is not None:
            self.t, self.y, self.w = inputs
        else:
            self.t = torch.as_tensor(np.ascontiguousarray(t, np.float64)).to(dev)
            self.y = torch.as_tensor(np.ascontiguousarray(y, np.float64)).to(dev)
            self.w = None if w is None else torch.as_tensor(np.ascontiguousarray(w, np.float64)).to(dev)
        nws = (self.plan.workspace_bytes + 255) // 256 * 256
        self.ws = torch.empty(nws + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        nf = self.plan.n_freq
        self.sr = torch.empty(nf, dtype=torch.float64, device=dev)
        self.best = torch.empty(nf * BEST_DTYPE.itemsize, dtype=torch.uint8, device=dev) if want_best else None
        self.snr = torch.empty(nf, dtype=torch.float64, device=dev) if want_snr else None
        self.result = torch.empty(self.plan.n_stars * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        self.stats = None
        self.fit = None
        self.plan.upload(self.ws_ptr, self.plan.workspace_bytes, _stream_handle())

    @classmethod
    def from_batch(cls, batch, params=None, **kw):
        return cls(batch.t, batch.y, batch.w, batch.offsets, batch.rho, batch.pmin, batch.pmax, params, **kw)

    def run_prepare(self, stream=None):
        self.plan.prepare(self.ws_ptr, self.t.data_ptr(), self.y.data_ptr(),
                          None if self.w is None else self.w.data_ptr(), stream=_stream_handle(stream))

    def run_search(self, stream=None, windows=None):
        """Full grid, or only the (star, i0, i1) frequency ranges of an int64 [n, 3]
        device tensor (ranges are clipped to the star's grid; empty ones are skipped;
        outputs outside the ranges are left untouched).  An empty work list does nothing
        (the C call treats a NULL list as the full grid, and an empty tensor has no
        storage)."""
        if windows is not None and int(windows.shape[0]) == 0:
            return
        h = _stream_handle(stream)
        self.plan.search(self.ws_ptr, self.sr.data_ptr(), None if self.best is None else self.best.data_ptr(),
                         None if windows is None else windows.data_ptr(),
                         0 if windows is None else int(windows.shape[0]), stream=h)

    def run_snr(self, stream=None):
        h = _stream_handle(stream)
        self.plan.snr(self.ws_ptr, self.sr.data_ptr(), None if self.best is None else self.best.data_ptr(),
                      None if self.snr is None else self.snr.data_ptr(), self.result.data_ptr(), stream=h)

    def run_stats(self, snr_min: float = 9.0, stream=None):
        """Per-star statistics and detection criteria at each star's detection
        (``bls_stats``; needs the best windows, i.e. ``want_best``)."""
        if self.best is None:
            raise RuntimeError("bls_stats needs the per-frequency best windows (want_best=True)")
        if self.stats is None:
            self.stats = torch.empty(self.plan.n_stars * _lib.STATS_DTYPE.itemsize, dtype=torch.uint8,
                                     device=self.device)
        self.plan.stats(self.ws_ptr, self.t.data_ptr(), self.y.data_ptr(),
                        None if self.w is None else self.w.data_ptr(), self.best.data_ptr(),
                        self.result.data_ptr(), self.stats.data_ptr(), snr_min, stream=_stream_handle(stream))

    def run_fit(self, snr_min: float = 9.0, pink_min: float = 9.0, stream=None):
        """Trapezoid fit, noise, S/N_pink and the detection criteria at each star's
        detection (``bls_fit``; starts from the results of ``run_snr`` with best windows)."""
        if self.fit is None:
            self.fit = torch.empty(self.plan.n_stars * _lib.FIT_DTYPE.itemsize, dtype=torch.uint8,
                                   device=self.device)
        self.plan.fit(self.ws_ptr, self.t.data_ptr(), self.y.data_ptr(),
                      None if self.w is None else self.w.data_ptr(), self.result.data_ptr(), self.fit.data_ptr(),
                      snr_min, pink_min, stream=_stream_handle(stream))

    def fit_host(self) -> np.ndarray:
        return self.fit.cpu().numpy().view(_lib.FIT_DTYPE)

    def stats_host(self) -> np.ndarray:
        return self.stats.cpu().numpy().view(_lib.STATS_DTYPE)

    def run(self, stream=None, windows=None):
        self.run_prepare(stream)
        self.run_search(stream, windows)
        self.run_snr(stream)

    def capture(self, windows=None):
        """Record prepare -> search -> S/N into a HIP graph (``torch.cuda.CUDAGraph``).

        The library allocates nothing and records no memset (the work counters are
        cleared by a kernel), so the sequence is capturable; ``graph.replay()``
        recomputes every output from the current contents of the input tensors.
        """
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            self.run(windows=windows)
        torch.cuda.current_stream().wait_stream(side)
        return g

    def capture_pipeline(self):
        """One HIP graph for the whole device path of this plan: the copies of t, y, w
        from pinned host buffers, prepare -> search -> S/N, and the copy of the
        per-star results back to a pinned host buffer.  Fill ``pipe.y_host`` (and, with
        the same first and last weighted times per star, ``w_host``) with new values,
        call ``pipe.replay()`` and read ``pipe.results()``: a serving loop over new
        fluxes of the same stars without per-call launches or allocations."""
        return _Pipeline(self)

    # ---- host copies ----
    def sr_host(self) -> np.ndarray:
        return self.sr.cpu().numpy()

    def best_host(self) -> np.ndarray:
        return self.best.cpu().numpy().view(BEST_DTYPE)

    def snr_host(self) -> np.ndarray:
        return self.snr.cpu().numpy()

    def results_host(self) -> np.ndarray:
        return self.result.cpu().numpy().view(RESULT_DTYPE)

    def star_slice(self, s: int) -> slice:
        fo = self.plan.freq_offsets
        return slice(int(fo[s]), int(fo[s + 1]))


class _Pipeline:
    """Pinned host staging buffers and the captured graph of ``capture_pipeline``."""

    def __init__(self, ds: DeviceSearch):
        self.ds = ds
        self.t_host = ds.t.cpu().pin_memory()
        self.y_host = ds.y.cpu().pin_memory()
        self.w_host = None if ds.w is None else ds.w.cpu().pin_memory()
        self.result_host = torch.empty(ds.result.numel(), dtype=torch.uint8, pin_memory=True)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=side):
            ds.t.copy_(self.t_host, non_blocking=True)
            ds.y.copy_(self.y_host, non_blocking=True)
            if ds.w is not None:
                ds.w.copy_(self.w_host, non_blocking=True)
            ds.run()
            self.result_host.copy_(ds.result, non_blocking=True)
        torch.cuda.current_stream().wait_stream(side)

    def replay(self):
        self.graph.replay()

    def results(self) -> np.ndarray:
        """Per-star results of the last replay (waits for it)."""
        torch.cuda.synchronize()
        return self.result_host.numpy().view(RESULT_DTYPE).copy()
