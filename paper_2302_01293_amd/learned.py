"""Learned period proposal on the GPU: resample -> CNN heatmap -> top-k period
windows -> restricted BLS with full-grid fallback -> windowed S/N.

Everything numeric runs in the library's HIP kernels (``include/mi355pp.h``);
this module allocates device buffers with PyTorch, passes pointers and streams,
and holds the training loop's bookkeeping (labels from the plain search, batches,
learning rate).  Labels follow the plain search: a light curve's class is the
log-period bin of its best-S/N plain peak when that peak has S/N >= 9 (the QLP
threshold, Sec. 2.2) and matches the injected period (or 2P, P/2) within 1%,
otherwise the null class.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib, synth
from ._lib import PP_MAX_WINDOWS, PP_NCLASS, PP_NPARAM, check
from .device import DeviceSearch, _stream_handle

NPB = PP_NCLASS - 1
SNR_MIN = 9.0


def period_bin(p: float) -> int:
    """Log-period bin (512 over [0.5, 100) d) of a period, or -1 outside."""
    if not (0.5 <= p < 100.0):
        return -1
    k = int(math.floor(math.log(p / 0.5) / math.log(200.0) * NPB))
    return min(max(k, 0), NPB - 1)


def soft_targets(labels: np.ndarray) -> np.ndarray:
    """Class indices (period bin or -1 for null) -> targets smoothed over +-1 bin
    with Gaussian weights exp(-1/2) (rows sum to 1), FP32 [B, 513]."""
    B = len(labels)
    q = np.zeros((B, PP_NCLASS), np.float32)
    g = math.exp(-0.5)
    for i, k in enumerate(labels):
        k = int(k)
        if k < 0 or k >= NPB:
            q[i, NPB] = 1.0
            continue
        ws = [(k - 1, g), (k, 1.0), (k + 1, g)]
        tot = sum(v for j, v in ws if 0 <= j < NPB)
        for j, v in ws:
            if 0 <= j < NPB:
                q[i, j] = v / tot
    return q


def plain_labels(results: np.ndarray, truth: dict) -> np.ndarray:
    """Label of each star from the plain search's results and the injections."""
    out = np.full(len(results), -1, np.int64)
    for s in range(len(results)):
        if not bool(truth["injected"][s]):
            continue
        if results["status"][s] != 0 or not results["snr"][s] >= SNR_MIN:
            continue
        p, pt = float(results["period"][s]), float(truth["period"][s])
        if any(abs(p / (pt * m) - 1.0) < 0.01 for m in (1.0, 2.0, 0.5)):
            out[s] = period_bin(p)
    return out


class ProposalNet:
    """FP32 master weights and Adam moments of the proposal CNN on the device."""

    def __init__(self, theta: np.ndarray | None = None, seed: int = 0, device: str = "cuda"):
        th = synth.pp_init_params(seed) if theta is None else np.asarray(theta, np.float32)
        assert th.shape == (PP_NPARAM,)
        self.device = torch.device(device)
        self.theta = torch.as_tensor(th.copy()).to(self.device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0
        self.grad = torch.zeros_like(self.theta)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._scratch = {}

    def params_host(self) -> np.ndarray:
        return self.theta.cpu().numpy().copy()

    def forward(self, x: torch.Tensor, lag: torch.Tensor, act: torch.Tensor | None = None, stream=None):
        B = int(x.shape[0])
        logits = torch.empty((B, PP_NCLASS), dtype=torch.float32, device=self.device)
        check("pp_forward", _lib.lib().pp_forward(self.theta.data_ptr(), x.data_ptr(), lag.data_ptr(), B,
                                                   logits.data_ptr(), None if act is None else act.data_ptr(),
                                                   _stream_handle(stream)))
        return logits

    def _buffers(self, B: int):
        if B not in self._scratch:
            n = ctypes.c_int64()
            check("pp_act_bytes", _lib.lib().pp_act_bytes(B, ctypes.byref(n)))
            self._scratch[B] = (torch.empty(int(n.value), dtype=torch.uint8, device=self.device),
                                torch.empty((B, PP_NPARAM), dtype=torch.float32, device=self.device),
                                torch.empty(B, dtype=torch.float32, device=self.device))
        return self._scratch[B]

    def gradient(self, x, lag, target, stream=None):
        """Loss and gradient (into self.grad, self.loss) of a batch; returns logits."""
        B = int(x.shape[0])
        act, gpart, lpart = self._buffers(B)
        logits = self.forward(x, lag, act, stream)
        check("pp_backward", _lib.lib().pp_backward(self.theta.data_ptr(), x.data_ptr(), lag.data_ptr(),
                                                     target.data_ptr(), logits.data_ptr(), act.data_ptr(), B,
                                                     gpart.data_ptr(), lpart.data_ptr(), self.grad.data_ptr(),
                                                     self.loss.data_ptr(), _stream_handle(stream)))
        return logits

    def train_step(self, x, lag, target, lr: float, stream=None):
        self.gradient(x, lag, target, stream)
        self.step += 1
        check("pp_adam", _lib.lib().pp_adam(self.theta.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                             self.grad.data_ptr(), self.step, float(lr), _stream_handle(stream)))
        return self.loss


def resample(ds: DeviceSearch, stream=None):
    """BF16 network input [S, 2, 4096] and lag step [S] for every star of a search."""
    S = ds.plan.n_stars
    x = torch.empty((S, 2, _lib.PP_NBINS_IN), dtype=torch.int16, device=ds.device)
    lag = torch.empty(S, dtype=torch.float64, device=ds.device)
    check("pp_resample", _lib.lib().pp_resample(ds.plan.h, ds.ws_ptr, ds.t.data_ptr(), ds.y.data_ptr(),
                                                 None if ds.w is None else ds.w.data_ptr(), x.data_ptr(),
                                                 lag.data_ptr(), _stream_handle(stream)))
    return x, lag


class LearnedSearch:
    """The learned path over one batch: a fine plan (the paper's grid) and a coarse
    plan (samples per peak divided by ``coarse_factor``) over the same device
    inputs."""

    def __init__(self, batch, net: ProposalNet, params=None, coarse_factor: int = 16, topk: int = 8,
                 conf: float = 0.9, coarse_peaks: int = 0, halfwidth: int = 3, search_long: bool = True):
        """``coarse_peaks`` > 0: the windows of a confident star also cover that many
        peaks of the coarse S/N spectrum (``pp_propose_guided``), each widened by
        ``halfwidth`` coarse steps; ``search_long`` = False then drops the blanket
        window over periods beyond the network's 100-d range."""
        p = params if params is not None else _lib.default_params()
        self.fine = DeviceSearch.from_batch(batch, p)
        cp = _lib.default_params(**{f: getattr(p, f) for f, _ in _lib.BlsParams._fields_})
        cp.spp = p.spp / coarse_factor
        self.coarse_peaks, self.halfwidth = int(coarse_peaks), int(halfwidth)
        self.search_long = bool(search_long)
        self.coarse = DeviceSearch(batch.t, batch.y, batch.w, batch.offsets, batch.rho, batch.pmin, batch.pmax,
                                   cp, want_best=False, want_snr=self.coarse_peaks > 0,
                                   inputs=(self.fine.t, self.fine.y, self.fine.w))
        self.net = net
        self.topk, self.conf = int(topk), float(conf)
        S = self.fine.plan.n_stars
        dev = self.fine.device
        self.windows = torch.empty((S, PP_MAX_WINDOWS, 3), dtype=torch.int64, device=dev)
        self.fallback = torch.empty(S, dtype=torch.uint8, device=dev)
        self.confidence = torch.empty(S, dtype=torch.float32, device=dev)
        cap = ctypes.c_int64()
        check("pp_tile_capacity", _lib.lib().pp_tile_capacity(self.fine.plan.h, ctypes.byref(cap)))
        self.tiles = torch.empty((int(cap.value), 3), dtype=torch.int64, device=dev)
        self.logits = None

    def run(self, stream=None):
        h = _stream_handle(stream)
        L = _lib.lib()
        f, c = self.fine, self.coarse
        f.run_prepare(stream)
        c.run_prepare(stream)
        if self.coarse_peaks > 0:
            c.run_search(stream)
            c.run_snr(stream)
        x, lag = resample(f, stream)
        self.logits = self.net.forward(x, lag, None, stream)
        if self.coarse_peaks > 0:
            check("pp_propose_guided", L.pp_propose_guided(
                f.plan.h, f.ws_ptr, self.logits.data_ptr(), self.topk, self.conf, int(self.search_long),
                c.plan.h, c.ws_ptr,
                c.snr.data_ptr(), self.coarse_peaks, self.halfwidth, self.windows.data_ptr(),
                self.fallback.data_ptr(), self.confidence.data_ptr(), self.tiles.data_ptr(), h))
        else:
            check("pp_propose", L.pp_propose(f.plan.h, f.ws_ptr, self.logits.data_ptr(), self.topk, self.conf,
                                             self.windows.data_ptr(), self.fallback.data_ptr(),
                                             self.confidence.data_ptr(), self.tiles.data_ptr(), h))
            c.run_search(stream)
        f.run_search(stream, windows=self.tiles)
        check("pp_snr_windows", L.pp_snr_windows(f.plan.h, f.ws_ptr, f.sr.data_ptr(), f.best.data_ptr(),
                                                 c.plan.h, c.ws_ptr, c.sr.data_ptr(), self.windows.data_ptr(),
                                                 PP_MAX_WINDOWS, self.fallback.data_ptr(), f.result.data_ptr(),
                                                 h))

    def searched_fraction(self) -> float:
        """Fraction of the fine grid's frequencies inside the searched windows."""
        w = self.windows.cpu().numpy().reshape(-1, 3)
        w = w[w[:, 0] >= 0]
        return float(np.sum(w[:, 2] - w[:, 1])) / float(self.fine.plan.n_freq)


def labelled_inputs(batch, params=None):
    """Run the plain search on a batch; return (x, lag, labels, plain results)."""
    ds = DeviceSearch.from_batch(batch, params)
    ds.run()
    x, lag = resample(ds)
    torch.cuda.synchronize()
    res = ds.results_host()
    labels = plain_labels(res, batch.truth)
    return x, lag, labels, res


def train(net: ProposalNet, x: torch.Tensor, lag: torch.Tensor, labels: np.ndarray, epochs: int = 20,
          batch: int = 128, lr: float = 3e-3, seed: int = 0, log=None):
    """Adam on shuffled mini-batches; returns the per-epoch mean loss."""
    S = int(x.shape[0])
    target = torch.as_tensor(soft_targets(labels)).to(net.device)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(S)).to(net.device)
        tot = 0.0
        nb = 0
        for i in range(0, S - batch + 1, batch):
            idx = order[i:i + batch]
            loss = net.train_step(x[idx].contiguous(), lag[idx].contiguous(), target[idx].contiguous(), lr)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        if log:
            log("epoch %d loss %.4f" % (ep, hist[-1]))
    return hist


def recovery(plain_res: np.ndarray, learned_res: np.ndarray, truth: dict, tol_index: int = 2) -> dict:
    """Recovery of plain detections by the learned path.

    Plain detections: S/N >= 9 and the period matches the injection (P, 2P or P/2
    within 1%).  Recovered: the learned path reports S/N >= 9 at a frequency index
    within tol_index of the plain one."""
    det = plain_labels(plain_res, truth) >= 0
    # injections beyond the heatmap are detections too
    for s in range(len(plain_res)):
        if det[s] or not bool(truth["injected"][s]) or plain_res["status"][s] != 0:
            continue
        if plain_res["snr"][s] >= SNR_MIN:
            p, pt = float(plain_res["period"][s]), float(truth["period"][s])
            det[s] = any(abs(p / (pt * m) - 1.0) < 0.01 for m in (1.0, 2.0, 0.5))
    rec = det & (learned_res["snr"] >= SNR_MIN) & (np.abs(learned_res["i_snr"] - plain_res["i_snr"]) <= tol_index)
    exact = det & (learned_res["i_snr"] == plain_res["i_snr"])
    n = int(det.sum())
    return dict(plain_detections=n, recovered=int(rec.sum()), recovery=float(rec.sum()) / max(n, 1),
                exact_index=int(exact.sum()))


def time_paths(batch, net: ProposalNet, reps: int = 3, **kw) -> dict:
    """Device time of the plain path (prepare, full search, S/N) and of the learned
    path (prepare x2, resample, forward, propose, coarse search, windowed search,
    windowed S/N) on the same stars; median of ``reps`` runs each."""
    plain = DeviceSearch.from_batch(batch)
    learned = LearnedSearch(batch, net, **kw)
    stream = torch.cuda.current_stream()

    def timed(fn):
        ms = []
        fn()
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    t_plain = timed(plain.run)
    t_learn = timed(learned.run)
    pres = plain.results_host()
    lres = learned.fine.results_host()
    fb = learned.fallback.cpu().numpy()
    out = dict(plain_ms=t_plain, learned_ms=t_learn, speedup=t_plain / t_learn,
               fallback_fraction=float(fb.mean()), searched_fraction=learned.searched_fraction())
    out.update(recovery(pres, lres, batch.truth))
    return out, pres, lres
