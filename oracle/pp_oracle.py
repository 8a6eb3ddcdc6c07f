"""CPU FP64 oracle of the learned period proposal (resample, network, loss and
gradients, proposal windows, windowed S/N).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and the smoke check).  The
product path never imports it, and it shares no code with the HIP kernels.

The learned proposal is not in the paper (QLP Data Release Notes 003 searches the
full Keplerian grid of Sec. 2.1); it restricts that grid to a few period windows
and falls back to the full grid when unsure, so the plain search decides every detection.
Definitions followed here, in order:

* resample: 4096 uniform bins over the weighted baseline [t0, t_last] (Sec. 2.1
  defines the baseline); channel 0 is the weighted mean of (y - median y) / s with
  s = 1.4826 MAD(y) (the robust scale of Sec. 2.2 item 1), channel 1 is coverage;
* network: conv(2->16, k16, s2) ReLU, conv(16->16, k8, s2) ReLU, 1x1 conv to one
  channel, mean removed, autocorrelation normalised by lag 0, read at the lag of
  each of 512 log-period bins over [0.5, 100] d (linear interpolation), logits
  alpha*phi + beta, plus a null logit delta;
* BF16 points: input, conv weights and the two ReLU outputs are rounded to BF16
  (via FP32, round to nearest even) when ``bf16`` is set; everything else is FP64;
* loss: softmax cross entropy with soft targets, mean over the batch;
* proposal: top-8 bins, each widened by one bin on both sides, merged, clipped to
  [Pmin, Pmax], plus every period beyond 100 d; confidence = null probability +
  probability mass inside the windows; below the threshold the full grid is used;
* windowed S/N: trend and sigma from a coarse spectrum (Sturges bins, medians,
  linear interpolation, 1.4826 MAD; Sec. 2.2 item 1 and its footnote) applied to
  the SR of the window frequencies;
* coarse-peak windows (guided proposal): the n largest values of the coarse
  spectrum's S/N, each more than h coarse steps from every larger one chosen
  before it (ties to the lower index), each widened by h coarse steps on both sides
  and mapped to the fine grid (both grids are uniform in u = f^(1/3) from the same
  u_min), added to the network's windows; overlapping or touching ranges merged.
"""
from __future__ import annotations

import math

import numpy as np

L0, C_IN = 4096, 2
C1, K1, S1, P1 = 16, 16, 2, 7
C2, K2, S2, P2 = 16, 8, 2, 3
L1, L2 = L0 // S1, L0 // (S1 * S2)
NPB = 512                      # period bins
PB_LO, PB_HI = 0.5, 100.0      # days
EPS = 1e-6
TOPK = 8
CONF = 0.9
MAX_WIN = TOPK + 2             # windows per star in the proposal output

OFF = {}
_sizes = [("W1", C1 * C_IN * K1), ("b1", C1), ("W2", C2 * C1 * K2), ("b2", C2), ("w3", C2),
          ("alpha", 1), ("beta", NPB), ("delta", 1)]
_o = 0
for _n, _s in _sizes:
    OFF[_n] = (_o, _o + _s)
    _o += _s
NPARAM = _o


def unpack(theta):
    th = np.asarray(theta, np.float64)
    g = {k: th[a:b] for k, (a, b) in OFF.items()}
    return dict(W1=g["W1"].reshape(C1, C_IN, K1), b1=g["b1"], W2=g["W2"].reshape(C2, C1, K2), b2=g["b2"],
                w3=g["w3"], alpha=float(g["alpha"][0]), beta=g["beta"], delta=float(g["delta"][0]))


def pack(d) -> np.ndarray:
    th = np.zeros(NPARAM)
    for k, (a, b) in OFF.items():
        th[a:b] = np.asarray(d[k], np.float64).reshape(-1)
    return th


def bf16(x):
    """Round to BF16 through FP32 (both steps round to nearest even); FP64 values."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    f = bf16(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def period_edges() -> np.ndarray:
    i = np.arange(NPB + 1, dtype=np.float64)
    return PB_LO * np.power(PB_HI / PB_LO, i / NPB)


def period_centres() -> np.ndarray:
    k = np.arange(NPB, dtype=np.float64)
    return PB_LO * np.power(PB_HI / PB_LO, (k + 0.5) / NPB)


def period_bin(p: float) -> int:
    """Log-period bin of a period (days), or -1 outside [0.5, 100)."""
    if not (PB_LO <= p < PB_HI):
        return -1
    k = int(math.floor(math.log(p / PB_LO) / math.log(PB_HI / PB_LO) * NPB))
    return min(max(k, 0), NPB - 1)


# ---------------------------------------------------------------------------
# resample
# ---------------------------------------------------------------------------
def _median(v):
    v = np.sort(np.asarray(v, np.float64))
    n = len(v)
    if n == 0:
        return 0.0
    return float(v[n // 2]) if n % 2 else 0.5 * (float(v[n // 2 - 1]) + float(v[n // 2]))


def resample(t, y, w, nbins: int = L0):
    """One star -> (X [2, nbins] FP64 holding BF16 values, lag step in days)."""
    t, y, w = (np.asarray(a, np.float64) for a in (t, y, w))
    good = w > 0
    tg = t[good]
    t0, t1 = float(tg[0]), float(tg[-1])
    T = t1 - t0
    med = _median(y[good])
    mad = _median(np.abs(y[good] - med))
    s = 1.4826 * mad
    X = np.zeros((2, nbins))
    sw = np.zeros(nbins)
    swz = np.zeros(nbins)
    for i in range(len(t)):                     # point order, one bin each
        b = int(math.floor(((t[i] - t0) / T) * nbins)) if T > 0 else 0
        b = min(max(b, 0), nbins - 1)
        z = (y[i] - med) / s if s > 0 else 0.0
        sw[b] += w[i]
        swz[b] += w[i] * z
    occ = sw > 0
    X[0, occ] = swz[occ] / sw[occ]
    X[1, occ] = 1.0
    return bf16(X), T / (nbins // (S1 * S2))


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def _conv(x, W, b, stride, pad):
    """out[o, l] = b[o] + sum_{c,k} W[o,c,k] x[c, stride*l + k - pad] (zeros outside)."""
    Cout, Cin, K = W.shape
    Lin = x.shape[1]
    Lout = Lin // stride
    xp = np.zeros((Cin, Lin + 2 * K))
    xp[:, pad + K - pad: pad + K - pad + Lin] = x   # x[c, p] at xp[c, p + K]
    idx = stride * np.arange(Lout)[:, None] + np.arange(K)[None, :] - pad + K   # [Lout, K]
    cols = xp[:, idx]                                # [Cin, Lout, K]
    return b[:, None] + np.einsum("ock,clk->ol", W, cols)


def lags(dlag):
    """Fractional lag (in network steps) of each period-bin centre; NaN where unused."""
    tau = period_centres() / dlag
    tau[(tau < 2.0) | (tau > L2 - 1)] = np.nan
    return tau


def forward(X, theta, dlag, use_bf16=True):
    """One star.  Returns (logits [513], cache of intermediates)."""
    p = unpack(theta)
    r = bf16 if use_bf16 else (lambda v: np.asarray(v, np.float64))
    x = r(X)
    W1, W2 = r(p["W1"]), r(p["W2"])
    z1 = _conv(x, W1, p["b1"], S1, P1)
    a1 = r(np.maximum(z1, 0.0))
    z2 = _conv(a1, W2, p["b2"], S2, P2)
    a2 = r(np.maximum(z2, 0.0))
    s = p["w3"] @ a2
    sh = s - s.mean()
    full = np.correlate(sh, sh, mode="full")        # lag -(L-1) .. L-1
    A = full[L2 - 1:] / L2                           # A[tau] = sum_t sh[t] sh[t+tau] / L
    den = A[0] + EPS
    Ah = A / den
    tau = lags(dlag)
    phi = np.zeros(NPB)
    ok = ~np.isnan(tau)
    phi[ok] = np.interp(tau[ok], np.arange(L2), Ah)
    logits = np.empty(NPB + 1)
    logits[:NPB] = p["alpha"] * phi + p["beta"]
    logits[NPB] = p["delta"]
    cache = dict(x=x, W1=W1, W2=W2, z1=z1, a1=a1, z2=z2, a2=a2, sh=sh, A=A, den=den, Ah=Ah, tau=tau, phi=phi,
                 p=p)
    return logits, cache


def softmax(z):
    e = np.exp(z - z.max())
    return e / e.sum()


def soft_target(label: int) -> np.ndarray:
    """Class index (0..511 period bin, 512 = null) -> smoothed target distribution."""
    q = np.zeros(NPB + 1)
    if label < 0 or label >= NPB:
        q[NPB] = 1.0
        return q
    g = math.exp(-0.5)
    for k, v in ((label - 1, g), (label, 1.0), (label + 1, g)):
        if 0 <= k < NPB:
            q[k] = v
    return q / q.sum()


def loss_and_grad(Xs, theta, dlags, labels, use_bf16=True):
    """Mean softmax cross entropy over a batch and its gradient w.r.t. theta."""
    B = len(Xs)
    g = np.zeros(NPARAM)
    loss = 0.0
    for X, dl, lab in zip(Xs, dlags, labels):
        z, c = forward(X, theta, dl, use_bf16)
        q = soft_target(int(lab))
        pr = softmax(z)
        loss += -float(np.sum(q * np.log(np.maximum(pr, 1e-300))))
        g += backward(c, (pr - q))
    return loss / B, g / B


def backward(c, dz):
    """Gradient of one star's loss given dL/dlogits."""
    p = c["p"]
    gd = {k: np.zeros_like(np.asarray(p[k], np.float64)) for k in ("W1", "b1", "W2", "b2", "w3", "beta")}
    dphi = p["alpha"] * dz[:NPB]
    galpha = float(np.dot(dz[:NPB], c["phi"]))
    gd["beta"] = dz[:NPB].copy()
    gdelta = float(dz[NPB])
    # interpolation
    dAh = np.zeros(L2)
    tau = c["tau"]
    for k in range(NPB):
        if np.isnan(tau[k]):
            continue
        i0 = int(math.floor(tau[k]))
        fr = tau[k] - i0
        if i0 >= L2 - 1:
            dAh[L2 - 1] += dphi[k]
            continue
        dAh[i0] += (1.0 - fr) * dphi[k]
        dAh[i0 + 1] += fr * dphi[k]
    # normalisation Ah = A / (A0 + eps)
    A, den = c["A"], c["den"]
    dA = dAh / den
    dA[0] -= float(np.dot(dAh, A)) / (den * den)
    # autocorrelation A[tau] = sum_t sh[t] sh[t+tau] / L
    sh = c["sh"]
    dsh = np.zeros(L2)
    for tau_i in range(L2):
        if dA[tau_i] == 0.0:
            continue
        v = dA[tau_i] / L2
        dsh[:L2 - tau_i] += v * sh[tau_i:]
        dsh[tau_i:] += v * sh[:L2 - tau_i]
    ds = dsh - dsh.mean()
    a2 = c["a2"]
    gd["w3"] = a2 @ ds
    dz2 = np.outer(p["w3"], ds) * (c["z2"] > 0)
    gd["b2"] = dz2.sum(axis=1)
    gd["W2"], da1 = _conv_back(c["a1"], c["W2"], dz2, S2, P2)
    dz1 = da1 * (c["z1"] > 0)
    gd["b1"] = dz1.sum(axis=1)
    gd["W1"], _ = _conv_back(c["x"], c["W1"], dz1, S1, P1)
    out = dict(gd)
    out["alpha"] = np.array([galpha])
    out["delta"] = np.array([gdelta])
    return pack(out)


def _conv_back(x, W, dz, stride, pad):
    Cout, Cin, K = W.shape
    Lin = x.shape[1]
    Lout = dz.shape[1]
    xp = np.zeros((Cin, Lin + 2 * K))
    xp[:, K:K + Lin] = x
    idx = stride * np.arange(Lout)[:, None] + np.arange(K)[None, :] - pad + K
    cols = xp[:, idx]                                   # [Cin, Lout, K]
    dW = np.einsum("ol,clk->ock", dz, cols)
    dcols = np.einsum("ock,ol->clk", W, dz)
    dxp = np.zeros_like(xp)
    np.add.at(dxp, (slice(None), idx), dcols)
    return dW, dxp[:, K:K + Lin]


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba), in place on copies; returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# proposal
# ---------------------------------------------------------------------------
def propose(logits, pmin, pmax, umin, A, nf, topk=TOPK, conf=CONF, pb_hi_window=True):
    """Frequency-index ranges [i0, i1) to search for one star, confidence, fallback
    (``pb_hi_window``: include the window over periods beyond 100 d)."""
    pr = softmax(np.asarray(logits, np.float64))
    pb = pr[:NPB]
    order = sorted(range(NPB), key=lambda k: (-pb[k], k))[:topk]
    sel = np.zeros(NPB, bool)
    for k in order:
        sel[max(0, k - 1):min(NPB, k + 2)] = True
    c = float(pr[NPB] + pb[sel].sum())
    if c < conf:
        return [(0, nf)], c, True
    edges = period_edges()
    ivs = []
    k = 0
    while k < NPB:                                  # maximal runs of selected bins
        if sel[k]:
            k1 = k
            while k1 + 1 < NPB and sel[k1 + 1]:
                k1 += 1
            ivs.append((edges[k], edges[k1 + 1]))
            k = k1 + 1
        else:
            k += 1
    if pb_hi_window and pmax > PB_HI:
        ivs.append((PB_HI, pmax))
    out = []
    for lo, hi in ivs:
        lo, hi = max(lo, pmin), min(hi, pmax)
        if hi <= lo:
            continue
        f_lo, f_hi = 1.0 / hi, 1.0 / lo
        i0 = max(0, int(math.ceil((f_lo ** (1.0 / 3.0) - umin) / A)))
        i1 = min(nf - 1, int(math.floor((f_hi ** (1.0 / 3.0) - umin) / A)))
        if i1 >= i0:
            out.append((i0, i1 + 1))
    return out, c, False


def window_snr(f_coarse, sr_coarse, f_fine, sr_fine, ranges, sturges):
    """S/N of the window frequencies with trend and sigma from a coarse spectrum.

    Returns (index of the best S/N among the window frequencies, its S/N, sigma)."""
    f_coarse = np.asarray(f_coarse, np.float64)
    sr_coarse = np.asarray(sr_coarse, np.float64)
    n = len(f_coarse)
    f0, span = f_coarse[0], f_coarse[-1] - f_coarse[0]
    kb = np.zeros(n, np.int64) if span <= 0 else np.minimum(
        sturges - 1, np.floor(((f_coarse - f0) / span) * sturges).astype(np.int64))
    kx, ky = [], []
    for b in range(sturges):
        sel = kb == b
        if sel.any():
            kx.append(f0 + ((b + 0.5) * span) / sturges)
            ky.append(_median(sr_coarse[sel]))
    trend_c = np.interp(f_coarse, kx, ky)
    rho = sr_coarse - trend_c
    med = _median(rho)
    sigma = 1.4826 * _median(np.abs(rho - med))
    best_i, best_v = -1, -np.inf
    for i0, i1 in ranges:
        for i in range(i0, i1):
            v = (sr_fine[i] - float(np.interp(f_fine[i], kx, ky))) / sigma if sigma > 0 else 0.0
            if v > best_v:
                best_i, best_v = i, v
    return best_i, best_v, sigma


# ---------------------------------------------------------------------------
# guided proposal: coarse-peak windows
# ---------------------------------------------------------------------------
def coarse_peaks(snr_coarse, n_peaks: int, halfwidth: int):
    """Indices of the n_peaks largest coarse S/N values, largest first; each pick
    blocks the picks within halfwidth coarse steps of it; ties to the lower index."""
    v = np.asarray(snr_coarse, np.float64)
    picks = []
    for _ in range(n_peaks):
        best = -1
        for i in range(len(v)):
            if any(abs(i - q) <= halfwidth for q in picks):
                continue
            if best < 0 or v[i] > v[best]:
                best = i
        if best < 0:
            break
        picks.append(best)
    return picks


def coarse_windows(picks, umin_c, A_c, nf_c, umin, A, nf, halfwidth: int):
    """Fine index ranges [i0, i1) covering coarse indices pick +- halfwidth (clipped
    to the coarse grid): i0 = ceil((u_c(lo) - u_min) / A), i1 - 1 = floor((u_c(hi) -
    u_min) / A), clipped to [0, nf)."""
    out = []
    for ic in picks:
        lo, hi = max(0, ic - halfwidth), min(nf_c - 1, ic + halfwidth)
        a = math.ceil(((umin_c + lo * A_c) - umin) / A)
        e = math.floor(((umin_c + hi * A_c) - umin) / A)
        i0, i1 = max(0, a), min(nf - 1, e)
        if i1 >= i0:
            out.append((i0, i1 + 1))
    return out


def merge_ranges(ranges):
    """Union of index ranges as sorted disjoint ranges (touching ranges join)."""
    out = []
    for a, b in sorted(ranges):
        if out and a <= out[-1][1]:
            out[-1] = (out[-1][0], max(out[-1][1], b))
        else:
            out.append((a, b))
    return out


def propose_guided(logits, pmin, pmax, umin, A, nf, snr_coarse, umin_c, A_c, n_peaks, halfwidth,
                   topk=TOPK, conf=CONF, search_long=True):
    """The proposal of ``propose`` (topk may be 0) with the coarse-peak windows added
    to a confident star's windows (a star that falls back searches its full grid);
    ``search_long`` False drops the window over periods beyond 100 d."""
    if topk > 0:
        ranges, c, fb = propose(logits, pmin, pmax, umin, A, nf, topk, conf,
                                pb_hi_window=search_long)
    else:
        pr = softmax(np.asarray(logits, np.float64))
        c = float(pr[NPB])
        fb = c < conf
        ranges = [(0, nf)]
        if not fb:
            ranges = []
            if search_long and pmax > PB_HI:
                lo, hi = max(PB_HI, pmin), pmax
                if hi > lo:
                    i0 = max(0, int(math.ceil(((1.0 / hi) ** (1.0 / 3.0) - umin) / A)))
                    i1 = min(nf - 1, int(math.floor(((1.0 / lo) ** (1.0 / 3.0) - umin) / A)))
                    if i1 >= i0:
                        ranges.append((i0, i1 + 1))
    if fb:
        return [(0, nf)], c, True
    picks = coarse_peaks(snr_coarse, n_peaks, halfwidth)
    ranges = merge_ranges(list(ranges) + coarse_windows(picks, umin_c, A_c, len(snr_coarse), umin, A, nf,
                                                         halfwidth))
    return ranges, c, False
