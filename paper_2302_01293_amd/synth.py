"""Seeded synthetic TESS-like light curves.

This module only draws inputs: sampling times, white-noise fluxes and weights,
stellar densities and injected box or trapezoid transits.  It holds none of the
search's arithmetic and is shared by the tests, the benchmark and the training
data of the period-proposal network.

Conventions (stand-ins for the QLP multi-sector light curves and TIC densities,
which are not available here):
  * a sector lasts 27.4 d (the TESS sector length in the paper's abstract) with a
    1-day mid-sector gap at [13.2, 14.2) d; consecutive sectors are separated by
    a further 1-day gap (sector k starts at 28.4 k d);
  * times carry a BTJD-like offset of 2800 d, so the FP64 phase path is exercised;
  * flux = 1 + N(0, sigma^2), weight = 1/sigma^2 per point;
  * injected transits subtract a box (or a trapezoid) of depth delta; the central
    duration of a circular orbit comes from Kepler's third law for the star's
    density: D = (P/pi) asin(sqrt(1 - b^2) R*/a).
Seeds derive from SeedSequence(230201293) spawned per workload and per star, so
every star is reproducible on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 230201293
SECTOR_DAYS = 27.4
SECTOR_STRIDE = 28.4
GAP_START, GAP_END = 13.2, 14.2
T_OFFSET = 2800.0
CADENCE_200S = 200.0 / 86400.0
CADENCE_30MIN = 30.0 / 1440.0

# Physical constants used for injections (IAU 2015 nominal values).
_GM_SUN = 1.3271244e20
_R_SUN = 6.957e8
_DAY = 86400.0

WORKLOADS = {
    "cfg0": 0,
    "cfg1": 1,
    "cfg2": 2,
    "cfg3": 3,
    "cfg4": 4,
    "tiny": 5,
    "ragged": 6,
    "varied": 7,
}


@dataclass
class Batch:
    """A packed, ragged batch of light curves."""
    t: np.ndarray          # float64 [sum N]
    y: np.ndarray          # float64 [sum N]
    w: np.ndarray          # float64 [sum N]
    offsets: np.ndarray    # int64 [S+1]
    rho: np.ndarray        # float64 [S], solar units (NaN = unknown)
    pmin: np.ndarray       # float64 [S], 0 = derive from a_min
    pmax: np.ndarray       # float64 [S], 0 = derive from the stretches
    truth: dict = field(default_factory=dict)

    @property
    def n_stars(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_points(self) -> int:
        return int(self.offsets[-1])

    def star(self, s: int):
        a, b = self.offsets[s], self.offsets[s + 1]
        return self.t[a:b], self.y[a:b], self.w[a:b]

    def subset(self, stars) -> "Batch":
        stars = np.asarray(stars, dtype=np.int64)
        ts, ys, ws, offs = [], [], [], [0]
        for s in stars:
            t, y, w = self.star(int(s))
            ts.append(t); ys.append(y); ws.append(w)
            offs.append(offs[-1] + len(t))
        truth = {k: np.asarray(v)[stars] for k, v in self.truth.items()}
        return Batch(np.concatenate(ts), np.concatenate(ys), np.concatenate(ws),
                     np.asarray(offs, np.int64), self.rho[stars].copy(), self.pmin[stars].copy(),
                     self.pmax[stars].copy(), truth)


def concat(batches) -> Batch:
    """One batch holding the stars of several (truth keys common to all are kept)."""
    keys = set.intersection(*[set(b.truth) for b in batches])
    offs = [0]
    for b in batches:
        offs.extend(offs[-1] + np.asarray(b.offsets[1:]))
    return Batch(np.concatenate([b.t for b in batches]), np.concatenate([b.y for b in batches]),
                 np.concatenate([b.w for b in batches]), np.asarray(offs, np.int64),
                 np.concatenate([b.rho for b in batches]), np.concatenate([b.pmin for b in batches]),
                 np.concatenate([b.pmax for b in batches]),
                 {k: np.concatenate([np.asarray(b.truth[k]) for b in batches]) for k in sorted(keys)})


def _star_rngs(workload: str, n: int, start: int = 0):
    ss = np.random.SeedSequence(ROOT_SEED).spawn(len(WORKLOADS))[WORKLOADS[workload]]
    kids = ss.spawn(start + n)[start:]
    return [np.random.default_rng(k) for k in kids]


def sector_times(sectors, cadence: float) -> np.ndarray:
    """Sampling times of the listed sector indices (0-based within the span)."""
    base = np.arange(0.0, SECTOR_DAYS, cadence)
    keep = ~((base >= GAP_START) & (base < GAP_END))
    base = base[keep]
    return np.concatenate([T_OFFSET + SECTOR_STRIDE * k + base for k in sectors])


def a_over_rstar(period: float, rho: float) -> float:
    """Kepler III: a/R* for a period (days) and a density in solar units."""
    p_s = period * _DAY
    return (_GM_SUN * rho * p_s * p_s / (4.0 * math.pi * math.pi)) ** (1.0 / 3.0) / _R_SUN


def central_duration(period: float, rho: float, b: float = 0.0) -> float:
    """Duration (days) of a transit with impact parameter b on a circular orbit."""
    aor = a_over_rstar(period, rho)
    x = min(1.0, math.sqrt(max(0.0, 1.0 - b * b)) / aor)
    return period / math.pi * math.asin(x)


def box_mask(t: np.ndarray, period: float, epoch: float, duration: float) -> np.ndarray:
    ph = np.mod(t - epoch, period)
    half = 0.5 * duration
    return (ph < half) | (ph > period - half)


def trapezoid(t: np.ndarray, period: float, epoch: float, duration: float, depth: float,
              q_in: float) -> np.ndarray:
    """Flux deficit of a trapezoid: full depth in the centre, linear ingress/egress."""
    d = np.mod(t - epoch + 0.5 * period, period) - 0.5 * period
    x = 0.5 * duration - np.abs(d)
    ing = max(q_in * duration, 1e-12)
    return depth * np.clip(x / ing, 0.0, 1.0)


def _pack(ts, ys, ws, rho, pmin, pmax, truth) -> Batch:
    offs = np.zeros(len(ts) + 1, np.int64)
    offs[1:] = np.cumsum([len(t) for t in ts])
    return Batch(np.concatenate(ts), np.concatenate(ys), np.concatenate(ws), offs,
                 np.asarray(rho, np.float64), np.asarray(pmin, np.float64),
                 np.asarray(pmax, np.float64), {k: np.asarray(v) for k, v in truth.items()})


def _density(rng) -> float:
    return float(10.0 ** np.clip(rng.normal(0.0, 0.5), -1.5, 1.5))


def config0() -> Batch:
    """One star: 27.4 d at 30-min cadence with a 1-day gap at day 13.7, sigma = 1e-3,
    a box transit with P = 3.1 d and depth 2e-3 (duration from solar density);
    periods 0.5-13.7 d."""
    rng = _star_rngs("cfg0", 1)[0]
    t = sector_times([0], CADENCE_30MIN)
    sig = 1e-3
    y = 1.0 + rng.normal(0.0, sig, len(t))
    P, depth = 3.1, 2e-3
    dur = central_duration(P, 1.0)
    epoch = T_OFFSET + 1.234
    y[box_mask(t, P, epoch, dur)] -= depth
    w = np.full(len(t), 1.0 / sig**2)
    truth = dict(injected=[True], period=[P], epoch=[epoch], depth=[depth], duration=[dur],
                 sigma=[sig], n_sectors=[1])
    return _pack([t], [y], [w], [1.0], [0.5], [13.7], truth)


def _one_star(rng, sectors, cadence, inj_frac, pmax_inj_cap, p_lo=0.5, p_hi=13.0,
              depth_lo=5e-4, depth_hi=1e-2):
    t = sector_times(sectors, cadence)
    sig = float(np.exp(rng.uniform(np.log(2e-4), np.log(5e-3))))
    rho = _density(rng)
    y = 1.0 + rng.normal(0.0, sig, len(t))
    inj = bool(rng.uniform() < inj_frac)
    P = epoch = depth = dur = np.nan
    if inj:
        hi = min(p_hi, pmax_inj_cap)
        P = float(np.exp(rng.uniform(np.log(p_lo), np.log(hi))))
        depth = float(np.exp(rng.uniform(np.log(depth_lo), np.log(depth_hi))))
        dur = central_duration(P, rho)
        epoch = float(t[0] + rng.uniform(0.0, P))
        y[box_mask(t, P, epoch, dur)] -= depth
    w = np.full(len(t), 1.0 / sig**2)
    return t, y, w, rho, dict(injected=inj, period=P, epoch=epoch, depth=depth, duration=dur,
                              sigma=sig, n_sectors=len(sectors))


def _collect(rows, pmin=None, pmax=None):
    ts, ys, ws, rhos = [], [], [], []
    truth = {}
    for t, y, w, rho, tr in rows:
        ts.append(t); ys.append(y); ws.append(w); rhos.append(rho)
        for k, v in tr.items():
            truth.setdefault(k, []).append(v)
    S = len(rows)
    pmin = np.zeros(S) if pmin is None else pmin
    pmax = np.zeros(S) if pmax is None else pmax
    return _pack(ts, ys, ws, rhos, pmin, pmax, truth)


def config1(n_stars: int = 4096, start: int = 0) -> Batch:
    """One sector at 200-s cadence per star (11,405 points), sigma log-uniform in
    [2e-4, 5e-3], log10 density ~ N(0, 0.5) clipped to +-1.5 dex, 20% with a box
    (P log-uniform 0.5-13 d, depth log-uniform 5e-4-1e-2).  Pmin at a = 2 R*,
    Pmax from the data (13.7 d)."""
    rows = [_one_star(rng, [0], CADENCE_200S, 0.2, 13.0) for rng in _star_rngs("cfg1", n_stars, start)]
    return _collect(rows)


def _sector_pattern(rng, max_sectors: int, p_present: float):
    span = int(rng.integers(1, max_sectors + 1))
    present = [0] + [k for k in range(1, span) if rng.uniform() < p_present]
    return present


def config2(n_stars: int = 16384, start: int = 0) -> Batch:
    """Uneven lengths: a span of 1-13 sectors, each later sector present with
    probability 0.8; noise, density and 20% boxes as in config1."""
    rows = []
    for rng in _star_rngs("cfg2", n_stars, start):
        sectors = _sector_pattern(rng, 13, 0.8)
        rows.append(_one_star(rng, sectors, CADENCE_200S, 0.2, 13.0))
    return _collect(rows)


def config4(n_stars: int = 65536, start: int = 0) -> Batch:
    """Sector-scale mix: 1-26 contiguous sectors, 10% boxes with P log-uniform in
    [0.5, min(100, baseline/2)] d."""
    rows = []
    for rng in _star_rngs("cfg4", n_stars, start):
        span = int(rng.integers(1, 27))
        sectors = list(range(span))
        base = SECTOR_STRIDE * (span - 1) + SECTOR_DAYS
        rows.append(_one_star(rng, sectors, CADENCE_200S, 0.1, 0.5 * base, p_hi=100.0))
    return _collect(rows)


def config3(n_stars: int = 200_000, start: int = 0, cadence: float = CADENCE_200S,
            max_sectors: int = 13, inj_frac: float = 0.7) -> Batch:
    """Training / evaluation light curves of the period-proposal network: a span of
    1..max_sectors sectors (later sectors present with probability 0.8), noise and
    density as config1, and in inj_frac of the stars a trapezoid with P log-uniform
    in [0.5, min(100, baseline/2)] d, depth log-uniform in [3e-4, 1e-2], ingress
    fraction U[0, 0.5] of the duration and impact parameter U[0, 0.9]."""
    rows = []
    for rng in _star_rngs("cfg3", n_stars, start):
        sectors = _sector_pattern(rng, max_sectors, 0.8)
        t = sector_times(sectors, cadence)
        sig = float(np.exp(rng.uniform(np.log(2e-4), np.log(5e-3))))
        rho = _density(rng)
        y = 1.0 + rng.normal(0.0, sig, len(t))
        inj = bool(rng.uniform() < inj_frac)
        P = epoch = depth = dur = q_in = b = np.nan
        if inj:
            hi = min(100.0, 0.5 * (t[-1] - t[0]))
            P = float(np.exp(rng.uniform(np.log(0.5), np.log(hi))))
            depth = float(np.exp(rng.uniform(np.log(3e-4), np.log(1e-2))))
            q_in = float(rng.uniform(0.0, 0.5))
            b = float(rng.uniform(0.0, 0.9))
            dur = central_duration(P, rho, b)
            epoch = float(t[0] + rng.uniform(0.0, P))
            y -= trapezoid(t, P, epoch, dur, depth, q_in)
        w = np.full(len(t), 1.0 / sig**2)
        rows.append((t, y, w, rho, dict(injected=inj, period=P, epoch=epoch, depth=depth, duration=dur,
                                        sigma=sig, n_sectors=len(sectors), q_in=q_in, impact=b)))
    return _collect(rows)


def pp_init_params(seed: int = 0) -> np.ndarray:
    """Initial FP32 parameters of the period-proposal network (random numbers only):
    W1[16][2][16] ~ N(0, 1/32), b1 = 0, W2[16][16][8] ~ N(0, 1/128), b2 = 0,
    w3[16] ~ N(0, 1/16), alpha = 4, beta = 0, delta = 0 (3122 values)."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 7, seed]))
    parts = [rng.normal(0.0, math.sqrt(1.0 / 32.0), 16 * 2 * 16), np.zeros(16),
             rng.normal(0.0, math.sqrt(1.0 / 128.0), 16 * 16 * 8), np.zeros(16),
             rng.normal(0.0, 0.25, 16), [4.0], np.zeros(512), [0.0]]
    th = np.concatenate([np.asarray(p, np.float64) for p in parts]).astype(np.float32)
    assert th.size == 3122
    return th


def varied_weights(n_stars: int = 8, start: int = 0, max_sectors: int = 13, spread: float = 2.0,
                   cadence: float = CADENCE_200S) -> Batch:
    """Stars whose points carry their own errors: a span of 1..max_sectors sectors
    (later sectors present with probability 0.8), a star-level sigma log-uniform in
    [2e-4, 5e-3] times a per-point factor log-uniform over a range of ``spread``
    (sigma_n varies by that factor within the star), flux 1 + N(0, sigma_n^2) and
    weight 1/sigma_n^2, density as config1, and a box in half of the stars."""
    rows = []
    for rng in _star_rngs("varied", n_stars, start):
        sectors = _sector_pattern(rng, max_sectors, 0.8)
        t = sector_times(sectors, cadence)
        sig0 = float(np.exp(rng.uniform(np.log(2e-4), np.log(5e-3))))
        rho = _density(rng)
        sig = sig0 * np.exp(rng.uniform(-0.5, 0.5, len(t)) * np.log(spread))
        y = 1.0 + rng.normal(0.0, 1.0, len(t)) * sig
        inj = bool(rng.uniform() < 0.5)
        P = epoch = depth = dur = np.nan
        if inj:
            hi = min(13.0, 0.25 * (t[-1] - t[0]))
            P = float(np.exp(rng.uniform(np.log(0.5), np.log(hi))))
            depth = float(np.exp(rng.uniform(np.log(5e-4), np.log(1e-2))))
            dur = central_duration(P, rho)
            epoch = float(t[0] + rng.uniform(0.0, P))
            y[box_mask(t, P, epoch, dur)] -= depth
        rows.append((t, y, 1.0 / sig**2, rho, dict(injected=inj, period=P, epoch=epoch, depth=depth,
                                                   duration=dur, sigma=sig0, n_sectors=len(sectors))))
    return _collect(rows)


def ragged(n_stars: int = 12, start: int = 0, cadence: float = CADENCE_30MIN,
           max_sectors: int = 3) -> Batch:
    """Small ragged batch for tests: 1..max_sectors sector spans with missing
    sectors at coarse cadence, half of the stars with a box transit."""
    rows = []
    for rng in _star_rngs("ragged", n_stars, start):
        sectors = _sector_pattern(rng, max_sectors, 0.7)
        base = SECTOR_STRIDE * sectors[-1] + SECTOR_DAYS
        rows.append(_one_star(rng, sectors, cadence, 0.5, 0.5 * base))
    return _collect(rows)


def tiny(n_points: int = 24, seed: int = 0, span: float = 3.0, sigma: float = 1e-3) -> Batch:
    """A single tiny, irregularly sampled light curve for brute-force checks."""
    rng = _star_rngs("tiny", seed + 1)[seed]
    t = np.sort(T_OFFSET + rng.uniform(0.0, span, n_points))
    y = 1.0 + rng.normal(0.0, sigma, n_points)
    w = rng.uniform(0.5, 2.0, n_points) / sigma**2
    return _pack([t], [y], [w], [1.0], [0.0], [0.0], dict(injected=[False]))
