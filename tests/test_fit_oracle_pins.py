"""Pins of the trapezoid-fit / noise / S/N_pink oracle (oracle/fit_oracle.py) against
facts that do not depend on its code: a noiseless trapezoid is recovered from a
perturbed start, the depth integral of the model equals a numerical quadrature of
its profile, white noise gives sigma_w = its sigma and no red noise while noise
correlated on the transit time scale does, transit counts on hand-built gaps."""
import math

import numpy as np
import pytest

from oracle import fit_oracle as F


def _grid(span=30.0, cadence=10.0 / 1440.0, t0=2800.0):
    return t0 + np.arange(0.0, span, cadence)


def test_noiseless_trapezoid_is_recovered():
    P, T0, delta, q, qin, z = 3.3, 2801.1, 5e-3, 0.04, 0.25, 1.0002
    t = _grid()
    y = F.model(t, P, [T0, delta, q, qin, z])
    w = np.full(len(t), 1e6)
    th, chi2, it, nfit = F.fit(t, y, w, P, T0 + 0.01, 0.8 * delta, 1.2 * q)
    assert nfit > 0 and it < F.MAX_ITER
    for got, exp, tol in zip(th, [T0, delta, q, qin, z], [1e-9, 1e-8, 1e-8, 1e-7, 1e-12]):
        assert abs(got - exp) <= tol * max(1.0, abs(exp)) * (1.0 if exp != 0 else 1.0), (got, exp)
    assert chi2 <= 1e-20


def test_depth_integral_equals_quadrature():
    """delta (1 - q_in) is the model's mean depth over the duration: a numerical
    quadrature of the profile of a noiseless trapezoid, refitted by detect()."""
    P = 5.0
    for qin in (0.1, 0.33, 0.5):
        th = [2801.0, 2e-3, 0.05, qin, 1.0]
        D = th[2] * P
        tt = 2801.0 + np.linspace(-D / 2, D / 2, 200001)
        integ = np.trapezoid(1.0 - F.model(tt, P, th), tt) / D
        assert abs(integ - th[1] * (1 - qin)) <= 1e-8
        t = _grid(span=30.0, cadence=2.0 / 1440.0)
        y = F.model(t, P, th) + np.random.default_rng(9).normal(0, 1e-6, len(t))
        r = F.detect(t, y, np.full(len(t), 1e12), P, 2801.0 + 1e-3, 2e-3, 0.05, 10.0)
        # noise 1e-6 per 2-min point: the refitted depth integral within 1e-7
        assert abs(r["depth_eff"] - integ) <= 1e-7, (qin, r["depth_eff"], integ)


def test_box_limit():
    """A box (q_in = 0) seen at a cadence of 2 min over a 6-h transit: from a start
    of q_in = 0.2 (36 cadences of ramp) the fitted ingress shrinks below two cadences
    (a ramp shorter than the sampling is unresolved) and depth, width at half depth
    and mid-time are the box's."""
    P, D = 5.0, 0.25
    th = [2801.0, 2e-3, D / P, 0.0, 1.0]
    t = _grid(span=30.0, cadence=2.0 / 1440.0)
    y = F.model(t, P, th) + np.random.default_rng(9).normal(0, 1e-6, len(t))
    r = F.detect(t, y, np.full(len(t), 1e12), P, 2801.003, 1.8e-3, 0.052, 10.0)
    assert r["q_in"] * D < 2 * 2.0 / 1440.0
    assert abs(r["depth"] - 2e-3) < 1e-7 and abs(r["T0"] - 2801.0) < 2.0 / 1440.0
    # the trapezoid's width at half depth, D (1 - q_in), is the box's duration
    assert abs(r["q"] * P * (1.0 - r["q_in"]) - D) < 2.0 / 1440.0


def test_white_noise_has_no_red_component():
    rng = np.random.default_rng(5)
    t = _grid(span=60.0)
    r = rng.normal(0, 1e-3, len(t))
    sw, sr = F.noise(t, r, 0.12)
    assert abs(sw - 1e-3) < 3e-5
    # sigma_D^2 - sigma_w^2 / n_bar is a fluctuation of relative size sqrt(2 / bins)
    # around zero: sigma_r stays below a tenth of sigma_w
    assert sr < 1e-4


def test_noise_correlated_on_the_duration_scale_is_red():
    """Independent offsets of sigma_b per duration-long bin plus white noise: sigma_r
    approaches sigma_b."""
    rng = np.random.default_rng(6)
    t = _grid(span=200.0)
    D = 0.2
    k = np.floor((t - t[0]) / D).astype(int)
    off = rng.normal(0, 4e-4, k.max() + 1)
    r = off[k] + rng.normal(0, 1e-3, len(t))
    sw, sr = F.noise(t, r, D)
    assert abs(sr - 4e-4) < 4e-5
    assert abs(sw - math.sqrt(1e-6 + 1.6e-7)) < 3e-5


def test_transit_count_with_gaps():
    """Transits every 2 d from 2801.0; data only in [2800, 2804.9] and [2808.95, 2812]:
    transits at 2801, 2803 and 2809, 2811 have data; 2805 and 2807 do not."""
    P, T0 = 2.0, 2801.0
    t = np.concatenate([np.arange(2800.0, 2804.9, 0.01), np.arange(2808.95, 2812.0, 0.01)])
    th = [T0, 4e-3, 0.05, 0.2, 1.0]
    y = F.model(t, P, th)
    r = F.detect(t, y, np.ones_like(t), P, T0, 4e-3, 0.05, 30.0)
    assert r["N_t"] == 4
    assert r["n_t"] == int(np.sum(np.abs(F.time_from_mid(t, r["T0"], P)) < 0.5 * r["q"] * P))
    assert r["snr_pink"] == math.inf and r["candidate"]     # no residual scatter
    y2 = y + np.random.default_rng(4).normal(0, 2e-4, len(t))
    r2 = F.detect(t, y2, np.ones_like(t), P, T0, 4e-3, 0.05, 30.0)
    assert r2["N_t"] == 4 and r2["snr_pink"] > 9 and r2["candidate"]


def test_single_transit_is_not_a_candidate():
    P, T0 = 20.0, 2801.0
    t = np.arange(2800.0, 2815.0, 0.01)
    y = F.model(t, P, [T0, 4e-3, 0.01, 0.2, 1.0]) + np.random.default_rng(1).normal(0, 1e-4, len(t))
    r = F.detect(t, y, np.ones_like(t), P, T0, 4e-3, 0.01, 30.0)
    assert r["N_t"] == 1 and not r["candidate"]


def test_low_snr_is_not_a_candidate():
    P, T0 = 2.0, 2801.0
    t = _grid()
    y = F.model(t, P, [T0, 4e-3, 0.05, 0.2, 1.0]) + np.random.default_rng(2).normal(0, 1e-4, len(t))
    r = F.detect(t, y, np.ones_like(t), P, T0, 4e-3, 0.05, 8.5)
    assert r["N_t"] >= 2 and r["snr_pink"] > 9 and not r["candidate"]
