"""Pins of the oracle's two search variants of QLP Data Release Notes 003, Sec. 2.1
and its footnote: the exact circular-orbit duration (``exact_duration``) and the
per-duration rebinning (``rebin``: one bin set per duration of a continuous ladder,
windows of noverlap bins).

Each test checks the variant against geometry solved independently (a chord found
by bisection, no arcsine), a brute-force enumeration over points, a noiseless box
with a closed-form answer, or a special case that reduces to the plain search.
"""
import math

import numpy as np
import pytest

from paper_2302_01293_amd import synth


# ---------------------------------------------------------------------------
# Exact circular duration
# ---------------------------------------------------------------------------
def _chord_duty_cycle(aor: float) -> float:
    """Fraction of a circular orbit of radius a (in stellar radii) during which a
    central transit lasts: the planet's projected distance a |sin(2 pi phi)| stays
    below one stellar radius for |phi| < phi*, found by bisection."""
    lo, hi = 0.0, 0.25
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if aor * math.sin(2.0 * math.pi * mid) < 1.0:
            lo = mid
        else:
            hi = mid
    return 2.0 * lo


@pytest.mark.parametrize("aor,rho", [(2.0, 1.0), (3.0, 1.0), (7.5, 0.3), (40.0, 2.0), (400.0, 1.0)])
def test_exact_duty_cycle_is_the_chord(oracle, aor, rho):
    f = 1.0 / oracle.period_at_a(aor, rho)
    q = oracle.qcirc_exact(f, rho)
    assert abs(q / _chord_duty_cycle(aor) - 1.0) < 1e-12
    # the small-angle form is the leading term: asin(x) / x - 1 = x^2/6 + 3x^4/40 + O(x^6)
    qs = oracle.qcirc(f, rho)
    x = 1.0 / aor
    assert abs((q / qs - 1.0) - x ** 2 / 6.0 - 3.0 * x ** 4 / 40.0) < 0.1 * x ** 6 + 1e-13


def _star(span=27.0, seed=0):
    rng = np.random.default_rng(seed)
    t = synth.T_OFFSET + np.sort(rng.uniform(0.0, span, 1500))
    return t


def test_exact_bins_are_the_smallest_covering_count(oracle):
    t = _star()
    pe = oracle.params(exact_duration=1)
    fs, nbs, _ = oracle.grid(t, None, 1.0, oracle.params())
    fe, nbe, _ = oracle.grid(t, None, 1.0, pe)
    assert np.array_equal(fs, fe)                      # the grid itself is unchanged
    assert np.all(nbe <= nbs) and np.any(nbe < nbs)    # longer durations: fewer bins
    qlo = np.array([0.5 * oracle.qcirc_exact(f, 1.0) for f in fe])
    # nb = the fewest bins of width <= q_lo / noverlap
    assert np.all(3.0 / nbe <= qlo * (1 + 1e-15))
    assert np.all(3.0 / (nbe - 1) > qlo * (1 - 1e-15))


def test_exact_search_changes_only_the_bins(oracle):
    b = synth.tiny(40, seed=4, span=6.0)
    t, y, w = b.star(0)
    s0 = oracle.bls_star(t, y, w, 1.0, pmin=0.3, pmax=3.0)
    s1 = oracle.bls_star(t, y, w, 1.0, oracle.params(exact_duration=1), pmin=0.3, pmax=3.0)
    same = s0.nb == s1.nb
    assert np.array_equal(s0.f, s1.f) and same.any() and (~same).any()
    for k in ("sr", "m", "j", "r", "s"):
        assert np.array_equal(getattr(s0, k)[same], getattr(s1, k)[same]), k


# ---------------------------------------------------------------------------
# Per-duration rebinning
# ---------------------------------------------------------------------------
def test_rebin_ladder(oracle):
    g = oracle.rebin_ladder()
    # k = 0 .. ceil(ln(2.0 / 0.5) / 0.1) = 14, capped at qmax / qmin = 4
    assert len(g) == 15 and g[0] == 1.0 and g[-1] == 4.0
    k = np.arange(14)
    assert np.allclose(g[:14], np.exp(0.1 * k), rtol=1e-15, atol=0)
    assert np.all(np.diff(g) > 0)


def _rebin_bruteforce(t, y, w, f, t0, qlo, g, noverlap=3):
    """Best (power, k, j, nb) over every bin set and window, summing over points."""
    wt = w / w.sum()
    x = y - np.sum(wt * y)
    ph = (t - t0) * f
    ph = ph - np.floor(ph)
    best = (-1.0, 0, -1, 0)
    for k, gk in enumerate(g):
        nb = int(math.ceil(noverlap / (qlo * gk)))
        if noverlap >= nb:
            continue
        b = np.minimum(nb - 1, np.floor(ph * nb).astype(np.int64))
        for j in range(nb):
            inwin = ((b - j) % nb) < noverlap
            r, s = wt[inwin].sum(), (wt * x)[inwin].sum()
            if 0 < r < 1:
                p2 = s * s / (r * (1 - r))
                if p2 > best[0] * (1 + 1e-12):
                    best = (p2, k, j, nb)
    return best


@pytest.mark.parametrize("seed,exact", [(0, 0), (1, 0), (2, 1)])
def test_rebin_bruteforce(oracle, seed, exact):
    b = synth.tiny(24, seed=seed, span=3.0)
    t, y, w = b.star(0)
    p = oracle.params(rebin=1, exact_duration=exact)
    sp = oracle.bls_star(t, y, w, 1.0, p, pmin=0.4, pmax=1.5)
    g = oracle.rebin_ladder(p)
    for i in np.linspace(0, len(sp.f) - 1, 6).astype(int):
        f = sp.f[i]
        qlo = 0.5 * (oracle.qcirc_exact(f, 1.0) if exact else oracle.qcirc(f, 1.0))
        p2, k, j, nb = _rebin_bruteforce(t, y, w, f, sp.bounds.t0, qlo, g)
        assert abs(sp.sr[i] - math.sqrt(p2)) <= 1e-12 * math.sqrt(p2)
        assert (sp.m[i], sp.j[i], sp.nb[i]) == (k, j, nb)


def test_rebin_with_one_duration_is_the_plain_search_at_noverlap_bins(oracle):
    # qmax = qmin: the continuous ladder is {q_lo} and the plain ladder is {noverlap}
    # fine bins, so both search windows of noverlap bins of width q_lo / noverlap.
    b = synth.tiny(30, seed=7, span=4.0)
    t, y, w = b.star(0)
    kw = dict(qmax_fac=0.5)
    s0 = oracle.bls_star(t, y, w, 1.0, oracle.params(**kw), pmin=0.3, pmax=2.0)
    s1 = oracle.bls_star(t, y, w, 1.0, oracle.params(rebin=1, **kw), pmin=0.3, pmax=2.0)
    assert list(oracle.durations(oracle.params(**kw))) == [3]
    assert np.array_equal(s0.sr, s1.sr) and np.array_equal(s0.j, s1.j) and np.array_equal(s0.nb, s1.nb)
    assert np.all(s1.m == 0) and np.all(s0.m[s0.j >= 0] == 3)


def test_rebin_noiseless_box_closed_form_and_decode(oracle):
    # A box covering exactly window (k*, j0) of the k*-th bin set at a grid frequency
    # is found there with SR = depth sqrt(r (1 - r)), and decodes to its own mid-time,
    # duration noverlap / (nb_k f) and depth.
    p = oracle.params(rebin=1)
    t = synth.sector_times([0], synth.CADENCE_30MIN / 4)
    f, nb0, bd = oracle.grid(t, None, 1.0, p, pmin=0.5, pmax=13.7)
    i = int(np.argmin(np.abs(1.0 / f - 3.1)))
    fi = f[i]
    g = oracle.rebin_ladder(p)
    kstar, j0, depth = 6, 11, 2e-3
    nbk = int(math.ceil(3.0 / (0.5 * oracle.qcirc(fi, 1.0) * g[kstar])))
    ph = (t - bd.t0) * fi
    ph = ph - np.floor(ph)
    b = np.minimum(nbk - 1, np.floor(ph * nbk).astype(int))
    intr = ((b - j0) % nbk) < 3
    y = np.ones_like(t)
    y[intr] -= depth
    sp = oracle.bls_star(t, y, None, 1.0, p, pmin=0.5, pmax=13.7)
    r = intr.mean()
    expect = depth * math.sqrt(r * (1 - r))
    assert abs(sp.sr[i] - expect) <= 1e-12 * expect
    assert (sp.m[i], sp.j[i], sp.nb[i]) == (kstar, j0, nbk)
    assert abs(-sp.s[i] / (sp.r[i] * (1 - sp.r[i])) - depth) <= 1e-12 * depth
    # decode through the batch driver at this frequency (the S/N picks a frequency
    # of the tie set holding the injection; check the decode wherever it lands)
    out = oracle.batch(t, y, np.ones_like(t), np.array([0, len(t)]), pmin=np.array([0.5]),
                       pmax=np.array([13.7]), p=p)
    assert np.array_equal(out["f"], sp.f)
    res = dict(zip(oracle.RESULT_FIELDS, out["results"][0]))
    ii = int(res["i_snr"])
    k_, j_, nb_ = int(out["m"][ii]), int(out["j"][ii]), int(out["nb"][ii])
    fo = out["f"][ii]
    assert abs(res["duration"] - (3.0 / nb_) / fo) <= 1e-15 * res["duration"]
    c = ((j_ + 1.5) / nb_) % 1.0
    assert abs(res["t0"] - (bd.t0 + c / fo)) <= 1e-9
    if ii == i:
        assert (k_, j_, nb_) == (kstar, j0, nbk)
        assert abs(res["depth"] - depth) <= 1e-12 * depth


def test_exact_duration_below_contact_is_clamped(oracle):
    # an explicit minimum period below a = R* (R*/a > 1 at the highest frequencies):
    # the duty cycle stops at asin(1) / pi = 1/2, never NaN, and the counts stay
    # the fewest covering bins (never more than the small-angle count)
    t = _star(span=10.0)
    p_contact = oracle.period_at_a(1.0, 1.0)
    pe = oracle.params(exact_duration=1)
    f, nb, _ = oracle.grid(t, None, 1.0, pe, pmin=0.5 * p_contact, pmax=2.0)
    fs, nbs, _ = oracle.grid(t, None, 1.0, oracle.params(), pmin=0.5 * p_contact, pmax=2.0)
    assert f[-1] > 1.0 / p_contact                      # the grid reaches below contact
    assert oracle.qcirc_exact(f[-1], 1.0) == 0.5
    assert np.all(nb >= 1) and np.all(nb <= nbs)
    qlo = np.maximum([0.5 * oracle.qcirc_exact(x, 1.0) for x in f], [0.5 * oracle.qcirc(x, 1.0) for x in f])
    assert np.all(3.0 / nb <= qlo * (1 + 1e-15))


def test_rebin_without_a_valid_window(oracle):
    # a frequency whose every bin set has at most noverlap bins (durations of a third
    # of the period or more) has no window: SR 0, k 0, j -1, nb of the k = 0 set
    b = synth.tiny(20, seed=3, span=3.0)
    t, y, w = b.star(0)
    p = oracle.params(rebin=1, qmin_fac=8.0, qmax_fac=9.0)
    sp = oracle.bls_star(t, y, w, 1.0, p, pmin=0.3, pmax=1.0)
    qlo = np.array([8.0 * oracle.qcirc(x, 1.0) for x in sp.f])
    none = np.ceil(3.0 / qlo) <= 3
    assert none.any()
    assert np.all(sp.sr[none] == 0.0) and np.all(sp.j[none] == -1) and np.all(sp.m[none] == 0)
