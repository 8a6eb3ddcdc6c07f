"""GPU parity of the two search variants (Sec. 2.1 and its footnote) against the
CPU FP64 oracle: the exact circular duration (``exact_duration``) and the
per-duration rebinning (``rebin``).  Same contract as the plain path: SR within
1e-5 relative per frequency, argmax indices equal, best windows equal except at
near-ties of the oracle's own power; integer statistics exact.
"""
import math

import numpy as np
import pytest

from paper_2302_01293_amd import synth

import parity_util as pu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _geom(oracle, okw, rho):
    """(bins, window length) of a rebinning record (m = duration index k)."""
    p = oracle.params(**okw)
    g = oracle.rebin_ladder(p)

    def geom(f, k):
        q = oracle.qcirc_exact(f, rho) if okw.get("exact_duration") else oracle.qcirc(f, rho)
        return int(math.ceil(3.0 / ((0.5 * q) * g[int(k)]))), 3
    return geom


def _batch(workload):
    if workload == "cfg0":
        return synth.config0()
    if workload == "ragged":
        return synth.ragged(4, start=40)
    if workload == "varied":
        return synth.varied_weights(2, start=3, max_sectors=3)
    raise ValueError(workload)


CASES = [("cfg0", dict(exact_duration=1)), ("ragged", dict(exact_duration=1)),
         ("cfg0", dict(rebin=1)), ("ragged", dict(rebin=1)), ("varied", dict(rebin=1)),
         ("ragged", dict(rebin=1, exact_duration=1)), ("ragged", dict(rebin=1, dip_only=1))]


@pytest.mark.parametrize("workload,kw", CASES, ids=["%s-%s" % (w, "-".join(sorted(k))) for w, k in CASES])
def test_variant_parity(oracle, workload, kw):
    from paper_2302_01293_amd import _lib
    b = _batch(workload)
    _say("case variant parity:", workload, kw, "points", np.diff(b.offsets).tolist())
    ds = pu.fetch(pu.run_gpu(b, _lib.default_params(**kw)))
    orc = pu.run_oracle(oracle, b, okw=kw)
    worst = 0.0
    for s in range(b.n_stars):
        rho = float(b.rho[s]) if b.rho is not None else 1.0
        rho = 1.0 if not (rho > 0) else rho
        geom = _geom(oracle, kw, rho) if kw.get("rebin") else None
        st = pu.compare_star(ds, orc, s, s, b.star(s), "%s%s[%d]" % (workload, kw, s), geom=geom)
        worst = max(worst, st["max_rel_sr"])
    _say("variant", kw, workload, "max rel SR err", worst)


def test_rebin_wide_bin_sets_in_passes(oracle):
    # A dense star searched out to 300 d: the k = 0..2 bin sets hold more than 4096
    # bins (searched in passes over start-bin ranges), k >= 3 fit in one pass.
    import torch
    from paper_2302_01293_amd import _lib
    from paper_2302_01293_amd.device import DeviceSearch
    rng = np.random.default_rng(17)
    t = synth.sector_times([0, 1], synth.CADENCE_30MIN)
    y = 1.0 + rng.normal(0.0, 1e-3, len(t))
    y[synth.box_mask(t, 7.3, t[0] + 1.1, 0.2)] -= 3e-3
    w = np.full(len(t), 1e6)
    b = synth._pack([t], [y], [w], [3.0], [0.0], [300.0], {})
    kw = dict(rebin=1)
    p = oracle.params(**kw)
    idx = np.arange(6)
    o = oracle.bls_star_at(t, y, w, idx, 3.0, p, pmax=300.0)
    assert int(math.ceil(3.0 / (0.5 * oracle.qcirc(o.f[0], 3.0) * oracle.rebin_ladder(p)[2]))) > 4096
    ds = DeviceSearch.from_batch(b, _lib.default_params(**kw))
    win = torch.tensor([[0, 0, 6]], dtype=torch.int64, device="cuda")
    ds.sr.zero_()
    ds.run_prepare()
    ds.run_search(windows=win)
    torch.cuda.synchronize()
    sr = ds.sr_host()[:6]
    bb = ds.best_host()[:6]
    _say("case rebin passes: nb0 of the k=0 set", int(math.ceil(3.0 / (0.5 * oracle.qcirc(o.f[0], 3.0)))),
         "SR gpu", sr.tolist(), "oracle", o.sr.tolist())
    np.testing.assert_allclose(sr, o.sr, rtol=pu.EXACT_SR_RTOL, atol=0)
    geom = _geom(oracle, kw, 3.0)
    for i in range(6):
        if (bb["m"][i], bb["j"][i]) != (o.m[i], o.j[i]):
            nbg, _ = geom(o.f[i], bb["m"][i])
            pg = pu.window_power(t, y, w, t[0], o.f[i], nbg, 3, bb["j"][i])
            po = pu.window_power(t, y, w, t[0], o.f[i], int(o.nb[i]), 3, o.j[i])
            assert abs(pg - po) <= pu.NEAR_TIE_RTOL * po, (i, bb[i], o.m[i], o.j[i])


def test_rebin_windows_equal_the_full_search(oracle):
    import torch
    from paper_2302_01293_amd import _lib
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.ragged(3, start=7)
    prm = _lib.default_params(rebin=1)
    full = pu.fetch(pu.run_gpu(b, prm))
    ds = DeviceSearch.from_batch(b, prm)
    fo = ds.plan.freq_offsets
    wl = [[s, 5, min(40, int(fo[s + 1] - fo[s]))] for s in range(b.n_stars)]
    ds.sr.fill_(-1.0)
    ds.run_prepare()
    ds.run_search(windows=torch.tensor(wl, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    sr = ds.sr_host()
    bw = ds.best_host()
    for s, i0, i1 in wl:
        a, z = int(fo[s]) + i0, int(fo[s]) + i1
        assert np.array_equal(sr[a:z], full._sr_host[a:z])
        assert np.array_equal(bw[a:z], full._best_host[a:z])
        assert np.all(sr[int(fo[s]):a] == -1.0)


def test_rebin_stats_at_the_detection(oracle):
    from paper_2302_01293_amd import _lib
    b = synth.ragged(4, start=40)
    kw = dict(rebin=1)
    ds = pu.fetch(pu.run_gpu(b, _lib.default_params(**kw)))
    ds.run_stats()
    st = ds.stats_host()
    orc = pu.run_oracle(oracle, b, okw=kw)
    for s in range(b.n_stars):
        t, y, w = b.star(s)
        R = orc["results"][s]
        i = int(R[0])
        o0 = int(orc["fofs"][s])
        assert int(ds._res_host[s]["i_snr"]) == i
        assert (int(ds._best_host[o0 + i]["m"]), int(ds._best_host[o0 + i]["j"])) == \
            (int(orc["m"][o0 + i]), int(orc["j"][o0 + i]))
        t0 = t[np.nonzero(w > 0)[0][0]]
        o = oracle.stats(t, y, w, t0, orc["f"][o0 + i], int(orc["nb"][o0 + i]), 3, int(orc["j"][o0 + i]), R[7])
        got = {k: int(st[s][k]) for k in ("n_in", "n_before", "n_after", "n_transits", "candidate")}
        _say("rebin stats star", s, got)
        for k in got:
            assert got[k] == o[k], (s, k, got[k], o[k])


@pytest.mark.parametrize("case", ["exact_below_contact", "rebin_no_window"])
def test_variant_edges(oracle, case):
    """Periods below contact with the exact duration (the arcsine argument clamped at
    1), and rebinning durations so long that some frequencies have no valid window."""
    from paper_2302_01293_amd import _lib
    b = synth.tiny(400, seed=11, span=6.0)
    if case == "exact_below_contact":
        kw, okw = dict(exact_duration=1), dict(exact_duration=1)
        b.pmin[:] = 0.5 * oracle.period_at_a(1.0, 1.0)
        b.pmax[:] = 2.0
    else:
        kw = okw = dict(rebin=1, qmin_fac=8.0, qmax_fac=9.0)
        b.pmin[:] = 0.3
        b.pmax[:] = 2.0
    _say("case variant edge:", case, "points", b.n_points)
    ds = pu.fetch(pu.run_gpu(b, _lib.default_params(**kw)))
    orc = pu.run_oracle(oracle, b, okw=okw)
    geom = None
    if okw.get("rebin"):
        g = oracle.rebin_ladder(oracle.params(**okw))

        def geom(f, k):  # bins of set k with qmin_fac = 8
            return int(math.ceil(3.0 / ((8.0 * oracle.qcirc(f, 1.0)) * g[int(k)]))), 3
    st = pu.compare_star(ds, orc, 0, 0, b.star(0), case, geom=geom)
    if case == "rebin_no_window":
        assert np.any(ds._best_host["j"] == -1) and np.all(ds._sr_host[ds._best_host["j"] == -1] == 0.0)
    _say(case, "max rel SR err", st["max_rel_sr"])
