"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library loads and exports every symbol declared in include/mi355bls.h;
* the plan's grid (f_i, nb_i), period bounds and duration ladder are bit-identical
  to the oracle's own (independently written) computation;
* invalid inputs give the documented status codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2302_01293_amd import _lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in ("mi355bls.h", "mi355pp.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b((?:bls|pp)_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_matches_binding():
    assert set(_declared_functions()) == set(_lib.EXPORTS)


def test_library_exports_every_symbol():
    L = _lib.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_status_strings():
    L = _lib.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.bls_status_string(code)


def _plan_for(batch, **pk):
    return _lib.Plan(batch.t, batch.y, batch.w, batch.offsets, batch.rho, batch.pmin, batch.pmax,
                     _lib.default_params(**pk))


@pytest.mark.parametrize("which", ["cfg0", "ragged"])
def test_grid_bit_identical_to_oracle(oracle, which):
    b = synth.config0() if which == "cfg0" else synth.ragged(10, start=0)
    plan = _plan_for(b)
    for s in range(b.n_stars):
        t, y, w = b.star(s)
        f_o, nb_o, bd = oracle.grid(t, w, float(b.rho[s]), oracle.params(), float(b.pmin[s]), float(b.pmax[s]))
        f_p, nb_p = plan.frequencies(s)
        assert f_p.dtype == np.float64 and len(f_p) == len(f_o)
        assert np.array_equal(f_p.view(np.uint64), f_o.view(np.uint64))
        assert np.array_equal(nb_p, nb_o)
        info = plan.star_info(s)
        assert info["t0"] == bd.t0 and info["T"] == bd.T
        assert info["pmin"] == bd.pmin and info["pmax"] == bd.pmax
        assert info["umin"] == bd.umin and info["A"] == bd.A
        assert info["sturges"] == oracle.sturges(len(f_o))
    assert plan.n_freq == sum(int(plan.freq_offsets[s + 1] - plan.freq_offsets[s]) for s in range(b.n_stars))


def test_durations_match_oracle(oracle):
    b = synth.config0()
    for kw in ({}, {"dlogq": 0.05}, {"noverlap": 4}, {"qmax_fac": 1.5}):
        plan = _plan_for(b, **kw)
        assert list(plan.durations()) == list(oracle.durations(oracle.params(**kw)))


def test_a_min_three(oracle):
    b = synth.ragged(3, start=1)
    plan = _plan_for(b, a_min_rstar=3.0)
    for s in range(b.n_stars):
        t, y, w = b.star(s)
        _, bd = oracle.bounds(t, w, float(b.rho[s]), oracle.params(a_min=3.0))
        assert plan.star_info(s)["pmin"] == bd.pmin


def _raises(code, **mut):
    b = synth.ragged(2, start=0)
    t, y, w = b.t.copy(), b.y.copy(), b.w.copy()
    rho, pmin, pmax = b.rho.copy(), b.pmin.copy(), b.pmax.copy()
    loc = dict(t=t, y=y, w=w, rho=rho, pmin=pmin, pmax=pmax)
    for k, fn in mut.items():
        fn(loc[k])
    with pytest.raises(_lib.BlsError) as e:
        _lib.Plan(t, y, w, b.offsets, rho, pmin, pmax)
    assert e.value.code == code


def test_invalid_inputs():
    _raises(-2, t=lambda a: a.__setitem__(3, np.nan))
    _raises(-2, y=lambda a: a.__setitem__(5, np.inf))
    _raises(-2, w=lambda a: a.__setitem__(7, -1.0))
    _raises(-2, t=lambda a: a.__setitem__(10, a[9] - 1.0))        # not ascending
    _raises(-2, w=lambda a: a.__setitem__(slice(None), 0.0))      # no weight
    _raises(-3, pmin=lambda a: a.__setitem__(0, 50.0))           # Pmin >= Pmax


def test_first_failing_star_reported_from_threaded_plan():
    """The per-star checks run on host threads for batches of more than 2^20 points;
    the error returned is still that of the first failing star, whatever finishes
    first, and a valid batch gives the same plan as its stars planned one by one."""
    b = synth.concat([synth.config4(6, start=20), synth.config1(4, start=3)])
    assert b.n_points > (1 << 20)
    offs = b.offsets
    t = b.t.copy()
    t[offs[7] + 3] = t[offs[7] + 2] - 1.0      # star 7: times not sorted
    t[offs[2] + 10] = np.nan                    # star 2: non-finite time
    with pytest.raises(_lib.BlsError) as e:
        _lib.Plan(t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax)
    assert e.value.code == -2 and e.value.star == 2
    t = b.t.copy()
    t[offs[7] + 3] = t[offs[7] + 2] - 1.0
    with pytest.raises(_lib.BlsError) as e:
        _lib.Plan(t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax)
    assert e.value.star == 7
    whole = _lib.Plan(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax)
    nf = np.diff(whole.freq_offsets)
    for s in range(b.n_stars):
        one = b.subset([s])
        p1 = _lib.Plan(one.t, one.y, one.w, one.offsets, one.rho, one.pmin, one.pmax)
        assert p1.n_freq == nf[s]
        assert whole.star_info(s) == p1.star_info(0)


def test_zero_weight_points_excluded_from_baseline(oracle):
    b = synth.ragged(1, start=2)
    t, y, w = b.star(0)
    w = w.copy()
    w[:30] = 0.0
    w[-10:] = 0.0
    plan = _lib.Plan(t, y, w, np.array([0, len(t)]), b.rho[:1])
    _, bd = oracle.bounds(t, w, float(b.rho[0]), oracle.params())
    info = plan.star_info(0)
    assert info["t0"] == t[30] == bd.t0 and info["T"] == bd.T


def test_limits():
    lim = _lib.limits()
    # 26-sector baselines at solar density reach ~4000 fine bins
    assert lim["nb_max"] >= 4000 and lim["m_max"] >= 12


def test_wide_bin_counts_accepted():
    # a two-year baseline up to 400 d at solar density needs ~4300 fine bins: more
    # than the common workgroup shape holds (the large shape searches them)
    t = np.concatenate([synth.sector_times([s], 0.5) for s in range(26)])
    y = np.ones_like(t)
    plan = _lib.Plan(t, y, np.ones_like(t), np.array([0, len(t)]), np.array([1.0]), np.array([50.0]),
                     np.array([400.0]))
    f, nb = plan.frequencies(0)
    assert nb[0] > 4064 and nb[0] <= _lib.limits()["nb_max"]


def test_limits_cover_dense_stars_on_long_baselines():
    # rho = 10^1.5 and Pmax = 356 d need ~12,600 fine bins
    assert _lib.limits()["nb_max"] >= 13000


def test_tile_size_changes_only_the_work_list():
    b = synth.ragged(4, start=3)
    small = _plan_for(b, tile_cells=1 << 18)
    big = _plan_for(b, tile_cells=1 << 26)
    assert small.workspace_bytes > big.workspace_bytes  # more work items
    for s in range(b.n_stars):
        fa, na = small.frequencies(s)
        fb, nbb = big.frequencies(s)
        assert np.array_equal(fa, fb) and np.array_equal(na, nbb)


def test_autotune_cache_and_sampling(tmp_path):
    from paper_2302_01293_amd import autotune
    pts = np.array([100, 5000, 20000, 150000, 12000] * 100)
    idx = autotune.sample_stars(pts, 16)
    assert len(idx) <= 16 and pts[idx].min() == pts.min() and pts[idx].max() == pts.max()
    k1 = autotune.shape_key("gfx950", pts)
    assert k1 == autotune.shape_key("gfx950", pts[::-1].copy())
    path = str(tmp_path / "t.json")
    assert autotune.load_cache(path) == {}
    autotune.save_cache(path, {k1: {"tile_cells": 123}})
    assert autotune.load_cache(path)[k1]["tile_cells"] == 123


def test_concat_keeps_stars_and_common_truth():
    from paper_2302_01293_amd import synth
    a = synth.config3(5, start=0, max_sectors=2)
    b = synth.config1(3, start=100_000)
    c = synth.concat([a, b])
    assert c.n_stars == 8 and c.n_points == a.n_points + b.n_points
    for s in range(5):
        assert all(np.array_equal(u, v) for u, v in zip(c.star(s), a.star(s)))
    for s in range(3):
        assert all(np.array_equal(u, v) for u, v in zip(c.star(5 + s), b.star(s)))
    assert set(c.truth) == set(a.truth) & set(b.truth)
    assert np.array_equal(c.truth["period"][5:], b.truth["period"], equal_nan=True)


def test_noalloc_rejects_plan_larger_than_scratch():
    """bls_run_noalloc refuses a plan whose workspace exceeds its static scratch
    before it touches any pointer or the device (host check, no GPU needed)."""
    from paper_2302_01293_amd import _lib, synth
    b = synth.config1(300, start=0)          # 300 x 11,405 points x 24 B > 64 MiB
    pl = _lib.Plan(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax)
    assert pl.workspace_bytes > _lib.NOALLOC_SCRATCH_BYTES
    with pytest.raises(_lib.BlsError) as e:
        pl.run_noalloc(1, 1, None, 1, None, None, 1)
    assert e.value.code == -8
    assert _lib.lib().bls_status_string(-8).startswith(b"workspace larger")


@pytest.mark.parametrize("which", ["cfg0", "ragged"])
def test_exact_duration_bins_identical_to_oracle(oracle, which):
    # the host evaluates the exact duty cycle with the same libm asin as the oracle
    b = synth.config0() if which == "cfg0" else synth.ragged(6, start=3)
    plan = _plan_for(b, exact_duration=1)
    small = _plan_for(b)
    for s in range(b.n_stars):
        t, y, w = b.star(s)
        f_o, nb_o, _ = oracle.grid(t, w, float(b.rho[s]), oracle.params(exact_duration=1),
                                   float(b.pmin[s]), float(b.pmax[s]))
        f_p, nb_p = plan.frequencies(s)
        assert np.array_equal(f_p.view(np.uint64), f_o.view(np.uint64))
        assert np.array_equal(nb_p, nb_o)
        assert np.all(nb_p <= small.frequencies(s)[1])


def test_variant_parameters_checked():
    b = synth.ragged(2, start=0)
    for bad in (dict(rebin=1, precision=1), dict(rebin=1, dlogq=0.01)):   # packed sums; > 32 durations
        with pytest.raises(_lib.BlsError) as e:
            _plan_for(b, **bad)
        assert e.value.code == -7
    for bad in (dict(rebin=2), dict(exact_duration=-1)):
        with pytest.raises(_lib.BlsError) as e:
            _plan_for(b, **bad)
        assert e.value.code == -1
