"""GPU tests of the batching layer: HIP-graph capture and replay, restricted
frequency ranges (work lists of (star, i0, i1)), and the largest fine-bin count the
search kernel accepts."""
import numpy as np
import pytest

from paper_2302_01293_amd import synth

import parity_util as pu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_graph_replay_matches_eager():
    import torch
    b = synth.ragged(6, start=60)
    _say("case graph replay: 6 ragged stars")
    ds = pu.run_gpu(b)
    sr_e = ds.sr_host()
    res_e = ds.result.cpu().numpy().copy()
    snr_e = ds.snr_host()
    g = ds.capture()
    torch.cuda.synchronize()
    other = pu.run_gpu(synth.ragged(2, start=70))  # unrelated eager work between replays
    for rep in range(3):
        ds.sr.zero_()
        ds.snr.zero_()
        ds.result.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(ds.sr_host().view(np.uint64), sr_e.view(np.uint64)), rep
        assert np.array_equal(ds.snr_host().view(np.uint64), snr_e.view(np.uint64)), rep
        assert np.array_equal(ds.result.cpu().numpy(), res_e), rep
        other.run()
        torch.cuda.synchronize()


def test_pipeline_graph_with_copies_matches_eager():
    """H2D copies -> prepare -> search -> S/N -> D2H copy captured as one graph and
    replayed for three different flux vectors of the same stars (eager work and
    synchronisations between the replays): each replay's results equal an eager run
    of the same data."""
    import torch
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.ragged(6, start=75)
    _say("case pipeline graph: 6 ragged stars, three flux vectors")
    ds = DeviceSearch.from_batch(b)
    ds.run()
    torch.cuda.synchronize()
    pipe = ds.capture_pipeline()
    rng = np.random.default_rng(3)
    other = pu.run_gpu(synth.ragged(2, start=70))
    for rep in range(3):
        y = b.y + rng.normal(0, 5e-4, len(b.y))
        if rep == 1:
            y[(b.t - b.t[0]) % 2.7 < 0.1] -= 4e-3     # a planted dip in every star
        pipe.y_host.numpy()[...] = y
        pipe.replay()
        got = pipe.results()
        eager = DeviceSearch(b.t, y, b.w, b.offsets, b.rho, b.pmin, b.pmax)
        eager.run()
        torch.cuda.synchronize()
        exp = eager.results_host()
        assert np.array_equal(got.view(np.uint8), exp.view(np.uint8)), rep
        _say("replay", rep, "best periods", np.round(got["period"], 4).tolist())
        other.run()
        torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["equal", "mixed"])
def test_windows_match_full_grid(kind):
    """Caller windows give the full search's results bit for bit on the frequencies
    they cover and leave the rest untouched; "mixed" holds stars of equal weights
    (counts of weighted points) and of varied weights (weight prefixes), so both
    exact launches serve the windows."""
    import torch
    if kind == "equal":
        b = synth.ragged(5, start=80)
    else:
        b = synth.concat([synth.ragged(3, start=80), synth.varied_weights(2, start=4, max_sectors=2)])
    _say("case windows (%s weights): 5 stars" % kind)
    ds = pu.run_gpu(b)
    full = ds.sr_host()
    best_full = ds.best_host().copy()
    nfs = np.diff(ds.plan.freq_offsets)
    rng = np.random.default_rng(5)
    tri = []
    for s in range(b.n_stars):
        for _ in range(3):
            i0 = int(rng.integers(0, nfs[s]))
            i1 = int(min(nfs[s], i0 + rng.integers(1, 700)))
            tri.append((s, i0, i1))
    tri.append((0, 5, 5))                      # empty range
    tri.append((1, nfs[1] - 3, nfs[1] + 50))   # clipped at the end of the grid
    tri.append((2, -10, 7))                    # clipped at the start
    tri.append((99, 0, 10))                    # no such star: skipped
    tri.append((-1, 0, 10))
    wins = torch.tensor(np.array(tri, np.int64), device="cuda")
    ds.sr.fill_(-1.0)
    ds.run_search(windows=wins)
    torch.cuda.synchronize()
    part = ds.sr_host()
    best_part = ds.best_host()
    covered = np.zeros(len(full), bool)
    for s, i0, i1 in tri:
        if not 0 <= s < b.n_stars:
            continue
        i0, i1 = max(0, i0), min(nfs[s], i1)
        if i1 > i0:
            covered[ds.plan.freq_offsets[s] + i0: ds.plan.freq_offsets[s] + i1] = True
    assert np.array_equal(part[covered].view(np.uint64), full[covered].view(np.uint64))
    assert np.array_equal(best_part[covered], best_full[covered])
    assert np.all(part[~covered] == -1.0)
    # an empty work list launches nothing and leaves the outputs alone
    ds.run_search(windows=torch.zeros((0, 3), dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    assert np.array_equal(ds.sr_host().view(np.uint64), part.view(np.uint64))


@pytest.mark.parametrize("pmax, nb_lo, nb_hi", [(236.0, 3000, 3040), (350.0, 3900, 4000)])
def test_largest_bin_count(oracle, pmax, nb_lo, nb_hi):
    # a two-year baseline at 12-h cadence searched from 50 d: up to 236 d the first
    # frequency has just under 3040 fine bins, the most one pass over the 48 KB
    # accumulator window holds; up to 350 d ~3940, searched in passes
    t = np.concatenate([synth.sector_times([s], 0.5) for s in range(26)])
    rng = np.random.default_rng(9)
    y = 1.0 + rng.normal(0, 1e-3, len(t))
    w = np.full(len(t), 1e6)
    b = synth.Batch(t, y, w, np.array([0, len(t)]), np.array([1.0]), np.array([50.0]), np.array([pmax]))
    ds = pu.fetch(pu.run_gpu(b))
    f, nb = ds.plan.frequencies(0)
    _say("case largest nb: points", len(t), "nb0", int(nb[0]), "frequencies", len(f))
    from paper_2302_01293_amd import _lib
    assert nb_lo <= nb[0] <= min(nb_hi, _lib.limits()["nb_max"])
    orc = pu.run_oracle(oracle, b)
    pu.compare_star(ds, orc, 0, 0, b.star(0), "largest-nb")


def test_autotune_picks_a_candidate_and_results_do_not_change(tmp_path):
    import torch
    from paper_2302_01293_amd import autotune, _lib
    b = synth.ragged(8, start=90)
    _say("case autotune: 8 ragged stars")
    cands = (1 << 18, 1 << 21, 1 << 24)
    out = autotune.tune(b, candidates=cands, n_sample=8, reps=2, cache_path=str(tmp_path / "tune.json"))
    assert out["tile_cells"] in cands + (0,) and not out["cached"]   # 0: the default, also timed
    again = autotune.tune(b, candidates=cands, n_sample=8, reps=2, cache_path=str(tmp_path / "tune.json"))
    assert again["cached"] and again["tile_cells"] == out["tile_cells"]
    ref = pu.run_gpu(b)
    for c in cands:
        ds = pu.run_gpu(b, _lib.default_params(tile_cells=c))
        assert np.array_equal(ds.sr_host().view(np.uint64), ref.sr_host().view(np.uint64)), c
        assert np.array_equal(ds.results_host(), ref.results_host()), c


def test_autotune_three_axes_results_do_not_change(tmp_path):
    """Coordinate descent over the work-item size, the per-item frequency cap and the
    point count above which a star takes the large workgroup shape, on stars of 1-13
    sectors (some above 50,000 points): every candidate gives bit-identical spectra,
    best windows and results."""
    import torch
    from paper_2302_01293_amd import autotune, _lib
    b = synth.config2(12, start=500)
    pts = np.diff(b.offsets)
    _say("case autotune, three axes: points per star", pts.tolist())
    assert pts.max() > 50_000
    out = autotune.tune(b, candidates=(1 << 20, 6 << 20), n_sample=12, reps=1, cache_path=str(tmp_path / "t.json"),
                        axes=("tile_cells", "item_freqs", "big_points"), item_freqs=(64, 512),
                        big_points=(50_000, 1 << 40))
    _say("picks", {k: out[k] for k in ("tile_cells", "item_freqs", "big_points")})
    assert out["item_freqs"] in (0, 64, 512) and out["big_points"] in (0, 50_000, 1 << 40)
    ref = pu.run_gpu(b)
    for kw in (dict(item_freqs=64), dict(item_freqs=512), dict(big_points=50_000), dict(big_points=1 << 40),
               dict(tile_cells=1 << 20, item_freqs=4096, big_points=30_000)):
        ds = pu.run_gpu(b, _lib.default_params(**kw))
        assert np.array_equal(ds.sr_host().view(np.uint64), ref.sr_host().view(np.uint64)), kw
        assert np.array_equal(ds.best_host(), ref.best_host()), kw
        assert np.array_equal(ds.results_host(), ref.results_host()), kw


@pytest.mark.parametrize("precision", [0, 1])
def test_wide_bin_counts_in_passes(oracle, precision):
    # a dense star (rho = 10^1.5) over 26 sectors at 2-h cadence searched between
    # 300 and 350 d: ~12,000 fine bins, three passes over bin ranges per frequency
    from paper_2302_01293_amd import _lib
    t = np.concatenate([synth.sector_times([s], 1.0 / 12) for s in range(26)])
    rng = np.random.default_rng(21)
    y = 1.0 + rng.normal(0, 1e-3, len(t))
    y[((t - t[0]) % 317.0) < 0.6] -= 3e-3
    w = np.full(len(t), 1e6)
    b = synth.Batch(t, y, w, np.array([0, len(t)]), np.array([10 ** 1.5]), np.array([300.0]), np.array([350.0]))
    ds = pu.fetch(pu.run_gpu(b, _lib.default_params(precision=precision)))
    f, nb = ds.plan.frequencies(0)
    _say("case wide nb: points", len(t), "nb", int(nb[0]), "..", int(nb[-1]), "frequencies", len(f),
         "precision", precision)
    assert nb[-1] > 2 * 4096
    orc = pu.run_oracle(oracle, b)
    if precision == 0:
        pu.compare_star(ds, orc, 0, 0, b.star(0), "wide-nb")
    else:
        sr_o = orc["sr"]
        rel = np.abs(ds._sr_host - sr_o) / np.maximum(np.abs(sr_o), 1e-300)
        _say("wide packed max rel SR err %.3e" % rel.max())
        assert rel.max() <= 1e-5
        assert int(ds._res_host["i_snr"][0]) == int(orc["results"][0][0])


def test_streamed_batches_match_single_runs():
    # double-buffered stream of three batches: results equal those of each batch
    # searched on its own
    from paper_2302_01293_amd import stream
    batches = [synth.ragged(4, start=200 + 10 * i) for i in range(3)]
    res, stats = stream.run_stream(batches)
    _say("stream stats", stats)
    assert len(res) == 3 and stats["stars"] == 12
    for b, r in zip(batches, res):
        ref = pu.run_gpu(b).results_host()
        assert np.array_equal(r["i_snr"], ref["i_snr"])
        assert np.array_equal(r["snr"].view(np.uint64), ref["snr"].view(np.uint64))


@pytest.mark.parametrize("sectors, precision", [(3, 0), (3, 1), (9, 0), (9, 1)])
def test_large_shape_bin_counts(oracle, sectors, precision):
    # sectors at 200 s of a dense star (rho = 12) searched between 60 and 80 d: the
    # first frequencies have 3040-3370 fine bins, the rest fewer; few gap points
    # (telescoping form).  Three sectors (34,215 points): the large workgroup shape
    # takes the frequencies above 3040 bins, the common shape the rest; nine sectors
    # (102,645 points, a long star): the large shape takes every frequency.
    from paper_2302_01293_amd import _lib
    t = synth.sector_times(list(range(sectors)), synth.CADENCE_200S)
    rng = np.random.default_rng(31)
    y = 1.0 + rng.normal(0, 1e-3, len(t))
    y[((t - t[0]) % 71.3) < 0.4] -= 2e-3
    w = np.full(len(t), 1e6)
    b = synth.Batch(t, y, w, np.array([0, len(t)]), np.array([12.0]), np.array([60.0]), np.array([80.0]))
    ds = pu.fetch(pu.run_gpu(b, _lib.default_params(precision=precision)))
    f, nb = ds.plan.frequencies(0)
    _say("case large shape: sectors", sectors, "points", len(t), "nb", int(nb[0]), "..", int(nb[-1]),
         "frequencies", len(f), "precision", precision)
    assert nb[0] > 3040 >= nb[-1]
    orc = pu.run_oracle(oracle, b)
    if precision == 0:
        pu.compare_star(ds, orc, 0, 0, b.star(0), "large-shape")
    else:
        rel = np.abs(ds._sr_host - orc["sr"]) / np.maximum(np.abs(orc["sr"]), 1e-300)
        _say("large shape packed max rel SR err %.3e" % rel.max())
        assert rel.max() <= pu.SR_RTOL
