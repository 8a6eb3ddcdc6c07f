"""GPU parity of the learned period proposal (HIP kernels through the C ABI) against
the CPU FP64 oracle ``oracle/pp_oracle.py``, plus the end-to-end learned path.

Tolerances: the GPU accumulates the two convolutions in FP32 on the matrix cores and
rounds their outputs to BF16, the oracle accumulates in FP64 and rounds at the same
points; an activation whose FP32 and FP64 values straddle a BF16 rounding boundary
differs by one BF16 step (a few in 10^4 of the activations), so activations are
compared by the fraction of exact BF16 matches and the downstream values with a
relative tolerance of a few 10^-3.  Integer outputs (windows, fallback flags,
indices) are compared exactly, range ends within one grid index (the cube root of
the host library and of the device may differ in the last bit).
"""
import os

import numpy as np
import pytest

from oracle import pp_oracle as P
from paper_2302_01293_amd import synth

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(*a):
    print(*a, flush=True)


def _bits_to_f(bits):
    return (np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _rand_inputs(B, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((B, 2, P.L0))
    for b in range(B):
        cov = (rng.uniform(size=P.L0) < 0.85).astype(float)
        sig = rng.normal(0, 1, P.L0) * cov
        per = rng.uniform(20, 300)
        sig[(np.arange(P.L0) % int(per)) < 3] -= 4.0
        X[b, 0] = P.bf16(sig * cov)
        X[b, 1] = cov
    lag = rng.uniform(0.02, 0.2, B)
    theta = synth.pp_init_params(seed).astype(np.float64)
    theta[P.OFF["beta"][0]:P.OFF["beta"][1]] = rng.normal(0, 0.3, P.NPB)
    theta[P.OFF["b1"][0]:P.OFF["b1"][1]] = rng.normal(0, 0.2, P.C1)
    theta[P.OFF["b2"][0]:P.OFF["b2"][1]] = rng.normal(0, 0.2, P.C2)
    theta[P.OFF["delta"][0]] = 0.7
    return X, lag, theta.astype(np.float32).astype(np.float64)


def _device_inputs(X, lag, theta):
    import torch
    xb = P.bf16_bits(X.reshape(len(X), -1)).reshape(X.shape).view(np.int16)
    return (torch.as_tensor(xb.copy()).cuda(), torch.as_tensor(lag.copy()).cuda(),
            torch.as_tensor(theta.astype(np.float32)).cuda())


def test_resample_parity():
    import torch
    from paper_2302_01293_amd import learned
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.ragged(6, start=120, cadence=synth.CADENCE_200S * 3)
    w = b.w.copy()
    w[np.random.default_rng(1).uniform(size=len(w)) < 0.05] = 0.0
    b.w = w
    _say("case resample: 6 ragged stars, points", np.diff(b.offsets).tolist())
    ds = DeviceSearch.from_batch(b)
    x, lag = learned.resample(ds)
    torch.cuda.synchronize()
    xg = x.cpu().numpy().view(np.uint16)
    lg = lag.cpu().numpy()
    for s in range(b.n_stars):
        t, y, ww = b.star(s)
        Xo, lo = P.resample(t, y, ww)
        bits_o = P.bf16_bits(Xo)
        assert lg[s] == lo
        assert np.array_equal(xg[s, 1], bits_o[1])
        same = np.mean(xg[s, 0] == bits_o[0])
        assert same >= 0.999, (s, same)
        np.testing.assert_allclose(_bits_to_f(xg[s, 0]), Xo[0], rtol=2 ** -7, atol=1e-30)


def test_forward_parity():
    import torch
    from paper_2302_01293_amd import _lib
    B = 4
    X, lag, theta = _rand_inputs(B, 11)
    xd, ld, td = _device_inputs(X, lag, theta)
    logits = torch.empty((B, P.NPB + 1), dtype=torch.float32, device="cuda")
    act = torch.empty(B * _lib.PP_ACT_BYTES_PER_STAR, dtype=torch.uint8, device="cuda")
    _lib.check("pp_forward", _lib.lib().pp_forward(td.data_ptr(), xd.data_ptr(), ld.data_ptr(), B,
                                                   logits.data_ptr(), act.data_ptr(), 0))
    torch.cuda.synchronize()
    lg = logits.cpu().numpy().astype(np.float64)
    ab = act.cpu().numpy().reshape(B, -1)
    for b in range(B):
        zo, c = P.forward(X[b], theta, lag[b])
        a1 = ab[b, :65536].view(np.uint16).reshape(16, 2048)
        a2 = ab[b, 65536:98304].view(np.uint16).reshape(16, 1024)
        sg = ab[b, 98304:102400].view(np.float32).astype(np.float64)
        Ag = ab[b, 102400:106496].view(np.float32).astype(np.float64)
        m1 = np.mean(a1 == P.bf16_bits(c["a1"]))
        m2 = np.mean(a2 == P.bf16_bits(c["a2"]))
        _say("star", b, "a1 match %.5f a2 match %.5f" % (m1, m2))
        assert m1 >= 0.995 and m2 >= 0.995
        scale = np.max(np.abs(c["sh"]))
        assert np.max(np.abs(sg - c["sh"])) <= 5e-3 * scale
        assert np.max(np.abs(Ag - c["A"])) <= 5e-3 * abs(c["A"][0])
        assert np.max(np.abs(lg[b] - zo)) <= 5e-3 * max(1.0, np.max(np.abs(zo)))


def test_backward_parity():
    import torch
    from paper_2302_01293_amd import _lib, learned
    B = 4
    X, lag, theta = _rand_inputs(B, 12)
    labels = np.array([100, -1, 300, 7])
    xd, ld, td = _device_inputs(X, lag, theta)
    net = learned.ProposalNet(theta.astype(np.float32))
    tgt = torch.as_tensor(learned.soft_targets(labels)).cuda()
    net.gradient(xd, ld, tgt)
    torch.cuda.synchronize()
    g = net.grad.cpu().numpy().astype(np.float64)
    loss = float(net.loss.cpu().numpy()[0])
    lo, go = P.loss_and_grad(list(X), theta, list(lag), list(labels))
    _say("loss gpu %.6f oracle %.6f" % (loss, lo))
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    for name, (a, b_) in P.OFF.items():
        ga, gb = g[a:b_], go[a:b_]
        scale = max(float(np.max(np.abs(gb))), 1e-12)
        err = np.abs(ga - gb) / scale
        _say("grad %-5s element-wise: max |gpu - oracle| / max|oracle| %.2e, elements above 1e-5: %d of %d"
             % (name, err.max(), int(np.sum(err > 1e-5)), len(err)))
        # every element, not a norm: a wrong tap anywhere in a group fails (observed
        # at most 1.3e-6: FP32 accumulation of the backward against FP64, with the
        # BF16 activations rounded the same way on both sides)
        assert err.max() <= 1e-5, name
    # deterministic: same gradient bits on a second evaluation
    g1 = net.grad.clone()
    net.gradient(xd, ld, tgt)
    torch.cuda.synchronize()
    assert torch.equal(g1, net.grad)


def test_adam_parity():
    import torch
    from paper_2302_01293_amd import _lib
    rng = np.random.default_rng(13)
    th = rng.normal(size=P.NPARAM).astype(np.float32)
    m = np.zeros(P.NPARAM)
    v = np.zeros(P.NPARAM)
    td = torch.as_tensor(th.copy()).cuda()
    md = torch.zeros(P.NPARAM, dtype=torch.float32, device="cuda")
    vd = torch.zeros_like(md)
    tho = th.astype(np.float64)
    for step in range(1, 4):
        g = rng.normal(size=P.NPARAM).astype(np.float32)
        gd = torch.as_tensor(g).cuda()
        _lib.check("pp_adam", _lib.lib().pp_adam(td.data_ptr(), md.data_ptr(), vd.data_ptr(), gd.data_ptr(),
                                                 step, 1e-2, 0))
        tho, m, v = P.adam(tho, m, v, g.astype(np.float64), step, 1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(td.cpu().numpy(), tho, rtol=1e-5, atol=1e-6)


def _oracle_grid(oracle, b, s, spp=2.0):
    t, y, w = b.star(s)
    f, nb, bd = oracle.grid(t, w, float(b.rho[s]), oracle.params(spp=spp), float(b.pmin[s]), float(b.pmax[s]))
    return f, bd


def test_propose_parity(oracle):
    import torch
    from paper_2302_01293_amd import _lib
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.ragged(8, start=140, max_sectors=13)
    ds = DeviceSearch.from_batch(b)
    S = b.n_stars
    rng = np.random.default_rng(14)
    z = rng.normal(0, 1, (S, P.NPB + 1))
    for s in range(S):
        if s % 3 != 2:      # confident: a few sharp peaks
            for k in rng.choice(P.NPB, 3, replace=False):
                z[s, k] += 14.0
    z = z.astype(np.float32)
    zd = torch.as_tensor(z).cuda()
    win = torch.empty((S, _lib.PP_MAX_WINDOWS, 3), dtype=torch.int64, device="cuda")
    fb = torch.empty(S, dtype=torch.uint8, device="cuda")
    cf = torch.empty(S, dtype=torch.float32, device="cuda")
    import ctypes
    cap = ctypes.c_int64()
    _lib.check("pp_tile_capacity", _lib.lib().pp_tile_capacity(ds.plan.h, ctypes.byref(cap)))
    tiles = torch.empty((int(cap.value), 3), dtype=torch.int64, device="cuda")
    _lib.check("pp_propose", _lib.lib().pp_propose(ds.plan.h, ds.ws_ptr, zd.data_ptr(), 8, 0.9, win.data_ptr(),
                                                   fb.data_ptr(), cf.data_ptr(), tiles.data_ptr(), 0))
    torch.cuda.synchronize()
    wg, fg, cg = win.cpu().numpy(), fb.cpu().numpy(), cf.cpu().numpy()
    tg = tiles.cpu().numpy()
    # the tiled list covers exactly the windows of every star, in pieces of at most
    # the star's tile size
    for s in range(S):
        cov_w = set()
        for r in wg[s]:
            if r[0] == s:
                cov_w.update(range(r[1], r[2]))
        rows = tg[tg[:, 0] == s]
        cov_t = []
        for r in rows:
            cov_t.extend(range(r[1], r[2]))
        assert set(cov_t) == cov_w, s
        assert len(cov_t) <= len(cov_w) + _lib.PP_MAX_WINDOWS   # windows meet at most at one index
        assert np.all(rows[:, 2] > rows[:, 1])
    for s in range(S):
        f, bd = _oracle_grid(oracle, b, s)
        ro, co, fo = P.propose(z[s].astype(np.float64), bd.pmin, bd.pmax, bd.umin, bd.A, len(f))
        rows = [tuple(r[1:]) for r in wg[s] if r[0] == s]
        _say("star", s, "fallback", bool(fg[s]), "windows", rows)
        assert bool(fg[s]) == fo and abs(cg[s] - co) <= 1e-5
        assert len(rows) == len(ro)
        for (g0, g1), (o0, o1) in zip(rows, ro):
            assert abs(g0 - o0) <= 1 and abs(g1 - o1) <= 1
        assert all(r[0] == -1 for r in wg[s] if r[0] != s)


def test_snr_windows_parity(oracle):
    import torch
    from paper_2302_01293_amd import _lib
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.ragged(5, start=160)
    S = b.n_stars
    fine = DeviceSearch.from_batch(b)
    cp = _lib.default_params(spp=2.0 / 16)
    coarse = DeviceSearch(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax, cp, want_best=False,
                          want_snr=False, inputs=(fine.t, fine.y, fine.w))
    fine.run()
    coarse.run_prepare()
    coarse.run_search()
    nfs = np.diff(fine.plan.freq_offsets)
    rng = np.random.default_rng(15)
    W = np.full((S, _lib.PP_MAX_WINDOWS, 3), -1, np.int64)
    W[:, :, 1:] = 0
    fallback = np.zeros(S, np.uint8)
    ranges = {}
    for s in range(S):
        if s == 3:
            fallback[s] = 1
            W[s, 0] = (s, 0, nfs[s])
            continue
        rs = []
        for q in range(3):
            i0 = int(rng.integers(0, nfs[s] - 50))
            rs.append((i0, i0 + int(rng.integers(1, 400))))
        rs = [(a, min(c, nfs[s])) for a, c in rs]
        for q, (a, c) in enumerate(rs):
            W[s, q] = (s, a, c)
        ranges[s] = rs
    wd = torch.as_tensor(W).cuda()
    fd = torch.as_tensor(fallback).cuda()
    fine.run_search(windows=wd.view(-1, 3))
    plain = fine.results_host().copy()
    _lib.check("pp_snr_windows", _lib.lib().pp_snr_windows(
        fine.plan.h, fine.ws_ptr, fine.sr.data_ptr(), fine.best.data_ptr(), coarse.plan.h, coarse.ws_ptr,
        coarse.sr.data_ptr(), wd.data_ptr(), _lib.PP_MAX_WINDOWS, fd.data_ptr(), fine.result.data_ptr(), 0))
    torch.cuda.synchronize()
    res = fine.results_host()
    orc_f = oracle.batch(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax)
    orc_c = oracle.batch(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax, p=oracle.params(spp=2.0 / 16))
    for s in range(S):
        if fallback[s]:
            assert int(res["i_snr"][s]) == int(orc_f["results"][s][0])
            assert res["snr"][s] == plain["snr"][s]
            continue
        fc0, fc1 = int(orc_c["fofs"][s]), int(orc_c["fofs"][s + 1])
        ff0, ff1 = int(orc_f["fofs"][s]), int(orc_f["fofs"][s + 1])
        i, v, sig = P.window_snr(orc_c["f"][fc0:fc1], orc_c["sr"][fc0:fc1], orc_f["f"][ff0:ff1],
                                 orc_f["sr"][ff0:ff1], ranges[s], oracle.sturges(fc1 - fc0))
        _say("star", s, "gpu", int(res["i_snr"][s]), res["snr"][s], "oracle", i, v)
        assert int(res["i_snr"][s]) == i
        assert abs(res["snr"][s] - v) <= 1e-6 * max(1.0, abs(v))
        assert abs(res["sigma"][s] - sig) <= 1e-6 * sig


def test_learned_path_fallback_is_plain():
    # with a confidence threshold above 1 every star falls back: the learned path
    # must then reproduce the plain search exactly
    import torch
    from paper_2302_01293_amd import learned
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.config3(16, start=0, max_sectors=2)
    net = learned.ProposalNet(seed=1)
    ls = learned.LearnedSearch(b, net, conf=1.5)
    ls.run()
    plain = DeviceSearch.from_batch(b)
    plain.run()
    torch.cuda.synchronize()
    assert np.all(ls.fallback.cpu().numpy() == 1)
    rl, rp = ls.fine.results_host(), plain.results_host()
    assert np.array_equal(rl["i_snr"], rp["i_snr"])
    assert np.array_equal(rl["snr"].view(np.uint64), rp["snr"].view(np.uint64))
    assert abs(ls.searched_fraction() - 1.0) < 1e-12


@pytest.mark.parametrize("search_long", [1, 0])
def test_propose_guided_parity(oracle, search_long):
    """pp_propose_guided against the oracle's propose_guided: the network's windows,
    the coarse-peak windows and their merge, on stars whose coarse S/N spectrum has
    planted peaks (and ties), with the tiled list covering exactly the windows."""
    import ctypes

    import torch
    from paper_2302_01293_amd import _lib
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.ragged(8, start=170, max_sectors=13)
    ds = DeviceSearch.from_batch(b)
    cp = _lib.default_params()
    cp.spp = cp.spp / 16
    cs = DeviceSearch(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax, cp, want_best=False, want_snr=True,
                      inputs=(ds.t, ds.y, ds.w))
    S = b.n_stars
    rng = np.random.default_rng(21)
    z = rng.normal(0, 1, (S, P.NPB + 1))
    for s in range(S):
        if s % 4 != 3:
            for k in rng.choice(P.NPB, 2, replace=False):
                z[s, k] += 15.0
    z = z.astype(np.float32)
    snr_c = rng.normal(0, 1, cs.plan.n_freq)
    for s in range(S):
        a, e = int(cs.plan.freq_offsets[s]), int(cs.plan.freq_offsets[s + 1])
        for k in rng.choice(e - a, 3, replace=False):
            snr_c[a + k] = 20.0 + k % 2            # two may tie at 20
    zd = torch.as_tensor(z).cuda()
    sd = torch.as_tensor(snr_c).cuda()
    win = torch.empty((S, _lib.PP_MAX_WINDOWS, 3), dtype=torch.int64, device="cuda")
    fb = torch.empty(S, dtype=torch.uint8, device="cuda")
    cf = torch.empty(S, dtype=torch.float32, device="cuda")
    cap = ctypes.c_int64()
    _lib.check("pp_tile_capacity", _lib.lib().pp_tile_capacity(ds.plan.h, ctypes.byref(cap)))
    tiles = torch.empty((int(cap.value), 3), dtype=torch.int64, device="cuda")
    npk, hw = 4, 3
    _lib.check("pp_propose_guided", _lib.lib().pp_propose_guided(
        ds.plan.h, ds.ws_ptr, zd.data_ptr(), 8, 0.9, search_long, cs.plan.h, cs.ws_ptr, sd.data_ptr(), npk, hw,
        win.data_ptr(),
        fb.data_ptr(), cf.data_ptr(), tiles.data_ptr(), 0))
    torch.cuda.synchronize()
    wg, fg, cg, tg = win.cpu().numpy(), fb.cpu().numpy(), cf.cpu().numpy(), tiles.cpu().numpy()
    n_conf = 0
    for s in range(S):
        fi = ds.plan.star_info(s)
        ci = cs.plan.star_info(s)
        nf = int(fi["nf"])
        a, e = int(cs.plan.freq_offsets[s]), int(cs.plan.freq_offsets[s + 1])
        ro, co, fo = P.propose_guided(z[s].astype(np.float64), fi["pmin"], fi["pmax"], fi["umin"], fi["A"], nf,
                                      snr_c[a:e], ci["umin"], ci["A"], npk, hw, search_long=bool(search_long))
        rows = [tuple(r[1:]) for r in wg[s] if r[0] == s]
        _say("star", s, "fallback", bool(fg[s]), "windows", rows)
        assert bool(fg[s]) == fo and abs(cg[s] - co) <= 1e-5
        # the network's bin-edge mapping may differ by one index (cbrt); coarse peaks are exact
        assert len(rows) == len(ro), (rows, ro)
        for (g0, g1), (o0, o1) in zip(rows, ro):
            assert abs(g0 - o0) <= 1 and abs(g1 - o1) <= 1
        if not fo:
            n_conf += 1
            for ic in P.coarse_peaks(snr_c[a:e], npk, hw):
                i_f = int(round((ci["umin"] + ic * ci["A"] - fi["umin"]) / fi["A"]))
                if 0 <= i_f < nf:
                    assert any(g0 <= i_f < g1 for g0, g1 in rows), (s, ic, i_f)
        cov_w = set()
        for g0, g1 in rows:
            cov_w.update(range(g0, g1))
        cov_t = []
        for r in tg[tg[:, 0] == s]:
            cov_t.extend(range(r[1], r[2]))
        assert set(cov_t) == cov_w and len(cov_t) == len(cov_w), s   # merged: no index searched twice
    assert n_conf >= 3


def test_guided_learned_path_recovers_sector_scale_detections():
    """The guided learned path (network windows plus coarse-peak windows) on 64 stars
    of the 1-26-sector recipe (seeds disjoint from the benchmark's): every plain
    detection is reported again at its frequency index, while only a small part of
    the fine grid is searched."""
    import torch
    from paper_2302_01293_amd import learned
    b = synth.config4(64, start=200_000)
    net = learned.ProposalNet(np.load(os.path.join(ROOT, "paper_2302_01293_amd", "pp_weights.npy")))
    out, pres, lres = learned.time_paths(b, net, reps=1, topk=8, conf=0.5, coarse_peaks=2, search_long=False)
    torch.cuda.synchronize()
    _say("guided path on 64 sector-scale stars: recovery %d/%d, searched fraction %.4f, speed-up %.2fx"
         % (out["recovered"], out["plain_detections"], out["searched_fraction"], out["speedup"]))
    assert out["plain_detections"] >= 3
    assert out["recovered"] == out["plain_detections"]
    assert out["searched_fraction"] < 0.05
