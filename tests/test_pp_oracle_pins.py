"""Pins of the learned-proposal oracle (``oracle/pp_oracle.py``) against library
routines, brute force, closed forms and finite differences (CPU only)."""
import math

import numpy as np
import pytest

from oracle import pp_oracle as P


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 5000), [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9,
                                                                           -2.5, 0.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(P.bf16(x), ref)
    assert P.bf16(1 + 2 ** -8) == 1.0 and P.bf16(1 + 3 * 2 ** -9) == 1 + 2 ** -7   # ties to even


def test_resample_tiny_by_hand():
    t = np.array([10.0, 11.0, 12.0, 13.0, 13.0])
    y = np.array([1.0, 2.0, 3.0, 4.0, 6.0])
    w = np.array([1.0, 1.0, 1.0, 1.0, 3.0])
    X, dl = P.resample(t, y, w, nbins=4)
    # median 3, |y-3| = 2,1,0,1,3 -> MAD 1, s = 1.4826; bins 0,1,2,3,3
    s = 1.4826
    exp0 = [(1 - 3) / s, (2 - 3) / s, 0.0, (1 * (4 - 3) / s + 3 * (6 - 3) / s) / 4]
    assert np.array_equal(X[0], P.bf16(exp0))
    assert np.array_equal(X[1], [1, 1, 1, 1])
    assert dl == 3.0 / (4 // 4)


def test_resample_invariances_and_coverage():
    rng = np.random.default_rng(2)
    t = np.sort(rng.uniform(0, 27.4, 3000))
    y = 1 + rng.normal(0, 1e-3, 3000)
    w = rng.uniform(0.5, 2, 3000)
    w[100:400] = 0.0
    X, dl = P.resample(t, y, w)
    X2, _ = P.resample(t, 3.0 * y + 7.0, w)
    assert np.max(np.abs(X2[0] - X[0])) <= 2 ** -7 * np.max(np.abs(X[0]))  # affine invariance up to BF16
    good = w > 0
    T = t[good][-1] - t[good][0]
    b = np.clip(np.floor((t - t[good][0]) / T * P.L0).astype(int), 0, P.L0 - 1)
    cov = np.zeros(P.L0)
    cov[np.unique(b[good])] = 1
    assert np.array_equal(X[1], cov)
    assert dl == T / P.L2


def test_conv_matches_scipy_correlate():
    from scipy.signal import correlate
    rng = np.random.default_rng(3)
    x = rng.normal(size=(P.C_IN, 64))
    W = rng.normal(size=(5, P.C_IN, P.K1))
    b = rng.normal(size=5)
    out = P._conv(x, W, b, 2, P.P1)
    for o in range(5):
        acc = np.zeros(64 + P.K1 - 1)
        for c in range(P.C_IN):
            xp = np.concatenate([np.zeros(P.P1), x[c], np.zeros(P.K1)])
            acc = correlate(xp, W[o, c], mode="valid")[:64] + (acc[:64] if c else 0)
        np.testing.assert_allclose(out[o], b[o] + acc[::2][:32], rtol=1e-12, atol=1e-12)


def test_autocorrelation_brute_force():
    rng = np.random.default_rng(4)
    X = np.stack([rng.normal(size=P.L0), (rng.uniform(size=P.L0) < 0.8).astype(float)])
    theta = P.pack(_init(rng))
    _, c = P.forward(X, theta, 0.03, use_bf16=False)
    sh = c["sh"]
    for tau in (0, 1, 7, 100, 511, P.L2 - 1):
        direct = sum(sh[t] * sh[t + tau] for t in range(P.L2 - tau)) / P.L2
        assert abs(direct - c["A"][tau]) <= 1e-12 * max(1.0, abs(c["A"][0]))
    assert abs(sh.mean()) < 1e-12


def _init(rng):
    return dict(W1=rng.normal(0, 0.3, (P.C1, P.C_IN, P.K1)), b1=rng.normal(0, 0.1, P.C1),
                W2=rng.normal(0, 0.1, (P.C2, P.C1, P.K2)), b2=rng.normal(0, 0.1, P.C2),
                w3=rng.normal(0, 0.5, P.C2), alpha=3.0, beta=rng.normal(0, 0.1, P.NPB), delta=0.2)


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(5)
    theta = P.pack(_init(rng))
    Xs = [np.stack([rng.normal(size=P.L0), (rng.uniform(size=P.L0) < 0.9).astype(float)]) for _ in range(2)]
    dl = [0.027, 0.08]
    lab = [200, P.NPB]
    _, g = P.loss_and_grad(Xs, theta, dl, lab, use_bf16=False)
    h = 1e-6
    picks = []
    for name, (a, b) in P.OFF.items():
        for j in rng.choice(np.arange(a, b), size=min(4, b - a), replace=False):
            picks.append((name, int(j)))
    for name, j in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        lp, _ = P.loss_and_grad(Xs, tp, dl, lab, use_bf16=False)
        lm, _ = P.loss_and_grad(Xs, tm, dl, lab, use_bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * max(1e-3, abs(fd)), (name, j, fd, g[j])


def test_soft_target_and_bins():
    q = P.soft_target(0)
    assert abs(q.sum() - 1) < 1e-15 and q[0] > q[1] > 0 and q[P.NPB] == 0
    assert P.soft_target(-1)[P.NPB] == 1.0
    e = P.period_edges()
    assert e[0] == 0.5 and abs(e[-1] - 100.0) < 1e-12
    for k in (0, 17, 300, 511):
        assert P.period_bin(P.period_centres()[k]) == k
    assert P.period_bin(100.0) == -1 and P.period_bin(0.49) == -1


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(6)
    th = rng.normal(size=20)
    m = np.zeros(20)
    v = np.zeros(20)
    tt = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=20)
        th, m, v = P.adam(th, m, v, g, step, 1e-2)
        tt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(th, tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_propose_windows_and_fallback():
    umin, A = (1 / 13.7) ** (1 / 3), 1e-4
    nf = int(((1 / 0.35) ** (1 / 3) - umin) / A) + 1
    z = np.full(P.NPB + 1, -20.0)
    k = P.period_bin(3.1)
    z[k] = 10.0
    z[P.NPB] = 0.0
    rng_, c, fb = P.propose(z, 0.35, 13.7, umin, A, nf)
    assert not fb and c > 0.99
    e = P.period_edges()
    # the other seven of the top 8 tie at the lowest bins (ties go to the lower bin)
    assert len(rng_) == 2
    i0, i1 = [r for r in rng_ if 1 / (umin + r[0] * A) ** 3 > 3.1 > 1 / (umin + (r[1] - 1) * A) ** 3][0]
    f = (umin + np.arange(i0, i1) * A) ** 3
    assert np.all((1 / f >= e[k - 1] * (1 - 1e-9)) & (1 / f <= e[k + 2] * (1 + 1e-9)))
    assert 1 / ((umin + (i0 - 1) * A) ** 3) > e[k + 2] and 1 / ((umin + i1 * A) ** 3) < e[k - 1]
    # a flat heatmap is not confident: full grid
    rng_, c, fb = P.propose(np.zeros(P.NPB + 1), 0.35, 13.7, umin, A, nf)
    assert fb and rng_ == [(0, nf)] and c < 0.9
    # periods beyond the heatmap are always searched
    umin2 = (1 / 300.0) ** (1 / 3)
    nf2 = int(((1 / 0.35) ** (1 / 3) - umin2) / A) + 1
    rng_, c, fb = P.propose(z, 0.35, 300.0, umin2, A, nf2)
    assert not fb and any(r[0] == 0 for r in rng_) and len(rng_) == 3


def test_window_snr_equals_plain_snr_on_full_grid(oracle):
    # with the coarse spectrum equal to the fine one and one full-grid window the
    # windowed S/N is the plain S/N of the C oracle (an independent implementation)
    from paper_2302_01293_amd import synth
    b = synth.config0()
    t, y, w = b.star(0)
    f, nb, bd = oracle.grid(t, w, float(b.rho[0]), oracle.params(), float(b.pmin[0]), float(b.pmax[0]))
    sp = oracle.bls_star(t, y, w, float(b.rho[0]), oracle.params(), float(b.pmin[0]), float(b.pmax[0]))
    _, _, res = oracle.snr(f, sp.sr)
    i, v, sigma = P.window_snr(f, sp.sr, f, sp.sr, [(0, len(f))], oracle.sturges(len(f)))
    assert i == res.i_snr and abs(v - res.snr_max) <= 1e-12 * abs(res.snr_max)
    assert abs(sigma - res.sigma) <= 1e-14 * sigma


def test_coarse_peaks_hand_built():
    """Largest first, each pick blocks +-h, ties to the lower index."""
    v = np.zeros(40)
    v[10], v[12], v[30], v[5] = 5.0, 4.0, 3.0, 5.0   # 5 and 10 tie; 12 is within h=2 of 10
    assert P.coarse_peaks(v, 3, 2) == [5, 10, 30]
    assert P.coarse_peaks(v, 1, 2) == [5]
    assert P.coarse_peaks(v, 4, 2) == [5, 10, 30, 0]    # then the first free zero (0..2 free of 5+-2)
    assert P.coarse_peaks(np.ones(3), 5, 1) == [0, 2]   # the grid runs out


def test_coarse_windows_map_u_ranges_to_the_fine_grid():
    """A coarse grid with 16 times the fine step from the same u_min: coarse index i
    is fine index 16 i, so +-h coarse steps are fine [16 (i - h), 16 (i + h)]."""
    umin, A = 0.25, 1e-4
    nf = 5000
    w = P.coarse_windows([100, 3, 311, 313], umin, 16 * A, 314, umin, A, nf, 2)
    assert w[0] == (16 * 98, 16 * 102 + 1)
    assert w[1] == (16 * 1, 16 * 5 + 1)
    assert w[2] == (16 * 309, nf)                          # clipped to the fine grid (16 * 313 > nf - 1)
    assert w[3] == (16 * 311, nf)                          # and to the coarse grid (313 + 2 > 313)
    assert P.coarse_windows([0], umin, 16 * A, 313, umin, A, nf, 3) == [(0, 16 * 3 + 1)]


def test_merge_ranges_is_the_union():
    rng = np.random.default_rng(3)
    for _ in range(50):
        rs = []
        for _ in range(rng.integers(1, 9)):
            a = int(rng.integers(0, 200))
            rs.append((a, a + int(rng.integers(1, 30))))
        m = P.merge_ranges(rs)
        cov = set()
        for a, b in rs:
            cov.update(range(a, b))
        got = set()
        for a, b in m:
            got.update(range(a, b))
        assert got == cov
        assert all(m[i][1] < m[i + 1][0] for i in range(len(m) - 1))   # disjoint, not touching


def test_guided_proposal_adds_the_coarse_peak_and_keeps_fallback():
    """A confident network window elsewhere plus a coarse peak: both ranges are
    searched; a star that falls back still searches its full grid only."""
    umin, A = (1.0 / 13.7) ** (1 / 3), 2e-5
    nf = int(((1 / 0.35) ** (1 / 3) - umin) / A) + 1
    z = np.full(P.NPB + 1, -5.0)
    z[200] = 10.0
    snr_c = np.zeros(nf // 16)
    snr_c[1000] = 12.0
    r, c, fb = P.propose_guided(z, 0.35, 13.7, umin, A, nf, snr_c, umin, 16 * A, 1, 3)
    assert not fb
    base, _, _ = P.propose(z, 0.35, 13.7, umin, A, nf)
    cw = P.coarse_windows([1000], umin, 16 * A, len(snr_c), umin, A, nf, 3)
    assert r == P.merge_ranges(base + cw)
    assert any(a <= 16 * 1000 < b for a, b in r)
    r2, c2, fb2 = P.propose_guided(np.zeros(P.NPB + 1), 0.35, 13.7, umin, A, nf, snr_c, umin, 16 * A, 1, 3)
    assert fb2 and r2 == [(0, nf)]
    # topk = 0: the null probability alone is the confidence; only coarse windows
    z0 = np.full(P.NPB + 1, -20.0)
    z0[P.NPB] = 10.0
    r3, c3, fb3 = P.propose_guided(z0, 0.35, 13.7, umin, A, nf, snr_c, umin, 16 * A, 2, 3, topk=0, conf=0.5)
    assert not fb3 and c3 > 0.99
    assert r3 == P.merge_ranges(P.coarse_windows(P.coarse_peaks(snr_c, 2, 3), umin, 16 * A, len(snr_c),
                                                 umin, A, nf, 3))


def test_guided_proposal_without_the_long_period_window():
    """With Pmax > 100 d the plain proposal adds [100 d, Pmax]; search_long=False drops
    it and keeps the network's and the coarse peaks' windows."""
    umin, A = (1.0 / 300.0) ** (1 / 3), 2e-5
    nf = int(((1 / 0.35) ** (1 / 3) - umin) / A) + 1
    z = np.full(P.NPB + 1, -5.0)
    z[300] = 12.0
    snr_c = np.zeros(nf // 16)
    snr_c[2000] = 9.0
    i_long = int(((1 / 100.0) ** (1 / 3) - umin) / A)        # fine index of P = 100 d
    with_long, _, _ = P.propose_guided(z, 0.35, 300.0, umin, A, nf, snr_c, umin, 16 * A, 1, 3)
    without, _, _ = P.propose_guided(z, 0.35, 300.0, umin, A, nf, snr_c, umin, 16 * A, 1, 3, search_long=False)
    assert any(a == 0 and b >= i_long for a, b in with_long)          # [100 d, Pmax] starts at f0
    assert not any(a <= 10 for a, b in without)
    base, _, _ = P.propose(z, 0.35, 300.0, umin, A, nf, pb_hi_window=False)
    assert without == P.merge_ranges(base + P.coarse_windows([2000], umin, 16 * A, len(snr_c), umin, A, nf, 3))
