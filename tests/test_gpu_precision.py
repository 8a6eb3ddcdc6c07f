"""Reduced-precision mode (precision = 1: weights and residuals packed into one
64-bit fixed-point sum per bin, one LDS atomic per boundary) against the FP64
oracle on uneven multi-sector stars.  The SR error per result is reported as
max / p99 / median; the bound tested is the mode's stated accuracy (1e-5 relative
for the bulk of the spectrum, a few 1e-5 at worst)."""
import numpy as np
import pytest

from paper_2302_01293_amd import synth

import parity_util as pu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_packed_sr_error_vs_oracle(oracle):
    from paper_2302_01293_amd import _lib
    rows = synth.config2(48, start=300)
    n = np.diff(rows.offsets)
    pick = [int(i) for i in np.nonzero(n < 50000)[0][:12]]
    b = rows.subset(pick)
    _say("case packed: stars", len(pick), "points", np.diff(b.offsets).tolist())
    ds = pu.fetch(pu.run_gpu(b, _lib.default_params(precision=1)))
    orc = pu.run_oracle(oracle, b)
    rel_all = []
    same_snr = 0
    for s in range(b.n_stars):
        sl = ds.star_slice(s)
        o0, o1 = int(orc["fofs"][s]), int(orc["fofs"][s + 1])
        sr_g, sr_o = ds._sr_host[sl], orc["sr"][o0:o1]
        rel = np.abs(sr_g - sr_o) / np.maximum(np.abs(sr_o), 1e-300)
        rel_all.append(rel)
        same_snr += int(ds._res_host["i_snr"][s] == int(orc["results"][s][0]))
    rel = np.concatenate(rel_all)
    mx, p99, med = float(rel.max()), float(np.percentile(rel, 99)), float(np.median(rel))
    _say("packed SR rel err: max %.3e p99 %.3e median %.3e over %d frequencies; best-S/N index equal for %d/%d"
         % (mx, p99, med, len(rel), same_snr, b.n_stars))
    assert med <= 1e-6 and p99 <= 1e-5 and mx <= 1e-4
    assert same_snr >= b.n_stars - 1


def test_packed_sr_error_cfg2_stratified(oracle):
    """The mode's SR error on a stratified 256-star subset of the uneven 1-13-sector
    workload (up to 20 stars of each length class), at 64 sampled
    frequencies per star (the oracle searches each one in full)."""
    from paper_2302_01293_amd import _lib
    pool = synth.config2(2048, start=0)
    span = np.asarray(pool.truth["n_sectors"])
    n = np.diff(pool.offsets)
    # stratify by point count (sectors present): up to 20 stars of each of the 13
    # length classes, topped up to 256 from the longest classes
    cls = np.minimum(12, (n - 1) // 11405)
    pick = [int(i) for k in range(13) for i in np.nonzero(cls == k)[0][:20]]
    for k in range(12, -1, -1):
        for i in np.nonzero(cls == k)[0][20:]:
            if len(pick) < 256:
                pick.append(int(i))
    pick = np.asarray(pick)
    b = pool.subset(np.sort(pick))
    _say("case packed stratified: %d stars, %d points, sector counts %s" % (
        b.n_stars, b.n_points, np.bincount(span[np.sort(pick)]).tolist()))
    ds = pu.fetch(pu.run_gpu(b, _lib.default_params(precision=1), want_best=False, want_snr=False))
    rng = np.random.default_rng(11)
    rel_all = []
    from concurrent.futures import ThreadPoolExecutor

    def one(s):
        sl = ds.star_slice(s)
        sr = ds._sr_host[sl]
        idx = np.unique(rng.integers(0, len(sr), 64))
        t, y, w = b.star(s)
        o = oracle.bls_star_at(t, y, w, idx, float(b.rho[s]))
        return np.abs(sr[idx] - o.sr) / np.maximum(o.sr, 1e-300)

    with ThreadPoolExecutor(8) as ex:
        rel_all = list(ex.map(one, range(b.n_stars)))
    rel = np.concatenate(rel_all)
    mx, p99, med = float(rel.max()), float(np.percentile(rel, 99)), float(np.median(rel))
    _say("packed SR rel err, stratified cfg2 subset: max %.3e p99 %.3e median %.3e over %d results"
         % (mx, p99, med, len(rel)))
    assert med <= 1e-6 and p99 <= 1e-5 and mx <= 1e-4
