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
