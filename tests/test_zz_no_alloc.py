"""bls_run_noalloc (the entry point that allocates nothing) against the existing
entry points (bls_plan_upload, bls_prepare, bls_search_batch, bls_snr on a caller
workspace): bit-equal outputs on two calls in a row, the second with a smaller
batch, and the size check that rejects a plan larger than the static scratch."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _compare(batch, windows=None):
    import torch
    from paper_2302_01293_amd import _lib
    from paper_2302_01293_amd.device import DeviceSearch

    ref = DeviceSearch.from_batch(batch)
    assert ref.plan.workspace_bytes <= _lib.NOALLOC_SCRATCH_BYTES
    wdev = None
    if windows is not None:
        wdev = torch.as_tensor(np.asarray(windows, np.int64).reshape(-1, 3)).cuda()
    ref.run(windows=wdev)
    torch.cuda.synchronize()
    nf, S = ref.plan.n_freq, ref.plan.n_stars
    sr = torch.full((nf,), -1.0, dtype=torch.float64, device="cuda")
    best = torch.zeros(nf * _lib.BEST_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    snr = torch.full((nf,), -1.0, dtype=torch.float64, device="cuda")
    res = torch.zeros(S * _lib.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    if windows is not None:        # frequencies outside the windows are not written
        sr.copy_(ref.sr)
        best.copy_(ref.best)
    # A second plan of the same batch: the reference's plan stays uploaded to its own
    # workspace.
    pl = _lib.Plan(batch.t, batch.y, batch.w, batch.offsets, batch.rho, batch.pmin, batch.pmax)
    h = int(torch.cuda.current_stream().cuda_stream)
    pl.run_noalloc(ref.t.data_ptr(), ref.y.data_ptr(), ref.w.data_ptr(), sr.data_ptr(), best.data_ptr(),
                   snr.data_ptr(), res.data_ptr(), None if wdev is None else wdev.data_ptr(),
                   0 if wdev is None else int(wdev.shape[0]), stream=h)
    torch.cuda.synchronize()
    # integer bin sums: every output is bit-equal, not merely close
    assert torch.equal(sr.view(torch.int64), ref.sr.view(torch.int64))
    assert torch.equal(best, ref.best)
    assert torch.equal(snr.view(torch.int64), ref.snr.view(torch.int64))
    assert torch.equal(res, ref.result)
    r = ref.results_host()
    _say("stars %d, frequencies %d, workspace %.2f MB: outputs bit-equal; first star P = %.6f d S/N = %.2f"
         % (S, nf, pl.workspace_bytes / 1e6, r["period"][0], r["snr"][0]))
    pl.close()


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_noalloc_matches_workspace_path_two_calls():
    from paper_2302_01293_amd import synth
    big = synth.config2(10, start=40)        # 1-13 sectors: tens of MB of workspace
    small = synth.config1(3, start=7)        # then a smaller batch on the same scratch
    _say("call 1: %d stars, %d points" % (big.n_stars, big.n_points))
    _compare(big)
    _say("call 2: %d stars, %d points" % (small.n_stars, small.n_points))
    _compare(small)
    _say("call 3: windows (star, i0, i1) on the small batch")
    _compare(small, windows=[[0, 10, 900], [2, 0, 50], [1, 3000, 4000]])
