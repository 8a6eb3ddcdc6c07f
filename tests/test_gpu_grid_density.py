"""Grid density and S/N (Sec. 2.2, the paragraph on the detection criteria): on the
finer grid the injected transits found at their period come out with a higher S/N,
and so do the best peaks of stars without a signal, the reason the note gives for
requiring S/N > 9 for every star.  The same 512 one-sector stars are searched at 0.5
and 4 samples per peak; the number of frequencies scales with the samples per peak."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")
def test_snr_rises_with_grid_density():
    from paper_2302_01293_amd import grid_study, synth
    print("grid density study: 512 one-sector stars, spp 0.5 and 4", flush=True)
    b = synth.config1(512, start=3_100_000)
    coarse, fine = grid_study.study(b, [0.5, 4.0])
    assert fine["frequencies"] / coarse["frequencies"] == pytest.approx(8.0, rel=1e-3)
    assert coarse["injected"] == fine["injected"] > 50
    assert fine["found_at_period"] >= coarse["found_at_period"]
    assert fine["median_snr_found"] > coarse["median_snr_found"] * 1.05
    assert fine["noise_median_snr"] > coarse["noise_median_snr"]
    assert fine["noise_snr_above_5"] > coarse["noise_snr_above_5"]
    assert np.isfinite([fine["median_snr_found"], fine["noise_median_snr"]]).all()
