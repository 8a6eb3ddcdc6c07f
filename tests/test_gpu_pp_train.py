"""GPU tests of the trained proposal: training from scratch lowers the loss, and the
committed trained network gains over the untrained one on held-out light curves
(less of the grid searched, less device time) while recovering the plain
detections."""
import os

import numpy as np
import pytest

from paper_2302_01293_amd import synth

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2302_01293_amd",
                       "pp_weights.npy")


def _say(*a):
    print(*a, flush=True)


def test_training_lowers_loss():
    import torch
    from paper_2302_01293_amd import learned
    b = synth.config3(512, start=100_000, max_sectors=2)
    x, lag, labels, _ = learned.labelled_inputs(b)
    net = learned.ProposalNet(seed=3)
    hist = learned.train(net, x, lag, labels, epochs=6, batch=64, lr=0.03)
    torch.cuda.synchronize()
    _say("loss per epoch", ["%.3f" % h for h in hist])
    assert np.all(np.isfinite(hist)) and hist[-1] < 0.8 * hist[0]


def test_trained_network_gains_over_untrained():
    from paper_2302_01293_amd import learned
    b = synth.config3(1024, start=200_000, max_sectors=3)
    trained = learned.ProposalNet(np.load(WEIGHTS))
    untrained = learned.ProposalNet(seed=0)
    out_t, _, _ = learned.time_paths(b, trained, conf=0.95, topk=12)
    out_u, _, _ = learned.time_paths(b, untrained, conf=0.95, topk=12)
    _say("trained", out_t)
    _say("untrained", out_u)
    # the untrained network is never confident: it searches the whole grid
    assert out_u["fallback_fraction"] == 1.0 and out_u["recovery"] == 1.0
    # the trained one searches less of the grid, in less time, and keeps >= 99% of
    # the plain detections
    assert out_t["searched_fraction"] < 0.8 * out_u["searched_fraction"]
    assert out_t["learned_ms"] < out_u["learned_ms"]
    assert out_t["recovery"] >= 0.99
