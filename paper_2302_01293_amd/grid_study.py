"""S/N of injected transits against the density of the frequency grid.

    python -m paper_2302_01293_amd.grid_study --stars 2048 --spp 0.25,0.5,1,2,4

QLP Data Release Notes 003, Sec. 2.2 (the paragraph on the detection criteria):
transit-like signals come out with higher S/N on the finer grid of the GPU search,
so the S/N threshold became 9 for every star.  This study searches the same
synthetic stars (one sector at 200 s, 20% boxes) at several samples per peak and
reports, per grid density, the frequencies searched, the median S/N of the injected
signals found at their period (within 1%), how many reach S/N > 9 and > 5 there, and
the S/N of the detections of stars without a signal (the noise peaks, whose level
rises with the number of frequencies tried).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def study(batch, spps, params_kw=None) -> list[dict]:
    import torch

    from . import _lib
    from .device import DeviceSearch
    inj = np.asarray(batch.truth["injected"], bool)
    pt = np.asarray(batch.truth["period"])
    rows = []
    for spp in spps:
        ds = DeviceSearch.from_batch(batch, _lib.default_params(spp=float(spp), **(params_kw or {})),
                                     want_snr=False)
        ds.run()
        torch.cuda.synchronize()
        r = ds.results_host()
        hit = np.zeros(batch.n_stars, bool)
        hit[inj] = np.abs(r["period"][inj] / pt[inj] - 1.0) < 0.01
        snr_inj = r["snr"][hit]
        noise = r["snr"][~inj]
        rows.append(dict(spp=float(spp), frequencies=int(ds.plan.n_freq),
                         injected=int(inj.sum()), found_at_period=int(hit.sum()),
                         median_snr_found=float(np.median(snr_inj)) if len(snr_inj) else float("nan"),
                         found_snr_above_9=int(np.sum(snr_inj > 9.0)), found_snr_above_5=int(np.sum(snr_inj > 5.0)),
                         noise_median_snr=float(np.median(noise)) if len(noise) else float("nan"),
                         noise_snr_above_9=int(np.sum(noise > 9.0)), noise_snr_above_5=int(np.sum(noise > 5.0)),
                         noise_stars=int((~inj).sum())))
        del ds
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--stars", type=int, default=2048)
    ap.add_argument("--start", type=int, default=3_000_000)
    ap.add_argument("--spp", default="0.25,0.5,1,2,4")
    args = ap.parse_args(argv)
    import torch

    from . import synth
    assert torch.cuda.is_available(), "needs the GPU"
    b = synth.config1(args.stars, start=args.start)
    rows = study(b, [float(x) for x in args.spp.split(",")])
    for r in rows:
        print("spp %-5g %9d frequencies: injected found at their period %d/%d, median S/N %.2f, S/N > 9: %d, "
              "> 5: %d; stars without a signal: median best S/N %.2f, above 9: %d, above 5: %d of %d"
              % (r["spp"], r["frequencies"], r["found_at_period"], r["injected"], r["median_snr_found"],
                 r["found_snr_above_9"], r["found_snr_above_5"], r["noise_median_snr"], r["noise_snr_above_9"],
                 r["noise_snr_above_5"], r["noise_stars"]), file=sys.stderr, flush=True)
    print(json.dumps(dict(stars=b.n_stars, workload="one sector at 200 s, 20% boxes (cfg1 recipe)", rows=rows)),
          flush=True)


if __name__ == "__main__":
    main()
