"""Write ``sector_stars.json``: the oracle's full-spectrum results for three
full-size stars of the sector-scale mix (20-26 sectors at 200-s cadence).

Calls only ``oracle/`` (and the seeded input generator): nothing here comes from
the HIP path.  The stars are indices of ``synth.config4(256, start=0)``, the first
batch the benchmark times:
  *   8: 24 sectors, 273,720 points, density 4.5 solar: 305,851 frequencies, up to
         6,372 fine bins (more than one LDS pass holds);
  * 109: 26 sectors, 296,530 points, a 6.9e-3 box at P = 80.3 d;
  * 114: 24 sectors, 273,720 points, a 7.3e-4 box at P = 3.30 d.
For each the file holds the per-star result (best-S/N index, best-SR index,
period, mid-transit time, duration, depth, SR, S/N, trend, sigma, status), the
32 largest SR and S/N values with their indices (to judge near-ties), and the
spectrum's length.  Run time: about 16 minutes on three cores.

    python tests/golden/make_sector_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2302_01293_amd import synth  # noqa: E402

STARS = (8, 109, 114)
BATCH = dict(n_stars=256, start=0)


def main():
    b = synth.config4(**BATCH)
    out = oracle.batch(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax, stars=list(STARS),
                       nthreads=len(STARS))
    rows = []
    for k, s in enumerate(STARS):
        o0, o1 = int(out["fofs"][k]), int(out["fofs"][k + 1])
        sr, snr = out["sr"][o0:o1], out["snr"][o0:o1]
        top_sr = np.argsort(-sr, kind="stable")[:32]
        top_snr = np.argsort(-snr, kind="stable")[:32]
        R = dict(zip(oracle.RESULT_FIELDS, out["results"][k].tolist()))
        rows.append(dict(star=s, n_points=int(b.offsets[s + 1] - b.offsets[s]), n_freq=o1 - o0,
                         n_sectors=int(b.truth["n_sectors"][s]), rho=float(b.rho[s]),
                         injected=bool(b.truth["injected"][s]), result=R,
                         top_sr=[[int(i), float(sr[i])] for i in top_sr],
                         top_snr=[[int(i), float(snr[i])] for i in top_snr],
                         nb_max=int(out["nb"][o0:o1].max())))
        print(s, R, flush=True)
    doc = dict(workload="synth.config4", batch=BATCH, params="paper defaults (oracle.params())",
               written_by="tests/golden/make_sector_golden.py (oracle only)", stars=rows)
    with open(os.path.join(HERE, "sector_stars.json"), "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
