"""Workload for profiling the learned path next to the plain path (rocprofv3).

    rocprofv3 --kernel-trace --stats -d out -o lp --output-format csv -- \
        python3 paper_2302_01293_amd/profile_learned.py

Runs the learned path (untrained network, so every star falls back to its full
grid and every kernel of the path runs at full size) and the plain path twice
each on 1024 held-out light curves of 1-3 sectors at 200-s cadence.
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import torch  # noqa: E402

from paper_2302_01293_amd import learned, synth  # noqa: E402
from paper_2302_01293_amd.device import DeviceSearch  # noqa: E402


def main():
    b = synth.config3(1024, start=4096, max_sectors=3)
    net = learned.ProposalNet(seed=0)
    ls = learned.LearnedSearch(b, net)
    plain = DeviceSearch.from_batch(b)
    for _ in range(2):
        ls.run()
        plain.run()
    torch.cuda.synchronize()
    print("done", flush=True)


if __name__ == "__main__":
    main()
