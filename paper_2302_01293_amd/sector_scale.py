"""Sector-scale throughput: stars/hour over a stream of mixed 1-26-sector stars.

    python -m paper_2302_01293_amd.sector_scale --batches 4 --batch-stars 1024 [--precision 1]
    python -m paper_2302_01293_amd.sector_scale --batches 64 --batch-stars 1024 --lazy

The light curves (``synth.config4``: 1-26 contiguous sectors at 200 s, 10% boxes)
are drawn before the clock starts, as they would be read from disk, or with
``--lazy`` on a host thread that stays at most two batches ahead (65,536 such stars
hold about 240 GB); the clock covers plan creation, host-to-device copies, prepare,
search, S/N and the results' return, with the copy of one batch overlapping the
search of the other (``stream.run_stream``).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _ahead(make, n, seen_points, depth: int = 2):
    """Batches make(0..n-1) produced on a host thread, at most ``depth`` ahead."""
    import queue
    import threading
    q = queue.Queue(maxsize=depth)

    def work():
        for i in range(n):
            q.put(make(i))
        q.put(None)

    threading.Thread(target=work, daemon=True).start()
    while True:
        b = q.get()
        if b is None:
            return
        seen_points.append(b.n_points)
        yield b


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--batches", type=int, default=4)
    ap.add_argument("--batch-stars", type=int, default=1024)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--lazy", action="store_true",
                    help="generate the batches on a host thread during the run (bounded memory)")
    args = ap.parse_args(argv)
    import torch
    from . import _lib, stream, synth
    assert torch.cuda.is_available(), "needs the GPU"
    def make(i):
        return synth.config4(args.batch_stars, start=i * args.batch_stars)

    seen_points = []
    if args.lazy:
        batches = _ahead(make, args.batches, seen_points)
    else:
        t0 = time.time()
        batches = [make(i) for i in range(args.batches)]
        seen_points.extend(b.n_points for b in batches)
        print("generated %d batches (%.1f s)" % (len(batches), time.time() - t0), file=sys.stderr, flush=True)
    params = _lib.default_params(precision=args.precision)
    # warm-up on a small batch (kernel loading, allocator)
    stream.run_stream([synth.config4(8, start=10_000_000)], params)
    torch.cuda.synchronize()
    res, stats = stream.run_stream(batches, params,
                                   log=lambda *a: print(*a, file=sys.stderr, flush=True))
    points = sum(seen_points)
    stats.update(batches=args.batches, batch_stars=args.batch_stars, points=points, precision=args.precision,
                 workload="cfg4 recipe: 1-26 contiguous sectors at 200 s, 10% boxes")
    print(json.dumps(stats), flush=True)


if __name__ == "__main__":
    main()
