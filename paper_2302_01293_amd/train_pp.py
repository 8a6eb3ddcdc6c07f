"""Train the period-proposal network on the GPU and compare the learned path with
the plain search on held-out light curves.

    python -m paper_2302_01293_amd.train_pp --n-train 8192 --n-eval 2048 \
        --max-sectors 3 --epochs 40 --out pp_weights.npy --report pp_report.json

Training light curves are the trapezoid-injection recipe of ``synth.config3``, or
with ``--recipe mixed`` half of them and half one-sector box-injection stars of
the ``synth.config1`` recipe (seeds disjoint from the benchmark's); labels come
from the plain search on each of them (``learned.plain_labels``).
The report gives, for the untrained and the trained network on the evaluation
stars: recovery of the plain detections, the fraction of stars that fell back
to the full grid, the searched fraction of the grid, and the device time of both
paths (learned and plain) with their ratio.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


# one-sector training and evaluation stars come from seeds far from the
# benchmark's (stars 0 .. 4095 of the same recipe)
CFG1_TRAIN_START = 100_000
CFG1_EVAL_START = 150_000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def labelled(batch, chunk: int = 2048):
    """Plain-search labels and network inputs of a batch, in chunks of stars."""
    import torch
    from . import learned
    xs, lags, labels, res = [], [], [], []
    for s0 in range(0, batch.n_stars, chunk):
        sub = batch.subset(np.arange(s0, min(batch.n_stars, s0 + chunk)))
        x, lag, lab, r = learned.labelled_inputs(sub)
        xs.append(x)
        lags.append(lag)
        labels.append(lab)
        res.append(r)
        torch.cuda.synchronize()
    return torch.cat(xs), torch.cat(lags), np.concatenate(labels), np.concatenate(res)


def labelled_streamed(make, n: int, start: int, chunk: int, threads: int):
    """Generate, label and resample n light curves in chunks (``make(count, start)``
    builds a batch): only the network inputs (16 KB per light curve, on the device)
    and the labels are kept, so the light curves never need to fit in memory at once.
    Generation of the next chunk (threads on the host) overlaps the labelling of the
    current one on the GPU."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from . import learned, synth

    def gen(s0):
        cnt = min(chunk, n - s0)
        per = (cnt + threads - 1) // threads
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(lambda k: make(min(per, cnt - k * per), start + s0 + k * per),
                                [k for k in range(threads) if k * per < cnt]))
        return synth.concat(parts)

    xs, lags, labels = [], [], []
    t0 = time.time()
    with ThreadPoolExecutor(1) as pool:
        fut = pool.submit(gen, 0)
        for s0 in range(0, n, chunk):
            b = fut.result()
            if s0 + chunk < n:
                fut = pool.submit(gen, s0 + chunk)
            x, lag, lab, _ = learned.labelled_inputs(b)
            torch.cuda.synchronize()
            xs.append(x)
            lags.append(lag)
            labels.append(lab)
            log("labelled %d / %d light curves (%d periods so far, %.0f s)"
                % (s0 + b.n_stars, n, int(sum((l >= 0).sum() for l in labels)), time.time() - t0))
            del b
    return torch.cat(xs), torch.cat(lags), np.concatenate(labels)


def evaluate(batch, net, tag: str, conf: float = 0.9, topk: int = 8, reps: int = 3):
    from . import learned
    out, _, _ = learned.time_paths(batch, net, reps=reps, conf=conf, topk=topk)
    log("%s: recovery %d/%d = %.4f, exact index %d, fallback %.3f, searched %.3f, plain %.1f ms, "
        "learned %.1f ms, speed-up %.2fx" % (tag, out["recovered"], out["plain_detections"], out["recovery"],
                                              out["exact_index"], out["fallback_fraction"],
                                              out["searched_fraction"], out["plain_ms"], out["learned_ms"],
                                              out["speedup"]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=8192)
    ap.add_argument("--n-eval", type=int, default=2048)
    ap.add_argument("--max-sectors", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--conf", type=float, default=0.9)
    ap.add_argument("--sweep", default="", help="comma-separated confidence thresholds to evaluate after training")
    ap.add_argument("--topk", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--recipe", choices=("cfg3", "mixed"), default="cfg3")
    ap.add_argument("--out", default="")
    ap.add_argument("--report", default="")
    ap.add_argument("--stream-chunk", type=int, default=0,
                    help="generate and label the training set in chunks of this many light curves (cfg3 recipe)")
    ap.add_argument("--threads", type=int, default=8, help="host threads generating light curves")
    ap.add_argument("--eval-reps", type=int, default=3)
    args = ap.parse_args(argv)

    import torch
    from . import learned, synth
    assert torch.cuda.is_available(), "training runs on the GPU"
    t0 = time.time()
    evalb = synth.config3(args.n_eval, start=args.n_train, max_sectors=args.max_sectors)
    eval1 = None
    if args.recipe == "mixed":
        half = args.n_train // 2
        train = synth.concat([synth.config3(half, start=0, max_sectors=args.max_sectors),
                              synth.config1(args.n_train - half, start=CFG1_TRAIN_START)])
        eval1 = synth.config1(args.n_eval, start=CFG1_EVAL_START)
    elif not args.stream_chunk:
        train = synth.config3(args.n_train, start=0, max_sectors=args.max_sectors)
    t1 = time.time()
    if args.stream_chunk:
        if args.recipe != "cfg3":
            raise SystemExit("--stream-chunk supports the cfg3 recipe")
        x, lag, labels = labelled_streamed(
            lambda c, st: synth.config3(c, start=st, max_sectors=args.max_sectors), args.n_train, 0,
            args.stream_chunk, args.threads)
        n_train = args.n_train
    else:
        log("generated %d + %d light curves (%.1f s)" % (train.n_stars, evalb.n_stars, time.time() - t0))
        x, lag, labels, _ = labelled(train)
        n_train = train.n_stars
    log("labelled by the plain search: %d periods, %d null (%.1f s)" % ((labels >= 0).sum(), (labels < 0).sum(),
                                                                        time.time() - t1))
    net = learned.ProposalNet(seed=args.seed)
    before = evaluate(evalb, net, "untrained", args.conf, reps=args.eval_reps)
    t2 = time.time()
    hist = learned.train(net, x, lag, labels, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=args.seed,
                         log=log)
    torch.cuda.synchronize()
    log("trained %d steps (%.1f s)" % (net.step, time.time() - t2))
    after = evaluate(evalb, net, "trained", args.conf, args.topk, reps=args.eval_reps)
    sweep = {}
    for c in [float(v) for v in args.sweep.split(",") if v]:
        sweep[str(c)] = evaluate(evalb, net, "trained, conf %.3f" % c, c, args.topk, reps=args.eval_reps)
    sweep1 = {}
    if eval1 is not None:
        for c in [args.conf] + [float(v) for v in args.sweep.split(",") if v]:
            sweep1[str(c)] = evaluate(eval1, net, "trained, one-sector boxes, conf %.3f" % c, c, args.topk)
    rep = dict(n_train=n_train, n_eval=evalb.n_stars, max_sectors=args.max_sectors, epochs=args.epochs,
               batch=args.batch, lr=args.lr, conf=args.conf, steps=net.step, loss_first=hist[0],
               loss_last=hist[-1], label_periods=int((labels >= 0).sum()), untrained=before, trained=after, sweep=sweep,
               topk=args.topk, recipe=args.recipe, sweep_one_sector=sweep1)
    if args.out:
        np.save(args.out, net.params_host())
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
