"""Benchmark of the MI355X BLS + S/N hot path.

One step = the whole path over one batch resident in HBM: bls_prepare (normalise,
fixed-point prefix sums) -> bls_search_batch (fold, boundary accumulation, duration/
phase scan) -> bls_snr (Sturges median-binned trend, MAD sigma, argmax).

Default workload: 4096 synthetic one-sector stars at 200-s cadence (11,405 points
each), per-star Keplerian grids (Pmin at a = 2 R*, Pmax from the data), plain
FP64-phase path.  Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "stars/hour at sector scale + BLS cells/s; learned vs plain recovery at 1 GPU"
# FP64 VALU issue rate of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12
# non-FMA FP64 operations per second (the 78.6 TFLOP/s figure counts an FMA as two).
FP64_OPS_PEAK = 256 * 64 * 2.4e9
OPS_PER_CELL = 4  # DMUL (dt f), FRACT, DMUL (phase nb), CVT (bin index)


COUNTERS = os.path.join(ROOT, "profiles", "k_search_cfg1_counters.json")


def search_sources_digest() -> str:
    """Digest of the code (comments and blank lines removed) of the sources that
    define the search kernel and its work items: the counters go stale when it
    changes."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in ("paper_2302_01293_amd/csrc/search.hip", "paper_2302_01293_amd/csrc/plan.hpp",
                "paper_2302_01293_amd/csrc/plan.cpp"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per k_search launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (scaled by a plain copy's readings), if they were taken on this
    workload with the current kernel sources; else None."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("workload") != workload or c.get("source_sha256") != search_sources_digest():
        return None
    return float(c["bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, n_stars: int = 0):
    from paper_2302_01293_amd import synth
    if name == "cfg0":
        return synth.config0(), "1 star, 27.4 d at 30-min cadence, P 0.5-13.7 d, plain FP64"
    if name == "cfg1":
        return synth.config1(), "4096 stars x 1 sector at 200 s (11,405 pts), Pmin a=2R*, plain FP64"
    if name == "cfg2":
        n = n_stars or 16384
        return synth.config2(n), "%d stars, 1-13 sectors at 200 s (uneven, missing sectors)" % n
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(batch, n_sample: int, seed: int = 7):
    """The oracle as it stands, on a bounded random sample of the same workload."""
    from oracle import oracle
    rng = np.random.default_rng(seed)
    S = batch.n_stars
    sample = np.sort(rng.choice(S, size=min(n_sample, S), replace=False))
    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.batch(batch.t, batch.y, batch.w, batch.offsets, batch.rho, batch.pmin, batch.pmax,
                 stars=sample, nthreads=cores)
    dt = time.perf_counter() - t0
    return dict(value=len(sample) / dt * 3600.0, unit="stars/hour", cores=cores, kind="oracle",
                sample="%d random stars of the %d-star workload, full spectrum + S/N each (%.1f s)"
                       % (len(sample), S, dt))


def learned_vs_plain(batch, conf: float, topk: int):
    """Recovery of the plain detections and device-time ratio of the learned path
    (committed trained weights) on the benchmark's own stars."""
    from paper_2302_01293_amd import learned
    path = os.path.join(ROOT, "paper_2302_01293_amd", "pp_weights.npy")
    net = learned.ProposalNet(np.load(path))
    r, _, _ = learned.time_paths(batch, net, reps=3, conf=conf, topk=topk)
    r.update(conf=conf, topk=topk, weights="paper_2302_01293_amd/pp_weights.npy")
    log("learned: recovery %d/%d, speed-up %.2fx, fallback %.3f, searched %.3f" % (
        r["recovered"], r["plain_detections"], r["speedup"], r["fallback_fraction"], r["searched_fraction"]))
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--stars", type=int, default=0, help="use only the first N stars of the workload")
    ap.add_argument("--precision", type=int, default=0,
                    help="0: exact int64 bin sums (plain FP64 path); 1: packed reduced-precision sums")
    ap.add_argument("--cpu-sample", type=int, default=768)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal comparison (trained weights vs the plain path)")
    ap.add_argument("--learned-conf", type=float, default=0.95)
    ap.add_argument("--learned-topk", type=int, default=12)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size kernel "
                         "for scaling the profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(stars shard independently; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_01293_amd.device import DeviceSearch

    assert torch.cuda.is_available(), "no GPU"
    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written" % (args.copy_calibration_mib,
                                                                  args.copy_calibration_mib))
        del src, dst
    log("generating workload", args.workload)
    batch, desc = make_workload(args.workload, args.stars if args.workload == "cfg2" else 0)
    if args.stars and args.stars < batch.n_stars:
        batch = batch.subset(np.arange(args.stars))
        desc += " (first %d stars)" % args.stars
    log("stars", batch.n_stars, "points", batch.n_points)
    from paper_2302_01293_amd import _lib
    ds = DeviceSearch.from_batch(batch, _lib.default_params(precision=args.precision))
    if args.precision:
        desc += ", packed reduced-precision sums"
    nfs = np.diff(ds.plan.freq_offsets)
    npts = np.diff(batch.offsets)
    cells = float(np.sum(nfs.astype(np.float64) * npts))
    log("frequencies", int(nfs.sum()), "cells %.3e" % cells)

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ds.run()
    torch.cuda.synchronize()
    log("warmup done")
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        e = ev[k]
        e[0].record(stream)
        ds.run_prepare()
        e[1].record(stream)
        ds.run_search()
        e[2].record(stream)
        ds.run_snr()
        e[3].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prep = np.mean([ev[k][0].elapsed_time(ev[k][1]) for k in range(args.steps)])
    srch = np.mean([ev[k][1].elapsed_time(ev[k][2]) for k in range(args.steps)])
    snr = np.mean([ev[k][2].elapsed_time(ev[k][3]) for k in range(args.steps)])
    step_ms = np.mean([ev[k][0].elapsed_time(ev[k][3]) for k in range(args.steps)])
    log("per step ms: prepare %.3f search %.3f snr %.3f total %.3f (wall/step %.3f)"
        % (prep, srch, snr, step_ms, wall * 1e3 / args.steps))
    res = ds.results_host()
    inj = np.asarray(batch.truth.get("injected", np.zeros(batch.n_stars, bool)), bool)
    if inj.any():
        hit = np.abs(res["period"][inj] / np.asarray(batch.truth["period"])[inj] - 1) < 0.01
        log("injections recovered at the best-S/N period: %d / %d" % (hit.sum(), inj.sum()))

    achieved = OPS_PER_CELL * cells / (srch * 1e-3) / 1e12
    peak = FP64_OPS_PEAK / 1e12
    out = {
        "metric": METRIC,
        "value": batch.n_stars / (step_ms * 1e-3) * 3600.0,
        "unit": "stars/hour",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + desc, "stars": batch.n_stars,
                   "points": batch.n_points, "frequencies": int(nfs.sum()), "cells": cells},
        "cells_per_s": cells / (srch * 1e-3),
        "kernel_ms": {"prepare": prep, "search": srch, "snr": snr},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(args.workload) if not (args.stars or args.precision) else None,
                     "kernel": "k_search (fold + boundary accumulation + scan)"},
    }
    if not args.no_learned:
        log("learned proposal vs plain on the same stars ...")
        out["learned"] = learned_vs_plain(batch, args.learned_conf, args.learned_topk)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on a sample ...")
        out["cpu_baseline"] = cpu_baseline(batch, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
