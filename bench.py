"""Benchmark of the MI355X BLS + S/N hot path.

One step = the whole path over one batch of stars whose light curves are already
resident in HBM: the host plan (C++: bounds, Keplerian grid, work items; built
while the previous step runs on the GPU), the descriptor upload, bls_prepare
(normalise, fixed-point prefix sums), bls_search_batch (fold, boundary
accumulation, duration/phase scan), bls_snr (Sturges median-binned trend, MAD
sigma, argmax) and the copy of the per-star results back to the host.

Default workload: the sector-scale mix -- every step is a new batch of 256 stars
of 1-26 contiguous TESS sectors at 200-s cadence (11k-297k points, up to ~2 yr
baselines, periods up to half the longest stretch, 10% injected boxes), per-star
Keplerian grids (Pmin at a = 2 R*), plain FP64-phase path with exact bin sums.
``--workload cfg1`` (4096 one-sector stars, the same batch every step) and
``cfg2`` / ``cfg0`` remain available.  Prints ONE JSON line on stdout; progress
goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
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


def counters_path(workload: str) -> str:
    return os.path.join(ROOT, "profiles", "k_search_%s_counters.json" % workload)


def search_sources_digest() -> str:
    """Digest of the code (comments and blank lines removed) of the sources that
    define the search kernel and its work items: the counters go stale when it
    changes."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in ("paper_2302_01293_amd/csrc/search.hip", "paper_2302_01293_amd/csrc/counts.hpp",
                "paper_2302_01293_amd/csrc/plan.hpp", "paper_2302_01293_amd/csrc/plan.cpp"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(workload: str, key: dict, cells_per_launch: float):
    """HBM bytes per search call from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs (scaled by a plain copy's readings), if they were taken on this workload
    (same batch shape) with the current kernel sources; else None.  Runs that record
    bytes per cell (a workload whose batches differ from step to step) are scaled to
    the timed calls' mean cells."""
    try:
        with open(counters_path(workload)) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256") != search_sources_digest() or c.get("key") != key:
        return None
    if "bytes_per_cell" in c:
        return float(c["bytes_per_cell"]) * cells_per_launch
    return float(c["bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _threads() -> int:
    """Host threads for generation and the CPU baseline: the process's CPU share
    (affinity), capped by OMP_NUM_THREADS when it is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def measure_ceilings(copy_mib: int = 2048) -> dict:
    """Unit rates measured on this GPU by libmi355ceil.so (csrc/ceilings.hip): the
    FP64 multiply / fract / convert issue costs, the 64-bit LDS atomic cost per wave
    instruction, and an HBM copy rate, next to which the vendor peaks are quoted."""
    import ctypes
    path = os.path.join(ROOT, "paper_2302_01293_amd", "libmi355ceil.so")
    L = ctypes.CDLL(path)
    L.mi355_ceilings.restype = ctypes.c_int
    L.mi355_ceilings.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    out = np.zeros(9)
    st = L.mi355_ceilings(out.ctypes.data, int(copy_mib) << 20)
    if st != 0:
        raise RuntimeError("mi355_ceilings failed (hipError %d)" % st)
    clk = out[7] * 1e9
    return {"dmul_simd_cycles": out[0], "fract_simd_cycles": out[1], "cvt_plus_xor_simd_cycles": out[2],
            "iadd_simd_cycles": out[3], "lds_add_u64_cu_cycles_64_lanes": out[4],
            "lds_add_u64_cu_cycles_1_lane": out[5], "lds_add_u32_cu_cycles_64_lanes": out[8],
            "hbm_copy_GBps": out[6], "clock_GHz": out[7],
            "fp64_ops_per_s": 1024 * 64 / out[0] * clk,
            "lds_atomic_instr_per_s": 256 / out[4] * clk}


def equal_weights(batch) -> np.ndarray:
    """Stars whose points of nonzero weight all carry the same weight: the search
    accumulates counts of weighted points for them (their fixed-point weights are
    then equal too)."""
    out = np.zeros(batch.n_stars, bool)
    for s in range(batch.n_stars):
        w = batch.star(s)[2]
        w = w[w > 0]
        out[s] = len(w) > 0 and bool(np.all(w == w[0]))
    return out


def make_workload(name: str, n_stars: int, batch_stars: int, steps: int):
    """List of batches (one per step for the sector-scale mix; one shared batch
    otherwise) and a description."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2302_01293_amd import synth
    if name == "cfg0":
        return [synth.config0()], "1 star, 27.4 d at 30-min cadence, P 0.5-13.7 d, plain FP64"
    if name == "cfg1":
        b = synth.config1(n_stars or 4096)
        return [b], "%d stars x 1 sector at 200 s (11,405 pts), Pmin a=2R*, plain FP64" % b.n_stars
    if name == "cfg2":
        n = n_stars or 16384
        return [synth.config2(n)], "%d stars, 1-13 sectors at 200 s (uneven, missing sectors)" % n
    if name == "cfg4":
        B = batch_stars

        def gen(k):
            return synth.config4(B, start=k * B)

        total = B * steps
        with ThreadPoolExecutor(_threads()) as ex:
            batches = list(ex.map(gen, range(steps)))
        return batches, ("sector-scale mix: %d new stars per step (%d in all), 1-26 contiguous sectors "
                         "at 200 s (11k-297k pts), 10%% boxes, Pmin a=2R*, plain FP64" % (B, total))
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline_cells(batches, stride: int, cells_per_star: float, params=None):
    """The oracle as it stands on a bounded sample of the benchmark's stars: one star
    per sector count (stratified), every ``stride``-th frequency of its grid (each
    frequency searched in full: fold, bins, every window).  Throughput in cells/s
    is extrapolated to stars/hour with the workload's mean cells per star.  The same
    stars are then searched on the GPU with the benchmark's parameters and the SR at
    those frequencies compared with the oracle's (relative error per result, and the
    share of equal best windows)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle
    seen = {}
    for bi, b in enumerate(batches):
        for s in range(b.n_stars):
            k = int(b.truth["n_sectors"][s])
            if k not in seen:
                seen[k] = (bi, s)
    picks = [seen[k] for k in sorted(seen)]
    jobs = []
    for bi, s in picks:
        b = batches[bi]
        t, y, w = b.star(s)
        st, bd = oracle.bounds(t, w, float(b.rho[s]))
        idx = np.arange(0, bd.nf, stride, dtype=np.int64)
        jobs.append((t, y, w, float(b.rho[s]), idx, len(t) * len(idx)))
    cores = _threads()

    def run(j):
        t, y, w, rho, idx, _ = j
        return oracle.bls_star_at(t, y, w, idx, rho)

    oracle.lib()
    order = sorted(range(len(jobs)), key=lambda i: -jobs[i][5])
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        specs = list(ex.map(run, [jobs[i] for i in order]))
    dt = time.perf_counter() - t0
    spec_of = {i: sp for i, sp in zip(order, specs)}
    cells = float(sum(j[5] for j in jobs))
    cps = cells / dt
    sr_err = None
    if params is not None:
        import torch
        from paper_2302_01293_amd import synth
        from paper_2302_01293_amd.device import DeviceSearch
        sub = synth.concat([batches[bi].subset([s]) for bi, s in picks])
        ds = DeviceSearch.from_batch(sub, params, want_snr=False)
        ds.run()
        torch.cuda.synchronize()
        sr_g, best_g = ds.sr_host(), ds.best_host()
        rels, same, tot = [], 0, 0
        for i, (t, y, w, rho, idx, _) in enumerate(jobs):
            f0 = int(ds.plan.freq_offsets[i])
            o = spec_of[i]
            g = sr_g[f0 + idx]
            rels.append(np.abs(g - o.sr) / np.maximum(np.abs(o.sr), 1e-300))
            bg = best_g[f0 + idx]
            same += int(np.sum((bg["m"] == o.m) & (bg["j"] == o.j)))
            tot += len(idx)
        rel = np.concatenate(rels)
        sr_err = dict(results=int(tot), stars=len(jobs), max_rel=float(rel.max()),
                      p99_rel=float(np.percentile(rel, 99)), median_rel=float(np.median(rel)),
                      best_window_equal=same / tot)
        del ds
    return dict(value=cps / cells_per_star * 3600.0, unit="stars/hour", cores=cores, kind="oracle",
                sample=("%d stars of the workload (one per sector count %d-%d), 1 in %d grid frequencies "
                        "of each: %.3g cells in %.1f s = %.3g cells/s, extrapolated with the workload's "
                        "%.3g cells per star (the S/N step, O(N_f log N_f), is not timed)"
                        % (len(jobs), min(seen), max(seen), stride, cells, dt, cps, cells_per_star)),
                cells_per_s=cps, nproc=os.cpu_count(), cpu_model=cpu_model(),
                single_core_s_per_star=cells_per_star / (cps / cores), sr_vs_oracle=sr_err)


def cpu_baseline_full(batch, n_sample: int, seed: int = 7):
    """The oracle as it stands on a bounded random sample of whole stars."""
    from oracle import oracle
    rng = np.random.default_rng(seed)
    S = batch.n_stars
    sample = np.sort(rng.choice(S, size=min(n_sample, S), replace=False))
    cores = _threads()
    t0 = time.perf_counter()
    oracle.batch(batch.t, batch.y, batch.w, batch.offsets, batch.rho, batch.pmin, batch.pmax,
                 stars=sample, nthreads=cores)
    dt = time.perf_counter() - t0
    return dict(value=len(sample) / dt * 3600.0, unit="stars/hour", cores=cores, kind="oracle",
                sample="%d random stars of the %d-star workload, full spectrum + S/N each (%.1f s)"
                       % (len(sample), S, dt), nproc=os.cpu_count(), cpu_model=cpu_model())


class Step:
    """One batch on the device: input tensors, plan, and the per-step buffers."""

    def __init__(self, batch, dev):
        import torch
        self.batch = batch
        self.t = torch.as_tensor(batch.t).to(dev)
        self.y = torch.as_tensor(batch.y).to(dev)
        self.w = torch.as_tensor(batch.w).to(dev)
        self.plan = None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg4")
    ap.add_argument("--stars", type=int, default=0, help="cfg1/cfg2: number of stars")
    ap.add_argument("--batch-stars", type=int, default=256, help="cfg4: new stars per step")
    ap.add_argument("--precision", type=int, default=0,
                    help="0: exact int64 bin sums (plain FP64 path); 1: packed reduced-precision sums")
    ap.add_argument("--cpu-sample", type=int, default=768, help="cfg1/cfg2: whole stars timed on the CPU")
    ap.add_argument("--cpu-stride", type=int, default=32,
                    help="cfg4: the CPU baseline searches every n-th frequency of its sample stars")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal comparison (trained weights vs the plain path)")
    ap.add_argument("--learned-batches", type=int, default=8,
                    help="cfg4: steps' batches on which the learned path is compared with the plain one")
    ap.add_argument("--learned-points", default="0.9:8:4,0.5:8:4,0.9:8:0,0:0:4,0:0:2,0:8:2",
                    help="operating points of the learned path, conf:topk:coarse_peaks (coarse_peaks > 0: "
                         "windows guided by that many peaks of the coarse S/N spectrum, no blanket window "
                         "beyond 100 d; topk 0: no network windows); the first is the headline")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the unit-rate microbenchmarks")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip timing the exact-duration and rebinning search variants")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default schedule instead of tuning it on the first batch")
    ap.add_argument("--tune-sample", type=int, default=0,
                    help="stars of the first batch the autotuner times (0: the whole batch)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size kernel "
                         "for scaling the profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(stars shard independently; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_01293_amd import _lib

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda")
    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written" % (args.copy_calibration_mib,
                                                                  args.copy_calibration_mib))
        del src, dst
    t_gen = time.perf_counter()
    log("generating workload", args.workload)
    batches, desc = make_workload(args.workload, args.stars, args.batch_stars, args.steps)
    log("generated %d batch(es), %d stars, %d points (%.1f s)" % (
        len(batches), sum(b.n_stars for b in batches), sum(b.n_points for b in batches),
        time.perf_counter() - t_gen))
    params = _lib.default_params(precision=args.precision)
    if args.precision:
        desc += ", packed reduced-precision sums"
    tuned = None
    if not args.no_autotune:
        # Schedule (work-item size, per-item frequency cap, large-shape threshold)
        # by coordinate descent on the first batch (the default schedule among the
        # candidates), before the clock; results do not depend on it.
        from paper_2302_01293_amd import autotune
        t_tune = time.perf_counter()
        tuned = autotune.tune(batches[0], params, n_sample=args.tune_sample or batches[0].n_stars, reps=1,
                              use_cache=False, axes=("tile_cells", "item_freqs", "big_points"),
                              candidates=(3 << 20, 12 << 20), item_freqs=(64, 256), big_points=(50_000, 200_000),
                              warmup=False)
        # adopt the pick only when it beats the default by more than timing noise, so
        # that the timed schedule (and the committed counters taken with it) is stable
        d_ms, b_ms = tuned.get("default_ms"), tuned.get("best_ms")
        tuned["adopted"] = bool(d_ms and b_ms and b_ms < 0.98 * d_ms)
        if tuned["adopted"]:
            for k in ("tile_cells", "item_freqs", "big_points"):
                setattr(params, k, int(tuned[k]))
        tuned["seconds"] = time.perf_counter() - t_tune
        log("autotuner: best tile_cells %d, item_freqs %d, big_points %d at %.1f ms against the default's %.1f ms "
            "on the first batch: %s (%.1f s)" % (tuned["tile_cells"], tuned["item_freqs"], tuned["big_points"], b_ms,
                                               d_ms, "adopted" if tuned["adopted"] else "default kept", tuned["seconds"]))

    # Every batch's light curves go to HBM before the clock starts.
    steps = [Step(b, dev) for b in batches]
    # Per-step sizes (the plans are built again inside the timed loop for a new batch).
    sizes = []
    for st in steps:
        pl = _lib.Plan(st.batch.t, st.batch.y, st.batch.w, st.batch.offsets, st.batch.rho,
                       st.batch.pmin, st.batch.pmax, params)
        nfs = np.diff(pl.freq_offsets)
        star_cells = nfs.astype(np.float64) * np.diff(st.batch.offsets)
        sizes.append(dict(nf=int(pl.n_freq), ws=int(pl.workspace_bytes), cells=float(np.sum(star_cells)),
                          equal_weight_cells=float(np.sum(star_cells[equal_weights(st.batch)]))))
        if len(steps) == 1:
            st.plan = pl
        else:
            pl.close()
    ws_bytes = max(s["ws"] for s in sizes)
    nf_max = max(s["nf"] for s in sizes)
    s_max = max(b.n_stars for b in batches)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    sr = torch.empty(nf_max, dtype=torch.float64, device=dev)
    best = torch.empty(nf_max * _lib.BEST_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    res_dev = torch.empty(s_max * _lib.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    h = int(stream.cuda_stream)
    n_batches = len(steps)
    log("per-step batch: %.3g cells on average, %d frequencies at most, workspace %.2f GB"
        % (np.mean([s["cells"] for s in sizes]), nf_max, ws_bytes / 1e9))

    def run_step(k, ev=None, res_host=None):
        st = steps[k % n_batches]
        b = st.batch
        if n_batches > 1 or st.plan is None:
            st.plan = _lib.Plan(b.t, b.y, b.w, b.offsets, b.rho, b.pmin, b.pmax, params)
        pl = st.plan
        if ev is not None:
            ev[0].record(stream)
        pl.upload(ws_ptr, ws_bytes, h)
        pl.prepare(ws_ptr, st.t.data_ptr(), st.y.data_ptr(), st.w.data_ptr(), h)
        if ev is not None:
            ev[1].record(stream)
        pl.search(ws_ptr, sr.data_ptr(), best.data_ptr(), None, 0, h)
        if ev is not None:
            ev[2].record(stream)
        pl.snr(ws_ptr, sr.data_ptr(), best.data_ptr(), None, res_dev.data_ptr(), h)
        if ev is not None:
            ev[3].record(stream)
        if res_host is not None:
            res_host.copy_(res_dev[:b.n_stars * _lib.RESULT_DTYPE.itemsize], non_blocking=True)
        return pl

    keep = []
    for k in range(args.warmup):
        keep.append(run_step(k))
        keep = keep[-2:]
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    res_host = [torch.empty(steps[k % n_batches].batch.n_stars * _lib.RESULT_DTYPE.itemsize,
                            dtype=torch.uint8, pin_memory=True) for k in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        keep.append(run_step(k, ev[k], res_host[k]))
        keep = keep[-2:]          # a plan's host descriptors stay alive while its copy may run
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    del keep
    prep = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(args.steps)])
    srch = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(args.steps)])
    snr = np.array([ev[k][2].elapsed_time(ev[k][3]) for k in range(args.steps)])
    dev_ms = np.array([ev[k][0].elapsed_time(ev[k][3]) for k in range(args.steps)])
    step_ms = wall * 1e3 / args.steps
    n_timed = sum(steps[k % n_batches].batch.n_stars for k in range(args.steps))
    cells = float(sum(sizes[k % n_batches]["cells"] for k in range(args.steps)))
    log("per step ms (device): prepare %.3f search %.3f snr %.3f total %.3f; wall/step %.3f"
        % (prep.mean(), srch.mean(), snr.mean(), dev_ms.mean(), step_ms))
    results = [res_host[k].numpy().view(_lib.RESULT_DTYPE).copy() for k in range(args.steps)]
    # Post-BLS statistics of the last step's batch (outside the timed step): per-star
    # counts and criteria (bls_stats) and the trapezoid fit with noise and S/N_pink
    # (bls_fit), timed with HIP events on the stream.
    post = None
    last = steps[(args.steps - 1) % n_batches]
    if last.plan is not None:
        nS = last.batch.n_stars
        st_dev = torch.empty(nS * _lib.STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        fit_dev = torch.empty(nS * _lib.FIT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        last.plan.stats(ws_ptr, last.t.data_ptr(), last.y.data_ptr(), last.w.data_ptr(), best.data_ptr(),
                        res_dev.data_ptr(), st_dev.data_ptr(), 9.0, h)
        e1.record(stream)
        last.plan.fit(ws_ptr, last.t.data_ptr(), last.y.data_ptr(), last.w.data_ptr(), res_dev.data_ptr(),
                      fit_dev.data_ptr(), 9.0, 9.0, h)
        e2.record(stream)
        torch.cuda.synchronize()
        fr = fit_dev.cpu().numpy().view(_lib.FIT_DTYPE)
        post = {"stars": nS, "stats_ms": e0.elapsed_time(e1), "fit_ms": e1.elapsed_time(e2),
                "candidates": int(fr["candidate"].sum()),
                "fit_iterations_mean": float(fr["iterations"][fr["status"] == 0].mean())
                if np.any(fr["status"] == 0) else 0.0}
        log("post-BLS statistics of %d stars: bls_stats %.3f ms, bls_fit %.3f ms, %d candidates"
            % (nS, post["stats_ms"], post["fit_ms"], post["candidates"]))
    n_inj = n_hit = 0
    for k in range(args.steps):
        b = steps[k % n_batches].batch
        inj = np.asarray(b.truth.get("injected", np.zeros(b.n_stars, bool)), bool)
        if inj.any():
            p = results[k]["period"][inj]
            pt = np.asarray(b.truth["period"])[inj]
            n_hit += int(np.sum(np.abs(p / pt - 1) < 0.01))
            n_inj += int(inj.sum())
    log("injections recovered at the best-S/N period: %d / %d" % (n_hit, n_inj))

    search_s = float(srch.sum()) * 1e-3
    achieved = OPS_PER_CELL * cells / search_s / 1e12
    peak = FP64_OPS_PEAK / 1e12
    key = dict(workload=args.workload, batch_stars=args.batch_stars if args.workload == "cfg4" else None,
               stars=args.stars or None, precision=args.precision, tile_cells=int(params.tile_cells),
               item_freqs=int(params.item_freqs), big_points=int(params.big_points))
    traffic = measured_traffic(args.workload, key, cells / args.steps)
    out = {
        "metric": METRIC,
        "value": n_timed / (wall) * 3600.0,
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
        "config": {"workload": args.workload + ": " + desc, "stars_timed": n_timed,
                   "points_timed": int(sum(steps[k % n_batches].batch.n_points for k in range(args.steps))),
                   "frequencies_timed": int(sum(sizes[k % n_batches]["nf"] for k in range(args.steps))),
                   "cells_timed": cells},
        "cells_per_s": cells / search_s,
        "cells_per_s_end_to_end": cells / wall,
        "kernel_ms_per_step": {"prepare": float(prep.mean()), "search": float(srch.mean()),
                               "snr": float(snr.mean()), "device_total": float(dev_ms.mean())},
        "injections_recovered": [n_hit, n_inj],
        "post_bls": post,
        "schedule": None if tuned is None else {k: tuned[k] for k in ("tile_cells", "item_freqs", "big_points",
                                                                       "times_ms", "default_ms", "best_ms",
                                                                       "adopted", "seconds")},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_search (fold + boundary accumulation + scan; all launches of "
                               "bls_search_batch)"},
    }
    # HBM fractions of the two streaming kernels of the step (algorithmic bytes: the
    # preparation reads t, y, w and writes dt and the two prefix sums, 48 B per point;
    # the S/N step reads SR once, 8 B per frequency, and writes 88 B per star); the
    # preparation interval also holds the plan's descriptor upload
    pts_step = float(np.mean([steps[k % n_batches].batch.n_points for k in range(args.steps)]))
    nf_step = float(np.mean([sizes[k % n_batches]["nf"] for k in range(args.steps)]))
    st_step = float(np.mean([steps[k % n_batches].batch.n_stars for k in range(args.steps)]))
    other = {}
    for name, by, ms in (("k_prepare", 48.0 * pts_step, float(prep.mean())),
                         ("k_snr", 8.0 * nf_step + 88.0 * st_step, float(snr.mean()))):
        gbs = by / (ms * 1e-3) / 1e9
        other[name] = {"bound": "hbm", "bytes_per_step": by, "ms": ms, "achieved": gbs, "peak": 8000.0,
                       "unit": "GB/s", "frac": gbs / 8000.0}
    out["other_kernels"] = other
    if not args.no_ceilings:
        c = measure_ceilings()
        out["ceilings"] = c
        out["roofline"]["measured_peak"] = c["fp64_ops_per_s"] / 1e12
        out["roofline"]["frac_of_measured"] = achieved / (c["fp64_ops_per_s"] / 1e12)
        # The fold's other bound: each wave-step (64 points at one frequency) adds the
        # boundary's values to LDS whenever any of its lanes enters a new bin, which
        # on these grids is every step (3-25 points per bin visit): two ds_add_u64
        # (weight and residual prefixes), or one ds_add_u64 and one ds_add_u32 for
        # stars of equal weights (counts of weighted points); at the measured cycles
        # per such instruction, weighted by the cells of each kind of star, the LDS
        # caps the search at this many cells/s.
        c64, c32 = c["lds_add_u64_cu_cycles_64_lanes"], c["lds_add_u32_cu_cycles_64_lanes"]
        if args.precision == 1:  # one packed 64-bit sum per boundary
            cyc, basis = c64, "1 ds_add_u64 (packed sums) per 64-cell wave-step at %.2f CU-cycles" % c64
        else:
            eq = float(sum(sizes[k % n_batches]["equal_weight_cells"] for k in range(args.steps))) / cells
            cyc = eq * (c64 + c32) + (1.0 - eq) * 2.0 * c64
            basis = ("per 64-cell wave-step, ds_add_u64 (%.2f CU-cycles) + ds_add_u32 (%.2f) on the %.1f%% of cells "
                     "in stars of equal weights, 2 ds_add_u64 on the rest" % (c64, c32, 100.0 * eq))
        lds_cap = 256 * c["clock_GHz"] * 1e9 / cyc * 64.0
        out["roofline"]["lds_atomic_bound"] = {"cells_per_s": lds_cap, "frac": (cells / search_s) / lds_cap,
                                               "basis": basis}
        log("ceilings: DMUL %.2f FRACT %.2f SIMD-cycles per wave instruction; 64-bit LDS atomic %.2f CU-cycles; "
            "copy %.0f GB/s" % (c["dmul_simd_cycles"], c["fract_simd_cycles"], c["lds_add_u64_cu_cycles_64_lanes"],
                                c["hbm_copy_GBps"]))
    if not args.no_learned:
        out["learned"] = learned_vs_plain(args, steps, results, dev_ms, params)
    if not args.no_variants:
        out["variants"] = measure_variants()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on a sample ...")
        if args.workload == "cfg4":
            out["cpu_baseline"] = cpu_baseline_cells([s.batch for s in steps], args.cpu_stride,
                                                     cells / n_timed, params)
            e = out["cpu_baseline"]["sr_vs_oracle"]
            log("GPU SR against the oracle at the sampled frequencies: max %.2e, p99 %.2e, median %.2e relative "
                "over %d results; best windows equal for %.6f" % (e["max_rel"], e["p99_rel"], e["median_rel"],
                                                                   e["results"], e["best_window_equal"]))
        else:
            out["cpu_baseline"] = cpu_baseline_full(batches[0], args.cpu_sample)
        log("cpu baseline: %.4g stars/hour" % out["cpu_baseline"]["value"])
    print(json.dumps(out), flush=True)


def measure_variants(n_stars: int = 1024) -> dict:
    """Search time of the two search variants (exact circular duration; per-duration
    rebinning) beside the plain search on the same one-sector stars (the 200-s
    one-sector recipe), each the best of three calls timed with HIP events on the
    launch stream, inputs resident in HBM."""
    import torch
    from paper_2302_01293_amd import _lib, synth
    from paper_2302_01293_amd.device import DeviceSearch
    b = synth.config1(n_stars, start=7_000_000)
    out = {"stars": b.n_stars, "points": int(b.n_points), "workload": "one-sector stars at 200 s (cfg1 recipe)"}
    for name, kw in (("plain", {}), ("exact_duration", dict(exact_duration=1)), ("rebin", dict(rebin=1))):
        ds = DeviceSearch.from_batch(b, _lib.default_params(**kw), want_snr=False)
        ds.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best_ms = None
        for _ in range(3):
            ds.run_prepare()
            e0.record()
            ds.run_search()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best_ms = ms if best_ms is None else min(best_ms, ms)
        cells = float(np.sum(np.diff(b.offsets) * np.diff(ds.plan.freq_offsets)))
        out[name] = {"search_ms": best_ms, "cells": cells, "cells_per_s": cells / (best_ms * 1e-3)}
        del ds
    log("variants on %d one-sector stars: plain %.1f ms, exact duration %.1f ms, rebinning %.1f ms"
        % (b.n_stars, out["plain"]["search_ms"], out["exact_duration"]["search_ms"], out["rebin"]["search_ms"]))
    return out


def learned_vs_plain(args, steps, plain_results, plain_ms, params):
    """Recovery of the plain detections and device-time ratio of the learned path
    (committed trained weights) on the benchmark's own stars: the plain results and
    device times are those of the timed steps."""
    import torch

    from paper_2302_01293_amd import learned
    path = os.path.join(ROOT, "paper_2302_01293_amd", "pp_weights.npy")
    net = learned.ProposalNet(np.load(path))
    nb = min(args.learned_batches, args.steps) if len(steps) > 1 else 1
    stream = torch.cuda.current_stream()
    out = dict(weights="paper_2302_01293_amd/pp_weights.npy", batches=nb,
               stars=int(sum(steps[k].batch.n_stars for k in range(nb))), points=[])
    for spec in args.learned_points.split(","):
        parts = spec.split(":")
        conf, topk = float(parts[0]), int(parts[1])
        peaks = int(parts[2]) if len(parts) > 2 else 0
        kw = dict(topk=topk, conf=conf, coarse_peaks=peaks, search_long=peaks == 0)
        t_l = t_p = 0.0
        agg = dict(plain_detections=0, recovered=0, exact_index=0)
        fb = searched = nf_all = 0.0
        conf_stats = dict(confident_detections=0, confident_recovered=0)
        for k in range(nb):
            b = steps[k].batch
            ls = learned.LearnedSearch(b, net, params=params, **kw)
            ls.run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ls.run()
            e1.record(stream)
            torch.cuda.synchronize()
            t_l += e0.elapsed_time(e1)
            t_p += float(plain_ms[k])
            lres = ls.fine.results_host()
            r = learned.recovery(plain_results[k], lres, b.truth)
            for q in agg:
                agg[q] += r[q]
            f = ls.fallback.cpu().numpy().astype(bool)
            rc = learned.recovery(plain_results[k][~f], lres[~f],
                                  {q: np.asarray(v)[~f] for q, v in b.truth.items()})
            conf_stats["confident_detections"] += rc["plain_detections"]
            conf_stats["confident_recovered"] += rc["recovered"]
            fb += float(f.sum())
            searched += ls.searched_fraction() * ls.fine.plan.n_freq
            nf_all += ls.fine.plan.n_freq
            del ls
        n_stars = out["stars"]
        kind = ("network windows" if peaks == 0 else
                "coarse-peak windows only (no network)" if topk == 0 else "network + coarse-peak windows")
        pt = dict(conf=conf, topk=topk, coarse_peaks=peaks, kind=kind, plain_ms=t_p, learned_ms=t_l,
                  speedup=t_p / t_l,
                  fallback_fraction=fb / n_stars, recovery=agg["recovered"] / max(agg["plain_detections"], 1),
                  **agg, **conf_stats)
        pt["searched_fraction"] = searched / nf_all
        log("learned conf %.2f top-%d coarse peaks %d: recovery %d/%d (confident stars %d/%d), speed-up %.2fx, "
            "fallback %.3f" % (conf, topk, peaks, agg["recovered"], agg["plain_detections"],
                               conf_stats["confident_recovered"], conf_stats["confident_detections"], pt["speedup"],
                               pt["fallback_fraction"]))
        out["points"].append(pt)
    # The network's forward pass on the first batch's resampled light curves: the
    # two convolutions are the MFMA work, 2*2048*16*(2*16) + 2*1024*16*(16*8) =
    # 6.29 MFLOP per light curve on BF16 inputs (the autocorrelation and head, FP32
    # and FP64, are in the same launch and not counted).
    b0 = steps[0].batch
    ls = learned.LearnedSearch(b0, net, params=params)
    ls.fine.run_prepare()
    x, lag = learned.resample(ls.fine)
    net.forward(x, lag)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(stream)
    for _ in range(reps):
        net.forward(x, lag)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    flops = 6.291456e6 * b0.n_stars
    out["k_forward"] = {"light_curves": b0.n_stars, "ms": fwd_ms, "mfma_flops": flops, "bound": "mfma",
                        "achieved": flops / (fwd_ms * 1e-3) / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": flops / (fwd_ms * 1e-3) / 1e12 / 2500.0}
    log("network forward on %d light curves: %.3f ms, %.2f TFLOP/s of BF16 MFMA work (%.2e of peak)"
        % (b0.n_stars, fwd_ms, out["k_forward"]["achieved"], out["k_forward"]["frac"]))
    del ls
    h = out["points"][0]
    out["headline"] = dict(kind=h["kind"], conf=h["conf"], topk=h["topk"], coarse_peaks=h["coarse_peaks"],
                           recovery=h["recovery"], speedup=h["speedup"],
                           stars_per_hour=out["stars"] / (h["learned_ms"] * 1e-3) * 3600.0)
    return out


if __name__ == "__main__":
    main()
