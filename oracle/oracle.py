"""Python access to the CPU FP64 oracle (``bls_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The product path never imports it.

The C file is compiled with gcc (``-O2 -fopenmp -ffp-contract=off``) into
``oracle/liboracle_bls.so`` the first time it is needed, or by ``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bls_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_bls.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    """Search parameters; defaults are the paper's (Sec. 2.1 and its footnote)."""
    _fields_ = [
        ("spp", ctypes.c_double),
        ("qmin_fac", ctypes.c_double),
        ("qmax_fac", ctypes.c_double),
        ("dlogq", ctypes.c_double),
        ("noverlap", ctypes.c_int32),
        ("dip_only", ctypes.c_int32),
        ("mad_of_raw", ctypes.c_int32),
        ("exact_duration", ctypes.c_int32),
        ("a_min", ctypes.c_double),
        ("sector_days", ctypes.c_double),
        ("rebin", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


def params(**kw) -> Params:
    p = Params(spp=2.0, qmin_fac=0.5, qmax_fac=2.0, dlogq=0.1, noverlap=3, dip_only=0,
               mad_of_raw=0, exact_duration=0, a_min=2.0, sector_days=27.4, rebin=0, pad_=0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Bounds(ctypes.Structure):
    _fields_ = [
        ("t0", ctypes.c_double), ("tlast", ctypes.c_double), ("T", ctypes.c_double),
        ("pmin", ctypes.c_double), ("pmax", ctypes.c_double), ("krho", ctypes.c_double),
        ("umin", ctypes.c_double), ("umax", ctypes.c_double), ("A", ctypes.c_double),
        ("nf", ctypes.c_int64),
    ]


class Spectrum(ctypes.Structure):
    _fields_ = [
        ("sr", ctypes.c_void_p), ("m", ctypes.c_void_p), ("j", ctypes.c_void_p),
        ("r", ctypes.c_void_p), ("s", ctypes.c_void_p), ("nb", ctypes.c_void_p),
        ("f", ctypes.c_void_p),
    ]


class SnrResult(ctypes.Structure):
    _fields_ = [
        ("i_snr", ctypes.c_int64), ("i_sr", ctypes.c_int64), ("snr_max", ctypes.c_double),
        ("sr_max", ctypes.c_double), ("trend_at", ctypes.c_double), ("sigma", ctypes.c_double),
        ("median_resid", ctypes.c_double), ("status", ctypes.c_int32),
        ("nbins_sturges", ctypes.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.orc_k_sun.restype = d
        L.orc_krho.restype = d
        L.orc_krho.argtypes = [d]
        L.orc_period_at_a.restype = d
        L.orc_period_at_a.argtypes = [d, d]
        L.orc_qcirc.restype = d
        L.orc_qcirc.argtypes = [d, d]
        L.orc_qcirc_exact.restype = d
        L.orc_qcirc_exact.argtypes = [d, d]
        L.orc_rebin_ladder.restype = i32
        L.orc_rebin_ladder.argtypes = [ctypes.POINTER(Params), vp, i32]
        L.orc_bounds.restype = ctypes.c_int
        L.orc_bounds.argtypes = [vp, vp, i64, d, ctypes.POINTER(Params), d, d, ctypes.POINTER(Bounds)]
        L.orc_grid.restype = i64
        L.orc_grid.argtypes = [ctypes.POINTER(Bounds), ctypes.POINTER(Params), vp, vp, i64]
        L.orc_durations.restype = i32
        L.orc_durations.argtypes = [ctypes.POINTER(Params), vp, i32]
        L.orc_bls_star.restype = ctypes.c_int
        L.orc_bls_star.argtypes = [vp, vp, vp, i64, d, ctypes.POINTER(Params), d, d,
                                   ctypes.POINTER(Spectrum), i64, ctypes.POINTER(Bounds)]
        L.orc_bls_star_at.restype = ctypes.c_int
        L.orc_bls_star_at.argtypes = [vp, vp, vp, i64, d, ctypes.POINTER(Params), d, d, vp, i64,
                                      ctypes.POINTER(Spectrum), ctypes.POINTER(Bounds)]
        L.orc_stats.restype = ctypes.c_int
        L.orc_stats.argtypes = [vp, vp, vp, i64, d, d, i32, i32, i32, d, vp]
        L.orc_median.restype = d
        L.orc_median.argtypes = [vp, i64]
        L.orc_sturges.restype = i32
        L.orc_sturges.argtypes = [i64]
        L.orc_snr.restype = ctypes.c_int
        L.orc_snr.argtypes = [vp, vp, i64, ctypes.POINTER(Params), vp, vp, ctypes.POINTER(SnrResult)]
        L.orc_batch_sizes.restype = ctypes.c_int
        L.orc_batch_sizes.argtypes = [i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Params), vp, vp]
        L.orc_batch_run.restype = ctypes.c_int
        L.orc_batch_run.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Params), vp,
                                    vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]
        L.orc_max_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# Small wrappers
# ----------------------------------------------------------------------------
def k_sun() -> float:
    return lib().orc_k_sun()


def krho(rho: float) -> float:
    return lib().orc_krho(rho)


def period_at_a(a_min: float, rho: float = 1.0) -> float:
    return lib().orc_period_at_a(a_min, rho)


def qcirc(f: float, rho: float = 1.0) -> float:
    return lib().orc_qcirc(f, rho)


def qcirc_exact(f: float, rho: float = 1.0) -> float:
    return lib().orc_qcirc_exact(f, rho)


def rebin_ladder(p: Params | None = None) -> np.ndarray:
    """Factors g_k of the continuous duration ladder (q_k = g_k q_lo) of the
    per-duration rebinning."""
    p = p or params()
    out = np.zeros(64)
    n = lib().orc_rebin_ladder(ctypes.byref(p), _ptr(out), 64)
    if n < 0:
        raise ValueError("bad duration parameters")
    return out[:n].copy()


def sturges(n: int) -> int:
    return lib().orc_sturges(n)


def median(v) -> float:
    v = _f64(v)
    return lib().orc_median(_ptr(v), len(v))


def durations(p: Params | None = None) -> np.ndarray:
    p = p or params()
    out = np.zeros(64, np.int32)
    n = lib().orc_durations(ctypes.byref(p), _ptr(out), 64)
    if n < 0:
        raise ValueError("bad duration parameters")
    return out[:n].copy()


def bounds(t, w=None, rho=1.0, p: Params | None = None, pmin=0.0, pmax=0.0):
    """Per-star baseline, period bounds and grid description.  Returns (status, Bounds)."""
    p = p or params()
    t = _f64(t)
    w = _f64(w)
    b = Bounds()
    st = lib().orc_bounds(_ptr(t), _ptr(w), len(t), rho, ctypes.byref(p), pmin, pmax, ctypes.byref(b))
    return st, b


def grid(t, w=None, rho=1.0, p: Params | None = None, pmin=0.0, pmax=0.0):
    """Frequencies (1/day) and fine-bin counts of the star's Keplerian grid."""
    p = p or params()
    st, b = bounds(t, w, rho, p, pmin, pmax)
    if st != 0:
        raise ValueError("oracle bounds status %d" % st)
    f = np.zeros(b.nf, np.float64)
    nb = np.zeros(b.nf, np.int32)
    lib().orc_grid(ctypes.byref(b), ctypes.byref(p), _ptr(f), _ptr(nb), b.nf)
    return f, nb, b


@dataclass
class StarSpectrum:
    f: np.ndarray
    nb: np.ndarray
    sr: np.ndarray
    m: np.ndarray
    j: np.ndarray
    r: np.ndarray
    s: np.ndarray
    bounds: Bounds


def bls_star(t, y, w=None, rho=1.0, p: Params | None = None, pmin=0.0, pmax=0.0) -> StarSpectrum:
    """Full BLS spectrum of one star (FP64, index-order sums)."""
    p = p or params()
    t, y, w = _f64(t), _f64(y), _f64(w)
    st, b = bounds(t, w, rho, p, pmin, pmax)
    if st != 0:
        raise ValueError("oracle bounds status %d" % st)
    nf = b.nf
    arr = dict(sr=np.zeros(nf), m=np.zeros(nf, np.int32), j=np.zeros(nf, np.int32),
               r=np.zeros(nf), s=np.zeros(nf), nb=np.zeros(nf, np.int32), f=np.zeros(nf))
    sp = Spectrum(*[_ptr(arr[k]) for k in ("sr", "m", "j", "r", "s", "nb", "f")])
    b2 = Bounds()
    st = lib().orc_bls_star(_ptr(t), _ptr(y), _ptr(w), len(t), rho, ctypes.byref(p), pmin, pmax,
                            ctypes.byref(sp), nf, ctypes.byref(b2))
    if st != 0:
        raise ValueError("oracle bls status %d" % st)
    return StarSpectrum(bounds=b2, **arr)


def bls_star_at(t, y, w, idx, rho=1.0, p: Params | None = None, pmin=0.0, pmax=0.0) -> StarSpectrum:
    """The star's BLS at the listed grid indices only (outputs indexed like ``idx``);
    each frequency is searched exactly as in ``bls_star``."""
    p = p or params()
    t, y, w = _f64(t), _f64(y), _f64(w)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    k = len(idx)
    arr = dict(sr=np.zeros(k), m=np.zeros(k, np.int32), j=np.zeros(k, np.int32),
               r=np.zeros(k), s=np.zeros(k), nb=np.zeros(k, np.int32), f=np.zeros(k))
    sp = Spectrum(*[_ptr(arr[n]) for n in ("sr", "m", "j", "r", "s", "nb", "f")])
    b = Bounds()
    st = lib().orc_bls_star_at(_ptr(t), _ptr(y), _ptr(w), len(t), rho, ctypes.byref(p), pmin, pmax,
                               _ptr(idx), k, ctypes.byref(sp), ctypes.byref(b))
    if st != 0:
        raise ValueError("oracle bls status %d" % st)
    return StarSpectrum(bounds=b, **arr)


def snr(f, sr, p: Params | None = None):
    """S/N spectrum, trend and summary of one SR spectrum."""
    p = p or params()
    f, sr = _f64(f), _f64(sr)
    n = len(f)
    out = np.zeros(n)
    tr = np.zeros(n)
    res = SnrResult()
    st = lib().orc_snr(_ptr(f), _ptr(sr), n, ctypes.byref(p), _ptr(out), _ptr(tr), ctypes.byref(res))
    if st != 0:
        raise ValueError("oracle snr status %d" % st)
    return out, tr, res


RESULT_FIELDS = ("i_snr", "i_sr", "period", "t0", "duration", "depth", "sr", "snr", "trend",
                 "sigma", "status", "nf")


def batch(t, y, w, offsets, rho=None, pmin=None, pmax=None, p: Params | None = None,
          nthreads: int = 0, stars=None):
    """Run the oracle over a packed batch (optionally only the listed star indices).

    Returns a dict with per-star ``results`` [S, 12] (fields ``RESULT_FIELDS``) and
    ragged per-frequency arrays with their offsets ``fofs``.
    """
    p = p or params()
    t, y, w = _f64(t), _f64(y), _f64(w)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    rho = None if rho is None else _f64(rho)
    pmin = None if pmin is None else _f64(pmin)
    pmax = None if pmax is None else _f64(pmax)
    if stars is not None:
        stars = np.asarray(stars, dtype=np.int64)
        segs_t, segs_y, segs_w, offs = [], [], [], [0]
        for s in stars:
            a, b = offsets[s], offsets[s + 1]
            segs_t.append(t[a:b]); segs_y.append(y[a:b]); segs_w.append(w[a:b])
            offs.append(offs[-1] + (b - a))
        t, y, w = np.concatenate(segs_t), np.concatenate(segs_y), np.concatenate(segs_w)
        offsets = np.asarray(offs, dtype=np.int64)
        rho = None if rho is None else rho[stars].copy()
        pmin = None if pmin is None else pmin[stars].copy()
        pmax = None if pmax is None else pmax[stars].copy()
    S = len(offsets) - 1
    nf = np.zeros(S, np.int64)
    stat = np.zeros(S, np.int32)
    L = lib()
    L.orc_batch_sizes(S, _ptr(offsets), _ptr(t), _ptr(w), _ptr(rho), _ptr(pmin), _ptr(pmax),
                      ctypes.byref(p), _ptr(nf), _ptr(stat))
    if np.any(stat != 0):
        raise ValueError("oracle bounds failed for stars %s" % np.nonzero(stat)[0][:10])
    fofs = np.zeros(S + 1, np.int64)
    fofs[1:] = np.cumsum(nf)
    tot = int(fofs[-1])
    out = dict(f=np.zeros(tot), nb=np.zeros(tot, np.int32), sr=np.zeros(tot),
               m=np.zeros(tot, np.int32), j=np.zeros(tot, np.int32), r=np.zeros(tot),
               s=np.zeros(tot), snr=np.zeros(tot), trend=np.zeros(tot), results=np.zeros((S, 12)))
    st = L.orc_batch_run(S, _ptr(offsets), _ptr(t), _ptr(y), _ptr(w), _ptr(rho), _ptr(pmin),
                         _ptr(pmax), ctypes.byref(p), _ptr(fofs), _ptr(out["f"]), _ptr(out["nb"]),
                         _ptr(out["sr"]), _ptr(out["m"]), _ptr(out["j"]), _ptr(out["r"]),
                         _ptr(out["s"]), _ptr(out["snr"]), _ptr(out["trend"]),
                         _ptr(out["results"]), int(nthreads))
    if st != 0:
        raise ValueError("oracle batch failed")
    out["fofs"] = fofs
    return out


STATS_FIELDS = ("n_in", "n_before", "n_after", "n_transits", "candidate", "oot_level")


def stats(t, y, w, t0: float, f: float, nb: int, m: int, j: int, snr: float) -> dict:
    """Points in, before and after transit, transit count, candidate flag and the
    out-of-transit level at one best window (Sec. 2.2 item 5 and the detection
    criteria)."""
    t, y, w = _f64(t), _f64(y), _f64(w)
    out = np.zeros(6)
    st = lib().orc_stats(_ptr(t), _ptr(y), _ptr(w), len(t), t0, f, nb, m, j, snr, _ptr(out))
    if st != 0:
        raise ValueError("oracle stats status %d" % st)
    r = dict(zip(STATS_FIELDS, out.tolist()))
    for k in STATS_FIELDS[:5]:
        r[k] = int(r[k])
    return r


def max_threads() -> int:
    return lib().orc_max_threads()
