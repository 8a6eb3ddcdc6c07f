"""ctypes binding of ``libmi355bls.so`` (the C ABI declared in ``include/mi355bls.h``).

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  If the shared
library is missing, loading raises immediately; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmi355bls.so")

BLS_OK = 0
STATUS_NAMES = {0: "BLS_OK", -1: "BLS_E_ARG", -2: "BLS_E_INPUT", -3: "BLS_E_EMPTY_GRID",
                -4: "BLS_E_NOMEM", -5: "BLS_E_HIP", -6: "BLS_E_STATE", -7: "BLS_E_UNSUPPORTED",
                -8: "BLS_E_SCRATCH"}

EXPORTS = ("bls_default_params", "bls_plan_create", "bls_plan_query", "bls_plan_star_info",
           "bls_plan_frequencies", "bls_plan_durations", "bls_plan_upload", "bls_prepare", "bls_search_batch",
           "bls_snr", "bls_stats", "bls_fit", "bls_run_noalloc", "bls_plan_destroy", "bls_status_string", "bls_limits", "bls_last_hip_error",
           # learned period proposal (include/mi355pp.h)
           "pp_act_bytes", "pp_resample", "pp_forward", "pp_backward", "pp_adam", "pp_propose", "pp_propose_guided",
           "pp_tile_capacity", "pp_snr_windows")

PP_NPARAM = 3122
PP_NCLASS = 513
PP_NBINS_IN = 4096
PP_MAX_WINDOWS = 16
PP_ACT_BYTES_PER_STAR = 106496


class BlsParams(ctypes.Structure):
    _fields_ = [("spp", ctypes.c_double), ("qmin_fac", ctypes.c_double),
                ("qmax_fac", ctypes.c_double), ("dlogq", ctypes.c_double),
                ("noverlap", ctypes.c_int32), ("dip_only", ctypes.c_int32),
                ("mad_of_raw", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("a_min_rstar", ctypes.c_double), ("sector_days", ctypes.c_double),
                ("tile_cells", ctypes.c_int64), ("big_points", ctypes.c_int64),
                ("item_freqs", ctypes.c_int32), ("exact_duration", ctypes.c_int32),
                ("rebin", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BlsStar(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("rho_solar", ctypes.c_double),
                ("pmin_days", ctypes.c_double), ("pmax_days", ctypes.c_double)]


BEST_DTYPE = np.dtype([("m", np.int32), ("j", np.int32), ("r", np.float64), ("s", np.float64)])
RESULT_DTYPE = np.dtype([("i_snr", np.int64), ("i_sr", np.int64), ("period", np.float64),
                         ("t0", np.float64), ("duration", np.float64), ("depth", np.float64),
                         ("sr", np.float64), ("snr", np.float64), ("trend", np.float64),
                         ("sigma", np.float64), ("status", np.int32), ("nbins", np.int32)])
STATS_DTYPE = np.dtype([("n_in", np.int64), ("n_before", np.int64), ("n_after", np.int64),
                        ("n_transits", np.int64), ("oot_level", np.float64), ("candidate", np.int32),
                        ("status", np.int32)])
FIT_DTYPE = np.dtype([("t0", np.float64), ("depth", np.float64), ("q", np.float64), ("q_in", np.float64),
                      ("level", np.float64), ("chi2", np.float64), ("sigma_w", np.float64),
                      ("sigma_r", np.float64), ("depth_eff", np.float64), ("snr_pink", np.float64),
                      ("n_fit", np.int64), ("n_t", np.int64), ("n_transits", np.int64),
                      ("iterations", np.int32), ("candidate", np.int32), ("status", np.int32), ("pad", np.int32)])
assert BEST_DTYPE.itemsize == 24 and RESULT_DTYPE.itemsize == 88 and STATS_DTYPE.itemsize == 48
assert FIT_DTYPE.itemsize == 120

_lib = None


class BlsError(RuntimeError):
    def __init__(self, where: str, code: int, star: int | None = None):
        msg = "%s failed: %s (%d)" % (where, STATUS_NAMES.get(code, "?"), code)
        if star is not None and star >= 0:
            msg += " at star %d" % star
        if code == -5 and _lib is not None:
            msg += " (hipError %d)" % int(_lib.bls_last_hip_error())
        super().__init__(msg)
        self.code = code
        self.star = star


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmi355bls.so not built: run `python -m paper_2302_01293_amd.build` "
                              "(or __graft_entry__.build())")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 (same soname
        # as the system one the library links).  Loading torch first makes the
        # library bind to torch's copy; loading the library first would bring in a
        # second runtime, and then one of the two finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.bls_default_params.restype = i32
        L.bls_default_params.argtypes = [ctypes.POINTER(BlsParams)]
        L.bls_plan_create.restype = i32
        L.bls_plan_create.argtypes = [ctypes.POINTER(BlsParams), i32, ctypes.POINTER(BlsStar), vp, vp, vp,
                                      ctypes.POINTER(vp), ctypes.POINTER(i32)]
        L.bls_plan_query.restype = i32
        L.bls_plan_query.argtypes = [vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64)]
        L.bls_plan_star_info.restype = i32
        L.bls_plan_star_info.argtypes = [vp, i32, vp]
        L.bls_plan_frequencies.restype = i32
        L.bls_plan_frequencies.argtypes = [vp, i32, vp, vp]
        L.bls_plan_durations.restype = i32
        L.bls_plan_durations.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.bls_plan_upload.restype = i32
        L.bls_plan_upload.argtypes = [vp, vp, i64, vp]
        L.bls_prepare.restype = i32
        L.bls_prepare.argtypes = [vp, vp, vp, vp, vp, vp]
        L.bls_search_batch.restype = i32
        L.bls_search_batch.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.bls_snr.restype = i32
        L.bls_snr.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.bls_stats.restype = i32
        L.bls_stats.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp, vp]
        L.bls_fit.restype = i32
        L.bls_fit.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp]
        L.bls_run_noalloc.restype = i32
        L.bls_run_noalloc.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        L.bls_plan_destroy.restype = None
        L.bls_plan_destroy.argtypes = [vp]
        L.bls_status_string.restype = ctypes.c_char_p
        L.bls_status_string.argtypes = [i32]
        L.bls_limits.restype = i32
        L.bls_limits.argtypes = [vp]
        L.bls_last_hip_error.restype = i32
        L.bls_last_hip_error.argtypes = []
        f32 = ctypes.c_float
        L.pp_act_bytes.restype = i32
        L.pp_act_bytes.argtypes = [i32, ctypes.POINTER(i64)]
        L.pp_resample.restype = i32
        L.pp_resample.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.pp_forward.restype = i32
        L.pp_forward.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.pp_backward.restype = i32
        L.pp_backward.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp]
        L.pp_adam.restype = i32
        L.pp_adam.argtypes = [vp, vp, vp, vp, i32, f32, vp]
        L.pp_propose.restype = i32
        L.pp_propose.argtypes = [vp, vp, vp, i32, f32, vp, vp, vp, vp, vp]
        L.pp_propose_guided.restype = i32
        L.pp_propose_guided.argtypes = [vp, vp, vp, i32, f32, i32, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp]
        L.pp_tile_capacity.restype = i32
        L.pp_tile_capacity.argtypes = [vp, ctypes.POINTER(i64)]
        L.pp_snr_windows.restype = i32
        L.pp_snr_windows.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp]
        _lib = L
    return _lib


def default_params(**kw) -> BlsParams:
    p = BlsParams()
    st = lib().bls_default_params(ctypes.byref(p))
    if st != BLS_OK:
        raise BlsError("bls_default_params", st)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def limits() -> dict:
    out = np.zeros(3, np.int64)
    lib().bls_limits(out.ctypes.data)
    return dict(nb_max=int(out[0]), m_max=int(out[1]), points_max=int(out[2]))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Plan:
    """A host plan for one packed batch (owns the C ``bls_plan``)."""

    def __init__(self, t, y=None, w=None, offsets=None, rho=None, pmin=None, pmax=None,
                 params: BlsParams | None = None):
        self.params = params if params is not None else default_params()
        t, y, w = _f64(t), _f64(y), _f64(w)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        S = len(offsets) - 1
        stars = (BlsStar * S)()
        n = np.diff(offsets)
        for s in range(S):
            stars[s].n_points = int(n[s])
            stars[s].rho_solar = float(rho[s]) if rho is not None else 1.0
            stars[s].pmin_days = float(pmin[s]) if pmin is not None else 0.0
            stars[s].pmax_days = float(pmax[s]) if pmax is not None else 0.0
        h = ctypes.c_void_p()
        bad = ctypes.c_int32(-1)
        self._keep = (t, y, w)
        st = lib().bls_plan_create(ctypes.byref(self.params), S, stars, t.ctypes.data,
                                   None if y is None else y.ctypes.data,
                                   None if w is None else w.ctypes.data, ctypes.byref(h), ctypes.byref(bad))
        if st != BLS_OK:
            raise BlsError("bls_plan_create", st, bad.value)
        self.h = h
        self.n_stars = S
        nft = ctypes.c_int64()
        wsb = ctypes.c_int64()
        fofs = np.zeros(S + 1, np.int64)
        st = lib().bls_plan_query(self.h, ctypes.byref(nft), fofs.ctypes.data, ctypes.byref(wsb))
        if st != BLS_OK:
            raise BlsError("bls_plan_query", st)
        self.n_freq = int(nft.value)
        self.freq_offsets = fofs
        self.workspace_bytes = int(wsb.value)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().bls_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def star_info(self, s: int) -> dict:
        o = np.zeros(10)
        st = lib().bls_plan_star_info(self.h, s, o.ctypes.data)
        if st != BLS_OK:
            raise BlsError("bls_plan_star_info", st)
        keys = ("t0", "T", "pmin", "pmax", "krho", "umin", "A", "nf", "nb_max", "sturges")
        return dict(zip(keys, o.tolist()))

    def frequencies(self, s: int):
        nf = int(self.freq_offsets[s + 1] - self.freq_offsets[s])
        f = np.zeros(nf)
        nb = np.zeros(nf, np.int32)
        st = lib().bls_plan_frequencies(self.h, s, f.ctypes.data, nb.ctypes.data)
        if st != BLS_OK:
            raise BlsError("bls_plan_frequencies", st)
        return f, nb

    def durations(self) -> np.ndarray:
        n = ctypes.c_int32()
        lib().bls_plan_durations(self.h, None, 0, ctypes.byref(n))
        m = np.zeros(n.value, np.int32)
        st = lib().bls_plan_durations(self.h, m.ctypes.data, n.value, ctypes.byref(n))
        if st != BLS_OK:
            raise BlsError("bls_plan_durations", st)
        return m

    # ---- device calls (pointers are integers from torch tensors) ----
    def upload(self, d_ws: int, ws_bytes: int, stream: int = 0):
        st = lib().bls_plan_upload(self.h, d_ws, ws_bytes, stream or None)
        if st != BLS_OK:
            raise BlsError("bls_plan_upload", st)

    def prepare(self, d_ws: int, d_t: int, d_y: int, d_w: int | None, stream: int = 0):
        st = lib().bls_prepare(self.h, d_ws, d_t, d_y, d_w or None, stream or None)
        if st != BLS_OK:
            raise BlsError("bls_prepare", st)

    def search(self, d_ws: int, d_sr: int, d_best: int | None, d_windows: int | None = None,
               n_windows: int = 0, stream: int = 0):
        st = lib().bls_search_batch(self.h, d_ws, d_windows or None, n_windows, d_sr, d_best or None,
                                    stream or None)
        if st != BLS_OK:
            raise BlsError("bls_search_batch", st)

    def snr(self, d_ws: int, d_sr: int, d_best: int | None, d_snr: int | None, d_result: int, stream: int = 0):
        st = lib().bls_snr(self.h, d_ws, d_sr, d_best or None, d_snr or None, d_result, stream or None)
        if st != BLS_OK:
            raise BlsError("bls_snr", st)

    def stats(self, d_ws: int, d_t: int, d_y: int, d_w: int | None, d_best: int, d_result: int,
              d_stats: int, snr_min: float = 9.0, stream: int = 0):
        st = lib().bls_stats(self.h, d_ws, d_t, d_y, d_w or None, d_best, d_result, float(snr_min), d_stats,
                             stream or None)
        if st != BLS_OK:
            raise BlsError("bls_stats", st)

    def fit(self, d_ws: int, d_t: int, d_y: int, d_w: int | None, d_result: int, d_fit: int,
            snr_min: float = 9.0, pink_min: float = 9.0, stream: int = 0):
        st = lib().bls_fit(self.h, d_ws, d_t, d_y, d_w or None, d_result, float(snr_min), float(pink_min), d_fit,
                           stream or None)
        if st != BLS_OK:
            raise BlsError("bls_fit", st)

    def run_noalloc(self, d_t: int, d_y: int, d_w: int | None, d_sr: int, d_best: int | None,
                    d_snr: int | None, d_result: int, d_windows: int | None = None, n_windows: int = 0,
                    stream: int = 0):
        """upload -> prepare -> search -> S/N on the library's static device scratch
        (``bls_run_noalloc``: no workspace argument, nothing allocated)."""
        st = lib().bls_run_noalloc(self.h, d_t, d_y, d_w or None, d_windows or None, n_windows, d_sr,
                                   d_best or None, d_snr or None, d_result, stream or None)
        if st != BLS_OK:
            raise BlsError("bls_run_noalloc", st)


NOALLOC_SCRATCH_BYTES = 64 << 20


def check(name: str, st: int):
    """Raise BlsError unless a library call returned BLS_OK."""
    if st != BLS_OK:
        raise BlsError(name, st)
