"""ctypes wrapper of ``ffa_oracle.c`` -- the plain CPU reference.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.  Never imported by the GPU library.

Float input is carried in double precision, uint8 input in int64.  See the C
source for the passage of the paper each function follows.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

IN_F32 = 0
IN_U8 = 1
ALG1 = 1
ALG2 = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def library(path: str):
    """Temporarily use another build of the oracle source (mutation tests)."""
    global _lib
    old = _lib
    _lib = _configure(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = old


def _configure(lib):
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    lib.oracle_plan.restype = ctypes.c_int
    lib.oracle_plan.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                i32p, i32p, i32p, i32p, i64p]
    lib.oracle_downsample_f64.argtypes = [f64p, ctypes.c_int64, ctypes.c_int32, f64p]
    lib.oracle_downsample_i64.argtypes = [i64p, ctypes.c_int64, ctypes.c_int32, i64p]
    lib.oracle_fold_f64.argtypes = [f64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, f64p]
    lib.oracle_fold_i64.argtypes = [i64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, i64p]
    for name in ("oracle_alg1_f64", "oracle_alg2_f64"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_double
        fn.argtypes = [f64p, ctypes.c_int32, i32p, ctypes.c_int32, i32p]
    for name in ("oracle_alg1_i64", "oracle_alg2_i64"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_double
        fn.argtypes = [i64p, ctypes.c_int32, i32p, ctypes.c_int32, i32p]
    lib.oracle_default_widths.restype = ctypes.c_int32
    lib.oracle_default_widths.argtypes = [ctypes.c_int32, i32p]
    lib.oracle_search.restype = ctypes.c_int
    lib.oracle_search.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                  i32p, i32p, i32p, i32p, i64p, ctypes.c_int32, i32p,
                                  i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_float), i32p]
    lib.oracle_fold_step.restype = ctypes.c_int
    lib.oracle_fold_step.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, vp]
    lib.oracle_dered_default_window.restype = ctypes.c_int32
    lib.oracle_dered_default_window.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.oracle_deredden_f64.restype = ctypes.c_int
    lib.oracle_deredden_f64.argtypes = [f64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, f64p]
    lib.oracle_sift.restype = ctypes.c_int64
    lib.oracle_sift.argtypes = [ctypes.POINTER(ctypes.c_float), i32p, ctypes.c_int64, ctypes.c_int32,
                                i32p, i32p, i32p, i32p, i64p, ctypes.c_double,
                                ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_int32, ctypes.c_float, i64p, f64p,
                                ctypes.POINTER(ctypes.c_float), i32p]
    lib.oracle_snr_histogram.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_mad_constant.restype = ctypes.c_double
    lib.oracle_score_profiles.restype = ctypes.c_int
    lib.oracle_score_profiles.argtypes = [f64p, ctypes.c_int64, ctypes.c_int32, i32p, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def mad_constant() -> float:
    """K of sigma = K*MAD as the oracle uses it."""
    return float(_load().oracle_mad_constant())


@dataclass
class Plan:
    """Step list of a search: one FFA execution per (octave factor f, P0)."""

    f: np.ndarray
    P0: np.ndarray
    m: np.ndarray
    M: np.ndarray
    first: np.ndarray
    tsamp: float

    @property
    def n_steps(self) -> int:
        return int(self.f.size)

    @property
    def n_trials(self) -> int:
        return int(self.M.sum()) if self.M.size else 0

    def periods(self) -> np.ndarray:
        """Trial periods in seconds: f*tsamp*(P0 + k/(M-1)) (Eq. 2, N -> M*P0)."""
        out = np.empty(self.n_trials, dtype=np.float64)
        for s in range(self.n_steps):
            M = int(self.M[s])
            k = np.arange(M, dtype=np.float64)
            out[self.first[s]:self.first[s] + M] = (
                float(self.f[s]) * self.tsamp * (float(self.P0[s]) + k / (M - 1)))
        return out


def plan(N: int, tsamp: float, pmin: float, pmax: float, bins_min: int,
         max_octaves: int = 0) -> Plan:
    lib = _load()
    n = lib.oracle_plan(N, tsamp, pmin, pmax, bins_min, max_octaves, 0,
                        None, None, None, None, None)
    if n < 0:
        raise ValueError("invalid plan arguments")
    f = np.zeros(n, np.int32)
    P0 = np.zeros(n, np.int32)
    m = np.zeros(n, np.int32)
    M = np.zeros(n, np.int32)
    first = np.zeros(n, np.int64)
    i32 = ctypes.c_int32
    lib.oracle_plan(N, tsamp, pmin, pmax, bins_min, max_octaves, n, _ptr(f, i32), _ptr(P0, i32),
                    _ptr(m, i32), _ptr(M, i32), _ptr(first, ctypes.c_int64))
    return Plan(f, P0, m, M, first, float(tsamp))


def downsample(x: np.ndarray, octave: int) -> np.ndarray:
    """Series at factor 2**octave by successive pairwise sums."""
    lib = _load()
    if np.issubdtype(x.dtype, np.integer):
        xi = np.ascontiguousarray(x, dtype=np.int64)
        out = np.zeros(max(xi.size >> octave, 0), np.int64)
        lib.oracle_downsample_i64(_ptr(xi, ctypes.c_int64), xi.size, octave,
                                  _ptr(out, ctypes.c_int64))
        return out
    xd = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(max(xd.size >> octave, 0), np.float64)
    lib.oracle_downsample_f64(_ptr(xd, ctypes.c_double), xd.size, octave,
                              _ptr(out, ctypes.c_double))
    return out


def fold(x: np.ndarray, P0: int, m: int, M: int) -> np.ndarray:
    """FFA profiles (M, P0) of the rows of ``x`` (already at the step's octave)."""
    lib = _load()
    if m * P0 > x.size or m > M or M & (M - 1):
        raise ValueError("bad fold shape")
    if np.issubdtype(x.dtype, np.integer):
        xi = np.ascontiguousarray(x, dtype=np.int64)
        out = np.zeros((M, P0), np.int64)
        lib.oracle_fold_i64(_ptr(xi, ctypes.c_int64), P0, m, M, _ptr(out, ctypes.c_int64))
        return out
    xd = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((M, P0), np.float64)
    lib.oracle_fold_f64(_ptr(xd, ctypes.c_double), P0, m, M, _ptr(out, ctypes.c_double))
    return out


def fold_step(series: np.ndarray, f: int, P0: int, m: int, M: int, dered_window: int = 0,
              dered_stride: int = 0) -> np.ndarray:
    """Profiles of one step straight from the raw series (uint8 -> int64, f32 -> f64;
    float64 whenever the series is dereddened)."""
    lib = _load()
    if series.dtype == np.uint8:
        dt, out = IN_U8, np.zeros((M, P0), np.float64 if dered_window > 0 else np.int64)
    elif series.dtype == np.float32:
        dt, out = IN_F32, np.zeros((M, P0), np.float64)
    else:
        raise TypeError("series must be uint8 or float32")
    s = np.ascontiguousarray(series)
    rc = lib.oracle_fold_step(s.ctypes.data, dt, s.size, f, P0, m, M, dered_window, dered_stride,
                              out.ctypes.data)
    if rc != 0:
        raise ValueError("bad step")
    return out


def default_widths(P0: int) -> list[int]:
    buf = np.zeros(32, np.int32)
    n = _load().oracle_default_widths(P0, _ptr(buf, ctypes.c_int32))
    return [int(v) for v in buf[:n]]


def _score(fn_f, fn_i, profile: np.ndarray, widths) -> tuple[float, int]:
    w = np.ascontiguousarray(widths, dtype=np.int32)
    bw = np.zeros(1, np.int32)
    if np.issubdtype(profile.dtype, np.integer) and fn_i is not None:
        p = np.ascontiguousarray(profile, dtype=np.int64)
        v = fn_i(_ptr(p, ctypes.c_int64), p.size, _ptr(w, ctypes.c_int32), w.size,
                 _ptr(bw, ctypes.c_int32))
    else:
        p = np.ascontiguousarray(profile, dtype=np.float64)
        v = fn_f(_ptr(p, ctypes.c_double), p.size, _ptr(w, ctypes.c_int32), w.size,
                 _ptr(bw, ctypes.c_int32))
    return float(v), int(bw[0])


def alg1(profile: np.ndarray, widths) -> tuple[float, int]:
    """Algorithm 1 score and width of one profile (integer profiles exactly)."""
    lib = _load()
    return _score(lib.oracle_alg1_f64, lib.oracle_alg1_i64, profile, widths)


def score_profiles(profiles: np.ndarray, alg: int, widths=None, threads: int = 0) -> np.ndarray:
    """Scores (float32) of the rows of ``profiles`` (n x P0, float64) with
    Algorithm ``alg``; ``widths`` None = the default rule for P0."""
    p = np.ascontiguousarray(profiles, dtype=np.float64)
    n, P0 = p.shape
    w = np.ascontiguousarray(widths if widths is not None else [], dtype=np.int32)
    out = np.empty(n, np.float32)
    rc = _load().oracle_score_profiles(_ptr(p, ctypes.c_double), n, P0,
                                        _ptr(w, ctypes.c_int32) if w.size else None, w.size, alg, threads,
                                        _ptr(out, ctypes.c_float))
    if rc != 0:
        raise ValueError("bad arguments")
    return out


def alg2(profile: np.ndarray, widths) -> tuple[float, int]:
    """Algorithm 2 score and width of one profile (integer profiles exactly)."""
    lib = _load()
    return _score(lib.oracle_alg2_f64, lib.oracle_alg2_i64, profile, widths)


def dered_default_window(tsamp: float, pmin: float, pmax: float) -> int:
    """The dereddening window the paper uses by default (Sec. 2.3.1), in
    samples of the input series."""
    return int(_load().oracle_dered_default_window(tsamp, pmin, pmax))


def deredden(x: np.ndarray, window: int, stride: int = 0) -> np.ndarray:
    """Running-median dereddening of one series (see oracle_deredden_f64)."""
    xd = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(xd)
    rc = _load().oracle_deredden_f64(_ptr(xd, ctypes.c_double), xd.size, window, stride,
                                     _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("bad dereddening arguments")
    return out


def search(series: np.ndarray, p: Plan, widths=None, alg: int = ALG1, steps=None,
           threads: int = 0, dered_window: int = 0, dered_stride: int = 0
           ) -> tuple[np.ndarray, np.ndarray]:
    """Periodogram (S/N float32, width int32) over all trials of plan ``p``.

    ``steps`` selects a subset of step indices; entries of other steps are NaN / -1.
    ``dered_window`` > 0 dereddens every octave series first (window in its
    own samples; ``dered_stride`` 0 or 1 = the exact running median at every
    sample, > 1 = medians at knots that far apart, interpolated).
    """
    lib = _load()
    if series.dtype == np.uint8:
        dt = IN_U8
    elif series.dtype == np.float32:
        dt = IN_F32
    else:
        raise TypeError("series must be uint8 or float32")
    s = np.ascontiguousarray(series)
    snr = np.full(p.n_trials, np.nan, np.float32)
    wid = np.full(p.n_trials, -1, np.int32)
    i32 = ctypes.c_int32
    if widths is None or len(widths) == 0:
        w = np.zeros(1, np.int32)
        nw = 0
    else:
        w = np.ascontiguousarray(widths, dtype=np.int32)
        nw = w.size
    if steps is None:
        sel = None
        nsel = 0
    else:
        sel_arr = np.ascontiguousarray(steps, dtype=np.int32)
        if sel_arr.size == 0:
            return snr, wid
        sel = _ptr(sel_arr, i32)
        nsel = sel_arr.size
    rc = lib.oracle_search(s.ctypes.data, dt, s.size, p.n_steps, _ptr(p.f, i32), _ptr(p.P0, i32),
                           _ptr(p.m, i32), _ptr(p.M, i32), _ptr(p.first, ctypes.c_int64),
                           nsel, sel, _ptr(w, i32), nw, alg, threads, dered_window, dered_stride,
                           _ptr(snr, ctypes.c_float), _ptr(wid, i32))
    if rc != 0:
        raise ValueError("oracle_search failed")
    return snr, wid


SIFT_DTYPE = np.dtype([("trial", "<i8"), ("period", "<f8"), ("snr", "<f4"), ("width", "<i4")])


def sift(snr: np.ndarray, width: np.ndarray, p: Plan, min_snr: float = 9.0, frac_fall: float = 0.1,
         abs_fall: float = 1.0, group_widths: float = 0.0, harmonic_primes: int = 0,
         harmonic_tol: float = 1e-5) -> np.ndarray:
    """Candidates of a periodogram (see oracle_sift), strongest first."""
    lib = _load()
    s = np.ascontiguousarray(snr, dtype=np.float32)
    w = np.ascontiguousarray(width, dtype=np.int32)
    n = s.size
    tr = np.zeros(max(n, 1), np.int64)
    pe = np.zeros(max(n, 1), np.float64)
    sn = np.zeros(max(n, 1), np.float32)
    wi = np.zeros(max(n, 1), np.int32)
    i32 = ctypes.c_int32
    k = lib.oracle_sift(_ptr(s, ctypes.c_float), _ptr(w, i32), n, p.n_steps, _ptr(p.f, i32),
                        _ptr(p.P0, i32), _ptr(p.m, i32), _ptr(p.M, i32), _ptr(p.first, ctypes.c_int64),
                        p.tsamp, min_snr, frac_fall, abs_fall, group_widths, harmonic_primes,
                        harmonic_tol, _ptr(tr, ctypes.c_int64), _ptr(pe, ctypes.c_double),
                        _ptr(sn, ctypes.c_float), _ptr(wi, i32))
    if k < 0:
        raise ValueError("bad sift arguments")
    out = np.zeros(k, SIFT_DTYPE)
    out["trial"], out["period"], out["snr"], out["width"] = tr[:k], pe[:k], sn[:k], wi[:k]
    return out


# ------------------------------------------------ false-alarm statistics

def snr_histogram(snr: np.ndarray, lo: float, bins_per_unit: float, n_bins: int,
                  hist: np.ndarray | None = None) -> np.ndarray:
    """Counts of S/N values per bin (see oracle_snr_histogram), added to
    ``hist`` (uint64) when given."""
    s = np.ascontiguousarray(snr, dtype=np.float32).ravel()
    if hist is None:
        hist = np.zeros(n_bins, np.uint64)
    if hist.dtype != np.uint64 or hist.size != n_bins or not hist.flags.c_contiguous:
        raise ValueError("hist must be a contiguous uint64 array of n_bins counts")
    _load().oracle_snr_histogram(_ptr(s, ctypes.c_float), s.size, lo, bins_per_unit, n_bins,
                                 _ptr(hist, ctypes.c_uint64))
    return hist


def _tails(hist: np.ndarray) -> np.ndarray:
    """tail[b] = number of values in bins b and above (exact integers)."""
    h = np.asarray(hist, dtype=np.uint64)
    return np.cumsum(h[::-1], dtype=np.uint64)[::-1]


def sigma_gauss(hist: np.ndarray) -> np.ndarray:
    """Gaussian-equivalent sigma at the lower edge of every bin (Sec. 4.1.2):
    the fraction Q of values at or above the edge, mapped through the normal
    quantile so that a standard normal variable exceeds sigma with
    probability Q.  Bin 0 (Q = 1) maps to -inf, an edge no value reaches to
    +inf."""
    from scipy.stats import norm

    tail = _tails(hist)
    total = float(tail[0])
    if total <= 0:
        raise ValueError("empty histogram")
    return norm.isf(tail.astype(np.float64) / total)


def sigma_threshold(hist: np.ndarray, lo: float, bins_per_unit: float, sigma: float) -> float:
    """The S/N that a sigma-sigma detection needs (Sec. 4.1.2): the lowest
    inner bin edge lo + b / bins_per_unit (b >= 1) at or above which at most
    a fraction Phi(-sigma) of the values lie (count <= Phi(-sigma) * total,
    in double)."""
    from scipy.stats import norm

    tail = _tails(hist)
    total = float(tail[0])
    if total <= 0:
        raise ValueError("empty histogram")
    limit = float(norm.sf(sigma)) * total
    for b in range(1, tail.size):
        if float(tail[b]) <= limit:
            return float(lo) + float(b) / float(bins_per_unit)
    raise ValueError("the histogram's top bin holds more than the allowed fraction; widen it")
