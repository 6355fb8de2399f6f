"""Python binding of libffa.so (ctypes).  Argument marshalling only: every step
of the search runs in the library's HIP kernels.  PyTorch supplies device
memory and streams (``tensor.data_ptr()``, ``torch.cuda.current_stream()``).

Importing this module loads the in-tree ``libffa.so`` and raises ImportError
when it has not been built (``python -m paper_1703_05581_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffa.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1703_05581_amd.build`")

# torch ships its own HIP runtime and loads it by file name.  Importing torch
# first lets libffa.so's libamdhip64.so.7 dependency resolve to that same
# runtime by soname, so the process holds one HIP runtime and torch's device
# pointers and streams are valid in the library.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

FFA_OK = 0
FFA_ERR_INVALID = -1
FFA_ERR_NOMEM = -2
FFA_ERR_DEVICE = -3
FFA_ERR_UNSUPPORTED = -4
FFA_ERR_BUSY = -5
FFA_ERR_TIMEOUT = -6
FFA_IN_F32 = 0
FFA_IN_U8 = 1
FFA_SNR_ALG1_MAD = 1
FFA_SNR_ALG2_OFFPULSE = 2

# every symbol include/ffa.h declares
EXPORTS = (
    "ffa_plan_create", "ffa_plan_create_opts", "ffa_plan_destroy", "ffa_plan_upload", "ffa_search_noalloc", "ffa_plan_query", "ffa_plan_step", "ffa_plan_passes",
    "ffa_plan_periods", "ffa_prepare", "ffa_search_prepared", "ffa_search", "ffa_fold", "ffa_best",
    "ffa_sift", "ffa_snr_histogram", "ffa_sigma_gauss", "ffa_sigma_threshold", "ffa_batch_workspace",
    "ffa_search_batch", "ffa_batch_create", "ffa_batch_destroy", "ffa_batch_query", "ffa_batch_search",
    "ffa_batch_prepare", "ffa_batch_search_prepared", "ffa_server_create", "ffa_server_submit", "ffa_server_wait",
    "ffa_server_destroy", "ffa_debug_server_fail", "ffa_status_str", "ffa_last_error",
)


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64),
        ("tsamp_s", ctypes.c_double),
        ("pmin_s", ctypes.c_double),
        ("pmax_s", ctypes.c_double),
        ("widths", ctypes.POINTER(ctypes.c_int32)),
        ("n_widths", ctypes.c_int32),
        ("bins_min", ctypes.c_int32),
        ("max_octaves", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("snr", ctypes.c_int32),
        ("dered_window", ctypes.c_int32),
        ("dered_stride", ctypes.c_int32),
    ]


class PlanOpts(ctypes.Structure):
    """ffa_plan_opts: launch options (zero = default); they never change a result."""

    _fields_ = [
        ("tile_lds_bytes", ctypes.c_int32),
        ("window_tiles", ctypes.c_int32),
        ("ring_mb", ctypes.c_int32),
        ("steps_per_window", ctypes.c_int32),
        ("no_u16", ctypes.c_int32),
        ("no_split_occupancy", ctypes.c_int32),
        ("select_iters", ctypes.c_int32),
        ("select_cand", ctypes.c_int32),
    ]


OPT_NAMES = tuple(f[0] for f in PlanOpts._fields_)


class SiftParams(ctypes.Structure):
    _fields_ = [
        ("min_snr", ctypes.c_float),
        ("frac_fall", ctypes.c_float),
        ("abs_fall", ctypes.c_float),
        ("group_widths", ctypes.c_float),
        ("harmonic_primes", ctypes.c_int32),
        ("harmonic_tol", ctypes.c_float),
    ]


class Candidate(ctypes.Structure):
    _fields_ = [
        ("trial", ctypes.c_int64),
        ("period_s", ctypes.c_double),
        ("snr", ctypes.c_float),
        ("width", ctypes.c_int32),
    ]


assert ctypes.sizeof(Candidate) == 24

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_P = ctypes.POINTER

_lib.ffa_plan_create.argtypes = [_P(PlanDesc), _P(_vp)]
_lib.ffa_plan_create_opts.argtypes = [_P(PlanDesc), _P(PlanOpts), _P(_vp)]
_lib.ffa_plan_destroy.argtypes = [_vp]
_lib.ffa_plan_upload.argtypes = [_vp]
_lib.ffa_search_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.ffa_plan_query.argtypes = [_vp, _P(_i64), _P(_i32), _P(_sz)]
_lib.ffa_plan_step.argtypes = [_vp, _i32, _P(_i32), _P(_i32), _P(_i32), _P(_i32), _P(_i64)]
_lib.ffa_plan_passes.argtypes = [_vp, _i32, _P(_i32), _P(_i32)]
_lib.ffa_plan_periods.argtypes = [_vp, _P(ctypes.c_double)]
_lib.ffa_search.argtypes = [_vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.ffa_prepare.argtypes = [_vp, _vp, _vp, _sz, _vp]
_lib.ffa_search_prepared.argtypes = [_vp, _vp, _vp, _vp, _sz, _vp]
_lib.ffa_fold.argtypes = [_vp, _vp, _i32, _vp, _vp, _sz, _vp]
_lib.ffa_best.argtypes = [_vp, _i64, _vp, _vp]
_lib.ffa_sift.argtypes = [_vp, _vp, _vp, _P(SiftParams), _vp, _i32, _vp, _vp, _sz, _vp]
_lib.ffa_snr_histogram.argtypes = [_vp, _i64, ctypes.c_float, ctypes.c_float, _i32, _vp, _vp]
_lib.ffa_sigma_gauss.argtypes = [_P(ctypes.c_uint64), _i32, _P(ctypes.c_double)]
_lib.ffa_sigma_threshold.argtypes = [_P(ctypes.c_uint64), _i32, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_double, _P(ctypes.c_double)]
_lib.ffa_batch_workspace.argtypes = [_i32, _P(_vp), _P(_sz)]
_lib.ffa_search_batch.argtypes = [_i32, _P(_vp), _P(_vp), _P(_vp), _P(_vp), _vp, _sz, _vp]
_lib.ffa_batch_create.argtypes = [_i32, _P(_vp), _P(_vp)]
_lib.ffa_batch_destroy.argtypes = [_vp]
_lib.ffa_batch_query.argtypes = [_vp, _P(_sz), _P(_i64), _P(_i32)]
_lib.ffa_batch_search.argtypes = [_vp, _P(_vp), _P(_vp), _P(_vp), _vp, _sz, _vp]
_lib.ffa_batch_prepare.argtypes = [_vp, _P(_vp), _vp, _sz, _vp]
_lib.ffa_batch_search_prepared.argtypes = [_vp, _P(_vp), _P(_vp), _vp, _sz, _vp]
_lib.ffa_server_create.argtypes = [_sz, _i32, _i32, _P(_vp)]
_lib.ffa_server_submit.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp, _P(_i64)]
_lib.ffa_server_wait.argtypes = [_vp, _i64, _i64, _vp, _vp, _P(ctypes.c_double)]
_lib.ffa_server_destroy.argtypes = [_vp]
_lib.ffa_debug_server_fail.argtypes = [_vp, _i64]
_lib.ffa_status_str.argtypes = [ctypes.c_int]
_lib.ffa_status_str.restype = ctypes.c_char_p
_lib.ffa_last_error.argtypes = []
_lib.ffa_last_error.restype = ctypes.c_char_p
for _n in EXPORTS:
    if _n not in ("ffa_status_str", "ffa_last_error"):
        getattr(_lib, _n).restype = ctypes.c_int


class FFAError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = _lib.ffa_last_error().decode(errors="replace")
        name = _lib.ffa_status_str(status).decode()
        super().__init__(f"{where}: {name} ({detail})")


def _check(st: int, where: str) -> None:
    if st != FFA_OK:
        raise FFAError(st, where)


def lib() -> ctypes.CDLL:
    return _lib


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


@dataclass
class StepInfo:
    f: int
    P0: int
    m: int
    M: int
    first_trial: int


def plan_opts(opts: dict | None) -> PlanOpts | None:
    """A PlanOpts from a dict of its field names (None or {}: the defaults)."""
    if not opts:
        return None
    bad = set(opts) - set(OPT_NAMES)
    if bad:
        raise ValueError(f"unknown plan options {sorted(bad)}")
    return PlanOpts(**{k: int(v) for k, v in opts.items()})


class Plan:
    """A search plan (ffa_plan_create).  ``dtype`` is "f32" or "u8";
    ``opts`` a dict of ffa_plan_opts fields (launch options)."""

    def __init__(self, N: int, tsamp: float, pmin: float, pmax: float, bins_min: int,
                 widths=None, dtype: str = "f32", snr: int = FFA_SNR_ALG1_MAD, max_octaves: int = 0,
                 dered_window: int = 0, dered_stride: int = 0, opts: dict | None = None):
        self._h = _vp()
        w = list(widths) if widths else []
        self._warr = (ctypes.c_int32 * max(len(w), 1))(*w)
        desc = PlanDesc(N=N, tsamp_s=tsamp, pmin_s=pmin, pmax_s=pmax,
                        widths=ctypes.cast(self._warr, _P(ctypes.c_int32)) if w else None,
                        n_widths=len(w), bins_min=bins_min, max_octaves=max_octaves,
                        dtype=FFA_IN_U8 if dtype == "u8" else FFA_IN_F32, snr=snr,
                        dered_window=dered_window, dered_stride=dered_stride)
        o = plan_opts(opts)
        _check(_lib.ffa_plan_create_opts(ctypes.byref(desc), ctypes.byref(o) if o is not None else None,
                                         ctypes.byref(self._h)), "ffa_plan_create_opts")
        self.opts = dict(opts or {})
        self.N = N
        self.tsamp = tsamp
        self.dtype = dtype
        self.dered_window = dered_window
        nt, ns, ws = _i64(), _i32(), _sz()
        _check(_lib.ffa_plan_query(self._h, ctypes.byref(nt), ctypes.byref(ns), ctypes.byref(ws)),
               "ffa_plan_query")
        self.n_trials, self.n_steps, self.ws_bytes = nt.value, ns.value, ws.value

    @classmethod
    def from_args(cls, pa, snr: int = FFA_SNR_ALG1_MAD, opts: dict | None = None) -> "Plan":
        """From a ``synth.PlanArgs``."""
        return cls(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min, pa.widths, pa.dtype, snr,
                   pa.max_octaves, getattr(pa, "dered_window", 0), getattr(pa, "dered_stride", 0), opts)

    @property
    def handle(self) -> int:
        return self._h.value

    def close(self) -> None:
        if self._h:
            _lib.ffa_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def step(self, s: int) -> StepInfo:
        f, P0, m, M = _i32(), _i32(), _i32(), _i32()
        ft = _i64()
        _check(_lib.ffa_plan_step(self._h, s, ctypes.byref(f), ctypes.byref(P0), ctypes.byref(m),
                                  ctypes.byref(M), ctypes.byref(ft)), "ffa_plan_step")
        return StepInfo(f.value, P0.value, m.value, M.value, ft.value)

    def passes(self, s: int) -> list[int]:
        n = _i32()
        d = (ctypes.c_int32 * 8)()
        _check(_lib.ffa_plan_passes(self._h, s, ctypes.byref(n), d), "ffa_plan_passes")
        return [d[i] for i in range(n.value)]

    def periods(self):
        import numpy as np

        out = np.empty(self.n_trials, dtype=np.float64)
        _check(_lib.ffa_plan_periods(self._h, out.ctypes.data_as(_P(ctypes.c_double))),
               "ffa_plan_periods")
        return out

    # ------------------------------------------------------------ device calls

    def workspace(self, device=None):
        import torch

        return torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device or "cuda")

    @staticmethod
    def _aligned(ws) -> int:
        p = ws.data_ptr()
        return (p + 255) // 256 * 256

    def search(self, series, snr=None, width=None, ws=None, stream=None):
        """Periodogram of ``series`` (a cuda tensor).  Returns (snr f32, width i32)."""
        import torch

        self._check_series(series)
        dev = series.device
        if snr is None:
            snr = torch.empty(self.n_trials, dtype=torch.float32, device=dev)
        if width is None:
            width = torch.empty(self.n_trials, dtype=torch.int32, device=dev)
        if ws is None:
            ws = self.workspace(dev)
        base = self._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        _check(_lib.ffa_search(self._h, series.data_ptr(), snr.data_ptr(), width.data_ptr(), base,
                               avail, _stream_ptr(stream)), "ffa_search")
        return snr, width

    def upload(self) -> None:
        """ffa_plan_upload: the plan's device tables on the current GPU."""
        _check(_lib.ffa_plan_upload(self._h), "ffa_plan_upload")

    def search_noalloc(self, series, snr, width, stream=None):
        """ffa_search_noalloc: the periodogram of ``series`` into ``snr`` and
        ``width`` (preallocated), with the library's fixed scratch as the
        workspace; nothing is allocated.  Needs upload() (or a search) first."""
        self._check_series(series)
        if snr.numel() != self.n_trials or width.numel() != self.n_trials:
            raise ValueError("outputs must hold n_trials entries")
        _check(_lib.ffa_search_noalloc(self._h, series.data_ptr(), snr.data_ptr(), width.data_ptr(),
                                       _stream_ptr(stream)), "ffa_search_noalloc")
        return snr, width

    def prepare(self, series, ws, stream=None):
        """ffa_prepare: octave series of ``series`` into ``ws`` (from workspace())."""
        self._check_series(series)
        base = self._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        _check(_lib.ffa_prepare(self._h, series.data_ptr(), base, avail, _stream_ptr(stream)),
               "ffa_prepare")

    def search_prepared(self, snr, width, ws, stream=None):
        """ffa_search_prepared: every FFA pass and the scoring, on the octave
        series the last prepare() left in ``ws``."""
        if snr.numel() != self.n_trials or width.numel() != self.n_trials:
            raise ValueError("outputs must hold n_trials entries")
        base = self._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        _check(_lib.ffa_search_prepared(self._h, snr.data_ptr(), width.data_ptr(), base, avail,
                                        _stream_ptr(stream)), "ffa_search_prepared")
        return snr, width

    def fold(self, series, step: int, out=None, ws=None, stream=None):
        """Raw profiles (M, P0) of step ``step`` (f32 or exact int32)."""
        import torch

        self._check_series(series)
        info = self.step(step)
        dt = torch.int32 if self.dtype == "u8" and not self.dered_window else torch.float32
        if out is None:
            out = torch.empty((info.M, info.P0), dtype=dt, device=series.device)
        if ws is None:
            ws = self.workspace(series.device)
        base = self._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        _check(_lib.ffa_fold(self._h, series.data_ptr(), step, out.data_ptr(), base, avail,
                             _stream_ptr(stream)), "ffa_fold")
        return out

    def sift(self, snr, width, min_snr: float = 9.0, frac_fall: float = 0.1, abs_fall: float = 1.0,
             group_widths: float = 0.0, harmonic_primes: int = 0, harmonic_tol: float = 1e-5,
             max_cands: int = 1024, ws=None, stream=None, raw: bool = False):
        """ffa_sift: candidates of a periodogram (cuda tensors from search()),
        strongest first.  Returns a numpy record array (trial, period, snr,
        width), or with ``raw`` the device buffer (max_cands, 24 bytes) and the
        one-element int32 count, both on the GPU and not yet synchronised."""
        import numpy as np
        import torch

        if snr.numel() != self.n_trials or width.numel() != self.n_trials:
            raise ValueError("snr and width must hold n_trials entries")
        if snr.dtype != torch.float32 or width.dtype != torch.int32:
            raise ValueError("snr must be float32 and width int32")
        dev = snr.device
        if ws is None:
            ws = self.workspace(dev)
        base = self._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        prm = SiftParams(min_snr, frac_fall, abs_fall, group_widths, harmonic_primes, harmonic_tol)
        cands = torch.empty((max(max_cands, 1), ctypes.sizeof(Candidate)), dtype=torch.uint8, device=dev)
        n = torch.empty(1, dtype=torch.int32, device=dev)
        _check(_lib.ffa_sift(self._h, snr.data_ptr(), width.data_ptr(), ctypes.byref(prm),
                             cands.data_ptr(), max_cands, n.data_ptr(), base, avail,
                             _stream_ptr(stream)), "ffa_sift")
        if raw:
            return cands, n
        k = int(n.item())
        if k < 0:
            raise RuntimeError("ffa_sift: more than 16384 peaks pass the thresholds; raise min_snr")
        k = min(k, max_cands)
        host = cands[:k].cpu().numpy()
        rec = np.frombuffer(host.tobytes(), dtype=np.dtype(
            [("trial", "<i8"), ("period", "<f8"), ("snr", "<f4"), ("width", "<i4")]))
        return rec.copy()

    def _check_series(self, series):
        import torch

        want = torch.uint8 if self.dtype == "u8" else torch.float32
        if series.dtype != want or series.numel() != self.N or not series.is_contiguous():
            raise ValueError(f"series must be a contiguous {want} tensor of {self.N} samples")
        if not series.is_cuda:
            raise ValueError("series must be on the GPU")


def best(snr, stream=None, out=None):
    """Index of the best trial of a periodogram (first on ties), computed on the
    GPU.  Returns it as an int, or, given ``out`` (a one-element int64 cuda
    tensor), writes it there asynchronously and returns ``out``."""
    import torch

    res = out if out is not None else torch.empty(1, dtype=torch.int64, device=snr.device)
    _check(_lib.ffa_best(snr.data_ptr(), snr.numel(), res.data_ptr(), _stream_ptr(stream)), "ffa_best")
    return out if out is not None else int(res.item())


def snr_histogram(snr, lo: float, bins_per_unit: float, n_bins: int, hist=None, stream=None):
    """ffa_snr_histogram: adds the scores of ``snr`` (a float32 cuda tensor)
    to ``hist`` (an int64 cuda tensor of n_bins counts, zeroed when created
    here) and returns it."""
    import torch

    if snr.dtype != torch.float32 or not snr.is_contiguous():
        raise ValueError("snr must be a contiguous float32 tensor")
    if hist is None:
        hist = torch.zeros(n_bins, dtype=torch.int64, device=snr.device)
    if hist.dtype != torch.int64 or hist.numel() != n_bins or not hist.is_contiguous():
        raise ValueError("hist must be a contiguous int64 tensor of n_bins counts")
    _check(_lib.ffa_snr_histogram(snr.data_ptr(), snr.numel(), lo, bins_per_unit, n_bins, hist.data_ptr(),
                                  _stream_ptr(stream)), "ffa_snr_histogram")
    return hist


def _host_counts(hist):
    import numpy as np

    if hasattr(hist, "cpu"):
        hist = hist.cpu().numpy()
    h = np.ascontiguousarray(hist)
    if h.dtype == np.int64:
        h = h.view(np.uint64)
    if h.dtype != np.uint64:
        raise ValueError("counts must be int64 or uint64")
    return h


def sigma_gauss(hist):
    """ffa_sigma_gauss: Gaussian-equivalent sigma at every bin's lower edge."""
    import numpy as np

    h = _host_counts(hist)
    out = np.empty(h.size, np.float64)
    _check(_lib.ffa_sigma_gauss(h.ctypes.data_as(_P(ctypes.c_uint64)), h.size,
                                out.ctypes.data_as(_P(ctypes.c_double))), "ffa_sigma_gauss")
    return out


def sigma_threshold(hist, lo: float, bins_per_unit: float, sigma: float) -> float:
    """ffa_sigma_threshold: the S/N a ``sigma``-sigma detection needs."""
    h = _host_counts(hist)
    out = ctypes.c_double()
    _check(_lib.ffa_sigma_threshold(h.ctypes.data_as(_P(ctypes.c_uint64)), h.size, lo, bins_per_unit, sigma,
                                    ctypes.byref(out)), "ffa_sigma_threshold")
    return out.value


def batch_workspace_bytes(plans) -> int:
    arr = (_vp * len(plans))(*[p.handle for p in plans])
    ws = _sz()
    _check(_lib.ffa_batch_workspace(len(plans), arr, ctypes.byref(ws)), "ffa_batch_workspace")
    return ws.value


def search_batch(plans, series, ws=None, outs=None, stream=None):
    """ffa_search_batch: periodograms of many series (cuda tensors), one plan
    each, run as one work queue.  Returns a list of (snr, width) tensors."""
    import torch

    n = len(plans)
    if n != len(series) or n == 0:
        raise ValueError("need one plan per series")
    for p, x in zip(plans, series):
        p._check_series(x)
    dev = series[0].device
    if outs is None:
        outs = [(torch.empty(p.n_trials, dtype=torch.float32, device=dev),
                 torch.empty(p.n_trials, dtype=torch.int32, device=dev)) for p in plans]
    need = batch_workspace_bytes(plans)
    if ws is None:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    base = Plan._aligned(ws)
    avail = ws.numel() - (base - ws.data_ptr())
    ph = (_vp * n)(*[p.handle for p in plans])
    sp = (_vp * n)(*[x.data_ptr() for x in series])
    so = (_vp * n)(*[o[0].data_ptr() for o in outs])
    wo = (_vp * n)(*[o[1].data_ptr() for o in outs])
    _check(_lib.ffa_search_batch(n, ph, sp, so, wo, base, avail, _stream_ptr(stream)), "ffa_search_batch")
    return outs


class Batch:
    """A planned batch of searches (ffa_batch_create): one work queue over the
    steps of every series.  The plans must outlive it."""

    def __init__(self, plans):
        self.plans = list(plans)
        if not self.plans:
            raise ValueError("need at least one plan")
        h = _vp()
        arr = (_vp * len(self.plans))(*[p.handle for p in self.plans])
        _check(_lib.ffa_batch_create(len(self.plans), arr, ctypes.byref(h)), "ffa_batch_create")
        self._h = h
        ws, nt, nl = _sz(), _i64(), _i32()
        _check(_lib.ffa_batch_query(self._h, ctypes.byref(ws), ctypes.byref(nt), ctypes.byref(nl)),
               "ffa_batch_query")
        self.ws_bytes, self.n_tiles, self.n_launches = ws.value, nt.value, nl.value

    @property
    def handle(self) -> int:
        return self._h.value

    def workspace(self, device=None):
        import torch

        return torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device or "cuda")

    def outputs(self, device=None):
        import torch

        dev = device or "cuda"
        return [(torch.empty(p.n_trials, dtype=torch.float32, device=dev),
                 torch.empty(p.n_trials, dtype=torch.int32, device=dev)) for p in self.plans]

    def search(self, series, outs=None, ws=None, stream=None):
        """ffa_batch_search of ``series`` (cuda tensors, one per plan).
        Returns the list of (snr, width) tensors."""
        n = len(self.plans)
        if len(series) != n:
            raise ValueError("need one series per plan")
        for p, x in zip(self.plans, series):
            p._check_series(x)
        if outs is None:
            outs = self.outputs(series[0].device)
        if ws is None:
            ws = self.workspace(series[0].device)
        base = Plan._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        sp = (_vp * n)(*[x.data_ptr() for x in series])
        so = (_vp * n)(*[o[0].data_ptr() for o in outs])
        wo = (_vp * n)(*[o[1].data_ptr() for o in outs])
        _check(_lib.ffa_batch_search(self._h, sp, so, wo, base, avail, _stream_ptr(stream)), "ffa_batch_search")
        return outs

    def prepare(self, series, ws, stream=None):
        """ffa_batch_prepare: every series' octave series into ``ws``."""
        n = len(self.plans)
        if len(series) != n:
            raise ValueError("need one series per plan")
        for p, x in zip(self.plans, series):
            p._check_series(x)
        base = Plan._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        sp = (_vp * n)(*[x.data_ptr() for x in series])
        _check(_lib.ffa_batch_prepare(self._h, sp, base, avail, _stream_ptr(stream)), "ffa_batch_prepare")

    def search_prepared(self, outs, ws, stream=None):
        """ffa_batch_search_prepared into ``outs`` (as from outputs())."""
        n = len(self.plans)
        if len(outs) != n:
            raise ValueError("need one output pair per plan")
        base = Plan._aligned(ws)
        avail = ws.numel() - (base - ws.data_ptr())
        so = (_vp * n)(*[o[0].data_ptr() for o in outs])
        wo = (_vp * n)(*[o[1].data_ptr() for o in outs])
        _check(_lib.ffa_batch_search_prepared(self._h, so, wo, base, avail, _stream_ptr(stream)),
               "ffa_batch_search_prepared")
        return outs

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.ffa_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


class Server:
    """Continuous-batching search server (ffa_server_*): one HBM pool of
    ``hbm_budget_bytes`` on the current GPU and ``n_streams`` streams.  A
    request that does not fit may be passed by up to ``max_bypass`` later
    ones that do (0, the default: strict arrival order, which kept the tail
    latency lower under heavy load)."""

    def __init__(self, hbm_budget_bytes: int, n_streams: int = 4, max_bypass: int = 0):
        h = _vp()
        _check(_lib.ffa_server_create(ctypes.c_size_t(hbm_budget_bytes), n_streams, max_bypass, ctypes.byref(h)),
               "ffa_server_create")
        self._h = h.value
        self._plans = {}

    def submit(self, plan: Plan, series) -> int:
        """Queue a search of ``series``: a numpy array (copied now) or a cuda
        tensor (read when the request runs, after the work queued on the
        current torch stream so far).  Returns the ticket."""
        import numpy as np

        want = np.uint8 if plan.dtype == "u8" else np.float32
        t = _i64()
        if isinstance(series, np.ndarray):
            if series.dtype != want or series.size != plan.N:
                raise ValueError(f"series must hold {plan.N} {np.dtype(want).name} samples")
            arr = np.ascontiguousarray(series)
            st = _lib.ffa_server_submit(self._h, plan.handle, arr.ctypes.data, 0, None, ctypes.byref(t))
        else:
            import torch

            plan._check_series(series)
            producer = torch.cuda.current_stream(series.device).cuda_stream
            st = _lib.ffa_server_submit(self._h, plan.handle, series.data_ptr(), 1, producer, ctypes.byref(t))
        _check(st, "ffa_server_submit")
        self._plans[t.value] = (plan, series)  # keep both alive until the wait
        return t.value

    def wait(self, ticket: int, timeout_s: float | None = None):
        """Block until ``ticket`` is done.  Returns (snr, width, latency_s) as
        numpy arrays and seconds.  Raises FFAError(FFA_ERR_TIMEOUT) on time-out."""
        import numpy as np

        plan, _ = self._plans[ticket]
        snr = np.empty(plan.n_trials, np.float32)
        wid = np.empty(plan.n_trials, np.int32)
        lat = ctypes.c_double()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        st = _lib.ffa_server_wait(self._h, ticket, us, snr.ctypes.data, wid.ctypes.data, ctypes.byref(lat))
        if st != FFA_ERR_TIMEOUT:
            self._plans.pop(ticket, None)
        _check(st, "ffa_server_wait")
        return snr, wid, lat.value

    def fail_ticket(self, ticket: int) -> None:
        """Test hook (ffa_debug_server_fail): that request fails on admission."""
        _check(_lib.ffa_debug_server_fail(self._h, ticket), "ffa_debug_server_fail")

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.ffa_server_destroy(self._h)
            self._h = None
            self._plans.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
