"""Autotuning of a plan's launch options, cached per GPU architecture and
shape class.

A setting is a dict of ``ffa_plan_opts`` fields, passed to the planner at
plan creation: the LDS budget of a tile (``tile_lds_bytes``, which sets the
pass split and the tile depth, so the rows each workgroup holds), the target
tiles per window group (``window_tiles``), the ring budget (``ring_mb``) and
16-bit first passes for uint8 input (``no_u16``).  None of them changes a
periodogram: uint8 searches stay bit-exact and float searches agree within
rounding.  ``autotune`` times a search of the caller's series under each
candidate setting and keeps the fastest; ``tuned_plan`` creates a plan with
the cached setting of its shape class (the defaults if there is none).
"""
from __future__ import annotations

import json
import math
import os

from . import ffa

KNOBS = ("tile_lds_bytes", "window_tiles", "ring_mb", "no_u16")

# Candidate settings tried by default (the first is the built-in default).
DEFAULT_CANDIDATES = (
    {},
    {"window_tiles": 65536},
    {"window_tiles": 16384},
    {"ring_mb": 8192, "window_tiles": 65536},
    {"ring_mb": 2048},
    {"tile_lds_bytes": 131072},
    {"no_u16": 1},
)


def default_cache_path() -> str:
    return os.environ.get("FFA_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ffa_mi355x_tune.json"))


def shape_class(pa, snr: int = ffa.FFA_SNR_ALG1_MAD) -> str:
    """Plans of one class share a tuned setting: the input type, the
    algorithm, dereddening on or off, log2 N, the base-period floor B and the
    number of period octaves searched."""
    octaves = max(1, math.ceil(math.log2(max(pa.pmax / max(pa.pmin, 1e-12), 1.0 + 1e-9))))
    dered = "dered" if getattr(pa, "dered_window", 0) else "raw"
    return f"{pa.dtype}/alg{snr}/{dered}/n{round(math.log2(pa.N))}/b{pa.bins_min}/oct{octaves}"


def arch_name() -> str:
    import torch

    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def make_plan(pa, setting: dict, snr: int = ffa.FFA_SNR_ALG1_MAD) -> ffa.Plan:
    """A plan with the launch options of ``setting`` (only KNOBS are taken)."""
    opts = {k: int(v) for k, v in (setting or {}).items() if k in KNOBS}
    return ffa.Plan.from_args(pa, snr=snr, opts=opts)


def load_cache(path: str | None = None) -> dict:
    path = path or default_cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or default_cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_setting(pa, snr: int = ffa.FFA_SNR_ALG1_MAD, arch: str | None = None,
                   path: str | None = None) -> dict | None:
    entry = load_cache(path).get(arch or arch_name(), {}).get(shape_class(pa, snr))
    return dict(entry["knobs"]) if entry else None


def tuned_plan(pa, snr: int = ffa.FFA_SNR_ALG1_MAD, path: str | None = None) -> ffa.Plan:
    """A plan with the cached setting of its class, else the defaults."""
    return make_plan(pa, cached_setting(pa, snr, path=path) or {}, snr)


def autotune(pa, series, snr: int = ffa.FFA_SNR_ALG1_MAD, candidates=DEFAULT_CANDIDATES, reps: int = 3,
             path: str | None = None, save: bool = True) -> dict:
    """Time a search of ``series`` (a cuda tensor of the plan's input type)
    under each candidate setting, best of ``reps`` after one warm-up, and
    cache the fastest for the plan's shape class.  Returns
    {"knobs": ..., "ms": ..., "trials": [(setting, ms), ...]}."""
    import torch

    trials = []
    for setting in candidates:
        plan = make_plan(pa, setting, snr)
        snr_t = torch.empty(plan.n_trials, dtype=torch.float32, device=series.device)
        wid_t = torch.empty(plan.n_trials, dtype=torch.int32, device=series.device)
        ws = plan.workspace(series.device)
        plan.search(series, snr_t, wid_t, ws)
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.search(series, snr_t, wid_t, ws)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        trials.append((dict(setting), best))
        del ws, snr_t, wid_t
        plan.close()
    knobs_best, ms = min(trials, key=lambda t: t[1])
    result = {"knobs": knobs_best, "ms": ms, "trials": trials}
    if save:
        data = load_cache(path)
        data.setdefault(arch_name(), {})[shape_class(pa, snr)] = {"knobs": knobs_best, "ms": ms}
        save_cache(data, path)
    return result
