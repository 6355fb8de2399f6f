"""Comparison of the GPU search with the oracle (shared by the GPU tests,
smoke() and the benchmark's self-check).

Tolerances (uint8 input is exact; float32 follows the stated bounds):
  uint8 : profiles bit-exact (int32 vs int64); S/N bit-exact as float32;
          widths identical.
  f32   : profiles |g - o| <= 1e-5 * max|o| per profile; S/N |g - o| <= 1e-4;
          width identical unless the oracle's S/N at the GPU's width is within
          2e-4 of its best; best trial identical unless the oracle's S/N there
          is within 2e-4 of its maximum.
"""
from __future__ import annotations

import numpy as np

SNR_ATOL = 1e-4
TIE_ATOL = 2e-4
PROFILE_RTOL = 1e-5


def step_trials(plan_o, steps) -> np.ndarray:
    idx = [np.arange(plan_o.first[s], plan_o.first[s] + plan_o.M[s]) for s in steps]
    return np.concatenate(idx) if idx else np.zeros(0, np.int64)


def _trial_step(plan_o, trial: int) -> tuple[int, int]:
    s = int(np.searchsorted(plan_o.first, trial, side="right") - 1)
    return s, int(trial - plan_o.first[s])


def check_periodogram(oracle, series, plan_o, widths, snr_g, w_g, snr_o, w_o, idx, exact: bool,
                      alg: int = 1, dered_window: int = 0, dered_stride: int = 0) -> dict:
    """Assert parity on trials ``idx``; return a summary."""
    sg, so = snr_g[idx], snr_o[idx]
    wg, wo = w_g[idx], w_o[idx]
    assert np.isfinite(sg).all(), "non-finite GPU S/N"
    if exact:
        bad = np.nonzero((sg != so) | (wg != wo))[0]
        assert bad.size == 0, (
            f"{bad.size} trials differ; first trial {idx[bad[0]]}: gpu ({sg[bad[0]]!r}, {wg[bad[0]]}) "
            f"oracle ({so[bad[0]]!r}, {wo[bad[0]]})")
    else:
        d = np.abs(sg.astype(np.float64) - so.astype(np.float64))
        assert d.max(initial=0.0) <= SNR_ATOL, f"max |dS/N| {d.max()} at trial {idx[int(np.argmax(d))]}"
        mism = np.nonzero(wg != wo)[0]
        for i in mism[:200]:
            t = int(idx[i])
            s, k = _trial_step(plan_o, t)
            prof = oracle.fold_step(series, int(plan_o.f[s]), int(plan_o.P0[s]), int(plan_o.m[s]),
                                    int(plan_o.M[s]), dered_window=dered_window,
                                    dered_stride=dered_stride)[k]
            fn = oracle.alg1 if alg == 1 else oracle.alg2
            at_gpu = fn(prof, [int(wg[i])])[0]
            assert abs(at_gpu - float(so[i])) <= TIE_ATOL, (t, int(wg[i]), int(wo[i]), at_gpu, so[i])
        assert mism.size <= max(5, idx.size // 1000), f"{mism.size} width mismatches"
    # best trial
    bo = int(np.argmax(so))
    bg = int(np.argmax(sg))
    if exact:
        assert bg == bo
    elif bg != bo:
        assert float(so[bg]) >= float(so[bo]) - TIE_ATOL, (idx[bg], idx[bo])
    return {"trials": int(idx.size), "max_abs_dsnr": float(np.abs(sg.astype(np.float64) - so).max(initial=0)),
            "best_trial": int(idx[bo]), "best_snr": float(so[bo])}


def check_profiles(prof_g: np.ndarray, prof_o: np.ndarray, exact: bool) -> float:
    assert prof_g.shape == prof_o.shape, (prof_g.shape, prof_o.shape)
    if exact:
        assert np.array_equal(prof_g.astype(np.int64), prof_o), "integer profiles differ"
        return 0.0
    scale = np.maximum(np.abs(prof_o).max(axis=1, keepdims=True), 1e-30)
    rel = (np.abs(prof_g.astype(np.float64) - prof_o) / scale).max()
    assert rel <= PROFILE_RTOL, f"profile relative error {rel}"
    return float(rel)


def pulsar_snr(periods, snr, period_s, rel=1e-3):
    """Largest S/N over the trials whose period lies within a relative
    ``rel`` of ``period_s`` (an injected pulsar's own peak, wherever the
    periodogram's maximum is)."""
    near = np.abs(periods / period_s - 1.0) < rel
    assert near.any(), period_s
    return float(np.max(snr[near]))
