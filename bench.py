"""Benchmark of the FFA search on one MI355X.

Workload: one 2^20-sample uint8 series (tsamp 1 ms, N(128, 16^2) noise with
three pulsars), base periods P0 in [256, 512) bins over octaves f = 1, 2, 4
(0.256-2.048 s), ten boxcar widths; 768 FFA executions, 1,835,008 trials.
One step = one ffa_search of that series (downsampling, every FFA butterfly
level, Algorithm 1 scoring of every folded profile, periodogram written), with
the series already resident in HBM.

Metric: trial*samples/s = sum over executions of M*(m*P0) per second.

Prints one JSON line.  `--gpus N` with N > 1 is refused: this build runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit VALU operations (no packed
# form is used), in tera-operations per second.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=48,
                    help="FFA executions the oracle times for the CPU baseline")
    ap.add_argument("--check", action="store_true", help="check sampled trials against the oracle")
    return ap.parse_args()


def workload_units(plan):
    """trial*samples, algorithmic bytes and algorithmic operations of one search."""
    ts = 0
    in_bytes = 0
    ops = 0
    trials = plan.n_trials
    for s in range(plan.n_steps):
        st = plan.step(s)
        L = st.M.bit_length() - 1
        elts = st.M * st.P0
        ts += st.M * st.m * st.P0
        # one read of the step's m*P0 samples: uint8 at f = 1, int32 sums above
        in_bytes += st.m * st.P0 * (1 if st.f == 1 else 4)
        # butterfly: L adds per profile bin; Algorithm 1: 2 ops per bin per
        # width (boxcar difference, running max), 1 prefix add, |x - median|,
        # and two exact selections at 2 comparisons per bin each.
        ops += elts * (L + 2 * 10 + 1 + 1 + 4)
    return ts, in_bytes + 8 * trials, ops


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1703_05581_amd import ffa, synth

    torch.cuda.init()
    dev = torch.device("cuda:0")
    series = synth.workload2(0)
    pa = series.plan
    plan = ffa.Plan.from_args(pa)
    x = torch.from_numpy(series.data).to(dev)
    snr = torch.empty(plan.n_trials, dtype=torch.float32, device=dev)
    wid = torch.empty(plan.n_trials, dtype=torch.int32, device=dev)
    ws = plan.workspace(dev)
    ts, alg_bytes, alg_ops = workload_units(plan)

    for _ in range(a.warmup):
        plan.search(x, snr, wid, ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(a.steps):
        plan.search(x, snr, wid, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / a.steps
    sec = ms / 1e3

    out = {
        "metric": "FFA trial*samples/s incl. boxcar S/N (Algorithm 1)",
        "value": ts / sec,
        "unit": "trial*samples/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8->i32",
        "data": "synthetic (seeded; workload 2 of paper_1703_05581_amd.synth)",
        "config": {"workload": "uint8 series 2^20 samples, tsamp 1 ms, P0 256..511 at f=1,2,4, "
                               "10 widths, 768 FFA executions, 1835008 trials",
                   "N": pa.N, "trials": plan.n_trials, "executions": plan.n_steps,
                   "trial_samples": ts},
        "roofline": {
            "bound": "alu",
            "achieved": alg_ops / sec / 1e12,
            "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": alg_ops / sec / 1e12 / VALU_PEAK_TOPS,
            "traffic": None,
        },
        "hbm": {"algorithmic_bytes": alg_bytes, "achieved_GBs": alg_bytes / sec / 1e9,
                "frac_of_8TBs": alg_bytes / sec / 1e9 / HBM_PEAK_GBS},
        "wall_s": wall,
    }
    best = ffa.best(snr)
    per = plan.periods()
    out["best_trial"] = {"index": best, "period_s": float(per[best]),
                         "snr": float(snr[best].item()), "width": int(wid[best].item())}

    if a.check or not a.no_cpu_baseline:
        import oracle

        op = oracle.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
        g = np.random.default_rng(1)
        sel = np.sort(g.choice(op.n_steps, size=min(a.cpu_steps, op.n_steps), replace=False))
        threads = os.cpu_count() or 1
        t0 = time.perf_counter()
        snr_o, w_o = oracle.search(series.data, op, list(pa.widths), steps=sel, threads=threads)
        cpu_s = time.perf_counter() - t0
        sample_ts = int(sum(int(op.M[s]) * int(op.m[s]) * int(op.P0[s]) for s in sel))
        out["cpu_baseline"] = {"value": sample_ts / cpu_s, "unit": "trial*samples/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{sel.size} of {op.n_steps} FFA executions (seeded pick), "
                                         f"{sample_ts:.3e} trial*samples in {cpu_s:.1f} s"}
        if a.check:
            sys.path.insert(0, os.path.join(ROOT, "tests"))
            from parity import check_periodogram, step_trials

            idx = step_trials(op, sel)
            check_periodogram(oracle, series.data, op, list(pa.widths), snr.cpu().numpy(),
                              wid.cpu().numpy(), snr_o, w_o, idx, exact=True)
            out["check"] = f"{idx.size} trials bit-exact"
    print(json.dumps(out))


if __name__ == "__main__":
    main()
