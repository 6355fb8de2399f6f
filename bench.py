"""Benchmark of the FFA search on one MI355X.

Headline (default): the batched workload -- 256 float32 series of 2^18 to
2^22 samples (tsamp 0.512 ms), each with its own period range (Pmin 0.2-1 s,
Pmax 5-30 s), white plus power-law red noise, a pulsar in about 30% of
them, each dereddened by its plan's exact running median (the paper's
default window) -- searched as one batch (ffa_batch_prepare +
ffa_batch_search_prepared: one work queue over every series' steps).  One
step = one search of all 256 series, inputs resident in HBM.  Beside it:
the plain path (ffa_search per series, one after another) on the same
series, with its outputs checked equal; the served stream (Poisson requests
of 2^20..2^23 float32 samples at 0.7 of the measured capacity, p50/p99);
and one search of the 2^20-sample uint8 workload.

Metric: trial*samples/s = sum over FFA executions of M*(m*P0) per second.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the library searches on
one GPU.

Profiling helpers (run under rocprofv3, then summarised by this script):
  --calibrate-copy      after the timed steps, copy 256 MiB device-to-device
                        three times (a plain copy of known size, to scale the
                        HBM byte counters)
  --pmc-summary DB      print per-kernel averages of the counters in a
                        rocprofv3 database and exit
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit VALU operations (no packed
# form is used), in tera-operations per second.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# the sources that decide what the FFA kernel does and how it is launched
PATH_SRC = [os.path.join(ROOT, "paper_1703_05581_amd", "csrc", f)
            for f in ("ffa_kernels.hip", "ffa_plan.cpp", "ffa_batch.cpp")]
TRAFFIC_FILES = {"batch256": os.path.join(ROOT, "profiles", "ffa_tile_kernel.batch256_f32.traffic.md"),
                 "u8_2e20": os.path.join(ROOT, "profiles", "ffa_tile_kernel.u8_2e20.traffic.md")}
COPY_BYTES = 256 << 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=768,
                    help="FFA executions the oracle times for the CPU baseline")
    ap.add_argument("--cpu-steps-1core", type=int, default=48,
                    help="FFA executions timed on one core for the single-core oracle figure (0: skip)")
    ap.add_argument("--check", action="store_true", help="check sampled trials against the oracle")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--pmc-summary", metavar="DB", nargs="+")
    ap.add_argument("--searches", type=int, default=0,
                    help="with --pmc-summary: searches the profiled run made")
    ap.add_argument("--workload", type=int, choices=[1, 2, 3], default=2,
                    help="search and graph modes: workload 2 (the metric's configuration), 3 (HTRU-like, "
                         "dereddened) or 1 (small, launch-bound)")
    ap.add_argument("--alg", type=int, choices=[1, 2], default=1,
                    help="profile score: 1 = Algorithm 1 (the headline), 2 = Algorithm 2")
    ap.add_argument("--mode", choices=["headline", "search", "batch", "served", "null", "graph", "tune"],
                    default="headline",
                    help="headline: the batched workload with plain, served and uint8 figures beside it "
                         "(default); search: one workload's single search; batch: batched against plain "
                         "searches over workload-4 series; served: the request server under "
                         "Poisson arrivals of workload-5 requests")
    ap.add_argument("--series", type=int, default=256, help="headline and batch: series in the batch")
    ap.add_argument("--plain-steps", type=int, default=3, help="headline: passes timed on the plain path")
    ap.add_argument("--no-served", action="store_true", help="headline: skip the served stream")
    ap.add_argument("--no-plain", action="store_true", help="headline: skip the plain path")
    ap.add_argument("--no-u8", action="store_true", help="headline: skip the uint8 workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="headline: CPU time budget of the oracle baseline (whole series, in order)")
    ap.add_argument("--requests", type=int, default=1000, help="served: timed requests")
    ap.add_argument("--max-bypass", type=int, default=0,
                    help="served: later requests that may pass a head that does not fit (0: strict order)")
    ap.add_argument("--load", type=float, nargs="+", default=[0.7],
                    help="served: offered loads / capacity, run in turn")
    return ap.parse_args()


WORKLOAD_TEXT = {
    1: "f32 series 2^16 samples, tsamp 1 ms, P0 500..999 (0.5-1.0 s), one octave, 10 widths, 500 FFA executions",
    2: "uint8 series 2^20 samples, tsamp 1 ms, P0 256..511 at f=1,2,4, 10 widths, 768 FFA executions, "
       "1835008 trials",
    3: "f32 series 2^23 samples (71.6 min at 0.512 ms) with red noise, 0.5-30 s, P0 256..511 at f=2..128, "
       "dereddened with the default 2 s window, 10 widths",
}


def host_threads() -> int:
    """Host threads this process may use (all of them for the oracle)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def workload_units(plan, u8: bool = True, n_widths: int = 10, alg: int = 1):
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
        in_bytes += st.m * st.P0 * (1 if st.f == 1 and u8 else 4)
        # butterfly: L adds per profile bin; Algorithm 1: 2 ops per bin per
        # width (boxcar difference, running max), 1 prefix add, |x - median|,
        # and two exact selections at 2 comparisons per bin each.  Algorithm 2:
        # 1 prefix add and, per width, the box difference, the running max,
        # the kept sum, the deviation and its squared sum (5 ops).
        if alg == 2:
            ops += elts * (L + 1 + 5 * n_widths)
        else:
            ops += elts * (L + 2 * n_widths + 1 + 1 + 4)
    return ts, in_bytes + 8 * trials, ops


def source_hash() -> str:
    """Hash of the kernel and planner sources: counter summaries taken on other
    sources (another kernel, or other launches) are not used."""
    h = hashlib.sha256()
    for path in PATH_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(which: str):
    """HBM bytes per search of the FFA kernel from the committed counter
    summary of a workload, if it was taken on the current kernel source;
    else None."""
    try:
        text = open(TRAFFIC_FILES[which]).read()
    except OSError:
        return None
    h = re.search(r"^path_source_sha256_16: (\w+)", text, re.M)
    b = re.search(r"^traffic_bytes_per_search: ([0-9.eE+]+)", text, re.M)
    if not h or not b or h.group(1) != source_hash():
        return None
    return float(b.group(1))


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def pmc_summary(db_paths, searches: int) -> None:
    """Per-kernel counter means of rocprofv3 databases.  With FETCH_SIZE and
    WRITE_SIZE present (each from its own run with --calibrate-copy), also the
    FFA kernel's HBM bytes per search, each counter scaled by what it reads
    for the 256 MiB device copy."""
    import sqlite3

    print(f"path_source_sha256_16: {source_hash()}")
    print("| kernel | counter | dispatches | mean per dispatch | total |")
    print("|---|---|---|---|---|")
    per_search = {}
    scale = {}
    for path in db_paths:
        db = sqlite3.connect(path)
        rows = db.execute("select kernel_name, counter_name, count(*), sum(value) from counters_collection "
                          "group by kernel_name, counter_name").fetchall()
        for name, ctr, n, total in sorted(rows, key=lambda r: -r[3]):
            print(f"| {_short(name)} | {ctr} | {n} | {total / n:.6g} | {total:.6g} |")
            if "ffa_tile_kernel" in name and searches:
                per_search[ctr] = per_search.get(ctr, 0.0) + total / searches
        # calibration: the copies that moved COPY_BYTES
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = [v for (v,) in db.execute(
                "select value from counters_collection where kernel_name like '%copyBuffer%' "
                "and counter_name = ? and grid_size = ?", (ctr, COPY_BYTES // 2048))]
            if vals:
                scale[ctr] = (COPY_BYTES / 1024) / (sum(vals) / len(vals))
    for ctr, v in sorted(per_search.items()):
        unit = "_KiB" if ctr.endswith("_SIZE") else ""
        print(f"{ctr}{unit}_per_search: {v:.6g}")
    for ctr, f in sorted(scale.items()):
        print(f"{ctr}_scale_from_copy: {f:.4f}")
    if searches and "FETCH_SIZE" in per_search and "WRITE_SIZE" in per_search and len(scale) == 2:
        t = 1024 * (per_search["FETCH_SIZE"] * scale["FETCH_SIZE"] + per_search["WRITE_SIZE"] * scale["WRITE_SIZE"])
        print(f"traffic_bytes_per_search: {t:.6g}")


def copy_bandwidth(dev) -> float:
    """Measured streaming peak: a 256 MiB device copy, read + write bytes per
    second (GB/s)."""
    import torch

    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    gbs = 2 * 5 * COPY_BYTES / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst
    return gbs


def trial_samples(plan) -> int:
    return sum(plan.step(s).M * plan.step(s).m * plan.step(s).P0 for s in range(plan.n_steps))


def run_batch(a) -> dict:
    """Batched (ffa_search_batch over library streams) against plain
    (ffa_search per series, one stream) on the first --series series of
    workload 4; same outputs, checked equal."""
    import torch

    from paper_1703_05581_amd import ffa, synth

    series = [synth.workload4(i) for i in range(a.series)]
    plans = [ffa.Plan.from_args(s.plan) for s in series]
    xs = [torch.from_numpy(s.data).cuda() for s in series]
    outs = [(torch.empty(p.n_trials, dtype=torch.float32, device="cuda"),
             torch.empty(p.n_trials, dtype=torch.int32, device="cuda")) for p in plans]
    wsb = torch.empty(ffa.batch_workspace_bytes(plans) + 256, dtype=torch.uint8, device="cuda")
    ws1 = torch.empty(max(p.ws_bytes for p in plans) + 256, dtype=torch.uint8, device="cuda")
    ts = sum(trial_samples(p) for p in plans)

    def plain():
        for p, x, o in zip(plans, xs, outs):
            p.search(x, o[0], o[1], ws1)

    def batched():
        ffa.search_batch(plans, xs, ws=wsb, outs=outs)

    res = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / a.steps / 1e3
        res[name + "_out"] = [(o[0].clone(), o[1].clone()) for o in outs]
    same = all(torch.equal(x[0], y[0]) and torch.equal(x[1], y[1])
               for x, y in zip(res["plain_out"], res["batched_out"]))
    return {"metric": "FFA trial*samples/s, batched search (workload 4 series)",
            "value": ts / res["batched"], "unit": "trial*samples/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": res["batched"] * 1e3, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic (seeded; workload 4 of paper_1703_05581_amd.synth)",
            "config": {"workload": f"first {a.series} series of workload 4 (f32, 2^18..2^22 samples, "
                                   "own period ranges)", "trial_samples": ts},
            "plain_value": ts / res["plain"], "plain_ms": res["plain"] * 1e3,
            "speedup": res["plain"] / res["batched"], "outputs_equal": same}


def run_graph(a) -> dict:
    """One search captured in a HIP graph and replayed, against the same
    search launched eagerly; every replay's periodogram is checked equal to
    the eager one."""
    import torch

    from paper_1703_05581_amd import ffa, synth

    series = synth.workload(a.workload, 0)
    plan = ffa.Plan.from_args(series.plan, snr=a.alg)
    x = torch.from_numpy(series.data).cuda()
    snr = torch.empty(plan.n_trials, dtype=torch.float32, device="cuda")
    wid = torch.empty(plan.n_trials, dtype=torch.int32, device="cuda")
    ws = plan.workspace()
    for _ in range(max(1, a.warmup)):
        plan.search(x, snr, wid, ws)  # also makes the plan's device tables
    torch.cuda.synchronize()
    ref = (snr.clone(), wid.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.search(x, snr, wid, ws)
    torch.cuda.synchronize()
    same = True
    for _ in range(3):  # replays with eager work in between
        snr.zero_()
        wid.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same &= torch.equal(snr, ref[0]) and torch.equal(wid, ref[1])
    res = {}
    for name, fn in (("eager", lambda: plan.search(x, snr, wid, ws)), ("graph", g.replay)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / a.steps
    same &= torch.equal(snr, ref[0]) and torch.equal(wid, ref[1])
    ts = trial_samples(plan)
    return {"metric": "FFA trial*samples/s, search replayed from a HIP graph",
            "value": ts / (res["graph"] / 1e3), "unit": "trial*samples/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": res["graph"], "higher_is_better": True,
            "dtype": "i32" if series.plan.dtype == "u8" else "f32",
            "data": f"synthetic (seeded; workload {a.workload} of paper_1703_05581_amd.synth)",
            "config": {"workload": WORKLOAD_TEXT[a.workload], "trial_samples": ts},
            "eager_ms": res["eager"], "speedup": res["eager"] / res["graph"], "outputs_equal": same}


def run_tune(a) -> dict:
    """Autotune the plan knobs of the chosen workload (tune.DEFAULT_CANDIDATES)
    and report every candidate's time; the choice goes to the tuning cache."""
    import torch

    from paper_1703_05581_amd import synth, tune

    series = synth.workload(a.workload, 0)
    x = torch.from_numpy(series.data).cuda()
    res = tune.autotune(series.plan, x, snr=a.alg, reps=max(1, a.steps))
    default_ms = res["trials"][0][1]
    return {"metric": "FFA autotuning of the plan knobs", "value": res["ms"], "unit": "ms",
            "higher_is_better": False, "n_gpus": 1, "steps": a.steps,
            "data": f"synthetic (seeded; workload {a.workload} of paper_1703_05581_amd.synth)",
            "config": {"workload": WORKLOAD_TEXT[a.workload], "shape_class": tune.shape_class(series.plan, a.alg),
                       "arch": tune.arch_name()},
            "best_knobs": res["knobs"], "default_ms": default_ms, "speedup_vs_default": default_ms / res["ms"],
            "trials": [{"knobs": k, "ms": ms} for k, ms in res["trials"]]}


HIST_LO, HIST_BPU, HIST_BINS = -8.0, 256.0, 16384  # S/N -8 .. 56 in steps of 1/256


def run_null(a) -> dict:
    """False-alarm statistics of Sec. 4.1.2 on workload 6 (26 white-noise
    series, about 10^8 trials): batched searches with Algorithms 1 and 2, the
    S/N histogram of every periodogram on the GPU, then the S/N each
    Gaussian-equivalent sigma needs.  One step = both algorithms over all
    series, histograms included."""
    import torch

    from paper_1703_05581_amd import ffa, synth

    series = [synth.workload6(i) for i in range(synth.NULL_SERIES)]
    pa = series[0].plan
    xs = [torch.from_numpy(s.data).cuda() for s in series]
    plans = {alg: ffa.Plan.from_args(pa, snr=alg) for alg in (1, 2)}
    nt = plans[1].n_trials
    outs = [(torch.empty(nt, dtype=torch.float32, device="cuda"), torch.empty(nt, dtype=torch.int32, device="cuda"))
            for _ in series]
    wsb = torch.empty(max(ffa.batch_workspace_bytes([p] * len(series)) for p in plans.values()) + 256,
                      dtype=torch.uint8, device="cuda")
    hists = {alg: torch.zeros(HIST_BINS, dtype=torch.int64, device="cuda") for alg in (1, 2)}

    def step():
        for alg in (1, 2):
            hists[alg].zero_()
            ffa.search_batch([plans[alg]] * len(series), xs, ws=wsb, outs=outs)
            for o in outs:
                ffa.snr_histogram(o[0], HIST_LO, HIST_BPU, HIST_BINS, hists[alg])

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / a.steps / 1e3
    trials = 2 * nt * len(series)
    res = {}
    for alg in (1, 2):
        h = hists[alg].cpu().numpy().view("uint64")
        assert int(h.sum()) == nt * len(series), "every trial is counted once"
        res[alg] = {f"{k:g}": round(ffa.sigma_threshold(h, HIST_LO, HIST_BPU, k), 4)
                    for k in (-2.0, -1.0, 0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 5.5)}
    return {"metric": "white-noise false-alarm calibration, S/N trials/s", "value": trials / sec,
            "unit": "trials/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": sec * 1e3,
            "higher_is_better": True, "dtype": "f32",
            "data": "synthetic (seeded; workload 6 of paper_1703_05581_amd.synth)",
            "config": {"workload": "26 white-noise f32 series, 2^21 x 2.048 ms, 1-20 s, base 488 bins, "
                                   "default widths, Algorithms 1 and 2",
                       "trials_per_algorithm": nt * len(series),
                       "histogram": {"lo": HIST_LO, "bins_per_unit": HIST_BPU, "bins": HIST_BINS}},
            "snr_at_sigma_alg1": res[1], "snr_at_sigma_alg2": res[2],
            "paper_5sigma_white_noise": {"alg1": 6.6, "alg2": 7.1}}


def run_served(a, runs_spec=None) -> dict:
    """Request server under Poisson arrivals at a load x its measured
    capacity; latency = submit to the end of the search on the GPU.
    ``runs_spec`` lists (load, max_bypass) pairs, run in turn on a fresh
    server each; by default every --load with --max-bypass."""
    import threading

    import numpy as np

    from paper_1703_05581_amd import ffa, synth, tune

    pool = [synth.workload5(i) for i in range(16)]
    plans = {}
    # the 16 GiB pool holds more large requests with 2 GiB rings than with
    # the default 4 GiB (more requests in flight, higher capacity)
    for s in pool:
        if s.plan.N not in plans:
            plans[s.plan.N] = tune.make_plan(s.plan, {"ring_mb": 2048})
    reqs = [pool[i % len(pool)] for i in range(a.requests + 100)]
    srv = ffa.Server(16 << 30, 4, a.max_bypass)
    # capacity: a closed burst of the same mix
    t0 = time.perf_counter()
    ts = [srv.submit(plans[r.plan.N], r.data) for r in reqs[:64]]
    for t in ts:
        srv.wait(t)
    cap = 64 / (time.perf_counter() - t0)
    srv.close()

    runs = []
    for li, (load, bypass) in enumerate(runs_spec or [(x, a.max_bypass) for x in a.load]):
        srv = ffa.Server(16 << 30, 4, bypass)
        rate = load * cap
        arrivals = synth.poisson_arrivals(7 + li, rate, len(reqs))
        lat, done = [], []
        tickets = []
        lock = threading.Lock()

        def collector():
            i = 0
            while i < len(reqs):
                with lock:
                    have = len(tickets)
                if i >= have:
                    time.sleep(1e-4)
                    continue
                _, _, l = srv.wait(tickets[i])
                if i >= 100:
                    lat.append(l)
                done.append(time.perf_counter())
                i += 1

        th = threading.Thread(target=collector)
        th.start()
        start = time.perf_counter()
        for r, at in zip(reqs, arrivals):
            now = time.perf_counter() - start
            if at > now:
                time.sleep(at - now)
            t = srv.submit(plans[r.plan.N], r.data)
            with lock:
                tickets.append(t)
        th.join()
        srv.close()
        span = done[-1] - done[100]
        served_ts = sum(trial_samples(plans[r.plan.N]) for r in reqs[101:])
        lat = np.array(lat)
        runs.append({"load": load, "max_bypass": bypass, "offered_rate_hz": rate,
                     "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                     "served_trial_samples_per_s": served_ts / span})
        print(f"served load {load} max_bypass {bypass}: p50 {runs[-1]['p50_s'] * 1e3:.1f} ms "
              f"p99 {runs[-1]['p99_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    first = runs[0]
    return {"metric": "FFA served requests: submit-to-result latency (workload 5)",
            "value": first["p50_s"], "unit": "s", "higher_is_better": False,
            "n_gpus": 1, "p50_s": first["p50_s"], "p99_s": first["p99_s"],
            "requests": a.requests, "warmup_requests": 100, "capacity_hz": cap, "loads": runs,
            "dtype": "f32", "data": "synthetic (seeded; workload 5 of paper_1703_05581_amd.synth)",
            "config": {"workload": "Poisson arrivals of f32 requests, 2^20..2^23 samples, "
                                   "P0 256..511 at f=1,2,4; 16 GiB pool, 4 streams"}}


def load_workload4(count: int):
    """The first ``count`` series of workload 4, generated in parallel."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_1703_05581_amd import synth

    with ThreadPoolExecutor(max(1, min(16, host_threads()))) as ex:
        return list(ex.map(synth.workload4, range(count)))


def run_headline(a) -> dict:
    """The batched workload (all 256 series of workload 4 as one batch), the
    plain path beside it, the served stream and the uint8 workload."""
    import numpy as np
    import torch

    from paper_1703_05581_amd import ffa

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    series = load_workload4(a.series)
    plans = [ffa.Plan.from_args(s.plan) for s in series]
    xs = [torch.from_numpy(s.data).to(dev) for s in series]
    gen_s = time.perf_counter() - t_gen
    batch = ffa.Batch(plans)
    outs = batch.outputs(dev)
    ws = batch.workspace(dev)
    ts, alg_bytes, alg_ops = 0, 0, 0
    for s, p in zip(series, plans):
        t, b, o = workload_units(p, False, len(s.plan.widths), 1)
        ts, alg_bytes, alg_ops = ts + t, alg_bytes + b, alg_ops + o
    trials = sum(p.n_trials for p in plans)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        batch.prepare(xs, ws)
        batch.search_prepared(outs, ws)
    torch.cuda.synchronize()
    # e0..e1 brackets the octave series and dereddening of every series,
    # e1..e2 exactly the FFA kernel launches (and the output table) of a step
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        batch.prepare(xs, ws)
        e1.record(stream)
        batch.search_prepared(outs, ws)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[0][0].elapsed_time(ev[-1][2]) / a.steps
    sec = ms / 1e3
    kern_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / a.steps
    prep_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / a.steps
    ksec = kern_ms / 1e3
    out = {
        "metric": "FFA trial*samples/s incl. boxcar S/N (batched vs plain); served p50/p99 latency",
        "value": ts / sec,
        "unit": "trial*samples/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; workload 4 of paper_1703_05581_amd.synth)",
        "config": {"workload": f"batched: {a.series} f32 series of 2^18..2^22 samples (tsamp 0.512 ms), "
                               "own period ranges (Pmin 0.2-1 s, Pmax 5-30 s), white + red noise, exact "
                               "running-median dereddening (default window), 10 widths, Algorithm 1, "
                               "one batch (ffa_batch_search)",
                   "series": a.series, "N_total": int(sum(p.N for p in plans)), "trials": int(trials),
                   "executions": int(sum(p.n_steps for p in plans)), "trial_samples": int(ts),
                   "batch_tiles": batch.n_tiles, "batch_launches": batch.n_launches},
        "roofline": {
            "bound": "alu",
            "kernel": "ffa_tile_kernel (all launches of one batched search)",
            "achieved": alg_ops / ksec / 1e12,
            "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": alg_ops / ksec / 1e12 / VALU_PEAK_TOPS,
            "traffic": stored_traffic("batch256") if a.series == 256 else None,
            "kernel_ms_per_search": kern_ms,
        },
        "prepare_ms_per_search": prep_ms,
        "hbm": {"algorithmic_bytes": alg_bytes, "achieved_GBs": alg_bytes / sec / 1e9,
                "frac_of_8TBs": alg_bytes / sec / 1e9 / HBM_PEAK_GBS},
        "wall_s": wall,
        "generate_s": gen_s,
    }
    if a.calibrate_copy:  # a plain copy of known size for the byte counters
        src = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    else:
        out["hbm"]["copy_GBs"] = copy_bandwidth(dev)
        out["hbm"]["frac_of_copy"] = out["hbm"]["achieved_GBs"] / out["hbm"]["copy_GBs"]
    if not a.no_plain:
        wsp = torch.empty(max(p.ws_bytes for p in plans) + 256, dtype=torch.uint8, device=dev)
        pouts = [(torch.empty(p.n_trials, dtype=torch.float32, device=dev),
                  torch.empty(p.n_trials, dtype=torch.int32, device=dev)) for p in plans]

        def plain():
            for p, x, o in zip(plans, xs, pouts):
                p.search(x, o[0], o[1], wsp)

        plain()
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for _ in range(a.plain_steps):
            plain()
        p1.record(stream)
        torch.cuda.synchronize()
        plain_ms = p0.elapsed_time(p1) / a.plain_steps
        same = all(torch.equal(o[0], q[0]) and torch.equal(o[1], q[1]) for o, q in zip(outs, pouts))
        out["plain"] = {"value": ts / (plain_ms / 1e3), "ms_per_step": plain_ms, "steps": a.plain_steps,
                        "path": "ffa_search per series, one after another on one stream"}
        out["speedup"] = plain_ms / ms
        out["outputs_equal_plain"] = bool(same)
        del wsp, pouts
    # the oracle on whole series, in order, within the time budget; those
    # series' GPU periodograms are checked against it on the way
    if not a.no_cpu_baseline:
        import oracle

        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import check_periodogram, step_trials

        threads = host_threads()
        done, cpu_ts, cpu_s, worst, ok = 0, 0, 0.0, 0.0, True
        for s, p, o in zip(series, plans, outs):
            pa = s.plan
            op = oracle.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
            W = oracle.dered_default_window(pa.tsamp, pa.pmin, pa.pmax)
            c0 = time.perf_counter()
            so, wo = oracle.search(s.data, op, list(pa.widths), alg=1, threads=threads, dered_window=W,
                                   dered_stride=pa.dered_stride)
            cpu_s += time.perf_counter() - c0
            cpu_ts += trial_samples(p)
            done += 1
            try:
                summ = check_periodogram(oracle, s.data, op, list(pa.widths), o[0].cpu().numpy(),
                                         o[1].cpu().numpy(), so, wo, step_trials(op, range(op.n_steps)),
                                         exact=False, dered_window=W, dered_stride=pa.dered_stride)
                worst = max(worst, summ["max_abs_dsnr"])
            except AssertionError as e:  # reported, not raised: the line must still print
                ok = False
                out["check_error"] = str(e)[:300]
            if cpu_s >= a.cpu_seconds:
                break
        out["cpu_baseline"] = {"value": cpu_ts / cpu_s, "unit": "trial*samples/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"series 0..{done - 1} of the {a.series} (whole searches, dereddening "
                                         f"included), {cpu_ts:.3e} trial*samples in {cpu_s:.1f} s",
                               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        out["check"] = {"series": done, "trials": int(sum(p.n_trials for p in plans[:done])),
                        "max_abs_dsnr": worst, "within_tolerance": ok}
        # the oracle on one core: every 16th step of series 0 (dereddening included)
        s0, plan0 = series[0], plans[0]
        pa = s0.plan
        op = oracle.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
        sel = list(range(0, op.n_steps, 16))
        W = oracle.dered_default_window(pa.tsamp, pa.pmin, pa.pmax)
        c0 = time.perf_counter()
        oracle.search(s0.data, op, list(pa.widths), alg=1, threads=1, dered_window=W,
                      dered_stride=pa.dered_stride, steps=sel)
        one_s = time.perf_counter() - c0
        one_ts = sum(plan0.step(k).M * plan0.step(k).m * plan0.step(k).P0 for k in sel)
        out["cpu_baseline"]["one_core"] = {
            "value": one_ts / one_s, "unit": "trial*samples/s", "cores": 1,
            "sample": f"every 16th step of series 0 ({len(sel)} of {op.n_steps}, dereddening of its octaves "
                      f"included), {one_ts:.3e} trial*samples in {one_s:.1f} s"}
    if not a.no_u8:
        u8 = run_search(argparse.Namespace(**{**vars(a), "workload": 2, "alg": 1, "check": False}), cpu=False)
        out["workload2_single_search"] = {
            "workload": u8["config"]["workload"], "value": u8["value"], "ms_per_step": u8["ms_per_step"],
            "dtype": "i32", "roofline": u8["roofline"], "hbm": u8["hbm"], "best_trial": u8["best_trial"]}
    if not a.no_served:
        # 0.7 x capacity with the chosen admission (strict arrival order by
        # default), then 0.9 x capacity in strict order and with backfill
        srv = run_served(a, [(0.7, a.max_bypass), (0.5, a.max_bypass), (0.9, 0), (0.9, 4)])
        out["served"] = {k: srv[k] for k in ("p50_s", "p99_s", "capacity_hz", "requests", "warmup_requests", "config")}
        out["served"]["served_trial_samples_per_s"] = srv["loads"][0]["served_trial_samples_per_s"]
        out["served"]["load"] = 0.7
        out["served"]["max_bypass"] = a.max_bypass
        out["served"]["at_0.5"] = {"p50_s": srv["loads"][1]["p50_s"], "p99_s": srv["loads"][1]["p99_s"]}
        out["served"]["admission_at_0.9"] = {
            ("strict" if r["max_bypass"] == 0 else f"backfill_{r['max_bypass']}"):
                {"p50_s": r["p50_s"], "p99_s": r["p99_s"]} for r in srv["loads"][2:]}
    return out


def run_search(a, cpu: bool = True) -> dict:
    """One search of one workload per step (prepare, every FFA pass and the
    scoring, best trial), with the series resident in HBM."""
    import numpy as np
    import torch

    from paper_1703_05581_amd import ffa, synth

    dev = torch.device("cuda:0")
    series = synth.workload(a.workload, 0)
    pa = series.plan
    plan = ffa.Plan.from_args(pa, snr=a.alg)
    x = torch.from_numpy(series.data).to(dev)
    snr = torch.empty(plan.n_trials, dtype=torch.float32, device=dev)
    wid = torch.empty(plan.n_trials, dtype=torch.int32, device=dev)
    ws = plan.workspace(dev)
    ts, alg_bytes, alg_ops = workload_units(plan, pa.dtype == "u8", len(pa.widths), a.alg)

    best_t = torch.empty(1, dtype=torch.int64, device=dev)
    for _ in range(a.warmup):
        plan.prepare(x, ws)
        plan.search_prepared(snr, wid, ws)
        ffa.best(snr, out=best_t)
    torch.cuda.synchronize()
    # The library launches on torch's current stream, where the events are
    # recorded: e_mid..e_end brackets exactly the FFA kernel launches of a step.
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e_beg, e_mid, e_end, e_best in ev:
        e_beg.record(stream)
        plan.prepare(x, ws)
        e_mid.record(stream)
        plan.search_prepared(snr, wid, ws)
        e_end.record(stream)
        ffa.best(snr, out=best_t)
        e_best.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[0][0].elapsed_time(ev[-1][3]) / a.steps
    sec = ms / 1e3
    kern_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / a.steps
    prep_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / a.steps
    best_ms = sum(e[2].elapsed_time(e[3]) for e in ev) / a.steps
    ksec = kern_ms / 1e3
    traffic = stored_traffic("u8_2e20") if a.workload == 2 and a.alg == 1 else None

    out = {
        "metric": f"FFA trial*samples/s incl. boxcar S/N (Algorithm {a.alg})",
        "value": ts / sec,
        "unit": "trial*samples/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32" if pa.dtype == "u8" else "f32",
        "data": f"synthetic (seeded; workload {a.workload} of paper_1703_05581_amd.synth)",
        "config": {"workload": WORKLOAD_TEXT[a.workload],
                   "N": pa.N, "trials": plan.n_trials, "executions": plan.n_steps,
                   "trial_samples": ts},
        "roofline": {
            "bound": "alu",
            "kernel": "ffa_tile_kernel (all launches of one search)",
            "achieved": alg_ops / ksec / 1e12,
            "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": alg_ops / ksec / 1e12 / VALU_PEAK_TOPS,
            "traffic": traffic,
            "kernel_ms_per_search": kern_ms,
        },
        "prepare_ms_per_search": prep_ms,
        "best_ms_per_search": best_ms,
        "hbm": {"algorithmic_bytes": alg_bytes, "achieved_GBs": alg_bytes / sec / 1e9,
                "frac_of_8TBs": alg_bytes / sec / 1e9 / HBM_PEAK_GBS},
        "wall_s": wall,
    }
    best = int(best_t.item())
    per = plan.periods()
    out["best_trial"] = {"index": best, "period_s": float(per[best]),
                         "snr": float(snr[best].item()), "width": int(wid[best].item())}

    if a.calibrate_copy:
        src = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    else:
        copy_gbs = copy_bandwidth(dev)
        out["hbm"]["copy_GBs"] = copy_gbs
        out["hbm"]["frac_of_copy"] = out["hbm"]["achieved_GBs"] / copy_gbs

    if a.check or (cpu and not a.no_cpu_baseline):
        import oracle

        op = oracle.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
        g = np.random.default_rng(1)
        sel = np.sort(g.choice(op.n_steps, size=min(a.cpu_steps, op.n_steps), replace=False))
        threads = host_threads()
        t0 = time.perf_counter()
        dw = oracle.dered_default_window(pa.tsamp, pa.pmin, pa.pmax) if pa.dered_window == -1 else pa.dered_window
        snr_o, w_o = oracle.search(series.data, op, list(pa.widths), alg=a.alg, steps=sel, threads=threads,
                                   dered_window=dw, dered_stride=pa.dered_stride)
        cpu_s = time.perf_counter() - t0
        sample_ts = int(sum(int(op.M[s]) * int(op.m[s]) * int(op.P0[s]) for s in sel))
        out["cpu_baseline"] = {"value": sample_ts / cpu_s, "unit": "trial*samples/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{sel.size} of {op.n_steps} FFA executions of the same "
                                         f"series, {sample_ts:.3e} trial*samples in {cpu_s:.1f} s",
                               "cpu_model": cpu_model()}
        if a.cpu_steps_1core > 0 and not a.check:
            sel1 = sel[:: max(1, sel.size // a.cpu_steps_1core)][: a.cpu_steps_1core]
            t1 = time.perf_counter()
            oracle.search(series.data, op, list(pa.widths), alg=a.alg, steps=sel1, threads=1, dered_window=dw,
                          dered_stride=pa.dered_stride)
            s1 = time.perf_counter() - t1
            ts1 = int(sum(int(op.M[s]) * int(op.m[s]) * int(op.P0[s]) for s in sel1))
            out["cpu_baseline"]["one_core"] = {"value": ts1 / s1, "unit": "trial*samples/s",
                                               "sample": f"{sel1.size} FFA executions, {ts1:.3e} "
                                                         f"trial*samples in {s1:.1f} s"}
        if a.check:
            sys.path.insert(0, os.path.join(ROOT, "tests"))
            from parity import check_periodogram, step_trials

            idx = step_trials(op, sel)
            exact = pa.dtype == "u8" and not pa.dered_window
            summ = check_periodogram(oracle, series.data, op, list(pa.widths), snr.cpu().numpy(),
                                     wid.cpu().numpy(), snr_o, w_o, idx, exact=exact, alg=a.alg,
                                     dered_window=dw, dered_stride=pa.dered_stride)
            out["check"] = (f"{idx.size} trials bit-exact" if exact else
                            f"{idx.size} trials, max |dS/N| {summ['max_abs_dsnr']:.2e}")
    return out


def torch_init():
    import torch

    torch.cuda.init()


def main():
    a = parse()
    if a.pmc_summary:
        pmc_summary(a.pmc_summary, a.searches)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the FFA search runs on one GPU; --gpus must be 1 "
                                   "(no multi-GPU path is built)"}))
        sys.exit(2)
    torch_init()
    fn = {"headline": run_headline, "search": run_search, "batch": run_batch, "served": run_served,
          "null": run_null, "graph": run_graph, "tune": run_tune}[a.mode]
    print(json.dumps(fn(a)))


if __name__ == "__main__":
    main()
