"""GPU search and fold against the oracle, through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

from parity import check_periodogram, check_profiles, pulsar_snr, step_trials

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def ffa():
    from paper_1703_05581_amd import ffa as mod

    return mod


def _sample_steps(plan_o, count: int) -> list[int]:
    n = plan_o.n_steps
    if n <= count:
        return list(range(n))
    picks = set(np.linspace(0, n - 1, count).round().astype(int).tolist())
    # every octave's first and last step
    for f in np.unique(plan_o.f):
        where = np.nonzero(plan_o.f == f)[0]
        picks.update([int(where[0]), int(where[-1])])
    return sorted(picks)


def run_case(torch, ffa, oracle, x, N, tsamp, pmin, pmax, B, widths, dtype, steps_max=None,
             check_fold=0, max_octaves=0, alg=1, dered_window=0, dered_stride=0, opts=None):
    # uint8 input is folded and scored from exact integers by both
    # algorithms; a dereddened series is real-valued, so it is compared
    # within the float tolerance also for uint8 input.
    exact = dtype == "u8" and dered_window == 0
    print(f"case N={N} tsamp={tsamp} P=[{pmin},{pmax}) B={B} widths={widths} {dtype} alg{alg} "
          f"dered={dered_window}/{dered_stride}", flush=True)
    plan = ffa.Plan(N, tsamp, pmin, pmax, B, widths, dtype, snr=alg, max_octaves=max_octaves,
                    dered_window=dered_window, dered_stride=dered_stride, opts=opts)
    W = oracle.dered_default_window(tsamp, pmin, pmax) if dered_window == -1 else dered_window
    xt = torch.from_numpy(x).cuda()
    snr, wid = plan.search(xt)
    torch.cuda.synchronize()
    snr_g, w_g = snr.cpu().numpy(), wid.cpu().numpy()
    op = oracle.plan(N, tsamp, pmin, pmax, B, max_octaves)
    steps = list(range(op.n_steps)) if steps_max is None else _sample_steps(op, steps_max)
    snr_o, w_o = oracle.search(x, op, widths, alg=alg, steps=steps, dered_window=W,
                               dered_stride=dered_stride)
    idx = step_trials(op, steps)
    summary = check_periodogram(oracle, x, op, widths, snr_g, w_g, snr_o, w_o, idx, exact, alg=alg,
                                dered_window=W, dered_stride=dered_stride)
    for s in steps[:: max(1, len(steps) // max(check_fold, 1))][:check_fold]:
        prof = plan.fold(xt, s).cpu().numpy()
        ref = oracle.fold_step(x, int(op.f[s]), int(op.P0[s]), int(op.m[s]), int(op.M[s]),
                               dered_window=W, dered_stride=dered_stride)
        check_profiles(prof, ref, exact)
    return plan, summary


W10 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]

# (N, tsamp, pmin, pmax, B, widths) -- small searches that cover: m = 2, m a
# power of two and one above it, odd and prime P0, P0 in every register class
# (<= 64, 128, 256, 512, 1024, 2048), one, two and three passes, widths above P0.
SMALL = [
    (1000, 1e-3, 0.300, 0.600, 300, [1, 2, 4]),            # m = 2 and 3 (L = 1, 2)
    (6000, 1e-3, 0.020, 0.120, 20, [1, 2, 4, 8, 16, 32, 64]),  # P0 < 64, widths > P0 dropped
    (20000, 1e-3, 0.070, 0.250, 70, W10),                   # P0 in (64, 140)
    (65536, 1e-3, 0.5, 1.0, 500, W10),                      # P0 500..999, 2-pass
    (30000, 1e-3, 0.200, 0.520, 200, W10),                  # 256 < P0 < 512 and below
    (50000, 1e-3, 1.900, 2.200, 1000, [1, 2, 4, 8]),        # P0 near 2047, 2 passes
]


@pytest.mark.parametrize("case", SMALL, ids=[f"N{c[0]}_B{c[4]}" for c in SMALL])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_small_search_and_fold(torch_cuda, ffa, oracle_mod, case, dtype):
    from paper_1703_05581_amd import synth

    N, tsamp, pmin, pmax, B, widths = case
    x = synth.random_series(7 + N, N, dtype)
    run_case(torch_cuda, ffa, oracle_mod, x, N, tsamp, pmin, pmax, B, widths, dtype,
             steps_max=40, check_fold=4)


def test_three_pass_u8(torch_cuda, ffa, oracle_mod):
    """Large P0 with enough rows to need three passes."""
    from paper_1703_05581_amd import synth

    N, B = 600000, 1000
    plan = ffa.Plan(N, 1e-3, 1.990, 2.010, B, [1, 2, 4, 8])
    assert max(len(plan.passes(s)) for s in range(plan.n_steps)) >= 3
    x = synth.random_series(99, N, "u8")
    run_case(torch_cuda, ffa, oracle_mod, x, N, 1e-3, 1.990, 2.010, B, [1, 2, 4, 8], "u8",
             steps_max=3, check_fold=2)


def test_default_widths_and_octave_limit(torch_cuda, ffa, oracle_mod):
    from paper_1703_05581_amd import synth

    x = synth.random_series(3, 100000, "u8")
    run_case(torch_cuda, ffa, oracle_mod, x, 100000, 1e-3, 0.1, 1.6, 100, None, "u8",
             steps_max=30, max_octaves=3)


def test_mad_zero(torch_cuda, ffa, oracle_mod):
    """A constant series folds to constant profiles: MAD = 0 gives S/N 0, width 0."""
    x = np.full(20000, 128, np.uint8)
    plan, _ = run_case(torch_cuda, ffa, oracle_mod, x, 20000, 1e-3, 0.3, 0.6, 300, [1, 2, 4], "u8")
    snr, wid = plan.search(torch_cuda.from_numpy(x).cuda())
    assert float(snr.abs().max()) == 0.0 and int(wid.abs().max()) == 0


def test_f32_large_offset(torch_cuda, ffa, oracle_mod):
    """Float series with a large mean (128, sd 16): centring keeps float32 S/N
    within tolerance."""
    from paper_1703_05581_amd import synth

    x = synth.random_series(17, 1 << 18, "f32", mean=128.0, sd=16.0)
    run_case(torch_cuda, ffa, oracle_mod, x, 1 << 18, 1e-3, 0.256, 2.048, 256, W10, "f32",
             steps_max=16, check_fold=2)


# ----------------------------------------------------------------- workloads

def test_workload1_full(torch_cuda, ffa, oracle_mod):
    """65536 f32 samples, P0 = 500..999: every trial against the oracle."""
    from paper_1703_05581_amd import synth

    s = synth.workload1()
    pa = s.plan
    _, summ = run_case(torch_cuda, ffa, oracle_mod, s.data, pa.N, pa.tsamp, pa.pmin, pa.pmax,
                       pa.bins_min, list(pa.widths), "f32", check_fold=3)
    # the injected 733.3-sample pulsar is the best trial
    op = oracle_mod.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
    best_p = op.periods()[summ["best_trial"]] / pa.tsamp
    assert abs(best_p - 733.3) < 0.1 and summ["best_snr"] > 10


def test_workload2_sampled(torch_cuda, ffa, oracle_mod):
    """2^20 uint8 samples, three octaves: sampled steps bit-exact."""
    from paper_1703_05581_amd import synth

    s = synth.workload2()
    pa = s.plan
    plan, _ = run_case(torch_cuda, ffa, oracle_mod, s.data, pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min,
                       list(pa.widths), "u8", steps_max=24, check_fold=3)
    _assert_recovered(torch_cuda, plan, s, 10.0)


def test_workload3_sampled(torch_cuda, ffa, oracle_mod):
    """2^23 float32 samples with red noise, 0.5-30 s, dereddened with the
    paper's default window: sampled steps, including the three-pass ones."""
    from paper_1703_05581_amd import synth

    s = synth.workload3()
    pa = s.plan
    plan, _ = run_case(torch_cuda, ffa, oracle_mod, s.data, pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min,
                       list(pa.widths), "f32", steps_max=10, check_fold=2, dered_window=pa.dered_window,
                       dered_stride=pa.dered_stride)
    _assert_recovered(torch_cuda, plan, s, 6.6)


def _assert_recovered(torch, plan, series, floor):
    """Every injected pulsar peaks at its own period at or above ``floor``
    (6.6 is Algorithm 1's 5-sigma white-noise level of Sec. 4.1.2) and at
    or above 60% of its injected S/N (what the discrete widths, the trial
    grid and the dereddening may cost)."""
    snr, _ = plan.search(torch.from_numpy(series.data).cuda())
    snr = snr.cpu().numpy()
    periods = plan.periods()
    for p in series.pulsars:
        peak = pulsar_snr(periods, snr, p.period_s)
        print(f"pulsar P={p.period_s:.4f} s duty={p.duty:.3f} injected S/N {p.snr:.1f}: found {peak:.2f}",
              flush=True)
        assert peak >= max(floor, 0.6 * p.snr), (p, peak)


def test_deterministic(torch_cuda, ffa):
    from paper_1703_05581_amd import synth

    s = synth.workload1()
    plan = ffa.Plan.from_args(s.plan)
    x = torch_cuda.from_numpy(s.data).cuda()
    a = [t.clone() for t in plan.search(x)]
    b = plan.search(x)
    assert torch_cuda.equal(a[0], b[0]) and torch_cuda.equal(a[1], b[1])


def _first_max(v):
    """Index of the largest non-NaN value, first on ties (-0 == +0); 0 if all NaN."""
    ok = ~np.isnan(v)
    if not ok.any():
        return 0
    m = v[ok].max()
    return int(np.nonzero(ok & (v == m))[0][0])


def test_best(torch_cuda, ffa):
    g = np.random.default_rng(3)
    for n in (1, 5, 1000, 300001, 1835008):
        v = g.standard_normal(n).astype(np.float32)
        v[g.integers(0, n, size=3)] = 9.0  # ties: first wins
        t = torch_cuda.from_numpy(v).cuda()
        assert ffa.best(t) == int(np.argmax(v)) == _first_max(v)
    cases = [
        np.array([np.nan, 1.0, np.nan, 1.0], np.float32),
        np.array([np.nan, np.nan], np.float32),
        np.array([-0.0, 0.0, -0.0], np.float32),
        np.array([0.0, -0.0], np.float32),
        np.array([-np.inf, np.nan, -np.inf], np.float32),
        np.array([-3.0, -1.0, -2.0, -1.0], np.float32),
        np.array([np.nan] * 70000 + [5.0, np.inf, 7.0, np.inf], np.float32),
    ]
    for v in cases:
        assert ffa.best(torch_cuda.from_numpy(v).cuda()) == _first_max(v), v[:8]


@pytest.mark.parametrize("knob", [("select_iters", -1), ("select_cand", 1), ("select_cand", 8)])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_selection_paths(torch_cuda, ffa, oracle_mod, knob, dtype):
    """The median/MAD selection's other exits: the full-sort fallback (no
    counting rounds), bisection down to one candidate, and a small in-lane
    select; each must give the same periodogram."""
    from paper_1703_05581_amd import synth

    opts = dict([knob])
    N = 30000
    x = synth.random_series(5 + N, N, dtype)
    run_case(torch_cuda, ffa, oracle_mod, x, N, 1e-3, 0.2, 0.52, 200, W10, dtype, steps_max=12, opts=opts)
    xs = (x // 16 * 16) if dtype == "u8" else np.round(x * 4) / 4  # many ties
    run_case(torch_cuda, ffa, oracle_mod, xs.astype(x.dtype), N, 1e-3, 0.2, 0.52, 200, W10, dtype,
             steps_max=6, opts=opts)


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_selection_open_ends(torch_cuda, ffa, oracle_mod, sign, dtype):
    """Sparse large spikes at random positions make every profile's bins
    skewed (most bins hold none, a few hold one or more), which puts the
    profiles' mean, about which the selections' first pivots are placed, far
    from their median (above it for positive spikes, below for negative
    ones). The pivots then miss and the open end of the bracket is closed from
    the keys' extremes; the periodogram still equals the oracle's."""
    g = np.random.default_rng(71 + sign)
    N = 40000
    pos = g.choice(N, N // 400, replace=False)
    if dtype == "u8":
        x = np.clip(np.rint(g.standard_normal(N) * 2.0 + 128), 0, 255)
        x[pos] = 255 if sign > 0 else 0
        x = x.astype(np.uint8)
    else:
        x = g.standard_normal(N) * 10.0
        x[pos] += sign * 1000.0
        x = x.astype(np.float32)
    op = oracle_mod.plan(N, 1e-3, 0.2, 0.9, 200)
    far = tot = 0
    for s in range(0, op.n_steps, max(1, op.n_steps // 6)):
        prof = oracle_mod.fold_step(x, int(op.f[s]), int(op.P0[s]), int(op.m[s]), int(op.M[s]))
        for F in prof[:: max(1, len(prof) // 4)]:
            med = np.median(F)
            mad = np.median(np.abs(F - med))
            tot += 1
            far += abs(F.mean() - med) > 3.0 * 1.4826 * mad / np.sqrt(F.size)
    assert far >= 0.8 * tot, (far, tot)  # the input does what the test is about
    run_case(torch_cuda, ffa, oracle_mod, x, N, 1e-3, 0.2, 0.9, 200, W10, dtype, steps_max=12)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_window_sizes_agree(torch_cuda, ffa, oracle_mod, dtype):
    """The periodogram does not depend on how the queue is cut into launches
    or where the ring places each step: one step per window group, three, a
    4 MB ring with small groups (the arena wraps many times) and the default
    agree bit for bit."""
    from paper_1703_05581_amd import synth

    N = 300000
    x = torch_cuda.from_numpy(synth.random_series(77, N, dtype)).cuda()
    outs = []
    for opts in ({"steps_per_window": 1}, {"steps_per_window": 3}, {"ring_mb": 4, "window_tiles": 500}, {}):
        plan = ffa.Plan(N, 1e-3, 0.2, 2.0, 100, W10, dtype, opts=opts)
        print("queue", opts, flush=True)
        outs.append([t.clone() for t in plan.search(x)])
        torch_cuda.cuda.synchronize()
    for o in outs[1:]:
        assert torch_cuda.equal(o[0], outs[0][0]) and torch_cuda.equal(o[1], outs[0][1])


# ------------------------------------------------------------- Algorithm 2

@pytest.mark.parametrize("case", SMALL, ids=[f"N{c[0]}_B{c[4]}" for c in SMALL])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_alg2_small(torch_cuda, ffa, oracle_mod, case, dtype):
    """Algorithm 2 (off-pulse window) on the small cases: every register class,
    one to two passes, widths above P0."""
    from paper_1703_05581_amd import synth

    N, tsamp, pmin, pmax, B, widths = case
    x = synth.random_series(11 + N, N, dtype)
    if dtype == "f32":
        # A box of nearly the whole profile leaves two or three bins to
        # estimate sigma from (P0 = 34, w = 32 scores about 1600); float32
        # profile rounding is then amplified about A^2-fold, past the 1e-4
        # tolerance.  The paper's width rule stays below 0.4*P0.  uint8
        # profiles, scored from exact integers, cover those widths bit for bit.
        widths = [w for w in widths if 2 * w <= B]
    run_case(torch_cuda, ffa, oracle_mod, x, N, tsamp, pmin, pmax, B, widths, dtype,
             steps_max=30, alg=2)


def test_alg2_workload1_full_and_ref(torch_cuda, ffa, oracle_mod):
    """Workload 1 with Algorithm 2 on every trial; then the fixed-width "Ref"
    variant (one width matched to the pulse); both find the pulsar."""
    from paper_1703_05581_amd import synth

    s = synth.workload1()
    pa = s.plan
    op = oracle_mod.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
    for widths in (list(pa.widths), [24]):
        _, summ = run_case(torch_cuda, ffa, oracle_mod, s.data, pa.N, pa.tsamp, pa.pmin, pa.pmax,
                           pa.bins_min, widths, "f32", alg=2)
        best_p = op.periods()[summ["best_trial"]] / pa.tsamp
        assert abs(best_p - 733.3) < 0.1 and summ["best_snr"] > 8, (widths, best_p, summ)


def test_alg2_workload2_sampled(torch_cuda, ffa, oracle_mod):
    from paper_1703_05581_amd import synth

    s = synth.workload2()
    pa = s.plan
    run_case(torch_cuda, ffa, oracle_mod, s.data, pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min,
             list(pa.widths), "u8", steps_max=16, alg=2)


def test_u16_first_passes_agree(torch_cuda, ffa):
    """uint8 steps whose first pass keeps 16-bit sums give the same
    periodogram, bit for bit, as with 32-bit rows everywhere."""
    from tile_emu import phases

    from paper_1703_05581_amd import synth

    s = synth.workload2(0)
    x = torch_cuda.from_numpy(s.data).cuda()
    outs = []
    for flag in ("1", "0"):
        plan = ffa.Plan.from_args(s.plan, opts={"no_u16": 0 if flag == "1" else 1})
        n16 = int(phases(plan)["u16"].sum())
        assert (n16 > 0) == (flag == "1"), n16
        print("u16", flag, "phases", n16, flush=True)
        outs.append([t.clone() for t in plan.search(x)])
        torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(outs[0][0], outs[1][0]) and torch_cuda.equal(outs[0][1], outs[1][1])


def test_fold_u16_first_pass_steps(torch_cuda, ffa, oracle_mod):
    """ffa_fold of uint8 steps whose first pass keeps 16-bit rows: the fold
    sizes each pass's LDS at the element size the planner used, so these
    steps fold, bit-exact against the oracle."""
    from tile_emu import phases

    from paper_1703_05581_amd import synth

    s = synth.workload2(0)
    pa = s.plan
    plan = ffa.Plan.from_args(pa)
    ph = phases(plan)
    u16_steps = sorted(set(int(v) for v in ph["step"][ph["u16"] == 1]))
    assert len(u16_steps) > 100, len(u16_steps)
    op = oracle_mod.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
    x = torch_cuda.from_numpy(s.data).cuda()
    ws = plan.workspace()
    picks = u16_steps[:: max(1, len(u16_steps) // 6)][:6] + [u16_steps[-1]]
    for st in picks:
        print("fold u16 step", st, plan.step(st), plan.passes(st), flush=True)
        prof = plan.fold(x, st, ws=ws).cpu().numpy()
        ref = oracle_mod.fold_step(s.data, int(op.f[st]), int(op.P0[st]), int(op.m[st]), int(op.M[st]))
        check_profiles(prof, ref, True)
