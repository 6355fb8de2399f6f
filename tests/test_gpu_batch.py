"""Batched search (one persistent launch over many series) against the
single-series search and the oracle."""
import numpy as np
import pytest

from parity import check_periodogram, step_trials

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1703_05581_amd import ffa, synth

    assert torch.cuda.is_available()
    return torch, ffa, synth


W10 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_batch_equals_single(env, oracle_mod, dtype):
    torch, ffa, synth = env
    g = np.random.default_rng(42)
    cases = []
    for i in range(7):
        N = int(g.choice([20000, 65536, 150000, 300000]))
        B = int(g.choice([64, 100, 256, 500]))
        tsamp = 1e-3
        pmin = B * tsamp * float(g.uniform(1.0, 1.5))
        pmax = pmin * float(g.uniform(2.0, 12.0))
        widths = None if i % 3 == 0 else W10
        cases.append((N, tsamp, pmin, pmax, B, widths))
    plans, xs, xnp = [], [], []
    for i, (N, ts, pmin, pmax, B, w) in enumerate(cases):
        print("series", i, N, ts, pmin, pmax, B, w, dtype, flush=True)
        plans.append(ffa.Plan(N, ts, pmin, pmax, B, w, dtype))
        x = synth.random_series(300 + i, N, dtype)
        xnp.append(x)
        xs.append(torch.from_numpy(x).cuda())
    outs = ffa.search_batch(plans, xs)
    torch.cuda.synchronize()
    for i, (p, x) in enumerate(zip(plans, xs)):
        s1, w1 = p.search(x)
        torch.cuda.synchronize()
        assert torch.equal(outs[i][0], s1) and torch.equal(outs[i][1], w1), f"series {i}"
    # and a few steps of two series against the oracle
    for i in (0, 3):
        N, ts, pmin, pmax, B, w = cases[i]
        op = oracle_mod.plan(N, ts, pmin, pmax, B)
        steps = sorted(set(np.linspace(0, op.n_steps - 1, 6).round().astype(int).tolist()))
        so, wo = oracle_mod.search(xnp[i], op, w, steps=steps)
        check_periodogram(oracle_mod, xnp[i], op, w, outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy(),
                          so, wo, step_trials(op, steps), exact=dtype == "u8")


def test_batch_workload4_subset(env, oracle_mod):
    """Eight series of the batched workload (lengths 2^18..2^22, own period
    ranges, red noise, dereddened by their plans): batch equals single,
    sampled steps equal the oracle."""
    torch, ffa, synth = env
    series = [synth.workload4(i) for i in range(8)]
    plans = [ffa.Plan.from_args(s.plan) for s in series]
    xs = [torch.from_numpy(s.data).cuda() for s in series]
    outs = ffa.search_batch(plans, xs)
    torch.cuda.synchronize()
    for i in range(8):
        s1, w1 = plans[i].search(xs[i])
        torch.cuda.synchronize()
        assert torch.equal(outs[i][0], s1) and torch.equal(outs[i][1], w1), f"series {i}"
    s = series[1]
    pa = s.plan
    op = oracle_mod.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
    steps = sorted(set(np.linspace(0, op.n_steps - 1, 5).round().astype(int).tolist()))
    W = oracle_mod.dered_default_window(pa.tsamp, pa.pmin, pa.pmax)
    so, wo = oracle_mod.search(s.data, op, list(pa.widths), steps=steps, dered_window=W)
    check_periodogram(oracle_mod, s.data, op, list(pa.widths), outs[1][0].cpu().numpy(),
                      outs[1][1].cpu().numpy(), so, wo, step_trials(op, steps), exact=False,
                      dered_window=W)


def test_batch_mixed_types_and_prepared(env):
    """A batch may mix uint8 and float32 plans; search equals prepare +
    search_prepared."""
    torch, ffa, synth = env
    plans, xs = [], []
    for i, dt in enumerate(["u8", "f32", "u8", "f32", "f32"]):
        N = 40000 + 7000 * i
        plans.append(ffa.Plan(N, 1e-3, 0.2, 0.9, 200, W10, dt))
        xs.append(torch.from_numpy(synth.random_series(50 + i, N, dt)).cuda())
    outs = ffa.search_batch(plans, xs)
    torch.cuda.synchronize()
    for i, (p, x) in enumerate(zip(plans, xs)):
        ws = p.workspace()
        s1 = torch.empty(p.n_trials, dtype=torch.float32, device="cuda")
        w1 = torch.empty(p.n_trials, dtype=torch.int32, device="cuda")
        p.prepare(x, ws)
        p.search_prepared(s1, w1, ws)
        torch.cuda.synchronize()
        assert torch.equal(outs[i][0], s1) and torch.equal(outs[i][1], w1), f"series {i}"
