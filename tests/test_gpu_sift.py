"""Candidate sifting (after ffa2best, paper Sec. 2.3.3) on the GPU against the
oracle, through the C ABI: synthetic periodograms fed to both sides, and the
periodogram of a real search, which is bit-exact for uint8 input, so each side
sifts its own."""
import numpy as np
import pytest

from sift_inputs import SIFT_PLAN, synthetic_periodogram

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


@pytest.fixture(scope="module")
def plans(ffa, oracle_mod):
    N, tsamp, pmin, pmax, B = SIFT_PLAN
    return ffa.Plan(N, tsamp, pmin, pmax, B, dtype="u8"), oracle_mod.plan(N, tsamp, pmin, pmax, B)


def _same(got, want):
    assert got.size == want.size, (got.size, want.size)
    np.testing.assert_array_equal(got["trial"], want["trial"])
    np.testing.assert_array_equal(got["width"], want["width"])
    np.testing.assert_array_equal(got["snr"].view(np.uint32), want["snr"].view(np.uint32))
    np.testing.assert_array_equal(got["period"].view(np.uint64), want["period"].view(np.uint64))


# (min_snr, frac_fall, abs_fall, group_widths, harmonic_primes, harmonic_tol)
PARAMS = [
    (9.0, 0.1, 1.0, 0.0, 0, 1e-5),      # peaks only
    (9.0, 0.1, 1.0, 2.0, 0, 1e-5),      # + grouping
    (9.0, 0.1, 1.0, 2.0, 31, 1e-5),     # + harmonics, the paper's prime limit
    (8.0, 0.05, 0.5, 30.0, 31, 1e-3),   # wide groups, loose harmonics
    (10.0, 0.0, 0.0, 0.0, 7, 2e-4),     # a fall of zero closes a peak
    (6.5, 0.1, 0.5, 1.0, 31, 1e-5),     # several thousand peaks
]


@pytest.mark.parametrize("prm", PARAMS, ids=[f"p{i}" for i in range(len(PARAMS))])
@pytest.mark.parametrize("quantised", [False, True], ids=["cont", "ties"])
def test_sift_synthetic(torch_cuda, ffa, oracle_mod, plans, prm, quantised):
    torch = torch_cuda
    gp, op = plans
    snr, width = synthetic_periodogram(op, seed=11 + quantised, quantised=quantised)
    want = oracle_mod.sift(snr, width, op, *prm)
    # the GPU holds at most 16384 peaks before grouping
    assert 0 < want.size and oracle_mod.sift(snr, width, op, *prm[:3]).size <= 16384
    print(f"sift synthetic prm={prm} quantised={quantised} n={want.size}", flush=True)
    got = gp.sift(torch.from_numpy(snr).cuda(), torch.from_numpy(width).cuda(), *prm, max_cands=16384)
    _same(got, want)


def test_sift_truncated_empty_overflow(torch_cuda, ffa, oracle_mod, plans):
    torch = torch_cuda
    gp, op = plans
    snr, width = synthetic_periodogram(op, seed=5)
    ds, dw = torch.from_numpy(snr).cuda(), torch.from_numpy(width).cuda()
    want = oracle_mod.sift(snr, width, op, 9.0)
    assert want.size > 7
    # only the first max_cands are written; the count is the full one
    cands, n = gp.sift(ds, dw, 9.0, max_cands=7, raw=True)
    assert int(n.item()) == want.size
    got = gp.sift(ds, dw, 9.0, max_cands=7)
    _same(got, want[:7])
    # max_cands 0: only the count
    cands, n = gp.sift(ds, dw, 9.0, max_cands=0, raw=True)
    assert int(n.item()) == want.size
    # nothing above the threshold
    got = gp.sift(ds, dw, 1e9)
    assert got.size == 0 and oracle_mod.sift(snr, width, op, 1e9).size == 0
    # more peaks than the scratch holds: count -1 and an error from the binding
    assert oracle_mod.sift(snr, width, op, -50.0, 0.0, 0.0).size > 16384
    cands, n = gp.sift(ds, dw, -50.0, 0.0, 0.0, raw=True)
    assert int(n.item()) == -1
    with pytest.raises(RuntimeError):
        gp.sift(ds, dw, -50.0, 0.0, 0.0)
    # a workspace from another call is reused: the result does not change
    ws = gp.workspace()
    gp.search(torch.zeros(gp.N, dtype=torch.uint8, device="cuda"), ws=ws)
    _same(gp.sift(ds, dw, 9.0, 0.1, 1.0, 2.0, 31, ws=ws), oracle_mod.sift(snr, width, op, 9.0, 0.1, 1.0, 2.0, 31))


def test_sift_argument_errors(torch_cuda, ffa, plans):
    torch = torch_cuda
    gp, _ = plans
    ds = torch.zeros(gp.n_trials, dtype=torch.float32, device="cuda")
    dw = torch.ones(gp.n_trials, dtype=torch.int32, device="cuda")
    for bad in [dict(frac_fall=1.5), dict(frac_fall=-0.1), dict(abs_fall=-1.0), dict(group_widths=-1.0),
                dict(harmonic_tol=-1e-3), dict(min_snr=float("nan")), dict(max_cands=-1)]:
        with pytest.raises(ffa.FFAError):
            gp.sift(ds, dw, **bad)
    with pytest.raises(ffa.FFAError):
        gp.sift(ds, dw, ws=torch.empty(64, dtype=torch.uint8, device="cuda"))


def test_sift_search_output(torch_cuda, ffa, oracle_mod):
    """A uint8 search with three injected pulsars: the GPU periodogram equals
    the oracle's bit for bit, and so do the candidates each side sifts from its
    own periodogram."""
    from paper_1703_05581_amd import synth

    torch = torch_cuda
    g = synth.rng(77)
    N, tsamp, pmin, pmax, B = SIFT_PLAN
    x = 128.0 + 16.0 * g.standard_normal(N)
    psrs = [synth.Pulsar(0.3, 0.02, 25.0, float(g.random())),
            synth.Pulsar(0.77, 0.04, 20.0, float(g.random())),
            synth.Pulsar(1.6, 0.05, 20.0, float(g.random()))]
    for p in psrs:
        x += synth.pulse_train(N, tsamp, p, 16.0)
    x = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    widths = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]
    gp = ffa.Plan(N, tsamp, pmin, pmax, B, widths, dtype="u8")
    op = oracle_mod.plan(N, tsamp, pmin, pmax, B)
    snr, width = gp.search(torch.from_numpy(x).cuda())
    osnr, owidth = oracle_mod.search(x, op, widths)
    np.testing.assert_array_equal(snr.cpu().numpy().view(np.uint32), osnr.astype(np.float32).view(np.uint32))
    np.testing.assert_array_equal(width.cpu().numpy(), owidth)
    prm = (8.0, 0.1, 1.0, 2.0, 31, 1e-4)
    want = oracle_mod.sift(osnr.astype(np.float32), owidth.astype(np.int32), op, *prm)
    got = gp.sift(snr, width, *prm)
    _same(got, want)
    # each injected pulsar is among the five strongest candidates
    top = got["period"][:5]
    for p in psrs:
        assert np.min(np.abs(top - p.period_s) / p.period_s) < 2e-3, (p.period_s, top)


@pytest.mark.parametrize("seed", range(20))
def test_sift_random_parameters(torch_cuda, ffa, oracle_mod, plans, seed):
    """Random thresholds, group widths, prime limits and tolerances on random
    synthetic periodograms: identical candidate lists."""
    torch = torch_cuda
    gp, op = plans
    g = np.random.default_rng(500 + seed)
    snr, width = synthetic_periodogram(op, seed=900 + seed, quantised=bool(g.random() < 0.3))
    prm = (float(g.uniform(6.0, 12.0)), float(g.choice([0.0, 0.02, 0.1, 0.3])), float(g.choice([0.0, 0.25, 1.0, 2.0])),
           float(g.choice([0.0, 0.5, 2.0, 10.0])), int(g.choice([0, 2, 3, 7, 31, 97])),
           float(g.choice([1e-6, 1e-5, 1e-4, 1e-3])))
    want = oracle_mod.sift(snr, width, op, *prm)
    if oracle_mod.sift(snr, width, op, *prm[:3]).size > 16384:
        pytest.skip("more peaks than the GPU scratch holds")
    got = gp.sift(torch.from_numpy(snr).cuda(), torch.from_numpy(width).cuda(), *prm, max_cands=16384)
    _same(got, want)
