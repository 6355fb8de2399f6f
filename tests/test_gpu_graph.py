"""A search captured in a HIP graph (through torch's graph capture on the
stream the C ABI is given) and replayed: every replay, with eager work and
synchronisations in between, gives the eager periodogram bit for bit, and a
replay after new data is copied into the captured input buffer gives the
eager periodogram of that data."""
import numpy as np
import pytest

from test_gpu_parity import W10

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("dtype,alg,dered", [("u8", 1, 0), ("f32", 1, 0), ("f32", 2, 0), ("f32", 1, -1)])
def test_graph_replay_matches_eager(torch_cuda, dtype, alg, dered):
    torch = torch_cuda
    from paper_1703_05581_amd import ffa, synth

    N = 200000
    plan = ffa.Plan(N, 1e-3, 0.2, 2.0, 100, W10, dtype, snr=alg, dered_window=dered)
    x = torch.from_numpy(synth.random_series(91, N, dtype)).cuda()
    snr = torch.empty(plan.n_trials, dtype=torch.float32, device="cuda")
    wid = torch.empty(plan.n_trials, dtype=torch.int32, device="cuda")
    ws = plan.workspace()
    plan.search(x, snr, wid, ws)  # eager, and it makes the plan's device tables
    torch.cuda.synchronize()
    ref = (snr.clone(), wid.clone())
    print("capture", dtype, alg, dered, plan.n_trials, flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.search(x, snr, wid, ws)
    torch.cuda.synchronize()
    other_snr, other_wid = torch.empty_like(snr), torch.empty_like(wid)
    for i in range(3):
        snr.fill_(-1.0)
        wid.fill_(-1)
        plan.search(x, other_snr, other_wid, plan.workspace())  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(snr, ref[0]) and torch.equal(wid, ref[1]), f"replay {i}"
        assert torch.equal(other_snr, ref[0]) and torch.equal(other_wid, ref[1])
    # new data in the captured input buffer
    x.copy_(torch.from_numpy(synth.random_series(92, N, dtype)).cuda())
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    s2, w2 = plan.search(x, other_snr, other_wid, ws)
    torch.cuda.synchronize()
    assert torch.equal(snr, s2) and torch.equal(wid, w2)
    assert not torch.equal(snr, ref[0])


def test_graph_replay_batch(torch_cuda):
    """A batched search (uint8 and dereddened float32 series) captured and
    replayed equals the eager batch, replay after replay."""
    torch = torch_cuda
    from paper_1703_05581_amd import ffa, synth

    plans, xs = [], []
    for i, (dt, dw) in enumerate([("u8", 0), ("f32", -1), ("f32", 0), ("f32", -1)]):
        N = 60000 + 20000 * i
        plans.append(ffa.Plan(N, 1e-3, 0.15, 1.2, 120, W10, dt, dered_window=dw))
        xs.append(torch.from_numpy(synth.random_series(130 + i, N, dt)).cuda())
    b = ffa.Batch(plans)
    ws = b.workspace()
    outs = b.outputs()
    b.search(xs, outs=outs, ws=ws)  # eager, and it makes the batch's device tables
    torch.cuda.synchronize()
    ref = [(s.clone(), w.clone()) for s, w in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.search(xs, outs=outs, ws=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        for s, w in outs:
            s.fill_(-1.0)
            w.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, ((s, w), (s0, w0)) in enumerate(zip(outs, ref)):
            assert torch.equal(s, s0) and torch.equal(w, w0), (rep, i)
    b.close()
