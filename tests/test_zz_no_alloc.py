"""The allocation-free search (ffa_search_noalloc), through the C ABI, against
ffa_search on the same plan and series: two calls in a row, the second with
a smaller input, each bit-exact (uint8) or identical (float32, same kernels
and order); and its refusals (no device tables yet, a workspace above the
scratch)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

W10 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1703_05581_amd import ffa, synth

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, ffa, synth


def _pair(torch, ffa, plan, x):
    print("noalloc plan", plan.N, plan.dtype, plan.n_trials, plan.ws_bytes, flush=True)
    s0, w0 = plan.search(x)
    s1 = torch.full((plan.n_trials,), -7.0, dtype=torch.float32, device="cuda")
    w1 = torch.full((plan.n_trials,), -7, dtype=torch.int32, device="cuda")
    plan.search_noalloc(x, s1, w1)
    torch.cuda.synchronize()
    assert torch.equal(s0, s1) and torch.equal(w0, w1)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_noalloc_equals_search_twice(env, dtype):
    torch, ffa, synth = env
    big = ffa.Plan(1 << 18, 1e-3, 0.2, 1.6, 200, W10, dtype, opts={"ring_mb": 16})
    small = ffa.Plan(60000, 1e-3, 0.15, 0.9, 150, None, dtype, opts={"ring_mb": 16})
    for p in (big, small):
        assert p.ws_bytes <= 64 << 20, p.ws_bytes
        p.upload()
    for p, seed in ((big, 1), (small, 2)):  # the second call on a smaller input
        x = torch.from_numpy(synth.random_series(seed, p.N, dtype)).cuda()
        _pair(torch, ffa, p, x)


def test_noalloc_dereddened_and_alg2(env):
    torch, ffa, synth = env
    p = ffa.Plan(100000, 1e-3, 0.3, 1.5, 150, W10, "f32", snr=2, dered_window=-1, opts={"ring_mb": 16})
    p.upload()
    x = torch.from_numpy(synth.random_series(9, p.N, "f32", mean=3.0)).cuda()
    _pair(torch, ffa, p, x)


def test_noalloc_refusals(env):
    torch, ffa, synth = env
    lib = ffa.lib()
    p = ffa.Plan(50000, 1e-3, 0.2, 0.9, 200, W10, "u8", opts={"ring_mb": 8})
    x = torch.zeros(p.N, dtype=torch.uint8, device="cuda")
    s = torch.empty(p.n_trials, dtype=torch.float32, device="cuda")
    w = torch.empty(p.n_trials, dtype=torch.int32, device="cuda")
    # no device tables on this GPU yet: refused before anything is enqueued
    assert lib.ffa_search_noalloc(p.handle, x.data_ptr(), s.data_ptr(), w.data_ptr(), None) == ffa.FFA_ERR_INVALID
    assert b"ffa_plan_upload" in lib.ffa_last_error()
    assert lib.ffa_search_noalloc(p.handle, None, s.data_ptr(), w.data_ptr(), None) == ffa.FFA_ERR_INVALID
    # a plan whose workspace exceeds the 64 MiB scratch
    huge = ffa.Plan(1 << 22, 1e-3, 0.3, 3.0, 256, W10, "f32")
    assert huge.ws_bytes > 64 << 20
    huge.upload()
    xs = torch.zeros(huge.N, dtype=torch.float32, device="cuda")
    sh = torch.empty(huge.n_trials, dtype=torch.float32, device="cuda")
    wh = torch.empty(huge.n_trials, dtype=torch.int32, device="cuda")
    assert lib.ffa_search_noalloc(huge.handle, xs.data_ptr(), sh.data_ptr(), wh.data_ptr(),
                                  None) == ffa.FFA_ERR_UNSUPPORTED
    assert b"64 MiB" in lib.ffa_last_error()
    torch.cuda.synchronize()
