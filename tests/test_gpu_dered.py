"""Dynamic running-median dereddening (paper Sec. 2.3.1) on the GPU against
the oracle, through the C ABI."""
import numpy as np
import pytest

from test_gpu_parity import W10, run_case

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


def _drift_series(seed, N, dtype, amp=1.0):
    """Noise on a slow baseline swing of ``amp`` * 30 sigma (red-noise stand-in)."""
    g = np.random.default_rng(seed)
    t = np.arange(N)
    x = g.standard_normal(N) * 10.0 + amp * (300.0 * np.sin(2 * np.pi * t / 37000.0) + 100.0 * (t / N) ** 2)
    if dtype == "u8":
        return np.clip(np.rint(x * 0.3 + 128), 0, 255).astype(np.uint8)
    return x.astype(np.float32)


# (window, stride): the paper's default, the plain per-sample running median,
# an odd window with a short stride, an even window, one longer than the series
WINDOWS = [(-1, 0), (301, 1), (37, 5), (200, 0), (500000, 0)]


@pytest.mark.parametrize("win", WINDOWS, ids=[f"W{w}_s{s}" for w, s in WINDOWS])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_dered_search_and_fold(torch_cuda, ffa, oracle_mod, win, dtype):
    N = 100000
    # A window longer than the series removes only a constant (the median of
    # the whole series), so a swing would stay in the float32 fold, whose
    # rounding then exceeds the 1e-4 S/N tolerance; that case checks the
    # clipped window on a series without a swing.
    x = _drift_series(5 + win[0] % 97, N, dtype, amp=0.0 if win[0] > N else 1.0)
    run_case(torch_cuda, ffa, oracle_mod, x, N, 1e-3, 0.3, 1.5, 150, W10, dtype, steps_max=24,
             check_fold=3, dered_window=win[0], dered_stride=win[1])


def test_dered_alg2(torch_cuda, ffa, oracle_mod):
    N = 80000
    x = _drift_series(8, N, "f32")
    run_case(torch_cuda, ffa, oracle_mod, x, N, 1e-3, 0.2, 1.0, 100, W10, "f32", steps_max=20,
             alg=2, dered_window=-1)


def test_dered_recovers_pulsar(torch_cuda, ffa, oracle_mod):
    """A weak pulsar on a strong slow swing is the best trial once the series is
    dereddened (default window), as in the oracle."""
    g = np.random.default_rng(26)
    N, ts, pmin, pmax, B = 1 << 16, 1e-3, 0.5, 1.0, 500
    t = np.arange(N)
    x = g.standard_normal(N) + 40.0 * np.sin(2 * np.pi * t / 20000.0)
    P = 733.3
    x = (x + 1.2 * np.exp(-0.5 * (((t % P) - 100.0) / 7.0) ** 2)).astype(np.float32)
    _, summ = run_case(torch_cuda, ffa, oracle_mod, x, N, ts, pmin, pmax, B, [1, 2, 4, 8, 16, 32],
                       "f32", dered_window=-1)
    op = oracle_mod.plan(N, ts, pmin, pmax, B)
    assert abs(op.periods()[summ["best_trial"]] / ts - P) < 0.5
