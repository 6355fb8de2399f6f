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


# (window, stride): the paper's default (the exact running median), the same
# with stride 1, an odd and an even window, windows shorter than the kernel's
# block of outputs, one too long to stage in LDS, one longer than the series,
# and the knot approximation with short and long strides
WINDOWS = [(-1, 0), (301, 1), (200, 0), (37, 0), (2, 0), (20000, 0), (500000, 0), (37, 5), (1001, 125)]


@pytest.mark.parametrize("win", WINDOWS, ids=[f"W{w}_s{s}" for w, s in WINDOWS])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_dered_search_and_fold(torch_cuda, ffa, oracle_mod, win, dtype):
    N = 100000
    # A window as long as the swing's period (or longer than the series)
    # cannot follow the swing, so most of it would stay in the float32 fold,
    # whose rounding then exceeds the 1e-4 S/N tolerance; those windows are
    # checked on a series without a swing.
    x = _drift_series(5 + win[0] % 97, N, dtype, amp=0.0 if win[0] >= 20000 else 1.0)
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


def test_dered_many_ties(torch_cuda, ffa, oracle_mod):
    """uint8 input with only a few distinct values: the running median's
    candidate pool overflows and every output is selected on its own, still
    equal to the oracle."""
    g = np.random.default_rng(31)
    N = 60000
    x = (127 + g.integers(0, 3, N)).astype(np.uint8)
    x[20000:21000] = 200  # a block of one value
    run_case(torch_cuda, ffa, oracle_mod, x, N, 1e-3, 0.3, 1.2, 150, W10, "u8", steps_max=12,
             check_fold=2, dered_window=1500, dered_stride=0)


@pytest.mark.parametrize("window", [301, 1500])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_dered_constant_stretch(torch_cuda, ffa, oracle_mod, window, dtype):
    """A stretch of one repeated value longer than the window plus a block of
    outputs: the blocks inside it have a core of a single value (one bucket
    holds every core value; the pool is that value), the blocks at its edges
    a core of mixed values; the dereddened series still folds to the
    oracle's profiles and the periodogram matches it."""
    g = np.random.default_rng(47 + window)
    N = 60000
    x = g.standard_normal(N) * 10.0
    x[20000:32000] = 0.0
    if dtype == "u8":
        x = np.clip(np.rint(x + 128), 0, 255).astype(np.uint8)
    else:
        x = (x + 5.0).astype(np.float32)
    run_case(torch_cuda, ffa, oracle_mod, x, N, 1e-3, 0.3, 1.2, 150, W10, dtype, steps_max=12,
             check_fold=3, dered_window=window, dered_stride=0)
