"""The host-side sigma mapping of the C ABI (Sec. 4.1.2) against the
oracle's, on CPU-made histograms (no GPU call)."""
import ctypes

import numpy as np
import pytest

from paper_1703_05581_amd import ffa


def _hists():
    g = np.random.default_rng(41)
    yield np.bincount(np.clip((g.standard_normal(200000) * 40 + 300).astype(np.int64), 0, 1023),
                      minlength=1024).astype(np.uint64)
    h = np.zeros(100, np.uint64)
    h[0], h[50], h[90] = 10**8 - 29, 1, 28
    yield h
    yield np.array([0, 1, 1, 1, 1, 0, 0, 0, 0, 0], np.uint64)
    yield (g.integers(0, 1000, 16384) ** 2).astype(np.uint64)


@pytest.mark.parametrize("case", range(4))
def test_sigma_gauss_matches_oracle(oracle_mod, case):
    h = list(_hists())[case]
    got = ffa.sigma_gauss(h)
    want = oracle_mod.sigma_gauss(h)
    fin = np.isfinite(want)
    assert np.array_equal(np.isinf(got), np.isinf(want)) and np.array_equal(np.sign(got[~fin]),
                                                                           np.sign(want[~fin]))
    assert np.max(np.abs(got[fin] - want[fin])) < 1e-9


@pytest.mark.parametrize("case", range(4))
@pytest.mark.parametrize("sigma", [-2.0, 0.0, 1.5, 3.0, 5.0])
def test_sigma_threshold_matches_oracle(oracle_mod, case, sigma):
    h = list(_hists())[case]
    lo, bpu = -3.0, 32.0
    try:
        want = oracle_mod.sigma_threshold(h, lo, bpu, sigma)
    except ValueError:
        with pytest.raises(ffa.FFAError):
            ffa.sigma_threshold(h, lo, bpu, sigma)
        return
    assert ffa.sigma_threshold(h, lo, bpu, sigma) == want


def test_stats_argument_errors():
    lib = ffa.lib()
    h = np.zeros(8, np.uint64)
    out = (ctypes.c_double * 8)()
    hp = h.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    assert lib.ffa_sigma_gauss(hp, 8, out) == ffa.FFA_ERR_INVALID  # empty
    assert lib.ffa_sigma_gauss(None, 8, out) == ffa.FFA_ERR_INVALID
    assert lib.ffa_sigma_gauss(hp, 0, out) == ffa.FFA_ERR_INVALID
    d = ctypes.c_double()
    assert lib.ffa_sigma_threshold(hp, 8, 0.0, 1.0, 5.0, ctypes.byref(d)) == ffa.FFA_ERR_INVALID
    h[0] = 5
    assert lib.ffa_sigma_threshold(hp, 8, 0.0, 1.0, float("nan"), ctypes.byref(d)) == ffa.FFA_ERR_INVALID
    # everything in bin 0: edge 1 already satisfies any sigma
    assert lib.ffa_sigma_threshold(hp, 8, 0.0, 1.0, 5.0, ctypes.byref(d)) == ffa.FFA_OK and d.value == 1.0
    # the histogram kernel's arguments are checked before any device call
    fake = 4096
    assert lib.ffa_snr_histogram(fake, 10, 0.0, 1.0, 0, fake, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_snr_histogram(fake, 10, 0.0, 1.0, 16385, fake, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_snr_histogram(fake, 10, 0.0, 0.0, 8, fake, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_snr_histogram(fake, 10, float("inf"), 1.0, 8, fake, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_snr_histogram(fake, -1, 0.0, 1.0, 8, fake, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_snr_histogram(None, 10, 0.0, 1.0, 8, fake, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_snr_histogram(fake, 10, 0.0, 1.0, 8, None, None) == ffa.FFA_ERR_INVALID
