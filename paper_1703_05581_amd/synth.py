"""Seeded synthetic inputs for the FFA search.

This module holds no part of the search itself (no folding, no S/N): it only
makes time series and plan arguments.  The GPU tests, the oracle tests and the
benchmark all draw their inputs from here, with numpy's PCG64 generator and
seed = 1000 * workload + series index.

Workloads (the surveys the paper uses are not available, so these stand in for
them; the shapes follow Sec. 2.4 and Sec. 4 of the paper):

  1 "plain"   : f32[65536], tsamp 1 ms, N(0,1) noise, P0 = 500..999 bins (0.5-1 s),
                one Gaussian pulse train, period 733.3 samples, 3% duty cycle,
                folded S/N about 15.
  2 "u8"      : u8[2^20], tsamp 1 ms, N(128, 16^2) rounded and clipped to 0..255,
                P0 in [256, 512) over octaves f = 1, 2, 4 (0.256-2.048 s), pulsars at
                0.4, 0.9, 1.7 s with duty 2%, 3.5%, 5%, folded S/N about 15 each.
  3 "htru"    : f32[2^23], tsamp 0.512 ms (~71.6 min), white N(0,1) plus power-law red
                noise (power spectral index -2, same rms as the white part), 0.5-30 s,
                P0 in [256, 512), 10 pulsars with log-uniform periods, duty 1-10%,
                S/N 10-30; the plan dereddens with the paper's default window.
  4 "batch"   : 256 f32 series, N from {2^18 .. 2^22}, tsamp 0.512 ms, Pmin U(0.2, 1) s,
                Pmax U(5, 30) s, noise as workload 3 (dereddened by the plan), 30% with
                one pulsar of S/N 15.
  5 "served"  : f32 series of N from {2^20 .. 2^23}, tsamp 1 ms, workload 2's plan and
                noise model (unclipped floats), workload 2's pulsars in 30% of requests.
  6 "null"    : 26 f32 series of white N(0,1) noise for the false-alarm statistics of
                Sec. 4.1.2: 2^21 samples of 2.048 ms (an HTRU-length observation of 64 us
                samples downsampled by 2^5), 1-20 s, base period 488 bins (1 s, the lowest
                trial period in samples), the paper's default widths; 1.03e8 trials over the 26.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

WIDTHS = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32)
FWHM_PER_SIGMA = 2.0 * np.sqrt(2.0 * np.log(2.0))  # Gaussian FWHM = this * std (Sec. 3.3.1)


@dataclass
class PlanArgs:
    """Arguments of a search plan (the fields of the C plan descriptor)."""

    N: int
    tsamp: float
    pmin: float
    pmax: float
    bins_min: int
    widths: tuple = WIDTHS
    dtype: str = "f32"  # "f32" or "u8"
    max_octaves: int = 0
    dered_window: int = 0  # 0: off, -1: the paper's default window, > 0: samples
    dered_stride: int = 0


@dataclass
class Pulsar:
    period_s: float
    duty: float  # FWHM / period
    snr: float   # target matched-filter S/N of the whole series
    phase: float = 0.0  # in [0, 1)


@dataclass
class Series:
    data: np.ndarray
    plan: PlanArgs
    pulsars: list = field(default_factory=list)
    seed: int = 0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def pulse_train(n: int, tsamp: float, p: Pulsar, sigma_noise: float) -> np.ndarray:
    """Gaussian pulse train whose ideal matched-filter S/N over the whole series
    is ``p.snr`` in white noise of standard deviation ``sigma_noise``.

    A pulse of peak a and standard deviation c (samples) folded over n_p turns
    has matched-filter S/N a*sqrt(n_p * c * sqrt(pi)) / sigma (sum of g^2 for a
    sampled unit Gaussian is c*sqrt(pi)); the peak is solved from that.
    """
    P = p.period_s / tsamp  # samples
    c = p.duty * P / FWHM_PER_SIGMA
    n_p = n / P
    amp = p.snr * sigma_noise / np.sqrt(n_p * c * np.sqrt(np.pi))
    t = np.arange(n, dtype=np.float64)
    ph = np.mod(t - p.phase * P, P)
    d = np.minimum(ph, P - ph)
    return amp * np.exp(-0.5 * (d / c) ** 2)


def red_noise(n: int, g: np.random.Generator, index: float = -2.0) -> np.ndarray:
    """Power-law noise: white noise shaped in the Fourier domain so its power
    spectrum goes as f**index (amplitude f**(index/2)), no DC, unit rms."""
    w = g.standard_normal(n)
    spec = np.fft.rfft(w)
    fr = np.fft.rfftfreq(n)
    shape = np.zeros_like(fr)
    shape[1:] = fr[1:] ** (index / 2.0)
    out = np.fft.irfft(spec * shape, n)
    return out / np.sqrt(np.mean(out ** 2))


# ------------------------------------------------------------- workloads

def plan_args(workload: int) -> PlanArgs:
    if workload == 1:
        return PlanArgs(N=65536, tsamp=1e-3, pmin=0.5, pmax=1.0, bins_min=500)
    if workload == 2:
        return PlanArgs(N=1 << 20, tsamp=1e-3, pmin=0.256, pmax=2.048, bins_min=256, dtype="u8")
    if workload == 3:
        return PlanArgs(N=1 << 23, tsamp=0.512e-3, pmin=0.5, pmax=30.0, bins_min=256, dered_window=-1)
    raise ValueError("workloads 4 and 5 have per-series plans")


def workload1(index: int = 0) -> Series:
    seed = 1000 * 1 + index
    g = rng(seed)
    pa = plan_args(1)
    x = g.standard_normal(pa.N)
    psr = Pulsar(period_s=733.3 * pa.tsamp, duty=0.03, snr=15.0, phase=float(g.random()))
    x = x + pulse_train(pa.N, pa.tsamp, psr, 1.0)
    return Series(x.astype(np.float32), pa, [psr], seed)


def _u8(x: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def workload2(index: int = 0) -> Series:
    seed = 1000 * 2 + index
    g = rng(seed)
    pa = plan_args(2)
    x = 128.0 + 16.0 * g.standard_normal(pa.N)
    psrs = [Pulsar(0.4, 0.02, 15.0, float(g.random())),
            Pulsar(0.9, 0.035, 15.0, float(g.random())),
            Pulsar(1.7, 0.05, 15.0, float(g.random()))]
    for p in psrs:
        x += pulse_train(pa.N, pa.tsamp, p, 16.0)
    return Series(_u8(x), pa, psrs, seed)


def _htru_noise(n: int, tsamp: float, g: np.random.Generator) -> np.ndarray:
    x = g.standard_normal(n) + red_noise(n, g, -2.0)
    return x


def workload3(index: int = 0, n: int | None = None) -> Series:
    seed = 1000 * 3 + index
    g = rng(seed)
    pa = plan_args(3)
    if n is not None:
        pa.N = n
    x = _htru_noise(pa.N, pa.tsamp, g)
    psrs = []
    for _ in range(10):
        P = float(np.exp(g.uniform(np.log(0.5), np.log(30.0))))
        psrs.append(Pulsar(P, float(g.uniform(0.01, 0.10)), float(g.uniform(10, 30)),
                           float(g.random())))
    for p in psrs:
        x += pulse_train(pa.N, pa.tsamp, p, 1.0)
    return Series(x.astype(np.float32), pa, psrs, seed)


def workload4(index: int, count: int = 256) -> Series:
    """Series ``index`` of the batched workload (each with its own plan)."""
    if not 0 <= index < count:
        raise IndexError(index)
    seed = 1000 * 4 + index
    g = rng(seed)
    N = int(1 << int(g.integers(18, 23)))
    tsamp = 0.512e-3
    pmin = float(g.uniform(0.2, 1.0))
    pmax = float(g.uniform(5.0, 30.0))
    pa = PlanArgs(N=N, tsamp=tsamp, pmin=pmin, pmax=pmax, bins_min=256, dered_window=-1)
    x = _htru_noise(N, tsamp, g)
    psrs = []
    if g.random() < 0.3:
        P = float(np.exp(g.uniform(np.log(pmin), np.log(pmax))))
        psrs.append(Pulsar(P, float(g.uniform(0.01, 0.10)), 15.0, float(g.random())))
        x += pulse_train(N, tsamp, psrs[0], 1.0)
    return Series(x.astype(np.float32), pa, psrs, seed)


def workload5(index: int, sizes=(20, 21, 22, 23)) -> Series:
    """Request ``index`` of the served stream."""
    seed = 1000 * 5 + index
    g = rng(seed)
    N = int(1 << int(g.choice(sizes)))
    pa = PlanArgs(N=N, tsamp=1e-3, pmin=0.256, pmax=2.048, bins_min=256)
    x = 128.0 + 16.0 * g.standard_normal(N)
    psrs = []
    if g.random() < 0.3:
        psrs = [Pulsar(0.4, 0.02, 15.0, float(g.random())),
                Pulsar(0.9, 0.035, 15.0, float(g.random())),
                Pulsar(1.7, 0.05, 15.0, float(g.random()))]
        for p in psrs:
            x += pulse_train(N, pa.tsamp, p, 16.0)
    return Series(x.astype(np.float32), pa, psrs, seed)


NULL_SERIES = 26


def plan_args_null() -> PlanArgs:
    return PlanArgs(N=1 << 21, tsamp=2.048e-3, pmin=1.0, pmax=20.0, bins_min=488, widths=())


def workload6(index: int) -> Series:
    """Series ``index`` (0..25) of the white-noise false-alarm set."""
    if not 0 <= index < NULL_SERIES:
        raise IndexError(index)
    seed = 1000 * 6 + index
    g = rng(seed)
    pa = plan_args_null()
    return Series(g.standard_normal(pa.N).astype(np.float32), pa, [], seed)


def workload(wl: int, index: int = 0) -> Series:
    return {1: workload1, 2: workload2, 3: workload3, 4: workload4, 5: workload5, 6: workload6}[wl](index)


# ------------------------------------------------------ small random cases

def random_series(seed: int, n: int, dtype: str, mean: float = 0.0, sd: float = 1.0) -> np.ndarray:
    """Plain noise for parity sweeps: f32 N(mean, sd) or u8 uniform 0..255."""
    g = rng(seed)
    if dtype == "u8":
        return g.integers(0, 256, size=n, dtype=np.uint8)
    return (mean + sd * g.standard_normal(n)).astype(np.float32)


def poisson_arrivals(seed: int, rate_hz: float, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process."""
    g = rng(seed)
    return np.cumsum(g.exponential(1.0 / rate_hz, size=count))
