"""Seeded synthetic periodograms for the sifting tests (shared by both sides:
random numbers and placement only, none of the sifting arithmetic)."""
import numpy as np

# N, tsamp, pmin, pmax, bins_min of the sifting plan (uint8, three octaves)
SIFT_PLAN = (1 << 18, 1e-3, 0.256, 2.048, 256)

_W10 = np.array([1, 2, 3, 4, 6, 8, 12, 16, 24, 32], np.int32)


def synthetic_periodogram(plan, seed: int, quantised: bool = False):
    """(snr float32, width int32) over ``plan``'s trials: smoothed noise around
    S/N 4 with a few NaNs, plus families of bumps at a base period and its
    ratios n/x (so grouping and harmonic matching both have work).  With
    ``quantised`` the S/N takes steps of 1/4, which makes ties common."""
    g = np.random.default_rng(seed)
    n = plan.n_trials
    z = g.standard_normal(n + 4)
    smooth = (z[:-4] + z[1:-3] + z[2:-2] + z[3:-1] + z[4:]) / np.sqrt(5.0)
    snr = 4.0 + 1.3 * smooth
    periods = plan.periods()
    lo, hi = periods.min(), periods.max()
    for _ in range(6):
        base = float(np.exp(g.uniform(np.log(lo), np.log(hi))))
        height = g.uniform(8.0, 30.0)
        for ratio in (1.0, 0.5, 2.0, 1 / 3, 2 / 3, 1.5, 3.0, 0.4, 2.5, 5 / 7):
            p = base * ratio
            if not lo <= p <= hi:
                continue
            i = int(np.argmin(np.abs(periods - p)))
            h = height * (1.0 if ratio == 1.0 else g.uniform(0.4, 0.9))
            for d in range(-4, 5):
                if 0 <= i + d < n:
                    snr[i + d] += h * (1.0 - abs(d) / 5.0)
    snr[g.integers(0, n, 20)] = np.nan
    if quantised:
        snr = np.round(snr * 4.0) / 4.0
    width = g.choice(_W10, n).astype(np.int32)
    return snr.astype(np.float32), width
