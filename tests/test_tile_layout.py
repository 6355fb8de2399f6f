"""Host-side check of the FFA kernel's addressing and launch order (no GPU)."""
import numpy as np
import pytest

from paper_1703_05581_amd import ffa, synth
from tile_emu import check


@pytest.mark.parametrize("wl", [1, 2])
def test_workload_plans(wl):
    check(ffa.Plan.from_args(synth.plan_args(wl)))


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_random_plans(dtype):
    g = np.random.default_rng(42)
    W10 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]
    for i in range(7):
        N = int(g.choice([20000, 65536, 150000, 300000]))
        B = int(g.choice([64, 100, 256, 500]))
        pmin = B * 1e-3 * float(g.uniform(1.0, 1.5))
        pmax = pmin * float(g.uniform(2.0, 12.0))
        check(ffa.Plan(N, 1e-3, pmin, pmax, B, None if i % 3 == 0 else W10, dtype))


def test_three_pass_and_small_windows():
    # one step per window group stresses the ring reuse and pass order checks
    p = ffa.Plan(600000, 1e-3, 1.990, 2.010, 1000, [1, 2, 4, 8], opts={"steps_per_window": 1})
    assert max(len(p.passes(s)) for s in range(p.n_steps)) >= 3
    L = check(p)
    assert L["lookahead"] == 1
    check(ffa.Plan(300000, 1e-3, 0.2, 2.0, 100, None, opts={"steps_per_window": 3}))


@pytest.mark.parametrize("lds_kb", [24, 48, 96, 160])
def test_lds_budgets(lds_kb):
    """Smaller tile LDS budgets give shallower tiles, more passes and a
    different halo room (so a different mix of radix-2 and radix-4 levels);
    every tile still fits and every dependency is met."""
    for args in [(150000, 1e-3, 0.1, 1.5, 97, None, "f32"), (300000, 1e-3, 0.3, 3.0, 300, None, "u8"),
                 (80000, 1e-3, 0.01, 0.2, 8, [1, 2, 4], "u8")]:
        p = ffa.Plan(*args, opts={"tile_lds_bytes": lds_kb * 1024})
        L = check(p)
        assert L["lds_bytes"] <= lds_kb * 1024


@pytest.mark.parametrize("ring_mb,tiles", [(1, 64), (4, 500), (16, 3000), (64, 100000)])
def test_ring_arena_budgets(ring_mb, tiles):
    """Small ring budgets and window targets cut the steps into many small
    groups whose ranges wrap around the arena again and again; no two steps
    whose launches overlap may share ring space, and the ring stays within
    the budget unless one step alone needs more."""
    for args in [(600000, 1e-3, 1.990, 2.010, 1000, [1, 2, 4, 8], "f32"),
                 (300000, 1e-3, 0.2, 2.0, 100, None, "u8"),
                 (400000, 1e-3, 0.05, 3.0, 64, None, "f32")]:
        p = ffa.Plan(*args, opts={"ring_mb": ring_mb, "window_tiles": tiles})
        L = check(p)
        largest = max((p.step(s).M * p.step(s).P0 * (2 if len(p.passes(s)) > 2 else 1)
                       for s in range(p.n_steps) if len(p.passes(s)) > 1), default=0)
        assert L["ring_elems"] * 4 <= max(ring_mb << 20, 3 * 4 * (largest + 64) * 2), (args, L["ring_elems"])


def test_plan_options_are_checked():
    """Out-of-range launch options are refused at plan creation."""
    for bad in ({"tile_lds_bytes": 1000}, {"tile_lds_bytes": 200000}, {"window_tiles": -1},
                {"ring_mb": -5}, {"steps_per_window": 5000}, {"no_u16": 2}, {"select_cand": 65}):
        with pytest.raises(ffa.FFAError) as e:
            ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, None, opts=bad)
        assert e.value.status == ffa.FFA_ERR_INVALID, bad
    with pytest.raises(ValueError):
        ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, None, opts={"no_such_option": 1})
