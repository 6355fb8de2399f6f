"""Host-side check of the FFA kernel's addressing and launch order, and of
the dereddening plan (no GPU)."""
import ctypes

import numpy as np
import pytest

import tile_emu
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


def _dered_plan(plan):
    lib = ffa.lib()
    lib.ffa_debug_dered.restype = ctypes.c_int64
    lib.ffa_debug_dered.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    nl = ctypes.c_int64()
    ns = lib.ffa_debug_dered(plan.handle, None, 0, ctypes.byref(nl))
    buf = np.zeros(6 * ns + 3 * nl.value, np.int64)
    assert lib.ffa_debug_dered(plan.handle, buf.ctypes.data, buf.size, ctypes.byref(nl)) == ns
    return buf[:6 * ns].reshape(-1, 6), buf[6 * ns:].reshape(-1, 3)


@pytest.mark.parametrize("seed", range(6))
def test_dered_plan_covers_octaves(seed):
    """Float plans with the exact filter dereddening every folded octave at
    once: each octave from the lowest folded one is one segment (its double
    raw series in, its float series out, inside the workspace), blocks of
    256 outputs numbered without gaps across the launches, each launch's
    LDS within the CU's and at least what its segments stage."""
    g = np.random.default_rng(500 + seed)
    N = int(g.integers(3000, 1 << 21))
    B = int(g.integers(16, 300))
    pmin = B * 1e-3 * float(g.uniform(1.0, 3.0))
    plan = ffa.Plan(N, 1e-3, pmin, pmin * float(g.uniform(2.0, 40.0)), B, None, "f32",
                    dered_window=int(g.choice([-1, 37, 5000, 40000])))
    segs, launches = _dered_plan(plan)
    L = tile_emu.layout(plan)
    octs = tile_emu.octaves(plan)
    first = min(plan.step(s).f for s in range(plan.n_steps)).bit_length() - 1
    assert len(segs) == len(octs) - first
    blk = 0
    for k, (x_off, out_off, n, block0, window, use_stage) in enumerate(segs):
        assert (out_off, n) in [tuple(o) for o in octs[first:]]
        assert x_off + 2 * n <= L["ring_off"] and out_off + n <= x_off or x_off + 2 * n <= out_off
        assert block0 == blk and window > 0
        stage_n = min(window + 255, n)
        assert use_stage == (stage_n <= 16384)
        blk += -(-n // 256)
    assert launches[0][0] == 0 and sum(int(b) for _, b, _ in launches) == blk
    for (b0, nb, lds), nxt in zip(launches, list(launches[1:]) + [None]):
        assert 0 < lds <= 160 * 1024
        if nxt is not None:
            assert nxt[0] == b0 + nb
        inside = [s for s in segs if b0 <= s[3] < b0 + nb]
        assert inside and all(s[3] + -(-s[2] // 256) <= b0 + nb for s in inside)


def test_dered_plan_absent_without_exact_float_filter():
    """uint8 input, knots, or no dereddening: no dereddening plan."""
    for dt, dw, st in (("u8", -1, 0), ("f32", -1, 8), ("f32", 0, 0)):
        plan = ffa.Plan(1 << 16, 1e-3, 0.2, 1.0, 100, None, dt, dered_window=dw, dered_stride=st)
        segs, launches = _dered_plan(plan)
        assert len(segs) == 0 and len(launches) == 0
