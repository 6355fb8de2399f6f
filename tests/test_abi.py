"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every declared entry point, validates arguments, and plans exactly the steps
the oracle plans."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1703_05581_amd import ffa, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "ffa.h")).read()
    return sorted(set(re.findall(r"\b(ffa_[a-z_]+)\s*\(", hdr)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 17
    lib = ffa.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ffa.EXPORTS)


def test_status_strings():
    assert ffa.lib().ffa_status_str(0) == b"FFA_OK"
    assert ffa.lib().ffa_status_str(-5) == b"FFA_ERR_BUSY"


@pytest.mark.parametrize("wl", [1, 2, 3])
def test_plan_matches_oracle(oracle_mod, wl):
    pa = synth.plan_args(wl)
    p = ffa.Plan.from_args(pa)
    o = oracle_mod.plan(pa.N, pa.tsamp, pa.pmin, pa.pmax, pa.bins_min)
    assert p.n_steps == o.n_steps and p.n_trials == o.n_trials
    for s in range(p.n_steps):
        st = p.step(s)
        assert (st.f, st.P0, st.m, st.M, st.first_trial) == (
            o.f[s], o.P0[s], o.m[s], o.M[s], o.first[s]), s
        d = p.passes(s)
        assert sum(d) == int(o.M[s]).bit_length() - 1 and all(x >= 1 for x in d)
    assert np.array_equal(p.periods(), o.periods())


def test_plan_matches_oracle_random(oracle_mod):
    g = np.random.default_rng(5)
    for _ in range(40):
        N = int(g.integers(100, 300000))
        tsamp = float(g.choice([1e-3, 0.512e-3, 6.4e-5, 2.5e-4]))
        B = int(g.integers(2, 300))
        pmin = float(g.uniform(B * tsamp * 0.5, B * tsamp * 4))
        pmax = pmin * float(g.uniform(1.01, 40))
        mo = int(g.integers(0, 4))
        try:
            p = ffa.Plan(N, tsamp, pmin, pmax, B, [1, 2, 4], max_octaves=mo)
        except ffa.FFAError as e:
            assert e.status == ffa.FFA_ERR_INVALID
            assert oracle_mod.plan(N, tsamp, pmin, pmax, B, mo).n_steps == 0
            continue
        o = oracle_mod.plan(N, tsamp, pmin, pmax, B, mo)
        assert p.n_steps == o.n_steps and p.n_trials == o.n_trials
        got = np.array([tuple(vars(p.step(s)).values()) for s in range(p.n_steps)])
        ref = np.stack([o.f, o.P0, o.m, o.M, o.first], axis=1)
        assert np.array_equal(got, ref)


def _desc(**kw):
    base = dict(N=65536, tsamp_s=1e-3, pmin_s=0.5, pmax_s=1.0, widths=None, n_widths=0,
                bins_min=500, max_octaves=0, dtype=0, snr=1)
    base.update(kw)
    return ffa.PlanDesc(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(N=1), ffa.FFA_ERR_INVALID),
    (dict(tsamp_s=0.0), ffa.FFA_ERR_INVALID),
    (dict(pmax_s=0.4), ffa.FFA_ERR_INVALID),
    (dict(bins_min=1), ffa.FFA_ERR_INVALID),
    (dict(bins_min=2000), ffa.FFA_ERR_INVALID),
    (dict(dtype=7), ffa.FFA_ERR_INVALID),
    (dict(snr=9), ffa.FFA_ERR_INVALID),
    (dict(dered_window=-2), ffa.FFA_ERR_INVALID),
    (dict(dered_stride=-1), ffa.FFA_ERR_INVALID),
    (dict(n_widths=40), ffa.FFA_ERR_INVALID),
    (dict(n_widths=3), ffa.FFA_ERR_INVALID),           # NULL widths
    (dict(pmin_s=50.0, pmax_s=60.0), ffa.FFA_ERR_INVALID),  # no step
    (dict(N=1 << 24, dtype=1, pmin_s=0.5, pmax_s=1.0), ffa.FFA_ERR_UNSUPPORTED),
])
def test_plan_create_rejects(kw, status):
    h = ctypes.c_void_p()
    d = _desc(**kw)
    assert ffa.lib().ffa_plan_create(ctypes.byref(d), ctypes.byref(h)) == status
    assert not h
    assert ffa.lib().ffa_last_error()


def test_plan_rejects_widths_all_above_p0():
    w = (ctypes.c_int32 * 1)(600)
    d = _desc(widths=ctypes.cast(w, ctypes.POINTER(ctypes.c_int32)), n_widths=1)
    h = ctypes.c_void_p()
    assert ffa.lib().ffa_plan_create(ctypes.byref(d), ctypes.byref(h)) == ffa.FFA_ERR_INVALID


def test_null_arguments_rejected_before_gpu():
    lib = ffa.lib()
    assert lib.ffa_plan_query(None, None, None, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_search(None, None, None, None, None, 0, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_fold(None, None, 0, None, None, 0, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_best(None, 0, None, None) == ffa.FFA_ERR_INVALID
    p = ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, [1, 2, 4])
    # a small workspace is refused on the host, before any device call
    assert lib.ffa_search(p.handle, 1, 2, 3, 256, 16, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_search(p.handle, 1, 2, 3, 257, p.ws_bytes, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_fold(p.handle, 1, p.n_steps, 3, 256, p.ws_bytes, None) == ffa.FFA_ERR_INVALID


def test_batch_workspace():
    """A batch workspace holds the output table, every series' own region of
    octave series and one intermediate ring per queue; ffa_batch_workspace
    equals an explicit batch's size; the batch's queue is walked like a
    plan's (tile_emu); an empty batch or a null plan is refused."""
    from tile_emu import check_batch

    a = ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, [1, 2], "u8")
    b = ffa.Plan(200000, 1e-3, 0.5, 1.0, 500, [1, 2], "f32")
    ws = ctypes.c_size_t()
    lib = ffa.lib()
    for plans in ([a], [a, b], [a, b, a, b, a, b]):
        arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
        assert lib.ffa_batch_workspace(len(plans), arr, ctypes.byref(ws)) == ffa.FFA_OK
        bt = ffa.Batch(plans)
        assert ws.value == bt.ws_bytes
        assert bt.n_tiles == sum(len(tile_phases(p)) for p in plans)
        qs = check_batch(bt)
        assert len(qs) == len({p.dtype for p in plans})
        bt.close()
    arr = (ctypes.c_void_p * 1)(a.handle)
    assert lib.ffa_batch_workspace(0, arr, ctypes.byref(ws)) == ffa.FFA_ERR_INVALID
    assert lib.ffa_batch_workspace(1, None, ctypes.byref(ws)) == ffa.FFA_ERR_INVALID
    assert lib.ffa_search_batch(1, arr, None, None, None, None, 0, None) == ffa.FFA_ERR_INVALID
    arr2 = (ctypes.c_void_p * 2)(a.handle, None)
    assert lib.ffa_batch_workspace(2, arr2, ctypes.byref(ws)) == ffa.FFA_ERR_INVALID


def tile_phases(plan):
    from tile_emu import layout

    return range(int(layout(plan)["n_tiles"]))


def test_batch_of_random_plans_walks_clean():
    """Batches of random plans (both sample types, both algorithms, tiny ring
    budgets that make the shared arena wrap) pass the host walk of every
    tile's reads, writes and launch order."""
    from tile_emu import check_batch

    g = np.random.default_rng(7)
    W10 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]
    for rep in range(3):
        plans = []
        for i in range(6):
            N = int(g.choice([20000, 65536, 150000, 300000]))
            B = int(g.choice([64, 100, 256, 500]))
            pmin = B * 1e-3 * float(g.uniform(1.0, 1.5))
            pmax = pmin * float(g.uniform(2.0, 12.0))
            opts = {"ring_mb": 4, "window_tiles": 500} if rep == 1 else {}
            plans.append(ffa.Plan(N, 1e-3, pmin, pmax, B, None if i % 3 == 0 else W10,
                                  "u8" if g.random() < 0.5 else "f32", snr=1 + int(g.random() < 0.3), opts=opts))
        check_batch(ffa.Batch(plans))


def test_server_argument_errors_before_gpu():
    """Bad server arguments are refused on the host, before any device call."""
    lib = ffa.lib()
    h = ctypes.c_void_p()
    assert lib.ffa_server_create(1 << 30, 4, 0, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_server_create(1 << 30, 0, 0, ctypes.byref(h)) == ffa.FFA_ERR_INVALID
    assert lib.ffa_server_create(1 << 30, 17, 0, ctypes.byref(h)) == ffa.FFA_ERR_INVALID
    assert lib.ffa_server_create(100, 2, 0, ctypes.byref(h)) == ffa.FFA_ERR_INVALID
    assert lib.ffa_server_create(1 << 30, 2, -1, ctypes.byref(h)) == ffa.FFA_ERR_INVALID
    t = ctypes.c_int64()
    assert lib.ffa_server_submit(None, None, None, 0, None, ctypes.byref(t)) == ffa.FFA_ERR_INVALID
    assert lib.ffa_debug_server_fail(None, 1) == ffa.FFA_ERR_INVALID
    assert lib.ffa_server_wait(None, 1, 0, None, None, None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_server_destroy(None) == ffa.FFA_ERR_INVALID


def test_alg2_plans():
    """Algorithm 2 plans build like Algorithm 1 plans (same steps, same
    workspace)."""
    a = ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, [1, 2, 4], "f32", snr=ffa.FFA_SNR_ALG1_MAD)
    b = ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, [1, 2, 4], "f32", snr=ffa.FFA_SNR_ALG2_OFFPULSE)
    assert (a.n_trials, a.n_steps, a.ws_bytes) == (b.n_trials, b.n_steps, b.ws_bytes)


def test_dered_plans():
    """Dereddening moves a uint8 plan to float folding, so the uint8 length
    bound no longer applies; the workspace grows by the knot medians."""
    big = dict(N=1 << 24, dtype=1, pmin_s=0.5, pmax_s=1.0, bins_min=500)
    d = _desc(**big)
    h = ctypes.c_void_p()
    assert ffa.lib().ffa_plan_create(ctypes.byref(d), ctypes.byref(h)) == ffa.FFA_ERR_UNSUPPORTED
    d = _desc(dered_window=-1, **big)
    assert ffa.lib().ffa_plan_create(ctypes.byref(d), ctypes.byref(h)) == ffa.FFA_OK
    ffa.lib().ffa_plan_destroy(h)
    a = ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, [1, 2], "u8")
    b = ffa.Plan(65536, 1e-3, 0.5, 1.0, 500, [1, 2], "u8", dered_window=-1)
    assert b.ws_bytes > a.ws_bytes and a.n_trials == b.n_trials


def test_sift_argument_errors_before_gpu():
    """ffa_sift checks its pointers, limits and workspace before any GPU call."""
    p = ffa.Plan(65536, 1e-3, 0.5, 1.0, 500)
    lib = ffa.lib()
    good = ffa.SiftParams(9.0, 0.1, 1.0, 2.0, 31, 1e-5)
    fake = 4096
    assert lib.ffa_sift(p.handle, None, fake, ctypes.byref(good), fake, 8, fake, fake, p.ws_bytes,
                        None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_sift(p.handle, fake, fake, ctypes.byref(good), None, 8, fake, fake, p.ws_bytes,
                        None) == ffa.FFA_ERR_INVALID
    assert lib.ffa_sift(p.handle, fake, fake, ctypes.byref(good), fake, -1, fake, fake, p.ws_bytes,
                        None) == ffa.FFA_ERR_INVALID
    for field, value in [("frac_fall", 1.5), ("frac_fall", -0.1), ("abs_fall", -1.0),
                         ("group_widths", float("inf")), ("harmonic_tol", -1e-3),
                         ("min_snr", float("nan")), ("harmonic_primes", 5000)]:
        bad = ffa.SiftParams(9.0, 0.1, 1.0, 2.0, 31, 1e-5)
        setattr(bad, field, value)
        assert lib.ffa_sift(p.handle, fake, fake, ctypes.byref(bad), fake, 8, fake, fake, p.ws_bytes,
                            None) == ffa.FFA_ERR_INVALID, field
    assert lib.ffa_sift(p.handle, fake, fake, ctypes.byref(good), fake, 8, fake, fake, 64,
                        None) == ffa.FFA_ERR_INVALID
    p.close()
