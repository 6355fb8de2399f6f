"""The plan autotuner: shape classes, the cache and the launch options on
the host, and on the GPU that every candidate setting gives the same
periodogram (uint8: bit for bit) and that the cached choice is what
tuned_plan uses."""
import pytest

from paper_1703_05581_amd import synth, tune


def test_shape_class_and_cache(tmp_path):
    pa = synth.plan_args(2)
    c = tune.shape_class(pa)
    assert c == "u8/alg1/raw/n20/b256/oct3"
    assert tune.shape_class(synth.plan_args(3)).startswith("f32/alg1/dered/n23/b256/")
    path = str(tmp_path / "cache.json")
    assert tune.load_cache(path) == {}
    tune.save_cache({"gfx950": {c: {"knobs": {"window_tiles": 65536}, "ms": 1.0}}}, path)
    assert tune.cached_setting(pa, arch="gfx950", path=path) == {"window_tiles": 65536}
    assert tune.cached_setting(synth.plan_args(1), arch="gfx950", path=path) is None


def test_settings_are_plan_options():
    """A setting reaches the planner through ffa_plan_opts, not the process
    environment: two plans made with different settings coexist."""
    pa = synth.plan_args(2)
    a = tune.make_plan(pa, {"window_tiles": 500})
    b = tune.make_plan(pa, {})
    assert a.opts == {"window_tiles": 500} and b.opts == {}
    from tile_emu import layout

    assert len(layout(a)["launches"]) > len(layout(b)["launches"])


def test_settings_change_the_plan_layout():
    pa = synth.plan_args(2)
    a = tune.make_plan(pa, {})
    b = tune.make_plan(pa, {"ring_mb": 2048})
    assert a.n_trials == b.n_trials and a.ws_bytes > b.ws_bytes


@pytest.mark.gpu
def test_autotune_candidates_agree(tmp_path):
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pa = synth.PlanArgs(N=300000, tsamp=1e-3, pmin=0.2, pmax=2.0, bins_min=100,
                        widths=(1, 2, 3, 4, 6, 8, 12, 16, 24, 32), dtype="u8", max_octaves=0,
                        dered_window=0, dered_stride=0)
    x = torch.from_numpy(synth.random_series(5, pa.N, "u8")).cuda()
    path = str(tmp_path / "cache.json")
    cands = ({}, {"window_tiles": 500}, {"tile_lds_bytes": 49152, "ring_mb": 64}, {"no_u16": 1})
    res = tune.autotune(pa, x, candidates=cands, reps=2, path=path)
    print("autotune", res, flush=True)
    assert len(res["trials"]) == len(cands) and res["knobs"] in [dict(c) for c in cands]
    assert tune.cached_setting(pa, path=path) == res["knobs"]
    outs = []
    for setting in cands:
        plan = tune.make_plan(pa, setting)
        outs.append([t.clone() for t in plan.search(x)])
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])
    plan = tune.tuned_plan(pa, path=path)
    s, w = plan.search(x)
    torch.cuda.synchronize()
    assert torch.equal(s, outs[0][0]) and torch.equal(w, outs[0][1])
