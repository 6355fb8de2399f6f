"""A seeded sweep of random search configurations on the GPU against the
oracle, through the C ABI: series length, base period, period range, width
set (given or the paper's default rule), sample type, scoring algorithm,
dereddening and the LDS budget of a tile (which changes the pass split and
the radix-4 pairing of levels) are all drawn per case."""
import numpy as np
import pytest

from test_gpu_parity import run_case

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


def _case(seed, oracle):
    """Draw a configuration whose plan has at least one step."""
    g = np.random.default_rng(seed)
    while True:
        N = int(g.integers(2000, 80000))
        B = int(g.choice([8, 13, 30, 64, 97, 150, 256, 300, 511, 600]))
        tsamp = 1e-3
        pmin = B * tsamp * float(g.uniform(1.0, 1.6))
        pmax = pmin * float(g.uniform(1.3, 8.0))
        if g.random() < 0.5:
            widths = sorted(set(int(w) for w in g.integers(1, 40, size=int(g.integers(1, 9)))))
        else:
            widths = None
        dtype = "u8" if g.random() < 0.5 else "f32"
        alg = 1 if g.random() < 0.6 else 2
        dered = int(g.choice([0, 0, 0, 31, 400]))
        lds = int(g.choice([160 * 1024, 96 * 1024, 48 * 1024, 24 * 1024]))
        op = oracle.plan(N, tsamp, pmin, pmax, B)
        if op.n_steps == 0 or (widths is not None and min(widths) > B):
            continue
        return dict(N=N, B=B, tsamp=tsamp, pmin=pmin, pmax=pmax, widths=widths, dtype=dtype, alg=alg,
                    dered=dered, lds=lds, seed=seed)


@pytest.mark.parametrize("seed", range(32))
def test_random_configuration(torch_cuda, ffa, oracle_mod, seed):
    from paper_1703_05581_amd import synth

    c = _case(1000 + seed, oracle_mod)
    print("random case", c, flush=True)
    x = synth.random_series(c["seed"], c["N"], c["dtype"])
    widths = c["widths"]
    if c["alg"] == 2 and widths and (c["dtype"] == "f32" or c["dered"]):
        # float profiles: a box over half the profile leaves too few
        # off-pulse bins for a float32 sigma (its rounding is amplified about
        # A^2-fold); exact integer profiles keep every width
        widths = [w for w in widths if 2 * w <= c["B"]] or [1]
    if c["dered"] and c["dtype"] == "f32":
        x = (x + 5.0 * np.sin(np.arange(c["N"]) / 900.0)).astype(np.float32)
    run_case(torch_cuda, ffa, oracle_mod, x, c["N"], c["tsamp"], c["pmin"], c["pmax"], c["B"], widths,
             c["dtype"], steps_max=10, check_fold=1, alg=c["alg"], dered_window=c["dered"],
             opts={"tile_lds_bytes": c["lds"]})
