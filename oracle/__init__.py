"""CPU oracle of the FFA search (test infrastructure only).

Only the test-suite (with its fixture scripts under tests/golden/),
``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    ALG1,
    ALG2,
    IN_F32,
    IN_U8,
    Plan,
    alg1,
    alg2,
    build,
    default_widths,
    dered_default_window,
    deredden,
    downsample,
    fold,
    fold_step,
    library,
    mad_constant,
    plan,
    search,
    score_profiles,
    sift,
    sigma_gauss,
    sigma_threshold,
    snr_histogram,
)
