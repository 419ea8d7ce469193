"""CPU oracle for the Binary Stereo Matching hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is a thin ctypes
wrapper over ``liboracle.so`` (built from ``bsm_oracle.c``), which is a plain
CPU definition of Zhang et al., "Binary Stereo Matching", Section 3,
Eq. 1-8, plus the right-reference map and the left/right check that open
Section 3's refinement step.  It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    INVALID_COST,
    cost_volume,
    describe,
    lab8,
    lab8_tables,
    load,
    lr_check,
    luma,
    make_pattern,
    mask,
    match,
    match_right,
    normal_draws,
    set_threads,
    get_threads,
    splitmix64,
    vote_refine,
    weights,
    wta,
)
