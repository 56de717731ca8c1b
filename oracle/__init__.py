"""Double-precision CPU oracle of the micro-DPD hot path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path never imports
this package.  See ``lhmm_oracle.c`` for what each function follows.
"""
from .oracle import (  # noqa: F401
    ERR_ARG,
    ERR_BOND,
    ERR_CELL,
    ERR_NONFINITE,
    OracleBox,
    afbc_noise,
    afbc_region,
    build,
    check_gradient,
    core_fraction,
    expL,
    forces,
    lib,
    max_threads,
    pairs,
    philox4x32_10,
    reduce_cell,
    run_batch,
    run_box,
    run_box_afbc,
    sph_accel,
    sph_density,
    sph_F,
    sph_gradv,
    sph_params_vector,
    sph_polymer_stress,
    sph_step,
    sph_W,
    theta,
    uniform23,
    widths,
)
