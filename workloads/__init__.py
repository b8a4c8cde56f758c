"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side tests.

This package holds parameter sets and seeded random-number draws only. It
contains none of the parquet arithmetic (no Green's functions, no bubbles, no
vertex algebra), so that the CPU oracle and the GPU path share nothing but
their inputs.
"""
from .synthetic import (  # noqa: F401
    ModelParams,
    CONFIGS,
    config,
    rand_complex,
    bse_microbench_gamma,
    random_phi,
    random_sigma,
    lowrank_phi_factors,
    lambda_box_parts,
    parameter_draws,
    batch_draws,
)
