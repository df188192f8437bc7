"""Seeded synthetic workloads shared by the oracle side and the HIP side.

This package only draws random inputs (matrices, right-hand sides, Gaussian
projections).  It holds none of the sketching, factorisation or solving
arithmetic, so that both sides of every parity test start from the same bytes
without sharing any of the method's code.
"""

from .gen import (  # noqa: F401
    CSR,
    bf16_round,
    bf16_to_f32,
    csr_uniform_rows,
    dense_gaussian,
    gaussian_matrix,
    lstsq_small,
    sketch_csr,
    sketch_csr_int,
    sketch_dense,
    pareto_rows,
    learned_family,
    learned_rhs,
    planted_lowrank_sparse,
    lp_sparse,
    lp_dense,
    SKETCH_SEED_BASE,
    data_seed,
    sketch_seed,
)
