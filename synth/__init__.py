"""Seeded synthetic inputs for the unaligned RKHS (infinite-mode) CP-HIFI subproblem.

This module only draws random numbers and lays out problem data: design points,
the kernel matrix K evaluated at them, the observation set Omega (as time-major
CSR), the fixed factor matrices of the other modes and the observed values y.
It contains none of the solver's arithmetic, and it is shared by the CPU
oracle, the tests and the benchmark so that both sides see identical inputs.
"""

from .generator import (  # noqa: F401
    Problem,
    BatchMember,
    gaussian_kernel,
    matern32_kernel,
    make_unaligned,
    make_aligned,
    make_small,
    make_batch,
    batch_members,
    make_paper_standin,
    AlsProblem,
    make_als_problem,
    config_c1,
    config_c2,
    config_c3,
    config_c5,
    drop_observations,
    sample_rows,
    probe_matrices,
)
