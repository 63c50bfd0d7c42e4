"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input generation only: molecule-shaped model Hamiltonians in
Cholesky form, trial determinants, and the counter-based random stream from
which the auxiliary fields and the population-control uniforms are drawn.  It
contains none of the AFQMC arithmetic (overlaps, Green's functions, force bias,
propagation, local energy, weights); those live separately in ``oracle/``
(CPU reference) and in the HIP library (GPU path), which share no code.
"""

from .hamiltonian import (  # noqa: F401
    CONFIGS,
    SyntheticSystem,
    config_system,
    diagonal_system,
    gen_system,
    random_walkers,
)
from .fields import (  # noqa: F401
    STREAM_COMB,
    STREAM_FIELDS,
    comb_uniform,
    gaussian_fields,
    philox_u64,
    u64_to_unit,
)
from .trials import excitation_trial, noci_trial, occupation_det, rhf_trial  # noqa: F401
from .workloads import batch_workload, serving_trace  # noqa: F401
