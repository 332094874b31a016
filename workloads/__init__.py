"""Seeded synthetic inputs shared by the CPU oracle tests and the HIP path.

This package holds input generation only: a counter-based random generator,
the analytic test problems of the paper (right-hand sides, boundary data and
exact solutions), and the workload configurations.  It contains none of the
solver's arithmetic (no stencil weights, no transforms, no tridiagonal solves),
so the oracle and the device path can both take their inputs from here while
sharing no solver code.
"""
from .gen import (  # noqa: F401
    splitmix64_u64,
    uniform01,
    uniform_pm1,
    gaussian,
)
from .problems import (  # noqa: F401
    Problem,
    paper_variable_k,
    paper_cd,
    manufactured_sin3,
    config1,
    config2,
    config3,
    config5,
    batch_members,
    noise_problem,
    complex_noise_problem,
    manufactured_cos2,
    neumann_noise_problem,
    config5_absorbing,
    K_ABSORB,
    robin_noise_problem,
    manufactured_robin,
)
