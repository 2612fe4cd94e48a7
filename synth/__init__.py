"""Seeded synthetic inputs (potential, strain, field, lever arms) for the hole
k.p eigensolver.  Shared by the tests, the benchmark and the smoke check; holds
none of the eigensolver's arithmetic.
"""

from .inputs import (  # noqa: F401
    Workload, WORKLOADS, workload, smooth_field, fin_potential, random_block, SPDevice,
    sp_device,
)
