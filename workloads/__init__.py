"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws and places particles. It holds none of the method's
arithmetic (no kernel, no expansion, no summation): the vortex-particle state
(x, alpha, sigma) it returns is what both the FP64 oracle and the HIP library
consume. All arrays are float32, structure-of-arrays, C-contiguous.
"""
from .gen import (  # noqa: F401
    lattice_positions,
    taylor_green_case,
    turbulence_case,
    ring_case,
    ring_batch,
    random_cloud,
    clustered_cloud,
    varcore_case,
    corner_lattice,
    jittered,
    graded_cores,
    checksum,
    checksum_matches,
    case_arrays,
)
