"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package draws spot clouds, request streams and the fixed optical
constants of the workloads. It holds none of the hologram arithmetic
(no phases, no propagation, no weight update): both the GPU library and
the CPU oracle receive what it draws as plain arrays.
"""
from .spots import (  # noqa: F401
    Grid, Optics, Spots, OPTICS, PUPIL_OPTICS, PITCH_MM, lateral_half_range_mm,
    spot_cloud, mixed_batch, poisson_stream, Workload, WORKLOADS, PUPIL_WORKLOAD,
)
from .scenarios import (  # noqa: F401
    SCENARIOS, random_rotation, rotating_grid, two_cubes, scenario,
)
