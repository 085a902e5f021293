"""CPU FP64 oracle for RS, WGS and CS-WGS point-cloud holograms.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that
the GPU library is checked against.  Only the test suite, the smoke check of
the build entry point and the CPU-baseline leg of the benchmark may import
it.  The product path (the HIP library and its Python binding) never imports,
calls or links anything here, and this package imports nothing from the
product path.

Parity status of each function is stated in the module headers:
  philox.py  - pinned to numpy.random.Philox (library routine)
  sampler.py - pinned by brute-force bijectivity / partition properties
  hg.py      - pinned by closed forms, invariants, FFT and mpmath brute force
               (tests/test_oracle_*.py); the full CS-WGS trajectory has no
               printed worked example in the paper and is pinned only
               through those pieces.
  slm.py     - phase-to-gray lookup from the bin definition (FP64, exact at
               bin edges), pinned by 60-digit arithmetic on the bins
"""
from .philox import philox4x64_10, PHILOX_M, PHILOX_W  # noqa: F401
from .sampler import (  # noqa: F401
    half_bits, round_tables, feistel, permute, subset_size, subset, theta0, ORDER_KEY,
)
from .hg import (  # noqa: F401
    pixel_offsets_mm, spot_phase, backward, forward, update, rs, wgs, cswgs,
    metrics, Trace, pupil_pixels, illumination, efficiency, uniformity,
)
from .slm import gray_index, gray_levels, gray_bin, fp32_edge_tolerance  # noqa: F401
