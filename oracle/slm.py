"""Phase-to-gray conversion of the SLM output, plain and slow.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's GPU-implementation section lists, among the fixed parameters
uploaded once at start-up, the phase to gray scale lookup table of the SLM:
the hologram Phi is shown on the SLM as gray levels through that table.

Reading: a table of L gray levels g[0..L-1] covers one period of phase, bin k
holding the phases with k/L <= frac(Phi / 2 pi) < (k + 1)/L, so that phases
that differ by a whole turn show the same gray level and a negative phase
wraps into [0, 2 pi).

The bin index is an integer decided by floating-point arithmetic, so it is
taken here in the same precision as on the device, FP32, in these steps:
    t = fl32(Phi * fl32(1 / (2 pi)))     (one rounded product)
    t = fl32(t - floor(t))               (exact for t >= 0; one rounded
                                          difference for t < 0)
    k = floor(fl32(t * L))               (one rounded product)
    k = min(k, L - 1)                    (t rounds up to 1.0 just below a
                                          whole turn)
Parity is pinned by exact arithmetic on the bins (tests/test_oracle_slm.py):
away from a bin edge the index is the exact bin of Phi; within FP32
rounding of an edge it is one of its two neighbours.
"""
from __future__ import annotations

import numpy as np

INV_TWO_PI_F32 = np.float32(1.0 / (2.0 * np.pi))


def gray_index(Phi, levels: int) -> np.ndarray:
    """Table index (int64) of each phase Phi (radians, any real)."""
    phi = np.asarray(Phi, dtype=np.float32)
    L = int(levels)
    with np.errstate(over="ignore", invalid="ignore"):
        t = phi * INV_TWO_PI_F32                   # float32 product
        t = (t - np.floor(t)).astype(np.float32)   # float32 difference
        k = np.floor(t * np.float32(L)).astype(np.int64)
    return np.minimum(k, L - 1)


def gray_levels(Phi, table) -> np.ndarray:
    """Gray level g[k] of each phase, in the table's dtype."""
    table = np.asarray(table)
    return table[gray_index(Phi, table.shape[0])]
