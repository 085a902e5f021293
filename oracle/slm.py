"""Phase-to-gray conversion of the SLM output, from the bin definition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's GPU-implementation section lists, among the fixed parameters
uploaded once at start-up, the phase to gray scale lookup table of the SLM:
the hologram Phi is shown on the SLM as gray levels through that table.

Reading: a table of L gray levels g[0..L-1] covers one period of phase, bin k
holding the phases with k/L <= frac(Phi / 2 pi) < (k + 1)/L, so that phases
that differ by a whole turn show the same gray level and a negative phase
wraps into [0, 2 pi).

This module computes that definition for the phase value as given (an FP32
hologram converts to FP64 exactly):
    y = L * frac(Phi / 2 pi),    k = floor(y)
first in FP64 (numpy), where every step is within a few units of 2^-53 of
the exact value, then, for every phase whose y lies within 1e-9 of an
integer (a bin edge), again with 2 pi to 50 digits (mpmath), so the bin is
the exact one everywhere.  `gray_bin` also returns the distance of y to the
nearest bin edge, in bins: an implementation that takes the bin in lower
precision may land in either bin that meets at an edge when the phase lies
within its rounding of that edge, and a comparison needs that distance to
decide whether a neighbouring bin is acceptable.

Pins: tests/test_oracle_slm.py (exact arithmetic at 60 digits on random
phases over many turns of both signs, bin centres, range, table lookup, and
planted mistakes).
"""
from __future__ import annotations

import math

import numpy as np

_EDGE = 1e-9  # in bins: phases this close to an edge are redone at 50 digits


def _exact(phi: float, L: int):
    import mpmath
    with mpmath.workdps(50):
        x = mpmath.mpf(phi) / (2 * mpmath.pi)
        f = x - mpmath.floor(x)
        y = f * L
        k = int(mpmath.floor(y))
        d = min(y - mpmath.floor(y), mpmath.ceil(y) - y)
        return k % L, float(d)


def gray_bin(Phi, levels: int):
    """Exact bin index (int64) of each phase Phi (radians, any finite real)
    and the distance of L*frac(Phi/2pi) to the nearest bin edge, in bins."""
    L = int(levels)
    phi = np.asarray(Phi, dtype=np.float64).ravel()
    t = phi / (2.0 * math.pi)
    f = t - np.floor(t)
    y = f * L
    k = np.floor(y).astype(np.int64) % L
    d = np.minimum(y - np.floor(y), np.ceil(y) - y)
    for i in np.flatnonzero(d < _EDGE):
        k[i], d[i] = _exact(float(phi[i]), L)
    shape = np.shape(Phi)
    return k.reshape(shape), d.reshape(shape)


def gray_index(Phi, levels: int) -> np.ndarray:
    """Table index (int64) of each phase Phi: the exact bin."""
    return gray_bin(Phi, levels)[0]


def gray_levels(Phi, table) -> np.ndarray:
    """Gray level g[k] of each phase, in the table's dtype."""
    table = np.asarray(table)
    return table[gray_index(Phi, table.shape[0])]


def fp32_edge_tolerance(Phi, levels: int) -> np.ndarray:
    """Distance to a bin edge, in bins, within which a bin taken in FP32
    (t = fl(Phi * fl(1/2pi)), t = fl(t - floor(t)), k = floor(fl(t * L)))
    may fall on either side of the edge: the rounding of Phi/2pi
    (|t| 2^-23), of the wrap (2^-25) and of the scaling (2^-24), in bins,
    doubled for margin."""
    t = np.abs(np.asarray(Phi, dtype=np.float64)) / (2.0 * math.pi)
    return int(levels) * (t + 1.0) * 2.0 ** -22
