"""Seeded random draws of the method: initial spot phases and the pixel subsets
of the compressed iterations.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, algorithm section: RS takes random initial phases theta_n^0; CS-WGS sums
the forward projection over a random subset of the pixels in each iteration.
Paper, GPU implementation section (compressed sensing): the pixels are put in
one random order at start-up and each iteration works on a contiguous run of
c*M entries of that order.  The paper names no generator, so both sides use
one counter-based construction, defined here:

* Block B(ctr, key) is Philox4x64-10 (oracle/philox.py).
* theta_n^0 = 2*pi * u_n, u_n = (B((n,0,0,0), (seed,0))[0] >> 11) * 2^-53, so
  u_n is uniform on [0, 1) with 53 random bits.
* The random pixel order is a keyed Feistel permutation pi of [0, M):
  h = smallest integer >= 1 with 4^h >= M; six rounds on the two h-bit halves
  (L, R) of x < 4^h, round r mapping (L, R) -> (R, L xor F_r[R]) with
  F_r[R] = B((R, r, 0, 0), (seed, 1))[0] mod 2^h.  Values >= M are walked
  along their cycle (apply the rounds again) until they land in [0, M), which
  keeps pi a bijection of [0, M).
* m = ceil(c * M) in FP64; the subset of iteration j (j >= 1) is
  Omega^j = [ pi(((j - 1) * m + q) mod M) for q in 0..m-1 ], in q order: a
  window sliding along the one fixed order, wrapping at M.
* The order is made once, at start-up, for the SLM (its grid and pupil) and
  serves every hologram: the algorithms key it with ORDER_KEY, not with the
  hologram's seed, which draws theta^0 alone.

Pins: bijectivity of pi by brute force, the partition of [0, M) by
consecutive windows when m divides M, and uniformity of the subsets
(tests/test_oracle_sampler.py).  theta^0 is pinned through the Philox pin.
"""
from __future__ import annotations

import functools
import math

import numpy as np

from .philox import philox4x64_10

FEISTEL_ROUNDS = 6
ORDER_KEY = 0  # key of the one random pixel order that the algorithms use


def theta0(seed: int, n: int) -> np.ndarray:
    """Initial phases theta_n^0 in radians, uniform on [0, 2*pi)."""
    out = np.empty(n, dtype=np.float64)
    for k in range(n):
        word = philox4x64_10((k, 0, 0, 0), (seed, 0))[0]
        out[k] = 2.0 * math.pi * ((word >> 11) * 2.0**-53)
    return out


def half_bits(M: int) -> int:
    """Smallest h >= 1 with 4^h >= M."""
    h = 1
    while (1 << (2 * h)) < M:
        h += 1
    return h


@functools.lru_cache(maxsize=16)
def _round_tables_cached(seed: int, h: int) -> bytes:
    size = 1 << h
    t = np.empty((FEISTEL_ROUNDS, size), dtype=np.uint64)
    mask = size - 1
    for r in range(FEISTEL_ROUNDS):
        for R in range(size):
            t[r, R] = philox4x64_10((R, r, 0, 0), (seed, 1))[0] & mask
    return t.tobytes()


def round_tables(seed: int, h: int) -> np.ndarray:
    """F_r[R] for r < 6, R < 2^h, as uint64 array of shape (6, 2^h)."""
    return np.frombuffer(_round_tables_cached(int(seed), int(h)),
                         dtype=np.uint64).reshape(FEISTEL_ROUNDS, 1 << h)


def feistel(x: np.ndarray, tables: np.ndarray, h: int) -> np.ndarray:
    """Six Feistel rounds on x < 4^h (vectorised over x)."""
    x = np.asarray(x, dtype=np.uint64)
    mask = np.uint64((1 << h) - 1)
    L = x >> np.uint64(h)
    R = x & mask
    for r in range(FEISTEL_ROUNDS):
        L, R = R, L ^ tables[r][R]
    return (L << np.uint64(h)) | R


def permute(k: np.ndarray, M: int, seed: int) -> np.ndarray:
    """pi(k) for k in [0, M): Feistel with cycle walking."""
    h = half_bits(M)
    tables = round_tables(seed, h)
    y = feistel(np.asarray(k, dtype=np.uint64), tables, h)
    out_of_range = y >= np.uint64(M)
    while np.any(out_of_range):
        y[out_of_range] = feistel(y[out_of_range], tables, h)
        out_of_range = y >= np.uint64(M)
    return y.astype(np.int64)


def subset_size(M: int, c: float) -> int:
    """m = ceil(c * M), evaluated in FP64."""
    return int(math.ceil(float(c) * float(M)))


def subset(M: int, seed: int, j: int, c: float) -> np.ndarray:
    """Omega^j: pixel indices of the compressed iteration j (j >= 1), q order."""
    m = subset_size(M, c)
    k = ((j - 1) * m + np.arange(m, dtype=np.int64)) % M
    return permute(k, M, seed)
