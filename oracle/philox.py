"""Philox4x64-10 counter-based generator, written from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11, section on the Philox family).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

One block maps a 256-bit counter (four 64-bit words) and a 128-bit key (two
64-bit words) to four 64-bit outputs through 10 rounds.  Each round multiplies
words 0 and 2 by two fixed odd constants, keeps the high and low halves of the
128-bit products, and mixes the high halves with words 1 and 3 and the key.
The key is advanced by two Weyl constants between rounds.

Pin: numpy.random.Philox implements the same generator; tests compare raw
blocks bit for bit (numpy emits block c+1 first when started at counter c).
Plain Python integers are used so the arithmetic is exact and readable.
"""
from __future__ import annotations

from typing import Sequence, Tuple

MASK64 = (1 << 64) - 1
# Round multipliers and key increments of Philox4x64 (published constants).
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def _mulhilo(a: int, b: int) -> Tuple[int, int]:
    prod = a * b
    return prod >> 64, prod & MASK64


def philox4x64_10(counter: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    """One Philox4x64 block with 10 rounds."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W[0]) & MASK64
            k1 = (k1 + PHILOX_W[1]) & MASK64
        hi0, lo0 = _mulhilo(PHILOX_M[0], c0)
        hi1, lo1 = _mulhilo(PHILOX_M[1], c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3
