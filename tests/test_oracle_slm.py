"""Pins of the oracle's phase-to-gray lookup (oracle/slm.py) against exact
arithmetic on the table's bins, independently of its FP32 steps:

* bin k holds the phases with k/L <= frac(Phi / 2 pi) < (k+1)/L: checked
  with 2 pi to 60 digits (mpmath) on random FP32 phases over many turns,
  both signs; away from a bin edge (farther than the FP32 rounding of
  Phi / 2 pi) the index is the exact bin, next to an edge it is one of the
  two bins that meet there;
* bin centres of every bin, in the first turn, in later turns and at
  negative phases (wrap), map to that bin;
* the index is always in [0, L) and the gray level is the table entry.
Planted mistakes (rounding instead of flooring, no wrap of negative phases,
no clamp below a whole turn, a half-bin shift) each fail a pin.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
import oracle.slm as S

mpmath.mp.dps = 60
TWO_PI = 2 * mpmath.pi


def exact_bin(phi32, L):
    """(bin, distance of L*frac to the nearest bin edge) in exact arithmetic."""
    x = mpmath.mpf(float(phi32)) / TWO_PI
    f = x - mpmath.floor(x)
    y = f * L
    k = int(mpmath.floor(y))
    return k % L, float(min(y - mpmath.floor(y), mpmath.ceil(y) - y))


def pin_random_phases_exact_bins():
    rng = np.random.default_rng(5)
    for L in (256, 1024, 4096, 7):
        phi = rng.uniform(-40 * math.pi, 40 * math.pi, 3000).astype(np.float32)
        k = S.gray_index(phi, L)
        for p, kk in zip(phi, k):
            kx, dist = exact_bin(p, L)
            t = abs(float(p)) / (2 * math.pi)
            tol = 4 * L * max(t, 1.0) * 2.0 ** -24
            if dist > tol:
                assert kk == kx, (L, float(p), kk, kx)
            else:
                assert kk in (kx, (kx - 1) % L, (kx + 1) % L), (L, float(p), kk, kx)


def pin_bin_centres_and_wrap():
    for L in (2, 16, 256, 1000):
        k = np.arange(L)
        for turn in (0, 1, 5, -1, -3):
            centres = (2 * np.pi * ((k + 0.5) / L + turn)).astype(np.float32)
            assert np.array_equal(S.gray_index(centres, L), k), (L, turn)


def pin_range_and_table_lookup():
    L = 256
    phi = np.array([0.0, -0.0, -1e-30, -1e-9, 2 * np.pi, -2 * np.pi, 1e5, -1e5, np.pi, -np.pi],
                   dtype=np.float32)
    k = S.gray_index(phi, L)
    assert np.all((k >= 0) & (k < L))
    table = (np.arange(L, dtype=np.uint16) * 7 + 3) % 251
    assert np.array_equal(S.gray_levels(phi, table), table[k])
    assert S.gray_levels(phi, table).dtype == np.uint16
    # just below a whole turn: the last bin, never L
    below = np.nextafter(np.float32(2 * np.pi), np.float32(0))
    assert S.gray_index(np.array([below], dtype=np.float32), L)[0] == L - 1
    assert S.gray_index(np.array([-1e-9], dtype=np.float32), L)[0] == L - 1


PINS = [pin_random_phases_exact_bins, pin_bin_centres_and_wrap, pin_range_and_table_lookup]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


def _mut_round(Phi, levels):
    phi = np.asarray(Phi, dtype=np.float32)
    t = phi * S.INV_TWO_PI_F32
    t = t - np.floor(t)
    return np.minimum(np.rint(t * np.float32(levels)).astype(np.int64), levels - 1)


def _mut_no_wrap(Phi, levels):
    phi = np.asarray(Phi, dtype=np.float32)
    t = np.abs(phi * S.INV_TWO_PI_F32)
    t = t - np.floor(t)
    return np.minimum(np.floor(t * np.float32(levels)).astype(np.int64), levels - 1)


def _mut_no_clamp(Phi, levels):
    phi = np.asarray(Phi, dtype=np.float32)
    t = phi * S.INV_TWO_PI_F32
    t = t - np.floor(t)
    return np.floor(t * np.float32(levels)).astype(np.int64) % levels


def _mut_half_bin(Phi, levels):
    phi = np.asarray(Phi, dtype=np.float32) + np.float32(np.pi / levels)
    t = phi * S.INV_TWO_PI_F32
    t = t - np.floor(t)
    return np.minimum(np.floor(t * np.float32(levels)).astype(np.int64), levels - 1)


MUTANTS = {"round": _mut_round, "no_wrap": _mut_no_wrap, "no_clamp": _mut_no_clamp,
           "half_bin": _mut_half_bin}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    monkeypatch.setattr(S, "gray_index", MUTANTS[name])
    caught = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, name


def test_exports():
    assert oracle.gray_index is S.gray_index or callable(oracle.gray_index)
