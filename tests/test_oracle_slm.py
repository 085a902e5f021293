"""Pins of the oracle's phase-to-gray lookup (oracle/slm.py) against exact
arithmetic on the table's bins, independently of its own steps:

* bin k holds the phases with k/L <= frac(Phi / 2 pi) < (k+1)/L: checked
  with 2 pi to 60 digits (mpmath) on random FP32 phases over many turns, both
  signs, and on adversarial phases (every bin edge of a 256-level table and
  its FP32 neighbours): the oracle's bin is the exact bin everywhere, and its
  distance to the nearest edge is the exact distance;
* bin centres of every bin, in the first turn, in later turns and at
  negative phases (wrap), map to that bin;
* the index is always in [0, L) and the gray level is the table entry;
* the FP32 edge tolerance covers the rounding of an FP32 bin decision
  (emulated here with numpy float32 steps): outside it, FP32 finds the exact
  bin.
Planted mistakes (rounding instead of flooring, no wrap of negative phases,
a half-bin shift, a period of pi) each fail a pin.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
import oracle.slm as S

def exact_bin(phi, L):
    """(bin, distance of L*frac to the nearest bin edge) at 60 digits."""
    with mpmath.workdps(60):
        x = mpmath.mpf(float(phi)) / (2 * mpmath.pi)
        f = x - mpmath.floor(x)
        y = f * L
        k = int(mpmath.floor(y))
        return k % L, float(min(y - mpmath.floor(y), mpmath.ceil(y) - y))


def adversarial(L):
    edges = 2 * np.pi * (np.arange(-3 * L, 3 * L) / float(L))
    e32 = edges.astype(np.float32)
    return np.concatenate([e32, np.nextafter(e32, np.float32(np.inf)),
                           np.nextafter(e32, np.float32(-np.inf))])


def pin_random_phases_exact_bins():
    rng = np.random.default_rng(5)
    for L in (256, 1024, 4096, 7):
        phi = rng.uniform(-40 * math.pi, 40 * math.pi, 1500).astype(np.float32)
        k, d = S.gray_bin(phi, L)
        for p, kk, dd in zip(phi, k, d):
            kx, dx = exact_bin(p, L)
            assert kk == kx, (L, float(p), kk, kx)
            assert abs(dd - dx) < 1e-9, (L, float(p), dd, dx)


def pin_edges_exact_bins():
    for L in (256, 6):
        phi = adversarial(L)
        k, d = S.gray_bin(phi, L)
        for p, kk, dd in zip(phi, k, d):
            kx, dx = exact_bin(p, L)
            assert kk == kx, (L, float(p), kk, kx)
            assert abs(dd - dx) < 1e-12, (L, float(p), dd, dx)


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
    assert S.gray_index(np.array([0.0], dtype=np.float32), L)[0] == 0
    # one level: every phase in bin 0
    assert np.all(S.gray_index(phi, 1) == 0)


def _fp32_bin(phi, L):
    """An FP32 bin decision: t = fl(Phi fl(1/2pi)), t = fl(t - floor t),
    k = min(floor(fl(t L)), L - 1)."""
    phi = np.asarray(phi, dtype=np.float32)
    t = phi * np.float32(1.0 / (2.0 * np.pi))
    t = (t - np.floor(t)).astype(np.float32)
    return np.minimum(np.floor(t * np.float32(L)).astype(np.int64), L - 1)


def pin_fp32_tolerance_covers_fp32_rounding():
    rng = np.random.default_rng(9)
    for L in (256, 4096, 65536):
        adv = adversarial(256)
        phi = np.concatenate([adv, rng.uniform(-200, 200, 20000).astype(np.float32)])
        k, d = S.gray_bin(phi, L)
        k32 = _fp32_bin(phi, L)
        tol = S.fp32_edge_tolerance(phi, L)
        far = d > tol
        assert np.array_equal(k32[far], k[far]), L
        near = ~far
        assert np.all((k32[near] == k[near]) | (k32[near] == (k[near] + 1) % L)
                      | (k32[near] == (k[near] - 1) % L)), L
        # on random phases the tolerance stays a small part of a bin where
        # FP32 resolves the bins (65536 bins over 30 turns it does not)
        if L <= 4096:
            frac = near[adv.shape[0]:].mean()
            assert frac < 0.05, (L, frac)


PINS = [pin_random_phases_exact_bins, pin_edges_exact_bins, pin_bin_centres_and_wrap,
        pin_range_and_table_lookup, pin_fp32_tolerance_covers_fp32_rounding]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


def _mut_round(Phi, levels):
    t = np.asarray(Phi, dtype=np.float64) / (2 * np.pi)
    y = (t - np.floor(t)) * levels
    return np.rint(y).astype(np.int64) % levels, np.abs(y - np.rint(y))


def _mut_no_wrap(Phi, levels):
    t = np.abs(np.asarray(Phi, dtype=np.float64)) / (2 * np.pi)
    y = (t - np.floor(t)) * levels
    return np.floor(y).astype(np.int64) % levels, np.minimum(y - np.floor(y), np.ceil(y) - y)


def _mut_half_bin(Phi, levels):
    t = (np.asarray(Phi, dtype=np.float64) + np.pi / levels) / (2 * np.pi)
    y = (t - np.floor(t)) * levels
    return np.floor(y).astype(np.int64) % levels, np.minimum(y - np.floor(y), np.ceil(y) - y)


def _mut_period_pi(Phi, levels):
    t = np.asarray(Phi, dtype=np.float64) / np.pi
    y = (t - np.floor(t)) * levels
    return np.floor(y).astype(np.int64) % levels, np.minimum(y - np.floor(y), np.ceil(y) - y)


MUTANTS = {"round": _mut_round, "no_wrap": _mut_no_wrap, "half_bin": _mut_half_bin,
           "period_pi": _mut_period_pi}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    monkeypatch.setattr(S, "gray_bin", MUTANTS[name])
    caught = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, name


def test_exports():
    assert oracle.gray_index is S.gray_index
    assert oracle.gray_bin is S.gray_bin
