"""Pins of the oracle's seeded draws: theta^0 against numpy's Philox words,
the Feistel permutation by brute force (bijection of [0, M)), the sliding
windows of the compressed iterations (a partition of the pixels when m
divides M) and the spatial uniformity of a subset."""
import math

import numpy as np
import pytest

from oracle import sampler
from oracle.philox import MASK64


def test_theta0_against_numpy_words():
    seed = 1234567
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                          counter=np.full(4, MASK64, dtype=np.uint64))
    raw = bg.random_raw(4 * 50).reshape(50, 4)
    want = 2.0 * math.pi * ((raw[:, 0] >> np.uint64(11)).astype(np.float64) * 2.0**-53)
    got = sampler.theta0(seed, 50)
    assert np.array_equal(got, want)
    assert np.all((got >= 0) & (got < 2 * math.pi))


def test_theta0_uniform():
    th = sampler.theta0(7, 4000) / (2 * math.pi)
    hist = np.histogram(th, bins=20, range=(0, 1))[0]
    chi2 = ((hist - 200.0) ** 2 / 200.0).sum()
    assert chi2 < 19 + 6 * math.sqrt(2 * 19)


@pytest.mark.parametrize("M,h", [(1, 1), (2, 1), (4, 1), (5, 2), (16, 2), (17, 3),
                                 (65536, 8), (1152 * 1152, 11), (1920 * 1152, 11),
                                 (2048 * 2048, 11), (2048 * 2048 + 1, 12)])
def test_half_bits(M, h):
    assert sampler.half_bits(M) == h
    assert 4 ** h >= M and (h == 1 or 4 ** (h - 1) < M)


@pytest.mark.parametrize("M", [1, 2, 3, 7, 1000, 65536, 512 * 512, 1152 * 1152, 1920 * 1152])
def test_permutation_is_bijection(M):
    pi = sampler.permute(np.arange(M), M, seed=11)
    assert pi.min() >= 0 and pi.max() < M
    assert np.array_equal(np.sort(pi), np.arange(M))


def test_feistel_is_bijection_on_full_domain():
    h = 5
    t = sampler.round_tables(3, h)
    x = np.arange(1 << (2 * h), dtype=np.uint64)
    y = sampler.feistel(x, t, h)
    assert np.array_equal(np.sort(y), x)
    assert not np.array_equal(y, x)


def test_permutation_depends_on_seed():
    M = 65536
    a = sampler.permute(np.arange(M), M, 1)
    b = sampler.permute(np.arange(M), M, 2)
    assert (a == b).mean() < 0.01


@pytest.mark.parametrize("M,c,m", [(65536, 1 / 16, 4096), (1152 * 1152, 1 / 16, 82944),
                                   (1920 * 1152, 1 / 16, 138240), (1000, 0.3, 300),
                                   (7, 0.5, 4), (5, 1.0, 5), (3, 1e-9, 1)])
def test_subset_size(M, c, m):
    assert sampler.subset_size(M, c) == m


def test_windows_partition_pixels():
    M = 256 * 256
    c = 1 / 16
    parts = [sampler.subset(M, 5, j, c) for j in range(1, 17)]
    allp = np.concatenate(parts)
    assert np.array_equal(np.sort(allp), np.arange(M))
    # iteration 17 starts the order again
    assert np.array_equal(sampler.subset(M, 5, 17, c), parts[0])


def test_window_wraps_at_M():
    M, c = 1000, 0.3       # m = 300; window 4 covers order positions 900..1199
    pi = sampler.permute(np.arange(M), M, 9)
    w4 = sampler.subset(M, 9, 4, c)
    want = pi[(900 + np.arange(300)) % M]
    assert np.array_equal(w4, want)


def test_subset_spatially_uniform():
    W = H = 1152
    p = sampler.subset(W * H, 3, 1, 1 / 16)
    assert len(np.unique(p)) == p.size
    for counts in (np.bincount(p // W, minlength=H), np.bincount(p % W, minlength=W)):
        exp = p.size / counts.size
        chi2 = ((counts - exp) ** 2 / exp).sum()
        dof = counts.size - 1
        assert chi2 < dof + 6 * math.sqrt(2 * dof)
