"""Pins of the oracle's pupil (illumination amplitude and round aperture,
oracle/hg.py: pupil_pixels, illumination, forward, metrics, the schedule)
against what the geometry and the mathematics fix, independently of the
oracle's own code:

* the aperture, by exact rational arithmetic on the pixel centres (half-pixel
  offsets, not the oracle's doubled integers), on odd, even and mixed grids;
* the aperture count of the paper's 1152-pixel disk against pi D^2 / 4
  within the Gauss circle bound;
* the Gaussian amplitude at pixels of known radius (scalar math.exp);
* eq. (3) with the pupil by scalar brute force (cmath loops) on a tiny grid;
* eq. (3) with the pupil against numpy.fft.fft2 for spots on the DFT lattice;
* one spot under the pupil: stationary, and e = mean(A)^2 / mean(A^2) from an
  independent loop over the disk;
* the pupil defaults (no waist, no aperture) reduce every observable to the
  uniform rectangle bit for bit;
* CS-WGS subsets lie in the aperture and consecutive windows partition it.

A mutation test plants plausible pupil mistakes in the oracle (on the CPU)
and checks that at least one of these pins catches each.
"""
import cmath
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import oracle.hg as H
import oracle.sampler as S
from workload import Grid, Optics, OPTICS, Spots, spot_cloud


def inside_exact(W, Hh, D):
    """Pixel indices whose centre is within D/2 pixels of the grid centre,
    by exact rational arithmetic on half-pixel offsets."""
    out = []
    r2 = Fraction(D) ** 2 / 4
    for j in range(Hh):
        dy = Fraction(2 * j - (Hh - 1), 2)
        for i in range(W):
            dx = Fraction(2 * i - (W - 1), 2)
            if dx * dx + dy * dy <= r2:
                out.append(j * W + i)
    return np.array(out, dtype=np.int64)


def pin_aperture_exact():
    for W, Hh in ((37, 29), (36, 28), (37, 28), (16, 41)):
        for D in (0.0, 9.0, 25.0, 25.5, 29.0, 60.0):
            got = H.pupil_pixels(Grid(W, Hh), Optics(aperture_px=D))
            want = np.arange(W * Hh) if D == 0.0 else inside_exact(W, Hh, Fraction(D))
            assert np.array_equal(got, want), (W, Hh, D)


def pin_aperture_area():
    D = 1152
    n = H.pupil_pixels(Grid(1152, 1152), Optics(aperture_px=D)).shape[0]
    assert abs(n - math.pi * D * D / 4) < 2 * D


def pin_illumination_radius():
    g = Grid(101, 101)
    w = 0.2
    o = Optics(waist_mm=w)
    c = 50  # centre pixel of the odd grid
    for k in (0, 1, 7, 30, 50):
        p = np.array([c * g.W + c + k, (c + k) * g.W + c], dtype=np.int64)
        r = k * g.pitch_mm
        want = math.exp(-(r * r) / (w * w))
        assert np.abs(H.illumination(g, o, p) - want).max() < 1e-15
    assert np.array_equal(H.illumination(g, OPTICS, np.arange(g.M)), np.ones(g.M))


def _phase_scalar(g, o, s, p, n):
    i, j = p % g.W, p // g.W
    xp = (i - (g.W - 1) / 2) * g.pitch_mm
    yp = (j - (g.H - 1) / 2) * g.pitch_mm
    lf = o.lambda_mm * o.focal_mm
    return (2 * math.pi / lf) * (xp * s.x_mm[n] + yp * s.y_mm[n]) + \
        (2 * math.pi / (lf * o.focal_mm)) * (xp * xp + yp * yp) * s.z_mm[n]


def pin_forward_bruteforce_pupil():
    g = Grid(9, 7)
    o = Optics(waist_mm=0.02, aperture_px=6.5)
    s = spot_cloud(4, 3, g, z_half_mm=0.2)
    rng = np.random.default_rng(5)
    Phi = rng.uniform(-math.pi, math.pi, g.M)
    inside = inside_exact(g.W, g.H, Fraction(13, 2))
    V = H.forward(g, o, s, Phi[inside], inside)
    for n in range(s.n):
        acc = 0j
        for p in inside:
            i, j = p % g.W, p // g.W
            r2 = (((i - (g.W - 1) / 2) ** 2 + (j - (g.H - 1) / 2) ** 2)) * g.pitch_mm ** 2
            A = math.exp(-r2 / o.waist_mm ** 2)
            acc += A * cmath.exp(1j * (Phi[p] - _phase_scalar(g, o, s, int(p), n)))
        assert abs(V[n] - acc / len(inside)) < 1e-13
    # the default set is the aperture
    assert np.array_equal(H.forward(g, o, s, Phi[inside]), V)


def lattice_spots(grid, optics, kxs, kys):
    kxs = np.asarray(kxs, dtype=np.float64)
    kys = np.asarray(kys, dtype=np.float64)
    x = kxs * optics.lambda_mm * optics.focal_mm / (grid.W * grid.pitch_mm)
    y = kys * optics.lambda_mm * optics.focal_mm / (grid.H * grid.pitch_mm)
    n = kxs.size
    return Spots(x, y, np.zeros(n), np.full(n, 1 / math.sqrt(n)))


def pin_forward_fft_pupil():
    g = Grid(48, 40)
    o = Optics(waist_mm=0.12, aperture_px=37.0)
    kx = np.array([3, -7, 11, 0, -20])
    ky = np.array([-5, 2, 0, 9, 19])
    s = lattice_spots(g, o, kx, ky)
    rng = np.random.default_rng(7)
    Phi = rng.uniform(-math.pi, math.pi, g.M)
    inside = inside_exact(g.W, g.H, Fraction(37))
    mask = np.zeros(g.M)
    mask[inside] = 1.0
    cx, cy = (g.W - 1) / 2.0, (g.H - 1) / 2.0
    ii, jj = np.meshgrid(np.arange(g.W) - cx, np.arange(g.H) - cy)
    A = np.exp(-((ii ** 2 + jj ** 2) * g.pitch_mm ** 2) / o.waist_mm ** 2)
    f = (mask.reshape(g.H, g.W) * A) * np.exp(1j * Phi).reshape(g.H, g.W)
    F = np.fft.fft2(f) / inside.shape[0]
    want = F[ky % g.H, kx % g.W] * np.exp(2j * math.pi * (kx * cx / g.W + ky * cy / g.H))
    V = H.forward(g, o, s, Phi[inside], inside)
    assert np.abs(V - want).max() < 1e-12


def pin_single_spot_pupil():
    g = Grid(48, 40)
    o = Optics(waist_mm=0.15, aperture_px=36.0)
    s = spot_cloud(6, 1, g)
    tr = oracle.Trace()
    Phi = oracle.cswgs(g, o, s, 4, 0.5, 77, tr)
    th0 = oracle.theta0(77, 1)
    inside = inside_exact(g.W, g.H, Fraction(36))
    # mean and mean square of A over the disk, by a scalar loop
    a1 = a2 = 0.0
    for p in inside:
        i, j = p % g.W, p // g.W
        r2 = (((i - (g.W - 1) / 2) ** 2 + (j - (g.H - 1) / 2) ** 2)) * g.pitch_mm ** 2
        A = math.exp(-r2 / o.waist_mm ** 2)
        a1 += A
        a2 += A * A
    a1 /= len(inside)
    a2 /= len(inside)
    for V, w, th in zip(tr.V, tr.w, tr.theta):
        assert abs(w[0] - 1) < 1e-12
        assert np.abs(np.angle(np.exp(1j * (th - th0)))).max() < 1e-12
    assert abs(abs(tr.V[-1][0]) - a1) < 1e-12  # the last forward runs over the whole disk
    e, u, _ = oracle.metrics(g, o, s, Phi)
    assert abs(e - a1 * a1 / a2) < 1e-12 and abs(u - 1) < 1e-15


def pin_defaults_are_uniform_rectangle():
    g = Grid(40, 36)
    s = spot_cloud(9, 6, g)
    o = Optics(waist_mm=0.0, aperture_px=0.0)
    a = oracle.cswgs(g, OPTICS, s, 3, 0.25, 5)
    b = oracle.cswgs(g, o, s, 3, 0.25, 5)
    assert np.array_equal(a, b)
    # an aperture covering the whole grid and a very wide beam change nothing
    big = Optics(waist_mm=1e9, aperture_px=1e6)
    c = oracle.cswgs(g, big, s, 3, 0.25, 5)
    assert np.abs(np.angle(np.exp(1j * (c - a)))).max() < 1e-9


def pin_subsets_in_aperture():
    g = Grid(50, 44)
    o = Optics(aperture_px=40.0)
    inside = inside_exact(g.W, g.H, Fraction(40))
    K = inside.shape[0]
    d = next(k for k in range(4, 64) if K % k == 0)  # windows that divide |Omega|
    c = 1.0 / d
    m = S.subset_size(K, c)
    assert m * d == K
    seen = []
    for j in range(1, d + 1):
        sub = inside[S.subset(K, 3, j, c)]
        assert np.isin(sub, inside).all()
        seen.append(sub)
    assert np.array_equal(np.sort(np.concatenate(seen)), inside)
    # the schedule's forward sums use exactly the windows of the SLM's one
    # order (key ORDER_KEY), whatever the hologram's seed
    s = spot_cloud(2, 5, g)
    tr = oracle.Trace()
    oracle.cswgs(g, o, s, 3, c, 3, tr)
    w = np.ones(s.n)
    th = oracle.theta0(3, s.n)
    p1 = inside[S.subset(K, S.ORDER_KEY, 1, c)]
    V1 = H.forward(g, o, s, H.backward(g, o, s, w, th, p1), p1)
    assert np.array_equal(V1, tr.V[0])


PINS = [pin_aperture_exact, pin_aperture_area, pin_illumination_radius,
        pin_forward_bruteforce_pupil, pin_forward_fft_pupil, pin_single_spot_pupil,
        pin_defaults_are_uniform_rectangle, pin_subsets_in_aperture]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


# ------------------------------------------------------- mutation test ---

_orig_illumination = H.illumination
_orig_pupil = H.pupil_pixels
_orig_metrics = H.metrics


def _mut_illumination_intensity(grid, optics, p):
    return _orig_illumination(grid, optics, p) ** 2  # intensity instead of amplitude


def _mut_aperture_radius(grid, optics):
    # the diameter taken as the radius
    o = Optics(optics.lambda_mm, optics.focal_mm, optics.waist_mm, 2 * optics.aperture_px)
    return _orig_pupil(grid, o)


def _mut_aperture_strict(grid, optics):
    # boundary pixels left out
    p = _orig_pupil(grid, optics)
    D = optics.aperture_px
    if D <= 0:
        return p
    Lx = 2 * (p % grid.W) - (grid.W - 1)
    Ly = 2 * (p // grid.W) - (grid.H - 1)
    return p[Lx * Lx + Ly * Ly < D * D]


def _mut_metrics_no_power(grid, optics, spots, Phi):
    pupil = _orig_pupil(grid, optics)
    V = H.forward(grid, optics, spots, np.asarray(Phi)[pupil], pupil)
    I = np.abs(V) ** 2
    return float(I.sum()), float(1 - (I.max() - I.min()) / (I.max() + I.min())), I


def _mut_illumination_in_mm_half(grid, optics, p):
    p = np.asarray(p, dtype=np.int64)
    if optics.waist_mm <= 0:
        return np.ones(p.shape[0])
    xp, yp = H._pixels(grid, p)
    return np.exp(-(xp * xp + yp * yp) / (2 * optics.waist_mm ** 2))  # 1/e^2 intensity misread


MUTANTS = {
    "illumination_intensity": ("illumination", _mut_illumination_intensity),
    "aperture_radius": ("pupil_pixels", _mut_aperture_radius),
    "aperture_strict": ("pupil_pixels", _mut_aperture_strict),
    "metrics_no_power": ("metrics", _mut_metrics_no_power),
    "illumination_sigma": ("illumination", _mut_illumination_in_mm_half),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(H, attr, fn)
    if attr == "metrics":
        monkeypatch.setattr(oracle, "metrics", fn)
    caught = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, IndexError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
