"""Pins of the FP64 oracle (oracle/hg.py) against what the paper and the
mathematics fix, independently of the oracle's own code:

* eq. (2) at 50 digits in mpmath from the pixel-grid definition;
* eq. (2) structure: separable in x' and y', odd under reflection through the
  grid centre when z = 0;
* eqs. (1) and (3) by scalar brute force (cmath loops) on a tiny non-square grid;
* eq. (1) closed forms for one spot (Phi = phi_1 + theta_1) and two equal spots;
* eq. (1) invariants: a common shift of theta shifts Phi; a common scale of
  the amplitudes changes nothing;
* eq. (3) against numpy.fft.fft2 for spots on the DFT lattice (z = 0, and with a
  common defocus removed by a chirp);
* eqs. (4)-(6) on a hand-worked example; one spot is stationary with e = u = 1;
* schedule identities: I = 0 is RS, c = 1 is WGS, CS-WGS with I = 1 is WGS;
* efficiency: e <= 1 for distinct lattice spots (Parseval), two equal spots
  give the binary-grating value 8/pi^2, many random spots give pi/4;
* eq. (7) and the efficiency on hand-worked intensities, and on a sinusoidal
  phase grating whose orders carry Bessel-function amplitudes J_m(a)
  (Jacobi-Anger), which fixes unequal intensities in closed form;
* the paper's qualitative claims (RS e,u > 0.2; converged WGS on a regular
  grid e,u > 0.9) as smoke checks.

A mutation test plants plausible mistakes in the oracle (on the CPU) and
checks that at least one pin catches each.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import oracle.hg as H
from workload import Grid, Optics, Spots, OPTICS, spot_cloud

mp = pytest.importorskip("mpmath")


def wrap(a):
    return np.angle(np.exp(1j * np.asarray(a)))


def wrapped_err(a, b):
    return np.abs(wrap(np.asarray(a) - np.asarray(b)))


def lattice_spots(grid, optics, kxs, kys, z=0.0, amp=None):
    """Spots whose lateral phase ramps complete an integer number of turns
    over the grid: x_n = k * lambda f / (W * pitch)."""
    kxs = np.asarray(kxs, dtype=np.float64)
    kys = np.asarray(kys, dtype=np.float64)
    x = kxs * optics.lambda_mm * optics.focal_mm / (grid.W * grid.pitch_mm)
    y = kys * optics.lambda_mm * optics.focal_mm / (grid.H * grid.pitch_mm)
    n = kxs.size
    a = np.full(n, 1 / math.sqrt(n)) if amp is None else np.asarray(amp, dtype=np.float64)
    return Spots(x, y, np.full(n, float(z)), a)


# ---------------------------------------------------------------- pins ----

def pin_phase_mpmath():
    mp.mp.dps = 50
    g = Grid(37, 23)
    s = spot_cloud(4, 5, g, z_half_mm=0.2)
    rng = np.random.default_rng(0)
    p = rng.integers(0, g.M, 40)
    got = H.spot_phase(g, OPTICS, s, p)
    lam, f, pitch = mp.mpf(OPTICS.lambda_mm), mp.mpf(OPTICS.focal_mm), mp.mpf(g.pitch_mm)
    for a, pp in enumerate(p):
        i, j = int(pp) % g.W, int(pp) // g.W
        xp = (i - mp.mpf(g.W - 1) / 2) * pitch
        yp = (j - mp.mpf(g.H - 1) / 2) * pitch
        for n in range(s.n):
            ref = (2 * mp.pi / (lam * f)) * (mp.mpf(s.x_mm[n]) * xp + mp.mpf(s.y_mm[n]) * yp) \
                + (2 * mp.pi / (lam * f * f)) * (xp * xp + yp * yp) * mp.mpf(s.z_mm[n])
            assert abs(float(ref) - got[a, n]) < 1e-12 * max(1.0, abs(float(ref)))


def pin_phase_structure():
    g = Grid(16, 9)
    s = spot_cloud(1, 3, g, z_half_mm=0.3)
    phi = H.spot_phase(g, OPTICS, s, np.arange(g.M)).reshape(g.H, g.W, s.n)
    # separable: phi(i,j) = a(i) + b(j)
    sep = phi - phi[:, :1] - phi[:1, :] + phi[:1, :1]
    assert np.abs(sep).max() < 1e-10
    # the linear part is odd and the quadratic part even under p -> M-1-p
    s0 = Spots(s.x_mm, s.y_mm, np.zeros(s.n), s.amp)
    lin = H.spot_phase(g, OPTICS, s0, np.arange(g.M))
    assert np.abs(lin + lin[::-1]).max() < 1e-10
    quad = phi.reshape(g.M, s.n) - lin
    assert np.abs(quad - quad[::-1]).max() < 1e-10
    # along x the phase grows with x_n, along y with y_n
    d_i = phi[0, 1] - phi[0, 0]
    d_j = phi[1, 0] - phi[0, 0]
    k = 2 * math.pi * g.pitch_mm / (OPTICS.lambda_mm * OPTICS.focal_mm)
    c = 2 * math.pi * g.pitch_mm ** 2 / (OPTICS.lambda_mm * OPTICS.focal_mm ** 2)
    # second differences isolate the defocus curvature: 2 c z_n per pixel^2
    assert np.allclose(phi[0, 2] - 2 * phi[0, 1] + phi[0, 0], 2 * c * s.z_mm, atol=1e-12)
    assert np.allclose(phi[2, 0] - 2 * phi[1, 0] + phi[0, 0], 2 * c * s.z_mm, atol=1e-12)
    # first differences at the centre line give the prism slope k x_n
    i0 = g.W // 2
    slope = phi[0, i0] - phi[0, i0 - 1] - c * s.z_mm * ((i0 - (g.W - 1) / 2) ** 2 - (i0 - 1 - (g.W - 1) / 2) ** 2)
    assert np.allclose(slope, k * s.x_mm, atol=1e-12)
    assert np.all(np.isfinite(d_j))


def _brute_phase(g, opt, s, i, j, n):
    xp = (i - (g.W - 1) / 2.0) * g.pitch_mm
    yp = (j - (g.H - 1) / 2.0) * g.pitch_mm
    return (2 * math.pi / (opt.lambda_mm * opt.focal_mm)) * (s.x_mm[n] * xp + s.y_mm[n] * yp) \
        + (2 * math.pi / (opt.lambda_mm * opt.focal_mm ** 2)) * (xp * xp + yp * yp) * s.z_mm[n]


def pin_bruteforce_tiny():
    g = Grid(5, 4, 0.05)
    s = spot_cloud(2, 3, g, z_half_mm=0.5)
    s.amp[:] = [0.3, 0.5, 0.9]
    w = np.array([1.0, 0.7, 1.3])
    th = np.array([0.1, 2.0, -1.0])
    Phi = H.backward(g, OPTICS, s, w, th)
    V = H.forward(g, OPTICS, s, Phi)
    Vb = [0j] * s.n
    for j in range(g.H):
        for i in range(g.W):
            acc = 0j
            for n in range(s.n):
                acc += w[n] * s.amp[n] * cmath.exp(1j * (_brute_phase(g, OPTICS, s, i, j, n) + th[n]))
            ph = math.atan2(acc.imag, acc.real)
            assert abs(cmath.exp(1j * ph) - cmath.exp(1j * Phi[j * g.W + i])) < 1e-12
            for n in range(s.n):
                Vb[n] += cmath.exp(1j * (ph - _brute_phase(g, OPTICS, s, i, j, n))) / g.M
    assert np.abs(np.array(Vb) - V).max() < 1e-12


def pin_one_spot_closed_form():
    g = Grid(64, 48)
    s = spot_cloud(3, 1, g)
    th = np.array([1.234])
    Phi = H.backward(g, OPTICS, s, [1.0], th)
    phi = H.spot_phase(g, OPTICS, s, np.arange(g.M))[:, 0]
    assert wrapped_err(Phi, phi + th[0]).max() < 1e-12
    V = H.forward(g, OPTICS, s, Phi)
    assert abs(V[0] - cmath.exp(1j * th[0])) < 1e-12


def pin_two_spot_closed_form():
    g = Grid(40, 30)
    s = spot_cloud(8, 2, g, z_half_mm=0.1)
    th = np.array([0.3, 2.9])
    Phi = H.backward(g, OPTICS, s, [1.0, 1.0], th)
    phi = H.spot_phase(g, OPTICS, s, np.arange(g.M))
    A, B = phi[:, 0] + th[0], phi[:, 1] + th[1]
    want = (A + B) / 2 + np.where(np.cos((A - B) / 2) < 0, math.pi, 0.0)
    ok = np.abs(np.cos((A - B) / 2)) > 1e-9
    assert wrapped_err(Phi[ok], want[ok]).max() < 1e-11


def pin_invariants():
    g = Grid(32, 24)
    s = spot_cloud(5, 7, g)
    rng = np.random.default_rng(1)
    w = rng.uniform(0.5, 1.5, s.n)
    th = rng.uniform(0, 2 * math.pi, s.n)
    P = H.backward(g, OPTICS, s, w, th)
    assert wrapped_err(H.backward(g, OPTICS, s, w, th + 0.7), P + 0.7).max() < 1e-11
    assert wrapped_err(H.backward(g, OPTICS, s, 3.5 * w, th), P).max() < 1e-11
    V = H.forward(g, OPTICS, s, P)
    V2 = H.forward(g, OPTICS, s, P + 0.7)
    assert np.abs(V2 - V * cmath.exp(0.7j)).max() < 1e-12


def pin_forward_fft():
    g = Grid(48, 40)
    kx = np.array([3, -7, 11, 0, -20])
    ky = np.array([-5, 2, 0, 9, 19])
    rng = np.random.default_rng(2)
    Phi = rng.uniform(-math.pi, math.pi, g.M)
    U = np.exp(1j * Phi).reshape(g.H, g.W)
    cx, cy = (g.W - 1) / 2.0, (g.H - 1) / 2.0
    for z in (0.0, 0.04):
        s = lattice_spots(g, OPTICS, kx, ky, z=z)
        V = H.forward(g, OPTICS, s, Phi)
        if z:
            # remove the common defocus with a chirp over the pixel radius
            ii, jj = np.meshgrid(np.arange(g.W) - cx, np.arange(g.H) - cy)
            r2 = (ii ** 2 + jj ** 2) * g.pitch_mm ** 2
            Uc = U * np.exp(-1j * 2 * math.pi * z * r2 / (OPTICS.lambda_mm * OPTICS.focal_mm ** 2))
        else:
            Uc = U
        F = np.fft.fft2(Uc) / g.M
        want = F[ky % g.H, kx % g.W] * np.exp(2j * math.pi * (kx * cx / g.W + ky * cy / g.H))
        assert np.abs(V - want).max() < 1e-12


def pin_update():
    w = np.array([1.0, 2.0, 0.5])
    V = np.array([1.0 + 0j, 2j, -3.0])
    w2, th = H.update(w, V)
    mean = (1 + 2 + 3) / 3.0
    assert np.allclose(w2, [1.0 * mean / 1, 2.0 * mean / 2, 0.5 * mean / 3], rtol=0, atol=1e-15)
    assert np.allclose(th, [0.0, math.pi / 2, math.pi], atol=1e-15)


def pin_single_spot_stationary():
    g = Grid(48, 32)
    s = spot_cloud(6, 1, g)
    tr = oracle.Trace()
    Phi = oracle.wgs(g, OPTICS, s, 4, 77, tr)
    th0 = oracle.theta0(77, 1)
    for V, w, th in zip(tr.V, tr.w, tr.theta):
        assert abs(abs(V[0]) - 1) < 1e-12
        assert abs(w[0] - 1) < 1e-12
        assert wrapped_err(th, th0).max() < 1e-12
    e, u, _ = oracle.metrics(g, OPTICS, s, Phi)
    assert abs(e - 1) < 1e-12 and abs(u - 1) < 1e-15


def pin_schedules():
    g = Grid(40, 36)
    s = spot_cloud(9, 6, g)
    assert np.array_equal(oracle.wgs(g, OPTICS, s, 0, 5), oracle.rs(g, OPTICS, s, 5))
    assert np.array_equal(oracle.cswgs(g, OPTICS, s, 0, 0.25, 5), oracle.rs(g, OPTICS, s, 5))
    a = oracle.wgs(g, OPTICS, s, 3, 5)
    b = oracle.cswgs(g, OPTICS, s, 3, 1.0, 5)
    assert wrapped_err(a, b).max() < 1e-10
    c = oracle.cswgs(g, OPTICS, s, 1, 0.1, 5)
    d = oracle.wgs(g, OPTICS, s, 1, 5)
    assert np.array_equal(c, d)
    # a compressed run really uses the subsets
    e = oracle.cswgs(g, OPTICS, s, 3, 0.25, 5)
    assert wrapped_err(a, e).max() > 1e-6


def pin_efficiency():
    g = Grid(64, 64)
    # distinct lattice spots: Parseval bounds the power in them by the total
    s = lattice_spots(g, OPTICS, [3, -9, 14, 0, 22, -17], [1, 5, -12, 20, -3, 8])
    e, u, I = oracle.metrics(g, OPTICS, s, oracle.rs(g, OPTICS, s, 4))
    assert 0 < e <= 1 + 1e-12 and 0 <= u <= 1
    # two equal spots: a binary phase grating, 8/pi^2 in the two orders
    g2 = Grid(256, 64)
    s2 = lattice_spots(g2, OPTICS, [8, -8], [0, 0])
    e2, u2, _ = oracle.metrics(g2, OPTICS, s2, oracle.rs(g2, OPTICS, s2, 1))
    assert abs(e2 - 8 / math.pi ** 2) < 0.01 and u2 > 0.999


def pin_efficiency_many_spots():
    # many spots with random phases: the phase-only field keeps pi/4 of the power
    g = Grid(256, 256)
    s = spot_cloud(12, 120, g)
    e, _, _ = oracle.metrics(g, OPTICS, s, oracle.rs(g, OPTICS, s, 12))
    assert abs(e - math.pi / 4) < 0.02


def pin_metrics_hand_worked():
    """eq. (7) and the efficiency on intensities worked out by hand."""
    assert abs(H.uniformity([1.0, 4.0, 2.0]) - 0.4) < 1e-15       # 1 - 3/5
    assert abs(H.uniformity([1.0, 9.0]) - 0.2) < 1e-15            # 1 - 8/10
    assert abs(H.uniformity([0.25, 0.25, 0.25]) - 1.0) < 1e-15
    assert abs(H.uniformity([0.5, 0.3, 0.1, 0.3]) - (1.0 - 0.4 / 0.6)) < 1e-15
    assert abs(H.efficiency([1.0, 4.0, 2.0]) - 7.0) < 1e-15
    assert abs(H.efficiency([0.1, 0.2, 0.3], power=0.5) - 1.2) < 1e-15


def pin_metrics_bessel_grating():
    """e and u of a hologram with unequal spot intensities known in closed
    form: the sinusoidal phase grating Phi = a cos(2 pi k i / W) diffracts
    into orders m k with amplitudes J_m(a) (Jacobi-Anger expansion), so spots
    on the lattice at orders m = 0..3 have I_m = J_m(a)^2 (aliased orders
    m + 32 q contribute J_32(a) ~ 1e-36)."""
    from scipy.special import jv
    g = Grid(256, 8)
    k = 8
    orders = np.array([0, 1, 2, 3])
    s = lattice_spots(g, OPTICS, orders * k, np.zeros(4), amp=np.full(4, 0.5))
    i = np.arange(g.M) % g.W
    for a in (1.5, 2.0):
        Phi = a * np.cos(2 * math.pi * k * i / g.W)
        e, u, I = oracle.metrics(g, OPTICS, s, Phi)
        want = jv(orders, a) ** 2
        assert np.abs(I - want).max() < 1e-13, (a, I, want)
        assert abs(e - want.sum()) < 1e-13
        u_want = 1.0 - (want.max() - want.min()) / (want.max() + want.min())
        assert abs(u - u_want) < 1e-12, (a, u, u_want)


PINS = [pin_phase_mpmath, pin_phase_structure, pin_bruteforce_tiny, pin_one_spot_closed_form,
        pin_two_spot_closed_form, pin_invariants, pin_forward_fft, pin_update,
        pin_single_spot_stationary, pin_schedules, pin_efficiency, pin_efficiency_many_spots,
        pin_metrics_hand_worked, pin_metrics_bessel_grating]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


# -------------------------------------------------- paper's claims ----

def test_paper_claim_rs_quality():
    """RS holograms have e > 0.2 and u > 0.2 (introduction)."""
    g = Grid(128, 128)
    s = spot_cloud(3, 16, g)
    e, u, _ = oracle.metrics(g, OPTICS, s, oracle.rs(g, OPTICS, s, 3))
    assert e > 0.2 and u > 0.2


def test_paper_claim_converged_wgs_on_grid():
    """Converged WGS gives e > 0.9 and u > 0.9 (introduction); checked on a
    regular 6 x 6 grid of spots like the paper's test scenarios."""
    g = Grid(256, 256)
    k = (np.arange(6) - 2.5) * 12
    KX, KY = np.meshgrid(k, k)
    s = lattice_spots(g, OPTICS, KX.ravel(), KY.ravel())
    e0, u0, _ = oracle.metrics(g, OPTICS, s, oracle.rs(g, OPTICS, s, 3))
    e, u, _ = oracle.metrics(g, OPTICS, s, oracle.wgs(g, OPTICS, s, 50, 3))
    assert e > 0.9 and u > 0.9
    assert e > e0 and u > u0


def test_cswgs_improves_on_rs():
    g = Grid(128, 128)
    s = spot_cloud(21, 24, g)
    _, u0, _ = oracle.metrics(g, OPTICS, s, oracle.rs(g, OPTICS, s, 2))
    _, u1, _ = oracle.metrics(g, OPTICS, s, oracle.cswgs(g, OPTICS, s, 20, 1 / 8, 2))
    assert u1 > u0 and u1 > 0.95


def test_reading_literal_sign_flips_theta():
    """Reading of eq. (3): with the printed sign e^{-i(Phi - phi_n)}, the
    field of a one-spot hologram Phi = phi_1 + theta_1 has arg -theta_1, so
    eq. (6) would flip theta every iteration; with the + sign it is kept."""
    g = Grid(40, 30)
    s = spot_cloud(3, 1, g)
    th = 1.1
    Phi = H.backward(g, OPTICS, s, [1.0], [th])
    phi = H.spot_phase(g, OPTICS, s, np.arange(g.M))[:, 0]
    literal = np.exp(-1j * (Phi - phi)).mean()
    assert abs(np.angle(literal) + th) < 1e-12
    assert abs(np.angle(H.forward(g, OPTICS, s, Phi)[0]) - th) < 1e-12


# ------------------------------------------------------ mutations ----

def _mut_forward_sign(grid, optics, spots, Phi_p, p=None):
    p = np.arange(grid.M) if p is None else np.asarray(p)
    phi = H.spot_phase(grid, optics, spots, p)
    return np.exp(-1j * (np.asarray(Phi_p)[:, None] - phi)).mean(axis=0)


def _mut_pixels_transposed(grid, p):
    p = np.asarray(p, dtype=np.int64)
    xs, ys = H.pixel_offsets_mm(grid)
    xs2 = (np.arange(max(grid.W, grid.H)) - (grid.W - 1) / 2.0) * grid.pitch_mm
    ys2 = (np.arange(max(grid.W, grid.H)) - (grid.H - 1) / 2.0) * grid.pitch_mm
    return xs2[p // grid.W], ys2[p % grid.W]


def _mut_offsets_half_pixel(grid):
    xs = (np.arange(grid.W) - grid.W / 2.0) * grid.pitch_mm
    ys = (np.arange(grid.H) - grid.H / 2.0) * grid.pitch_mm
    return xs, ys


def _mut_no_defocus(grid, optics, spots, p):
    xp, yp = H._pixels(grid, p)
    lf = optics.lambda_mm * optics.focal_mm
    return (2 * math.pi / lf) * (np.outer(xp, spots.x_mm) + np.outer(yp, spots.y_mm))


def _mut_update_inverted(w, V):
    mag = np.abs(V)
    return np.asarray(w) * (mag / mag.mean()), np.angle(V)


def _mut_backward_no_theta(grid, optics, spots, w, theta, p=None):
    return _orig_backward(grid, optics, spots, w, np.zeros_like(np.asarray(theta)), p)


def _mut_backward_amp_squared(grid, optics, spots, w, theta, p=None):
    return _orig_backward(grid, optics, spots, np.asarray(w) ** 2, theta, p)


def _mut_uniformity_over_max(I):
    I = np.asarray(I)
    return 1.0 - (I.max() - I.min()) / I.max()


def _mut_uniformity_of_magnitudes(I):
    A = np.sqrt(np.asarray(I))
    return 1.0 - (A.max() - A.min()) / (A.max() + A.min())


def _mut_uniformity_min_over_max(I):
    I = np.asarray(I)
    return I.min() / I.max()


def _mut_efficiency_mean(I, power=1.0):
    return float(np.mean(I)) / power


def _mut_efficiency_of_magnitudes(I, power=1.0):
    return float(np.sum(np.sqrt(np.asarray(I)))) / power


_orig_backward = H.backward

MUTANTS = {
    "forward_sign": ("forward", _mut_forward_sign),
    "pixels_transposed": ("_pixels", _mut_pixels_transposed),
    "offsets_half_pixel": ("pixel_offsets_mm", _mut_offsets_half_pixel),
    "no_defocus": ("spot_phase", _mut_no_defocus),
    "update_inverted": ("update", _mut_update_inverted),
    "backward_no_theta": ("backward", _mut_backward_no_theta),
    "backward_w_squared": ("backward", _mut_backward_amp_squared),
    "uniformity_over_max": ("uniformity", _mut_uniformity_over_max),
    "uniformity_of_magnitudes": ("uniformity", _mut_uniformity_of_magnitudes),
    "uniformity_min_over_max": ("uniformity", _mut_uniformity_min_over_max),
    "efficiency_mean": ("efficiency", _mut_efficiency_mean),
    "efficiency_of_magnitudes": ("efficiency", _mut_efficiency_of_magnitudes),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(H, attr, fn)
    caught = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, IndexError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
