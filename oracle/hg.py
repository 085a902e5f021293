"""RS, WGS and CS-WGS phase-only holograms of 3-D spot clouds, in plain FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Written from the paper (Pozzi & Mapelli, arXiv 2003.05293), section 2:

* eq. (2) lens-and-prism phase of spot n at pixel (x', y'):
      phi_n = 2*pi/(lambda f) (x_n x' + y_n y') + 2*pi/(lambda f^2) (x'^2 + y'^2) z_n
  taken literally, including the factor 2*pi of the defocus term.
* eq. (1) back-propagation: Phi = arg( sum_n a_n e^{i (phi_n + theta_n)} ),
  with a_n = w_n a_n^0 (eq. 5).
* eq. (3) forward projection, read as the mean over the pixel set Omega of
  e^{+i (Phi - phi_n)} with uniform illumination A = 1.  The printed sign is
  e^{-i(...)}; only the + sign makes theta_n = arg E_n (eq. 6) a fixed point
  of eq. (1) (for one spot, Phi = phi_1 + theta_1 is then kept by every
  iteration), so the + sign is used.  A mean instead of a sum divides every
  E_n by the same |Omega|; it cancels in eq. (4) and in arg.
* eqs. (4)-(6) weight update: w_n <- w_n * mean_k |E_k| / |E_n|,
  theta_n <- arg E_n, with w_n = 1 before the first iteration.
* RS: eq. (1) with the random theta^0 and w = 1.
* WGS: RS, then I iterations of forward (all pixels), update, back-prop.
* CS-WGS: as WGS, but the forward sum of iteration j < I runs over the random
  subset Omega^j (oracle/sampler.py); iteration I uses all pixels.  The paper
  lets the phase be computed only on the pixels the next forward step reads,
  except in the last two iterations; this oracle does exactly that: Phi^{j}
  is evaluated on Omega^{j+1} for j <= I-2 and on all pixels for j >= I-1.
* Efficiency e and uniformity u (eq. 7): the spot fields of the final
  hologram over all pixels, V*_n; I_n = |V*_n|^2; e = sum_n I_n (the fraction
  of the SLM power that lands in the spots: with the mean normalisation a
  single spot gets all of it); u = 1 - (max I - min I)/(max I + min I).
* The pupil (experimental setup section: a Gaussian beam of waist radius w
  on the SLM, and the round aperture of the optical system): with a waist,
  eq. (3) weights each pixel by the illumination amplitude
  A(x', y') = exp(-(x'^2 + y'^2) / w^2); with an aperture of diameter D
  pixels, Omega is the set of pixels whose centre lies within D/2 pixels of
  the grid centre, and every pixel set of the method (the full set and the
  random order of CS-WGS) is taken within it.  The phase of eq. (1) is still
  computed on every pixel of the grid.  The efficiency divides by the power
  on the SLM: e = sum_n I_n / mean_Omega(A^2), which is 1 for a single spot
  under uniform illumination and at most 1 in general.

Pixel grid: x'_i = (i - (W-1)/2) * pitch, y'_j = (j - (H-1)/2) * pitch, and
pixel p = j*W + i (row-major [H][W]).

Numbers are numpy float64 / complex128 with libm exp and atan2 (np.angle);
arg(0) is 0.  Pixel sets are processed in fixed chunks only to bound memory.

Pins: tests/test_oracle_hg.py (mpmath brute force of eq. 2, one- and two-spot
closed forms, the theta-shift invariant, an FFT pin of the forward sum,
I=0 == RS, c=1 == WGS, stationarity of a single spot, e=u=1 for one spot,
e and u of eq. 7 on hand-worked intensities and on a sinusoidal phase
grating, whose diffraction orders carry Bessel-function amplitudes).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import sampler

CHUNK = 1 << 15


def pixel_offsets_mm(grid):
    """x'_i for i < W and y'_j for j < H, in mm (centred grid)."""
    xs = (np.arange(grid.W, dtype=np.float64) - (grid.W - 1) / 2.0) * grid.pitch_mm
    ys = (np.arange(grid.H, dtype=np.float64) - (grid.H - 1) / 2.0) * grid.pitch_mm
    return xs, ys


def _pixels(grid, p):
    p = np.asarray(p, dtype=np.int64)
    xs, ys = pixel_offsets_mm(grid)
    return xs[p % grid.W], ys[p // grid.W]


def spot_phase(grid, optics, spots, p) -> np.ndarray:
    """eq. (2): phi_n at the pixels p, shape (len(p), N), radians."""
    xp, yp = _pixels(grid, p)
    lf = optics.lambda_mm * optics.focal_mm
    lf2 = optics.lambda_mm * optics.focal_mm ** 2
    lin = (2.0 * math.pi / lf) * (np.outer(xp, spots.x_mm) + np.outer(yp, spots.y_mm))
    quad = (2.0 * math.pi / lf2) * np.outer(xp * xp + yp * yp, spots.z_mm)
    return lin + quad


def _all(grid):
    return np.arange(grid.M, dtype=np.int64)


def pupil_pixels(grid, optics) -> np.ndarray:
    """Omega: the pixels inside the round aperture, in index order (all
    pixels without an aperture).  With doubled integer offsets
    Lx = 2i - (W-1), Ly = 2j - (H-1) a pixel centre lies within D/2 pixels of
    the grid centre exactly when Lx^2 + Ly^2 <= D^2."""
    D = float(getattr(optics, "aperture_px", 0.0))
    if D <= 0.0:
        return _all(grid)
    Lx = 2 * np.arange(grid.W, dtype=np.int64) - (grid.W - 1)
    Ly = 2 * np.arange(grid.H, dtype=np.int64) - (grid.H - 1)
    inside = (Lx[None, :] ** 2 + Ly[:, None] ** 2) <= D * D
    return np.flatnonzero(inside.ravel()).astype(np.int64)


def illumination(grid, optics, p) -> np.ndarray:
    """Illumination amplitude A at the pixels p: exp(-r^2 / w^2) with r the
    distance of the pixel centre from the grid centre in mm (1 without a
    waist)."""
    p = np.asarray(p, dtype=np.int64)
    w = float(getattr(optics, "waist_mm", 0.0))
    if w <= 0.0:
        return np.ones(p.shape[0])
    xp, yp = _pixels(grid, p)
    return np.exp(-(xp * xp + yp * yp) / (w * w))


def backward(grid, optics, spots, w, theta, p=None) -> np.ndarray:
    """eq. (1): Phi at pixels p (default all), with a_n = w_n a_n^0."""
    p = _all(grid) if p is None else np.asarray(p, dtype=np.int64)
    coef = np.asarray(w, dtype=np.float64) * spots.amp
    th = np.asarray(theta, dtype=np.float64)
    out = np.empty(p.shape[0], dtype=np.float64)
    for s in range(0, p.shape[0], CHUNK):
        phi = spot_phase(grid, optics, spots, p[s:s + CHUNK])
        field = np.exp(1j * (phi + th)) @ coef       # sum over n of eq. (1)
        out[s:s + CHUNK] = np.angle(field)
    return out


def forward(grid, optics, spots, Phi_p, p=None) -> np.ndarray:
    """eq. (3): V_n = mean over p of A(p) e^{i(Phi(p) - phi_n(p))}, complex
    (N,).  p defaults to Omega (pupil_pixels); Phi_p holds Phi at the pixels
    p, in the order of p."""
    p = pupil_pixels(grid, optics) if p is None else np.asarray(p, dtype=np.int64)
    Phi_p = np.asarray(Phi_p, dtype=np.float64)
    assert Phi_p.shape == p.shape
    A = illumination(grid, optics, p)
    V = np.zeros(spots.n, dtype=np.complex128)
    for s in range(0, p.shape[0], CHUNK):
        phi = spot_phase(grid, optics, spots, p[s:s + CHUNK])
        V += (A[s:s + CHUNK, None] * np.exp(1j * (Phi_p[s:s + CHUNK, None] - phi))).sum(axis=0)
    return V / p.shape[0]


def update(w, V):
    """eqs. (4)-(6): new weights and phases from the spot fields V."""
    mag = np.abs(V)
    w_new = np.asarray(w, dtype=np.float64) * (mag.mean() / mag)
    return w_new, np.angle(V)


@dataclasses.dataclass
class Trace:
    """Per-iteration state: V[j-1] is the spot field of iteration j, and
    w[j-1], theta[j-1] the weights and phases it produces."""
    V: List[np.ndarray] = dataclasses.field(default_factory=list)
    w: List[np.ndarray] = dataclasses.field(default_factory=list)
    theta: List[np.ndarray] = dataclasses.field(default_factory=list)


def rs(grid, optics, spots, seed: int) -> np.ndarray:
    """Random superposition: eq. (1) with theta^0 from the seed, w = 1."""
    return backward(grid, optics, spots, np.ones(spots.n), sampler.theta0(seed, spots.n))


def _iterate(grid, optics, spots, iterations: int, seed: int, c: Optional[float],
             trace: Optional[Trace]):
    I = int(iterations)
    pupil = pupil_pixels(grid, optics)
    compressed = c is not None

    def forward_set(j):  # pixel set of the forward sum of iteration j
        if compressed and j < I:  # the SLM's one random order (made at start-up)
            return pupil[sampler.subset(pupil.shape[0], sampler.ORDER_KEY, j, c)]
        return pupil  # Omega

    w = np.ones(spots.n)
    theta = sampler.theta0(seed, spots.n)
    p_next = forward_set(1) if I >= 1 else None
    Phi = backward(grid, optics, spots, w, theta, p_next)       # Phi^0
    for j in range(1, I + 1):
        V = forward(grid, optics, spots, Phi, p_next)            # E^j from Phi^{j-1}
        w, theta = update(w, V)
        if trace is not None:
            trace.V.append(V)
            trace.w.append(w.copy())
            trace.theta.append(theta.copy())
        p_next = forward_set(j + 1) if j < I else None          # None: all pixels
        Phi = backward(grid, optics, spots, w, theta, p_next)   # Phi^j
    return Phi


def wgs(grid, optics, spots, iterations: int, seed: int,
        trace: Optional[Trace] = None) -> np.ndarray:
    """Weighted Gerchberg-Saxton: RS, then `iterations` full iterations."""
    return _iterate(grid, optics, spots, iterations, seed, None, trace)


def cswgs(grid, optics, spots, iterations: int, compression: float, seed: int,
          trace: Optional[Trace] = None) -> np.ndarray:
    """Compressed-sensing WGS with subset fraction `compression` = c."""
    if not (0.0 < compression <= 1.0):
        raise ValueError("compression must be in (0, 1]")
    return _iterate(grid, optics, spots, iterations, seed, compression, trace)


def efficiency(I, power: float = 1.0) -> float:
    """The fraction of the SLM's power that lands in the spots (section 2,
    last paragraph): sum_n I_n over the power on the SLM, mean_Omega(A^2)
    (1 under uniform illumination)."""
    return float(np.sum(np.asarray(I, dtype=np.float64))) / float(power)


def uniformity(I) -> float:
    """eq. (7): u = 1 - (max_n I_n - min_n I_n) / (max_n I_n + min_n I_n),
    with I_n the spot intensities |V*_n|^2."""
    I = np.asarray(I, dtype=np.float64)
    hi, lo = float(I.max()), float(I.min())
    return 1.0 - (hi - lo) / (hi + lo)


def metrics(grid, optics, spots, Phi):
    """Efficiency e, uniformity u (eq. 7) and spot intensities I_n of the
    hologram Phi (all pixels, index order), over Omega."""
    pupil = pupil_pixels(grid, optics)
    V = forward(grid, optics, spots, np.asarray(Phi, dtype=np.float64)[pupil], pupil)
    I = np.abs(V) ** 2
    power = float(np.mean(illumination(grid, optics, pupil) ** 2))
    return efficiency(I, power), uniformity(I), I
