"""Seeded spot clouds and request streams for the hologram workloads.

The paper's own spot patterns (two rotating grids and two cubes, in its
results section) are described in words only, with no coordinates, so every
workload here is a synthetic stand-in: spots drawn uniformly in a box that
fills 0.4 of the addressable lateral field and a thin axial slab.

Optics for every workload: pixel pitch 9.2 um (the paper's SLM, experimental
setup section), wavelength 0.488 um, focal length 20 mm.  The addressable
lateral half-field of a pixelated SLM is lambda*f/(2*pitch) (Nyquist); spots
are kept within 0.4 of it.

Everything is drawn with numpy's PCG64 generator so that the same seed gives
the same cloud on every machine.  The draw order is fixed: x, then y, then z.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

PITCH_MM = 9.2e-3


@dataclasses.dataclass(frozen=True)
class Grid:
    """SLM pixel grid: W columns (x'), H rows (y'), square pixels of pitch_mm."""
    W: int
    H: int
    pitch_mm: float = PITCH_MM

    @property
    def M(self) -> int:
        return self.W * self.H


@dataclasses.dataclass(frozen=True)
class Optics:
    """Wavelength and focal length of the Fourier lens, both in mm, and the
    pupil on the SLM: the waist radius of a Gaussian illumination beam in mm
    (0: uniform illumination) and the diameter of a round aperture centred on
    the grid, in pixels (0: the whole rectangle)."""
    lambda_mm: float = 0.488e-3
    focal_mm: float = 20.0
    waist_mm: float = 0.0
    aperture_px: float = 0.0


OPTICS = Optics()
# The paper's pupil (experimental setup section): a laser expanded to a beam
# waist radius of 6 mm at the SLM panel, and the round aperture of the
# optical system, 1152 pixels across (the short side of the panel).
PUPIL_OPTICS = Optics(waist_mm=6.0, aperture_px=1152.0)


@dataclasses.dataclass
class Spots:
    """N target spots: coordinates in mm in the focal volume and the target
    amplitudes a_n^0 (the paper's relative intensities are |a_n^0|^2)."""
    x_mm: np.ndarray
    y_mm: np.ndarray
    z_mm: np.ndarray
    amp: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x_mm.shape[0])

    def __post_init__(self):
        for name in ("x_mm", "y_mm", "z_mm", "amp"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name), dtype=np.float64))


def lateral_half_range_mm(grid: Grid, optics: Optics = OPTICS, fill: float = 0.4) -> float:
    """Half-width of the lateral spot box: fill * lambda*f / (2*pitch)."""
    return fill * optics.lambda_mm * optics.focal_mm / (2.0 * grid.pitch_mm)


def spot_cloud(seed: int, n: int, grid: Grid, optics: Optics = OPTICS,
               z_half_mm: float = 0.05, fill: float = 0.4) -> Spots:
    """n spots uniform in [-r, r]^2 x [-z_half, z_half] with equal amplitudes
    1/sqrt(n), drawn from PCG64(seed) in the order x, y, z."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    r = lateral_half_range_mm(grid, optics, fill)
    x = rng.uniform(-r, r, n)
    y = rng.uniform(-r, r, n)
    z = rng.uniform(-z_half_mm, z_half_mm, n)
    amp = np.full(n, 1.0 / math.sqrt(n))
    return Spots(x, y, z, amp)


# Sizes of the mixed batch: the three square SLM sub-apertures and the full
# 1920 x 1152 panel of the paper's SLM.
BATCH_SIZES = ((512, 512), (1024, 1024), (1152, 1152), (1920, 1152))


@dataclasses.dataclass
class Job:
    grid: Grid
    spots: Spots
    iterations: int
    compression: float
    seed: int


def mixed_batch(seed: int, count: int = 64, iterations: int = 30,
                compression: float = 1.0 / 16, n_range=(8, 200),
                sizes=BATCH_SIZES, z_half_mm: float = 0.1) -> List[Job]:
    """count independent holograms with sizes drawn uniformly from `sizes`,
    N uniform in the closed range n_range, z within +-z_half_mm.  Each job
    gets its own cloud seed and algorithm seed derived from `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for k in range(count):
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        job_seed = int(rng.integers(0, 2**63))
        g = Grid(W, H)
        jobs.append(Job(g, spot_cloud(job_seed, n, g, z_half_mm=z_half_mm),
                        iterations, compression, job_seed))
    return jobs


@dataclasses.dataclass
class Request:
    arrival_s: float
    job: Job


def poisson_stream(seed: int, rate_hz: float = 60.0, duration_s: float = 30.0,
                   iterations: int = 20, compression: float = 1.0 / 16,
                   n_range=(10, 150), sizes=((1152, 1152), (1920, 1152)),
                   z_half_mm: float = 0.05) -> List[Request]:
    """Poisson arrivals (exponential gaps of mean 1/rate_hz) over duration_s,
    each a fresh random spot cloud."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        job_seed = int(rng.integers(0, 2**63))
        g = Grid(W, H)
        out.append(Request(t, Job(g, spot_cloud(job_seed, n, g, z_half_mm=z_half_mm),
                                  iterations, compression, job_seed)))
    return out


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    grid: Grid
    n: int
    iterations: int
    compression: float
    z_half_mm: float = 0.05


WORKLOADS = {
    # RS + plain WGS, small enough for the FP64 oracle to run in seconds.
    "wgs_256x256_n16_i20": Workload("wgs_256x256_n16_i20", Grid(256, 256), 16, 20, 1.0),
    # The headline case: 1152 x 1152 SLM (the paper's round aperture is
    # 1152 px across), 100 spots, 30 iterations, 1/16 of the pixels per
    # compressed iteration.
    "cswgs_1152x1152_n100_i30_c16": Workload("cswgs_1152x1152_n100_i30_c16",
                                             Grid(1152, 1152), 100, 30, 1.0 / 16),
}
# The headline case under the paper's pupil (PUPIL_OPTICS): Gaussian
# illumination on the round 1152-pixel aperture.
PUPIL_WORKLOAD = "cswgs_1152x1152_n100_i30_c16_pupil"
