"""Synthetic stand-ins for the three test scenarios of the paper's results
section, which describes them in words only (no coordinates):

* ``grid100``: a regularly spaced planar grid of 10 x 10 spots rotating in 3-D
  (the worst case for uniformity; the paper's WGS fits one iteration in its
  frame time);
* ``grid36``: the same with 6 x 6 spots (WGS fits five iterations);
* ``cubes``: a less regular 3-D pattern of spots organised in two cubes.

Recipe (every draw from numpy's PCG64(seed), in the order written here):

* a rotation is a uniform random unit quaternion (Shoemake's subgroup
  algorithm: three uniforms u1, u2, u3) turned into a 3 x 3 matrix;
* a grid of n x n spots spans [-h, h]^2 in its own plane with
  h = r / sqrt(2), r the lateral half-range of ``spot_cloud`` (0.4 of the
  Nyquist half-field): a rotated corner stays within r of the optical axis,
  so every spot stays inside the lateral box;
* the two cubes are 3 x 3 x 3 lattices without their centre (26 spots each),
  of edges 0.45 r and 0.35 r, centred at (-0.45 r, -0.1 r, 0) and
  (0.45 r, 0.2 r, 0); each is rotated about its centre by its own rotation
  (first cube first), then every coordinate of every spot (cube order, spot
  order, x y z) moves by U(-0.1, 0.1) lattice spacings;
* the axial coordinate after rotation is scaled by ``z_scale`` = 0.25, which
  keeps |z| within about 0.053 mm, the slab of ``spot_cloud``;
* amplitudes are equal, 1/sqrt(N).

A different seed gives a different orientation, as in the paper's repeats
(which also change theta^0: the seed of the hologram run).
"""
from __future__ import annotations

import math

import numpy as np

from .spots import OPTICS, Grid, Optics, Spots, lateral_half_range_mm

SCENARIOS = ("grid100", "grid36", "cubes")
Z_SCALE = 0.25


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation: a unit quaternion from three uniforms
    (Shoemake), as a 3 x 3 matrix."""
    u1, u2, u3 = rng.uniform(0.0, 1.0, 3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    w, x = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    y, z = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _spots(p: np.ndarray, z_scale: float) -> Spots:
    n = p.shape[0]
    return Spots(p[:, 0], p[:, 1], p[:, 2] * z_scale, np.full(n, 1.0 / math.sqrt(n)))


def rotating_grid(n_side: int, seed: int, grid: Grid, optics: Optics = OPTICS,
                  fill: float = 0.4, z_scale: float = Z_SCALE) -> Spots:
    """n_side x n_side regularly spaced spots in a plane, rotated in 3-D."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = lateral_half_range_mm(grid, optics, fill) / math.sqrt(2.0)
    u = np.linspace(-h, h, n_side) if n_side > 1 else np.zeros(1)
    gx, gy = np.meshgrid(u, u, indexing="xy")
    p = np.stack([gx.ravel(), gy.ravel(), np.zeros(n_side * n_side)], axis=1)
    return _spots(p @ random_rotation(rng).T, z_scale)


def _cube_lattice(edge: float) -> np.ndarray:
    """3 x 3 x 3 lattice of the given edge centred at 0, without its centre."""
    t = np.array([-0.5, 0.0, 0.5]) * edge
    pts = np.array([(a, b, c) for c in t for b in t for a in t])
    return pts[np.any(pts != 0.0, axis=1)]


def two_cubes(seed: int, grid: Grid, optics: Optics = OPTICS, fill: float = 0.4,
              z_scale: float = Z_SCALE) -> Spots:
    """Two rotated, jittered cubic lattices of 26 spots each (52 spots)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = lateral_half_range_mm(grid, optics, fill)
    cubes = ((0.45 * r, np.array([-0.45 * r, -0.1 * r, 0.0])),
             (0.35 * r, np.array([0.45 * r, 0.2 * r, 0.0])))
    rots = [random_rotation(rng) for _ in cubes]
    parts = []
    for (edge, centre), R in zip(cubes, rots):
        parts.append(_cube_lattice(edge) @ R.T + centre)
    jitter = rng.uniform(-0.1, 0.1, (sum(p.shape[0] for p in parts), 3))
    spacing = np.concatenate([np.full(p.shape[0], edge / 2.0) for p, (edge, _) in zip(parts, cubes)])
    p = np.concatenate(parts) + jitter * spacing[:, None]
    return _spots(p, z_scale)


def scenario(name: str, seed: int, grid: Grid, optics: Optics = OPTICS) -> Spots:
    """Spots of one of SCENARIOS for the given seed (orientation)."""
    if name == "grid100":
        return rotating_grid(10, seed, grid, optics)
    if name == "grid36":
        return rotating_grid(6, seed, grid, optics)
    if name == "cubes":
        return two_cubes(seed, grid, optics)
    raise ValueError(f"unknown scenario {name!r}; expected one of {SCENARIOS}")
