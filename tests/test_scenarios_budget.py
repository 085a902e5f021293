"""CPU checks of the scenario stand-ins (workload/scenarios.py) and of the
fixed-work budget rule of the algorithm comparison
(paper_2003_05293_amd/budget.py)."""
import math

import numpy as np
import pytest

from paper_2003_05293_amd import budget as B
from workload import Grid, OPTICS, SCENARIOS, lateral_half_range_mm, random_rotation, scenario
from workload.scenarios import Z_SCALE, _cube_lattice


G = Grid(1152, 1152)
R = lateral_half_range_mm(G, OPTICS)


@pytest.mark.parametrize("seed", [0, 1, 7, 12345])
def test_rotation_is_proper_orthogonal(seed):
    rot = random_rotation(np.random.Generator(np.random.PCG64(seed)))
    assert np.allclose(rot @ rot.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(rot) - 1.0) < 1e-14


def test_rotations_are_uniform_on_average():
    """The mean of a uniform random rotation matrix is 0 (Haar measure)."""
    rng = np.random.Generator(np.random.PCG64(3))
    mean = sum(random_rotation(rng) for _ in range(4000)) / 4000
    assert np.max(np.abs(mean)) < 0.05


@pytest.mark.parametrize("name,n", [("grid100", 100), ("grid36", 36), ("cubes", 52)])
def test_scenario_shape_and_bounds(name, n):
    for seed in range(5):
        s = scenario(name, seed, G)
        assert s.n == n
        assert np.max(np.abs(s.x_mm)) <= R + 1e-12 and np.max(np.abs(s.y_mm)) <= R + 1e-12
        assert np.max(np.abs(s.z_mm)) <= Z_SCALE * R + 1e-12
        assert np.allclose(s.amp, 1 / math.sqrt(n))


@pytest.mark.parametrize("name,side", [("grid100", 10), ("grid36", 6)])
def test_grid_is_a_rotated_regular_lattice(name, side):
    """Undo the axial scale: the spots are a square lattice of spacing
    2h/(side-1), h = r/sqrt(2), in some plane (all pairwise distances are
    lattice distances, and the points are coplanar)."""
    s = scenario(name, 11, G)
    p = np.stack([s.x_mm, s.y_mm, s.z_mm / Z_SCALE], axis=1)
    c = p - p.mean(axis=0)
    sv = np.linalg.svd(c, compute_uv=False)
    assert sv[2] < 1e-12 * sv[0]                      # coplanar
    h = R / math.sqrt(2)
    step = 2 * h / (side - 1)
    d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)) / step
    k = np.rint(d ** 2)
    assert np.allclose(d ** 2, k, atol=1e-9)           # squared distances are integers
    assert math.isclose(d.max(), math.sqrt(2) * (side - 1), rel_tol=1e-12)


def test_cubes_lattice_and_jitter():
    lat = _cube_lattice(1.0)
    assert lat.shape == (26, 3) and not np.any(np.all(lat == 0, axis=1))
    s = scenario("cubes", 4, G)
    p = np.stack([s.x_mm, s.y_mm, s.z_mm / Z_SCALE], axis=1)
    # the two cubes' centroids are where the recipe puts them (jitter is
    # zero-mean and the lattice is symmetric about its centre)
    c1, c2 = p[:26].mean(axis=0), p[26:].mean(axis=0)
    assert np.allclose(c1, [-0.45 * R, -0.1 * R, 0], atol=0.02 * R)
    assert np.allclose(c2, [0.45 * R, 0.2 * R, 0], atol=0.02 * R)


def test_scenarios_are_seeded():
    for name in SCENARIOS:
        a, b, c = scenario(name, 5, G), scenario(name, 5, G), scenario(name, 6, G)
        assert np.array_equal(a.x_mm, b.x_mm) and np.array_equal(a.z_mm, b.z_mm)
        assert not np.array_equal(a.x_mm, c.x_mm)
    with pytest.raises(ValueError):
        scenario("sphere", 0, G)


# ---------------------------------------------------------------- budget ---

def test_budget_reproduces_the_papers_anchors():
    """WGS fits one iteration at N = 100 and five at N = 36 (results
    section), for any pupil size."""
    for M in (65536, 1042224, 1327104):
        assert B.iterations_for_budget("wgs", M, 100) == 1
        assert B.iterations_for_budget("wgs", M, 36) == 5


@pytest.mark.parametrize("M", [51472, 1042224, 1327104])
@pytest.mark.parametrize("N", [36, 52, 100, 144, 150])
def test_budget_iterations_are_the_largest_that_fit(M, N):
    budget = B.BUDGET_TERMS_PER_PIXEL * M
    I = B.iterations_for_budget("wgs", M, N)
    if I > 0:
        assert B.terms("wgs", M, N, I) <= budget
    assert B.terms("wgs", M, N, I + 1) > budget
    for c in B.COMPRESSIONS:
        I = B.iterations_for_budget("cswgs", M, N, c)
        if I > 0:
            assert B.terms("cswgs", M, N, I, c) <= budget
        assert B.terms("cswgs", M, N, I + 1, c) > budget


def test_terms_match_the_schedule():
    """CS-WGS with I iterations: I - 1 compressed iterations of two window
    passes each (forward on Omega^j, back-propagation on the next window),
    plus three full passes; I = 1 is WGS."""
    M, N, c = 1000, 7, 0.25
    m = 250
    assert B.terms("cswgs", M, N, 1, c) == B.terms("wgs", M, N, 1) == 3 * M * N
    assert B.terms("cswgs", M, N, 5, c) == (2 * 4 * m + 3 * M) * N
    assert B.terms("rs", M, N) == M * N
    # the paper's linear estimate 2MN + cMN(I-2) is the same schedule counted
    # once per (pixel, spot) and iteration: both grow by 2 m N per iteration
    assert (B.terms("cswgs", M, N, 9, c) - B.terms("cswgs", M, N, 8, c)) == 2 * m * N
