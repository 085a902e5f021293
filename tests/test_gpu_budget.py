"""Fixed-work comparison of RS, WGS and CS-WGS on the scenario stand-ins
(paper, results section), on the GPU through the C ABI.

* Parity: scenario holograms at the budget's iteration counts against the
  FP64 oracle on a 256 x 256 grid under a pupil: final e and u within 1e-3.
* The paper's comparison, at 1152 x 1152 under its pupil (6 mm waist, round
  1152-pixel aperture), 10 orientations and theta^0 per scenario, every
  algorithm at the largest iteration count within 432 |Omega| (pixel, spot)
  terms (WGS: one iteration at N = 100, five at N = 36):
  - for both grids, CS-WGS at every compression 2^-1 .. 2^-8 beats WGS in
    mean efficiency and in mean uniformity;
  - for the two cubes, every compression beats WGS in mean efficiency and
    the best compression beats it in mean uniformity;
  - WGS run to 100 iterations (no budget) has the highest mean uniformity.
Each case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import paper_2003_05293_amd as hg
from paper_2003_05293_amd import budget
from workload import Grid, Optics, PUPIL_OPTICS, scenario

pytestmark = pytest.mark.gpu

EU_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hg.load()
    yield
    torch.cuda.synchronize()


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("name,alg,c", [("grid100", "wgs", None), ("grid100", "cswgs", 1 / 16),
                                        ("grid36", "cswgs", 1 / 4), ("cubes", "cswgs", 1 / 32)])
def test_scenario_runs_vs_oracle(name, alg, c):
    g = Grid(256, 256)
    opt = Optics(waist_mm=1.0, aperture_px=256.0)
    s = scenario(name, 2, g, opt)
    M = oracle.pupil_pixels(g, opt).shape[0]
    I = budget.iterations_for_budget(alg, M, s.n, c)
    if alg == "wgs":
        phi_o = oracle.wgs(g, opt, s, I, 2)
    else:
        phi_o = oracle.cswgs(g, opt, s, I, c, 2)
    eo, uo, _ = oracle.metrics(g, opt, s, phi_o)
    say("scenario parity", name, alg, c, "I", I)
    phi = hg.wgs(g, opt, s, I, 2) if alg == "wgs" else hg.cswgs(g, opt, s, I, c, 2)
    e, u, _ = hg.metrics(g, opt, s, phi)
    print(name, alg, c, I, "e", e, eo, "u", u, uo)
    assert abs(e - eo) <= EU_TOL and abs(u - uo) <= EU_TOL


@pytest.fixture(scope="module")
def sweep_results():
    say("budget sweep 1152x1152 pupil, 3 scenarios x 11 algorithms x 10 repeats")
    return budget.sweep(Grid(1152, 1152), PUPIL_OPTICS, ("grid100", "grid36", "cubes"),
                        repeats=10)


def _split(rows):
    by = {(r["algorithm"], r["compression"]): r for r in rows}
    wgs = by[("wgs", None)]
    cs = [by[("cswgs", c)] for c in budget.COMPRESSIONS]
    return by, wgs, cs


@pytest.mark.parametrize("name", ["grid100", "grid36"])
def test_cswgs_beats_wgs_on_grids(sweep_results, name):
    by, wgs, cs = _split(sweep_results[name])
    for r in cs:
        print(name, r["compression"], r["iterations"], r["e"]["mean"], r["u"]["mean"],
              "WGS", wgs["iterations"], wgs["e"]["mean"], wgs["u"]["mean"])
        assert r["e"]["mean"] > wgs["e"]["mean"]
        assert r["u"]["mean"] > wgs["u"]["mean"]


def test_cswgs_on_cubes(sweep_results):
    by, wgs, cs = _split(sweep_results["cubes"])
    for r in cs:
        assert r["e"]["mean"] > wgs["e"]["mean"]
    assert max(r["u"]["mean"] for r in cs) > wgs["u"]["mean"]


@pytest.mark.parametrize("name", ["grid100", "grid36", "cubes"])
def test_converged_wgs_is_the_uniformity_ceiling(sweep_results, name):
    by, wgs, cs = _split(sweep_results[name])
    conv = by[("wgs_converged", None)]
    assert conv["u"]["mean"] >= max(r["u"]["mean"] for r in cs + [wgs, by[("rs", None)]])


def test_budget_iterations_as_planned(sweep_results):
    rows = {r["algorithm"] + str(r["compression"]): r for r in sweep_results["grid100"]}
    assert rows["wgsNone"]["iterations"] == 1
    assert rows["cswgs0.0625"]["iterations"] == 11
    rows = {r["algorithm"] + str(r["compression"]): r for r in sweep_results["grid36"]}
    assert rows["wgsNone"]["iterations"] == 5
    for name in ("grid100", "grid36", "cubes"):
        for r in sweep_results[name]:
            if r["algorithm"] != "wgs_converged":
                assert r["terms_per_pixel"] <= budget.BUDGET_TERMS_PER_PIXEL
