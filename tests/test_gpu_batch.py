"""Batched form: many holograms per launch (one launch per iteration round),
and the reusable batch whose schedule is captured once as a HIP graph.

Bars: every hologram of a batch is bit-identical to the same hologram
computed alone (the launch geometry of a hologram's passes depends only on
that hologram); graph replays are bit-identical to the eager run, replay
after replay, also with eager work between them and after the spot inputs
change; and e, u of a batched hologram match the FP64 oracle within 1e-3.
"""
import json
import os

import numpy as np
import pytest

import oracle
import paper_2003_05293_amd as hg
from workload import Grid, OPTICS, spot_cloud, mixed_batch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available()
    hg.load()
    yield
    torch.cuda.synchronize()


# (W, H, N, I, c, z_half, seed): ragged sizes, N below and above one wave of
# spots, WGS (c = 1), RS (I = 0), one compressed iteration (I = 1)
CASES = [
    (256, 256, 16, 20, 1 / 16, 0.05, 1),
    (300, 170, 37, 8, 0.1, 0.1, 2),
    (512, 512, 200, 10, 1 / 16, 0.1, 3),
    (128, 96, 65, 5, 1.0, 0.05, 4),
    (97, 61, 9, 0, 0.5, 0.05, 5),
    (160, 120, 129, 1, 0.25, 0.05, 6),
    (1152, 1152, 100, 30, 1 / 16, 0.05, 7),
    (64, 48, 1, 6, 0.5, 0.05, 8),
]


def _jobs(cases):
    jobs = []
    for W, H, N, I, c, zh, seed in cases:
        g = Grid(W, H)
        s = spot_cloud(seed, N, g, z_half_mm=zh)
        jobs.append((g, s, I, c, seed))
    return jobs


def _alone(jobs):
    import torch
    out = []
    for g, s, I, c, seed in jobs:
        out.append(hg.cswgs(g, OPTICS, s, I, c, seed).clone())
    torch.cuda.synchronize()
    return out


def test_batch_equals_alone_bitwise():
    import torch
    jobs = _jobs(CASES)
    say("batch of", len(jobs), "vs alone")
    ref = _alone(jobs)
    dj = [hg.DeviceJob.from_spots(g, OPTICS, s, I, c, seed) for g, s, I, c, seed in jobs]
    hg.cswgs_batch(dj)
    torch.cuda.synchronize()
    for k, (j, r) in enumerate(zip(dj, ref)):
        assert torch.equal(j.phi, r), k


def test_batch_order_does_not_matter():
    import torch
    jobs = _jobs(CASES[:5])
    say("batch order")
    a = [hg.DeviceJob.from_spots(g, OPTICS, s, I, c, seed) for g, s, I, c, seed in jobs]
    b = [hg.DeviceJob.from_spots(g, OPTICS, s, I, c, seed) for g, s, I, c, seed in jobs[::-1]]
    hg.cswgs_batch(a)
    hg.cswgs_batch(b)
    torch.cuda.synchronize()
    for x, y in zip(a, b[::-1]):
        assert torch.equal(x.phi, y.phi)


def test_graph_replays_match_eager():
    import torch
    jobs = _jobs(CASES)
    say("graph replay")
    ref = _alone(jobs)
    dj = [hg.DeviceJob.from_spots(g, OPTICS, s, I, c, seed) for g, s, I, c, seed in jobs]
    stream = torch.cuda.Stream()
    batch = hg.Batch(dj, use_graph=True)
    try:
        for rep in range(4):
            for j in dj:
                j.phi.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                batch.run(stream)
            stream.synchronize()
            for k, (j, r) in enumerate(zip(dj, ref)):
                assert torch.equal(j.phi, r), (rep, k)
            # eager work between replays on the default stream
            _ = hg.cswgs(jobs[0][0], OPTICS, jobs[0][1], 3, 0.5, 99)
            torch.cuda.synchronize()
        # new spot values in the same buffers: the next replay computes them
        g, s, I, c, seed = jobs[0]
        s2 = spot_cloud(1234, s.n, g)
        new = torch.tensor(np.stack([s2.x_mm, s2.y_mm, s2.z_mm, s2.amp]), dtype=torch.float64,
                           device="cuda")
        dj[0].spots_dev.copy_(new)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            batch.run(stream)
        stream.synchronize()
        want = hg.cswgs(g, OPTICS, s2, I, c, seed)
        torch.cuda.synchronize()
        assert torch.equal(dj[0].phi, want)
        for k in range(1, len(dj)):
            assert torch.equal(dj[k].phi, ref[k])
    finally:
        batch.close()


def test_mixed_batch_against_stored_oracle():
    """A mixed batch (sizes from the paper's SLM, N from 8 to 200) that
    contains the stored full-size 1920 x 1152 case; its e, u must match the
    oracle's within 1e-3."""
    import torch
    path = os.path.join(GOLDEN, "cswgs_1920x1152_n150_i20_c16_seed3.json")
    gd = json.load(open(path))
    g = Grid(gd["W"], gd["H"])
    s = spot_cloud(gd["seed"], gd["n"], g, z_half_mm=gd["z_half_mm"])
    others = mixed_batch(5, count=11, iterations=20)
    say("mixed batch with the 1920x1152 stored case")
    dj = [hg.DeviceJob.from_spots(j.grid, OPTICS, j.spots, j.iterations, j.compression, j.seed)
          for j in others]
    target = hg.DeviceJob.from_spots(g, OPTICS, s, gd["iterations"], gd["compression"],
                                     gd["seed"])
    dj.insert(6, target)
    hg.cswgs_batch(dj)
    torch.cuda.synchronize()
    e, u, _ = hg.metrics(g, OPTICS, s, target.phi)
    print("batched 1920x1152: e", e, gd["e"], "u", u, gd["u"])
    assert abs(e - gd["e"]) <= 1e-3 and abs(u - gd["u"]) <= 1e-3
    # and the small members against the oracle directly
    for j, d in zip(others[:6], dj[:6]):
        if j.grid.M > 300_000:
            continue
        eo, uo, _ = oracle.metrics(j.grid, OPTICS, j.spots,
                                   oracle.cswgs(j.grid, OPTICS, j.spots, j.iterations,
                                                j.compression, j.seed))
        eg, ug, _ = hg.metrics(j.grid, OPTICS, j.spots, d.phi)
        assert abs(eg - eo) <= 1e-3 and abs(ug - uo) <= 1e-3


def test_launch_geometry_does_not_change_results():
    """Partial sums are kept per tile of pixels whichever block computes the
    tile, so the block caps (the autotuner's parameters) leave every result
    bit-identical, also when blocks take several tiles each."""
    import torch
    g = Grid(1152, 1152)
    s = spot_cloud(3, 100, g)
    say("geometry invariance 1152 N=100")
    ref = hg.cswgs(g, OPTICS, s, 10, 1 / 16, 3).clone()
    for cap in (1, 64, 300, 1024, 4096):
        out = hg.cswgs(g, OPTICS, s, 10, 1 / 16, 3,
                       tune={"subset_block_cap": cap, "full_block_cap": cap})
        torch.cuda.synchronize()
        assert torch.equal(out, ref), cap
    g2 = Grid(300, 170)
    s2 = spot_cloud(4, 37, g2)
    ref2 = hg.cswgs(g2, OPTICS, s2, 6, 0.25, 4, direct=True).clone()
    for cap in (7, 100, 4096):
        out = hg.cswgs(g2, OPTICS, s2, 6, 0.25, 4, direct=True,
                       tune={"subset_block_cap": cap, "full_block_cap": cap})
        torch.cuda.synchronize()
        assert torch.equal(out, ref2), cap


def test_autotuner_picks_a_measured_candidate(tmp_path):
    from paper_2003_05293_amd import autotune
    g = Grid(512, 512)
    s = spot_cloud(5, 60, g)
    say("autotune 512 N=60")
    table = autotune.Table(str(tmp_path / "tune.json"))
    t = table.single(g, OPTICS, s, 8, 1 / 16, reps=2, subset_caps=(64, 256, 1024))
    entry = table.entries[autotune.single_key(g, 60, 8, 1 / 16, "fp32")]
    assert t["subset_block_cap"] in (64, 256, 1024)
    assert entry["ms"] == min(entry["sweep_ms"].values())
    again = autotune.Table(str(tmp_path / "tune.json"))
    assert again.single(g, OPTICS, s, 8, 1 / 16) == t  # cached, not re-timed


def test_shared_exponential_form_alone_equals_batch():
    import torch
    form = {"full_block_cap": 0, "subset_block_cap": 0, "pass_form": 1}
    jobs = _jobs(CASES[:4])
    say("shared-e batch vs alone")
    alone = [hg.cswgs(g, OPTICS, s, I, c, seed, tune=form).clone() for g, s, I, c, seed in jobs]
    dj = [hg.DeviceJob.from_spots(g, OPTICS, s, I, c, seed) for g, s, I, c, seed in jobs]
    out = hg.cswgs_batch(dj, tune=form)
    torch.cuda.synchronize()
    for k in range(len(jobs)):
        assert torch.equal(out[k], alone[k]), k
