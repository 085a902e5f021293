"""Deferred weight updates between compressed passes, and the split of a
round's per-pixel passes into a one-unit and a wide launch.

A compressed pass that is followed by another compressed pass of the same
hologram leaves its weight update (eqs. 4-6) to the next pass, whose blocks
apply it at their start.  The update's arithmetic and summation order are
unchanged, so the bars are bit-identity:
- against the chained launch, which hands the updated state over inside one
  launch and defers nothing: I = 3 (one deferring and one pending pass), 4
  and 7; N = 1, 5, 100 and 256 (the largest deferred N);
- the traced spot fields of every iteration, against the chained launch;
- two holograms in a row on one stream (the rotating rows of pass totals
  start each hologram at zero);
- a hologram alone against the same hologram in a batch beside a hologram
  of 300 spots (four spot units per wave): holograms of one unit per wave
  run in their own launch of each round, so they sum in the same order;
  likewise for requests of 5, 100, 256 and 300 spots served together by
  the engine.
Parity of the results with the FP64 oracle is covered by the parity suites.
"""
import numpy as np
import pytest

import paper_2003_05293_amd as hg
from workload import Grid, OPTICS, PUPIL_OPTICS, spot_cloud

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available()
    hg.load()
    yield
    torch.cuda.synchronize()


G = Grid(256, 192)


@pytest.mark.parametrize("N", [1, 5, 100, 256, 257])
@pytest.mark.parametrize("I", [2, 3, 4, 7])
def test_alone_equals_batch_without_deferral(N, I):
    import torch
    say("alone vs batch", N, I)
    s = spot_cloud(N, N, G)
    alone = hg.cswgs(G, OPTICS, s, I, 0.25, 11).cpu().numpy()
    # a job of 300 spots needs four spot units per wave: it runs in the wide launch
    jobs = [hg.DeviceJob.from_spots(G, OPTICS, s, I, 0.25, 11),
            hg.DeviceJob.from_spots(G, OPTICS, spot_cloud(7, 300, G), 3, 0.25, 2)]
    hg.cswgs_batch(jobs)
    torch.cuda.synchronize()
    assert np.array_equal(alone, jobs[0].phi.cpu().numpy())


@pytest.mark.parametrize("N", [1, 5, 100, 256])
@pytest.mark.parametrize("I", [3, 4, 7])
def test_deferred_equals_chained(N, I):
    say("deferred vs chained", N, I)
    s = spot_cloud(N + 1, N, G)
    dfr = hg.cswgs(G, OPTICS, s, I, 0.25, 3, tune={"chain_passes": 0}).cpu().numpy()
    chn = hg.cswgs(G, OPTICS, s, I, 0.25, 3, tune={"chain_passes": 1}).cpu().numpy()
    assert np.array_equal(dfr, chn)


@pytest.mark.parametrize("optics", [OPTICS, PUPIL_OPTICS], ids=["uniform", "pupil"])
def test_traced_fields_equal_chained_launch(optics):
    say("trace vs chained", optics is PUPIL_OPTICS)
    g = Grid(384, 320)
    s = spot_cloud(3, 100, g)
    phi_d, V_d = hg.cswgs(g, optics, s, 9, 1 / 8, 5, trace=True)
    phi_c, V_c = hg.cswgs(g, optics, s, 9, 1 / 8, 5, trace=True, tune={"chain_passes": 1})
    assert np.array_equal(phi_d.cpu().numpy(), phi_c.cpu().numpy())
    assert np.array_equal(np.asarray(V_d), np.asarray(V_c))
    assert np.all(np.isfinite(np.asarray(V_d)))


def test_back_to_back_holograms():
    import torch
    say("back to back")
    s1, s2 = spot_cloud(1, 64, G), spot_cloud(2, 200, G)
    ref1 = hg.cswgs(G, OPTICS, s1, 6, 0.25, 1).cpu().numpy()
    ref2 = hg.cswgs(G, OPTICS, s2, 5, 0.25, 2).cpu().numpy()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = hg.cswgs(G, OPTICS, s1, 6, 0.25, 1, stream=st)
        b = hg.cswgs(G, OPTICS, s2, 5, 0.25, 2, stream=st)
        c = hg.cswgs(G, OPTICS, s1, 6, 0.25, 1, stream=st)
    st.synchronize()
    assert np.array_equal(a.cpu().numpy(), ref1)
    assert np.array_equal(b.cpu().numpy(), ref2)
    assert np.array_equal(c.cpu().numpy(), ref1)


def test_engine_mix_of_unit_widths_equals_alone():
    import torch
    say("engine 100 + 300 + 5 spots")
    specs = [(100, 6, 1), (300, 4, 2), (5, 7, 3), (256, 5, 4)]
    alone = [hg.cswgs(G, OPTICS, spot_cloud(40 + k, n, G), it, 0.25, seed).cpu().numpy()
             for k, (n, it, seed) in enumerate(specs)]
    e = hg.Engine(1 << 28, 8)
    st = torch.cuda.Stream()
    phis, tickets = [], []
    for k, (n, it, seed) in enumerate(specs):
        p = torch.empty(G.M, dtype=torch.float32, device="cuda")
        phis.append(p)
        tickets.append(e.submit(G, OPTICS, spot_cloud(40 + k, n, G), it, 0.25, seed, p))
    done = set()
    for _ in range(100):
        e.step(stream=st)
        for t in tickets:
            if t not in done and e.poll(t):
                done.add(t)
        if len(done) == len(tickets):
            break
    st.synchronize()
    e.close()
    assert len(done) == len(tickets)
    for k in range(len(specs)):
        assert np.array_equal(phis[k].cpu().numpy(), alone[k]), specs[k]
