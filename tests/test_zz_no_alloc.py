"""hg_cswgs_static, the entry point that allocates nothing (its scratch is a
static per-GPU device array), against hg_cswgs_ex on the same inputs.

Both run the same kernels on the same inputs, so the bar is bit identity of
the hologram (and of the gray image where one is asked for).  Calls follow
each other on one stream, each smaller than the one before, so every call
reuses the array that the previous call left behind: the first is the
1152^2, N = 100 CS-WGS workload, then smaller grids with fewer spots, in
both precisions, under a pupil, and with the gray-image output.  A hologram
whose scratch exceeds the array is rejected with HG_ENOMEM before anything
runs, and its output is left untouched.  Each case prints its name before
touching the GPU.
"""
import numpy as np
import pytest

import paper_2003_05293_amd as hg
from workload import Grid, OPTICS, PUPIL_OPTICS, spot_cloud

pytestmark = pytest.mark.gpu

CASES = [  # W, H, N, I, c, seed, precision, pupil
    (1152, 1152, 100, 30, 1 / 16, 0, "fp32", False),
    (512, 384, 60, 12, 0.1, 5, "fp32", False),
    (300, 200, 37, 9, 0.25, 11, "mixed", False),
    (256, 256, 16, 20, 1 / 16, 2, "fp32", True),
    (96, 64, 1500, 4, 0.25, 3, "fp32", False),
    (64, 48, 5, 6, 0.5, 7, "mixed", True),
]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hg.load()
    yield
    torch.cuda.synchronize()


def say(*a):
    print("[case]", *a, flush=True)


def spots_dev(s):
    import torch
    return torch.tensor(np.stack([s.x_mm, s.y_mm, s.z_mm, s.amp]), dtype=torch.float64,
                        device="cuda")


def test_static_matches_ex_on_consecutive_calls():
    import torch
    stream = torch.cuda.current_stream()
    for W, H, N, I, c, seed, prec, pupil in CASES:
        g = Grid(W, H)
        optics = PUPIL_OPTICS if pupil else OPTICS
        sd = spots_dev(spot_cloud(seed, N, g))
        say("static vs ex", W, H, N, I, c, seed, prec, "pupil" if pupil else "")
        ref = hg.cswgs_device(g, optics, sd, I, c, seed, stream=stream, precision=prec)
        phi = torch.full((W * H,), 7.0, dtype=torch.float32, device="cuda")
        hg.cswgs_static(g, optics, sd, I, c, seed, phi, stream=stream, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(phi, ref), (W, H, N, prec)


def test_static_twice_same_input_and_gray_output():
    """The same hologram twice in a row (the second call sees the first
    one's leftovers at every address), and the fused gray image."""
    import torch
    g = Grid(320, 240)
    sd = spots_dev(spot_cloud(4, 50, g))
    lut = hg.Lut(np.arange(256, dtype=np.uint16), bits=8)
    say("static twice with gray image", g.W, g.H, 50)
    ref_gray = lut.new_image(g)
    ref = hg.cswgs_device(g, OPTICS, sd, 10, 0.125, 4, lut=lut, gray=ref_gray)
    outs = []
    for _ in range(2):
        phi = torch.empty(g.W * g.H, dtype=torch.float32, device="cuda")
        gray = lut.new_image(g)
        hg.cswgs_static(g, OPTICS, sd, 10, 0.125, 4, phi, lut=lut, gray=gray)
        outs.append((phi, gray))
    torch.cuda.synchronize()
    for phi, gray in outs:
        assert torch.equal(phi, ref)
        assert torch.equal(gray, ref_gray)


def test_static_rejects_oversized_request():
    import torch
    g = Grid(4096, 4096)
    sd = spots_dev(spot_cloud(1, 100, g))
    phi = torch.full((g.W * g.H,), 3.0, dtype=torch.float32, device="cuda")
    say("static oversized", g.W, g.H)
    with pytest.raises(hg.HGError) as ei:
        hg.cswgs_static(g, OPTICS, sd, 30, 1 / 16, 1, phi)
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((phi == 3.0).all())
    # a request that fits still runs after the rejection
    g2 = Grid(128, 96)
    sd2 = spots_dev(spot_cloud(2, 12, g2))
    ref = hg.cswgs_device(g2, OPTICS, sd2, 8, 0.25, 2)
    phi2 = torch.empty(g2.W * g2.H, dtype=torch.float32, device="cuda")
    hg.cswgs_static(g2, OPTICS, sd2, 8, 0.25, 2, phi2)
    torch.cuda.synchronize()
    assert torch.equal(phi2, ref)
