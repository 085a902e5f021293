"""GPU parity of the pupil (paper section 4: a Gaussian illumination of waist
radius w on the SLM and the round aperture of the optics) against the FP64
oracle, through the C ABI.

With a pupil the forward sums of eq. (3) weight each pixel by the
illumination amplitude A = exp(-r^2 / w^2), the full set of every iteration
is the set Omega of pixels inside the aperture, the random order of CS-WGS
runs over the |Omega| pupil pixels in index order, and the metrics divide
the efficiency by mean_Omega(A^2).  The hologram is still computed on every
pixel.

Bars (those of the uniform-pupil tests; every term still has magnitude
<= 1, so the error bounds carry over with |Omega| in place of W*H):
* subset pixel indices: bit-exact;
* forward with Phi held fixed and one fused pass with (w, theta) held fixed:
  |V_n| relative error <= 1e-5 (FP32) and, mixed precision, |dV| <=
  8 2^-11 / sqrt(|Omega|) (forward) and |V_n| relative error <= 1e-3 (pass);
* FP64 metrics on the same Phi: e and u within 1e-9, I_n within 1e-10;
* final e and u of WGS / CS-WGS in every pass form: within 1e-3 of the
  oracle's, V of the first iteration within 1e-5 (FP32) / 1e-3 (mixed);
* an aperture that holds the whole grid with no waist gives the same bits as
  no pupil; a pupil hologram alone, in a batch and through the serving
  engine gives the same bits.
Each case prints its name before touching the GPU.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import paper_2003_05293_amd as hg
from oracle import sampler
from workload import Grid, OPTICS, Optics, PUPIL_OPTICS, spot_cloud

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
REL_V = 1e-5
REL_V_MX = 1e-3
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


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def to_dev(a, dtype="float32"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a).astype(dtype), device="cuda")


def wrapped(a, b):
    return np.abs(np.angle(np.exp(1j * (np.asarray(a) - np.asarray(b)))))


def rel_mag_err(Vg, Vo):
    return float(np.max(np.abs(np.abs(Vg) - np.abs(Vo)) / np.abs(Vo)))


def pupil(D, w):
    return Optics(waist_mm=w, aperture_px=D)


# ------------------------------------------------------- random order ---

SUBSET_CASES = [
    (256, 256, 0, 1, 1 / 16, 256.0), (256, 256, 0, 17, 1 / 16, 200.5),
    (1152, 1152, 7, 3, 1 / 16, 1152.0), (1920, 1152, 3, 5, 1 / 16, 1152.0),
    (300, 170, 4, 4, 0.3, 150.0), (7, 5, 1, 3, 0.5, 4.0), (64, 48, 2, 1, 1.0, 3.0),
    (33, 20, 5, 2, 0.9, 1e6),
]


@pytest.mark.parametrize("W,H,seed,j,c,D", SUBSET_CASES)
def test_pupil_subset_bit_exact(W, H, seed, j, c, D):
    g = Grid(W, H)
    opt = pupil(D, 0.0)
    say("pupil subset", W, H, seed, j, c, D)
    got = to_np(hg.subset(g, seed, j, c, optics=opt)).astype(np.int64)
    omega = oracle.pupil_pixels(g, opt)
    want = omega[sampler.subset(omega.shape[0], seed, j, c)]
    assert got.shape == want.shape
    assert np.array_equal(got, want)


# ------------------------------------------------------- single passes ---

FWD_CASES = [(256, 256, 16, 0, 256.0, 1.0), (1152, 1152, 100, 1, 1152.0, 6.0),
             (300, 170, 70, 4, 150.0, 0.8), (1920, 1152, 129, 6, 1152.0, 6.0),
             (200, 150, 20, 3, 0.0, 0.5), (200, 150, 20, 3, 120.0, 0.0)]


@pytest.mark.parametrize("W,H,N,seed,D,w", FWD_CASES)
def test_pupil_forward_phi_held_fixed(W, H, N, seed, D, w):
    g = Grid(W, H)
    opt = pupil(D, w)
    s = spot_cloud(seed, N, g)
    phi32 = oracle.backward(g, opt, s, np.ones(N), oracle.theta0(seed, N)).astype(np.float32)
    omega = oracle.pupil_pixels(g, opt)
    Vo = oracle.forward(g, opt, s, phi32.astype(np.float64)[omega], omega)
    say("pupil forward", W, H, N, D, w)
    Vg = hg.forward(g, opt, s, to_dev(phi32))
    e = rel_mag_err(Vg, Vo)
    say("pupil forward mixed", W, H, N, D, w)
    Vm = hg.forward(g, opt, s, to_dev(phi32), precision="mixed")
    dm = float(np.max(np.abs(Vm - Vo)))
    bound = 8 * 2.0 ** -11 / math.sqrt(omega.shape[0])
    print("pupil forward |V| rel err", W, H, N, D, w, e, "mixed |dV|", dm, "bound", bound)
    assert e <= REL_V
    assert dm <= bound


def test_pupil_forward_explicit_pixels_weighted_not_masked():
    """An explicit pixel list is taken as given (the aperture does not drop
    any of its pixels); the illumination still weights them."""
    g = Grid(256, 200)
    opt = pupil(120.0, 0.7)
    s = spot_cloud(2, 24, g)
    phi32 = oracle.backward(g, opt, s, np.ones(24), oracle.theta0(2, 24)).astype(np.float32)
    idx = oracle.subset(g.M, 2, 3, 0.2)  # pixels inside and outside the aperture
    say("pupil forward explicit pixels")
    Vg = hg.forward(g, opt, s, to_dev(phi32), idx=to_dev(idx, "int32"))
    Vo = oracle.forward(g, opt, s, phi32.astype(np.float64)[idx], idx)
    assert rel_mag_err(Vg, Vo) <= REL_V


STEP_CASES = [(256, 256, 16, 0, 256.0, 1.0, False), (256, 256, 16, 0, 256.0, 1.0, True),
              (1152, 1152, 100, 4, 1152.0, 6.0, False), (1152, 1152, 100, 4, 1152.0, 6.0, True),
              (333, 129, 65, 9, 129.0, 0.5, False), (200, 70, 129, 5, 90.0, 0.0, False),
              (64, 64, 1, 2, 40.0, 0.2, True)]


@pytest.mark.parametrize("W,H,N,seed,D,w,direct", STEP_CASES)
def test_pupil_step_state_held_fixed(W, H, N, seed, D, w, direct):
    g = Grid(W, H)
    opt = pupil(D, w)
    s = spot_cloud(seed, N, g)
    rng = np.random.default_rng(seed + 100)
    wt = rng.uniform(0.6, 1.4, N)
    th = rng.uniform(0, 2 * math.pi, N)
    omega = oracle.pupil_pixels(g, opt)
    Vo = oracle.forward(g, opt, s, oracle.backward(g, opt, s, wt, th, omega), omega)
    say("pupil step", W, H, N, D, w, "direct" if direct else "separable")
    Vg = hg.step(g, opt, s, wt, th, direct=direct)
    e = rel_mag_err(Vg, Vo)
    print("pupil step |V| rel err", W, H, N, D, w, direct, e)
    assert e <= REL_V
    if not direct:
        say("pupil step mixed", W, H, N, D, w)
        em = rel_mag_err(hg.step(g, opt, s, wt, th, precision="mixed"), Vo)
        print("pupil mixed step |V| rel err", em)
        assert em <= REL_V_MX


@pytest.mark.parametrize("W,H,N,seed,D,w", [(256, 256, 16, 0, 256.0, 1.0),
                                            (1152, 1152, 100, 1, 1152.0, 6.0),
                                            (130, 77, 5, 2, 70.0, 0.3)])
def test_pupil_metrics_fp64(W, H, N, seed, D, w):
    g = Grid(W, H)
    opt = pupil(D, w)
    s = spot_cloud(seed, N, g)
    say("pupil metrics", W, H, N, D, w)
    phi = hg.rs(g, opt, s, seed)
    e, u, inten = hg.metrics(g, opt, s, phi)
    eo, uo, io = oracle.metrics(g, opt, s, to_np(phi))
    print("pupil metrics", W, H, N, e, eo, u, uo)
    assert abs(e - eo) < 1e-9 and abs(u - uo) < 1e-9
    assert np.max(np.abs(inten - io)) < 1e-10


# ------------------------------------------------------- algorithms ---

SHARED_E = {"pass_form": 1}
CHAINED = {"chain_passes": 1}


_ORACLE_RUNS = {}


def _oracle_run(g, opt, s, I, c, seed):
    """(V^1, e, u) of the oracle, once per case (shared by the pass forms)."""
    key = (g.W, g.H, s.n, I, c, seed, opt.aperture_px, opt.waist_mm)
    if key not in _ORACLE_RUNS:
        tr = oracle.Trace()
        if c is None:
            phi_o = oracle.wgs(g, opt, s, I, seed, tr)
        else:
            phi_o = oracle.cswgs(g, opt, s, I, c, seed, tr)
        eo, uo, _ = oracle.metrics(g, opt, s, phi_o)
        _ORACLE_RUNS[key] = (tr.V[0], eo, uo)
    return _ORACLE_RUNS[key]


def _run_and_compare(g, opt, s, I, c, seed, tag, **kw):
    V1o, eo, uo = _oracle_run(g, opt, s, I, c, seed)
    say(tag, g.W, g.H, s.n, I, c, opt.aperture_px, opt.waist_mm, kw)
    mixed = kw.get("precision") == "mixed"
    phi_g, Vg = hg.cswgs(g, opt, s, I, 1.0 if c is None else c, seed, trace=True, **kw)
    if c is None and not kw:
        phi_g = hg.wgs(g, opt, s, I, seed)  # every pass over the whole grid
    eg, ug, _ = hg.metrics(g, opt, s, phi_g)
    e1 = rel_mag_err(Vg[0], V1o)
    print(tag, "e", eg, eo, "u", ug, uo, "V^1 rel", e1)
    assert abs(eg - eo) <= EU_TOL and abs(ug - uo) <= EU_TOL
    assert e1 <= (REL_V_MX if mixed else REL_V)


ALGO_CASES = [(256, 256, 16, 20, 1 / 16, 0, 256.0, 1.0), (256, 256, 16, 12, None, 0, 256.0, 1.0),
              (300, 170, 37, 8, 0.1, 11, 160.7, 0.9), (512, 512, 200, 10, 1 / 16, 4, 512.0, 2.0)]


@pytest.mark.parametrize("W,H,N,I,c,seed,D,w", ALGO_CASES)
@pytest.mark.parametrize("form", ["default", "direct", "shared_e", "chained", "mixed"])
def test_pupil_algorithms_vs_oracle(W, H, N, I, c, seed, D, w, form):
    g = Grid(W, H)
    s = spot_cloud(seed, N, g, z_half_mm=0.1)
    kw = {"default": {}, "direct": {"direct": True}, "shared_e": {"tune": SHARED_E},
          "chained": {"tune": CHAINED}, "mixed": {"precision": "mixed"}}[form]
    _run_and_compare(g, pupil(D, w), s, I, c, seed, "pupil " + form, **kw)


def test_pupil_full_size_against_stored_oracle():
    name = "cswgs_1152x1152_n100_i30_c16_pupil_seed0"
    path = os.path.join(GOLDEN, name + ".json")
    with open(path) as f:
        gd = json.load(f)
    g = Grid(gd["W"], gd["H"])
    opt = Optics(waist_mm=gd["waist_mm"], aperture_px=gd["aperture_px"])
    assert opt == PUPIL_OPTICS
    s = spot_cloud(gd["seed"], gd["n"], g, z_half_mm=gd["z_half_mm"])
    say("pupil full size", name)
    phi, V = hg.cswgs(g, opt, s, gd["iterations"], gd["compression"], gd["seed"], trace=True)
    e, u, _ = hg.metrics(g, opt, s, phi)
    V1 = np.array(gd["V1"])
    V1 = V1[:, 0] + 1j * V1[:, 1]
    e1 = rel_mag_err(V[0], V1)
    pix = np.array(gd["sample_pixels"])
    d = wrapped(to_np(phi)[pix], np.array(gd["sample_phi"]))
    print(name, "e", e, gd["e"], "u", u, gd["u"], "V^1 rel", e1, "Phi sample rms",
          float(np.sqrt((d ** 2).mean())))
    assert abs(e - gd["e"]) <= EU_TOL and abs(u - gd["u"]) <= EU_TOL
    assert e1 <= REL_V


# ------------------------------------------------------- identities ---

@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_aperture_over_whole_grid_is_no_pupil(precision):
    """An aperture holding every pixel, with no waist, changes nothing: the
    random order, the sets and the sums are those of the uniform pupil."""
    import torch
    g = Grid(300, 170)
    s = spot_cloud(3, 37, g)
    say("whole-grid aperture identity", precision)
    a = hg.cswgs(g, OPTICS, s, 8, 0.1, 11, precision=precision, trace=True)
    b = hg.cswgs(g, pupil(1e6, 0.0), s, 8, 0.1, 11, precision=precision, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_pupil_alone_batch_and_engine_identical():
    import torch
    g1, g2 = Grid(256, 256), Grid(300, 170)
    o1, o2 = pupil(256.0, 1.0), pupil(160.7, 0.9)
    s1, s2 = spot_cloud(0, 16, g1), spot_cloud(3, 37, g2)
    say("pupil alone vs batch vs engine")
    ref1 = hg.cswgs(g1, o1, s1, 20, 1 / 16, 0).clone()
    ref2 = hg.cswgs(g2, o2, s2, 8, 0.1, 11).clone()
    ref3 = hg.cswgs(g1, OPTICS, s1, 20, 1 / 16, 0).clone()
    jobs = [hg.DeviceJob.from_spots(g1, o1, s1, 20, 1 / 16, 0),
            hg.DeviceJob.from_spots(g2, o2, s2, 8, 0.1, 11),
            hg.DeviceJob.from_spots(g1, OPTICS, s1, 20, 1 / 16, 0)]
    out = hg.cswgs_batch(jobs)
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(out, (ref1, ref2, ref3))):
        assert torch.equal(o, r), k
    eng = hg.Engine(1 << 30, max_slots=4)
    try:
        phis = [torch.full((g.M,), float("nan"), dtype=torch.float32, device="cuda")
                for g in (g1, g2, g1)]
        t = [eng.submit(g1, o1, s1, 20, 1 / 16, 0, phis[0])]
        eng.step()
        t.append(eng.submit(g2, o2, s2, 8, 0.1, 11, phis[1]))
        eng.step()
        t.append(eng.submit(g1, OPTICS, s1, 20, 1 / 16, 0, phis[2]))
        steps = 0
        while not all(eng.poll(x) for x in t):
            eng.step()
            steps += 1
            assert steps < 1000
        torch.cuda.synchronize()
    finally:
        eng.close()
    for k, (o, r) in enumerate(zip(phis, (ref1, ref2, ref3))):
        assert torch.equal(o, r), k
