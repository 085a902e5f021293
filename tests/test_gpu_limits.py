"""GPU parity at the limits the C ABI accepts: N up to HG_MAX_SPOTS = 4096,
more pixels than the on-chip Feistel tables cover (M > 4^11, where the random
order reads its round tables from global memory), grids up to 8192 pixels on
a side, and the 64-hologram mixed batch against the same holograms alone.

Bars (FP32 form), and where they come from:
* subset indices: bit-exact (integer work);
* forward projection with Phi held fixed, one fused pass with (w, theta)
  held fixed, V^1 of a run: max_n ||V_n| - |V_n(oracle)|| <= REL_V = 1e-5
  times the mean spot magnitude mean_n |V_n(oracle)|.  The absolute error of
  a spot's field does not depend on its magnitude, and with thousands of
  spots the weakest field is a small fraction of the mean, so the error is
  measured against the mean (for N <= 300 the suite's other files bound it
  spot by spot).  The bar holds while the phase of a (pixel, spot) term
  stays within T_REF = 256 turns, as on the 1920 x 1152 panel; beyond, the
  FP32 phase t = cx Lx + cy Ly + cz Q (and its FP32 coefficients) carries a
  rounding error proportional to |t|, so the bar scales with the largest
  |t| of the case, t_max / T_REF.  And a pass over m pixels averages
  independent per-term roundings of a few 2^-24 |t| turns, which leaves an
  error of about that over sqrt(m) against a mean magnitude of about
  N^-1/2: where 4 2 pi 2^-24 t_max sqrt(N / m) is larger (thousands of
  spots on a few thousand pixels), it is the bar;
* Phi of a back-propagation: wrapped error RMS <= max(1e-4, PHI_PER_TURN *
  t_max), 99.9th percentile <= 20 x that, with PHI_PER_TURN = 2 pi 6 2^-24
  rad per turn (three FMAs and three coefficient roundings, each at most
  half an FP32 ulp of |t|);
* final e and u: within 1e-3 of the oracle's;
* mixed precision: the bars of the mixed form (|Delta V_n| <= 8 2^-11 /
  sqrt(M) with Phi fixed, magnitude error <= 1e-3 of the mean for one pass,
  e, u within 1e-3);
* a batch: every hologram bit-identical to the same hologram alone.
Each case prints its name before touching the GPU.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2003_05293_amd as hg
from workload import Grid, OPTICS, spot_cloud, mixed_batch

pytestmark = pytest.mark.gpu

REL_V = 1e-5
ROUND_V = 4 * 2 * math.pi * 2.0 ** -24  # four FP32 roundings of the phase, per turn
REL_V_MX = 1e-3
EU_TOL = 1e-3
T_REF = 256.0
PHI_PER_TURN = 2 * math.pi * 6 * 2.0 ** -24


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


def err_stats(d):
    d = np.asarray(d)
    return dict(rms=float(np.sqrt((d ** 2).mean())), p999=float(np.quantile(d, 0.999)),
                max=float(d.max()))


def rel_mag_err(Vg, Vo):
    """Largest spot-magnitude error over the mean spot magnitude."""
    return float(np.max(np.abs(np.abs(Vg) - np.abs(Vo))) / np.mean(np.abs(Vo)))


def t_max(g, s):
    """Largest |phase| in turns of any (pixel, spot) term, bounded term by
    term: (|x| |x'| + |y| |y'|) / (lambda f) + |z| (x'^2 + y'^2) / (lambda f^2)
    at the grid's outermost pixel centres."""
    xm = (g.W - 1) / 2 * g.pitch_mm
    ym = (g.H - 1) / 2 * g.pitch_mm
    lf = OPTICS.lambda_mm * OPTICS.focal_mm
    t = (np.abs(s.x_mm) * xm + np.abs(s.y_mm) * ym) / lf \
        + np.abs(s.z_mm) * (xm * xm + ym * ym) / (lf * OPTICS.focal_mm)
    return float(t.max())


def v_bar(g, s, m):
    """FP32 bar of |V_n| over the mean spot magnitude for a pass over m
    pixels: REL_V (scaled by t_max / T_REF beyond T_REF turns), or, where
    larger, ROUND_V t_max sqrt(N / m): each term's FP32 phase carries a
    rounding error of a few 2^-24 |t| turns, independent from term to term,
    so the mean over m terms errs by about that over sqrt(m), while the mean
    spot magnitude is about 1 / sqrt(N)."""
    return max(REL_V * max(1.0, t_max(g, s) / T_REF), ROUND_V * t_max(g, s) * math.sqrt(s.n / m))


def phi_bars(g, s):
    rms = max(1e-4, PHI_PER_TURN * t_max(g, s))
    return rms, 20 * rms


def rs_phase_on(g, s, seed, p):
    """FP32 grid holding the oracle's RS phase at pixels p and 0 elsewhere: a
    realistic hologram where the forward sum reads it."""
    phi = np.zeros(g.M, dtype=np.float32)
    phi[p] = oracle.backward(g, OPTICS, s, np.ones(s.n), oracle.theta0(seed, s.n), p)
    return phi


# ---------------------------------------------------- many spots ---

# N above 1024 runs the wide pass form (16 spot units per wave); 4096 is the
# ABI's maximum.  A 96 x 64 grid keeps the oracle at a few seconds.
BIG_N = [1500, 4096]


@pytest.mark.parametrize("N", BIG_N)
@pytest.mark.parametrize("sub", [None, 0.25])
def test_many_spots_forward_phi_held_fixed(N, sub):
    g = Grid(96, 64)
    s = spot_cloud(N, N, g, z_half_mm=0.1)
    p = np.arange(g.M) if sub is None else oracle.subset(g.M, N, 1, sub)
    phi = rs_phase_on(g, s, N, p)
    say("many spots forward", N, sub)
    Vg = hg.forward(g, OPTICS, s, to_dev(phi), idx=None if sub is None else to_dev(p, "int32"))
    Vo = oracle.forward(g, OPTICS, s, phi.astype(np.float64)[p], p)
    e = rel_mag_err(Vg, Vo)
    print("many spots forward |V| rel err", N, sub, e, "bar", v_bar(g, s, p.size))
    assert e <= v_bar(g, s, p.size)
    if sub is None:  # the mixed form's single-pass calls take the whole grid
        Vm = hg.forward(g, OPTICS, s, to_dev(phi), precision="mixed")
        dm = float(np.max(np.abs(Vm - Vo)))
        print("many spots forward mixed |dV|", N, dm, "bar", 8 * 2.0 ** -11 / math.sqrt(p.size))
        assert dm <= 8 * 2.0 ** -11 / math.sqrt(p.size)


def mx_bar(N, m):
    """Bar of the mixed form for one pass over m pixels, against the mean
    spot magnitude: 1e-3, or 8 FP16 unit roundoffs of the typical term
    scaled by sqrt(N / m) when that is larger (|dV_n| ~ 2^-11 / sqrt(m) per
    spot while the mean |V_n| falls as 1 / sqrt(N))."""
    return max(REL_V_MX, 8 * 2.0 ** -11 * math.sqrt(N / m))


@pytest.mark.parametrize("N", BIG_N)
@pytest.mark.parametrize("sub", [None, 0.25])
def test_many_spots_step_state_held_fixed(N, sub):
    g = Grid(96, 64)
    s = spot_cloud(N + 1, N, g, z_half_mm=0.1)
    rng = np.random.default_rng(N)
    w = rng.uniform(0.6, 1.4, N)
    th = rng.uniform(0, 2 * math.pi, N)
    p = np.arange(g.M) if sub is None else oracle.subset(g.M, N, 2, sub)
    idx = None if sub is None else to_dev(p, "int32")
    say("many spots step", N, sub)
    Vo = oracle.forward(g, OPTICS, s, oracle.backward(g, OPTICS, s, w, th, p), p)
    for direct in ((False, True) if sub is None else (False,)):
        Vg = hg.step(g, OPTICS, s, w, th, idx=idx, direct=direct)
        e = rel_mag_err(Vg, Vo)
        print("many spots step |V| rel err", N, sub, "direct" if direct else "", e)
        assert e <= v_bar(g, s, p.size)
    if sub is None:
        Vm = hg.step(g, OPTICS, s, w, th, precision="mixed")
        em = rel_mag_err(Vm, Vo)
        print("many spots step mixed |V| rel err", N, em, "bar", mx_bar(N, p.size))
        assert em <= mx_bar(N, p.size)


@pytest.mark.parametrize("N", BIG_N)
def test_many_spots_backward(N):
    g = Grid(96, 64)
    s = spot_cloud(N + 2, N, g, z_half_mm=0.1)
    rng = np.random.default_rng(N + 2)
    w = rng.uniform(0.5, 1.5, N)
    th = rng.uniform(-math.pi, math.pi, N)
    want = oracle.backward(g, OPTICS, s, w, th)
    rms_bar, p999_bar = phi_bars(g, s)
    say("many spots backward", N)
    for direct in (False, True):
        st = err_stats(wrapped(to_np(hg.backward(g, OPTICS, s, w, th, direct=direct)), want))
        print("many spots backward", N, "direct" if direct else "separable", st)
        assert st["rms"] <= rms_bar and st["p999"] <= p999_bar
    p = oracle.subset(g.M, N, 3, 0.25)
    st = err_stats(wrapped(to_np(hg.backward(g, OPTICS, s, w, th, idx=to_dev(p, "int32"))),
                           want[p]))
    print("many spots backward, subset", N, st)
    assert st["rms"] <= rms_bar and st["p999"] <= p999_bar


@pytest.mark.parametrize("N", BIG_N)
@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_many_spots_cswgs(N, precision):
    """A short CS-WGS run with more spots than the 96 x 64 grid resolves
    (about 0.16 M = 983 spot-sized cells in the spots' box): the problem is
    ill-conditioned, so two runs that differ by rounding drift apart, and
    e, u of the GPU's and the oracle's runs are not compared.  Each kernel
    of the run is checked instead: every V^{j+1} against the oracle's step
    from the state the GPU's own V^1..V^j imply, the final hologram against
    the oracle's back-propagation of the final state, and the FP64 metrics
    against the oracle's on the same hologram."""
    g = Grid(96, 64)
    s = spot_cloud(N + 3, N, g, z_half_mm=0.1)
    I, c, seed = 4, 0.25, N
    say("many spots cswgs", N, precision)
    phi, V = hg.cswgs(g, OPTICS, s, I, c, seed, trace=True, precision=precision)
    w, th = np.ones(N), oracle.theta0(seed, N)
    for j in range(1, I + 1):
        p = oracle.subset(g.M, oracle.ORDER_KEY, j, c) if j < I else np.arange(g.M)
        Vo = oracle.forward(g, OPTICS, s, oracle.backward(g, OPTICS, s, w, th, p), p)
        bar = v_bar(g, s, p.size) if precision == "fp32" else mx_bar(N, p.size)
        err = rel_mag_err(V[j - 1], Vo)
        print("many spots cswgs", N, precision, "V^%d" % j, err, "bar", bar)
        assert err <= bar
        w, th = oracle.update(w, V[j - 1])
    phi_np = to_np(phi)
    d = err_stats(wrapped(phi_np, oracle.backward(g, OPTICS, s, w, th)))
    rms_bar, p999_bar = phi_bars(g, s)
    if precision == "mixed":
        rms_bar, p999_bar = 2e-3, 2e-2  # the mixed form's full-grid phase bars
    print("many spots cswgs", N, precision, "final Phi", d)
    assert d["rms"] <= rms_bar and d["p999"] <= p999_bar
    e, u, _ = hg.metrics(g, OPTICS, s, phi)
    eo, uo, _ = oracle.metrics(g, OPTICS, s, phi_np)
    print("many spots cswgs", N, precision, "e", e, eo, "u", u, uo)
    assert abs(e - eo) <= 1e-9 * max(1.0, eo) and abs(u - uo) <= 1e-9


# ------------------------------------------- large and wide grids ---

# 2100^2 and 3000 x 1500 hold more than 4^11 pixels: the random order's
# Feistel tables no longer fit the LDS and are read from global memory.
# 3000, 8192 (the ABI's maximum width and height) exceed 2896, beyond which
# the doubled squared offset Q = Lx^2 + Ly^2 is no longer exact in FP32.
BIG_GRIDS = [(2100, 2100), (3000, 1500), (8192, 48), (40, 8192)]


@pytest.mark.parametrize("W,H", BIG_GRIDS)
def test_big_grid_subset_bit_exact(W, H):
    g = Grid(W, H)
    for seed, j, c in ((5, 1, 1 / 16), (6, 17, 1 / 16), (7, 3, 0.37)):
        say("big grid subset", W, H, seed, j, c)
        got = to_np(hg.subset(g, seed, j, c)).astype(np.int64)
        want = oracle.subset(g.M, seed, j, c)
        assert got.shape == want.shape
        assert np.array_equal(got, want)


@pytest.mark.parametrize("W,H", BIG_GRIDS)
def test_big_grid_forward_and_step(W, H):
    g = Grid(W, H)
    N, seed = 16, W + H
    s = spot_cloud(seed, N, g)
    p = oracle.subset(g.M, seed, 1, 1 / 16)
    phi = rs_phase_on(g, s, seed, p)
    say("big grid forward", W, H, "t_max", t_max(g, s))
    Vg = hg.forward(g, OPTICS, s, to_dev(phi), idx=to_dev(p, "int32"))
    Vo = oracle.forward(g, OPTICS, s, phi.astype(np.float64)[p], p)
    e = rel_mag_err(Vg, Vo)
    print("big grid forward |V| rel err", W, H, e, "bar", v_bar(g, s, p.size))
    assert e <= v_bar(g, s, p.size)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.6, 1.4, N)
    th = rng.uniform(0, 2 * math.pi, N)
    say("big grid step", W, H)
    Vg = hg.step(g, OPTICS, s, w, th, idx=to_dev(p, "int32"))
    Vo = oracle.forward(g, OPTICS, s, oracle.backward(g, OPTICS, s, w, th, p), p)
    e = rel_mag_err(Vg, Vo)
    print("big grid step |V| rel err", W, H, e)
    assert e <= v_bar(g, s, p.size)


@pytest.mark.parametrize("W,H", BIG_GRIDS)
def test_big_grid_backward(W, H):
    g = Grid(W, H)
    N = 24
    s = spot_cloud(W + 2 * H, N, g, z_half_mm=0.1)
    rng = np.random.default_rng(W)
    w = rng.uniform(0.5, 1.5, N)
    th = rng.uniform(-math.pi, math.pi, N)
    pix = np.sort(rng.choice(g.M, 60000, replace=False))
    corners = np.array([0, g.W - 1, g.M - g.W, g.M - 1])
    pix = np.union1d(pix, corners)
    want = oracle.backward(g, OPTICS, s, w, th, pix)
    rms_bar, p999_bar = phi_bars(g, s)
    say("big grid backward", W, H, "t_max", t_max(g, s))
    full = to_np(hg.backward(g, OPTICS, s, w, th))
    st = err_stats(wrapped(full[pix], want))
    print("big grid backward separable", W, H, st, "bars", rms_bar, p999_bar)
    assert st["rms"] <= rms_bar and st["p999"] <= p999_bar
    st = err_stats(wrapped(to_np(hg.backward(g, OPTICS, s, w, th, idx=to_dev(pix, "int32"))),
                           want))
    print("big grid backward per pixel", W, H, st)
    assert st["rms"] <= rms_bar and st["p999"] <= p999_bar


@pytest.mark.parametrize("W,H", [(2100, 2100), (8192, 48), (40, 8192)])
def test_big_grid_cswgs(W, H):
    g = Grid(W, H)
    N, I, c, seed = 8, 3, 1 / 16, 11
    s = spot_cloud(seed, N, g)
    say("big grid cswgs", W, H)
    phi, V = hg.cswgs(g, OPTICS, s, I, c, seed, trace=True)
    tr = oracle.Trace()
    phi_o = oracle.cswgs(g, OPTICS, s, I, c, seed, tr)
    e, u, _ = hg.metrics(g, OPTICS, s, phi)
    eo, uo, _ = oracle.metrics(g, OPTICS, s, phi_o)
    e1 = rel_mag_err(V[0], tr.V[0])
    print("big grid cswgs", W, H, "e", e, eo, "u", u, uo, "V^1 rel", e1)
    assert abs(e - eo) <= EU_TOL and abs(u - uo) <= EU_TOL
    assert e1 <= v_bar(g, s, math.ceil(c * g.M))


def test_batch_with_big_grid_equals_alone():
    """A job whose random order reads its tables from global memory sets the
    table layout of the whole batch; every hologram still equals itself
    alone, bit for bit."""
    import torch
    cases = [(Grid(2100, 2100), 16, 5, 1 / 16, 1), (Grid(256, 256), 16, 20, 1 / 16, 2),
             (Grid(300, 170), 37, 8, 0.1, 3)]
    say("batch with a 2100^2 job vs alone")
    ref = [hg.cswgs(g, OPTICS, spot_cloud(sd, n, g), I, c, sd).clone() for g, n, I, c, sd in cases]
    jobs = [hg.DeviceJob.from_spots(g, OPTICS, spot_cloud(sd, n, g), I, c, sd)
            for g, n, I, c, sd in cases]
    hg.cswgs_batch(jobs)
    torch.cuda.synchronize()
    for k, (j, r) in enumerate(zip(jobs, ref)):
        assert torch.equal(j.phi, r), k


# ------------------------------------------- the 64-hologram batch ---

def test_mixed64_batch_equals_alone():
    """The 64-hologram mixed batch of the benchmark (sizes 512^2 to
    1920 x 1152, N in [8, 200], z within +-0.1 mm, I = 30, c = 1/16), as one
    graph-captured batch, against each hologram computed alone."""
    import torch
    mixed = mixed_batch(0, count=64)
    say("mixed64 batch vs alone")
    jobs = [hg.DeviceJob.from_spots(j.grid, OPTICS, j.spots, j.iterations, j.compression, j.seed)
            for j in mixed]
    batch = hg.Batch(jobs, use_graph=True)
    stream = torch.cuda.Stream()
    batch.run(stream)
    stream.synchronize()
    out = [j.phi.clone() for j in jobs]
    batch.run(stream)  # a replay of the captured graph
    stream.synchronize()
    batch.close()
    for k, j in enumerate(mixed):
        alone = hg.cswgs(j.grid, OPTICS, j.spots, j.iterations, j.compression, j.seed)
        torch.cuda.synchronize()
        assert torch.equal(out[k], alone), k
        assert torch.equal(jobs[k].phi, alone), k
