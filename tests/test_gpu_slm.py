"""SLM output: the phase-to-gray lookup on the GPU against the oracle's
(oracle/slm.py), through the C ABI.

The gray level is the table entry of the phase's bin (oracle/slm.py: the
exact bin of the phase value the device holds).  The device decides the bin
in FP32, so its gray level must be that of the exact bin, except for a phase
within the FP32 rounding of a bin edge (oracle.fp32_edge_tolerance), where
the bin on the other side of the edge is accepted too:
* hg_phase_to_gray on random and adversarial phases (bin edges, whole
  turns, negative phases), for 8- and 16-bit tables of several sizes, ragged
  counts and an image that is not 4-byte aligned;
* the gray image written by the final pass of CS-WGS (FP32 separable,
  per-pixel direct, mixed precision, under a pupil) equals the oracle's
  lookup of the hologram the same call returns, and that hologram is the one
  computed without a table;
* batch and serving engine: the same bits as alone.
Each case prints its name before touching the GPU.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2003_05293_amd as hg
from workload import Grid, OPTICS, Optics, spot_cloud

pytestmark = pytest.mark.gpu


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
    return t.detach().cpu().numpy()


def slm_table(levels, bits, gamma=0.8):
    """A nonlinear SLM response: g(k) = round(G (k / (levels - 1))^gamma)."""
    G = 255 if bits == 8 else 4095
    k = np.arange(levels) / max(levels - 1, 1)
    return np.rint(G * k ** gamma).astype(np.uint16)


def assert_gray_matches(got, phi, table):
    """got[p] is table[k] for the exact bin k of phi[p], or a neighbouring
    bin's entry where phi[p] lies within FP32 rounding of the edge between
    them."""
    L = table.shape[0]
    phi = np.asarray(phi, dtype=np.float32)
    k, d = oracle.gray_bin(phi, L)
    tab = table.astype(np.int64)
    exact = got == tab[k]
    near = d <= oracle.fp32_edge_tolerance(phi, L)
    nb = near & ((got == tab[(k + 1) % L]) | (got == tab[(k - 1) % L]))
    bad = np.flatnonzero(~(exact | nb))
    assert bad.size == 0, [(float(phi[i]), int(got[i]), int(k[i]), float(d[i])) for i in bad[:5]]
    return int(np.count_nonzero(~exact))


def adversarial_phases(n, seed):
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-math.pi, math.pi, n), rng.uniform(-60, 60, n // 4)]
    edges = 2 * np.pi * (np.arange(-300, 300) / 256.0)    # bin edges of L = 256
    parts += [edges, np.nextafter(edges.astype(np.float32), np.float32(np.inf)),
              np.nextafter(edges.astype(np.float32), np.float32(-np.inf))]
    parts += [np.array([0.0, -0.0, math.pi, -math.pi, 2 * math.pi, -2 * math.pi, -1e-7, 1e-7,
                        -1e-30, 6.2831855, -6.2831855])]
    return np.concatenate([np.asarray(p, dtype=np.float32) for p in parts])


@pytest.mark.parametrize("levels,bits", [(256, 8), (1024, 16), (7, 8), (4096, 16), (1, 8),
                                         (65536, 16)])
@pytest.mark.parametrize("count_off", [0, 1, 3])
def test_phase_to_gray_bit_exact(levels, bits, count_off):
    import torch
    table = slm_table(levels, bits)
    phi = adversarial_phases(20000, levels)
    phi = phi[:phi.shape[0] - count_off] if count_off else phi
    say("phase_to_gray", levels, bits, phi.shape[0])
    lut = hg.Lut(table, bits=bits)
    try:
        d_phi = torch.as_tensor(phi, device="cuda")
        gray = hg.phase_to_gray(lut, d_phi)
        got = to_np(gray).astype(np.int64) & (0xFF if bits == 8 else 0xFFFF)
        off = assert_gray_matches(got, phi, table)
        print(f"  {phi.shape[0]} phases, {off} in the neighbouring bin of an edge", flush=True)
        if bits == 8:
            # an image one byte off 4-byte alignment, and a tiny count: the
            # same levels as the aligned image
            buf = torch.zeros(phi.shape[0] + 1, dtype=torch.uint8, device="cuda")
            hg.phase_to_gray(lut, d_phi, gray=buf[1:])
            assert np.array_equal(to_np(buf[1:]).astype(np.int64), got)
            assert to_np(buf)[0] == 0
            g3 = hg.phase_to_gray(lut, d_phi[:3])
            assert np.array_equal(to_np(g3).astype(np.int64), got[:3])
    finally:
        lut.close()


def _gray_of(gray, bits):
    return to_np(gray).astype(np.int64) & (0xFF if bits == 8 else 0xFFFF)


@pytest.mark.parametrize("form", ["separable", "direct", "mixed", "pupil"])
@pytest.mark.parametrize("bits", [8, 16])
def test_final_pass_writes_gray_image(form, bits):
    import torch
    g = Grid(300, 170)
    s = spot_cloud(3, 37, g)
    opt = Optics(waist_mm=0.9, aperture_px=160.0) if form == "pupil" else OPTICS
    kw = {"separable": {}, "direct": {"direct": True}, "mixed": {"precision": "mixed"},
          "pupil": {}}[form]
    table = slm_table(256 if bits == 8 else 1024, bits)
    lut = hg.Lut(table, bits=bits)
    try:
        gray = lut.new_image(g)
        say("final pass gray image", form, bits)
        phi = hg.cswgs(g, opt, s, 8, 0.1, 11, lut=lut, gray=gray, **kw)
        ref = hg.cswgs(g, opt, s, 8, 0.1, 11, **kw)
        torch.cuda.synchronize()
        assert torch.equal(phi, ref)
        assert_gray_matches(_gray_of(gray, bits), to_np(phi), table)
        # the fused epilogue and the standalone conversion agree bit for bit
        assert np.array_equal(_gray_of(gray, bits), _gray_of(hg.phase_to_gray(lut, phi), bits))
    finally:
        lut.close()


def test_gray_image_alone_batch_engine():
    import torch
    g1, g2 = Grid(256, 256), Grid(300, 170)
    s1, s2 = spot_cloud(0, 16, g1), spot_cloud(3, 37, g2)
    table = slm_table(256, 8)
    lut = hg.Lut(table, bits=8)
    try:
        say("gray image alone vs batch vs engine")
        a1, a2 = lut.new_image(g1), lut.new_image(g2)
        hg.cswgs(g1, OPTICS, s1, 20, 1 / 16, 0, lut=lut, gray=a1)
        hg.cswgs(g2, OPTICS, s2, 8, 0.1, 11, lut=lut, gray=a2)
        b1, b2 = lut.new_image(g1), lut.new_image(g2)
        jobs = [hg.DeviceJob.from_spots(g1, OPTICS, s1, 20, 1 / 16, 0, lut=lut, gray=b1),
                hg.DeviceJob.from_spots(g2, OPTICS, s2, 8, 0.1, 11, lut=lut, gray=b2)]
        hg.cswgs_batch(jobs)
        torch.cuda.synchronize()
        assert torch.equal(a1, b1) and torch.equal(a2, b2)
        c1 = lut.new_image(g1)
        eng = hg.Engine(1 << 30, max_slots=4)
        try:
            phi = torch.empty(g1.M, dtype=torch.float32, device="cuda")
            t = eng.submit(g1, OPTICS, s1, 20, 1 / 16, 0, phi, lut=lut, gray=c1)
            steps = 0
            while not eng.poll(t):
                eng.step()
                steps += 1
                assert steps < 1000
            torch.cuda.synchronize()
        finally:
            eng.close()
        assert torch.equal(a1, c1)
    finally:
        lut.close()
