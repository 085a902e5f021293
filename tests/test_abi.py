"""CPU checks of the C ABI: libhg.so loads, exports every function declared
in include/hg.h, and rejects invalid arguments before touching the GPU
(argument validation runs before any HIP call, so these run without one)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2003_05293_amd as hg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hg.lib_path()):
        from paper_2003_05293_amd import build
        build.build()
    return hg.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 13
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version(lib):
    assert "gfx950" in hg.version()


def _args(W=64, H=48, pitch=9.2e-3, lam=0.488e-3, f=20.0, n=3, x=None, amp=None, waist=0.0,
          aperture=0.0):
    g = hg._Grid(W, H, pitch)
    o = hg._Optics(lam, f, waist, aperture)
    xs = np.zeros(n) if x is None else np.asarray(x, dtype=np.float64)
    a = np.full(n, 0.5) if amp is None else np.asarray(amp, dtype=np.float64)
    keep = [xs, np.zeros(n), np.zeros(n), a]
    s = hg._Spots(n, *[k.ctypes.data_as(hg._DP) for k in keep])
    return g, o, s, keep


def call_rs(lib, g, o, s, phi=1):
    return lib.hg_rs(ctypes.byref(g), ctypes.byref(o), ctypes.byref(s), 1,
                     ctypes.c_void_p(phi) if phi else None, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(W=0), "W and H"),
    (dict(H=9000), "W and H"),
    (dict(pitch=0.0), "pitch"),
    (dict(pitch=math.inf), "pitch"),
    (dict(lam=-1.0), "lambda"),
    (dict(f=math.nan), "focal"),
    (dict(n=0), "spot count"),
    (dict(n=5000), "spot count"),
    (dict(x=[0.0, math.nan, 0.0]), "coordinates"),
    (dict(amp=[0.5, 0.0, 0.5]), "amplitudes"),
    (dict(amp=[0.5, -1.0, 0.5]), "amplitudes"),
    (dict(waist=-1.0), "waist_mm"),
    (dict(waist=math.nan), "waist_mm"),
    (dict(aperture=-2.0), "aperture_px"),
    (dict(aperture=math.inf), "aperture_px"),
    # even W and H: the nearest pixel centres have Lx^2 + Ly^2 = 2 > 1.4^2
    (dict(aperture=1.4), "no pixel"),
])
def test_rs_rejects(lib, kw, msg):
    g, o, s, keep = _args(**kw)
    assert call_rs(lib, g, o, s) == 1
    assert msg in hg.last_error()


def test_null_arguments(lib):
    g, o, s, keep = _args()
    assert lib.hg_rs(None, ctypes.byref(o), ctypes.byref(s), 1, ctypes.c_void_p(1), None) == 1
    assert call_rs(lib, g, o, s, phi=0) == 1
    assert "phi_dev" in hg.last_error()


def test_iteration_and_compression_limits(lib):
    g, o, s, keep = _args()
    G, O, S = ctypes.byref(g), ctypes.byref(o), ctypes.byref(s)
    p = ctypes.c_void_p(1)
    assert lib.hg_wgs(G, O, S, -1, 1, p, None) == 1
    assert lib.hg_wgs(G, O, S, 100001, 1, p, None) == 1
    for c in (0.0, -0.5, 1.5, math.nan):
        assert lib.hg_cswgs(G, O, S, 10, c, 1, p, None) == 1
        assert "compression" in hg.last_error()
    params = hg._Params(10, 0.5, 1, 7, None)
    assert lib.hg_cswgs_ex(G, O, S, ctypes.byref(params), p, None) == 1
    assert "flags" in hg.last_error()
    assert lib.hg_cswgs_ex(G, O, S, None, p, None) == 1


def test_static_entry_point_validation(lib):
    """hg_cswgs_static takes device-resident spots and no trace; both, and
    every check of hg_cswgs_ex, are rejected before any HIP call."""
    g, o, s, keep = _args()
    G, O, S = ctypes.byref(g), ctypes.byref(o), ctypes.byref(s)
    p = ctypes.c_void_p(1)
    params = hg._Params(10, 0.5, 1, hg.PREC_FP32, None)
    assert lib.hg_cswgs_static(G, O, S, ctypes.byref(params), p, None) == 1
    assert "HG_SPOTS_ON_DEVICE" in hg.last_error()
    trace = np.zeros(10 * 3 * 2)
    params = hg._Params(10, 0.5, 1, hg.PREC_FP32 | hg.SPOTS_ON_DEVICE,
                        trace.ctypes.data_as(hg._DP))
    assert lib.hg_cswgs_static(G, O, S, ctypes.byref(params), p, None) == 1
    assert "trace" in hg.last_error()
    params = hg._Params(10, 1.5, 1, hg.PREC_FP32 | hg.SPOTS_ON_DEVICE, None)
    assert lib.hg_cswgs_static(G, O, S, ctypes.byref(params), p, None) == 1
    assert "compression" in hg.last_error()
    params = hg._Params(10, 0.5, 1, 7 | hg.SPOTS_ON_DEVICE, None)
    assert lib.hg_cswgs_static(G, O, S, ctypes.byref(params), p, None) == 1
    assert "flags" in hg.last_error()
    assert lib.hg_cswgs_static(G, O, S, None, p, None) == 1
    params = hg._Params(10, 0.5, 1, hg.PREC_FP32 | hg.SPOTS_ON_DEVICE, None)
    assert lib.hg_cswgs_static(G, O, S, ctypes.byref(params), None, None) == 1
    assert "phi" in hg.last_error()


def test_test_hook_validation(lib):
    g, o, s, keep = _args()
    G, O, S = ctypes.byref(g), ctypes.byref(o), ctypes.byref(s)
    out = np.zeros(8)
    assert lib.hg_theta0(1, 0, out.ctypes.data_as(hg._DP)) == 1
    assert lib.hg_theta0(1, 4097, out.ctypes.data_as(hg._DP)) == 1
    m = ctypes.c_int32()
    assert lib.hg_subset(G, None, 1, 0, 0.5, ctypes.c_void_p(1), ctypes.byref(m), None) == 1
    assert lib.hg_subset(G, O, 1, 1, 0.0, ctypes.c_void_p(1), ctypes.byref(m), None) == 1
    bad = hg._Optics(0.488e-3, 20.0, 0.0, math.nan)
    assert lib.hg_subset(G, ctypes.byref(bad), 1, 1, 0.5, ctypes.c_void_p(1), ctypes.byref(m),
                         None) == 1
    assert "aperture_px" in hg.last_error()
    V = np.zeros(6)
    # idx given with m out of range
    assert lib.hg_forward(G, O, S, ctypes.c_void_p(1), ctypes.c_void_p(1), 0, 0,
                          V.ctypes.data_as(hg._DP), None) == 1
    assert lib.hg_forward(G, O, S, ctypes.c_void_p(1), ctypes.c_void_p(1), 64 * 48 + 1, 0,
                          V.ctypes.data_as(hg._DP), None) == 1
    w = np.array([1.0, 0.0, 1.0])
    th = np.zeros(3)
    assert lib.hg_step(G, O, S, w.ctypes.data_as(hg._DP), th.ctypes.data_as(hg._DP), None, 0,
                       0, V.ctypes.data_as(hg._DP), None) == 1
    assert "w must be positive" in hg.last_error()
    e, u = ctypes.c_double(), ctypes.c_double()
    assert lib.hg_metrics(G, O, S, None, ctypes.byref(e), ctypes.byref(u), None, None) == 1


def test_binding_rejects_wrong_types():
    from workload import Grid, OPTICS, spot_cloud
    g = Grid(16, 16)
    s = spot_cloud(0, 3, g)
    with pytest.raises((TypeError, ValueError)):
        hg.backward(g, OPTICS, s, np.ones(2), np.zeros(3))
    with pytest.raises(ValueError):
        hg.cswgs(g, OPTICS, s, 3, 0.5, 1, phi=np.zeros(256, np.float32), precision="fp8")


def test_lut_validation(lib):
    gray = np.arange(256, dtype=np.uint16)
    P16 = ctypes.POINTER(ctypes.c_uint16)
    h = ctypes.c_void_p()
    for levels, bits in ((0, 8), (65537, 16), (256, 12)):
        assert lib.hg_lut_create(gray.ctypes.data_as(P16), levels, bits, ctypes.byref(h)) == 1
    big = np.full(4, 300, dtype=np.uint16)
    assert lib.hg_lut_create(big.ctypes.data_as(P16), 4, 8, ctypes.byref(h)) == 1
    assert "255" in hg.last_error()
    assert lib.hg_lut_create(None, 4, 8, ctypes.byref(h)) == 1
    assert lib.hg_lut_destroy(None) == 0
    assert lib.hg_phase_to_gray(None, ctypes.c_void_p(1), 4, ctypes.c_void_p(1), None) == 1
    # a table without an image (and the reverse) is rejected before any GPU work
    g, o, s, keep = _args()
    for lut, img in ((ctypes.c_void_p(8), None), (None, ctypes.c_void_p(8))):
        params = hg._Params(3, 0.5, 1, 0, None, hg._Tune(0, 0, 0, 0), lut, img)
        assert lib.hg_cswgs_ex(ctypes.byref(g), ctypes.byref(o), ctypes.byref(s),
                               ctypes.byref(params), ctypes.c_void_p(1), None) == 1
        assert "lut and gray_dev" in hg.last_error()
