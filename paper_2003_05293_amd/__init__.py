"""Python binding of libhg (include/hg.h): RS, WGS and CS-WGS holograms of
3-D spot clouds on AMD MI355X.

This module only marshals arguments: it converts grid/optics/spot objects
to the C structs, passes device pointers of torch tensors and the current
HIP stream, and turns non-zero status codes into HGError.  Every step of
the computation runs in the library's HIP kernels.  If libhg.so has not been
built, every call raises: there is no fallback path.

Grid, optics and spot arguments are duck-typed: any object with
  grid:   W, H, pitch_mm
  optics: lambda_mm, focal_mm (and optionally waist_mm, aperture_px: the
          pupil; 0 or absent means uniform illumination on the whole grid)
  spots:  x_mm, y_mm, z_mm, amp  (array-likes of equal length)
works (for example the classes of the workload package).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "HGError", "lib_path", "load", "version", "last_error", "release",
    "rs", "wgs", "cswgs", "metrics", "theta0", "subset", "forward", "backward", "step",
    "PREC_FP32", "PREC_MIXED", "cswgs_device", "cswgs_static", "timing_enable", "timing_reset", "timing_read",
    "DeviceJob", "cswgs_batch", "Batch", "Engine", "Lut", "phase_to_gray",
]

PREC_FP32 = 0
PREC_MIXED = 1
SPOTS_ON_DEVICE = 0x100
FULL_DIRECT = 0x200
_PREC = {"fp32": PREC_FP32, "mixed": PREC_MIXED}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhg.so")
_lib = None

STATUS = {0: "HG_OK", 1: "HG_EINVAL", 2: "HG_ENOMEM", 3: "HG_EBUSY", 4: "HG_ENUMERIC",
          5: "HG_EDEVICE"}


class HGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32), ("pitch_mm", ctypes.c_double)]


class _Optics(ctypes.Structure):
    _fields_ = [("lambda_mm", ctypes.c_double), ("focal_mm", ctypes.c_double),
                ("waist_mm", ctypes.c_double), ("aperture_px", ctypes.c_double)]


_DP = ctypes.POINTER(ctypes.c_double)


class _Spots(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("x_mm", _DP), ("y_mm", _DP), ("z_mm", _DP), ("amp", _DP)]


class _Job(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("optics", _Optics), ("spots", _Spots),
                ("iterations", ctypes.c_int32), ("compression", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("phi_dev", ctypes.c_void_p), ("trace_V", _DP),
                ("lut", ctypes.c_void_p), ("gray_dev", ctypes.c_void_p)]


class _Tune(ctypes.Structure):
    _fields_ = [("full_block_cap", ctypes.c_int32), ("subset_block_cap", ctypes.c_int32),
                ("pass_form", ctypes.c_int32), ("chain_passes", ctypes.c_int32)]


class _EngineConfig(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("tune", _Tune)]


class _Params(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("compression", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("trace_V", _DP),
                ("tune", _Tune), ("lut", ctypes.c_void_p), ("gray_dev", ctypes.c_void_p)]


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Loads libhg.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"libhg.so not found at {_LIB_PATH}; build it with "
                           "`python -m paper_2003_05293_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    c = ctypes
    vp, i32, u32, u64, dbl = c.c_void_p, c.c_int32, c.c_uint32, c.c_uint64, c.c_double
    G, O, S = c.POINTER(_Grid), c.POINTER(_Optics), c.POINTER(_Spots)
    sig = {
        "hg_rs": [G, O, S, u64, vp, vp],
        "hg_wgs": [G, O, S, i32, u64, vp, vp],
        "hg_cswgs": [G, O, S, i32, dbl, u64, vp, vp],
        "hg_cswgs_ex": [G, O, S, c.POINTER(_Params), vp, vp],
        "hg_cswgs_static": [G, O, S, c.POINTER(_Params), vp, vp],
        "hg_metrics": [G, O, S, vp, _DP, _DP, _DP, vp],
        "hg_theta0": [u64, i32, _DP],
        "hg_subset": [G, O, u64, i32, dbl, vp, c.POINTER(i32), vp],
        "hg_forward": [G, O, S, vp, vp, i32, u32, _DP, vp],
        "hg_backward": [G, O, S, _DP, _DP, vp, i32, u32, vp, vp],
        "hg_step": [G, O, S, _DP, _DP, vp, i32, u32, _DP, vp],
        "hg_release": [],
        "hg_cswgs_batch": [i32, c.POINTER(_Job), c.POINTER(_Tune), vp],
        "hg_batch_create": [i32, c.POINTER(_Job), c.POINTER(_Tune), i32, c.POINTER(vp)],
        "hg_batch_run": [vp, vp],
        "hg_batch_destroy": [vp],
        "hg_engine_create": [c.POINTER(_EngineConfig), c.POINTER(vp)],
        "hg_engine_submit": [vp, c.POINTER(_Job), c.POINTER(u64)],
        "hg_engine_step": [vp, vp, c.POINTER(i32)],
        "hg_engine_poll": [vp, u64, c.POINTER(i32)],
        "hg_engine_destroy": [vp],
        "hg_timing_enable": [c.c_int],
        "hg_timing_reset": [],
        "hg_timing_read": [c.c_char_p, _DP, c.POINTER(c.c_int64)],
        "hg_lut_create": [c.POINTER(c.c_uint16), i32, i32, c.POINTER(vp)],
        "hg_lut_destroy": [vp],
        "hg_phase_to_gray": [vp, vp, c.c_int64, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c.c_int
    lib.hg_last_error.restype = c.c_char_p
    lib.hg_last_error.argtypes = []
    lib.hg_version.restype = c.c_char_p
    lib.hg_version.argtypes = []
    _lib = lib
    atexit.register(_release_at_exit)
    return lib


# Library objects (batches with their graphs, engines, tables) still open;
# closed at interpreter exit, before the HIP runtime's own teardown.
_OPEN = weakref.WeakSet()


def _release_at_exit():
    """Closes the open batches, engines and tables, then frees the library's
    per-stream scratch (hg_release synchronises the device first), so that
    nothing of the library is left for the process's exit-time teardown."""
    if _lib is None:
        return
    for obj in list(_OPEN):
        try:
            obj.close()
        except Exception:
            pass
    try:
        _lib.hg_release()
    except Exception:
        pass


def version() -> str:
    return load().hg_version().decode()


def last_error() -> str:
    return load().hg_last_error().decode()


def _check(status: int):
    if status != 0:
        raise HGError(status, last_error())


def release():
    _check(load().hg_release())


# ----------------------------------------------------------- marshalling ---

def _grid(g) -> _Grid:
    return _Grid(int(g.W), int(g.H), float(g.pitch_mm))


def _optics(o) -> _Optics:
    return _Optics(float(o.lambda_mm), float(o.focal_mm),
                   float(getattr(o, "waist_mm", 0.0)), float(getattr(o, "aperture_px", 0.0)))


class _SpotArgs:
    """Keeps contiguous float64 copies alive for the duration of a call."""

    def __init__(self, s):
        self.arrays = [np.ascontiguousarray(getattr(s, k), dtype=np.float64)
                       for k in ("x_mm", "y_mm", "z_mm", "amp")]
        n = self.arrays[0].shape[0]
        for a in self.arrays:
            if a.ndim != 1 or a.shape[0] != n:
                raise ValueError("spot arrays must be 1-D and of equal length")
        self.n = n
        self.struct = _Spots(n, *[a.ctypes.data_as(_DP) for a in self.arrays])


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(t, numel: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 torch tensor on the GPU")
    if not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{name} must be contiguous with at least {numel} elements")
    return ctypes.c_void_p(t.data_ptr())


def _dev_i32(t, name: str):
    import torch
    if t is None:
        return None, 0
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda:
        raise TypeError(f"{name} must be an int32 torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr()), int(t.numel())


def _new_phi(grid, numel=None):
    import torch
    return torch.empty(int(numel if numel is not None else grid.W * grid.H),
                       dtype=torch.float32, device="cuda")


def _flags(precision: str) -> int:
    try:
        return _PREC[precision]
    except KeyError:
        raise ValueError(f"precision must be one of {sorted(_PREC)}") from None


def _f64(a, n: int, name: str):
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if arr.shape != (n,):
        raise ValueError(f"{name} must have shape ({n},)")
    return arr


# ------------------------------------------------------------------ calls ---

def rs(grid, optics, spots, seed: int, phi=None, stream=None):
    """Random superposition hologram (eq. 1).  Returns phi (float32 [H*W])."""
    lib = load()
    phi = _new_phi(grid) if phi is None else phi
    sa = _SpotArgs(spots)
    _check(lib.hg_rs(_grid(grid), _optics(optics), sa.struct, int(seed),
                     _dev_f32(phi, grid.W * grid.H, "phi"), _stream(stream)))
    return phi


def wgs(grid, optics, spots, iterations: int, seed: int, phi=None, stream=None):
    """Weighted Gerchberg-Saxton hologram after `iterations` iterations."""
    lib = load()
    phi = _new_phi(grid) if phi is None else phi
    sa = _SpotArgs(spots)
    _check(lib.hg_wgs(_grid(grid), _optics(optics), sa.struct, int(iterations), int(seed),
                      _dev_f32(phi, grid.W * grid.H, "phi"), _stream(stream)))
    return phi


def cswgs(grid, optics, spots, iterations: int, compression: float, seed: int, phi=None,
          stream=None, precision: str = "fp32", trace: bool = False, direct: bool = False,
          tune=None, lut=None, gray=None):
    """Compressed-sensing WGS hologram.  With trace=True returns (phi, V)
    where V[j-1] is the complex spot field of iteration j.  direct=True
    computes the full-grid passes with the per-pixel kernels.  tune: launch
    geometry {"full_block_cap", "subset_block_cap"} (see autotune).  lut (a
    Lut) and gray (a uint8 or int16 GPU tensor of W*H elements, by the
    table's bits): the final pass also writes the SLM's gray image."""
    lib = load()
    phi = _new_phi(grid) if phi is None else phi
    sa = _SpotArgs(spots)
    flags = _flags(precision) | (FULL_DIRECT if direct else 0)
    lp, gp = _lut_args(lut, gray, grid)
    if precision == "fp32" and not trace and not direct and tune is None and lut is None:
        _check(lib.hg_cswgs(_grid(grid), _optics(optics), sa.struct, int(iterations),
                            float(compression), int(seed),
                            _dev_f32(phi, grid.W * grid.H, "phi"), _stream(stream)))
        return phi
    tr = np.zeros((max(int(iterations), 1), sa.n, 2)) if trace else None
    params = _Params(int(iterations), float(compression), int(seed), flags,
                     tr.ctypes.data_as(_DP) if trace else None, _tune(tune) or _Tune(0, 0, 0, 0),
                     lp, gp)
    _check(lib.hg_cswgs_ex(_grid(grid), _optics(optics), sa.struct, ctypes.byref(params),
                           _dev_f32(phi, grid.W * grid.H, "phi"), _stream(stream)))
    if trace:
        return phi, (tr[..., 0] + 1j * tr[..., 1])[:int(iterations)]
    return phi


class Lut:
    """The SLM's phase-to-gray table on the GPU (hg_lut_create): gray values
    of `levels` equal phase bins covering one period; bits 8 or 16 sets the
    element type of the gray images."""

    def __init__(self, table, bits: int = 8):
        lib = load()
        arr = np.ascontiguousarray(table, dtype=np.uint16)
        if arr.ndim != 1:
            raise ValueError("table must be one-dimensional")
        h = ctypes.c_void_p()
        _check(lib.hg_lut_create(arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                 int(arr.shape[0]), int(bits), ctypes.byref(h)))
        self._h, self.levels, self.bits = h, int(arr.shape[0]), int(bits)
        _OPEN.add(self)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("the table has been closed")
        return self._h

    def new_image(self, grid):
        """An empty gray image of the grid, of the table's element type."""
        import torch
        return torch.empty(grid.W * grid.H, dtype=torch.uint8 if self.bits == 8 else torch.int16,
                           device="cuda")

    def close(self):
        if self._h:
            _check(load().hg_lut_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _gray_ptr(gray, lut, count: int, name: str = "gray"):
    import torch
    want = torch.uint8 if lut.bits == 8 else torch.int16
    if (not isinstance(gray, torch.Tensor) or not gray.is_cuda or gray.dtype != want
            or gray.numel() != count or not gray.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {want} GPU tensor of {count} elements")
    return ctypes.c_void_p(gray.data_ptr())


def _lut_args(lut, gray, grid):
    if lut is None and gray is None:
        return None, None
    if lut is None or gray is None:
        raise ValueError("lut and gray go together")
    return lut.handle, _gray_ptr(gray, lut, grid.W * grid.H)


def phase_to_gray(lut, phi, gray=None, stream=None):
    """Gray image of a hologram phi (float32 GPU tensor) through the table."""
    lib = load()
    count = int(phi.numel())
    if gray is None:
        import torch
        gray = torch.empty(count, dtype=torch.uint8 if lut.bits == 8 else torch.int16,
                           device="cuda")
    _check(lib.hg_phase_to_gray(lut.handle, _dev_f32(phi, count, "phi"), count,
                                _gray_ptr(gray, lut, count), _stream(stream)))
    return gray


def metrics(grid, optics, spots, phi, stream=None) -> Tuple[float, float, np.ndarray]:
    """FP64 efficiency e, uniformity u and spot intensities of a hologram."""
    lib = load()
    sa = _SpotArgs(spots)
    e, u = ctypes.c_double(), ctypes.c_double()
    inten = np.zeros(sa.n)
    _check(lib.hg_metrics(_grid(grid), _optics(optics), sa.struct,
                          _dev_f32(phi, grid.W * grid.H, "phi"), ctypes.byref(e),
                          ctypes.byref(u), inten.ctypes.data_as(_DP), _stream(stream)))
    return e.value, u.value, inten


def theta0(seed: int, n: int) -> np.ndarray:
    """Initial phases theta_n^0 (radians) computed on the GPU."""
    lib = load()
    out = np.zeros(int(n))
    _check(lib.hg_theta0(int(seed), int(n), out.ctypes.data_as(_DP)))
    return out


def subset(grid, seed: int, j: int, compression: float, stream=None, optics=None):
    """Pixel indices of Omega^j as an int32 GPU tensor (within the aperture of
    `optics`, if given)."""
    import torch
    lib = load()
    m_cap = int(np.ceil(float(compression) * grid.W * grid.H))
    idx = torch.empty(max(m_cap, 1), dtype=torch.int32, device="cuda")
    m = ctypes.c_int32()
    opt = ctypes.byref(_optics(optics)) if optics is not None else None
    _check(lib.hg_subset(_grid(grid), opt, int(seed), int(j), float(compression),
                         ctypes.c_void_p(idx.data_ptr()), ctypes.byref(m), _stream(stream)))
    return idx[:m.value]


def forward(grid, optics, spots, phi, idx=None, precision: str = "fp32",
            stream=None) -> np.ndarray:
    """Spot fields V_n (eq. 3) of the hologram phi over idx (default all)."""
    lib = load()
    sa = _SpotArgs(spots)
    ip, m = _dev_i32(idx, "idx")
    V = np.zeros(2 * sa.n)
    _check(lib.hg_forward(_grid(grid), _optics(optics), sa.struct,
                          _dev_f32(phi, grid.W * grid.H, "phi"), ip, m, _flags(precision),
                          V.ctypes.data_as(_DP), _stream(stream)))
    return V[0::2] + 1j * V[1::2]


def backward(grid, optics, spots, w, theta, idx=None, out=None, precision: str = "fp32",
             stream=None, direct: bool = False):
    """Phi (eq. 1) with weights w and phases theta at idx (compact) or at
    all pixels (separable products unless direct=True)."""
    lib = load()
    sa = _SpotArgs(spots)
    w = _f64(w, sa.n, "w")
    th = _f64(theta, sa.n, "theta")
    ip, m = _dev_i32(idx, "idx")
    count = m if idx is not None else grid.W * grid.H
    out = _new_phi(grid, count) if out is None else out
    _check(lib.hg_backward(_grid(grid), _optics(optics), sa.struct, w.ctypes.data_as(_DP),
                           th.ctypes.data_as(_DP), ip, m,
                           _flags(precision) | (FULL_DIRECT if direct else 0),
                           _dev_f32(out, count, "out"), _stream(stream)))
    return out


def step(grid, optics, spots, w, theta, idx=None, precision: str = "fp32",
         stream=None, direct: bool = False) -> np.ndarray:
    """One fused iteration body: back-propagate (w, theta) on the pixel set
    and return the forward spot fields over the same set (the full grid uses
    the separable products unless direct=True)."""
    lib = load()
    sa = _SpotArgs(spots)
    w = _f64(w, sa.n, "w")
    th = _f64(theta, sa.n, "theta")
    ip, m = _dev_i32(idx, "idx")
    V = np.zeros(2 * sa.n)
    _check(lib.hg_step(_grid(grid), _optics(optics), sa.struct, w.ctypes.data_as(_DP),
                       th.ctypes.data_as(_DP), ip, m,
                       _flags(precision) | (FULL_DIRECT if direct else 0),
                       V.ctypes.data_as(_DP), _stream(stream)))
    return V[0::2] + 1j * V[1::2]


def cswgs_device(grid, optics, spots_dev, iterations: int, compression: float, seed: int,
                 phi=None, stream=None, precision: str = "fp32", tune=None, lut=None, gray=None):
    """CS-WGS with the spot arrays already on the GPU: spots_dev is a float64
    GPU tensor of shape (4, N) holding x_mm, y_mm, z_mm, amp.  lut, gray: as
    in cswgs."""
    import torch
    lib = load()
    if (not isinstance(spots_dev, torch.Tensor) or spots_dev.dtype != torch.float64
            or not spots_dev.is_cuda or spots_dev.dim() != 2 or spots_dev.shape[0] != 4
            or not spots_dev.is_contiguous()):
        raise TypeError("spots_dev must be a contiguous float64 GPU tensor of shape (4, N)")
    n = int(spots_dev.shape[1])
    base = spots_dev.data_ptr()
    ptrs = [ctypes.cast(ctypes.c_void_p(base + 8 * n * k), _DP) for k in range(4)]
    sp = _Spots(n, *ptrs)
    phi = _new_phi(grid) if phi is None else phi
    lp, gp = _lut_args(lut, gray, grid)
    params = _Params(int(iterations), float(compression), int(seed),
                     _flags(precision) | SPOTS_ON_DEVICE, None, _tune(tune) or _Tune(0, 0, 0, 0),
                     lp, gp)
    _check(lib.hg_cswgs_ex(_grid(grid), _optics(optics), sp, ctypes.byref(params),
                           _dev_f32(phi, grid.W * grid.H, "phi"), _stream(stream)))
    return phi


def cswgs_static(grid, optics, spots_dev, iterations: int, compression: float, seed: int, phi,
                 stream=None, precision: str = "fp32", tune=None, lut=None, gray=None):
    """cswgs_device through hg_cswgs_static: the library allocates nothing
    and works in its static per-GPU scratch (calls that overlap on one GPU
    race).  phi (float32 GPU tensor of W*H) and, with lut, gray are the
    caller's; spots_dev as in cswgs_device."""
    import torch
    lib = load()
    if (not isinstance(spots_dev, torch.Tensor) or spots_dev.dtype != torch.float64
            or not spots_dev.is_cuda or spots_dev.dim() != 2 or spots_dev.shape[0] != 4
            or not spots_dev.is_contiguous()):
        raise TypeError("spots_dev must be a contiguous float64 GPU tensor of shape (4, N)")
    if phi is None:
        raise TypeError("phi must be given: cswgs_static allocates nothing")
    n = int(spots_dev.shape[1])
    base = spots_dev.data_ptr()
    ptrs = [ctypes.cast(ctypes.c_void_p(base + 8 * n * k), _DP) for k in range(4)]
    sp = _Spots(n, *ptrs)
    lp, gp = _lut_args(lut, gray, grid)
    params = _Params(int(iterations), float(compression), int(seed),
                     _flags(precision) | SPOTS_ON_DEVICE, None, _tune(tune) or _Tune(0, 0, 0, 0),
                     lp, gp)
    _check(lib.hg_cswgs_static(_grid(grid), _optics(optics), sp, ctypes.byref(params),
                               _dev_f32(phi, grid.W * grid.H, "phi"), _stream(stream)))
    return phi


def timing_enable(on: bool = True):
    """Bracket every iteration-kernel launch with HIP events (benchmarks)."""
    _check(load().hg_timing_enable(1 if on else 0))


def timing_reset():
    _check(load().hg_timing_reset())


def timing_read(name: str):
    """(total ms, launches) of a kernel family since the last reset."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(load().hg_timing_read(name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


# ---------------------------------------------------------------- batches ---

class DeviceJob:
    """One hologram of a batch with its spot arrays and output on the GPU.

    spots_dev: float64 GPU tensor (4, N) holding x_mm, y_mm, z_mm, amp;
    phi: float32 GPU tensor of W*H elements (allocated if None)."""

    def __init__(self, grid, optics, spots_dev, iterations: int, compression: float, seed: int,
                 phi=None, precision: str = "fp32", lut=None, gray=None):
        import torch
        if (not isinstance(spots_dev, torch.Tensor) or spots_dev.dtype != torch.float64
                or not spots_dev.is_cuda or spots_dev.dim() != 2 or spots_dev.shape[0] != 4
                or not spots_dev.is_contiguous()):
            raise TypeError("spots_dev must be a contiguous float64 GPU tensor of shape (4, N)")
        self.grid, self.optics, self.spots_dev = grid, optics, spots_dev
        self.iterations, self.compression, self.seed = int(iterations), float(compression), int(seed)
        self.phi = _new_phi(grid) if phi is None else phi
        self.flags = _flags(precision) | SPOTS_ON_DEVICE
        self.lut, self.gray = lut, gray
        _lut_args(lut, gray, grid)  # checks the pair

    @classmethod
    def from_spots(cls, grid, optics, spots, iterations, compression, seed, **kw):
        import torch
        dev = torch.tensor(np.stack([np.asarray(spots.x_mm), np.asarray(spots.y_mm),
                                     np.asarray(spots.z_mm), np.asarray(spots.amp)]),
                           dtype=torch.float64, device="cuda")
        return cls(grid, optics, dev, iterations, compression, seed, **kw)

    def _struct(self) -> _Job:
        n = int(self.spots_dev.shape[1])
        base = self.spots_dev.data_ptr()
        ptrs = [ctypes.cast(ctypes.c_void_p(base + 8 * n * k), _DP) for k in range(4)]
        lp, gp = _lut_args(self.lut, self.gray, self.grid)
        return _Job(_grid(self.grid), _optics(self.optics), _Spots(n, *ptrs), self.iterations,
                    self.compression, self.seed, self.flags,
                    _dev_f32(self.phi, self.grid.W * self.grid.H, "phi"), None, lp, gp)


def _tune(tune):
    if tune is None:
        return None
    if isinstance(tune, dict):
        return _Tune(int(tune.get("full_block_cap", 0)), int(tune.get("subset_block_cap", 0)),
                     int(tune.get("pass_form", 0)), int(tune.get("chain_passes", 0)))
    return _Tune(*(int(v) for v in tune))


def cswgs_batch(jobs, tune=None, stream=None):
    """Runs a list of DeviceJob together (one launch per iteration round)."""
    lib = load()
    arr = (_Job * len(jobs))(*[j._struct() for j in jobs])
    t = _tune(tune)
    _check(lib.hg_cswgs_batch(len(jobs), arr, ctypes.byref(t) if t else None, _stream(stream)))
    return [j.phi for j in jobs]


class Batch:
    """A reusable batch (planned once; runs replay a captured HIP graph when
    use_graph).  Keep the DeviceJob objects alive while the batch exists."""

    def __init__(self, jobs, tune=None, use_graph: bool = True):
        lib = load()
        self.jobs = list(jobs)
        arr = (_Job * len(self.jobs))(*[j._struct() for j in self.jobs])
        t = _tune(tune)
        h = ctypes.c_void_p()
        _check(lib.hg_batch_create(len(self.jobs), arr, ctypes.byref(t) if t else None,
                                   1 if use_graph else 0, ctypes.byref(h)))
        self._h = h
        _OPEN.add(self)

    def run(self, stream=None):
        _check(load().hg_batch_run(self._h, _stream(stream)))

    def close(self):
        if self._h:
            _check(load().hg_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- serving ---

class Engine:
    """Continuous-batching engine (hg_engine_*).  submit() queues a request
    (host spot arrays are copied; the phi tensor must stay alive until the
    request is done), step() admits and advances every request by one
    iteration on the given stream, poll() reports completion."""

    def __init__(self, mem_budget_bytes: int, max_slots: int = 64, tune=None):
        lib = load()
        t = _tune(tune) or _Tune(0, 0, 0, 0)
        cfg = _EngineConfig(int(mem_budget_bytes), int(max_slots), t)
        h = ctypes.c_void_p()
        _check(lib.hg_engine_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        _OPEN.add(self)
        self._keep = {}

    def submit(self, grid, optics, spots, iterations: int, compression: float, seed: int,
               phi, precision: str = "fp32", lut=None, gray=None) -> int:
        sa = _SpotArgs(spots)
        lp, gp = _lut_args(lut, gray, grid)
        job = _Job(_grid(grid), _optics(optics), sa.struct, int(iterations), float(compression),
                   int(seed), _flags(precision), _dev_f32(phi, grid.W * grid.H, "phi"), None,
                   lp, gp)
        t = ctypes.c_uint64()
        _check(load().hg_engine_submit(self._h, ctypes.byref(job), ctypes.byref(t)))
        self._keep[t.value] = (phi, gray, lut)
        return t.value

    def step(self, stream=None) -> int:
        n = ctypes.c_int32()
        _check(load().hg_engine_step(self._h, _stream(stream), ctypes.byref(n)))
        return n.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(load().hg_engine_poll(self._h, int(ticket), ctypes.byref(d)))
        if d.value:
            self._keep.pop(int(ticket), None)
        return bool(d.value)

    def close(self):
        if self._h:
            _check(load().hg_engine_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
