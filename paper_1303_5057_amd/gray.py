"""Python binding of libgray (include/gray.h): argument marshalling only.

Every step of the hot path runs in the HIP kernels of libgray.so; this module
mirrors the ABI structs with ctypes, exposes the entry points under their C
names, and offers ``Batch``, a small helper that owns the device buffers of
one batch of photons as torch tensors (torch is used for device memory and
streams only).

There is no CPU fallback: if libgray.so is missing this module raises on
import of the library, and every call that fails on the device raises
``GrayError``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

from .workloads import Camera, Params

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgray.so")

GRAY_OK, GRAY_EINVAL, GRAY_EDEVICE, GRAY_EWORKSPACE, GRAY_EUNSUPPORTED = 0, -1, -2, -3, -4
GRAY_FP64, GRAY_FP32C = 0, 1
RUNNING, CAPTURED, ESCAPED, UNFINISHED, NONFINITE = range(5)
GRAY_RECORD_DISK = 1
GRAY_SLOTS = 2
GRAY_WORKLIST = 4
GRAY_WORKLIST_SLACK = 1 << 20
# size of the library's static per-device workspace (gray_integrate_static)
GRAY_STATIC_WORKSPACE_BYTES = 32 << 20
PRECISIONS = {"fp64": GRAY_FP64, "fp32c": GRAY_FP32C}


GRAY_MAX_PHOTONS = 2147482623

# gray_params.pole_mode
GRAY_POLE_MONITOR, GRAY_POLE_EULER_CROSSING, GRAY_POLE_NONE = 0, 1, 2

# gray_camera.kind
GRAY_CAMERA_GRID = 0
GRAY_CAMERA_POLAR = 1

# gray_camera.metric
GRAY_METRIC_KERR = 0
GRAY_METRIC_DEFORMED = 1


class gray_camera(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("r_obs", ctypes.c_double), ("incl", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("alpha_lo", ctypes.c_double), ("alpha_hi", ctypes.c_double),
                ("beta_lo", ctypes.c_double), ("beta_hi", ctypes.c_double),
                ("first", ctypes.c_int64), ("kind", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("deform", ctypes.c_double), ("call_steps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gray_params(ctypes.Structure):
    _fields_ = [("step_frac", ctypes.c_double), ("horizon_eps", ctypes.c_double),
                ("r_escape", ctypes.c_double), ("xi_eps", ctypes.c_double),
                ("euler_div", ctypes.c_double), ("disk_rmin", ctypes.c_double),
                ("disk_rmax", ctypes.c_double), ("fp64_horizon", ctypes.c_double),
                ("fp64_pole", ctypes.c_double), ("fp64_turn", ctypes.c_double),
                ("max_steps", ctypes.c_int32),
                ("call_steps", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("pole_mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class gray_state(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("steps", ctypes.c_void_p), ("cam", ctypes.c_void_p), ("counters", ctypes.c_void_p),
                ("mark", ctypes.c_void_p), ("disk", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("stride", ctypes.c_int64), ("work_in", ctypes.c_void_p),
                ("work_out", ctypes.c_void_p), ("work_in_count", ctypes.c_void_p),
                ("work_out_count", ctypes.c_void_p), ("cam_done", ctypes.c_void_p),
                ("wave_iters", ctypes.c_void_p), ("stop", ctypes.c_void_p)]


class gray_result(ctypes.Structure):
    _fields_ = [("flag", ctypes.c_void_p), ("xf", ctypes.c_void_p), ("cons", ctypes.c_void_p),
                ("counts", ctypes.c_void_p)]


EXPORTS = ("gray_workspace_size", "gray_camera_init", "gray_camera_init_slot", "gray_integrate",
           "gray_integrate_static", "gray_classify", "gray_strerror", "gray_version",
           "gray_struct_size")


class GrayError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed: {msg} (code {code})")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libgray.so from the package directory (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1303_5057_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    C, P, S, R = (ctypes.POINTER(gray_camera), ctypes.POINTER(gray_params),
                  ctypes.POINTER(gray_state), ctypes.POINTER(gray_result))
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    L.gray_workspace_size.restype, L.gray_workspace_size.argtypes = sz, [i64, i32, P]
    L.gray_camera_init.restype, L.gray_camera_init.argtypes = ctypes.c_int, [C, i32, P, S, vp]
    L.gray_camera_init_slot.restype = ctypes.c_int
    L.gray_camera_init_slot.argtypes = [C, i32, i32, P, S, vp]
    L.gray_integrate.restype, L.gray_integrate.argtypes = ctypes.c_int, [C, i32, P, S, vp, sz, vp]
    L.gray_integrate_static.restype, L.gray_integrate_static.argtypes = ctypes.c_int, [C, i32, P, S, vp]
    L.gray_classify.restype, L.gray_classify.argtypes = ctypes.c_int, [C, i32, P, S, R, vp]
    L.gray_strerror.restype, L.gray_strerror.argtypes = ctypes.c_char_p, [ctypes.c_int]
    L.gray_version.restype, L.gray_version.argtypes = ctypes.c_int, []
    L.gray_struct_size.restype, L.gray_struct_size.argtypes = sz, [ctypes.c_int]
    for k, t in enumerate((gray_camera, gray_params, gray_state, gray_result)):
        if L.gray_struct_size(k) != ctypes.sizeof(t):
            raise ImportError(f"ABI mismatch for {t.__name__}: C {L.gray_struct_size(k)} bytes, "
                              f"binding {ctypes.sizeof(t)} bytes")
    _lib = L
    return L


def _check(fn: str, code: int) -> int:
    if code != GRAY_OK:
        raise GrayError(fn, code, load().gray_strerror(code).decode())
    return code


# ---------------------------------------------------------- C-named entry points
def gray_workspace_size(n: int, ncam: int, p: gray_params) -> int:
    return int(load().gray_workspace_size(n, ncam, ctypes.byref(p)))


def gray_camera_init(cams, ncam: int, p: gray_params, s: gray_state, stream: int = 0) -> int:
    return _check("gray_camera_init",
                  load().gray_camera_init(cams, ncam, ctypes.byref(p), ctypes.byref(s), stream))


def gray_camera_init_slot(cams, ncam: int, slot: int, p: gray_params, s: gray_state,
                          stream: int = 0) -> int:
    return _check("gray_camera_init_slot",
                  load().gray_camera_init_slot(cams, ncam, slot, ctypes.byref(p), ctypes.byref(s),
                                               stream))


def gray_integrate(cams, ncam: int, p: gray_params, s: gray_state, workspace: int,
                   workspace_bytes: int, stream: int = 0) -> int:
    return _check("gray_integrate",
                  load().gray_integrate(cams, ncam, ctypes.byref(p), ctypes.byref(s), workspace,
                                        workspace_bytes, stream))


def gray_integrate_static(cams, ncam: int, p: gray_params, s: gray_state, stream: int = 0) -> int:
    return _check("gray_integrate_static",
                  load().gray_integrate_static(cams, ncam, ctypes.byref(p), ctypes.byref(s), stream))


def gray_classify(cams, ncam: int, p: gray_params, s: gray_state, out: gray_result,
                  stream: int = 0) -> int:
    return _check("gray_classify",
                  load().gray_classify(cams, ncam, ctypes.byref(p), ctypes.byref(s),
                                       ctypes.byref(out), stream))


def gray_strerror(code: int) -> str:
    return load().gray_strerror(code).decode()


def gray_version() -> int:
    return int(load().gray_version())


# ----------------------------------------------------------------- marshalling
def camera_struct(c: Camera, first: int) -> gray_camera:
    return gray_camera(c.a, c.r_obs, c.incl, c.nx, c.ny, c.alpha_lo, c.alpha_hi, c.beta_lo,
                       c.beta_hi, first, c.kind, c.metric, c.deform)


def camera_array(cams: Sequence[Camera]):
    """ctypes array of gray_camera tiling photon ids [0, n) in order."""
    arr = (gray_camera * len(cams))()
    first = 0
    for k, c in enumerate(cams):
        arr[k] = camera_struct(c, first)
        first += c.nx * c.ny
    return arr


def params_struct(p: Params) -> gray_params:
    return gray_params(p.step_frac, p.horizon_eps, p.r_escape, p.xi_eps, p.euler_div, p.disk_rmin,
                       p.disk_rmax, p.fp64_horizon, p.fp64_pole, p.fp64_turn, p.max_steps,
                       p.call_steps, PRECISIONS[p.precision],
                       GRAY_RECORD_DISK if p.record_disk else 0, p.pole_mode, 0)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def current_stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


@dataclass
class Result:
    flag: "object"
    xf: "object" = None
    cons: "object" = None
    counts: "object" = None


class Batch:
    """Device buffers (torch tensors) for one batch of cameras, plus calls.

    Layout follows include/gray.h: component-major rows of `stride` elements.
    """

    def __init__(self, cams: Sequence[Camera], params: Params, device: str = "cuda",
                 counters: bool = True, mark: bool = True):
        import torch
        self.torch = torch
        self.cams = list(cams)
        self.params = params
        self.n = sum(c.nx * c.ny for c in self.cams)
        self.stride = max(64, (self.n + 63) // 64 * 64)
        self.device = device
        S = self.stride
        fp64 = params.precision == "fp64"
        dt = torch.float64 if fp64 else torch.float32
        self.x = torch.zeros(8 * S, dtype=dt, device=device)
        self.lo = None if fp64 else torch.zeros(8 * S, dtype=torch.float32, device=device)
        self.status = torch.zeros(S, dtype=torch.int32, device=device)
        self.steps = torch.zeros(S, dtype=torch.int32, device=device)
        self.cam = torch.zeros(S, dtype=torch.int32, device=device)
        self.counters = torch.zeros(3 * S, dtype=torch.int32, device=device) if counters else None
        self.mark = torch.zeros(8 * S, dtype=torch.float64, device=device) if mark else None
        self.disk = (torch.zeros(3 * S, dtype=torch.float64, device=device)
                     if params.record_disk else None)
        self.cam_arr = camera_array(self.cams)
        self.p = params_struct(params)
        ws = gray_workspace_size(self.n, len(self.cams), self.p)
        if ws == 0:
            raise GrayError("gray_workspace_size", GRAY_EINVAL, "invalid arguments")
        self._ws = torch.zeros(ws + 256, dtype=torch.uint8, device=device)
        off = (-self._ws.data_ptr()) % 256
        self.ws_ptr = self._ws.data_ptr() + off
        self.ws_bytes = ws
        # loop iterations of the integrator's waves (lane efficiency); the
        # integrator adds to it, callers zero it
        self.wave_iters = torch.zeros(1, dtype=torch.int64, device=device)
        self.state = gray_state(_ptr(self.x), _ptr(self.lo), _ptr(self.status), _ptr(self.steps),
                                _ptr(self.cam), _ptr(self.counters), _ptr(self.mark),
                                _ptr(self.disk), self.n, S)
        self.state.wave_iters = _ptr(self.wave_iters)

    def set_call_steps(self, k: int) -> None:
        self.p.call_steps = int(k)

    def set_stop_flag(self, ptr: Optional[int]) -> None:
        """Address of a uint32 stop request (gray_state.stop) that integrate
        calls read, or None: device memory, or host memory mapped for the
        device."""
        self.state.stop = ptr

    def camera_init(self, stream: Optional[int] = None) -> None:
        gray_camera_init(self.cam_arr, len(self.cams), self.p, self.state,
                         current_stream() if stream is None else stream)

    def integrate(self, stream: Optional[int] = None) -> None:
        gray_integrate(self.cam_arr, len(self.cams), self.p, self.state, self.ws_ptr, self.ws_bytes,
                       current_stream() if stream is None else stream)

    def integrate_static(self, stream: Optional[int] = None) -> None:
        """gray_integrate with the library's static workspace (no allocation)."""
        gray_integrate_static(self.cam_arr, len(self.cams), self.p, self.state,
                              current_stream() if stream is None else stream)

    def classify(self, xf: bool = True, cons: bool = True, counts: bool = True,
                 stream: Optional[int] = None) -> Result:
        torch = self.torch
        S = self.stride
        res = Result(flag=torch.zeros(S, dtype=torch.int8, device=self.device))
        if xf:
            res.xf = torch.zeros(8 * S, dtype=torch.float64, device=self.device)
        if cons:
            res.cons = torch.zeros(9 * S, dtype=torch.float64, device=self.device)
        if counts:
            res.counts = torch.zeros(5 * len(self.cams), dtype=torch.int32, device=self.device)
        out = gray_result(_ptr(res.flag), _ptr(res.xf), _ptr(res.cons), _ptr(res.counts))
        gray_classify(self.cam_arr, len(self.cams), self.p, self.state, out,
                      current_stream() if stream is None else stream)
        return res

    def run(self, xf: bool = True, cons: bool = True, counts: bool = True) -> Result:
        """One pass of the whole path: camera_init, integrate, classify."""
        self.camera_init()
        self.integrate()
        return self.classify(xf=xf, cons=cons, counts=counts)

    # ------------------------------------------------------------ host views
    def rows(self, t, nrows: int):
        """(nrows, n) host numpy view of a row-major device buffer."""
        return t.view(nrows, self.stride)[:, : self.n].cpu().numpy()
