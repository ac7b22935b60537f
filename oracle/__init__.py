"""Python access to the FP64 CPU oracle (``gray_oracle.c``).

TEST INFRASTRUCTURE ONLY. The oracle is the plain, slow reference that the
GPU path is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The product package
never imports it, and the two share no code.

Everything here is argument marshalling over ``ctypes``; the arithmetic is in
the C file, which follows Sec. 2 of Chan, Psaltis & Ozel (2013), "GRay".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gray_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RUNNING, CAPTURED, ESCAPED, UNFINISHED, NONFINITE = range(5)
STATUS_NAMES = {RUNNING: "running", CAPTURED: "captured", ESCAPED: "escaped",
                UNFINISHED: "unfinished", NONFINITE: "nonfinite"}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "gray_oracle.h"))):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("step_frac", ctypes.c_double), ("horizon_eps", ctypes.c_double),
                ("r_escape", ctypes.c_double), ("xi_eps", ctypes.c_double),
                ("euler_div", ctypes.c_double), ("disk_rmin", ctypes.c_double),
                ("disk_rmax", ctypes.c_double), ("max_steps", ctypes.c_int32),
                ("record_disk", ctypes.c_int32), ("pole_mode", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("eps3", ctypes.c_double)]


class CameraT(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("r_obs", ctypes.c_double), ("incl", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("alpha_lo", ctypes.c_double), ("alpha_hi", ctypes.c_double),
                ("beta_lo", ctypes.c_double), ("beta_hi", ctypes.c_double)]


POLE_MONITOR, POLE_EULER_CROSSING, POLE_NONE = 0, 1, 2
METRIC_KERR, METRIC_JP = 0, 1


def make_params(step_frac=1.0 / 32, horizon_eps=1e-3, r_escape=1000.0, xi_eps=1e-3,
                euler_div=9.0, max_steps=65536, record_disk=False, disk_rmin=-1.0,
                disk_rmax=50.0, pole_mode=POLE_MONITOR, metric=METRIC_KERR, eps3=0.0) -> Params:
    return Params(step_frac, horizon_eps, r_escape, xi_eps, euler_div, disk_rmin, disk_rmax,
                  int(max_steps), 1 if record_disk else 0, int(pole_mode), int(metric), float(eps3))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        P = ctypes.POINTER(Params)
        sig = {
            "oracle_horizon": (d, [d]),
            "oracle_r_isco": (d, [d]),
            "oracle_metric": (None, [d, d, d, _D]),
            "oracle_metric_deriv": (None, [d, d, d, _D, _D]),
            "oracle_christoffel": (None, [d, d, d, _D]),
            "oracle_rhs": (None, [d, _D, _D]),
            "oracle_camera": (None, [d, d, d, d, d, _D]),
            "oracle_camera_grid": (None, [ctypes.POINTER(CameraT), _D]),
            "oracle_step_size": (d, [d, d, _D]),
            "oracle_xi": (d, [d, _D]),
            "oracle_remap": (ctypes.c_int, [_D]),
            "oracle_step": (ctypes.c_int, [P, d, _D, _D]),
            "oracle_conserved": (None, [d, _D, _D]),
            "oracle_disk_redshift": (d, [d, d, d, d]),
            "oracle_metric_jp": (None, [d, d, d, d, _D]),
            "oracle_metric_deriv_jp": (None, [d, d, d, d, _D, _D]),
            "oracle_christoffel_jp": (None, [d, d, d, d, _D]),
            "oracle_rhs_jp": (None, [d, d, _D, _D]),
            "oracle_xi_jp": (d, [d, d, _D]),
            "oracle_camera_jp": (None, [d, d, d, d, d, d, _D]),
            "oracle_conserved_jp": (None, [d, d, _D, _D]),
            "oracle_trace": (ctypes.c_int, [P, d, _D, _I, _I, _I, _D]),
            "oracle_trace_path": (ctypes.c_int, [P, d, _D, i32, _D, _I, _I]),
            "oracle_run": (None, [P, i64, _D, _D, _I, _I, _I, _I, _D, _D, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def horizon(a: float) -> float:
    return lib().oracle_horizon(a)


def r_isco(a: float) -> float:
    return lib().oracle_r_isco(a)


def metric(a, r, th) -> np.ndarray:
    g = np.zeros(16)
    lib().oracle_metric(a, r, th, _dp(g))
    return g.reshape(4, 4)


def metric_deriv(a, r, th):
    dr, dth = np.zeros(16), np.zeros(16)
    lib().oracle_metric_deriv(a, r, th, _dp(dr), _dp(dth))
    return dr.reshape(4, 4), dth.reshape(4, 4)


def christoffel(a, r, th) -> np.ndarray:
    G = np.zeros(64)
    lib().oracle_christoffel(a, r, th, _dp(G))
    return G.reshape(4, 4, 4)


def rhs(a, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros(8)
    lib().oracle_rhs(a, _dp(x), _dp(f))
    return f


def camera(a, r_obs, incl, alpha, beta) -> np.ndarray:
    x = np.zeros(8)
    lib().oracle_camera(a, r_obs, incl, alpha, beta, _dp(x))
    return x


def camera_grid(a, r_obs, incl, nx, ny, alpha_lo, alpha_hi, beta_lo, beta_hi) -> np.ndarray:
    """Initial states of a cell-centred nx*ny grid, shape (ny*nx, 8)."""
    c = CameraT(a, r_obs, incl, nx, ny, alpha_lo, alpha_hi, beta_lo, beta_hi)
    x = np.zeros((nx * ny, 8))
    lib().oracle_camera_grid(ctypes.byref(c), _dp(x))
    return x


def step_size(rbh, step_frac, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().oracle_step_size(rbh, step_frac, _dp(x))


def xi(a, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().oracle_xi(a, _dp(x))


def remap(x):
    x = np.array(x, dtype=np.float64)
    applied = lib().oracle_remap(_dp(x))
    return x, applied


def step(params: Params, a, x):
    x = np.array(x, dtype=np.float64)
    h = ctypes.c_double(0.0)
    fl = lib().oracle_step(ctypes.byref(params), a, _dp(x), ctypes.byref(h))
    return x, fl, h.value


def conserved(a, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(3)
    lib().oracle_conserved(a, _dp(x), _dp(out))
    return out


# --------------------------------------- deformed Kerr metric (eps3 = 0: Kerr)
def metric_jp(a, eps3, r, th) -> np.ndarray:
    g = np.zeros(16)
    lib().oracle_metric_jp(a, eps3, r, th, _dp(g))
    return g.reshape(4, 4)


def metric_deriv_jp(a, eps3, r, th):
    dr, dth = np.zeros(16), np.zeros(16)
    lib().oracle_metric_deriv_jp(a, eps3, r, th, _dp(dr), _dp(dth))
    return dr.reshape(4, 4), dth.reshape(4, 4)


def christoffel_jp(a, eps3, r, th) -> np.ndarray:
    G = np.zeros(64)
    lib().oracle_christoffel_jp(a, eps3, r, th, _dp(G))
    return G.reshape(4, 4, 4)


def rhs_jp(a, eps3, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros(8)
    lib().oracle_rhs_jp(a, eps3, _dp(x), _dp(f))
    return f


def xi_jp(a, eps3, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().oracle_xi_jp(a, eps3, _dp(x))


def camera_jp(a, eps3, r_obs, incl, alpha, beta) -> np.ndarray:
    x = np.zeros(8)
    lib().oracle_camera_jp(a, eps3, r_obs, incl, alpha, beta, _dp(x))
    return x


def conserved_jp(a, eps3, x) -> np.ndarray:
    """E, L_z (constants of motion) and the Kerr expression for Q (not one)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(3)
    lib().oracle_conserved_jp(a, eps3, _dp(x), _dp(out))
    return out


def disk_redshift(a, rc, E, L) -> float:
    return lib().oracle_disk_redshift(a, rc, E, L)


@dataclass
class TraceResult:
    status: int
    x: np.ndarray
    steps: int
    n_euler: int
    n_remap: int
    disk: np.ndarray


def trace(params: Params, a, x0) -> TraceResult:
    x = np.array(x0, dtype=np.float64)
    s, ne, nr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    disk = np.zeros(3)
    st = lib().oracle_trace(ctypes.byref(params), a, _dp(x), ctypes.byref(s), ctypes.byref(ne),
                            ctypes.byref(nr), _dp(disk))
    return TraceResult(st, x, s.value, ne.value, nr.value, disk)


def trace_path(params: Params, a, x0, max_pts=200000):
    """Every accepted state along one ray: (status, path[n,8], flags[n])."""
    x = np.array(x0, dtype=np.float64)
    path = np.zeros((max_pts, 8))
    flags = np.zeros(max_pts, dtype=np.int32)
    npts = ctypes.c_int32()
    st = lib().oracle_trace_path(ctypes.byref(params), a, _dp(x), max_pts, _dp(path), _ip(flags),
                                 ctypes.byref(npts))
    n = npts.value
    return st, path[:n].copy(), flags[:n].copy()


@dataclass
class RunResult:
    status: np.ndarray
    x: np.ndarray
    steps: np.ndarray
    n_euler: np.ndarray
    n_remap: np.ndarray
    disk: np.ndarray | None
    mark: np.ndarray | None = None   # (n, 8): last state with r >= 2 r_bh before the last fall below


def run(params: Params, a, x0, nthreads: int = 0, want_disk: bool = False,
        want_mark: bool = False) -> RunResult:
    """Trace every photon of x0 (shape (n, 8)); a is a scalar or per-photon array."""
    x = np.array(x0, dtype=np.float64, order="C").reshape(-1, 8)
    n = x.shape[0]
    av = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)))
    status = np.zeros(n, dtype=np.int32)
    steps = np.zeros(n, dtype=np.int32)
    ne = np.zeros(n, dtype=np.int32)
    nr = np.zeros(n, dtype=np.int32)
    disk = np.zeros((n, 3)) if want_disk else None
    mark = np.zeros((n, 8)) if want_mark else None
    lib().oracle_run(ctypes.byref(params), n, _dp(av), _dp(x), _ip(status), _ip(steps), _ip(ne),
                     _ip(nr), _dp(disk) if disk is not None else None,
                     _dp(mark) if mark is not None else None, int(nthreads))
    return RunResult(status, x, steps, ne, nr, disk, mark)


def drift(E0, L0, Q0, E, L, Q):
    """Relative drifts of E, L_z and Q with floors that avoid 0/0 (dE, dL, dQ)."""
    dE = np.abs(E / E0 - 1.0)
    dL = np.abs(L - L0) / (np.abs(L0) + np.abs(E0))
    dQ = np.abs(Q - Q0) / (np.abs(Q0) + L0 * L0 + E0 * E0)
    return dE, dL, dQ
