"""Host-side checks of libgray's C ABI that need no GPU.

The library must load, export every function include/gray.h declares, agree
with the binding on struct layouts, and reject invalid arguments on the host
(GRAY_EINVAL / GRAY_EWORKSPACE) before it touches any device.
"""
import ctypes
import math
import os
import re

import pytest

from paper_1303_5057_amd import gray as G
from paper_1303_5057_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "gray.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gray_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(G.LIB_PATH):
        from paper_1303_5057_amd import build
        build.build()
    return G.load()


def test_exports_every_declared_function(lib):
    names = _declared_functions()
    assert set(names) == set(G.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts(lib):
    for k, t in enumerate((G.gray_camera, G.gray_params, G.gray_state, G.gray_result)):
        assert lib.gray_struct_size(k) == ctypes.sizeof(t)
    assert lib.gray_struct_size(99) == 0
    assert ctypes.sizeof(G.gray_camera) == 96


def test_strerror_and_version(lib):
    for code in (0, -1, -2, -3, -4, 7):
        assert isinstance(G.gray_strerror(code), str) and G.gray_strerror(code)
    assert G.gray_version() >= 100


def _state(n, stride, fp64=True, x=0x1000, status=0x2000, steps=0x3000, cam=0x4000, lo=None):
    # Fake, never-dereferenced addresses: every call below must fail validation first.
    return G.gray_state(x, lo, status, steps, cam, None, None, None, n, stride)


def _call_init(cams, p, s):
    arr = G.camera_array(cams)
    return G.load().gray_camera_init(arr, len(cams), ctypes.byref(p), ctypes.byref(s), None)


def _call_integrate(cams, p, s, ws=0x100000, wsb=1 << 20):
    arr = G.camera_array(cams)
    return G.load().gray_integrate(arr, len(cams), ctypes.byref(p), ctypes.byref(s), ws, wsb, None)


def _call_classify(cams, p, s, flag=0x5000):
    arr = G.camera_array(cams)
    out = G.gray_result(flag, None, None, None)
    return G.load().gray_classify(arr, len(cams), ctypes.byref(p), ctypes.byref(s),
                                  ctypes.byref(out), None)


CAM = W.Camera(0.5, 1000.0, 1.0, 8, 8, -5.0, 5.0, -5.0, 5.0)


@pytest.mark.parametrize("field,value", [
    ("step_frac", 0.0), ("step_frac", math.inf), ("horizon_eps", 0.0), ("r_escape", -1.0),
    ("xi_eps", 0.0), ("euler_div", 0.5), ("max_steps", 0), ("call_steps", -1), ("precision", 5),
    ("flags", 8), ("fp64_horizon", -1.0), ("fp64_pole", math.nan), ("fp64_turn", math.inf),
    ("pole_mode", 3), ("pole_mode", -1)])
def test_invalid_params_rejected(lib, field, value):
    p = G.params_struct(W.Params())
    setattr(p, field, value)
    s = _state(64, 64)
    assert _call_init([CAM], p, s) == G.GRAY_EINVAL
    assert _call_integrate([CAM], p, s) == G.GRAY_EINVAL
    assert _call_classify([CAM], p, s) == G.GRAY_EINVAL
    assert G.gray_workspace_size(64, 1, p) == 0


@pytest.mark.parametrize("cam", [
    W.Camera(1.0, 1000.0, 1.0, 8, 8, -5, 5, -5, 5),       # extremal spin
    W.Camera(-0.1, 1000.0, 1.0, 8, 8, -5, 5, -5, 5),      # negative spin
    W.Camera(0.5, 1.5, 1.0, 8, 8, -5, 5, -5, 5),          # observer inside the horizon
    W.Camera(0.5, 1000.0, 3.5, 8, 8, -5, 5, -5, 5),       # inclination > pi
    W.Camera(0.5, 1000.0, 1.0, 8, 8, -5, math.nan, -5, 5),
    W.Camera(0.5, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, kind=2),             # unknown camera kind
    W.Camera(0.5, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, metric=2),           # unknown metric
    W.Camera(0.5, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, deform=1.0),         # Kerr with a deviation
    W.Camera(0.5, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, metric=1, deform=-0.1),  # spinning, eps3 < 0
    W.Camera(0.0, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, metric=1, deform=-8.0),  # 1 + h = 0 at r = 2
    W.Camera(0.5, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, metric=1, deform=math.inf),
])
def test_invalid_camera_rejected(lib, cam):
    p = G.params_struct(W.Params())
    s = _state(64, 64)
    assert _call_init([cam], p, s) == G.GRAY_EINVAL
    assert _call_integrate([cam], p, s) == G.GRAY_EINVAL


def test_invalid_state_rejected(lib):
    p = G.params_struct(W.Params())
    assert _call_init([CAM], p, _state(64, 100)) == G.GRAY_EINVAL        # stride % 64
    assert _call_init([CAM], p, _state(64, 0)) == G.GRAY_EINVAL          # stride < n
    assert _call_init([CAM], p, _state(65, 128)) == G.GRAY_EINVAL        # cameras do not tile n
    assert _call_init([CAM], p, _state(64, 64, x=None)) == G.GRAY_EINVAL
    assert _call_init([CAM], p, _state(64, 64, lo=0x9000)) == G.GRAY_EINVAL  # lo with FP64
    p32 = G.params_struct(W.Params(precision="fp32c"))
    assert _call_init([CAM], p32, _state(64, 64)) == G.GRAY_EINVAL       # FP32C needs lo
    pd = G.params_struct(W.Params(record_disk=True))
    assert _call_init([CAM], pd, _state(64, 64)) == G.GRAY_EINVAL        # disk buffer missing
    assert _call_classify([CAM], p, _state(64, 64), flag=None) == G.GRAY_EINVAL
    # cameras that do not tile [0, n) in order
    arr = G.camera_array([CAM, CAM])
    arr[1].first = 0
    s = _state(128, 128)
    assert G.load().gray_camera_init(arr, 2, ctypes.byref(p), ctypes.byref(s), None) == G.GRAY_EINVAL


def test_negative_camera_step_budget_rejected(lib):
    p = G.params_struct(W.Params(call_steps=50))
    arr = G.camera_array([CAM])
    arr[0].call_steps = -1
    s = _state(64, 64)
    assert G.load().gray_camera_init(arr, 1, ctypes.byref(p), ctypes.byref(s), None) == G.GRAY_EINVAL
    with pytest.raises(G.GrayError) as e:
        G.gray_integrate(arr, 1, p, s, 0x1000, 1 << 20)
    assert e.value.code == G.GRAY_EINVAL


def test_fp32c_integrate_needs_counters(lib):
    """FP32C keeps each photon's FP64-step count (a photon that has taken FP64
    steps continues in FP64), so its integrate call requires the counters."""
    p = G.params_struct(W.Params(precision="fp32c"))
    s = _state(64, 64, lo=0x9000)
    assert _call_integrate([CAM], p, s) == G.GRAY_EINVAL
    s.counters = 0xA000
    assert _call_integrate([CAM], p, s, ws=None) == G.GRAY_EWORKSPACE


def test_fp32c_supports_only_the_production_pole_treatment(lib):
    p = G.params_struct(W.Params(precision="fp32c", pole_mode=G.GRAY_POLE_NONE))
    s = _state(64, 64, lo=0x9000)
    assert _call_init([CAM], p, s) == G.GRAY_EUNSUPPORTED
    assert _call_integrate([CAM], p, s) == G.GRAY_EUNSUPPORTED
    p64 = G.params_struct(W.Params(pole_mode=G.GRAY_POLE_EULER_CROSSING))
    assert G.gray_workspace_size(64, 1, p64) > 0


def test_photon_count_limit(lib):
    p = G.params_struct(W.Params())
    n = G.GRAY_MAX_PHOTONS
    assert G.gray_workspace_size(n, 1, p) > 0
    assert G.gray_workspace_size(n + 1, 1, p) == 0
    big = W.Camera(0.5, 1000.0, 1.0, 1, n + 1, -5, 5, -5, 5)
    s = _state(n + 1, (n + 1 + 63) // 64 * 64)
    assert _call_init([big], p, s) == G.GRAY_EINVAL
    assert _call_integrate([big], p, s) == G.GRAY_EINVAL
    assert _call_classify([big], p, s) == G.GRAY_EINVAL


def test_workspace_checked(lib):
    p = G.params_struct(W.Params())
    s = _state(64, 64)
    need = G.gray_workspace_size(64, 1, p)
    assert need >= 256 + 64
    assert _call_integrate([CAM], p, s, ws=None) == G.GRAY_EWORKSPACE
    assert _call_integrate([CAM], p, s, ws=0x100010) == G.GRAY_EWORKSPACE   # misaligned
    assert _call_integrate([CAM], p, s, wsb=need - 1) == G.GRAY_EWORKSPACE


def test_static_workspace_limit(lib):
    """gray_integrate_static rejects, on the host, a call whose workspace
    would not fit the library's static array, and checks its arguments as
    gray_integrate does."""
    p = G.params_struct(W.Params())
    cap = G.GRAY_STATIC_WORKSPACE_BYTES
    # largest dense-mode photon count that fits, and one photon-chunk more
    n_fit = 64
    while G.gray_workspace_size(n_fit * 2, 1, p) <= cap:
        n_fit *= 2
    big = n_fit * 2
    assert G.gray_workspace_size(big, 1, p) > cap
    cam = W.Camera(0.5, 1000.0, 1.0, 64, big // 64, -5, 5, -5, 5)
    s = _state(big, big)
    arr = G.camera_array([cam])
    assert lib.gray_integrate_static(arr, 1, ctypes.byref(p), ctypes.byref(s), None) == G.GRAY_EWORKSPACE
    bad = G.params_struct(W.Params())
    bad.step_frac = 0.0
    s = _state(64, 64)
    arr = G.camera_array([CAM])
    assert lib.gray_integrate_static(arr, 1, ctypes.byref(bad), ctypes.byref(s), None) == G.GRAY_EINVAL
    empty = G.gray_state(None, None, None, None, None, None, None, None, 0, 0)
    assert lib.gray_integrate_static(arr, 1, ctypes.byref(p), ctypes.byref(empty), None) == G.GRAY_OK


def test_empty_batch_is_a_no_op(lib):
    p = G.params_struct(W.Params())
    s = G.gray_state(None, None, None, None, None, None, None, None, 0, 0)
    assert _call_init([CAM], p, s) == G.GRAY_OK
    assert _call_integrate([CAM], p, s, ws=None, wsb=0) == G.GRAY_OK
    assert _call_classify([CAM], p, s, flag=None) == G.GRAY_OK


def test_camera_array_tiles_photon_ids():
    cams = [W.scaled(CAM, 3, 5), W.scaled(CAM, 7), W.scaled(CAM, 1)]
    arr = G.camera_array(cams)
    assert [arr[k].first for k in range(3)] == [0, 15, 64]


def test_deformed_metric_requirements(lib):
    """The deformed metric runs in FP64 with the production pole treatment and
    no disk recorder, and all cameras of a call share one metric kind."""
    dcam = W.Camera(0.5, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, metric=G.GRAY_METRIC_DEFORMED, deform=1.5)
    s = _state(64, 64)
    p = G.params_struct(W.Params())
    for bad in (W.Params(pole_mode=G.GRAY_POLE_NONE), W.Params(record_disk=True)):
        pb = G.params_struct(bad)
        sb = G.gray_state(0x1000, None, 0x2000, 0x3000, 0x4000, None, None, 0x6000, 64, 64)
        assert _call_init([dcam], pb, sb) == G.GRAY_EUNSUPPORTED
        assert _call_integrate([dcam], pb, sb) == G.GRAY_EUNSUPPORTED
    p32 = G.params_struct(W.Params(precision="fp32c"))
    s32 = _state(64, 64, lo=0x9000)
    assert _call_integrate([dcam], p32, s32) == G.GRAY_EUNSUPPORTED
    s2 = _state(128, 128)
    assert _call_init([dcam, CAM], p, s2) == G.GRAY_EUNSUPPORTED
    assert _call_classify([CAM, dcam], p, s2) == G.GRAY_EUNSUPPORTED
    # a = 0 admits a negative deviation while 1 + h stays positive outside r = 2
    ok = W.Camera(0.0, 1000.0, 1.0, 8, 8, -5, 5, -5, 5, metric=G.GRAY_METRIC_DEFORMED, deform=-1.0)
    assert _call_integrate([ok], p, _state(64, 64), ws=None) == G.GRAY_EWORKSPACE
