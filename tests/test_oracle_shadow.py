"""Pins of the oracle's capture/escape decisions against exact results.

* a = 0: a ray is captured iff its impact parameter b < sqrt(27) M.
* any a: captured iff Carter's radial potential R(r) has no turning point
  between the horizon and the observer (roots of a quartic, numpy).
* the shadow's outline is Bardeen's critical curve.
Rays within 1e-3 M of the critical curve (measured on the ray's own
constants of motion) are excluded: there the outcome depends on the
integration error, and several answers are correct.
"""
import numpy as np
import pytest

import analytic
from paper_1303_5057_amd import workloads as W

BAND = 1e-3


def _grid(orc, cam):
    return orc.camera_grid(cam.a, cam.r_obs, cam.incl, cam.nx, cam.ny, cam.alpha_lo, cam.alpha_hi,
                           cam.beta_lo, cam.beta_hi)


def _constants(orc, a, X):
    return np.array([orc.conserved(a, x) for x in X])


def test_schwarzschild_shadow_c1(orc):
    """Full 64 x 64 grid of the a = 0, i = 60 deg workload against b < sqrt(27)."""
    cam = W.C1
    X = _grid(orc, cam)
    res = orc.run(orc.make_params(), cam.a, X, nthreads=0)
    c = _constants(orc, cam.a, X)
    b = np.sqrt(c[:, 1] ** 2 + c[:, 2]) / c[:, 0]
    far = np.abs(b - analytic.SQRT27) > BAND
    expect = np.where(b < analytic.SQRT27, orc.CAPTURED, orc.ESCAPED)
    assert far.sum() >= 4090
    assert np.array_equal(res.status[far], expect[far])
    # plain pixel geometry gives the same count: screen b vs sqrt(27)
    ix, iy = np.meshgrid(np.arange(64), np.arange(64))
    al = -10 + 20 * (ix + 0.5) / 64
    be = -10 + 20 * (iy + 0.5) / 64
    assert (res.status == orc.CAPTURED).sum() == int((np.hypot(al, be) < analytic.SQRT27).sum())


@pytest.mark.parametrize("a,incl_deg,window,side", [(0.99, 90.0, 8.0, 40), (0.9375, 17.0, 12.0, 40),
                                                     (0.6, 45.0, 9.0, 32)])
def test_kerr_capture_matches_radial_potential(orc, a, incl_deg, window, side):
    cam = W.Camera(a, 1000.0, np.radians(incl_deg), side, side, -window, window, -window, window)
    X = _grid(orc, cam)
    res = orc.run(orc.make_params(), a, X, nthreads=0)
    c = _constants(orc, a, X)
    band = analytic.CriticalBand(a, cam.incl)
    d = band.distance(c[:, 0], c[:, 1], c[:, 2])
    far = d > BAND
    expect = np.array([orc.CAPTURED if analytic.captured_by_potential(a, L / E, Q / E ** 2, x[1])
                       else orc.ESCAPED for (E, L, Q), x in zip(c, X)])
    assert far.mean() > 0.99
    assert np.array_equal(res.status[far], expect[far])
    assert {orc.CAPTURED, orc.ESCAPED} <= set(res.status.tolist())


def test_kerr_shadow_edge_on_extent(orc):
    """a = 0.99, i = 90 deg: along beta ~ 0 the shadow spans alpha between
    -xi at the prograde and retrograde equatorial photon orbits (about
    [-2.2517, 6.9833]; the camera's flat screen at 1000 M shifts it by
    < 3e-3 M), i.e. it is shifted towards +alpha."""
    a = 0.99
    al_curve, be_curve = analytic.bardeen_curve(a, np.pi / 2)
    xi = lambda r: -(r ** 3 - 3 * r ** 2 + a * a * r + a * a) / (a * (r - 1))
    r_pro, r_ret = analytic.photon_orbit_radii(a)
    lo, hi = -xi(r_pro), -xi(r_ret)
    assert al_curve.min() == pytest.approx(lo, abs=1e-6) and al_curve.max() == pytest.approx(hi, abs=1e-6)
    assert lo == pytest.approx(-2.2517, abs=1e-4) and hi == pytest.approx(6.9833, abs=1e-4)
    p = orc.make_params()
    for al, expect in [(lo + 0.02, orc.CAPTURED), (lo - 0.02, orc.ESCAPED),
                       (hi - 0.02, orc.CAPTURED), (hi + 0.02, orc.ESCAPED), (2.0, orc.CAPTURED)]:
        x0 = orc.camera(a, 1000.0, np.pi / 2, al, 1e-3)
        assert orc.trace(p, a, x0).status == expect, al
    # top of the curve is at (2a, sqrt(27)) exactly (photon orbit r = 3)
    k = np.argmax(be_curve)
    assert al_curve[k] == pytest.approx(2 * a, abs=1e-4)
    assert be_curve[k] == pytest.approx(np.sqrt(27.0), abs=1e-8)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.99])
@pytest.mark.parametrize("incl", [0.3, 1.2, np.pi / 2])
def test_polar_turning_point_of_traced_rays(orc, a, incl):
    """analytic.polar_turning_sin (the zero of Kerr's polar potential, used to
    split drift statistics by how close a ray passes to the axis) against
    oracle paths at a fine step: no accepted state lies closer to the axis,
    and wherever k^theta changes sign (a turning point, not a remap) the
    state there sits at the predicted sin(theta)."""
    g = np.random.Generator(np.random.PCG64(20261203))
    p = orc.make_params(step_frac=1.0 / 128)
    turns = 0
    for _ in range(25):
        al, be = g.uniform(-9.0, 9.0, 2)
        x0 = orc.camera(a, 1000.0, incl, al, be)
        E, L, Q = orc.conserved(a, x0)
        pred = float(analytic.polar_turning_sin(a, E, L, Q))
        st, path, fl = orc.trace_path(p, a, x0)
        s = np.abs(np.sin(path[:, 2]))
        assert s.min() >= pred - 1e-7
        for j in np.nonzero((path[:-1, 6] * path[1:, 6] < 0) & ((fl[1:] & 2) == 0))[0]:
            assert min(s[j], s[j + 1]) == pytest.approx(pred, rel=1e-4)
            turns += 1
    assert turns >= 10
