"""Pins of the oracle's deformed-Kerr spacetime (the non-Kerr metrics of
Sec. 1, here the Johannsen-Psaltis deformation with deviation eps3), each
independent of the oracle's code:

* eps3 = 0 is Kerr: metric, derivatives, Christoffel symbols, right-hand side,
  null monitor, camera and whole traces equal the Kerr oracle's, which is
  pinned separately (test_oracle_spacetime.py, test_oracle_integrator.py);
* the complex-step metric derivatives equal central finite differences;
* det g = -Sigma^2 (1 + h)^2 sin^2(theta), an identity of the metric (any
  slip in g_tt, g_tphi, g_rr or g_phph breaks it);
* the Christoffel symbols equal their definition evaluated with numpy
  (finite-difference derivatives, numpy matrix inverse);
* along traced rays E, L_z and the null condition are conserved, while
  Carter's Q (in its Kerr form) is not once eps3 != 0;
* at a = 0 the deformed metric is static and spherically symmetric, with
  f(r) = (1 + eps3 / r^3)(1 - 2 / r), and a ray is captured iff its impact
  parameter is below min_r r / sqrt(f(r)) (closed form, scipy minimiser).
"""
import numpy as np
import pytest

import analytic
import oracle

rng = np.random.default_rng(20261203)


def _points(n=40):
    a = rng.uniform(0.0, 0.99, n)
    r = rng.uniform(2.2, 30.0, n)
    th = rng.uniform(0.05, np.pi - 0.05, n)
    e = rng.uniform(-0.5, 3.0, n)
    return zip(a, r, th, e)


def test_eps3_zero_is_kerr(orc):
    for a, r, th, _ in _points(20):
        assert np.allclose(orc.metric_jp(a, 0.0, r, th), orc.metric(a, r, th), rtol=1e-15, atol=1e-15)
        dr, dt = orc.metric_deriv_jp(a, 0.0, r, th)
        kr, kt = orc.metric_deriv(a, r, th)
        assert np.allclose(dr, kr, rtol=1e-12, atol=1e-13) and np.allclose(dt, kt, rtol=1e-12, atol=1e-13)
        assert np.allclose(orc.christoffel_jp(a, 0.0, r, th), orc.christoffel(a, r, th), rtol=1e-11, atol=1e-13)
    a = 0.8
    x0k = orc.camera(a, 1000.0, 1.1, 4.0, -2.5)
    x0j = orc.camera_jp(a, 0.0, 1000.0, 1.1, 4.0, -2.5)
    assert np.array_equal(x0k, x0j)
    assert orc.xi_jp(a, 0.0, x0k) == orc.xi(a, x0k)
    rk = orc.trace(orc.make_params(), a, x0k)
    rj = orc.trace(orc.make_params(metric=orc.METRIC_JP, eps3=0.0), a, x0j)
    assert rk.status == rj.status and rk.steps == rj.steps
    assert np.allclose(rk.x, rj.x, rtol=1e-9, atol=1e-9)


def test_complex_step_derivatives_match_finite_differences(orc):
    for a, r, th, e in _points():
        dr, dt = orc.metric_deriv_jp(a, e, r, th)
        hr, ht = 1e-5 * r, 1e-5
        fr = (orc.metric_jp(a, e, r + hr, th) - orc.metric_jp(a, e, r - hr, th)) / (2 * hr)
        ft = (orc.metric_jp(a, e, r, th + ht) - orc.metric_jp(a, e, r, th - ht)) / (2 * ht)
        scale = np.abs(orc.metric_jp(a, e, r, th)).max()
        assert np.abs(dr - fr).max() <= 1e-8 * scale
        assert np.abs(dt - ft).max() <= 1e-8 * scale


def test_determinant_identity(orc):
    for a, r, th, e in _points():
        g = orc.metric_jp(a, e, r, th)
        sig = r * r + (a * np.cos(th)) ** 2
        h = e * r / sig ** 2
        assert np.linalg.det(g) == pytest.approx(-(sig * (1 + h) * np.sin(th)) ** 2, rel=1e-11)
        # Lorentzian: the t-phi block has negative determinant outside the horizon
        assert g[0, 0] * g[3, 3] - g[0, 3] ** 2 < 0.0 and g[1, 1] > 0.0


def test_christoffel_symbols_by_definition(orc):
    for a, r, th, e in _points(15):
        g = orc.metric_jp(a, e, r, th)
        gi = np.linalg.inv(g)
        hr, ht = 1e-5 * r, 1e-5
        dg = np.zeros((4, 4, 4))        # dg[k] = d_k g
        dg[1] = (orc.metric_jp(a, e, r + hr, th) - orc.metric_jp(a, e, r - hr, th)) / (2 * hr)
        dg[2] = (orc.metric_jp(a, e, r, th + ht) - orc.metric_jp(a, e, r, th - ht)) / (2 * ht)
        low = 0.5 * (np.einsum("anb->nab", dg) + np.einsum("bna->nab", dg) - dg)   # Gamma_{n a b}
        G = np.einsum("mn,nab->mab", gi, low)
        assert np.allclose(orc.christoffel_jp(a, e, r, th), G, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("eps3", [0.0, 2.0])
def test_constants_along_deformed_rays(orc, eps3):
    """E, L_z and the null condition stay put; the Kerr-form Q only at eps3 = 0."""
    a = 0.6
    p = orc.make_params(metric=orc.METRIC_JP, eps3=eps3)
    dq = []
    for al, be in [(-6.5, 1.5), (7.0, -3.0), (2.5, 6.5), (-5.0, -5.5)]:
        x0 = orc.camera_jp(a, eps3, 1000.0, 1.2, al, be)
        c0 = orc.conserved_jp(a, eps3, x0)
        r = orc.trace(p, a, x0)
        assert r.status == orc.ESCAPED and r.n_euler == 0
        c1 = orc.conserved_jp(a, eps3, r.x)
        dE, dL, dQ = orc.drift(c0[0], c0[1], c0[2], c1[0], c1[1], c1[2])
        assert max(dE, dL) < 1e-6
        assert orc.xi_jp(a, eps3, r.x) == pytest.approx(-1.0, abs=1e-6)
        dq.append(dQ)
    if eps3 == 0.0:
        assert max(dq) < 1e-6
    else:
        assert max(dq) > 1e-4


@pytest.mark.parametrize("eps3", [2.0, -1.0])
def test_spherical_deformation_shadow_radius(orc, eps3):
    """a = 0, i = 60 deg, 48 x 48 over [-8, 8]^2: captured iff the ray's
    impact parameter sqrt(L^2 + Q) / E is below the critical value of the
    deformed static metric (rays within 2e-3 M of it are not checked)."""
    bc = analytic.deformed_static_critical_impact(eps3)
    assert abs(bc - np.sqrt(27.0)) > 0.05          # the deformation moves the shadow
    n = 48
    ax = -8.0 + 16.0 * (np.arange(n) + 0.5) / n
    X0 = np.array([orc.camera_jp(0.0, eps3, 1000.0, np.radians(60.0), al, be) for be in ax for al in ax])
    res = orc.run(orc.make_params(metric=orc.METRIC_JP, eps3=eps3), 0.0, X0)
    c = np.array([orc.conserved_jp(0.0, eps3, x) for x in X0])
    b = np.sqrt(c[:, 1] ** 2 + c[:, 2]) / c[:, 0]
    far = np.abs(b - bc) > 2e-3
    assert far.mean() > 0.98
    assert np.array_equal((res.status == orc.CAPTURED)[far], (b < bc)[far])
    assert np.all((res.status == orc.CAPTURED) | (res.status == orc.ESCAPED))
