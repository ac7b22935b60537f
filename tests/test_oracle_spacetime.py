"""Pins of the oracle's spacetime (Kerr metric, its derivatives, Christoffels).

Each check compares with something other than the oracle's own formulas:
textbook identities of the Kerr metric, the Schwarzschild limit, finite
differences, and a library matrix inverse.
"""
import numpy as np
import pytest

from analytic import photon_orbit_radii, r_horizon

RNG = np.random.default_rng(7)


def _points(n=60, a_max=0.999):
    for _ in range(n):
        a = RNG.uniform(0.0, a_max)
        r = RNG.uniform(r_horizon(a) + 0.05, 60.0)
        th = RNG.uniform(0.02, np.pi - 0.02)
        yield a, r, th


def test_metric_textbook_identities(orc):
    """det g = -Sigma^2 sin^2 and g_tphi^2 - g_tt g_phph = Delta sin^2 (Kerr in BL)."""
    for a, r, th in _points():
        g = orc.metric(a, r, th)
        sig = r * r + a * a * np.cos(th) ** 2
        dl = r * r - 2 * r + a * a
        s2 = np.sin(th) ** 2
        assert np.allclose(g, g.T)
        assert np.linalg.det(g) == pytest.approx(-sig * sig * s2, rel=1e-10)
        assert g[0, 3] ** 2 - g[0, 0] * g[3, 3] == pytest.approx(dl * s2, rel=1e-9)


def test_metric_schwarzschild_limit(orc):
    for _, r, th in _points(20):
        g = orc.metric(0.0, r, th)
        f = 1.0 - 2.0 / r
        assert np.allclose(g, np.diag([-f, 1.0 / f, r * r, (r * np.sin(th)) ** 2]), rtol=1e-14, atol=0)


def test_metric_static_limit_and_horizon(orc):
    """g_tt vanishes on the ergosurface r = 1 + sqrt(1 - a^2 cos^2); g^rr = 0 at r_bh."""
    for a in (0.3, 0.9, 0.99):
        for th in (0.3, 1.0, np.pi / 2):
            r_erg = 1 + np.sqrt(1 - a * a * np.cos(th) ** 2)
            assert abs(orc.metric(a, r_erg, th)[0, 0]) < 1e-14
        rbh = orc.horizon(a)
        assert rbh == pytest.approx(r_horizon(a), rel=1e-15)
        assert rbh * rbh - 2 * rbh + a * a == pytest.approx(0.0, abs=1e-14)


def test_metric_derivatives_finite_difference(orc):
    for a, r, th in _points():
        dr, dth = orc.metric_deriv(a, r, th)
        e = 1e-6
        fr = (orc.metric(a, r + e * r, th) - orc.metric(a, r - e * r, th)) / (2 * e * r)
        ft = (orc.metric(a, r, th + e) - orc.metric(a, r, th - e)) / (2 * e)
        scale = np.abs(orc.metric(a, r, th)).max() / r + 1e-12
        assert np.abs(dr - fr).max() < 1e-7 * scale * r
        assert np.abs(dth - ft).max() < 1e-7 * np.abs(orc.metric(a, r, th)).max()


def test_christoffel_from_finite_differences_and_library_inverse(orc):
    """Rebuild Gamma from central differences of g and numpy's matrix inverse."""
    for a, r, th in _points(30):
        e = 1e-6
        dg = np.zeros((4, 4, 4))
        dg[1] = (orc.metric(a, r * (1 + e), th) - orc.metric(a, r * (1 - e), th)) / (2 * e * r)
        dg[2] = (orc.metric(a, r, th + e) - orc.metric(a, r, th - e)) / (2 * e)
        gi = np.linalg.inv(orc.metric(a, r, th))
        ref = 0.5 * (np.einsum("mn,anb->mab", gi, dg) + np.einsum("mn,bna->mab", gi, dg)
                     - np.einsum("mn,nab->mab", gi, dg))
        G = orc.christoffel(a, r, th)
        assert np.allclose(G, np.swapaxes(G, 1, 2), rtol=0, atol=0)
        assert np.abs(G - ref).max() < 1e-6 * max(1.0, np.abs(ref).max())


def test_christoffel_schwarzschild_textbook(orc):
    """Nonzero Schwarzschild symbols (M = 1) as listed in textbooks."""
    r, th = 7.3, 1.1
    G = orc.christoffel(0.0, r, th)
    f = 1 - 2 / r
    expect = {
        (0, 0, 1): 1 / (r * r * f), (1, 0, 0): f / (r * r), (1, 1, 1): -1 / (r * r * f),
        (1, 2, 2): -r * f, (1, 3, 3): -r * f * np.sin(th) ** 2, (2, 1, 2): 1 / r,
        (2, 3, 3): -np.sin(th) * np.cos(th), (3, 1, 3): 1 / r, (3, 2, 3): np.cos(th) / np.sin(th),
    }
    ref = np.zeros((4, 4, 4))
    for (m, a_, b), v in expect.items():
        ref[m, a_, b] = ref[m, b, a_] = v
    assert np.allclose(G, ref, rtol=1e-13, atol=1e-15)


def test_circular_photon_orbits_are_fixed_points(orc):
    """Equatorial circular photon orbits at r_pro and r_retro (closed form) have
    zero radial acceleration; so does the a = 0 photon sphere r = 3 for any
    orbital plane."""
    for a in (0.0, 0.5, 0.99):
        for r in photon_orbit_radii(a):
            g = orc.metric(a, r, np.pi / 2)
            # null circular orbit: g_tt + 2 g_tphi W + g_phph W^2 = 0 for W = dphi/dt
            W = np.roots([g[3, 3], 2 * g[0, 3], g[0, 0]])
            for w in W.real:
                x = np.array([0, r, np.pi / 2, 0, 1.0, 0, 0, w])
                f = orc.rhs(a, x)
                if abs(f[5]) < 1e-9:
                    break
            else:
                pytest.fail(f"no circular photon orbit at r={r} for a={a}")
