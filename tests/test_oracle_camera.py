"""Pins of the oracle's image plane (camera) against plain geometry.

The screen is the flat plane through the observer perpendicular to the line
of sight; the ray through (alpha, beta) moves along the line of sight. These
tests rebuild the point and direction with numpy vectors and finite
differences of the spherical coordinates, and check the null condition and
the exact a = 0 invariants.
"""
import numpy as np
import pytest

RNG = np.random.default_rng(11)


def _screen(D, incl, alpha, beta):
    n = np.array([np.sin(incl), 0.0, np.cos(incl)])           # line of sight
    e_alpha = np.array([0.0, 1.0, 0.0])                       # +phi-hat at (incl, 0)
    e_beta = -np.array([np.cos(incl), 0.0, -np.sin(incl)])    # -theta-hat at (incl, 0)
    return D * n + alpha * e_alpha + beta * e_beta, n


def _spherical(P):
    r = np.linalg.norm(P)
    return r, np.arctan2(np.hypot(P[0], P[1]), P[2]), np.arctan2(P[1], P[0])


def test_camera_position_and_direction_match_vector_geometry(orc):
    for _ in range(200):
        a = RNG.uniform(0, 0.999)
        incl = RNG.uniform(0.05, np.pi - 0.05)
        al, be = RNG.uniform(-12, 12, 2)
        D = 1000.0
        x = orc.camera(a, D, incl, al, be)
        P, n = _screen(D, incl, al, be)
        r0, th0, ph0 = _spherical(P)
        assert x[0] == 0.0
        assert x[1] == pytest.approx(r0, rel=1e-15)
        assert x[2] == pytest.approx(th0, abs=1e-14)
        assert x[3] == pytest.approx(ph0, abs=1e-14)
        # d(r, theta, phi)/ds along the line, by central differences (p = -k)
        e = 1e-3
        fp, fm = np.array(_spherical(P + e * n)), np.array(_spherical(P - e * n))
        d = (fp - fm) / (2 * e)
        assert -x[5] == pytest.approx(d[0], rel=1e-8)
        assert -x[6] == pytest.approx(d[1], rel=1e-5, abs=1e-13)
        assert -x[7] == pytest.approx(d[2], rel=1e-5, abs=1e-13)


def test_camera_null_condition(orc):
    for _ in range(200):
        a = RNG.uniform(0, 0.999)
        x = orc.camera(a, 1000.0, RNG.uniform(0.01, 3.1), *RNG.uniform(-12, 12, 2))
        assert orc.xi(a, x) == pytest.approx(-1.0, abs=1e-14)
        g = orc.metric(a, x[1], x[2])
        k = x[4:]
        assert abs(k @ g @ k) < 1e-15 * (abs(g[0, 0]) * k[0] ** 2)
        assert x[4] < 0.0  # traced backwards in time


def test_camera_schwarzschild_invariants(orc):
    """a = 0: E^2 = 1 - 2 b^2 / r0^3, L = -alpha sin(i) and L^2 + Q = b^2
    exactly, since the flat unit direction has transverse part b / r0."""
    for _ in range(100):
        incl = RNG.uniform(0.05, np.pi - 0.05)
        al, be = RNG.uniform(-12, 12, 2)
        x = orc.camera(0.0, 1000.0, incl, al, be)
        E, L, Q = orc.conserved(0.0, x)
        b2 = al * al + be * be
        assert E * E == pytest.approx(1 - 2 * b2 / x[1] ** 3, rel=1e-14)
        assert L == pytest.approx(-al * np.sin(incl), rel=1e-12, abs=1e-14)
        assert L * L + Q == pytest.approx(b2, rel=1e-12)


def test_camera_grid_is_cell_centred(orc):
    X = orc.camera_grid(0.3, 1000.0, 1.0, 5, 3, -2.0, 3.0, -1.0, 2.0)
    assert X.shape == (15, 8)
    for iy in range(3):
        for ix in range(5):
            al = -2.0 + 5.0 * (ix + 0.5) / 5
            be = -1.0 + 3.0 * (iy + 0.5) / 3
            assert np.array_equal(X[iy * 5 + ix], orc.camera(0.3, 1000.0, 1.0, al, be))


def test_on_axis_ray_is_degenerate(orc):
    """Reading: the ray exactly on the spin axis (i = 0, alpha = beta = 0) sits
    on the Boyer-Lindquist coordinate singularity; it starts with theta = 0 and
    zero angular momenta, and its first step is non-finite."""
    x = orc.camera(0.5, 1000.0, 0.0, 0.0, 0.0)
    assert x[2] == 0.0 and x[6] == 0.0 and x[7] == 0.0 and x[3] == 0.0
    r = orc.trace(orc.make_params(), 0.5, x)
    assert r.status == orc.NONFINITE and r.steps == 1
