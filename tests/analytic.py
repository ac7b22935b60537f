"""Closed-form results the integrator approximates, used to pin the oracle.

Nothing here integrates a geodesic or calls the oracle: each function is a
textbook closed form or a one-dimensional quadrature, so that agreement with
the oracle is evidence about the oracle.

* Kerr radial potential R(r) (Carter): a ray arriving from the observer is
  captured iff R has no turning point between the horizon and the observer.
* Bardeen's critical curve (the shadow boundary for an observer at infinity).
* Schwarzschild orbit quadratures for the azimuthal sweep of a scattered ray
  and for the radius where a face-on ray crosses the equatorial plane.
* Circular-orbit kinematics of Bardeen, Press & Teukolsky (1972).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, optimize
from scipy.spatial import cKDTree

SQRT27 = np.sqrt(27.0)


# --------------------------------------------------------------- horizons
def r_horizon(a):
    return 1.0 + np.sqrt(1.0 - a * a)


def photon_orbit_radii(a):
    """Prograde and retrograde equatorial circular photon orbits."""
    r_pro = 2.0 * (1.0 + np.cos(2.0 / 3.0 * np.arccos(-a)))
    r_ret = 2.0 * (1.0 + np.cos(2.0 / 3.0 * np.arccos(a)))
    return r_pro, r_ret


# ------------------------------------------------------------ radial potential
def radial_potential_coeffs(a, lam, eta):
    """R(r) = r^4 + (a^2 - lam^2 - eta) r^2 + 2 (eta + (lam - a)^2) r - a^2 eta,
    for E = 1, lam = L/E, eta = Q/E^2 (coefficients, highest power first)."""
    return np.array([1.0, 0.0, a * a - lam * lam - eta, 2.0 * (eta + (lam - a) ** 2), -a * a * eta])


def captured_by_potential(a, lam, eta, r_start):
    """True iff R(r) has no real root in (r_bh, r_start): the inbound ray then
    meets no radial turning point and falls through the horizon."""
    rbh = r_horizon(a)
    roots = np.roots(radial_potential_coeffs(a, lam, eta))
    real = roots[np.abs(roots.imag) < 1e-9 * np.maximum(1.0, np.abs(roots.real))].real
    return not np.any((real > rbh) & (real < r_start))


# --------------------------------------------------------------- critical curve
def bardeen_curve(a, incl, n=400001):
    """Points (alpha, beta >= 0) of the critical curve seen at inclination incl.
    For a = 0 it is the circle of radius sqrt(27)."""
    if a == 0.0:
        t = np.linspace(0.0, np.pi, n)
        return SQRT27 * np.cos(t), SQRT27 * np.sin(t)
    r_pro, r_ret = photon_orbit_radii(a)
    # cluster samples at the ends, where beta grows like sqrt(r - r_end)
    u = np.linspace(0.0, np.pi, n)
    r = r_pro + (r_ret - r_pro) * 0.5 * (1.0 - np.cos(u))
    xi = -(r ** 3 - 3.0 * r ** 2 + a * a * r + a * a) / (a * (r - 1.0))
    eta = -r ** 3 * (r ** 3 - 6.0 * r ** 2 + 9.0 * r - 4.0 * a * a) / (a * a * (r - 1.0) ** 2)
    si, ci = np.sin(incl), np.cos(incl)
    if si == 0.0:
        keep = np.abs(xi) < 1e-3
        rad = np.sqrt(np.maximum(eta[keep] + xi[keep] ** 2 + a * a, 0.0)).mean()
        t = np.linspace(0.0, np.pi, n)
        return rad * np.cos(t), rad * np.sin(t)
    b2 = eta + a * a * ci * ci - xi * xi * (ci / si) ** 2
    if ci == 0.0 or abs(ci) < 1e-15:
        b2 = np.maximum(b2, 0.0)   # edge-on: the ends are exactly beta = 0
    ok = b2 >= 0.0
    return -xi[ok] / si, np.sqrt(b2[ok])


def effective_impact(a, incl, E, L, Q):
    """Asymptotic image-plane position (alpha, |beta|) of a ray with constants
    E, L, Q, in the same convention as the critical curve."""
    lam = L / E
    eta = Q / (E * E)
    si, ci = np.sin(incl), np.cos(incl)
    if si == 0.0:
        rad = np.sqrt(np.maximum(eta + lam * lam + a * a, 0.0))
        return rad, np.zeros_like(rad)
    alpha = -lam / si
    beta = np.sqrt(np.maximum(eta + a * a * ci * ci - lam * lam * (ci / si) ** 2, 0.0))
    return alpha, beta


def polar_turning_sin(a, E, L, Q):
    """sin(theta) at the polar turning point of a Kerr null geodesic: the
    smallest sin(theta) its path reaches. The polar potential
    Theta(theta) = Q - cos^2 (L^2 / sin^2 - a^2 E^2) vanishes there; with
    u = cos^2 it reads a^2 E^2 u^2 + (Q + L^2 - a^2 E^2) u - Q = 0 (times
    -(1 - u)), whose root in [0, 1] is the largest cos^2 reached."""
    E, L, Q = np.asarray(E, float), np.asarray(L, float), np.asarray(Q, float)
    b = Q + L * L - a * a * E * E
    if a == 0.0:
        u = Q / (Q + L * L)
    else:
        A = a * a * E * E
        # the root -b/2A + sqrt(b^2 + 4AQ)/2A without cancellation for b > 0
        disc = np.sqrt(b * b + 4.0 * A * Q)
        u = np.where(b > 0, 2.0 * Q / (b + disc), (disc - b) / (2.0 * A))
    return np.sqrt(np.clip(1.0 - u, 0.0, 1.0))


class CriticalBand:
    """Distance from a ray's effective image-plane point to the critical curve."""

    def __init__(self, a, incl):
        self.a, self.incl = a, incl
        al, be = bardeen_curve(a, incl)
        self.tree = cKDTree(np.column_stack([al, be]))
        self.pole_on = np.sin(incl) == 0.0
        if self.pole_on:
            self.radius = np.hypot(al[0], be[0])

    def distance(self, E, L, Q, upper=np.inf):
        """Distances; with a finite `upper`, those beyond it come back as inf
        (a bounded search, fast on millions of rays)."""
        al, be = effective_impact(self.a, self.incl, np.asarray(E), np.asarray(L), np.asarray(Q))
        if self.pole_on:
            d = np.abs(al - self.radius)
            return np.where(d <= upper, d, np.inf)
        d, _ = self.tree.query(np.column_stack([np.atleast_1d(al), np.atleast_1d(be)]),
                               distance_upper_bound=upper, workers=-1)
        return d


# ------------------------------------------------------- Schwarzschild orbits
def schw_turning_point(b):
    """Largest root of r^3 - b^2 (r - 2) = 0 (closest approach), b > sqrt(27)."""
    return optimize.brentq(lambda r: r ** 3 - b * b * (r - 2.0), 3.0, max(3.0 * b, 10.0))


def schw_sweep(b, r_from, r_to=None, through_turning=True):
    """Total orbital angle swept by a Schwarzschild null ray of impact parameter
    b > sqrt(27), moving in from r_from, through the turning point and out to
    r_to (through_turning=False: from r_from in to r_to only).

    With u = 1/r the orbit equation is dpsi/du = 1 / sqrt(P(u)),
    P(u) = 2 u^3 - u^2 + 1/b^2, whose smallest positive root u0 = 1/r_min is
    the turning point. Dividing out that root, P(u) = (u0 - u) S(u) with
    S(u) = -(2 u^2 + (2 u0 - 1) u + u0 (2 u0 - 1)) > 0 on [0, u0], and the
    substitution u = u0 - s^2 turns every leg into the integral of the
    smooth 2 / sqrt(S(u0 - s^2)) over s, with no end-point singularity and no
    cancellation near the turning point."""
    u0 = 1.0 / schw_turning_point(b)
    c1, c0 = 2.0 * u0 - 1.0, u0 * (2.0 * u0 - 1.0)

    def leg(r_hi, r_lo):
        s_lo = np.sqrt(max(u0 - 1.0 / r_lo, 0.0))   # the inner end (larger u)
        s_hi = np.sqrt(u0 - 1.0 / r_hi)
        g = lambda s: 2.0 / np.sqrt(-(2.0 * (u0 - s * s) ** 2 + c1 * (u0 - s * s) + c0))
        val, _ = integrate.quad(g, s_lo, s_hi, epsabs=1e-14, epsrel=1e-13, limit=400)
        return val

    if not through_turning:
        return leg(r_from, r_to)
    rmin = 1.0 / u0
    total = leg(r_from, rmin)
    if r_to is not None:
        total += leg(r_to, rmin)
    return total


# --------------------------------------------------- circular-orbit kinematics
def kerr_circular_ut(a, r):
    """u^t of a prograde equatorial circular geodesic (Bardeen, Press &
    Teukolsky 1972)."""
    return (r ** 1.5 + a) / (r ** 0.75 * np.sqrt(r ** 1.5 - 3.0 * r ** 0.5 + 2.0 * a))


def kerr_circular_energy(a, r):
    return (r ** 1.5 - 2.0 * r ** 0.5 + a) / (r ** 0.75 * np.sqrt(r ** 1.5 - 3.0 * r ** 0.5 + 2.0 * a))


def isco_by_energy_minimum(a):
    """r_ISCO as the minimum of the circular-orbit energy (no closed form used)."""
    lo = photon_orbit_radii(a)[0] + 1e-6
    res = optimize.minimize_scalar(lambda r: kerr_circular_energy(a, r), bounds=(lo, 12.0),
                                   method="bounded", options={"xatol": 1e-12})
    return res.x


# ------------------------------------------- deformed Kerr metric, a = 0
def deformed_static_critical_impact(eps3):
    """Critical impact parameter of the a = 0 deformed metric, which is static
    and spherically symmetric with -g_tt = f(r) = (1 + eps3 / r^3)(1 - 2 / r)
    and g_thth = r^2: a null ray of impact parameter b has a turning point
    where b^2 = r^2 / f(r), so it is captured iff b < min_{r > 2} r / sqrt(f)."""
    f = lambda r: (1.0 + eps3 / r ** 3) * (1.0 - 2.0 / r)
    res = optimize.minimize_scalar(lambda r: r / np.sqrt(f(r)), bounds=(2.05, 10.0), method="bounded",
                                   options={"xatol": 1e-12})
    return res.fun
