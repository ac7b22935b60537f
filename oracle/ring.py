"""Photon-ring oracle: the ring edge and ring measures of Sec. 4, computed
the slow and plain way on the CPU.

TEST INFRASTRUCTURE ONLY (like the rest of this package): used by the test
suite; the product never imports it.

* Pixels: the polar image-plane grid of the study: nr cell-centred radii
  R_k = r_lo + (r_hi - r_lo)(k + 1/2)/nr along each angle vartheta, and
  alpha = R cos(vartheta), beta = R sin(vartheta) (Sec. 4).
* Edge along an angle: the number of those rays, counted from the inside,
  that the FP64 oracle integrator captures before the first one that
  escapes. Found by bisection over the ray index, each probe a full oracle
  trace of that one ray, all angles of a configuration probed together.
  (Inside the shadow every ray is captured and outside every ray escapes,
  so the captured rays are the first ones; the bisection finds the
  boundary index.)
* Measures (Sec. 4): D = |alpha_min + alpha_max| / 2, the mean radius
  <R> = (1/2 pi) int R dvartheta and the asymmetry
  A = 2 [(1/2 pi) int (R - <R>)^2 dvartheta]^(1/2), with R the distance of
  the ring point from the ring's centre on the alpha axis and vartheta the
  polar angle about the image centre; the upper half of the ring is
  mirrored (beta -> -beta).
* The paper's fitting formulae for <R> and A (Sec. 4).
"""
from __future__ import annotations

import math

import numpy as np

from . import CAPTURED, ESCAPED, camera, make_params, run


def polar_pixels(nr: int, r_lo: float, r_hi: float, theta: float):
    radii = r_lo + (r_hi - r_lo) * (np.arange(nr) + 0.5) / nr
    return radii, radii * math.cos(theta), radii * math.sin(theta)


def edge_counts(a: float, r_obs: float, incl: float, thetas, nr: int, r_lo: float, r_hi: float,
                params=None, nthreads: int = 0) -> np.ndarray:
    """Per angle, the number of captured rays before the first escaped one
    (bisection over the ray index, probes traced by the oracle)."""
    params = params or make_params()
    thetas = np.asarray(thetas, dtype=np.float64)
    lo = np.zeros(len(thetas), dtype=np.int64)        # ray lo - 1 is captured (or lo == 0)
    hi = np.full(len(thetas), nr, dtype=np.int64)     # ray hi escapes (or hi == nr)
    cos_t, sin_t = np.cos(thetas), np.sin(thetas)
    while np.any(lo < hi):
        act = np.where(lo < hi)[0]
        mid = (lo[act] + hi[act]) // 2
        radii = r_lo + (r_hi - r_lo) * (mid + 0.5) / nr
        x0 = np.array([camera(a, r_obs, incl, R * cos_t[j], R * sin_t[j]) for R, j in zip(radii, act)])
        st = run(params, a, x0, nthreads=nthreads).status
        cap = st == CAPTURED
        lo[act[cap]] = mid[cap] + 1
        hi[act[~cap]] = mid[~cap]
    return lo


def ray_status(a: float, r_obs: float, incl: float, theta: float, idx, nr: int, r_lo: float,
               r_hi: float, params=None) -> np.ndarray:
    """Oracle status of the listed rays along one angle."""
    params = params or make_params()
    idx = np.asarray(idx, dtype=np.int64)
    radii = r_lo + (r_hi - r_lo) * (idx + 0.5) / nr
    x0 = np.array([camera(a, r_obs, incl, R * math.cos(theta), R * math.sin(theta)) for R in radii])
    return run(params, a, x0).status


def measures(thetas, radius) -> dict:
    """D, <R>, A of the ring r = radius(vartheta) given on vartheta in [0, pi]
    (uniform, both ends included), by the definitions of Sec. 4."""
    thetas = np.asarray(thetas, dtype=np.float64)
    radius = np.asarray(radius, dtype=np.float64)
    # whole circle: angles 0 .. 2 pi - step, the lower half from beta -> -beta
    t = list(thetas)
    r = list(radius)
    for j in range(len(thetas) - 2, 0, -1):
        t.append(2.0 * math.pi - thetas[j])
        r.append(radius[j])
    t = np.array(t)
    r = np.array(r)
    al = r * np.cos(t)
    be = r * np.sin(t)
    center = (al.min() + al.max()) / 2.0
    dist = np.sqrt((al - center) ** 2 + be ** 2)
    # periodic trapezoid rule on a uniform grid = the plain mean
    mean = float(np.sum(dist) / len(dist))
    var = float(np.sum((dist - mean) ** 2) / len(dist))
    return {"D": abs(float(center)), "center": float(center), "R_mean": mean, "A": 2.0 * math.sqrt(var)}


def fit_mean_radius(a: float, incl_deg: float) -> float:
    R0 = 5.2 - 0.209 * a + 0.445 * a * a - 0.567 * a ** 3
    R1 = (0.24 - 3.3 / ((a - 0.9017) ** 2 + 0.059)) * 1e-3
    return R0 + R1 * math.cos(math.radians(2.14 * incl_deg - 22.9))


def fit_asymmetry(a: float, incl_deg: float) -> float:
    A0 = 0.332 * a ** 3 + 0.176 * a ** 21.7 + 0.0756 * a ** 195
    n = 1.55 * (1.0 - a) ** -0.022 + 1.3 * (1.0 - a) ** 0.98
    return A0 * math.sin(math.radians(incl_deg)) ** n
