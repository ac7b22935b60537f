"""Seeded synthetic workloads: camera descriptors and integrator parameters.

This module is shared by the GPU path and the oracle tests and holds none of
the method's arithmetic: it only says which cameras (spin, inclination, image
plane window, grid size) and which integrator settings a workload uses, and
draws seeded random camera parameters for the sweep and serving workloads.

Every workload is a synthetic image-plane grid, as are the paper's own
(grid projection and ns-per-step benchmarks in Sec. 3, photon-ring study in
Sec. 4); no dataset exists or is needed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import List

import numpy as np

SEED_BASE = 20260000


@dataclass(frozen=True)
class Camera:
    """Kerr spin a, observer distance r_obs (M), inclination incl (radians),
    spacetime (metric, deform), and an nx x ny image-plane grid: kind 0,
    cell-centred over
    [alpha_lo, alpha_hi] x [beta_lo, beta_hi] (M); kind 1 (polar), nx
    cell-centred radii in [alpha_lo, alpha_hi] times ny angles from beta_lo
    to beta_hi inclusive (radians)."""
    a: float
    r_obs: float
    incl: float
    nx: int
    ny: int
    alpha_lo: float
    alpha_hi: float
    beta_lo: float
    beta_hi: float
    kind: int = 0
    # spacetime: 0 Kerr; 1 Kerr deformed by the Johannsen-Psaltis deviation
    # function with parameter `deform` (epsilon_3)
    metric: int = 0
    deform: float = 0.0

    @property
    def n(self) -> int:
        return self.nx * self.ny


@dataclass(frozen=True)
class Params:
    """Integrator settings. Defaults are the paper's Delta ~ 1/32 and
    epsilon ~ 1e-3 with the h/9 Euler fallback (Sec. 2), capture at
    r < r_bh (1 + 1e-3), escape beyond 1000 M moving outward."""
    step_frac: float = 1.0 / 32.0
    horizon_eps: float = 1e-3
    r_escape: float = 1000.0
    xi_eps: float = 1e-3
    euler_div: float = 9.0
    disk_rmin: float = -1.0      # < 0: r_ISCO of each camera's spin
    disk_rmax: float = 50.0
    max_steps: int = 65536
    call_steps: int = 0
    precision: str = "fp64"      # "fp64" or "fp32c"
    record_disk: bool = False
    # FP32C: a photon continues in double precision once it comes near the
    # horizon, a pole or a radial turning point (r < r_bh (1 + fp64_horizon),
    # sin(theta) < fp64_pole, |k^r| < fp64_turn |k^t|); only the horizon zone
    # is on by default.
    fp64_horizon: float = 0.02
    fp64_pole: float = 0.0
    fp64_turn: float = 0.0
    # treatment of the polar axis (Sec. 2): 0 the production null-condition
    # monitor, 1 the earlier Euler step on pole crossings, 2 none
    pole_mode: int = 0


def deg(x: float) -> float:
    return math.radians(x)


# Schwarzschild, i = 60 deg, 64 x 64 over [-10, 10]^2: the sqrt(27) shadow check.
C1 = Camera(0.0, 1000.0, deg(60.0), 64, 64, -10.0, 10.0, -10.0, 10.0)
# Kerr a = 0.99 edge-on, 512 x 512 over [-8, 8]^2: shadow vs the critical curve.
C2 = Camera(0.99, 1000.0, deg(90.0), 512, 512, -8.0, 8.0, -8.0, 8.0)
# Kerr a = 0.9375, i = 17 deg, 4096 x 4096 over [-12, 12]^2 with the
# equatorial-crossing recorder on, window [r_ISCO, 50 M].
C3 = Camera(0.9375, 1000.0, deg(17.0), 4096, 4096, -12.0, 12.0, -12.0, 12.0)
C3_PARAMS = Params(record_disk=True, disk_rmin=-1.0, disk_rmax=50.0, precision="fp32c")

# Grid projection (Sec. 3): a uniform Cartesian image-plane grid projected
# onto the equatorial plane (first crossing at any radius, recorder window
# [0, 1000] M) for spins 0 and 0.95 at inclinations 0 and 60 deg; the
# a = 0.95, i = 60 deg case is the paper's run-time-versus-n benchmark.
PROJECTION_CONFIGS = ((0.0, 0.0), (0.0, 60.0), (0.95, 0.0), (0.95, 60.0))
PROJECTION_HALF_WIDTH = 12.0
PROJECTION_PARAMS = Params(record_disk=True, disk_rmin=0.0, disk_rmax=1000.0)


def projection_camera(a: float, incl_deg: float, side: int,
                      half_width: float = PROJECTION_HALF_WIDTH) -> Camera:
    return Camera(a, 1000.0, deg(incl_deg), side, side, -half_width, half_width, -half_width,
                  half_width)


# The paper's pole test (Sec. 2): a = 0.99, r0 cos(theta0) = 1000 M,
# r0 sin(theta0) = 4.833605 M, phi0 = 0. With the observer on the axis
# (incl = 0) the screen point (alpha, beta) = (0, -4.833605) has exactly
# that position.
POLE_A = 0.99
POLE_R_SIN = 4.833605


def pole_camera(phi0: float = 0.0) -> Camera:
    """1x1 camera of the pole test rotated to azimuth phi0 (the paper notes the
    outcome does not depend on phi0)."""
    al = POLE_R_SIN * math.sin(phi0)
    be = -POLE_R_SIN * math.cos(phi0)
    return Camera(POLE_A, 1000.0, 0.0, 1, 1, al, al, be, be)


def scaled(cam: Camera, nx: int, ny: int | None = None) -> Camera:
    """Same window at a different resolution."""
    return replace(cam, nx=nx, ny=ny if ny is not None else nx)


def _rng(index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index))


def _log_uniform_side(g: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))


def sweep_cameras(count: int = 256, side_lo: int = 64, side_hi: int = 1024,
                  a_hi: float = 0.998, incl_lo_deg: float = 1.0, incl_hi_deg: float = 89.0,
                  window: float = 10.0, first_index: int = 0) -> List[Camera]:
    """Batched sweep: camera k uses seed SEED_BASE + k; side log-uniform in
    [side_lo, side_hi], spin uniform in [0, a_hi], inclination uniform in degrees."""
    cams = []
    for k in range(first_index, first_index + count):
        g = _rng(k)
        side = _log_uniform_side(g, side_lo, side_hi)
        a = g.uniform(0.0, a_hi)
        incl = deg(g.uniform(incl_lo_deg, incl_hi_deg))
        cams.append(Camera(a, 1000.0, incl, side, side, -window, window, -window, window))
    return cams


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    camera: Camera


def request_stream(count: int, qps: float, seed_offset: int = 100000, side_lo: int = 32,
                   side_hi: int = 2048, a_hi: float = 0.998, window: float = 10.0) -> List[Request]:
    """Serving workload: Poisson arrivals at rate qps; request k draws its camera
    from seed SEED_BASE + seed_offset + k (side log-uniform, spin and
    inclination uniform in [0, a_hi] and [0, 90] degrees)."""
    arr = np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset - 1))
    gaps = arr.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(count):
        g = _rng(seed_offset + k)
        side = _log_uniform_side(g, side_lo, side_hi)
        a = g.uniform(0.0, a_hi)
        incl = deg(g.uniform(0.0, 90.0))
        reqs.append(Request(k, float(t[k]), Camera(a, 1000.0, incl, side, side, -window, window,
                                                   -window, window)))
    return reqs


def subsample_ids(cam: Camera, every: int) -> np.ndarray:
    """Pixel ids (iy * nx + ix) of every `every`-th row and column."""
    iy, ix = np.meshgrid(np.arange(0, cam.ny, every), np.arange(0, cam.nx, every), indexing="ij")
    return (iy * cam.nx + ix).ravel().astype(np.int64)
