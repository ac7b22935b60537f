"""Photon-ring study (Sec. 4): the outline of the black-hole shadow for 16
spins a_j = 1 - 10^(-j/5) and 19 inclinations i = 0, 5, ..., 90 deg, traced
on a polar image-plane grid of 6000 radii in (1.5, 7.5) M times 181 angles
in [0, pi] with the image plane at r = 1000 M, and the ring measures the
paper defines from it: the horizontal displacement D, the mean radius <R>
and the asymmetry A, next to the paper's fitting formulae for <R> and A.

Every ray is traced by libgray (camera_init, integrate, classify): each
angle of each configuration is one polar camera of nx radii and one angle,
so the per-camera status counts that gray_classify returns give the number
of captured rays along that angle. The ring edge along the angle is then

    R_edge = R_lo + N_captured (R_hi - R_lo) / nx,

the boundary between the captured rays (inside the shadow, the first
N_captured radii) and the escaped ones. The measures use the full circle,
the upper half mirrored (the image of a Kerr hole is symmetric under
beta -> -beta), sampled every (pi / (nth - 1)) in the grid angle.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import gray as G
from .workloads import Camera, Params

SPINS: Tuple[float, ...] = tuple(1.0 - 10.0 ** (-j / 5.0) for j in range(16))
INCLS_DEG: Tuple[int, ...] = tuple(range(0, 91, 5))
NR, NTH = 6000, 181
R_LO, R_HI = 1.5, 7.5
R_OBS = 1000.0


def ring_cameras(a: float, incl_deg: float, nr: int = NR, nth: int = NTH, r_lo: float = R_LO,
                 r_hi: float = R_HI, r_obs: float = R_OBS) -> List[Camera]:
    """One polar camera per angle vartheta_j = j pi / (nth - 1), each a row
    of nr cell-centred radii in (r_lo, r_hi)."""
    incl = math.radians(incl_deg)
    thetas = np.linspace(0.0, math.pi, nth)
    return [Camera(a, r_obs, incl, nr, 1, r_lo, r_hi, float(t), float(t), kind=G.GRAY_CAMERA_POLAR)
            for t in thetas]


def ring_measures(thetas: np.ndarray, radius: np.ndarray) -> Dict[str, float]:
    """D, <R> and A of a ring given its edge radius along the grid angles
    thetas (upper half, 0 .. pi inclusive, uniform).

    Readings: the centre of the ring is (c, 0) with c = (alpha_min +
    alpha_max) / 2, and D = |c|; R is the distance of an edge point from
    that centre and the averages are over the grid angle vartheta (the
    polar angle about the image centre), on the full circle."""
    full_t = np.concatenate([thetas, 2.0 * math.pi - thetas[-2:0:-1]])
    full_r = np.concatenate([radius, radius[-2:0:-1]])
    alpha0 = full_r * np.cos(full_t)
    beta0 = full_r * np.sin(full_t)
    c = 0.5 * (alpha0.min() + alpha0.max())
    R = np.hypot(alpha0 - c, beta0)
    mean_r = float(R.mean())
    asym = float(2.0 * math.sqrt(np.mean((R - mean_r) ** 2)))
    return {"D": abs(float(c)), "center": float(c), "R_mean": mean_r, "A": asym}


def paper_fit_mean_radius(a: float, incl_deg: float) -> float:
    """The paper's fit for <R> (Sec. 4), arguments of cos in degrees."""
    r0 = 5.2 - 0.209 * a + 0.445 * a ** 2 - 0.567 * a ** 3
    r1 = (0.24 - 3.3 / ((a - 0.9017) ** 2 + 0.059)) * 1e-3
    return r0 + r1 * math.cos(math.radians(2.14 * incl_deg - 22.9))


def paper_fit_asymmetry(a: float, incl_deg: float) -> float:
    """The paper's fit for A (Sec. 4)."""
    a0 = 0.332 * a ** 3 + 0.176 * a ** 21.7 + 0.0756 * a ** 195
    n = 1.55 * (1.0 - a) ** (-0.022) + 1.3 * (1.0 - a) ** 0.98
    return a0 * math.sin(math.radians(incl_deg)) ** n


@dataclass
class RingResult:
    a: float
    incl_deg: float
    thetas: np.ndarray
    n_captured: np.ndarray      # per angle
    radius: np.ndarray          # edge radius per angle
    measures: Dict[str, float]
    unfinished: int             # rays that hit max_steps or went non-finite


def trace_rings(configs: Sequence[Tuple[float, float]], params: Params = Params(), nr: int = NR,
                nth: int = NTH, r_lo: float = R_LO, r_hi: float = R_HI) -> Tuple[List[RingResult], Dict]:
    """Trace every (a, incl_deg) configuration in ONE batch (one persistent
    integrate launch) and return the rings plus timing: integrate time from
    HIP events and the photon-steps it took."""
    import torch
    cams: List[Camera] = []
    for a, inc in configs:
        cams.extend(ring_cameras(a, inc, nr, nth, r_lo, r_hi))
    b = G.Batch(cams, params, counters=False, mark=False)
    t0 = time.perf_counter()
    b.camera_init()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.integrate()
    e1.record()
    res = b.classify(xf=False, cons=False, counts=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts = res.counts.view(len(cams), 5).cpu().numpy()
    steps = int(b.steps[: b.n].to(torch.int64).sum().item())
    thetas = np.linspace(0.0, math.pi, nth)
    dr = (r_hi - r_lo) / nr
    out = []
    for k, (a, inc) in enumerate(configs):
        c = counts[k * nth:(k + 1) * nth]
        ncap = c[:, G.CAPTURED].astype(np.int64)
        radius = r_lo + ncap * dr
        out.append(RingResult(a, inc, thetas, ncap, radius, ring_measures(thetas, radius),
                              int(c[:, G.UNFINISHED].sum() + c[:, G.NONFINITE].sum())))
    ms = e0.elapsed_time(e1)
    timing = {"rays": b.n, "cameras": len(cams), "photon_steps": steps, "integrate_ms": ms,
              "ns_per_photon_step": ms * 1e6 / max(1, steps), "wall_s": wall}
    del b, res
    return out, timing


def study(spins: Sequence[float] = SPINS, incls: Sequence[float] = INCLS_DEG, **kw):
    """The full parameter study: every (spin, inclination) pair in one batch."""
    return trace_rings([(a, i) for a in spins for i in incls], **kw)
