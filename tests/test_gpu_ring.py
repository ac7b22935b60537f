"""Photon-ring study (Sec. 4) on the GPU against the CPU oracle.

Each configuration is traced at the study's full resolution (6000 radii in
(1.5, 7.5) M times 181 angles in [0, pi], image plane at 1000 M) by libgray
through the C ABI: one polar camera per angle, the captured count per camera
from gray_classify. The oracle finds the same edge along every angle by
bisection over the same rays, each probe a full FP64 trace (oracle/ring.py).

* Edge counts: equal, except that a ray within rounding of the critical
  curve may fall either way (one ray), and within 5 deg of the beta axis,
  where rays with L_z ~ 0 cross the polar axis next to the critical curve
  and lock into Euler steps, the two integrators' errors may move the edge
  by up to 3 rays.
* Measures D, <R>, A from the GPU edges: within the grid spacing of the
  oracle's measures from the oracle's edges.
* A subset of the parameter study against the paper's fits for <R> and A
  (a consistency check: the fits are approximate; the exact critical curve
  differs from them by up to 0.025 M in <R> and ~10% in A).
"""
import math

import numpy as np
import pytest

from oracle import ring as OR
from paper_1303_5057_amd import ring as GR

pytestmark = pytest.mark.gpu

CONFIGS = [(0.0, 60.0), (0.9, 60.0), (0.99, 90.0), (0.6, 0.0), (GR.SPINS[15], 45.0)]


def test_ring_edges_and_measures_match_oracle():
    rings, timing = GR.trace_rings(CONFIGS)
    print(timing, flush=True)
    dr = (GR.R_HI - GR.R_LO) / GR.NR
    thetas = np.linspace(0.0, math.pi, GR.NTH)
    polar = np.abs(np.cos(thetas)) < math.sin(math.radians(5.0))
    for rg, (a, inc) in zip(rings, CONFIGS):
        assert rg.unfinished == 0
        want = OR.edge_counts(a, GR.R_OBS, math.radians(inc), thetas, GR.NR, GR.R_LO, GR.R_HI)
        diff = rg.n_captured - want
        print(a, inc, "mismatched angles", int(np.count_nonzero(diff)), "max", int(np.abs(diff).max()),
              flush=True)
        assert np.all(np.abs(diff[~polar]) <= 1)
        assert np.count_nonzero(diff[~polar]) <= 2
        assert np.all(np.abs(diff[polar]) <= 3)
        mo = OR.measures(thetas, GR.R_LO + want * dr)
        mg = rg.measures
        print(a, inc, "gpu", mg, "oracle", mo, flush=True)
        assert abs(mg["R_mean"] - mo["R_mean"]) <= dr
        assert abs(mg["D"] - mo["D"]) <= 2 * dr
        assert abs(mg["A"] - mo["A"]) <= 2 * dr
    # Schwarzschild: the sqrt(27) circle
    m0 = rings[0].measures
    assert abs(m0["R_mean"] - math.sqrt(27.0)) < 5e-3 and m0["D"] < 2 * dr and m0["A"] < 4 * dr


def test_ring_study_subset_vs_paper_fits():
    spins = [GR.SPINS[j] for j in (0, 5, 10, 13, 15)]
    incls = [0, 30, 60, 90]
    rings, timing = GR.trace_rings([(a, i) for a in spins for i in incls])
    print(timing, flush=True)
    for rg in rings:
        fr = OR.fit_mean_radius(rg.a, rg.incl_deg)
        fa = OR.fit_asymmetry(rg.a, rg.incl_deg)
        m = rg.measures
        print(f"a={rg.a:.4f} i={rg.incl_deg:2.0f} <R>={m['R_mean']:.4f} fit {fr:.4f} "
              f"A={m['A']:.4f} fit {fa:.4f} D={m['D']:.4f}", flush=True)
        assert rg.unfinished == 0
        # The fits are approximate: against the exact critical curve (which
        # the traced rings match to the grid spacing) they are off by up to
        # 0.025 M in <R> and ~10% in A at intermediate inclinations.
        assert abs(m["R_mean"] - fr) < 0.03
        assert abs(m["A"] - fa) < 0.02 + 0.15 * fa
