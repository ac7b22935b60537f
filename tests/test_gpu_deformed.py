"""GPU parity in the deformed Kerr metric (the non-Kerr spacetimes of Sec. 1):
the metric-generic right-hand side (forward-mode derivatives of the metric)
through the C ABI, against the FP64 oracle (complex-step derivatives, the
same metric written independently) and against closed forms.

* deform = 0 through the generic path equals the Kerr fast path and the
  oracle under the usual FP64 rules;
* deform = 1.5 at a = 0.6: flags equal the oracle's except on pixels whose
  oracle flag differs from a neighbour's (the shadow edge, where no closed
  form locates the critical curve), states match to 1e-5 where step counts
  agree, Euler and remap counters exactly;
* a = 0, deform = 2 and -1: flags follow the closed-form critical impact
  parameter of the static deformed metric, without the oracle;
* E and L_z are conserved by the GPU integration, Carter's Q is not.
"""
import numpy as np
import pytest

import analytic
from parity import RTOL, compare, run_gpu, run_oracle
from paper_1303_5057_amd import gray as G
from paper_1303_5057_amd import workloads as W

pytestmark = pytest.mark.gpu

DEF = G.GRAY_METRIC_DEFORMED


def _cam(a, incl_deg, n, m, deform, half=8.0, metric=DEF):
    return W.Camera(a, 1000.0, np.radians(incl_deg), n, m, -half, half, -half, half, metric=metric, deform=deform)


def test_generic_path_at_zero_deviation_matches_kerr():
    kerr = W.scaled(W.C2, 61, 53)
    gen = _cam(0.99, 90.0, 61, 53, 0.0)
    p = W.Params()
    gk = run_gpu([kerr], p)
    gg = run_gpu([gen], p)
    o = run_oracle(gen, p)
    rep = compare(gg.status, gg.steps, gg.x.T, gg.counters, o, RTOL["fp64"])
    print(rep, flush=True)
    assert rep.flag_mismatch == 0 and rep.state_bad == 0 and rep.counter_bad == 0
    assert rep.step_mismatch <= 0.002 * rep.n
    far = o.band_dist > 1e-3
    assert np.array_equal(gk.status[far], gg.status[far])
    same = (gk.steps == gg.steps) & (gk.status == gg.status)
    assert same.mean() > 0.99
    err = np.abs(gk.x[:, same] - gg.x[:, same]) / (np.abs(gk.x[:, same]) + 1.0)
    assert err.max() < 1e-8


def _edge_pixels(status, nx, ny):
    s = status.reshape(ny, nx)
    edge = np.zeros_like(s, dtype=bool)
    edge[:, 1:] |= s[:, 1:] != s[:, :-1]
    edge[:, :-1] |= s[:, 1:] != s[:, :-1]
    edge[1:, :] |= s[1:, :] != s[:-1, :]
    edge[:-1, :] |= s[1:, :] != s[:-1, :]
    return edge.ravel()


def test_deformed_spinning_hole_against_oracle():
    cam = _cam(0.6, 50.0, 64, 56, 1.5)
    p = W.Params()
    g = run_gpu([cam], p)
    o = run_oracle(cam, p)
    edge = _edge_pixels(o.status, cam.nx, cam.ny)
    assert edge.mean() < 0.1
    assert np.array_equal(g.status[~edge], o.status[~edge])
    same = (g.steps == o.steps) & (g.status == o.status)
    assert (~same).mean() <= 2e-3
    r = np.abs(o.x[:, 1])
    floor = np.stack([np.ones_like(r)] * 6 + [1.0 / r, 1.0 / r], axis=1)
    err = np.abs(g.x.T - o.x) / (np.abs(o.x) + floor)
    assert err[same].max() <= RTOL["fp64"], err[same].max()
    assert np.array_equal(g.counters[0][same], o.n_euler[same])
    assert np.array_equal(g.counters[1][same], o.n_remap[same])
    assert set(np.unique(g.status)) == {G.CAPTURED, G.ESCAPED}
    # constants of motion: E and L_z conserved, Carter's Q not (rows 6..8: drifts)
    clean = (g.status == G.ESCAPED) & (g.counters[0] == 0) & ~edge
    assert clean.sum() > 100
    assert g.cons[6, clean].max() <= 1e-5 and g.cons[7, clean].max() <= 1e-5
    assert g.cons[8, clean].max() > 1e-4


@pytest.mark.parametrize("deform", [2.0, -1.0])
def test_static_deformed_shadow_closed_form(deform):
    cam = _cam(0.0, 60.0, 72, 72, deform)
    g = run_gpu([cam], W.Params())
    b = np.sqrt(g.cons[1] ** 2 + g.cons[2]) / g.cons[0]      # E0, L0, Q0 at the camera
    bc = analytic.deformed_static_critical_impact(deform)
    far = np.abs(b - bc) > 2e-3
    assert far.mean() > 0.98
    assert np.array_equal((g.status == G.CAPTURED)[far], (b < bc)[far])
    assert abs(bc - np.sqrt(27.0)) > 0.05
