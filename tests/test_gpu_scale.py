"""Full-size workloads through the C ABI, checked against the oracle on
deterministic samples of their rays (gathered on the device), and a batch
of 2^27 photons for the large-index paths:

* the 4096 x 4096 a = 0.9375, i = 17 deg grid with the equatorial recorder
  on, in FP32C (the precision this workload is specified in);
* the 256-camera sweep (~48M rays) in one persistent launch.
"""
import numpy as np
import pytest

from parity import RTOL, STATE_BAND, compare, run_oracle
from paper_1303_5057_amd import gray as G
from paper_1303_5057_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gather(b, res, ids):
    import torch
    idx = torch.as_tensor(ids, dtype=torch.int64, device=b.x.device)
    rows = lambda t, k: t.view(k, b.stride)[:, idx].cpu().numpy()
    out = {"status": rows(b.status, 1)[0], "steps": rows(b.steps, 1)[0],
           "x": rows(res.xf, 8).T, "counters": rows(b.counters, 3)}
    if b.mark is not None:
        out["mark"] = rows(b.mark, 8).T
    if b.disk is not None:
        out["disk"] = rows(b.disk, 3).T
    return out


def test_c3_full_grid_fp32c_sampled():
    import torch
    cam, p = W.C3, W.C3_PARAMS
    b = G.Batch([cam], p, mark=False)
    res = b.run(cons=False)
    torch.cuda.synchronize()
    ids = W.subsample_ids(cam, 64)
    g = _gather(b, res, ids)
    o = run_oracle(cam, p, ids)
    rep = compare(g["status"], g["steps"], g["x"], g["counters"], o, RTOL["fp32c"],
                  STATE_BAND["fp32c"], skip_locked=True)
    print(rep, flush=True)
    assert rep.flag_mismatch == 0 and rep.state_bad == 0 and rep.counter_bad == 0
    assert rep.step_mismatch <= 0.002 * rep.n
    same = (g["steps"] == o.steps) & (g["status"] == o.status) & (o.band_dist > 1e-2)
    hit = same & (o.disk[:, 0] > 0)
    assert np.array_equal(g["disk"][same, 0] > 0, o.disk[same, 0] > 0)
    assert np.allclose(g["disk"][hit], o.disk[hit], rtol=1e-3, atol=1e-3)
    # every ray stops; the recorder saw a good part of the image
    st = b.status[: b.n]
    assert int((st == G.RUNNING).sum()) == 0
    assert float((b.disk.view(3, b.stride)[0, : b.n] > 0).float().mean()) > 0.2


def test_c4_sweep_one_launch_fp64_sampled():
    import torch
    cams = W.sweep_cameras()
    assert len(cams) == 256
    p = W.Params()
    b = G.Batch(cams, p, mark=False)
    res = b.run(cons=False)
    torch.cuda.synchronize()
    counts = res.counts.view(-1, 5).cpu().numpy()
    assert counts[:, G.RUNNING].sum() == 0
    assert np.array_equal(counts.sum(axis=1), [c.n for c in cams])
    first = np.cumsum([0] + [c.n for c in cams])
    bad = 0
    for k in range(0, 256, 8):                      # every 8th camera, 1 ray in 97
        cam = cams[k]
        local = np.arange(k % 97, cam.n, 97)
        g = _gather(b, res, first[k] + local)
        o = run_oracle(cam, p, local)
        rep = compare(g["status"], g["steps"], g["x"], g["counters"], o, RTOL["fp64"])
        bad += rep.flag_mismatch + rep.state_bad + rep.counter_bad
        assert rep.step_mismatch <= max(1, 0.002 * rep.n), (k, rep)
    assert bad == 0


def test_c4_sweep_one_launch_fp32c_sampled():
    """The 256-camera sweep in FP32C, one persistent launch, against the
    oracle on every 8th camera (1 ray in 97), under the FP32C rules: the
    excluded fraction, step mismatches and flipped fallback decisions are
    summed over the sample and bounded."""
    import torch
    cams = W.sweep_cameras()
    p = W.Params(precision="fp32c")
    b = G.Batch(cams, p)
    res = b.run(cons=False)
    torch.cuda.synchronize()
    counts = res.counts.view(-1, 5).cpu().numpy()
    assert counts[:, G.RUNNING].sum() == 0
    first = np.cumsum([0] + [c.n for c in cams])
    n = flag = state = steps = flips = 0
    excluded = excluded_esc = 0.0
    for k in range(0, 256, 8):
        cam = cams[k]
        local = np.arange(k % 97, cam.n, 97)
        g = _gather(b, res, first[k] + local)
        o = run_oracle(cam, p, local)
        rep = compare(g["status"], g["steps"], g["x"], g["counters"], o, RTOL["fp32c"], STATE_BAND["fp32c"],
                      skip_locked=True, g_mark=g["mark"])
        n += rep.n
        flag += rep.flag_mismatch
        state += rep.state_bad
        steps += rep.step_mismatch
        flips += rep.flips
        excluded += rep.excluded * rep.n
        excluded_esc += rep.excluded_escaped * rep.n
    print(f"FP32C sweep sample: rays {n} flag {flag} state {state} step mismatch {steps} flips {flips} "
          f"excluded {excluded / n:.4f} (escaped {excluded_esc / n:.4f})", flush=True)
    assert flag == 0 and state == 0
    assert steps <= 2e-3 * n and flips <= 1e-3 * n
    assert excluded / n <= 0.25 and excluded_esc / n <= 0.04


def test_large_batch_every_photon_advances_once_per_call():
    """2^27 photons in one batch (134M: ids, launch-order entries and queue
    positions span 1/16 of their 32-bit range, grabs are 512 ids): with
    call_steps = 1 each call advances every running photon by exactly one
    step."""
    import torch
    cam = W.Camera(0.6, 1000.0, W.deg(40.0), 8192, 16384, -12.0, 12.0, -12.0, 12.0)
    assert cam.n == 1 << 27
    b = G.Batch([cam], W.Params(call_steps=1), counters=False, mark=False)
    b.camera_init()
    for k in (1, 2):
        b.integrate()
        torch.cuda.synchronize()
        steps = b.steps[: b.n]
        assert int((steps == k).sum().item()) == b.n, k
    assert int((b.status[: b.n] == G.RUNNING).sum().item()) == b.n
    res = b.classify(xf=False, cons=False, counts=True)
    assert res.counts.view(-1, 5).cpu().numpy()[0].tolist() == [b.n, 0, 0, 0, 0]
    del b, res
    torch.cuda.empty_cache()


def test_c2_full_grid_fp32c_against_oracle():
    """Every ray of the 512 x 512 edge-on grid in FP32C against the FP64
    oracle, under the FP32C rules (tests/parity.py): flags exact outside the
    1e-3 M band; states to 1e-3 where step counts and fallback decisions
    agree, for rays outside the 2e-2 M band and not Euler-locked; the rays
    with another step count or a flipped fallback decision, and the rays left
    out, counted and bounded."""
    import analytic
    import torch
    from parity import state_close
    cam, p = W.C2, W.Params(precision="fp32c")
    b = G.Batch([cam], p)
    res = b.run()
    torch.cuda.synchronize()
    st, sp = b.rows(b.status, 1)[0], b.rows(b.steps, 1)[0]
    x, ctr = b.rows(res.xf, 8).T, b.rows(b.counters, 3)
    c0 = b.rows(res.cons, 9)[0:3]
    o = run_oracle(cam, p)
    mk = b.rows(b.mark, 8).T
    rep = compare(st, sp, x, ctr, o, RTOL["fp32c"], STATE_BAND["fp32c"], skip_locked=True, g_mark=mk)
    print(rep, flush=True)
    # where the mismatches fall (diagnostics)
    smin = analytic.polar_turning_sin(cam.a, c0[0], c0[1], c0[2])
    at_mark = (o.status == G.CAPTURED) & (o.mark[:, 1] > 0)
    ok, err = state_close(np.where(at_mark[:, None], mk, x), np.where(at_mark[:, None], o.mark, o.x), 1e-3)
    same = (sp == o.steps) & (st == o.status)
    flip = same & ((ctr[0] != o.n_euler) | (ctr[1] != o.n_remap))
    cons = (o.band_dist > STATE_BAND["fp32c"]) & (o.n_euler <= 0.1 * o.steps)
    e = np.where(same & cons & ~flip, err.max(axis=1), 0.0)
    for i in np.argsort(-e)[:5]:
        print(f"  worst compared ray {i}: err {e[i]:.2e} comp {err[i].argmax()} band {o.band_dist[i]:.3g} "
              f"sin_min {smin[i]:.3f} FP64 steps {ctr[2][i]} of {sp[i]}", flush=True)
    fl = np.nonzero(flip & cons)[0]
    print("flipped rays: euler GPU/oracle", [(int(ctr[0][i]), int(o.n_euler[i])) for i in fl[:10]], flush=True)
    assert rep.flag_mismatch == 0 and rep.state_bad == 0
    assert rep.flips <= 1e-3 * rep.n
    assert rep.step_mismatch <= 2e-3 * rep.n
    assert rep.excluded <= 0.25 and rep.excluded_escaped <= 0.04
