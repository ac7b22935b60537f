"""Serving (continuous batching) on the GPU: requests of uneven size, spin and
inclination share one resident pool and one persistent launch per
iteration; each request's result must be the same alone and in the mix, and
the same as a plain single-batch render of its camera."""
import numpy as np
import pytest

from paper_1303_5057_amd import gray as G
from paper_1303_5057_amd import workloads as W
from paper_1303_5057_amd.serve import Server, bytes_per_photon

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32c"]


def _stream():
    return W.request_stream(14, qps=400.0, side_lo=8, side_hi=56)


def _batch_render(cam, prec):
    import torch
    b = G.Batch([cam], W.Params(precision=prec))
    res = b.run()
    torch.cuda.synchronize()
    return b.rows(b.status, 1)[0], b.rows(b.steps, 1)[0], b.rows(res.xf, 8)


@pytest.mark.parametrize("prec", PRECS)
def test_alone_equals_mix_equals_batch(prec):
    reqs = _stream()
    big = max(r.camera.n for r in reqs)
    budget = int(2.5 * big) * bytes_per_photon(prec)     # admission binds: not all fit at once
    mix_srv = Server(budget, W.Params(precision=prec), max_slots=8, slice_ms=2.0, keep_results=True)
    mix = {r.rid: r for r in mix_srv.run(reqs, realtime=True)}
    assert len(mix) == len(reqs)
    assert mix_srv.max_active >= 2                      # requests really overlapped
    assert mix_srv.max_used <= mix_srv.capacity
    assert mix_srv.admit_order == sorted(mix_srv.admit_order)   # FIFO admission
    for target in (reqs[3], reqs[9]):
        alone_srv = Server(budget, W.Params(precision=prec), max_slots=8, slice_ms=0.5,
                           keep_results=True)
        alone = alone_srv.run([W.Request(0, 0.0, target.camera)], realtime=False)[0]
        m = mix[target.rid]
        assert np.array_equal(alone.status, m.status)
        assert np.array_equal(alone.steps, m.steps)
        assert np.array_equal(alone.x, m.x)
        st, steps, xf = _batch_render(target.camera, prec)
        assert np.array_equal(st, m.status)
        assert np.array_equal(steps, m.steps)
        assert np.array_equal(xf, m.x)
        assert np.all((m.status == G.CAPTURED) | (m.status == G.ESCAPED))


def test_pool_reuse_after_retire():
    """Ranges freed by finished requests are reused; stale photons there never
    run again (they stay terminal until a new camera initialises them)."""
    reqs = [W.Request(k, 0.0, W.scaled(W.C2, 24, 20)) for k in range(6)]
    srv = Server(700 * bytes_per_photon("fp64"), W.Params(precision="fp64"), max_slots=4,
                 slice_ms=1.0, keep_results=True)
    out = srv.run(reqs, realtime=False)
    assert len(out) == 6 and srv.max_active == 1       # only one 480-photon request fits
    ref = out[0]
    for r in out[1:]:
        assert np.array_equal(r.x, ref.x) and np.array_equal(r.steps, ref.steps)


@pytest.mark.parametrize("prec", PRECS)
def test_cancel_in_flight_and_waiting(prec):
    """A request cancelled while its photons run leaves every other result
    unchanged (bit for bit against a plain render of its camera), and its
    pool range goes to the requests waiting behind it; a request cancelled
    while waiting never runs."""
    cams = [W.scaled(W.C2, 40, 32), W.scaled(W.C2, 48, 40), W.scaled(W.C1, 24, 24),
            W.scaled(W.C2, 36, 30), W.scaled(W.C1, 20, 20)]
    reqs = [W.Request(k, 0.0, c) for k, c in enumerate(cams)]
    # the pool holds requests 0 and 1 only; 2-4 wait for a free range
    cap = sum((c.n + 63) // 64 * 64 for c in cams[:2])
    srv = Server(cap * bytes_per_photon(prec), W.Params(precision=prec), max_slots=4, slice_ms=1.0,
                 keep_results=True)
    out = {r.rid: r for r in srv.run(reqs, realtime=False, cancel={1: 2, 4: 0})}
    print(f"cancel {prec}: admitted {srv.admit_order}, iterations {srv.iterations}", flush=True)
    assert sorted(out) == list(range(5))
    assert out[1].cancelled and out[4].cancelled
    assert out[1].status is None and out[4].status is None
    assert srv.admit_order == [0, 1, 2, 3]               # 4 never ran; 2 and 3 took 1's range
    assert srv.max_used <= srv.capacity
    for rid in (0, 2, 3):
        m = out[rid]
        assert not m.cancelled
        st, steps, xf = _batch_render(cams[rid], prec)
        assert np.array_equal(st, m.status)
        assert np.array_equal(steps, m.steps)
        assert np.array_equal(xf, m.x)


@pytest.mark.parametrize("prec", PRECS)
def test_per_camera_step_budget(prec):
    """gray_camera.call_steps: a camera's own step budget replaces the call's
    for its photons; resuming reproduces one uninterrupted call bit for bit."""
    import torch
    cams = [W.scaled(W.C2, 40, 32), W.scaled(W.C1, 24, 24)]
    ref = G.Batch(cams, W.Params(precision=prec))
    ref.camera_init()
    ref.integrate()
    torch.cuda.synchronize()
    b = G.Batch(cams, W.Params(precision=prec, call_steps=50))
    b.cam_arr[1].call_steps = 200
    b.camera_init()
    b.integrate()
    torch.cuda.synchronize()
    n0 = cams[0].n
    steps = b.steps[: b.n].cpu().numpy()
    st = b.status[: b.n].cpu().numpy()
    print(f"budget {prec}: max steps {steps[:n0].max()} / {steps[n0:].max()}", flush=True)
    assert steps[:n0].max() == 50 and steps[n0:].max() == 200
    # a photon still running has taken exactly its camera's budget
    assert (steps[:n0][st[:n0] == G.RUNNING] == 50).all()
    assert (steps[n0:][st[n0:] == G.RUNNING] == 200).all()
    for _ in range(200):
        if not (b.status[: b.n] == G.RUNNING).any().item():
            break
        b.integrate()
        torch.cuda.synchronize()
    for name in ("status", "steps", "x"):
        got = getattr(b, name)[: b.n] if name != "x" else b.x.view(8, b.stride)[:, : b.n]
        want = getattr(ref, name)[: ref.n] if name != "x" else ref.x.view(8, ref.stride)[:, : ref.n]
        assert torch.equal(got, want), name
    if prec == "fp32c":
        assert torch.equal(b.lo.view(8, b.stride)[:, : b.n], ref.lo.view(8, ref.stride)[:, : ref.n])
