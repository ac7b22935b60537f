"""gray_integrate_static (the entry point for callers that cannot allocate)
against gray_integrate, through the C ABI.

Both calls run the same kernels; only the workspace differs (the library's
static per-device array instead of a caller buffer). A photon's result does
not depend on the workspace or the launch order, so every output must be
identical bit for bit. Two static calls run back to back, the second on a
smaller batch, so the second starts from the first one's leftovers in the
shared array; work-list mode is covered as well.
"""
import numpy as np
import pytest
import torch

from paper_1303_5057_amd import gray as G
from paper_1303_5057_amd import workloads as W

pytestmark = pytest.mark.gpu


def _outputs(b):
    torch.cuda.synchronize()
    out = {"status": b.status[: b.n].cpu().numpy(), "steps": b.steps[: b.n].cpu().numpy(),
           "x": b.x.view(8, b.stride)[:, : b.n].cpu().numpy(),
           "counters": b.counters.view(3, b.stride)[:, : b.n].cpu().numpy(),
           "mark": b.mark.view(8, b.stride)[:, : b.n].cpu().numpy()}
    if b.lo is not None:
        out["lo"] = b.lo.view(8, b.stride)[:, : b.n].cpu().numpy()
    return out


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), f"{what}: {k} differs"


def _pair(cams, prec, **kw):
    """(results of gray_integrate, results of gray_integrate_static) on the same batch."""
    params = W.Params(precision=prec, **kw)
    ref = G.Batch(cams, params)
    ref.camera_init()
    ref.integrate()
    r = _outputs(ref)
    del ref
    b = G.Batch(cams, params)
    b.camera_init()
    b.integrate_static()
    return r, _outputs(b)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_static_equals_workspace_call_twice_then_smaller(prec):
    big = [W.scaled(W.C2, 160, 128), W.scaled(W.C1, 37, 29)]
    small = [W.scaled(W.C2, 61, 43)]
    for what, cams in (("first call", big), ("second, smaller call", small)):
        print(f"no-alloc {prec} {what}: {sum(c.n for c in cams)} photons", flush=True)
        r, s = _pair(cams, prec)
        assert (r["status"] != G.RUNNING).all()
        _same(r, s, f"{prec} {what}")


def test_static_resumable_and_classify():
    """Resumed static calls (call_steps) reproduce one gray_integrate call."""
    cams = [W.scaled(W.C2, 48, 40)]
    params = W.Params()
    ref = G.Batch(cams, params)
    ref.camera_init()
    ref.integrate()
    r = _outputs(ref)
    b = G.Batch(cams, params)
    b.camera_init()
    b.set_call_steps(97)
    for _ in range(200):
        b.integrate_static()
        torch.cuda.synchronize()
        if not (b.status[: b.n] == G.RUNNING).any().item():
            break
    _same(r, _outputs(b), "resumed")
    res = b.classify()
    torch.cuda.synchronize()
    assert np.array_equal(b.rows(res.flag, 1)[0], r["status"])


def test_static_work_list_mode():
    """Work-list mode (the serving loop's): the static workspace holds only
    the header and camera table; lists are swapped between calls until no
    photon is left running."""
    cams = [W.scaled(W.C2, 40, 32)]
    params = W.Params()
    ref = G.Batch(cams, params)
    ref.camera_init()
    ref.integrate()
    r = _outputs(ref)
    b = G.Batch(cams, params)
    b.camera_init()
    n = b.n
    wl = [torch.full((n + G.GRAY_WORKLIST_SLACK,), -1, dtype=torch.int32, device="cuda") for _ in range(2)]
    wl[0][:n] = torch.arange(n, dtype=torch.int32, device="cuda")
    wc = torch.zeros(2, dtype=torch.int32, device="cuda")
    wc[0] = n
    pp = G.params_struct(params)
    pp.flags |= G.GRAY_WORKLIST
    pp.call_steps = 150
    k = 0
    for _ in range(500):
        st = G.gray_state(b.state.x, b.state.lo, b.state.status, b.state.steps, b.state.cam,
                          b.state.counters, b.state.mark, None, n, b.stride,
                          wl[k].data_ptr(), wl[1 - k].data_ptr(),
                          wc.data_ptr() + 4 * k, wc.data_ptr() + 4 * (1 - k))
        G.gray_integrate_static(b.cam_arr, 1, pp, st, G.current_stream())
        torch.cuda.synchronize()
        if int(wc[1 - k].item()) == 0:
            break
        k = 1 - k
    assert int(wc[1 - k].item()) == 0
    _same(r, _outputs(b), "work lists")


def test_static_rejects_oversized_batch():
    p = G.params_struct(W.Params())
    n = 1 << 23
    assert G.gray_workspace_size(n, 1, p) > G.GRAY_STATIC_WORKSPACE_BYTES
    cam = W.Camera(0.5, 1000.0, 1.0, 4096, n // 4096, -5, 5, -5, 5)
    # never dereferenced: the size check fails on the host first
    s = G.gray_state(0x1000, None, 0x2000, 0x3000, 0x4000, None, None, None, n, n)
    with pytest.raises(G.GrayError) as e:
        G.gray_integrate_static(G.camera_array([cam]), 1, p, s)
    assert e.value.code == G.GRAY_EWORKSPACE
