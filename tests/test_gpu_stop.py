"""The host-set stop request of gray_integrate (gray_state.stop, a watchdog),
through the C ABI.

A call that reads a set flag stores every photon after at most its next step
(GRAY_RUNNING, as at the end of call_steps); later calls then continue every
photon bit for bit, so the final results equal those of one uninterrupted
call. Covered: the flag set before the launch (dense and work-list mode) and
set by the host while the kernel runs (the flag in host memory mapped for
the device), in both precisions; in FP32C the photons of the FP64 waves are
paused too. Every kernel ends on its own either way; the flag only makes it
end sooner.
"""
import ctypes
import time

import numpy as np
import pytest
import torch

from paper_1303_5057_amd import gray as G
from paper_1303_5057_amd import workloads as W

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32c"]


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


def _reference(cams, params):
    ref = G.Batch(cams, params)
    ref.camera_init()
    ref.integrate()
    out = _outputs(ref)
    del ref
    return out


def _finish(b, what):
    for _ in range(20):
        b.integrate()
        torch.cuda.synchronize()
        if not (b.status[: b.n] == G.RUNNING).any().item():
            return
    raise AssertionError(f"{what}: photons still running")


@pytest.mark.parametrize("prec", PRECS)
def test_stop_set_before_launch(prec):
    cams = [W.scaled(W.C2, 96, 80)]
    params = W.Params(precision=prec)
    r = _reference(cams, params)
    b = G.Batch(cams, params)
    b.camera_init()
    flag = torch.ones(1, dtype=torch.int32, device="cuda")
    b.set_stop_flag(flag.data_ptr())
    b.integrate()
    torch.cuda.synchronize()
    st = b.status[: b.n].cpu().numpy()
    steps = b.steps[: b.n].cpu().numpy()
    print(f"stop before launch {prec}: running {int((st == G.RUNNING).sum())} of {b.n}, "
          f"steps taken {int(steps.sum())}", flush=True)
    # every photon paused after at most one step (in FP32C one that needs an
    # FP64 step first pauses without it)
    assert (st == G.RUNNING).all()
    assert steps.max() <= 1
    assert (steps == 1).sum() >= 0.99 * b.n
    flag.zero_()
    _finish(b, "after stop")
    _same(r, _outputs(b), f"{prec} resumed after a stop before launch")


@pytest.mark.parametrize("prec", PRECS)
def test_stop_in_work_list_mode(prec):
    """Every photon still running goes on to the next list; swapping the lists
    until none is left reproduces the uninterrupted call."""
    cams = [W.scaled(W.C2, 64, 48)]
    params = W.Params(precision=prec)
    r = _reference(cams, params)
    b = G.Batch(cams, params)
    b.camera_init()
    n = b.n
    wl = [torch.full((n + G.GRAY_WORKLIST_SLACK,), -1, dtype=torch.int32, device="cuda") for _ in range(2)]
    wl[0][:n] = torch.arange(n, dtype=torch.int32, device="cuda")
    wc = torch.zeros(2, dtype=torch.int32, device="cuda")
    wc[0] = n
    flag = torch.ones(1, dtype=torch.int32, device="cuda")
    pp = G.params_struct(params)
    pp.flags |= G.GRAY_WORKLIST
    k = 0
    for it in range(50):
        st = G.gray_state(b.state.x, b.state.lo, b.state.status, b.state.steps, b.state.cam,
                          b.state.counters, b.state.mark, None, n, b.stride,
                          wl[k].data_ptr(), wl[1 - k].data_ptr(),
                          wc.data_ptr() + 4 * k, wc.data_ptr() + 4 * (1 - k))
        st.stop = flag.data_ptr()
        G.gray_integrate(b.cam_arr, 1, pp, st, b.ws_ptr, b.ws_bytes, G.current_stream())
        torch.cuda.synchronize()
        left = int(wc[1 - k].item())
        if it == 0:
            out = wl[1 - k][:left].cpu().numpy()
            ids = np.sort(out[out >= 0])
            print(f"stop in list mode {prec}: {left} list entries, {ids.size} ids", flush=True)
            # every photon is still running and listed exactly once
            assert np.array_equal(ids, np.arange(n))
            assert (b.status[:n] == G.RUNNING).all().item()
            flag.zero_()
        if left == 0:
            break
        k = 1 - k
    assert int(wc[1 - k].item()) == 0
    _same(r, _outputs(b), f"{prec} work lists after a stop")


def _mapped_host_word():
    """A 4-byte word of pinned, coherent host memory and its device address,
    allocated with the HIP runtime the library itself uses."""
    lib = G.load()
    alloc, devptr = lib.hipHostMalloc, lib.hipHostGetDevicePointer
    alloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
    devptr.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_uint]
    lib.hipHostFree.argtypes = [ctypes.c_void_p]
    hp, dp = ctypes.c_void_p(), ctypes.c_void_p()
    mapped, coherent = 0x2, 0x40000000
    if alloc(ctypes.byref(hp), 64, mapped | coherent) != 0:
        pytest.skip("hipHostMalloc failed")
    if devptr(ctypes.byref(dp), hp, 0) != 0 or not dp.value:
        lib.hipHostFree(hp)
        pytest.skip("no device address for the host word")
    return lib, hp, dp


@pytest.mark.parametrize("prec", PRECS)
def test_stop_while_running(prec):
    """The host sets the flag about 1 ms into a call of several ms: the call
    ends early with photons paused, and the next call finishes them as if
    nothing had happened."""
    cams = [W.C2]
    params = W.Params(precision=prec)
    r = _reference(cams, params)
    lib, hp, dp = _mapped_host_word()
    try:
        word = ctypes.c_uint32.from_address(hp.value)
        word.value = 0
        b = G.Batch(cams, params)
        b.camera_init()
        b.set_stop_flag(dp.value)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.integrate()
        time.sleep(0.001)
        word.value = 1
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_mask = b.status[: b.n] == G.RUNNING
        running = int(run_mask.sum().item())
        # photons paused after FP64 steps (FP32C: by the block's FP64 wave)
        n64 = b.counters.view(3, b.stride)[2, : b.n]
        paused64 = int((run_mask & (n64 > 0)).sum().item())
        print(f"stop while running {prec}: call ended after {1e3 * (t1 - t0):.2f} ms with {running} of "
              f"{b.n} photons paused ({paused64} after FP64 steps)", flush=True)
        assert running > 0
        if prec == "fp32c":
            # the FP64 waves pause their photons too once their blocks' float
            # waves have exited, instead of running them to their end
            assert paused64 > 0
        word.value = 0
        _finish(b, "after a stop while running")
        _same(r, _outputs(b), f"{prec} resumed after a stop while running")
    finally:
        torch.cuda.synchronize()
        lib.hipHostFree(hp)
