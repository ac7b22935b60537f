#!/usr/bin/env python3
"""Benchmark of the Kerr photon-geodesic integrator on one MI355X.

One "step" is one pass of the whole hot path over the edge-on Kerr workload
(a = 0.99, i = 90 deg, 512 x 512 image-plane grid over [-8, 8]^2 M,
r_obs = 1000 M): gray_camera_init, gray_integrate, gray_classify, with the
inputs (camera descriptors) on the host and every photon's state resident in
HBM. The headline metric is ns per photon per step: wall time of a pass
divided by the accepted photon-steps it takes.

Prints one JSON line. Also reports the integrate kernel against the VALU
roofline (algorithmic flops per photon-step, counted by
paper_1303_5057_amd/csrc/flopcount.cpp, times accepted steps, over the
kernel time from HIP events on the launch stream), and the FP64 CPU oracle
timed on a bounded sample of the same rays on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic flops per accepted photon-step of the integrate kernel (common
# path: RK4 + step size + null-condition check), weights add/mul 1, fma 2,
# div/sqrt/sin/cos 1; produced by csrc/flopcount.cpp and checked by the tests.
F_STEP = {"fp64": 644, "fp32c": 644}
# MI355X published vector peaks, TFLOP/s (256 CUs at 2.4 GHz).
PEAK_TFLOPS = {"fp64": 78.6, "fp32c": 157.3}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1,
                    help="oracle traces every k-th row and column of the grid")
    return ap.parse_args()


def cpu_baseline(cam, params, every: int):
    """FP64 CPU oracle on a strided sample of the same rays, all host threads."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np
    import oracle
    from paper_1303_5057_amd import workloads as W

    if not os.path.exists(oracle._LIB):
        oracle.build()
    ids = W.subsample_ids(cam, every)
    iy, ix = ids // cam.nx, ids % cam.nx
    al = cam.alpha_lo + (cam.alpha_hi - cam.alpha_lo) * ((ix + 0.5) / cam.nx)
    be = cam.beta_lo + (cam.beta_hi - cam.beta_lo) * ((iy + 0.5) / cam.ny)
    X0 = np.array([oracle.camera(cam.a, cam.r_obs, cam.incl, x, y) for x, y in zip(al, be)])
    p = oracle.make_params(step_frac=params.step_frac, horizon_eps=params.horizon_eps,
                           r_escape=params.r_escape, xi_eps=params.xi_eps,
                           euler_div=params.euler_div, max_steps=params.max_steps)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    res = oracle.run(p, cam.a, X0, nthreads=threads)
    dt = time.perf_counter() - t0
    nsteps = int(res.steps.sum())
    return {"value": dt * 1e9 / nsteps, "unit": "ns/photon/step", "cores": threads,
            "kind": "oracle",
            "sample": f"every {every} row(s) and column(s) of the 512x512 grid "
                      f"({len(ids)} rays, {nsteps} photon-steps, {dt:.2f} s wall)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(photons are independent; a multi-GPU run would shard the ray ids).", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_1303_5057_amd import gray as G
    from paper_1303_5057_amd import workloads as W

    G.load()   # raises if libgray.so is not built: there is no fallback
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 3
    cam = W.C2
    params = W.Params(precision=args.precision)
    b = G.Batch([cam], params)

    def one_pass(ev0=None, ev1=None):
        b.camera_init()
        if ev0 is not None:
            ev0.record()
        b.integrate()
        if ev1 is not None:
            ev1.record()
        return b.classify(xf=False, cons=True, counts=True)

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        res = one_pass(e0, e1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    int_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    steps = b.steps[: b.n].to(torch.int64)
    total_steps = int(steps.sum().item())
    status = b.status[: b.n].cpu().numpy()
    cons = res.cons.view(9, b.stride)[:, : b.n].cpu().numpy()
    drift = {}
    for name, sel in (("escaped", status == G.ESCAPED), ("captured", status == G.CAPTURED)):
        d = cons[6:9, sel]
        drift[name] = {q: np.percentile(d, pq, axis=1).tolist()
                       for q, pq in (("p50", 50), ("p99", 99), ("max", 100))} if d.size else {}
    achieved = F_STEP[args.precision] * total_steps / (int_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]

    out = {
        "metric": "ns/photon/step",
        "value": ms_per_step * 1e6 / total_steps,
        "unit": "ns/photon/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f32c",
        "data": "synthetic",
        "config": {"workload": "kerr_a0.99_i90_512x512_r1000", "photons": b.n,
                   "grid": [cam.nx, cam.ny], "spin": cam.a, "incl_deg": 90.0,
                   "precision": args.precision, "step_frac": params.step_frac},
        "photon_steps_per_pass": total_steps,
        "photon_steps_per_s": total_steps / (ms_per_step * 1e-3),
        "integrate_ms": int_ms,
        "integrate_ns_per_photon_step": int_ms * 1e6 / total_steps,
        "status_counts": np.bincount(status, minlength=5).tolist(),
        "drift_ELQ": drift,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_integrate_fp64", "flops_per_photon_step": F_STEP[args.precision]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cam, params, args.cpu_sample)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
