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


def measure(G, W, torch, np, cam, prec: str, steps: int, warmup: int) -> dict:
    """Time `steps` passes (camera_init + integrate + classify) after `warmup`."""
    params = W.Params(precision=prec)
    b = G.Batch([cam], params)

    def one_pass(ev0=None, ev1=None):
        b.camera_init()
        if ev0 is not None:
            ev0.record()
        b.integrate()
        if ev1 is not None:
            ev1.record()
        return b.classify(xf=False, cons=True, counts=True)

    for _ in range(warmup):
        one_pass()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        res = one_pass(e0, e1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    ms_per_step = (t1 - t0) * 1e3 / steps
    int_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    total_steps = int(b.steps[: b.n].to(torch.int64).sum().item())
    counters = b.counters.view(3, b.stride)[:, : b.n].to(torch.int64).sum(dim=1).tolist()
    status = b.status[: b.n].cpu().numpy()
    cons = res.cons.view(9, b.stride)[:, : b.n].cpu().numpy()
    euler = b.counters.view(3, b.stride)[0, : b.n].cpu().numpy()
    drift = {}
    for name, sel in (("escaped", status == G.ESCAPED), ("captured", status == G.CAPTURED),
                      ("no_fallback", euler == 0)):
        d = cons[6:9, sel]
        drift[name] = {q: np.percentile(d, pq, axis=1).tolist()
                       for q, pq in (("p50", 50), ("p99", 99), ("max", 100))} if d.size else {}
    return {"params": params, "ms_per_step": ms_per_step, "integrate_ms": int_ms,
            "total_steps": total_steps, "status": np.bincount(status, minlength=5).tolist(),
            "euler_steps": counters[0], "fp64_steps": counters[2], "drift": drift, "n": b.n}


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
    head = measure(G, W, torch, np, cam, args.precision, args.steps, args.warmup)
    other_prec = "fp32c" if args.precision == "fp64" else "fp64"
    other = measure(G, W, torch, np, cam, other_prec, args.steps, args.warmup)
    t64 = head["integrate_ms"] if args.precision == "fp64" else other["integrate_ms"]
    t32 = other["integrate_ms"] if args.precision == "fp64" else head["integrate_ms"]

    total_steps = head["total_steps"]
    achieved = F_STEP[args.precision] * total_steps / (head["integrate_ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    kernel = "k_integrate<GRAY_FP64>" if args.precision == "fp64" else "k_integrate<GRAY_FP32C>"
    out = {
        "metric": "ns/photon/step",
        "value": head["ms_per_step"] * 1e6 / total_steps,
        "unit": "ns/photon/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f32c",
        "data": "synthetic",
        "config": {"workload": "kerr_a0.99_i90_512x512_r1000", "photons": head["n"],
                   "grid": [cam.nx, cam.ny], "spin": cam.a, "incl_deg": 90.0,
                   "precision": args.precision, "step_frac": head["params"].step_frac},
        "photon_steps_per_pass": total_steps,
        "photon_steps_per_s": total_steps / (head["ms_per_step"] * 1e-3),
        "integrate_ms": head["integrate_ms"],
        "integrate_ns_per_photon_step": head["integrate_ms"] * 1e6 / total_steps,
        "status_counts": head["status"],
        "euler_fallback_steps": head["euler_steps"],
        "drift_ELQ": head["drift"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": kernel,
                     "flops_per_photon_step": F_STEP[args.precision]},
        other_prec: {"ns_per_photon_step": other["ms_per_step"] * 1e6 / other["total_steps"],
                     "integrate_ms": other["integrate_ms"],
                     "photon_steps_per_pass": other["total_steps"],
                     "fp64_step_fraction": other["fp64_steps"] / other["total_steps"],
                     "status_counts": other["status"], "drift_ELQ": other["drift"]},
        "fp32c_speedup_vs_fp64": t64 / t32,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cam, head["params"], args.cpu_sample)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
