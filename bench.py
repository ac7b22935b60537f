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
F_STEP = {"fp64": 538, "fp32c": 538}
# MI355X published vector peaks, TFLOP/s: FP64 78.6 (256 CUs x 4 SIMDs x 16
# lanes x 2 flops x 2.4 GHz), FP32 157.3 (twice that). The FP32C integrator is
# held to the FP32 one: without packed FP32 a SIMD still issues FP32
# instructions whose operands are all vector registers through a second VALU
# path (measured with csrc/valu_peak.hip: non-packed FP32 FMA chains at 2.5
# cycles per wave64 instruction, 126 TFLOP/s; FP64 at 4.1-4.8 cycles).
PEAK_TFLOPS = {"fp64": 78.6, "fp32c": 157.3}
# Rays closer than this to the critical curve (M, on the ray's own constants of
# motion) may legitimately differ in outcome between two correct integrators.
BAND = 1e-3
# Rays whose path comes closer than this (sin theta) to the polar axis carry
# the largest RK4 truncation error of the scheme at Delta = 1/32; drift
# statistics are also reported without them.
AXIS_SIN = 0.02
# FP32C state comparison leaves out rays this close (M) to the critical curve
FP32C_STATE_BAND = 2e-2


def measured_traffic(prec: str):
    """HBM bytes per integrate launch on this workload from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when the kernel sources
    changed since those counters were taken."""
    from paper_1303_5057_amd.srchash import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "k_integrate_kerr512_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()[:2]
        vals[k] = v
    if vals.get("source_hash") != kernel_source_hash() or prec not in vals:
        return None
    return float(vals[prec])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1,
                    help="oracle traces every k-th row and column of the grid")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 256-camera sweep")
    ap.add_argument("--no-c3", action="store_true", help="skip the 4096x4096 recorder workload")
    ap.add_argument("--no-steady", action="store_true", help="skip the far-field steady-state workload")
    ap.add_argument("--no-deformed", action="store_true", help="skip the deformed-metric timing")
    ap.add_argument("--no-ring", action="store_true", help="skip the photon-ring study")
    ap.add_argument("--no-pole", action="store_true", help="skip the pole-treatment ablation")
    ap.add_argument("--no-floor", action="store_true",
                    help="skip tracing the longest photon alone (keeps a profile's integrator launches all 512^2 ones)")
    ap.add_argument("--no-nsweep", action="store_true",
                    help="skip the grid-projection run time versus number of rays")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain device copy of 256 MiB (read 256 MiB, write "
                         "256 MiB), the reference for the HBM traffic counters")
    ap.add_argument("--serve-requests", type=int, default=1100)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-precision", choices=["fp64", "fp32c"], default="fp32c")
    return ap.parse_args()


def sweep(G, W, torch, np) -> dict:
    """The 256-camera sweep (side log-uniform in [64, 1024], spin U[0, 0.998],
    inclination U[1, 89] deg, seeded per camera) in one persistent launch per
    precision: integrate time and ns per photon-step."""
    cams = W.sweep_cameras()
    out = {"cameras": len(cams), "photons": int(sum(c.n for c in cams))}
    t = {}
    for prec in ("fp64", "fp32c"):
        b = G.Batch(cams, W.Params(precision=prec), counters=True, mark=False)
        ms = []
        for rep in range(2):
            b.camera_init()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.integrate()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        steps = int(b.steps[: b.n].to(torch.int64).sum().item())
        t[prec] = min(ms)
        out[prec] = {"integrate_ms": min(ms), "photon_steps": steps,
                     "ns_per_photon_step": min(ms) * 1e6 / steps,
                     "tflops": F_STEP[prec] * steps / (min(ms) * 1e-3) / 1e12}
        del b
        torch.cuda.empty_cache()
    out["fp32c_speedup_vs_fp64"] = t["fp64"] / t["fp32c"]
    return out


def serving(args) -> dict:
    """Continuous batching of camera requests (side log-uniform in [32, 2048],
    spin U[0, 0.998], inclination U[0, 90] deg, Poisson arrivals): saturation
    throughput from a closed loop, then p50/p99 latency at 0.5x and 0.9x of
    the saturation request rate; the first serve-warmup requests are not
    counted."""
    import numpy as np
    from paper_1303_5057_amd import workloads as W
    from paper_1303_5057_amd.serve import Server, latency_stats

    budget = int(args.serve_budget_gb * (1 << 30))
    params = W.Params(precision=args.serve_precision)
    n = args.serve_requests
    def progress(tag):
        last = [time.perf_counter()]

        def cb(r):
            now = time.perf_counter()
            if now - last[0] > 5.0:
                print(f"bench: serving {tag}: request {r.rid} done", file=sys.stderr, flush=True)
                last[0] = now
        return cb

    closed = [W.Request(r.rid, 0.0, r.camera) for r in W.request_stream(n, qps=1.0)]
    srv = Server(budget, params)
    t0 = time.perf_counter()
    res = srv.run(closed, realtime=False, on_done=progress("closed loop"))
    wall = time.perf_counter() - t0
    qps_sat = len(res) / wall
    out = {"precision": args.serve_precision, "budget_gb": args.serve_budget_gb,
           "pool_photons": srv.capacity, "requests": n, "warmup": args.serve_warmup,
           "saturation": {"requests_per_s": qps_sat,
                          "photon_steps_per_s": sum(r.photon_steps for r in res) / wall,
                          "mean_photons_per_request": float(np.mean([r.photons for r in res])),
                          "max_in_flight": srv.max_active}}
    # each size class's floor: a few of its requests served alone, one after
    # the other, on an otherwise empty server
    from paper_1303_5057_amd.serve import SIZE_CLASSES, size_class
    floors = {}
    for name, _, _ in SIZE_CLASSES:
        picks = [r for r in closed if size_class(r.camera.nx * r.camera.ny) == name][:3]
        lat = []
        for r in picks:
            one = srv.run([W.Request(r.rid, 0.0, r.camera)], realtime=False)
            lat.append(one[0].latency_s * 1e3)
        if lat:
            floors[name] = {"requests": len(lat), "alone_ms": lat,
                            "photons": [r.camera.nx * r.camera.ny for r in picks]}
    out["alone_floor_by_size"] = floors
    for frac in (0.5, 0.9):
        reqs = W.request_stream(n, qps=frac * qps_sat)
        srv = Server(budget, params)
        res = srv.run(reqs, realtime=True, on_done=progress(f"{frac}x load"))
        st = latency_stats(res, skip=args.serve_warmup)
        out[f"load_{frac}"] = {"qps": frac * qps_sat, "p50_ms": st["p50_ms"],
                               "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
                               "photon_steps_per_s": st["photon_steps_per_s"],
                               "max_in_flight": srv.max_active, "iterations": srv.iterations,
                               "by_size": st["by_size"]}
    return out


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
    res = oracle.run(p, cam.a, X0, nthreads=threads, want_mark=True)
    dt = time.perf_counter() - t0
    nsteps = int(res.steps.sum())
    cons0 = np.array([oracle.conserved(cam.a, x) for x in X0])
    # one thread on the 64 x 64 Schwarzschild grid (full grid)
    c1 = W.C1
    X1 = oracle.camera_grid(c1.a, c1.r_obs, c1.incl, c1.nx, c1.ny, c1.alpha_lo, c1.alpha_hi,
                            c1.beta_lo, c1.beta_hi)
    t1 = time.perf_counter()
    r1 = oracle.run(p, c1.a, X1, nthreads=1)
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    summary = {"value": dt * 1e9 / nsteps, "unit": "ns/photon/step", "cores": threads,
               "kind": "oracle",
               "sample": f"every {every} row(s) and column(s) of the 512x512 grid "
                         f"({len(ids)} rays, {nsteps} photon-steps, {dt:.2f} s wall)",
               "per_core_ns_per_photon_step": dt * 1e9 / nsteps * threads,
               "single_thread_64x64_schwarzschild_ns_per_photon_step": dt1 * 1e9 / int(r1.steps.sum()),
               "nproc": os.cpu_count(), "cpu_model": model}
    ref = {"ids": ids, "status": res.status, "steps": res.steps, "x": res.x, "euler": res.n_euler,
           "mark": res.mark, "band": band_distance(cam, cons0[:, 0], cons0[:, 1], cons0[:, 2])}
    return summary, ref


def oracle_sample(cam, params, ids):
    """FP64 oracle traces of the listed pixels of `cam` (for C3's error check)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np
    import oracle

    if not os.path.exists(oracle._LIB):
        oracle.build()
    iy, ix = ids // cam.nx, ids % cam.nx
    al = cam.alpha_lo + (cam.alpha_hi - cam.alpha_lo) * ((ix + 0.5) / cam.nx)
    be = cam.beta_lo + (cam.beta_hi - cam.beta_lo) * ((iy + 0.5) / cam.ny)
    X0 = np.array([oracle.camera(cam.a, cam.r_obs, cam.incl, x, y) for x, y in zip(al, be)])
    p = oracle.make_params(step_frac=params.step_frac, horizon_eps=params.horizon_eps,
                           r_escape=params.r_escape, xi_eps=params.xi_eps,
                           euler_div=params.euler_div, max_steps=params.max_steps,
                           record_disk=params.record_disk, disk_rmin=params.disk_rmin,
                           disk_rmax=params.disk_rmax)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    res = oracle.run(p, cam.a, X0, nthreads=threads, want_disk=params.record_disk, want_mark=True)
    cons0 = np.array([oracle.conserved(cam.a, x) for x in X0])
    return {"ids": ids, "status": res.status, "steps": res.steps, "x": res.x, "euler": res.n_euler,
            "mark": res.mark, "band": band_distance(cam, cons0[:, 0], cons0[:, 1], cons0[:, 2]), "disk": res.disk}


def error_vs_oracle(np, g: dict, ref: dict, gathered: bool = False) -> dict:
    """Final states of one GPU run against the FP64 oracle's on the same rays.

    State error per ray: max over components of |x_gpu - x_ora| / (|x_ora| + f)
    with f = 1 for t, r, theta, phi, k^t, k^r and 1/r for k^theta, k^phi,
    over rays whose outcome and step count agree, outside the 1e-3 M band,
    at the horizon stop ("state_err") and, for captured rays, at their mark
    (the last state with r >= 2 r_bh, where the FP32C rule compares them).
    Also the step-count mismatches, the flipped Euler-fallback decisions
    (same step count, different count of fallbacks), the outcome mismatches
    outside the band, and what the FP32C rule leaves out of state comparison
    (within FP32C_STATE_BAND M of the critical curve, or more than 10% Euler
    steps in the oracle)."""
    ids = np.arange(len(ref["ids"])) if gathered else ref["ids"]
    st, sp, x = g["status"][ids], g["steps"][ids], g["x"][ids]
    far = ref["band"] > BAND
    same = (st == ref["status"]) & (sp == ref["steps"])

    def rel(xg, xo):
        r = np.abs(xo[:, 1])
        floor = np.stack([np.ones_like(r)] * 6 + [1.0 / np.maximum(r, 1e-300)] * 2, axis=1)
        return (np.abs(xg - xo) / (np.abs(xo) + floor)).max(axis=1)

    err = rel(x, ref["x"])
    flip = same & (g["euler"][ids] != ref["euler"])
    at_mark = (ref["status"] == 1) & (ref["mark"][:, 1] > 0) if ref.get("mark") is not None else None
    err_m = err.copy()
    if at_mark is not None and g.get("mark") is not None:
        err_m[at_mark] = rel(g["mark"][ids][at_mark], ref["mark"][at_mark])
    sel = same & far & ~flip
    e = err[sel]
    locked = ref["euler"] > 0.1 * ref["steps"]
    excluded = (ref["band"] <= FP32C_STATE_BAND) | locked
    mism = (~same) & far
    comp = sel & ~excluded
    return {"rays": int(len(ids)), "outside_band": int(far.sum()),
            "outcome_mismatch_outside_band": int(((st != ref["status"]) & far).sum()),
            "step_mismatch_fraction_outside_band": float(mism.sum() / max(1, far.sum())),
            "fallback_flips": int((flip & far).sum()),
            "step_mismatch_outside_fp32c_exclusions": int((mism & ~excluded).sum()),
            "state_err": {"p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99)),
                          "max": float(e.max())} if e.size else None,
            "state_err_fp32c_rule": {"p50": float(np.percentile(err_m[comp], 50)),
                                     "p99": float(np.percentile(err_m[comp], 99)),
                                     "max": float(err_m[comp].max()),
                                     "above_1e-3": int((err_m[comp] > 1e-3).sum())} if comp.any() else None,
            "fp32c_rule_excluded_fraction": float(excluded.mean()),
            "fp32c_rule_excluded": {"state_band_M": FP32C_STATE_BAND,
                                    "within_state_band": int((ref["band"] <= FP32C_STATE_BAND).sum()),
                                    "euler_locked": int(locked.sum())}}


def projection_nsweep(G, W, torch, np) -> dict:
    """The paper's first benchmark (Sec. 3): run time of the grid projection
    (a = 0.95, i = 60 deg, recorder on, FP64) against the number of rays n,
    from 8 x 8 to 4096 x 4096: the integrate call and the whole pass
    (camera_init + integrate + classify), medians of HIP-event timings."""
    rows = []
    for side in (8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096):
        cam = W.projection_camera(0.95, 60.0, side)
        b = G.Batch([cam], W.PROJECTION_PARAMS, counters=False, mark=False)
        reps = 7 if side <= 1024 else 3
        t_int, t_pass = [], []
        for rep in range(reps + 1):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            b.camera_init()
            ev[1].record()
            b.integrate()
            ev[2].record()
            b.classify(xf=False, cons=False, counts=True)
            ev[3].record()
            torch.cuda.synchronize()
            if rep:
                t_int.append(ev[1].elapsed_time(ev[2]))
                t_pass.append(ev[0].elapsed_time(ev[3]))
        steps = int(b.steps[: b.n].to(torch.int64).sum().item())
        hit = float((b.disk.view(3, b.stride)[0, : b.n] > 0).float().mean().item())
        ti, tp = float(np.median(t_int)), float(np.median(t_pass))
        rows.append({"side": side, "n": b.n, "integrate_ms": ti, "pass_ms": tp, "photon_steps": steps,
                     "ns_per_photon_step": ti * 1e6 / steps, "crossed_fraction": hit})
        del b
    return {"workload": "grid projection a=0.95 i=60deg, window +-12 M, FP64", "rows": rows}


def pole_ablation(G, W, torch, np) -> dict:
    """The paper's pole case (a = 0.99, r0 sin(theta0) = 4.833605 M) rotated
    to phi0 = 0..359 deg under the three treatments of the polar axis
    (Sec. 2, Fig. 2), FP64: outcome, step counts and the drift of E, L_z, Q
    at the last state with r >= 2 r_bh."""
    import math
    cams = [W.pole_camera(math.radians(d)) for d in range(360)]
    out = {}
    for name, mode in (("production_monitor", G.GRAY_POLE_MONITOR),
                       ("euler_on_crossing", G.GRAY_POLE_EULER_CROSSING),
                       ("none", G.GRAY_POLE_NONE)):
        b = G.Batch(cams, W.Params(pole_mode=mode))
        res = b.run()
        torch.cuda.synchronize()
        n = b.n
        status = b.status[:n].cpu().numpy()
        steps = b.steps[:n].cpu().numpy()
        ctr = b.counters.view(3, b.stride)[:, :n].cpu().numpy()
        drift = res.cons.view(9, b.stride)[6:9, :n].cpu().numpy()
        out[name] = {"status_counts": np.bincount(status, minlength=5).tolist(),
                     "steps_median": float(np.median(steps)), "steps_max": int(steps.max()),
                     "euler_steps_median": float(np.median(ctr[0])),
                     "remaps_median": float(np.median(ctr[1])),
                     "drift_ELQ_median": np.median(drift, axis=1).tolist(),
                     "drift_ELQ_max": drift.max(axis=1).tolist()}
        del b, res
    return out


def ring_study(np) -> dict:
    """The photon-ring parameter study (16 spins x 19 inclinations, 6000 x 181
    polar rays each, 3.3e8 rays) in one persistent launch: integrate time,
    ns per photon-step, and the ring measures against the paper's fits."""
    from paper_1303_5057_amd import ring as GR
    rings, timing = GR.study()
    dR = np.array([r.measures["R_mean"] - GR.paper_fit_mean_radius(r.a, r.incl_deg) for r in rings])
    dA = np.array([r.measures["A"] - GR.paper_fit_asymmetry(r.a, r.incl_deg) for r in rings])
    edge_on = [r for r in rings if r.incl_deg == 90]
    timing.update({
        "configs": len(rings),
        "tflops": F_STEP["fp64"] * timing["photon_steps"] / (timing["integrate_ms"] * 1e-3) / 1e12,
        "unfinished_rays": int(sum(r.unfinished for r in rings)),
        "mean_radius_minus_fit": {"max_abs": float(np.abs(dR).max()), "rms": float(np.sqrt((dR ** 2).mean()))},
        "asymmetry_minus_fit": {"max_abs": float(np.abs(dA).max()), "rms": float(np.sqrt((dA ** 2).mean()))},
        "edge_on": [{"a": r.a, "D": r.measures["D"], "R_mean": r.measures["R_mean"], "A": r.measures["A"]}
                    for r in edge_on],
    })
    return timing


def measure(G, W, torch, np, cam, prec: str, steps: int, warmup: int, floor: bool = True) -> dict:
    """Time `steps` passes (camera_init + integrate + classify) after `warmup`."""
    params = W.Params(precision=prec)
    b = G.Batch([cam], params)

    def one_pass(ev0=None, ev1=None):
        b.camera_init()
        b.wave_iters.zero_()
        if ev0 is not None:
            ev0.record()
        b.integrate()
        if ev1 is not None:
            ev1.record()
        return b.classify(xf=True, cons=True, counts=True)

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
    lane_eff = total_steps / (64.0 * max(1, int(b.wave_iters.item())))
    counters = b.counters.view(3, b.stride)[:, : b.n].to(torch.int64).sum(dim=1).tolist()
    status = b.status[: b.n].cpu().numpy()
    cons = res.cons.view(9, b.stride)[:, : b.n].cpu().numpy()
    euler = b.counters.view(3, b.stride)[0, : b.n].cpu().numpy()
    band = band_distance(cam, cons[0], cons[1], cons[2])
    drift = drift_groups(G, np, status, cons, euler, band, polar_turning(cam, cons[0], cons[1], cons[2]))
    # the pass's own results, copied before the floor measurement re-initialises the batch
    host = {"status": status, "steps": b.steps[: b.n].cpu().numpy(),
            "x": res.xf.view(8, b.stride)[:, : b.n].cpu().numpy().T if res.xf is not None else None,
            "mark": b.mark.view(8, b.stride)[:, : b.n].cpu().numpy().T if b.mark is not None else None,
            "euler": euler, "band": band}
    tail = longest_alone(G, W, torch, np, b, params) if floor else None
    return {"params": params, "ms_per_step": ms_per_step, "integrate_ms": int_ms,
            "total_steps": total_steps, "status": np.bincount(status, minlength=5).tolist(),
            "euler_steps": counters[0], "fp64_steps": counters[2], "drift": drift, "n": b.n,
            "lane_efficiency": lane_eff, "tail": tail, "host": host}


def band_distance(cam, E0, L0, Q0):
    """Distance (M) of each ray's asymptotic image-plane point, from its own
    constants of motion at the camera, to the Kerr critical curve; inf
    beyond 0.1 M (every use compares it with 1e-3 or 1e-2 M, and the bounded
    search keeps 16.8M rays to seconds)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import analytic
    return analytic.CriticalBand(cam.a, cam.incl).distance(E0, L0, Q0, upper=0.1)


def drift_groups(G, np, status, cons, euler, band, smin=None) -> dict:
    """Drift of E, L_z and Q (rows 6..8 of gray_classify's cons) per group of
    rays: outcome (escaped, captured) x position (outside or inside the 1e-3 M
    band around the critical curve) x Euler fallbacks (none, some). For each
    group: ray count, p50 / p99 / max of each drift, and how many rays exceed
    1e-5 in each quantity; with `smin` (sin theta at each ray's polar turning
    point) also the same counts and maxima over the rays that stay off the
    polar axis (smin >= 0.02)."""
    out = {}
    for oname, osel in (("escaped", status == G.ESCAPED), ("captured", status == G.CAPTURED)):
        for bname, bsel in (("outside_band", band > BAND), ("in_band", band <= BAND)):
            for ename, esel in (("no_euler", euler == 0), ("euler", euler > 0)):
                sel = osel & bsel & esel
                d = cons[6:9, sel]
                g = {"rays": int(sel.sum())}
                if d.size:
                    g.update({q: np.percentile(d, pq, axis=1).tolist()
                              for q, pq in (("p50", 50), ("p99", 99), ("max", 100))})
                    g["above_1e-5"] = (d > 1e-5).sum(axis=1).tolist()
                if smin is not None:
                    off = sel & (smin >= AXIS_SIN)
                    do = cons[6:9, off]
                    g["off_axis_rays"] = int(off.sum())
                    if do.size:
                        g["off_axis_max"] = do.max(axis=1).tolist()
                        g["off_axis_above_1e-5"] = (do > 1e-5).sum(axis=1).tolist()
                out[f"{oname}/{bname}/{ename}"] = g
    return out


def polar_turning(cam, E0, L0, Q0):
    """sin theta at each ray's polar turning point (closest approach to the
    spin axis) from its constants of motion at the camera."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import analytic
    return analytic.polar_turning_sin(cam.a, E0, L0, Q0)


def longest_alone(G, W, torch, np, b, params, reps: int = 3) -> dict:
    """The launch's floor: its longest photon traced alone (a one-photon work
    list, so one wave on an otherwise idle GPU). A launch cannot end before
    that photon does, and the photon cannot run faster than alone."""
    steps = b.steps[: b.n].cpu().numpy()
    pid = int(np.argmax(steps))
    wl = [torch.zeros(G.GRAY_WORKLIST_SLACK + 64, dtype=torch.int32, device="cuda") for _ in range(2)]
    wc = torch.zeros(2, dtype=torch.int32, device="cuda")
    pp = G.params_struct(params)
    pp.flags |= G.GRAY_WORKLIST
    # the launch's own counters and mark buffers, so the photon runs the same recorders
    st = G.gray_state(b.state.x, b.state.lo, b.state.status, b.state.steps, b.state.cam, b.state.counters,
                      b.state.mark, None, b.n, b.stride, wl[0].data_ptr(), wl[1].data_ptr(), wc.data_ptr(),
                      wc.data_ptr() + 4)
    ts = []
    for _ in range(reps):
        b.camera_init()
        wl[0][0] = pid
        wc.zero_()
        wc[0] = 1
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        G.gray_integrate(b.cam_arr, 1, pp, st, b.ws_ptr, b.ws_bytes, G.current_stream())
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    alone_steps = int(b.steps[pid].item())
    return {"photon": pid, "steps": int(steps[pid]), "alone_steps": alone_steps, "alone_ms": min(ts),
            "alone_us_per_step": min(ts) * 1e3 / max(1, alone_steps)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
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
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    cam = W.C2
    print("bench: timing the 512x512 workload", file=sys.stderr, flush=True)
    head = measure(G, W, torch, np, cam, args.precision, args.steps, args.warmup, not args.no_floor)
    other_prec = "fp32c" if args.precision == "fp64" else "fp64"
    other = measure(G, W, torch, np, cam, other_prec, args.steps, args.warmup, not args.no_floor)
    t64 = head["integrate_ms"] if args.precision == "fp64" else other["integrate_ms"]
    t32 = other["integrate_ms"] if args.precision == "fp64" else head["integrate_ms"]

    total_steps = head["total_steps"]
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
        "lane_efficiency": head["lane_efficiency"],
        # the launch's floor: its longest photon alone on the GPU
        "longest_photon": floor_block(head),
        "drift_ELQ": head["drift"],
        "roofline": roofline(args.precision, head, measured_traffic(args.precision)),
        other_prec: {"ns_per_photon_step": other["ms_per_step"] * 1e6 / other["total_steps"],
                     "integrate_ms": other["integrate_ms"],
                     "photon_steps_per_pass": other["total_steps"],
                     "fp64_step_fraction": other["fp64_steps"] / other["total_steps"],
                     "lane_efficiency": other["lane_efficiency"],
                     "status_counts": other["status"], "drift_ELQ": other["drift"],
                     "longest_photon": floor_block(other),
                     "roofline": roofline(other_prec, other, measured_traffic(other_prec))},
        "fp32c_speedup_vs_fp64": t64 / t32,
    }
    if args.precision == "fp32c":
        out["fp64_step_fraction"] = head["fp64_steps"] / total_steps
    if not args.no_steady:
        print("bench: far-field steady state", file=sys.stderr, flush=True)
        out["steady"] = steady_block(G, W, torch, np)
    if not args.no_c3:
        print("bench: 4096x4096 recorder workload", file=sys.stderr, flush=True)
        out["c3"] = c3_block(G, W, torch, np, with_oracle=not args.no_cpu_baseline)
    if not args.no_deformed:
        print("bench: deformed metric", file=sys.stderr, flush=True)
        out["deformed"] = deformed_block(G, W, torch, np)
    if not args.no_sweep:
        print("bench: 256-camera sweep", file=sys.stderr, flush=True)
        out["sweep"] = sweep(G, W, torch, np)
    if not args.no_nsweep:
        print("bench: grid-projection n-sweep", file=sys.stderr, flush=True)
        out["projection_nsweep"] = projection_nsweep(G, W, torch, np)
    if not args.no_pole:
        print("bench: pole-treatment ablation", file=sys.stderr, flush=True)
        out["pole_ablation"] = pole_ablation(G, W, torch, np)
    if not args.no_ring:
        print("bench: photon-ring study", file=sys.stderr, flush=True)
        out["ring_study"] = ring_study(np)
    if not args.no_serve:
        print("bench: serving", file=sys.stderr, flush=True)
        out["serving"] = serving(args)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"], ref = cpu_baseline(cam, head["params"], args.cpu_sample)
        # the same oracle traces, against both precisions' final states
        out["error_vs_oracle"] = {args.precision: error_vs_oracle(np, head["host"], ref),
                                  other_prec: error_vs_oracle(np, other["host"], ref)}
    print(json.dumps(out), flush=True)
    return 0


def roofline(prec: str, m: dict, traffic) -> dict:
    """The integrate kernel against the VALU peak: algorithmic flops per
    accepted photon-step times the launch's photon-steps over its HIP-event
    time."""
    achieved = F_STEP[prec] * m["total_steps"] / (m["integrate_ms"] * 1e-3) / 1e12
    kernel = "k_integrate<kPoleMonitor>" if prec == "fp64" else "k_integrate_c32"
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[prec], "traffic": traffic, "traffic_unit": "bytes per launch",
            "kernel": kernel, "flops_per_photon_step": F_STEP[prec]}


def floor_block(m: dict):
    if not m["tail"]:
        return None
    return dict(m["tail"], launch_ms=m["integrate_ms"], floor_fraction=m["tail"]["alone_ms"] / m["integrate_ms"])


def deformed_block(G, W, torch, np, reps: int = 3) -> dict:
    """The metric-generic path: a = 0.6, i = 50 deg, 512 x 512 over +-8 M in
    the deformed Kerr metric (deform = 1.5), and the same camera through the
    generic path at deform = 0 and through the Kerr fast path, FP64:
    integrate time, ns per photon-step, and drift of E and L_z (constants of
    motion of the deformed metric) and of the Kerr-form Q (not one)."""
    out = {"workload": "deformed_kerr_a0.6_i50_512x512_r1000"}
    for name, metric, deform in (("deformed_1.5", G.GRAY_METRIC_DEFORMED, 1.5),
                                 ("generic_0", G.GRAY_METRIC_DEFORMED, 0.0),
                                 ("kerr_fast_path", G.GRAY_METRIC_KERR, 0.0)):
        cam = W.Camera(0.6, 1000.0, W.deg(50.0), 512, 512, -8.0, 8.0, -8.0, 8.0, metric=metric, deform=deform)
        b = G.Batch([cam], W.Params(), counters=True, mark=True)
        ms = []
        for rep in range(reps):
            b.camera_init()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.integrate()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        res = b.classify(xf=False, cons=True, counts=True)
        torch.cuda.synchronize()
        n = b.n
        steps = int(b.steps[:n].to(torch.int64).sum().item())
        status = b.status[:n].cpu().numpy()
        cons = res.cons.view(9, b.stride)[:, :n].cpu().numpy()
        euler = b.counters.view(3, b.stride)[0, :n].cpu().numpy()
        clean = (status == G.ESCAPED) & (euler == 0)
        out[name] = {"integrate_ms": min(ms), "photon_steps": steps, "ns_per_photon_step": min(ms) * 1e6 / steps,
                     "status_counts": np.bincount(status, minlength=5).tolist(),
                     "escaped_no_euler_drift_max_E_L_Q": cons[6:9, clean].max(axis=1).tolist() if clean.any() else None}
        del b, res
        torch.cuda.empty_cache()
    out["generic_over_fast_path_time"] = out["generic_0"]["integrate_ms"] / out["kerr_fast_path"]["integrate_ms"]
    return out


def steady_block(G, W, torch, np, reps: int = 5) -> dict:
    """Throughput without a tail: a 2048 x 2048 grid aimed 200-300 M off the
    hole (a = 0.9, i = 60 deg), every ray advanced exactly 100 far-field steps
    (call_steps = 100), in both precisions: integrate time (best of `reps`,
    HIP events), ns per photon-step and the VALU roofline."""
    cam = W.Camera(0.9, 1000.0, W.deg(60.0), 2048, 2048, 200.0, 300.0, 200.0, 300.0)
    out = {"workload": "far_field_a0.9_i60_2048x2048_100_steps", "photons": cam.n}
    for prec in ("fp64", "fp32c"):
        b = G.Batch([cam], W.Params(precision=prec, call_steps=100), mark=False)
        ms = []
        for _ in range(reps):
            b.camera_init()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.integrate()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        steps = int(b.steps[: b.n].to(torch.int64).sum().item())
        m = {"integrate_ms": min(ms), "total_steps": steps}
        out[prec] = {"integrate_ms": min(ms), "photon_steps": steps, "ns_per_photon_step": min(ms) * 1e6 / steps,
                     "roofline": roofline(prec, m, None)}
        del b
        torch.cuda.empty_cache()
    out["fp32c_speedup_vs_fp64"] = out["fp64"]["integrate_ms"] / out["fp32c"]["integrate_ms"]
    return out


def c3_block(G, W, torch, np, with_oracle: bool, reps: int = 3) -> dict:
    """The 4096 x 4096 face-on-ish workload (a = 0.9375, i = 17 deg, window
    +-12 M, equatorial-crossing recorder over [r_ISCO, 50 M]) in FP32C (the
    precision it is specified in) and FP64: integrate time (best of `reps`,
    HIP events), ns per photon-step, the FP64-step fraction, drift groups, the
    fraction of rays that hit the recorder window, the roofline, and the
    error against the FP64 oracle on every 64th row and column."""
    cam = W.C3
    out = {"workload": "kerr_a0.9375_i17_4096x4096_r1000_disk", "photons": cam.n}
    ids = W.subsample_ids(cam, 64)
    ref = oracle_sample(cam, W.C3_PARAMS, ids) if with_oracle else None
    t = {}
    for prec in ("fp32c", "fp64"):
        params = W.Params(record_disk=True, disk_rmin=-1.0, disk_rmax=50.0, precision=prec)
        b = G.Batch([cam], params, counters=True, mark=True)
        ms = []
        for rep in range(reps):
            b.camera_init()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.integrate()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        res = b.classify(xf=True, cons=True, counts=True)
        torch.cuda.synchronize()
        n = b.n
        steps = int(b.steps[:n].to(torch.int64).sum().item())
        ctr = b.counters.view(3, b.stride)[:, :n].to(torch.int64).sum(dim=1).tolist()
        status = b.status[:n].cpu().numpy()
        cons = res.cons.view(9, b.stride)[:, :n].cpu().numpy()
        euler = b.counters.view(3, b.stride)[0, :n].cpu().numpy()
        band = band_distance(cam, cons[0], cons[1], cons[2])
        disk_r = b.disk.view(3, b.stride)[0, :n]
        m = {"integrate_ms": min(ms), "total_steps": steps}
        blk = {"integrate_ms": min(ms), "integrate_ms_all": ms, "photon_steps": steps,
               "ns_per_photon_step": min(ms) * 1e6 / steps, "photon_steps_per_s": steps / (min(ms) * 1e-3),
               "fp64_step_fraction": ctr[2] / steps, "euler_steps": ctr[0],
               "status_counts": np.bincount(status, minlength=5).tolist(),
               "disk_hit_fraction": float((disk_r > 0).float().mean().item()),
               "drift_ELQ": drift_groups(G, np, status, cons, euler, band,
                                         polar_turning(cam, cons[0], cons[1], cons[2])),
               "roofline": roofline(prec, m, None)}
        if ref is not None:
            # the sampled rays only, gathered on the device
            idx = torch.as_tensor(ids, dtype=torch.int64, device=b.x.device)
            g = {"status": b.status[idx].cpu().numpy(), "steps": b.steps[idx].cpu().numpy(),
                 "x": res.xf.view(8, b.stride)[:, idx].cpu().numpy().T,
                 "euler": b.counters.view(3, b.stride)[0, idx].cpu().numpy(),
                 "mark": b.mark.view(8, b.stride)[:, idx].cpu().numpy().T}
            blk["error_vs_oracle"] = error_vs_oracle(np, g, ref, gathered=True)
            dg = b.disk.view(3, b.stride)[:, idx].cpu().numpy().T
            agree = (g["status"] == ref["status"]) & (g["steps"] == ref["steps"])
            same = agree & (ref["disk"][:, 0] > 0) & (ref["band"] > 1e-2)
            de = np.abs(dg[same] - ref["disk"][same]) / (np.abs(ref["disk"][same]) + 1.0)
            blk["error_vs_oracle"]["disk_err_max"] = float(de.max()) if de.size else None
            blk["error_vs_oracle"]["disk_hit_mismatch"] = int(
                ((dg[:, 0] > 0) != (ref["disk"][:, 0] > 0))[agree].sum())
        out[prec] = blk
        t[prec] = min(ms)
        del b, res
        torch.cuda.empty_cache()
    out["fp32c_speedup_vs_fp64"] = t["fp64"] / t["fp32c"]
    return out


if __name__ == "__main__":
    sys.exit(main())
