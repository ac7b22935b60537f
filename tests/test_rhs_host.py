"""The integrator's geodesic right-hand side (csrc/kerr.hpp, built for the
host) against the oracle's RHS, which contracts the Christoffel symbols
computed from their definition: random Kerr states across spins, radii from
just outside the horizon to 1000 M, polar angles near the poles and the
equator, and arbitrary (not necessarily null) momenta, since the geodesic
equation holds for any k."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def host_rhs(tmp_path_factory):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rhs") / "rhs_host")
    csrc = os.path.join(ROOT, "paper_1303_5057_amd", "csrc")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-ffp-contract=off", "-I",
                    os.path.join(ROOT, "include"), "-I", csrc, os.path.join(ROOT, "tests", "rhs_host.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def test_rhs_matches_oracle(orc, host_rhs):
    g = np.random.Generator(np.random.PCG64(20261202))
    n = 4000
    a = g.uniform(0.0, 0.999, n)
    rbh = 1.0 + np.sqrt(1.0 - a * a)
    r = rbh * (1.0 + np.exp(g.uniform(np.log(1e-3), np.log(1000.0 / rbh), n)))
    th = np.concatenate([g.uniform(1e-4, 0.05, n // 4), g.uniform(0.05, np.pi - 0.05, n // 2),
                         np.pi - g.uniform(1e-4, 0.05, n - n // 4 - n // 2)])
    k = g.normal(size=(n, 4)) * np.array([1.0, 1.0, 0.3, 0.3])
    lines = "\n".join(" ".join(f"{v:.17g}" for v in row) for row in
                      np.column_stack([a, r, th, k]))
    out = subprocess.run([host_rhs], input=lines, check=True, capture_output=True, text=True).stdout
    got = np.array([[float(v) for v in ln.split()] for ln in out.strip().splitlines()])
    want = np.array([orc.rhs(a[i], np.array([0.0, r[i], th[i], 0.0, *k[i]]))[4:] for i in range(n)])
    # relative to the size of the terms that cancel in each component
    scale = np.abs(want) + 1e-12 * (1.0 + np.abs(k).sum(axis=1, keepdims=True) ** 2)
    err = np.abs(got - want) / scale
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() < 1e-9, (err.max(), worst, got[worst[0]], want[worst[0]])
    assert np.percentile(err, 99) < 1e-12
    assert np.median(err) < 1e-14


def test_null_condition_test_matches_oracle_xi(orc, host_rhs):
    """The integrator's division-free test of eq. (4) (metric components
    scaled by Sigma Delta) against the oracle's xi from its definition: for
    random states, with eps just below and just above the oracle's
    |xi + 1|, the test must report a violation and no violation."""
    g = np.random.Generator(np.random.PCG64(20261203))
    n = 3000
    a = g.uniform(0.0, 0.999, n)
    rbh = 1.0 + np.sqrt(1.0 - a * a)
    r = rbh * (1.0 + np.exp(g.uniform(np.log(1e-3), np.log(1000.0 / rbh), n)))
    th = g.uniform(1e-3, np.pi - 1e-3, n)
    k = g.normal(size=(n, 4)) * np.array([1.0, 1.0, 0.3, 0.3])
    dev = np.array([abs(orc.xi(a[i], np.array([0.0, r[i], th[i], 0.0, *k[i]])) + 1.0) for i in range(n)])
    keep = (dev > 1e-8) & (dev < 1e4)
    assert keep.sum() > n // 2
    rows = []
    for i in np.where(keep)[0]:
        for f in (1.0 - 1e-6, 1.0 + 1e-6):
            rows.append([a[i], r[i], th[i], *k[i], dev[i] * f])
    lines = "\n".join(" ".join(f"{v:.17g}" for v in row) for row in rows)
    out = subprocess.run([host_rhs, "xi"], input=lines, check=True, capture_output=True, text=True).stdout
    got = np.array([int(v) for v in out.split()]).reshape(-1, 2)
    assert np.all(got[:, 0] == 1), np.where(got[:, 0] != 1)
    assert np.all(got[:, 1] == 0), np.where(got[:, 1] != 0)
