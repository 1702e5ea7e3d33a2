"""The C ABI used from plain C: ``tests/c_client/fpt_c_client`` (built by
``__graft_entry__.build()`` with gcc against ``include/fpt.h`` and the HIP
runtime's C API, no Python or torch in the process) runs plans, the
allocation-free entry point and a server, and its results equal the Python
binding's for the same parameters: escape steps, histograms and integer
moments bit-exact, FP64 steps against the oracle at the usual bar."""

import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1802_05065_amd import api, workloads

pytestmark = pytest.mark.gpu

BINARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "fpt_c_client")
INT_MOMENTS = ("n_escaped", "n_censored", "n_overflow", "sum_k")


def _param_args(p):
    return [str(int(p["model"])), repr(float(p["alpha"])), repr(float(p["T"])),
            repr(float(p["V0"])), repr(float(p["gamma0"])), repr(float(p["ramp"])),
            repr(float(p["dt"])), repr(float(p["phi0"])), repr(float(p["v0"])),
            repr(float(p["threshold"])), str(int(p["max_steps"])), str(int(p["n_replicas"])),
            str(int(p["n_bins"])), str(int(p["hist_k_max"])), str(int(p["seed"]))]


def _run(mode, prec, third, p):
    if not os.path.exists(BINARY):
        pytest.fail(f"{BINARY} is missing: run __graft_entry__.build() first")
    cmd = [BINARY, mode, prec, str(third), *_param_args(p)]
    print("c client:", mode, prec, p["n_replicas"], "replicas, seed", p["seed"], flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=150)
    assert res.returncode == 0, res.stderr
    lines = {}
    for line in res.stdout.splitlines():
        head, _, rest = line.partition(" ")
        if head in ("job", "job_counts"):
            idx, _, rest = rest.partition(" ")
            head = f"{head} {idx}"
        lines[head] = rest.split()
    return lines


def _moments(fields):
    n_esc, n_cens, n_over, sum_k, lo, hi = (int(x) for x in fields[:6])
    return {"n_escaped": n_esc, "n_censored": n_cens, "n_overflow": n_over, "sum_k": sum_k,
            "sum_k2": (hi << 64) | lo, "mean_t": float(fields[6])}


def _check_equal(lines, res, n_bins, tag="", counts_key="counts"):
    counts = [int(x) for x in lines[counts_key]]
    assert len(counts) == n_bins
    assert counts == res.counts[0].tolist(), tag
    mom = _moments(lines["moments" if not tag else f"job {tag}"])
    for k in INT_MOMENTS:
        assert mom[k] == res.moments[0][k], (tag, k)
    assert mom["sum_k2"] == res.moments[0]["sum_k2"], tag
    if math.isfinite(res.moments[0]["mean_t"]):
        assert mom["mean_t"] == res.moments[0]["mean_t"], tag


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_c_client_plan_equals_binding(prec, tmp_path):
    p = workloads.plain_escape(n_replicas=4096, seed=11)
    path = tmp_path / "steps.bin"
    lines = _run("plan", prec, path, p)
    steps = np.fromfile(path, dtype=np.int64)
    assert steps.size == p["n_replicas"]
    res = api.simulate(p, prec)
    assert np.array_equal(steps, res.steps[0].cpu().numpy())
    _check_equal(lines, res, p["n_bins"])
    assert lines["device_counts"] == lines["counts"]
    assert int(lines["stats"][0]) == res.stats["replica_steps"]
    if prec == "fp64":
        ref = oracle.escape_steps(oracle.OracleParams(**workloads.to_oracle_kwargs(p)), 0, 1024)
        same = float(np.mean(steps[:1024] == ref))
        print(f"C client FP64 vs oracle: identical escape steps {same:.4f} (first 1024)")
        assert same >= 0.99


def test_c_client_noalloc_equals_binding(tmp_path):
    # the allocation-free entry point from C (the client allocates only its
    # outputs), against the binding's workspace run of the same tuning
    p = workloads.plain_escape(n_replicas=3000, seed=12)
    path = tmp_path / "steps.bin"
    lines = _run("noalloc", "fp32c", path, p)
    steps = np.fromfile(path, dtype=np.int64)
    res = api.simulate(p, "fp32c", dict(replicas_per_lane=1, waves_per_simd=2,
                                        steps_per_launch=4096))
    assert np.array_equal(steps, res.steps[0].cpu().numpy())
    _check_equal(lines, res, p["n_bins"])
    assert lines["device_counts"] == lines["counts"]


def test_c_client_server_jobs_equal_plans():
    # three jobs submitted at once to a server created from C: each job's
    # histogram and moments equal its own plan's
    p = workloads.plain_escape(n_replicas=2048, seed=21)
    n_jobs = 3
    lines = _run("serve", "fp32c", n_jobs, p)
    for i in range(n_jobs):
        alone = api.simulate(dict(p, seed=p["seed"] + i), "fp32c", record_steps=False)
        _check_equal(lines, alone, p["n_bins"], tag=str(i), counts_key=f"job_counts {i}")
