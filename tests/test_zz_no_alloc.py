"""fpt_simulate_noalloc, the entry point for callers that cannot allocate
(workspace in the library's static device array), against fpt_simulate with
a caller-owned workspace: the same escape steps, histograms and integer
moments, bit for bit, on two calls in a row (the second one smaller), in
both precisions; plans it cannot run are refused before any launch."""

import numpy as np
import pytest

from paper_1802_05065_amd import _lib, workloads

pytestmark = pytest.mark.gpu

TUNE = dict(replicas_per_lane=1, waves_per_simd=4, steps_per_launch=2048)
INT_MOMENTS = ("n_escaped", "n_censored", "n_overflow", "sum_k", "sum_k2")


def _torch():
    import torch

    assert torch.cuda.is_available()
    return torch


def _outputs(torch, sets):
    steps = [torch.full((int(s["n_replicas"]),), -7, dtype=torch.int64, device="cuda")
             for s in sets]
    hist = torch.full((sum(int(s["n_bins"]) for s in sets),), -7, dtype=torch.int64,
                      device="cuda")
    return steps, hist


def _run(sets, prec, noalloc, keep_hist_inside=False):
    torch = _torch()
    stream = torch.cuda.current_stream().cuda_stream
    h = _lib.fpt_plan(sets, prec, TUNE)
    try:
        steps, hist = _outputs(torch, sets)
        ptrs = [t.data_ptr() for t in steps]
        if noalloc:
            _lib.fpt_simulate_noalloc(h, ptrs, None if keep_hist_inside else hist.data_ptr(),
                                      stream)
        else:
            raw = torch.empty(_lib.fpt_plan_workspace(h) + 256, dtype=torch.uint8,
                              device="cuda")
            ws = raw.data_ptr() + (-raw.data_ptr()) % 256
            _lib.fpt_simulate(h, ws, ptrs, hist.data_ptr(), stream)
        counts, moments = _lib.fpt_histogram_all(h, [int(s["n_bins"]) for s in sets])
        stats = _lib.fpt_plan_stats(h)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in steps], counts, moments, stats
    finally:
        _lib.fpt_plan_destroy(h)


def _same(a, b, label):
    steps_a, counts_a, mom_a, st_a = a
    steps_b, counts_b, mom_b, st_b = b
    for i in range(len(steps_a)):
        assert np.array_equal(steps_a[i], steps_b[i]), (label, i)
        assert counts_a[i].tolist() == counts_b[i].tolist(), (label, i)
        for k in INT_MOMENTS:
            assert mom_a[i][k] == mom_b[i][k], (label, i, k)
    assert st_a["replica_steps"] == st_b["replica_steps"], label
    assert st_a["n_launches"] == st_b["n_launches"], label


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_noalloc_equals_workspace_run_twice(prec):
    # first a multi-set plan with more replicas than slots (work queue,
    # regroups while replicas wait, tail compaction), then a smaller
    # single-set plan with censoring and overflow: the array keeps the first
    # call's contents, which the second must not see
    big = workloads.batched_sets(n_sets=6, seed=31, log2_min=16, log2_max=17, ramp_scale=300.0)
    small = [dict(workloads.plain_escape(n_replicas=1000, seed=5), max_steps=9_999,
                  hist_k_max=5_000)]
    for label, sets in (("first, larger", big), ("second, smaller", small)):
        ref = _run(sets, prec, noalloc=False)
        got = _run(sets, prec, noalloc=True)
        print(f"{prec} {label}: {got[3]['n_launches']} launches, "
              f"{got[3]['n_compactions']} compactions, {got[3]['n_regroups']} regroups")
        _same(ref, got, label)
        assert all((s != -7).all() for s in got[0])
        if len(sets) > 1:
            assert got[3]["n_regroups"] >= 1 and got[3]["n_compactions"] >= 1
    # histograms kept in the array when no output buffer is given
    inside = _run(small, prec, noalloc=True, keep_hist_inside=True)
    ref = _run(small, prec, noalloc=False)
    assert inside[1][0].tolist() == ref[1][0].tolist()


def test_noalloc_refuses_what_it_cannot_run():
    p = workloads.switching_ramp(n_replicas=2 ** 21)
    # one replica per lane for 2^21 replicas: 2^21 slots of lane state (36 B
    # each), 72 MiB > 48 MiB
    h = _lib.fpt_plan([p], "fp32c", dict(schedule=1, replicas_per_lane=1, waves_per_simd=1,
                                         steps_per_launch=4096))
    try:
        with pytest.raises(_lib.FptError) as e:
            _lib.fpt_simulate_noalloc(h, None, None, None)
        assert e.value.status == _lib.FPT_E_NOMEM
        assert "static scratch" in e.value.message
    finally:
        _lib.fpt_plan_destroy(h)
    for tun in (dict(TUNE, waves_per_simd=0), dict(TUNE, use_graph=1)):
        h = _lib.fpt_plan([workloads.plain_escape(n_replicas=64)], "fp64", tun)
        try:
            with pytest.raises(_lib.FptError) as e:
                _lib.fpt_simulate_noalloc(h, None, None, None)
            assert e.value.status == _lib.FPT_E_INVAL
        finally:
            _lib.fpt_plan_destroy(h)
