"""Benchmark: replica-steps/s of the FP32-compensated integrator against the
FP64 one on the switching-current workload, at KS-pass accuracy.

Workload (the switching-current distribution under a linear ramp): 2^20
underdamped replicas, alpha 0.05, T 0.002, gamma(t) = 1e-6 t from 0,
dt 0.05, phi0 = v0 = 0, escape at phi > 2 pi, 256-bin histogram of the bias
at switching.  One step = one fpt_simulate of the whole workload (every
replica integrated until it switches, escape steps recorded, histogram and
moments reduced), inputs resident on the GPU.

Prints one JSON line.  Runs on one GPU only.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "replica-steps/s FP32-comp vs FP64 at KS-pass accuracy; p50/p99 job latency"

# Algorithmic VALU work per replica-step, in full-rate issue slots (a
# quarter-rate instruction counts 4).  Per 4-step block: Philox4x32-10 with a
# wave-uniform key = 10 rounds x (2 v_mad_u64_u32 + 4 v_xor) ; 4 uniforms
# (cvt + fma); 2 Box-Muller pairs (log, sqrt, sin, cos + 3 mul); per step:
# sin(phi) (scale + v_sin), gamma_k (f64 fma + cvt), Kahan phase (fma, add,
# 2 sub), velocity (mul, fma, sub, fma), threshold compare.
TRANS_COST = 4      # v_sin/v_cos/v_log/v_sqrt_f32 issue cost (full-rate slots)
MAD64_COST = 4      # v_mad_u64_u32 issue cost
OPS_FP32C = (10 * (2 * MAD64_COST + 4) + 4 * 2 + 2 * (4 * TRANS_COST + 3)
             + 4 * ((1 + TRANS_COST) + 2 + 4 + 4 + 1)) / 4.0
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock


def counter_traffic(slots: int):
    """HBM bytes per launch of the FP32C slice kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None when the kernel sources
    (or the launch shape) differ from those the counters were taken on."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "slice_kernel_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["kernel_sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != rec["kernel_sources_sha256"] or int(rec["slots"]) != slots:
            return None
        return float(rec["bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--replicas", type=int, default=2 ** 20,
                    help="replicas of the FP32C leg (the workload has 2^20)")
    ap.add_argument("--fp64-replicas", type=int, default=2 ** 18,
                    help="replicas of the FP64 comparison leg (independent seed); 0 runs "
                         "the FP32C leg alone and prints its figures only")
    ap.add_argument("--cpu-replicas", type=int, default=32,
                    help="replicas of the oracle CPU-baseline sample (0: skip)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes (0: min(16, host cores))")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (scale for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def copy_calibration():
    import torch

    n = 256 << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)


def cpu_baseline(n_rep: int, procs: int):
    import oracle
    from paper_1802_05065_amd import workloads

    oracle.build(force=False)
    p = workloads.switching_ramp(n_replicas=n_rep, seed=2)
    op = oracle.OracleParams(**workloads.to_oracle_kwargs(p))
    procs = max(1, min(procs, n_rep))
    chunks = [(i * n_rep // procs, (i + 1) * n_rep // procs) for i in range(procs)]
    t0 = time.perf_counter()
    children = []
    for a, b in chunks:
        args = [oracle.oracle._CLI, str(op.model), repr(op.alpha), repr(op.T), repr(op.V0),
                repr(op.gamma0), repr(op.ramp), repr(op.dt), repr(op.phi0), repr(op.v0),
                repr(op.threshold), str(op.max_steps), str(op.seed), str(a), str(b - a)]
        children.append(subprocess.Popen(args, stdout=subprocess.PIPE, text=True))
    total = 0
    for c in children:
        out, _ = c.communicate()
        if c.returncode != 0:
            raise RuntimeError("oracle CLI failed")
        total += int(out.split("\n")[0].split()[2])
    wall = time.perf_counter() - t0
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:
        pass
    return {"value": total / wall, "unit": "replica-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"switching-current workload, replicas 0..{n_rep - 1} (seed 2) in "
                      f"{procs} single-threaded oracle processes, {total} replica-steps, "
                      f"{wall:.1f} s wall; host CPU: {cpu}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import torch
    from scipy import stats

    from paper_1802_05065_amd import api, workloads

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    # library load and autotuning of both precisions (untimed): plans of the
    # same size and shape with a 1000x faster ramp, so the tuner sees the
    # real occupancy
    for prec, n in (("fp32c", args.replicas), ("fp64", args.fp64_replicas)):
        if n <= 0:
            continue
        api.simulate(workloads.switching_ramp(n_replicas=n, seed=99) | dict(
            ramp=1e-3, max_steps=20_100, hist_k_max=20_000), prec, record_steps=False)

    p32 = workloads.switching_ramp(n_replicas=args.replicas, seed=2)
    plan32 = api.Plan([p32], "fp32c", None, dev)
    for _ in range(args.warmup):
        plan32.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        runs.append(plan32.run())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rs32 = sum(r.stats["replica_steps"] for r in runs)
    value = rs32 / (t1 - t0)
    last = runs[-1]
    st = last.stats
    steps32 = last.steps[0].cpu().numpy()
    print(f"[bench] fp32c {args.replicas} replicas: {value:.4e} replica-steps/s, "
          f"{st['n_launches']} launches, tuning {st['tuning']}", file=sys.stderr, flush=True)

    if args.fp64_replicas <= 0:  # profiling runs: the FP32C leg only
        print(json.dumps({"value": value, "launches": st["n_launches"],
                          "kernel_ms": st["kernel_ms"], "replica_steps": st["replica_steps"],
                          "tuning": st["tuning"]}), flush=True)
        return

    # FP64 leg (independent seed) for the speed ratio and the KS test
    p64 = workloads.switching_ramp(n_replicas=args.fp64_replicas, seed=3)
    plan64 = api.Plan([p64], "fp64", None, dev)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    r64 = plan64.run()
    torch.cuda.synchronize()
    f1 = time.perf_counter()
    value64 = r64.stats["replica_steps"] / (f1 - f0)
    steps64 = r64.steps[0].cpu().numpy()
    print(f"[bench] fp64 {args.fp64_replicas} replicas: {value64:.4e} replica-steps/s",
          file=sys.stderr, flush=True)

    e32, e64 = steps32[steps32 > 0], steps64[steps64 > 0]
    ks = stats.ks_2samp(e32, e64)
    se = math.sqrt(e32.var() / e32.size + e64.var() / e64.size)
    dmean = float(e32.mean() - e64.mean())
    ks_info = {"pvalue": float(ks.pvalue), "statistic": float(ks.statistic),
               "pass": bool(ks.pvalue > 0.01 and abs(dmean) < 3 * se),
               "mean_switch_step_fp32c": float(e32.mean()), "mean_switch_step_fp64": float(e64.mean()),
               "mean_diff_over_se": dmean / se if se > 0 else None,
               "censored_fp32c": int((steps32 < 0).sum()), "censored_fp64": int((steps64 < 0).sum())}

    kernel_s = st["kernel_ms"] * 1e-3
    launches = max(st["n_launches"], 1)
    achieved = st["replica_steps"] * OPS_FP32C / kernel_s if kernel_s > 0 else 0.0
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
            "unit": "TOP/s", "frac": achieved / PEAK_LANE_OPS,
            "traffic": counter_traffic(
                torch.cuda.get_device_properties(0).multi_processor_count * 4 * 64
                * st["tuning"]["waves_per_simd"] * st["tuning"]["replicas_per_lane"]),
            "kernel": "slice_kernel<fp32c, underdamped>",
            "ops_per_replica_step": OPS_FP32C,
            "avg_launch_ms": st["kernel_ms"] / launches, "launches": st["n_launches"]}

    cpu = None
    if args.cpu_replicas > 0:
        procs = args.cpu_procs or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(args.cpu_replicas, procs)

    line = {
        "metric": METRIC, "value": value, "unit": "replica-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (t1 - t0) * 1e3 / max(args.steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "switching-current ramp: underdamped, alpha 0.05, T 0.002, "
                               "gamma = 1e-6 t from 0, dt 0.05, threshold 2 pi, 256 bins",
                   "replicas": args.replicas, "precision": "fp32c",
                   "tuning": st["tuning"]},
        "fp64": {"value": value64, "replicas": args.fp64_replicas,
                 "speedup_fp32c_over_fp64": value / value64 if value64 > 0 else None,
                 "tuning": r64.stats["tuning"]},
        "ks": ks_info,
        "latency": None,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
