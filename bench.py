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

# Algorithmic VALU lane-operations per replica-step of the FP32C path: the
# method's operations per 4-step block, one lane-op per instruction (sin and
# generator operations included):
#   Philox4x32-10: 10 rounds x (2 32x32->64 products + 2 three-input XORs) = 40
#   4 uniforms (radii: convert + scale; angles: one bit-field insert)       =  6
#   Box-Muller: 2 x (log, sqrt, cos, sin) + 2 noise scalings                = 10
#   bias: 1 FP64 fma + 1 convert per block + 3 FP32 increments              =  5
#   4 steps x (sin, phase advance fma, 3 velocity fma) + 3 phases of the
#     block + compensated fold of the block's advance (add, 2 subtractions) = 26
#   threshold: largest of the 4 phases (2) and one compare                  =  3
#   block counter (FP64 step count, 64-bit block index)                     =  2
OPS_FP32C = (40 + 6 + 10 + 5 + 26 + 3 + 2) / 4.0
# MI355X FP32 vector peak 157.3 TFLOP/s = 78.6e12 FMA lane-operations/s
# (256 CUs x 128 FP32 lanes per clock x 2.4 GHz)
PEAK_LANE_OPS = 256 * 128 * 2.4e9
# FP64 flops per replica-step of the FP64 kernel as compiled (its own sin,
# Box-Muller log, sqrt and sin/cos): 11.74 adds + 16.49 multiplies + 34.48
# FMAs (2 flops) per step from its SQ_INSTS_VALU_{ADD,MUL,FMA}_F64 counters
# (profiles/slice_kernel_fp64_switching_2p18.md); peak 78.6 TFLOP/s.
FP64_FLOPS_PER_STEP = 11.74 + 16.49 + 2 * 34.48
PEAK_FP64_FLOPS = 78.6e12


# Instructions per 4-step block of one replica as the FP32C underdamped kernel
# compiles them for gfx950 (its hot loop's disassembly), by issue class; each
# class is priced at the rate profiles/isa_rates_gfx950.txt measured for it.
FP32C_BLOCK_MIX = {
    "mad_u64_u32_s0": 18,  # Philox products (2 of rounds 0-1 formed once per one-set loop)
    "bitop3_b32_s": 16,    # Philox three-input XORs (rounds 2-9)
    "xor_b32": 3,          # what rounds 0-1 leave per block
    "sin_f32": 6, "cos_f32": 2, "log_f32": 2,
    "sqrt_f32_neg": 2,     # Box-Muller radius, negated operand (VOP3 form)
    "fmac_f32_s": 16,      # phase advance, noise, force, damping
    "add_f32": 10,         # phases of the block, fold, bias offsets; priced alike:
                           # near-threshold compare and 2 register copies
    "sub_f32": 2,          # error term of the fold
    "mul_f32": 2, "fmamk_f32": 2,
    "cvt_f32_u32": 2,      # uniforms of the radii
    "cvt_f32_f64": 1,      # the block's bias G_k to FP32
    "alignbit_b32": 2,     # uniforms of the angles
    "max_f32": 1, "max3_f32": 1,  # largest phase of the block
    "fma_f64": 1, "add_f64": 1,   # bias G_k and step count in FP64
    "add_u32": 2,          # block index
}


def mix_attainable(mix=FP32C_BLOCK_MIX):
    """Replica-steps/s the instruction mix can issue at the measured per-class
    rates (None without the rate table)."""
    path = os.path.join(ROOT, "profiles", "isa_rates_gfx950.txt")
    rates = {}
    try:
        for line in open(path):
            f = line.split()
            if len(f) == 4 and f[1] == "1":
                rates[f[0]] = float(f[2]) * 1e12
    except OSError:
        return None
    if not all(k in rates for k in mix):
        return None
    block_s = sum(n / rates[k] for k, n in mix.items())
    return 4.0 / block_s


def counter_traffic():
    """Mean HBM bytes per launch of the FP32C slice kernel over the timed run,
    from the committed FETCH_SIZE / WRITE_SIZE counter runs of this command,
    or None when the kernel sources differ from those the counters were
    taken on."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "slice_kernel_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["kernel_sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != rec["kernel_sources_sha256"]:
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
    ap.add_argument("--cpu-replicas", type=int, default=64,
                    help="replicas of the oracle CPU-baseline sample (0: skip)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes (0: min(16, host cores))")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="arrival window of the rate-scaled serving leg (0: skip)")
    ap.add_argument("--serve-drain", type=float, default=45.0,
                    help="longest wait for admitted jobs after the window")
    ap.add_argument("--literal-seconds", type=float, default=8.0,
                    help="window of the serving trace at its literal 50 jobs/s (0: skip)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched leg (256 sets, full ramps) of the benchmark line")
    ap.add_argument("--serve-steps", type=int, default=0,
                    help="steps per launch of the serving loop (0: the server's default)")
    ap.add_argument("--serve-rho", type=float, default=0.7,
                    help="offered load of the rate-scaled trace, as a fraction of the "
                         "measured FP32C throughput")
    ap.add_argument("--mode", choices=("switching", "uneven", "batched", "mt", "next", "serve",
                                       "identical"),
                    default="switching",
                    help="switching: the benchmark line (default); uneven: refill vs "
                         "one-replica-per-lane on the uneven overdamped workload; batched: "
                         "the 256-set workload in one graph-replayed persistent launch; mt: "
                         "the switching workload with per-replica MT19937 against Philox; "
                         "next: rates of the semi-implicit scheme and of the Arrhenius and "
                         "switching-distribution analyses; serve: the serving legs alone, "
                         "with --serve-seconds / --literal-seconds as given; identical: the "
                         "single-set against the multi-set kernel on identical sets")
    ap.add_argument("--capacity", type=float, default=1.43e12,
                    help="serve mode: the FP32C replica-steps/s the rate-scaled trace is "
                         "scaled to")
    ap.add_argument("--waves", default="7,8",
                    help="identical mode: waves per SIMD to run (comma separated)")
    ap.add_argument("--ramp-scale", type=float, default=1.0,
                    help="batched mode: multiply every ramp (shorter runs)")
    ap.add_argument("--no-regroup", action="store_true",
                    help="batched mode: never move the active replicas into set order")
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


def _host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            return next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:
        return ""


def _oracle_processes(tasks):
    """Run the oracle CLI once per task (params dict, first replica, count),
    all at once, one single-threaded process each.  Returns (replica-steps,
    wall seconds, per-process seconds from the oracle's own clock)."""
    import oracle
    from paper_1802_05065_amd import workloads

    oracle.build(force=False)
    t0 = time.perf_counter()
    children = []
    for p, first, n in tasks:
        op = oracle.OracleParams(**workloads.to_oracle_kwargs(p))
        args = [oracle.oracle._CLI, str(op.model), repr(op.alpha), repr(op.T), repr(op.V0),
                repr(op.gamma0), repr(op.ramp), repr(op.dt), repr(op.phi0), repr(op.v0),
                repr(op.threshold), str(op.max_steps), str(op.seed), str(first), str(n)]
        children.append(subprocess.Popen(args, stdout=subprocess.PIPE, text=True))
    total, secs = 0, []
    for c in children:
        out, _ = c.communicate()
        if c.returncode != 0:
            raise RuntimeError("oracle CLI failed")
        head = out.split("\n")[0].split()
        total += int(head[2])
        secs.append(float(head[4]))
    return total, time.perf_counter() - t0, secs


def cpu_baseline(n_rep: int, procs: int):
    """The FP64 oracle on the host cores: the benchmark workload's first
    `n_rep` replicas split over `procs` processes (the line's value), and
    per-workload rates: the plain fixed-bias workload in full (one process,
    about 0.1 s), 32768 replicas of the uneven overdamped workload and one
    replica of each of the batched workload's first 16 sets (16 processes
    each)."""
    from paper_1802_05065_amd import workloads

    procs = max(1, min(procs, n_rep))
    p2 = workloads.switching_ramp(n_replicas=n_rep, seed=2)
    tasks = [(p2, i * n_rep // procs, (i + 1) * n_rep // procs - i * n_rep // procs)
             for i in range(procs)]
    total, wall, secs = _oracle_processes(tasks)
    cpu = _host_cpu_model()
    per = {}

    def record(name, tasks_, note):
        rs, w, ss = _oracle_processes(tasks_)
        per[name] = {"replica_steps": rs, "processes": len(tasks_), "wall_s": w,
                     "replica_steps_per_s": rs / w,
                     "ns_per_replica_step_one_core": 1e9 * sum(ss) / rs,
                     "process_s_min": min(ss), "sample": note}

    record("plain_escape_full", [(workloads.plain_escape(), 0, 1024)],
           "fixed-bias workload, all 1024 replicas, one process")
    p3 = workloads.uneven_overdamped(n_replicas=32768)
    record("uneven_32768", [(p3, i * 2048, 2048) for i in range(16)],
           "uneven overdamped workload, replicas 0..32767, 16 processes of 2048")
    sets = workloads.batched_sets(n_sets=256, seed=4)
    record("batched_16_sets", [(s, 0, 1) for s in sets[:16]],
           "batched workload, replica 0 of sets 0..15, one process each")
    return {"value": total / wall, "unit": "replica-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"switching-current workload, replicas 0..{n_rep - 1} (seed 2) in "
                      f"{procs} single-threaded oracle processes, {total} replica-steps, "
                      f"{wall:.1f} s wall (each process {min(secs):.1f}-{max(secs):.1f} s)",
            "ns_per_replica_step_one_core": 1e9 * sum(secs) / total,
            "host_cores": os.cpu_count(), "host_cpu": cpu, "per_workload": per}


def serving_leg(capacity: float, window_s: float, drain_s: float, rho: float,
                steps_per_launch: int = 0, literal: bool = False):
    """Continuous batching on the serving trace (Poisson arrivals at 50
    jobs/s, ramp jobs with 2^10..2^18 replicas).  Rate-scaled (default): the
    arrival times are stretched so the trace offers `rho` of the measured
    capacity; jobs arriving in `window_s` are submitted and polled until done
    (at most `drain_s` more).  Literal: the trace at 50 jobs/s as written for
    `window_s`, then stop; what finished, and the backlog left.  Latency is
    submit-to-result; it is also given per unit of the job's own work
    (seconds per 10^12 replica-steps) and as a stretch (latency x capacity /
    work: 1 is a job that had the whole GPU's rate to itself)."""
    import numpy as np
    import torch

    from paper_1802_05065_amd import _lib, workloads

    trace = workloads.serving_trace(rate_per_s=50.0, duration_s=60.0, seed=5)
    # expected work of a job, bounded by the steps to gamma = 1 (hist_k_max)
    work = np.array([j["params"]["n_replicas"] * j["params"]["hist_k_max"] for j in trace],
                    dtype=np.float64)
    mean_work = float(work.mean())
    lam = 50.0 if literal else rho * capacity / mean_work
    stretch = 50.0 / lam
    pool_bytes = 1 << 30
    pool = torch.empty(pool_bytes + 256, dtype=torch.uint8, device="cuda")
    base = pool.data_ptr() + (-pool.data_ptr()) % 256
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    tun = dict(steps_per_launch=steps_per_launch) if steps_per_launch else None
    srv = _lib.fpt_server_create(base, pool_bytes, "fp32c", 0, tun, stream.cuda_stream)
    pending, lat, per_work, stretch_f, t_sub = {}, [], [], [], {}
    i = 0
    t0 = time.perf_counter()
    try:
        while True:
            now = time.perf_counter() - t0
            while i < len(trace) and trace[i]["t"] * stretch <= min(now, window_s):
                jid = _lib.fpt_submit(srv, trace[i]["params"])
                pending[jid] = trace[i]["params"]
                t_sub[jid] = time.perf_counter() - t0
                i += 1
            for jid in list(pending):
                p = pending[jid]
                r = _lib.fpt_poll(srv, jid, p["n_bins"])
                if r is not None:
                    m = r[1]
                    w = m["sum_k"] + m["n_censored"] * p["max_steps"]
                    lat.append(r[2])
                    per_work.append(r[2] / (w / 1e12))
                    stretch_f.append(r[2] * capacity / w)
                    del pending[jid]
            arrivals_done = i >= len(trace) or trace[i]["t"] * stretch > window_s
            if literal and now >= window_s:
                break
            if (now >= window_s and arrivals_done and not pending) or now > window_s + drain_s:
                break
            time.sleep(0.002)
        elapsed = time.perf_counter() - t0
        st = _lib.fpt_server_stats_get(srv)
    finally:
        _lib.fpt_server_destroy(srv)
    lat, per_work, stretch_f = np.array(lat), np.array(per_work), np.array(stretch_f)

    def pct(a, q):
        return float(np.percentile(a, q)) if a.size else None

    out = {
        "offered_jobs_per_s": lam, "window_s": window_s, "submitted": i,
        "finished": int(lat.size), "unfinished": len(pending),
        "p50_s": pct(lat, 50), "p99_s": pct(lat, 99), "max_s": float(lat.max()) if lat.size else None,
        "p50_s_per_1e12_replica_steps": pct(per_work, 50),
        "p99_s_per_1e12_replica_steps": pct(per_work, 99),
        "p50_stretch": pct(stretch_f, 50), "p99_stretch": pct(stretch_f, 99),
        "replica_steps_per_s": st["replica_steps"] / elapsed, "launches": st["n_launches"],
        "elapsed_s": elapsed,
    }
    if literal:
        out.update({"trace": "serving trace as written: Poisson arrivals at 50 jobs/s, ramp "
                             "jobs with 2^10..2^18 replicas, stopped at the end of the window",
                    "offered_replica_steps_per_s": 50.0 * mean_work,
                    "rho": 50.0 * mean_work / capacity,
                    "backlog_jobs": i - int(lat.size),
                    "queued_at_stop": st["queued"], "running_at_stop": st["running"]})
    else:
        out["trace"] = ("serving mix (Poisson, 2^10..2^18 replicas, ramp jobs) offered at "
                        f"rho={rho} of the measured FP32C capacity")
        if pending:
            # jobs still running at the drain cap: their latency is at least
            # their age then (lower bounds, not in the percentiles)
            out["unfinished_age_s"] = sorted(round(elapsed - t_sub[j], 2) for j in pending)
    return out


def uneven_mode(args):
    """Refill vs one replica per lane on the uneven overdamped workload
    (exponential-tailed escape times), with Appendix A's prediction."""
    import numpy as np
    import torch

    from paper_1802_05065_amd import api, workloads

    p = workloads.uneven_overdamped(n_replicas=args.replicas if args.replicas != 2 ** 20
                                    else 2 ** 22, seed=3)
    out = {"workload": "uneven overdamped: gamma 0.8, T 0.05, dt 0.01, threshold phi0 + 2 pi",
           "replicas": p["n_replicas"], "precision": "fp32c"}
    steps = None
    for sched in ("refill", "one_per_lane"):
        tun = dict(schedule=0 if sched == "refill" else 1)
        # untimed: library load and the tuner's trials, on the same replicas
        # (the tuner keys its cache by plan size), cut short by a step cap
        api.simulate(dict(p, seed=77, max_steps=20_000, hist_k_max=20_000), "fp32c", tun,
                     record_steps=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.simulate(p, "fp32c", tun)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = r.stats
        util = st["replica_steps"] / st["lane_steps"] if st["lane_steps"] else None
        out[sched] = {"replica_steps_per_s": st["replica_steps"] / (t1 - t0),
                      "wall_s": t1 - t0, "lane_utilization": util,
                      "launches": st["n_launches"], "compactions": st["n_compactions"],
                      "tuning": st["tuning"]}
        if steps is None:
            steps = r.steps[0].cpu().numpy()
        else:
            assert np.array_equal(steps, r.steps[0].cpu().numpy()), "schedules disagree"
    lanes = 64 * out["one_per_lane"]["tuning"]["replicas_per_lane"]
    k = steps[steps > 0].astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(0))
    emp = k.mean() / rng.choice(k, size=(20000, lanes)).max(axis=1).mean()
    per_slot = p["n_replicas"] / (out["refill"]["tuning"]["waves_per_simd"] * 4 * 64 *
                                  torch.cuda.get_device_properties(0).multi_processor_count *
                                  out["refill"]["tuning"]["replicas_per_lane"])
    # Appendix A's model: unit-exponential run times, so a thread with n_load
    # runs takes an Erlang(n_load, 1) time and the wavefront the largest of
    # its threads' times; efficiency = n_load / E[that maximum].  For one run
    # per thread E[max] is the harmonic number H_lanes; for a fixed share it
    # is estimated here by sampling.
    harmonic = sum(1.0 / i for i in range(1, lanes + 1))
    n_load = max(1, round(per_slot))
    static_eff = n_load / rng.gamma(n_load, size=(20000, lanes)).max(axis=1).mean()
    out["appendix_a"] = {
        "threads": lanes,
        "exponential_model_efficiency": 1.0 / harmonic,
        "empirical_escape_law_efficiency": float(emp),
        "static_partition_efficiency": float(static_eff),
        "static_partition_runs_per_thread": n_load,
        "static_partition_note": "Appendix A's model with each of the 64 threads of a "
                                 "wavefront given a fixed share of round(replicas per slot) "
                                 "jobs; refill assigns them dynamically instead",
        "note": "one replica per lane: a wavefront's slots wait for its slowest replica; "
                "Appendix A models escape times as unit exponentials (efficiency 1/H_N)"}
    out["identical_results_across_schedules"] = True
    print(json.dumps(out), flush=True)


def batched_roofline(st):
    """The headline's roofline terms for a multi-set run: algorithmic lane-ops
    per replica-step over the kernel time (with a graph, the captured groups,
    regroups included)."""
    kernel_s = st["kernel_ms"] * 1e-3
    if kernel_s <= 0:
        return None
    rate = st["replica_steps"] / kernel_s
    mix = mix_attainable()
    return {"bound": "alu", "achieved": rate * OPS_FP32C / 1e12, "peak": PEAK_LANE_OPS / 1e12,
            "unit": "TOP/s", "frac": rate * OPS_FP32C / PEAK_LANE_OPS,
            "ops_per_replica_step": OPS_FP32C,
            "frac_of_mix_attainable": rate / mix if mix else None}


def batched_mode(args):
    """The 256-set workload in one plan: persistent refill over all sets,
    launches replayed through a captured hipGraph."""
    import torch

    from paper_1802_05065_amd import api, workloads

    sets = workloads.batched_sets(n_sets=256, seed=4, ramp_scale=args.ramp_scale)
    res = {}
    for graph in (1, 0):
        tun = dict(use_graph=graph, no_regroup=int(args.no_regroup))
        api.simulate([dict(x, max_steps=min(x["max_steps"], 20_000),
                           hist_k_max=min(x["hist_k_max"] or x["max_steps"], 20_000))
                      for x in sets], "fp32c", tun, record_steps=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.simulate(sets, "fp32c", tun, record_steps=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = r.stats
        res["graph" if graph else "stream"] = {
            "replica_steps_per_s": st["replica_steps"] / (t1 - t0), "wall_s": t1 - t0,
            "replica_steps": st["replica_steps"], "launches": st["n_launches"],
            "kernel_s": st["kernel_ms"] / 1e3,
            "lane_utilization": st["replica_steps"] / max(st["lane_steps"], 1),
            "regroups": st["n_regroups"], "compactions": st["n_compactions"],
            # passes beyond one per wavefront block for lanes of other sets
            "extra_pass_fraction": st["extra_passes"] / max(st["lane_steps"] / 256, 1),
            "roofline": batched_roofline(st),
            "tuning": st["tuning"],
            "censored": int(sum(m["n_censored"] for m in r.moments))}
        if graph:
            hist_graph = [c.tolist() for c in r.counts]
        else:
            assert hist_graph == [c.tolist() for c in r.counts], "graph and stream disagree"
    print(json.dumps({"workload": "batched: 256 ramp sets", "ramp_scale": args.ramp_scale,
                      "replicas": sum(s["n_replicas"] for s in sets), "precision": "fp32c",
                      **res}), flush=True)


# MT19937 mode: per 4-step block a lane loads two 16-byte state groups and
# stores one (the lazily regenerated words), 12 bytes per replica-step.
MT_BYTES_PER_REPLICA_STEP = 48 / 4.0
PEAK_HBM = 8.0e12


def streaming_rate(reads: int) -> float:
    """Bytes/s of a plain device streaming kernel over 1 GiB operands with
    `reads` reads per write (torch copy for 1, elementwise add for 2): the
    rate an HBM-bound kernel with that read/write mix can attain here."""
    import torch

    n = 1 << 28
    a = torch.rand(n, device="cuda")
    b = torch.rand(n, device="cuda")
    c = torch.empty_like(a)
    fn = (lambda: c.copy_(a)) if reads == 1 else (lambda: torch.add(a, b, out=c))
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        fn()
    e1.record()
    torch.cuda.synchronize()
    rate = (reads + 1) * 4 * n / (e0.elapsed_time(e1) / 20 * 1e-3)
    del a, b, c
    torch.cuda.empty_cache()
    return rate


def mt_mode(args):
    """The switching workload drawn from Algorithm 2's generator (one MT19937
    per replica) against the same workload on Philox4x32-10, both FP32C."""
    import numpy as np
    import torch
    from scipy import stats

    from paper_1802_05065_amd import api, workloads

    n = args.replicas if args.replicas != 2 ** 20 else 2 ** 18
    out = {"workload": "switching-current ramp (as the benchmark line), FP32C",
           "replicas": n}
    samples = {}
    for rng in ("mt19937", "philox"):
        code = 1 if rng == "mt19937" else 0
        api.simulate(workloads.switching_ramp(n_replicas=n, seed=99) | dict(
            ramp=1e-3, max_steps=20_100, hist_k_max=20_000, rng=code), "fp32c",
            record_steps=False)
        p = workloads.switching_ramp(n_replicas=n, seed=2 if code else 3) | dict(rng=code)
        plan = api.Plan([p], "fp32c", None, torch.device("cuda", 0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = r.stats
        kernel_s = st["kernel_ms"] * 1e-3
        leg = {"replica_steps_per_s": st["replica_steps"] / (t1 - t0), "wall_s": t1 - t0,
               "launches": st["n_launches"], "tuning": st["tuning"],
               "avg_launch_ms": st["kernel_ms"] / max(st["n_launches"], 1)}
        if code:
            bw = st["replica_steps"] * MT_BYTES_PER_REPLICA_STEP / kernel_s
            # the generator state moves two 16 B reads per 16 B write
            attain = streaming_rate(2)
            leg["roofline"] = {"bound": "hbm", "achieved": bw / 1e9, "peak": PEAK_HBM / 1e9,
                               "unit": "GB/s", "frac": bw / PEAK_HBM,
                               "bytes_per_replica_step": MT_BYTES_PER_REPLICA_STEP,
                               "streaming_2r1w_GBps": attain / 1e9,
                               "frac_of_streaming": bw / attain}
        out[rng] = leg
        samples[rng] = r.steps[0].cpu().numpy()
        print(f"[bench] {rng}: {leg['replica_steps_per_s']:.4e} replica-steps/s",
              file=sys.stderr, flush=True)
    a, b = samples["mt19937"], samples["philox"]
    a, b = a[a > 0], b[b > 0]
    ks = stats.ks_2samp(a, b)
    out["mt_over_philox"] = (out["mt19937"]["replica_steps_per_s"]
                             / out["philox"]["replica_steps_per_s"])
    out["ks_mt_vs_philox"] = {"pvalue": float(ks.pvalue),
                              "mean_mt": float(a.mean()), "mean_philox": float(b.mean())}
    print(json.dumps(out), flush=True)


def next_mode(args):
    """Rates of the extensions beyond the plain method: the semi-implicit
    scheme on the benchmark workload (against the explicit one), an
    Arrhenius sweep (one batched plan over temperatures) and a
    switching-distribution run at the Li07 damping and temperature."""
    import torch

    from paper_1802_05065_amd import analysis, api, workloads

    n = args.replicas if args.replicas != 2 ** 20 else 2 ** 18
    out = {"replicas": n, "precision": "fp32c"}
    for scheme in (0, 1):
        api.simulate(workloads.switching_ramp(n_replicas=n, seed=99) | dict(
            ramp=1e-3, max_steps=20_100, hist_k_max=20_000, scheme=scheme), "fp32c",
            record_steps=False)
        plan = api.Plan([workloads.switching_ramp(n_replicas=n, seed=2) | dict(scheme=scheme)],
                        "fp32c", None, torch.device("cuda", 0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.run(record_steps=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = r.stats
        out["semi_implicit" if scheme else "explicit"] = {
            "replica_steps_per_s": st["replica_steps"] / (t1 - t0),
            "kernel_replica_steps_per_s": st["replica_steps"] / (st["kernel_ms"] * 1e-3),
            "mean_switch_step": r.moments[0]["sum_k"] / max(r.moments[0]["n_escaped"], 1),
            "tuning": st["tuning"]}
    g = 0.5
    du = float(analysis.barrier_height(g))
    temps = [du / x for x in (4.0, 5.0, 6.0, 7.0)]
    analysis.arrhenius_sweep(g, 0.5, temps, n_replicas=4096, dt=0.02,
                             max_steps=20_000)  # tuning on the same plan size, untimed
    t0 = time.perf_counter()
    arr = analysis.arrhenius_sweep(g, 0.5, temps, n_replicas=4096, dt=0.02)
    t1 = time.perf_counter()
    out["arrhenius"] = {"wall_s": t1 - t0, "replica_steps": arr["stats"]["replica_steps"],
                        "replica_steps_per_s": arr["stats"]["replica_steps"] / (t1 - t0),
                        "delta_U": arr["delta_U"], "delta_U_fit": arr["delta_U_arrhenius"]}
    for scheme in (1, 0):
        t0 = time.perf_counter()
        sw = analysis.switching_distribution(alpha=0.283, T=0.0673, ramp=1e-6, n_replicas=30000,
                                             dt=0.02, scheme=scheme)
        t1 = time.perf_counter()
        out[f"switching_cdf_scheme{scheme}"] = {
            "wall_s": t1 - t0, "replica_steps_per_s": sw["stats"]["replica_steps"] / (t1 - t0),
            "max_abs_diff_fd": sw["max_abs_diff"], "mean_gamma_sw": sw["mean_gamma_sw"]}
    print(json.dumps(out), flush=True)


def batched_leg():
    """The batched workload (256 ramp sets, 5.4e6 replicas, full ramps) in
    one FP32C plan: the multi-set kernel with its regroups, its launches
    replayed through a captured hipGraph, the tiling autotuned (the tuner's
    trials run first on the same plan with a 20000-step cap, untimed).
    Whole-run rate, kernel rate and the kernel's roofline terms."""
    import torch

    from paper_1802_05065_amd import api, workloads

    sets = workloads.batched_sets(n_sets=256, seed=4)
    api.simulate([dict(x, max_steps=min(x["max_steps"], 20_000),
                       hist_k_max=min(x["hist_k_max"] or x["max_steps"], 20_000))
                  for x in sets], "fp32c", None, record_steps=False)
    plan = api.Plan(sets, "fp32c", {"use_graph": 1})
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.run(record_steps=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    finally:
        plan.close()
    st = r.stats
    roof = batched_roofline(st)
    if roof is not None:
        roof["kernel"] = "slice_kernel<fp32c, underdamped, multi-set>"
        roof["avg_launch_ms"] = st["kernel_ms"] / max(st["n_launches"], 1)
    return {"workload": "batched: 256 ramp sets (alpha log-uniform [0.01, 1], T uniform "
                        "[1e-3, 5e-2], ramp log-uniform [1e-7, 1e-4]), 2^12..2^16 replicas each, "
                        "dt 0.05, FP32C, one plan, launches replayed through a hipGraph",
            "replicas": sum(s["n_replicas"] for s in sets),
            "replica_steps": st["replica_steps"], "wall_s": t1 - t0,
            "replica_steps_per_s": st["replica_steps"] / (t1 - t0),
            "kernel_replica_steps_per_s": st["replica_steps"] / (st["kernel_ms"] * 1e-3)
            if st["kernel_ms"] > 0 else None,
            "launches": st["n_launches"], "regroups": st["n_regroups"],
            "compactions": st["n_compactions"],
            "lane_utilization": st["replica_steps"] / max(st["lane_steps"], 1),
            "extra_pass_fraction": st["extra_passes"] / max(st["lane_steps"] / 256, 1),
            "censored": int(sum(m["n_censored"] for m in r.moments)),
            "tuning": st["tuning"], "roofline": roof}


def serving_legs(args, capacity):
    """The rate-scaled serving trace and the literal one, as the arguments
    ask (None when both are off)."""
    out = None
    if args.serve_seconds > 0:
        out = serving_leg(capacity, args.serve_seconds, args.serve_drain, args.serve_rho,
                          args.serve_steps)
        print(f"[bench] serving: {out['finished']} jobs, p50 {out['p50_s']} s, "
              f"p99 {out['p99_s']} s", file=sys.stderr, flush=True)
    if args.literal_seconds > 0:
        lit = serving_leg(capacity, args.literal_seconds, 0.0, args.serve_rho, args.serve_steps,
                          literal=True)
        print(f"[bench] literal trace: {lit['finished']} of {lit['submitted']} jobs done, "
              f"backlog {lit['backlog_jobs']}", file=sys.stderr, flush=True)
        out = dict(out or {}, literal_trace=lit)
    return out


def identical_mode(args):
    """The same work as one set and as 16 identical sets: 2^22 replicas of a
    1e-4 ramp (the benchmark workload's physics, 200000-step cap), FP32C,
    R = 1, 16384-step launches, at each wave count of --waves.  One plan per
    line, no untimed runs (the tuning is fixed), so a counter run sees only
    these launches; kernel lane-steps/s compare the single-set and the
    multi-set kernel issuing the same work."""
    import torch

    from paper_1802_05065_amd import api, workloads

    base = workloads.switching_ramp(n_replicas=2 ** 22, seed=11) | dict(
        ramp=1e-4, max_steps=201_000, hist_k_max=200_000)
    for w in (int(x) for x in args.waves.split(",")):
        tun = dict(replicas_per_lane=1, waves_per_simd=w, steps_per_launch=16384)
        for n_sets in (1, 16):
            sets = [dict(base, n_replicas=2 ** 22 // n_sets, seed=100 + i) for i in range(n_sets)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = api.simulate(sets, "fp32c", tun, record_steps=False)
            t1 = time.perf_counter()
            st = r.stats
            print(json.dumps({
                "waves_per_simd": w, "sets": n_sets, "lane_steps": st["lane_steps"],
                "replica_steps": st["replica_steps"], "launches": st["n_launches"],
                "kernel_lane_steps_per_s": st["lane_steps"] / (st["kernel_ms"] * 1e-3),
                "replica_steps_per_s": st["replica_steps"] / (t1 - t0),
                "lane_utilization": st["replica_steps"] / st["lane_steps"]}), flush=True)


def serve_mode(args):
    """The serving legs alone, against the capacity the benchmark line
    measured (`--capacity`, default 1.43e12 replica-steps/s)."""
    import torch

    torch.cuda.set_device(0)
    out = serving_legs(args, args.capacity)
    print(json.dumps({"capacity": args.capacity, "latency": out}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.mode == "uneven":
        uneven_mode(args)
        return
    if args.mode == "batched":
        batched_mode(args)
        return
    if args.mode == "mt":
        mt_mode(args)
        return
    if args.mode == "next":
        next_mode(args)
        return
    if args.mode == "serve":
        serve_mode(args)
        return
    if args.mode == "identical":
        identical_mode(args)
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
    for i in range(args.warmup):
        plan32.run()
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        # each run ends synchronized (its histogram readback); the progress
        # line costs microseconds of a multi-second step
        runs.append(plan32.run())
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
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
    f64_kernel = r64.stats["replica_steps"] / (r64.stats["kernel_ms"] * 1e-3)
    roof64 = {"bound": "alu", "achieved": f64_kernel * FP64_FLOPS_PER_STEP / 1e12,
              "peak": PEAK_FP64_FLOPS / 1e12, "unit": "TFLOP/s",
              "frac": f64_kernel * FP64_FLOPS_PER_STEP / PEAK_FP64_FLOPS,
              "flops_per_replica_step": FP64_FLOPS_PER_STEP}
    # same-seed paired error of FP32C against FP64: the FP64 oracle's
    # switching steps of the first 1024 replicas (seed 2), stored by
    # tests/golden/make_switching_golden.py
    paired = None
    gold_path = os.path.join(ROOT, "tests", "golden", "switching_fp64_seed2_first1024.json")
    if args.replicas >= 1024 and os.path.exists(gold_path):
        k64 = np.array(json.load(open(gold_path))["escape_steps"], dtype=np.int64)
        k32 = steps32[:k64.size]
        both = (k64 > 0) & (k32 > 0)
        dk = np.abs(k32[both] - k64[both]).astype(np.float64)
        paired = {"replicas": int(k64.size), "reference": "FP64 oracle, same seed",
                  "identical_fraction": float(np.mean(k32 == k64)),
                  "mean_abs_dk_steps": float(dk.mean()) if dk.size else None,
                  "median_abs_dk_steps_of_differing": float(np.median(dk[dk > 0]))
                  if (dk > 0).any() else 0.0,
                  "max_abs_dk_steps": float(dk.max()) if dk.size else None,
                  "max_abs_dgamma_sw": float(dk.max() * p64["ramp"] * p64["dt"])
                  if dk.size else None}
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

    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def lanes_of(tun):
        return cus * 4 * tun["waves_per_simd"] * 64 * tun["replicas_per_lane"]

    lanes32, lanes64 = lanes_of(st["tuning"]), lanes_of(r64.stats["tuning"])
    kernel_s = st["kernel_ms"] * 1e-3
    launches = max(st["n_launches"], 1)
    achieved = st["replica_steps"] * OPS_FP32C / kernel_s if kernel_s > 0 else 0.0
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
            "unit": "TOP/s", "frac": achieved / PEAK_LANE_OPS,
            "traffic": counter_traffic(),
            "kernel": "slice_kernel<fp32c, underdamped>",
            "ops_per_replica_step": OPS_FP32C,
            "mix_attainable_replica_steps_per_s": mix_attainable(),
            "frac_of_mix_attainable": (st["replica_steps"] / kernel_s / mix_attainable()
                                       if kernel_s > 0 and mix_attainable() else None),
            "avg_launch_ms": st["kernel_ms"] / launches, "launches": st["n_launches"]}

    def side_leg(name, fn):
        # a leg beside the headline: a library error there is reported in its
        # field and does not take the measured line with it
        try:
            return fn()
        except Exception as e:  # noqa: BLE001
            print(f"[bench] {name} leg failed: {type(e).__name__}: {e}", file=sys.stderr,
                  flush=True)
            return {"error": f"{type(e).__name__}: {e}"}

    batched = None
    if not args.no_batched:
        batched = side_leg("batched", batched_leg)
        if "error" not in batched:
            print(f"[bench] batched: {batched['replica_steps_per_s']:.4e} replica-steps/s, "
                  f"{batched['launches']} launches", file=sys.stderr, flush=True)

    latency = side_leg("serving", lambda: serving_legs(args, value))

    cpu = None
    if args.cpu_replicas > 0:
        procs = args.cpu_procs or min(16, os.cpu_count() or 1)
        cpu = side_leg("cpu_baseline", lambda: cpu_baseline(args.cpu_replicas, procs))

    line = {
        "metric": METRIC, "value": value, "unit": "replica-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (t1 - t0) * 1e3 / max(args.steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "switching-current ramp: underdamped, alpha 0.05, T 0.002, "
                               "gamma = 1e-6 t from 0, dt 0.05, threshold 2 pi, 256 bins",
                   "replicas": args.replicas, "precision": "fp32c",
                   "tuning": st["tuning"]},
        "kernel_value": st["replica_steps"] / kernel_s if kernel_s > 0 else None,
        "fp64": {"value": value64, "replicas": args.fp64_replicas,
                 "lanes": lanes64,
                 "note": "independent seed (3); the FP64 leg's replicas take "
                         f"{args.fp64_replicas / lanes64:.2f} rounds of its lanes, the FP32C "
                         f"leg's {args.replicas / lanes32:.2f}",
                 "kernel_value": f64_kernel,
                 "speedup_fp32c_over_fp64": value / value64 if value64 > 0 else None,
                 "tuning": r64.stats["tuning"], "roofline": roof64},
        "ks": ks_info,
        "paired_error_vs_fp64": paired,
        "batched": batched,
        "latency": latency,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
