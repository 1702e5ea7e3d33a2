"""Write the FP64 oracle's escape steps of the switching-current workload's
first 1024 replicas, for the two seeds the GPU tests compare against.

The workload is Algorithm 3 (SwitchingCurrent): underdamped, alpha 0.05,
T 0.002, gamma(t) = 1e-6 t from 0, dt 0.05, phi0 = v0 = 0, escape at
phi > 2 pi, cap 20.1e6 steps.  Seed 2 is the seed of the benchmark's FP32C
leg, seed 3 the seed of its FP64 leg.  Only ``oracle`` computes the values
(about 1.9e7 steps per replica; a few minutes on 8 host cores):

    python tests/golden/make_switching_golden.py
"""

from __future__ import annotations

import concurrent.futures
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1802_05065_amd import workloads  # noqa: E402  (inputs only)

N_FIRST = 1024
SEEDS = (2, 3)


def path_for(seed: int) -> str:
    return os.path.join(HERE, f"switching_fp64_seed{seed}_first{N_FIRST}.json")


def make(seed: int, workers: int) -> dict:
    p = workloads.switching_ramp(n_replicas=N_FIRST, seed=seed)
    op = oracle.OracleParams(**workloads.to_oracle_kwargs(p))
    chunk = 16
    starts = list(range(0, N_FIRST, chunk))
    # the oracle's C loop runs outside the GIL, so threads use every core
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(lambda a: oracle.escape_steps(op, a, min(chunk, N_FIRST - a)),
                            starts))
    steps = [int(k) for part in parts for k in part]
    return {
        "source": "FP64 oracle (oracle/fpt_oracle.c), Algorithm 3 replica loop",
        "workload": "switching-current ramp: underdamped, alpha 0.05, T 0.002, "
                    "gamma = 1e-6 t from 0, dt 0.05, phi0 = v0 = 0, threshold 2 pi, "
                    "cap 20100000 steps",
        "params": {k: p[k] for k in ("alpha", "T", "V0", "gamma0", "ramp", "dt", "phi0",
                                     "v0", "threshold", "max_steps", "seed")},
        "first_replica": 0,
        "escape_steps": steps,
    }


def main():
    oracle.build(force=False)
    workers = os.cpu_count() or 1
    for seed in SEEDS:
        rec = make(seed, workers)
        with open(path_for(seed), "w") as f:
            json.dump(rec, f, separators=(",", ":"))
            f.write("\n")
        print(f"seed {seed}: {len(rec['escape_steps'])} replicas written", flush=True)


if __name__ == "__main__":
    main()
