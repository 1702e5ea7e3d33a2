"""The oracle: plain FP64 reference implementation of arXiv:1802.05065's method.

TEST INFRASTRUCTURE ONLY -- imported by ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py``.  The GPU library never imports
it, and it never imports the GPU library.
"""

from .oracle import (  # noqa: F401
    OracleParams,
    build,
    derived,
    escape_steps,
    histogram,
    mt19937,
    normals,
    philox4x32_10,
    replica_steps,
    rng_words,
    run_cli,
    trajectory,
)
