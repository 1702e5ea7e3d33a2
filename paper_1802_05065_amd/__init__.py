"""MI355X (gfx950) first-passage-time library for Langevin replicas of a
Josephson junction in a tilted washboard potential (arXiv:1802.05065).

The compute path is the C ABI of ``include/fpt.h`` implemented in HIP
(``csrc/``); this package holds its ctypes binding (``_lib``), PyTorch
plumbing for device memory and streams (``api``), the physics analyses built
on it (``analysis``), the seeded workloads (``workloads``) and the build
script (``build``).
"""

from ._lib import (  # noqa: F401
    FPT_FP32C,
    FPT_FP64,
    FPT_EXPLICIT,
    FPT_OVERDAMPED,
    FPT_RNG_MT19937,
    FPT_RNG_PHILOX,
    FPT_SCHED_ONE_PER_LANE,
    FPT_SCHED_REFILL,
    FPT_SEMI_IMPLICIT,
    FPT_UNDERDAMPED,
    FptError,
    fpt_api_version,
    fpt_histogram,
    fpt_histogram_all,
    fpt_last_error,
    fpt_mt_words,
    fpt_normals,
    fpt_plan,
    fpt_plan_destroy,
    fpt_plan_stats,
    fpt_plan_workspace,
    fpt_poll,
    fpt_rng_words,
    fpt_server_create,
    fpt_server_destroy,
    fpt_server_stats_get,
    fpt_simulate,
    fpt_simulate_noalloc,
    fpt_submit,
    fpt_trajectory,
)
