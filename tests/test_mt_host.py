"""CPU check of the library's MT19937 state handling (regeneration 4 words at
a time, group-major layout, restore mid-regeneration) against the oracle's
generator: the header is built for the host with hipcc."""

import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_lazy_regeneration_matches_oracle(tmp_path, oracle_mod):
    exe = tmp_path / "mt_host_check"
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"),
                    os.path.join(HERE, "mt_host_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = np.array(out.split(), dtype=np.uint64).reshape(400, 3, 4).astype(np.uint32)
    for s, seed in enumerate([5489, 5490, 2**32 - 1]):
        ref = oracle_mod.mt19937(seed, 1600).reshape(400, 4)
        assert np.array_equal(got[:, s, :], ref), seed
