"""CPU check of the generator variant that the FP32C busy loop uses
(paper_1802_05065_amd/csrc/device_math.hpp, built for the host with hipcc):
with the parts of rounds 0 and 1 that do not depend on counter word 0 formed
beforehand, the words equal the oracle's Philox4x32-10 for the same counter
and key, over random counters and keys and the extreme word values."""

import os
import random
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

from oracle import oracle  # noqa: E402


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_fixed_part_words_equal_oracle_philox(tmp_path):
    exe = tmp_path / "philox_fixed_check"
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"),
                    os.path.join(HERE, "philox_fixed_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    rng = random.Random(5)
    edge = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF]
    cases = [tuple(rng.choice(edge) for _ in range(6)) for _ in range(300)]
    cases += [tuple(rng.getrandbits(32) for _ in range(6)) for _ in range(3000)]
    # consecutive blocks of one replica across a 2^32 crossing of word 0
    cases += [(c0, 7, 123456789, 0, 0xDEADBEEF, 0x01234567)
              for c0 in (0xFFFFFFFD, 0xFFFFFFFE, 0xFFFFFFFF, 0, 1)]
    text = "".join(" ".join(str(v) for v in c) + "\n" for c in cases)
    out = subprocess.run([str(exe)], input=text, check=True, capture_output=True,
                         text=True).stdout.split("\n")
    assert len([line for line in out if line]) == len(cases)
    for c, line in zip(cases, out):
        got = [int(v) for v in line.split()]
        want = oracle.philox4x32_10(np.array(c[:4], dtype=np.uint32),
                                    np.array(c[4:], dtype=np.uint32))
        assert got == [int(v) for v in want], c
