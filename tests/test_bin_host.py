"""CPU check of the library's histogram binning, floor((k-1) n_bins / k_hist)
for escape steps k in [1, k_hist], computed on the device from an FP64
estimate and an integer correction: built for the host with hipcc and
compared with exact integer division, at bin edges and up to k_hist = 2^50."""

import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_bin_is_exact_integer_division(tmp_path):
    exe = tmp_path / "bin_host_check"
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"),
                    os.path.join(HERE, "bin_host_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    rng = random.Random(11)
    cases = []
    for _ in range(20000):
        nb = rng.choice([1, 2, 3, 7, 64, 256, 1000, 4093, 4096])
        kh = rng.choice([1, 7, 999, 2 ** 20 + 3, rng.randrange(1, 2 ** 50)])
        k = rng.randrange(1, kh + 1)
        cases.append((k, nb, kh))
        # both sides of every bin edge: (k-1) n_bins = b k_hist (+-1)
        b = rng.randrange(0, nb)
        edge = -(-b * kh // nb) + 1  # smallest k with (k-1) nb >= b kh
        for kk in (edge - 1, edge, edge + 1):
            if 1 <= kk <= kh:
                cases.append((kk, nb, kh))
    cases += [(1, 4096, 2 ** 50), (2 ** 50, 4096, 2 ** 50), (2 ** 50 - 1, 4093, 2 ** 50)]
    text = "".join(f"{k} {nb} {kh}\n" for k, nb, kh in cases)
    out = subprocess.run([str(exe)], input=text, check=True, capture_output=True,
                         text=True).stdout.split()
    for (k, nb, kh), got in zip(cases, out):
        assert int(got) == (k - 1) * nb // kh, (k, nb, kh)
    assert len(out) == len(cases)
