"""Build ``tests/c_client/fpt_c_client``: a C program that uses libfpt through
``include/fpt.h`` and the HIP runtime's C API only (gcc, no C++ and no
Python).  It links against the in-tree ``paper_1802_05065_amd/libfpt.so``,
found at run time relative to the binary, so build the library first."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1802_05065_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SOURCE = os.path.join(HERE, "fpt_c_client.c")
BINARY = os.path.join(HERE, "fpt_c_client")


def build() -> str:
    # (the HIP runtime's C headers need C11 and are not -pedantic clean;
    # fpt.h alone is checked as pedantic C99 by the CPU tests)
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror",
           "-D_POSIX_C_SOURCE=200809L", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"), SOURCE, "-o", BINARY + ".tmp",
           "-L" + PKG, "-lfpt", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1802_05065_amd",
           "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"C client build failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(BINARY + ".tmp", BINARY)
    return BINARY


if __name__ == "__main__":
    print(build())
