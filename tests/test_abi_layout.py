"""The ctypes mirrors of the public structs (paper_1802_05065_amd/_lib.py)
against include/fpt.h as a C compiler lays it out: a generated C program
prints sizeof and, for every field the binding names, offsetof and size."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1802_05065_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CC = shutil.which("gcc") or shutil.which("cc")

STRUCTS = {
    "fpt_params": _lib.FptParams,
    "fpt_tuning": _lib.FptTuning,
    "fpt_moments": _lib.FptMoments,
    "fpt_run_stats": _lib.FptRunStats,
    "fpt_server_stats": _lib.FptServerStats,
}


@pytest.mark.skipif(CC is None, reason="no C compiler")
def test_ctypes_structs_match_the_header(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "fpt.h"',
             "int main(void) {"]
    expect = []
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        expect.append(f"{cname} {ctypes.sizeof(cls)}")
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu %zu\\n", offsetof({cname}, {fname}), '
                         f"sizeof((({cname}*)0)->{fname}));")
            f = getattr(cls, fname)
            expect.append(f"{cname}.{fname} {f.offset} {f.size}")
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([CC, "-std=c99", "-Wall", "-I" + os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    assert [g for g in got if g] == expect
