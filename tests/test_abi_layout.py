"""The ctypes mirrors of the C ABI's structures (paper_2204_00326_amd/ls.py) against include/ls.h:
a small C program built with gcc prints sizeof and every field's offsetof; they must equal what
ctypes computes, so a field added to one side only fails here (no GPU, no library load)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2204_00326_amd import ls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"ls_options": ls._Options, "ls_solve_info": ls._Info, "ls_stats_t": ls._Stats,
           "ls_plan_info": ls._PlanInfo, "ls_tune_info": ls._TuneInfo, "ls_nop_config": ls._NopConfig}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_ctypes_structures_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ls.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (ln.split() for ln in out if ln.strip())}
    for cname, py in STRUCTS.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
