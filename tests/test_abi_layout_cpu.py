"""The ctypes structures of the binding have the layout of the C structs
declared in include/spfas.h: a small C program built with gcc against the
header prints sizeof and every field's offsetof, and they must equal what
ctypes computes for the binding's mirror of each struct."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2005_01275_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["spfas_mesh", "spfas_coarsen_opts", "spfas_allocator", "spfas_problem", "spfas_solve_opts",
           "spfas_stats", "spfas_server_opts", "spfas_request_info", "spfas_server_counters"]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_binding_structs_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "spfas.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in getattr(N, name)._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            name, field, val = ln.split()
            got[(name, field)] = int(val)
    for name in STRUCTS:
        cls = getattr(N, name)
        assert got[(name, "sizeof")] == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
