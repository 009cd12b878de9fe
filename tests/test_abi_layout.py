"""The ctypes mirror of include/rid.h has the C layout (host only).

A small C program built with gcc against the header prints the size of
every ABI structure and the offset of each field; the binding's ctypes
structures must match them field by field, so that no argument is read at a
shifted address.
"""

import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NAMES = ["rid_allocator", "rid_problem_desc", "rid_solve_opts", "rid_stats", "rid_kernel_stat", "rid_request",
         "rid_result", "rid_server_opts", "rid_aux_basis_desc"]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_ctypes_layout_matches_the_header(tmp_path):
    from paper_2404_17133_amd import _binding as B

    STRUCTS = {name: getattr(B, name) for name in NAMES}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rid.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for fname, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, fname, name, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c = {}
    for line in out:
        if line:
            parts = line.split()
            c[(parts[0], parts[1])] = int(parts[2])
    for name, cls in STRUCTS.items():
        assert c[(name, "size")] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert c[(name, fname)] == getattr(cls, fname).offset, (name, fname)
