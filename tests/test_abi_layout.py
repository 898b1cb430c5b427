"""The ctypes structs of the binding against the C header, on the CPU: a
small C program compiled against include/cvo.h prints the size of every
struct of the ABI and the offset of each field the binding declares, and
they must equal ctypes' (a field added on one side only would make the
library read or write past the caller's struct)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1904_02266_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = (B.cvo_cloud, B.cvo_params, B.cvo_rgbd_frame, B.cvo_result, B.cvo_serving_counters)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a C compiler")
def test_struct_layouts_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cvo.h"', "int main(void) {"]
    for S in STRUCTS:
        name = S.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in S._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for S in STRUCTS:
        name = S.__name__
        assert got[(name, "size")] == ctypes.sizeof(S), name
        for f, _ in S._fields_:
            assert got[(name, f)] == getattr(S, f).offset, (name, f)
