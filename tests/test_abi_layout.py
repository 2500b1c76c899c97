"""The binding's ctypes structures against the C header's layout (no GPU):
a small C program built with the host compiler prints sizeof and offsetof of
every field of sos_adam_t, sos_solve_opts_t and sos_result_t, and each must
equal the ctypes mirror's."""
import ctypes
import os
import shutil
import subprocess

import pytest

S = pytest.importorskip("paper_2410_19844_amd")

INCLUDE = os.path.join(os.path.dirname(__file__), "..", "include")
MIRRORS = {"sos_adam_t": S._Adam, "sos_solve_opts_t": S._SolveOpts, "sos_result_t": S._Result}


def test_structure_layouts_match_the_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sos.h"', 'int main(void) {']
    for cname, mirror in MIRRORS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in mirror._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", INCLUDE, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, mirror in MIRRORS.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(mirror), cname
        for field, _ in mirror._fields_:
            assert got[(cname, field)] == getattr(mirror, field).offset, (cname, field)
