"""The binding's ctypes structures against the C header: every struct that
crosses the boundary by pointer has the same size and the same field
offsets on both sides.  A short ctypes buffer would otherwise be written past
its end by the library (bemfft_plan_get_info, bemfft_solve) without any
error.  A small C program built with gcc against include/bemfft.h prints
sizeof and offsetof; CPU only."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1809_00845_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [B.bemfft_grid, B.bemfft_plan_opts, B.bemfft_solve_opts, B.bemfft_solve_info, B.bemfft_plan_info]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "bemfft.h"', "int main(void) {"]
    for st in STRUCTS:
        name = st.__name__
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([gcc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        name, key, value = line.split()
        table[(name, key)] = int(value)
    return table


@pytest.mark.parametrize("st", STRUCTS, ids=lambda s: s.__name__)
def test_struct_matches_header(c_layout, st):
    name = st.__name__
    assert ctypes.sizeof(st) == c_layout[(name, "size")], name
    for field, _ in st._fields_:
        assert getattr(st, field).offset == c_layout[(name, field)], (name, field)
