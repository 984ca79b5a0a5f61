"""The Python binding's structs have the C header's layout: a C program built against
include/perm3.h prints each struct's size and field offsets, which must equal ctypes'."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2407_20205_amd import perm3 as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "perm_server_cfg": P.perm_server_cfg,
    "perm_done": P.perm_done,
    "perm_server_stats": P.perm_server_stats,
    "perm_tuning": P.perm_tuning,
    "perm_timing": P.perm_timing,
    "perm_device_info": P.perm_device_info,
}


def c_layout(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "perm3.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, key, value = line.split()
        got[(name, key)] = int(value)
    return got


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match_the_header(tmp_path):
    got = c_layout(tmp_path)
    for name, cls in STRUCTS.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
