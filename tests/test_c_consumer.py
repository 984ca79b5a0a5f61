"""The C ABI from plain C: tests/c_consumer.c includes include/perm3.h alone, is compiled as C99
with -pedantic -Werror and linked against libperm3.so.  Without a GPU it runs the calls that need
none; on a GPU it also computes permanents fixed by closed forms."""
import os
import subprocess

import pytest

from conftest import ROOT
from paper_2407_20205_amd import perm3 as P

SRC = os.path.join(ROOT, "tests", "c_consumer.c")


def build(tmp_path) -> str:
    exe = str(tmp_path / "c_consumer")
    libdir = os.path.dirname(P.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    "-o", exe, SRC, "-L", libdir, "-lperm3", f"-Wl,-rpath,{libdir}"], check=True)
    return exe


def test_c_consumer_host_calls(tmp_path):
    r = subprocess.run([build(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "host ok"


@pytest.mark.gpu
def test_c_consumer_on_gpu(tmp_path):
    r = subprocess.run([build(tmp_path), "gpu"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.split() == ["host", "ok", "gpu", "ok"]
