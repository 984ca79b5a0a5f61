"""C-ABI checks that need no GPU: the library loads, exports every function
include/perm3.h declares, and the host-side parts (argument checks, the phi
packer of Section 2) behave as documented."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT, read_golden
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

HEADER = os.path.join(ROOT, "include", "perm3.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(perm_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["perm_mod3", "perm_mod3_batch", "perm_mod3_batch_packed", "perm_mod3_range_tally",
                 "perm_mod3_pack", "perm_server_create", "perm_server_submit", "perm_server_poll",
                 "perm_server_destroy", "perm_strerror", "perm_last_error_index"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = P.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert {n for n, _, _ in P.EXPORTS} == set(declared_functions())


def test_library_is_built_for_gfx950_only(tmp_path):
    import shutil
    import subprocess
    bundler = "/opt/rocm/llvm/bin/clang-offload-bundler"
    if not (shutil.which("objcopy") and os.path.exists(bundler)):
        pytest.skip("objcopy or clang-offload-bundler unavailable")
    fat = tmp_path / "fatbin.bin"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", P.LIB_PATH, str(fat)], check=True)
    out = subprocess.run([bundler, "--list", "--type=o", f"--input={fat}"], capture_output=True, text=True,
                         check=True)
    targets = [t for t in out.stdout.split() if "amdgcn" in t]
    assert targets and all(t.endswith("gfx950") for t in targets)


def test_version_and_strerror():
    assert "gfx950" in P.version()
    assert P.strerror(P.PERM_OK) == "ok"
    for code in (P.PERM_EINVAL, P.PERM_EDOMAIN, P.PERM_ENOMEM, P.PERM_EDEVICE, P.PERM_EAGAIN, P.PERM_ESTATE):
        assert P.strerror(code) not in ("ok", "unknown status")
    assert P.strerror(12345) == "unknown status"


# ---------------------------------------------------------------- phi packer (host)

def test_pack_worked_example():
    row = read_golden("phi_worked_example.txt")[0]
    vec = [int(x) for x in row[0].split(",")]
    mag, sgn, alt = int(row[1], 16), int(row[2], 16), int(row[3], 16)
    # a 4x4 matrix whose first row is the example
    A = np.zeros((4, 4), np.uint8)
    A[0] = vec
    planes = P.perm_mod3_pack(A)
    assert int(planes[0]) == mag and int(planes[1]) == sgn
    # psi reads the alternative sgn word as the same vector
    for s in (sgn, alt):
        back = []
        for i in range(1, 5):                          # element i at bit n - i
            b = 4 - i
            back.append(0 if not (mag >> b) & 1 else (2 if (s >> b) & 1 else 1))
        assert back == vec


def test_pack_random_roundtrip():
    for n in (1, 5, 31, 32, 33, 63):
        A = W.uniform_matrix(n, 40 + n)
        planes = P.perm_mod3_pack(A)
        assert planes.shape == (2 * n,)
        for r in range(n):
            mag, sgn = int(planes[2 * r]), int(planes[2 * r + 1])
            assert mag >> n == 0 and sgn >> n == 0
            assert sgn & ~mag == 0                    # phi never emits the (0,1) zero
            for j in range(n):
                b = n - 1 - j
                v = 0 if not (mag >> b) & 1 else (2 if (sgn >> b) & 1 else 1)
                assert v == A[r, j]


def test_pack_rejects_bad_entries():
    A = W.uniform_matrix(6, 1)
    A[2, 3] = 7
    with pytest.raises(P.PermError) as e:
        P.perm_mod3_pack(A)
    assert e.value.code == P.PERM_EDOMAIN and e.value.index == 2 * 6 + 3


# ---------------------------------------------------------------- argument checks before any device work

def test_argument_errors_need_no_device():
    bad = W.uniform_matrix(5, 2)
    bad[4, 4] = 3
    with pytest.raises(P.PermError) as e:
        P.perm_mod3(bad)
    assert e.value.code == P.PERM_EDOMAIN and e.value.index == 24
    with pytest.raises(P.PermError) as e:
        P.perm_mod3_range_tally(W.uniform_matrix(5, 3), 3, 2)
    assert e.value.code == P.PERM_EINVAL
    with pytest.raises(P.PermError) as e:
        P.perm_mod3_range_tally(W.uniform_matrix(5, 3), 0, 33)
    assert e.value.code == P.PERM_EINVAL
    with pytest.raises(P.PermError) as e:
        P.perm_mod3_batch([W.uniform_matrix(3, 1), bad])
    assert e.value.code == P.PERM_EDOMAIN and e.value.index == 1
    big = np.zeros((64, 64), np.uint8)
    with pytest.raises(P.PermError) as e:
        P.perm_mod3(big)
    assert e.value.code == P.PERM_EINVAL
    L = P.lib()
    assert L.perm_mod3(None, 3, None) == P.PERM_EINVAL
    assert L.perm_mod3_batch_dev(None, None, None, -1, None, None, None) == P.PERM_EINVAL
    assert L.perm_mod3_batch_dev(None, None, None, 0, None, None, None) == P.PERM_OK
    # counts: 0 is an empty call, PERM_MAX_BATCH + 1 (the allocation-free call: its own limit + 1)
    # is refused before any pointer is looked at
    over = P.PERM_MAX_BATCH + 1
    for fn in (L.perm_mod3_batch_dev, L.perm_mod3_batch_packed):
        assert fn(None, None, None, over, None, None, None) == P.PERM_EINVAL
        assert fn(None, None, None, 0, None, None, None) == P.PERM_OK
    assert L.perm_mod3_batch_packed_noalloc(None, None, None, P.PERM_NOALLOC_MAX_COUNT + 1, None, None,
                                            None) == P.PERM_EINVAL
    assert L.perm_mod3_batch_packed_noalloc(None, None, None, 0, None, None, None) == P.PERM_OK
    assert L.perm_mod3_batch(None, None, over, None) == P.PERM_EINVAL
    assert L.perm_mod3_batch(None, None, 0, None) == P.PERM_OK
    assert P.perm_mod3_batch([]).shape == (0,)


def test_compute_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.PermError) as e:
        P.perm_mod3(W.uniform_matrix(4, 1))
    assert e.value.code == P.PERM_EDEVICE
