"""The autotuner and the tuning cache through the C ABI: per-class tunings found by timing on the
device, written to a cache file, read back, and every result unchanged against the oracle.  The
block decomposition of Section 3.1 is free: no tuning may change T(a, b) or perm mod 3."""
import os

import numpy as np
import pytest

import oracle
from gpu_util import flush_print, oracle_perms, require_gpu, to_dev
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def packed(b):
    import torch
    planes = np.concatenate([P.perm_mod3_pack(M) for M in b.mats]).view(np.int64)
    row_off = np.zeros(b.count, np.int64)
    row_off[1:] = np.cumsum(b.ns[:-1].astype(np.int64))
    return to_dev(planes, torch.int64), to_dev(row_off, torch.int64), to_dev(b.ns, torch.int32)


def all_classes():
    return [P.tuning_get_class(k) for k in range(P.PERM_TUNE_CLASSES)]


def check_results(b, want_b, singles):
    import torch
    planes, row_off, ns = packed(b)
    out = torch.zeros(b.count, dtype=torch.uint8, device="cuda")
    P.perm_mod3_batch_packed(planes, row_off, ns, out, None, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want_b)
    for A, want in singles:
        assert P.perm_mod3(A) == want, A.shape


def test_classes_start_at_defaults_or_cache():
    # every earlier test puts the tunings back as a new context makes them
    for t, src in all_classes():
        assert src in (P.PERM_TUNE_SRC_DEFAULT, P.PERM_TUNE_SRC_CACHE)
        assert 1 <= t.waves_per_simd <= 16
    with P.saved_tunings():
        P.tuning_set(P.tuning_get())
        assert all(src == P.PERM_TUNE_SRC_SET for _, src in all_classes())
    assert all(src in (P.PERM_TUNE_SRC_DEFAULT, P.PERM_TUNE_SRC_CACHE) for _, src in all_classes())


def test_set_class_is_per_class():
    with P.saved_tunings():
        P.tuning_reset()
        t, _ = P.tuning_get_class(P.PERM_TUNE_BATCH)
        t.tasks_per_wave = 7
        P.tuning_set_class(P.PERM_TUNE_BATCH, t)
        got = all_classes()
        assert got[P.PERM_TUNE_BATCH][0].tasks_per_wave == 7
        assert got[P.PERM_TUNE_BATCH][1] == P.PERM_TUNE_SRC_SET
        for k in (P.PERM_TUNE_SMALL, P.PERM_TUNE_MID, P.PERM_TUNE_LARGE):
            assert got[k][1] == P.PERM_TUNE_SRC_DEFAULT and got[k][0].tasks_per_wave != 7
        bad = P.perm_tuning()
        with pytest.raises(P.PermError) as e:
            P.tuning_set_class(P.PERM_TUNE_BATCH, bad)          # all zeros: out of range
        assert e.value.code == P.PERM_EINVAL
        with pytest.raises(P.PermError):
            P.tuning_set_class(P.PERM_TUNE_CLASSES, t)


def test_autotune_every_class_cache_round_trip(tmp_path):
    import torch
    b = W.batch_uniform(count=400, n_lo=12, n_hi=24, seed=7101)
    flush_print("oracle on 400 matrices, n in 12..24, and one matrix per class")
    want_b = np.array(oracle_perms(b.mats), np.uint8)
    singles = []
    for n, seed in ((20, 7102), (29, 7103), (33, 7104)):
        A = W.uniform_matrix(n, seed)
        singles.append((A, oracle.perm_mod3(A)))
    path = str(tmp_path / "perm3_tuning.txt")
    # a line of another device and a comment, which a save must keep
    foreign = "gfx942:sramecc+:xnack- 304 large waves_per_simd=3 body_log=5"
    with open(path, "w") as f:
        f.write("# kept\n" + foreign + "\n")
    with P.saved_tunings():
        P.tuning_reset()
        tuned = {}
        for n in (20, 29, 34):
            flush_print(f"autotune n = {n}")
            tuned[n] = P.autotune(n, budget_ms=2500)
        planes, row_off, ns = packed(b)
        out = torch.zeros(b.count, dtype=torch.uint8, device="cuda")
        flush_print("autotune batch")
        tb = P.autotune_batch(planes, row_off, ns, out, budget_ms=4000)
        assert np.array_equal(out.cpu().numpy(), want_b)   # the tuner's own last run
        now = all_classes()
        for k, n in ((P.PERM_TUNE_SMALL, 20), (P.PERM_TUNE_MID, 29), (P.PERM_TUNE_LARGE, 34)):
            assert now[k][1] == P.PERM_TUNE_SRC_AUTOTUNE
            assert now[k][0].as_dict() == tuned[n].as_dict()
        assert now[P.PERM_TUNE_BATCH][0].as_dict() == tb.as_dict()
        check_results(b, want_b, singles)

        P.tuning_cache_save(path)
        with open(path) as f:
            lines = f.read().splitlines()
        assert "# kept" in lines and foreign in lines
        arch = P.device_info().arch.decode()
        mine = [line for line in lines if line.startswith(arch + " ")]
        assert sorted(line.split()[2] for line in mine) == ["batch", "large", "mid", "small"]

        P.tuning_reset()
        assert all(src == P.PERM_TUNE_SRC_DEFAULT for _, src in all_classes())
        assert P.tuning_cache_load(path) == 4
        back = all_classes()
        for k in range(P.PERM_TUNE_CLASSES):
            assert back[k][1] == P.PERM_TUNE_SRC_CACHE
            assert back[k][0].as_dict() == now[k][0].as_dict()
        check_results(b, want_b, singles)

        # saving again rewrites this device's lines in place of the old ones
        P.tuning_cache_save(path)
        with open(path) as f:
            again = f.read().splitlines()
        assert sorted(again) == sorted(lines)


def test_cache_skips_bad_lines(tmp_path):
    arch = P.device_info().arch.decode()
    cus = P.device_info().compute_units
    path = str(tmp_path / "c.txt")
    with open(path, "w") as f:
        f.write(f"{arch} {cus} mid waves_per_simd=99\n")            # out of range: skipped
        f.write(f"{arch} {cus} nosuchclass waves_per_simd=4\n")     # unknown class: skipped
        f.write(f"{arch} {cus + 1} large waves_per_simd=4\n")       # another CU count: skipped
        f.write(f"{arch} {cus} small waves_per_simd=4 bogus=1 tasks_per_wave=x\n")   # unknown key, bad value
    with P.saved_tunings():
        P.tuning_reset()
        assert P.tuning_cache_load(path) == 1
        t, src = P.tuning_get_class(P.PERM_TUNE_SMALL)
        assert src == P.PERM_TUNE_SRC_CACHE and t.waves_per_simd == 4
        for k in (P.PERM_TUNE_MID, P.PERM_TUNE_LARGE, P.PERM_TUNE_BATCH):
            assert P.tuning_get_class(k)[1] == P.PERM_TUNE_SRC_DEFAULT
        A = W.uniform_matrix(22, 7105)
        assert P.perm_mod3(A) == oracle.perm_mod3(A)
    with pytest.raises(P.PermError) as e:
        P.tuning_cache_load(os.path.join(str(tmp_path), "missing.txt"))
    assert e.value.code == P.PERM_EINVAL
