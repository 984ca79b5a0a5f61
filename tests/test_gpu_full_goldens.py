"""The standard workloads at full size against expected values the CPU oracle wrote
(tests/golden/make_full_goldens.py: Ryser's identity, eq. (2), walked in Gray-code order over
unpacked residues, Section 3), element by element, in the launch configuration the benchmark
times: the 36 x 36 matrix over all 2^36 Gray indices (its exact tally T and perm mod 3), every
one of the 8192 Monte Carlo matrices with the per-n histogram, and every request of the serving
trace with n <= 28 run through the server.  Each golden names the SHA-256 of its inputs, so a
change of generator shows up as a stale golden, not as a wrong result."""
import os

import numpy as np
import pytest

from conftest import GOLDEN
from gpu_util import flush_print, require_gpu, to_dev
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def read_kv(name):
    """A golden of 'key value' lines; repeated keys ('results', 'hist') are collected in lists."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition(" ")
            if key in ("results", "hist"):
                out.setdefault(key, []).append(val)
            else:
                out[key] = val
    return out


def test_single36_full_range():
    import torch
    g = read_kv("full_single36.txt")
    A = W.single_36()
    assert W.sha256(A) == g["input_sha256"], "the 36x36 input changed: rerun make_full_goldens.py"
    flush_print("36x36: perm_mod3_range_tally over [0, 2^36)")
    assert P.perm_mod3_range_tally(A, 0, 1 << 36) == int(g["tally"])
    # the benchmark's call: device input on the NULL stream
    mats = torch.from_numpy(A.reshape(-1).copy()).cuda()
    offs = torch.zeros(1, dtype=torch.int64, device="cuda")
    ns = torch.full((1,), 36, dtype=torch.int32, device="cuda")
    out = torch.full((1,), 0xEE, dtype=torch.uint8, device="cuda")
    for _ in range(2):
        P.perm_mod3_batch_dev(mats, offs, ns, out)
        torch.cuda.synchronize()
        assert int(out.item()) == int(g["perm_mod3"])
    assert P.perm_mod3(A) == int(g["perm_mod3"])


def test_batch8192_every_result_and_histogram():
    import torch
    g = read_kv("full_batch8192.txt")
    b = W.batch_uniform()
    assert W.sha256(b.ns, *b.mats) == g["input_sha256"], "the batch input changed: rerun make_full_goldens.py"
    want = np.array([int(c) for c in "".join(g["results"])], np.uint8)
    assert want.size == b.count == int(g["count"])
    want_hist = np.zeros((64, 3), np.int64)
    for row in g["hist"]:
        n, *h = (int(x) for x in row.split())
        want_hist[n] = h
    planes = np.concatenate([P.perm_mod3_pack(M) for M in b.mats]).view(np.int64)
    row_off = np.zeros(b.count, np.int64)
    row_off[1:] = np.cumsum(b.ns[:-1].astype(np.int64))
    planes_d, row_off_d, ns_d = to_dev(planes, torch.int64), to_dev(row_off, torch.int64), to_dev(b.ns, torch.int32)
    out = torch.zeros(b.count, dtype=torch.uint8, device="cuda")
    hist = torch.zeros(64 * 3, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    # as the benchmark runs it: the first call captures the library's graph, later calls replay it
    for rep in range(3):
        flush_print(f"8192-matrix batch, call {rep}")
        out.fill_(0xEE)
        hist.zero_()
        P.perm_mod3_batch_packed(planes_d, row_off_d, ns_d, out, hist, stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, f"{bad.size} results differ, first at matrix {bad[:5]} (n = {b.ns[bad[:5]]})"
        assert np.array_equal(hist.cpu().numpy().reshape(64, 3), want_hist)
    # the host-input batch call on the same matrices
    assert np.array_equal(P.perm_mod3_batch(b.mats), want)


def test_serving_trace_small_requests():
    g = read_kv("full_serve_le28.txt")
    count = int(g["count"])
    tr = W.serve_trace(count=count)
    assert W.sha256(tr.ns, *tr.mats) == g["input_sha256"], "the trace changed: rerun make_full_goldens.py"
    want = "".join(g["results"])
    n_max = int(g["n_max"])
    idx = [k for k in range(count) if tr.ns[k] <= n_max]
    assert len(idx) == int(g["checked"]) and all(want[k] != "-" for k in idx)
    # every request of the trace through the server, submitted as fast as it accepts them; the
    # larger ones (n > 28, slots and ticks) run beside them and are checked against single calls
    big = [k for k in range(count) if tr.ns[k] > n_max][:40]
    sub = sorted(idx + big)
    flush_print(f"serving {len(sub)} requests ({len(idx)} with n <= {n_max})")
    done = {}
    with P.Server(max_slots=4096, queue_cap=1 << 16, work_budget=1 << 40) as srv:
        for k in sub:
            while not srv.submit(tr.mats[k], k):
                for d in srv.poll(4096, 0):
                    done[int(d.tag)] = int(d.result)
        while len(done) < len(sub):
            for d in srv.poll(4096, 200000):
                done[int(d.tag)] = int(d.result)
    wrong = [k for k in idx if done[k] != int(want[k])]
    assert not wrong, f"{len(wrong)} of {len(idx)} results differ, first {wrong[:5]}"
    for k in big:
        assert done[k] == P.perm_mod3(tr.mats[k]), k
