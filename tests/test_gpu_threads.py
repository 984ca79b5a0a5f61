"""Calls from several host threads at once (the C ABI promises thread safety, with the calls into
one device context serialised): every result equals the oracle's, while a server runs beside them.

Bar: exact equality."""
import threading
import time

import numpy as np
import pytest

import oracle
from gpu_util import flush_print, require_gpu
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def test_concurrent_calls_and_server():
    g = W.rng(2000)
    mats = [g.integers(0, 3, (n, n), dtype=np.uint8) for n in g.integers(10, 25, 48)]
    flush_print("oracle on 48 matrices, n in 10..24")
    want = [oracle.perm_mod3(M) for M in mats]
    ranges = [(int(g.integers(0, (1 << 24) - 5000)), 5000 + int(g.integers(0, 30000))) for _ in range(16)]
    big = W.uniform_matrix(24, 2001)
    want_tallies = [oracle.range_tally(big, a, a + c) for a, c in ranges]
    wide = W.rank_one_signs(100, 2002)
    wide_begin = (1 << 99) + 12345
    want_wide = oracle.range_tally_wide(wide, wide_begin, 1 << 15, threads=8)
    errors = []

    def singles(tid):
        try:
            for r in range(3):
                for k in range(tid, len(mats), 4):
                    got = P.perm_mod3(mats[k])
                    if got != want[k]:
                        errors.append(("single", tid, k, got, want[k]))
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(("single-exc", tid, repr(e)))

    def tallies(tid):
        try:
            for j in range(tid, len(ranges), 2):
                a, c = ranges[j]
                got = P.perm_mod3_range_tally(big, a, a + c)
                if got != want_tallies[j]:
                    errors.append(("tally", tid, j, got, want_tallies[j]))
                if P.perm_mod3_range_tally_wide(wide, wide_begin, 1 << 15) != want_wide:
                    errors.append(("wide", tid, j))
        except Exception as e:  # noqa: BLE001
            errors.append(("tally-exc", tid, repr(e)))

    def batches(tid):
        try:
            for r in range(4):
                got = P.perm_mod3_batch(mats[tid::3])
                if list(got) != want[tid::3]:
                    errors.append(("batch", tid, r))
        except Exception as e:  # noqa: BLE001
            errors.append(("batch-exc", tid, repr(e)))

    with P.Server(max_slots=32, work_budget=1 << 30, quantum=1 << 28) as srv:
        for k, M in enumerate(mats):
            while not srv.submit(M, k):
                time.sleep(0.001)
        threads = [threading.Thread(target=singles, args=(t,)) for t in range(4)]
        threads += [threading.Thread(target=tallies, args=(t,)) for t in range(2)]
        threads += [threading.Thread(target=batches, args=(t,)) for t in range(3)]
        for t in threads:
            t.start()
        got = {}
        t0 = time.time()
        while len(got) < len(mats) and time.time() - t0 < 120:
            for d in srv.poll(256, 20000):
                got[d.tag] = d
        for t in threads:
            t.join(timeout=240)
        assert not any(t.is_alive() for t in threads), "a worker thread did not finish"
    assert not errors, errors[:5]
    assert len(got) == len(mats)
    for k, d in got.items():
        assert d.status == 0 and d.result == want[k], k
