"""GPU parity for the serving loop: results equal the oracle, and each request's
result is the same alone as in a mix with others arriving while it runs."""
import time

import numpy as np
import pytest

from gpu_util import flush_print, oracle_perms, require_gpu
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def drain(srv, want_count, timeout_s=120.0):
    got = {}
    t0 = time.time()
    while len(got) < want_count:
        for d in srv.poll(1024, 20000):
            assert d.tag not in got
            got[d.tag] = d
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {want_count} finished"
    return got


_WANT = {}


def mixed_trace():
    tr = W.serve_trace(count=400, rate=1e9, seed=41, n_lo=0, n_hi=30)
    if "mixed" not in _WANT:
        flush_print("oracle on 400 requests, n in 0..30")
        _WANT["mixed"] = oracle_perms(tr.mats)
    return tr, _WANT["mixed"]


@pytest.mark.parametrize("fast_max_n", [0, -1, 18, 24])
@pytest.mark.parametrize("policy", [P.PERM_POLICY_SRPT, P.PERM_POLICY_FIFO])
def test_server_mixed_stream_vs_oracle(policy, fast_max_n):
    """With the fast lane at its default (its widest, n <= 28), off, and narrower."""
    tr, want = mixed_trace()
    with P.Server(max_slots=64, work_budget=1 << 33, quantum=1 << 30, policy=policy,
                  fast_max_n=fast_max_n) as srv:
        for k, M in enumerate(tr.mats):
            while not srv.submit(M, k):
                time.sleep(0.001)
        got = drain(srv, len(tr.mats))
        st = srv.stats()
    for k in range(len(tr.mats)):
        d = got[k]
        assert d.status == 0 and d.n == tr.ns[k]
        assert d.result == want[k], (k, int(tr.ns[k]))
        assert d.t_submit_ns <= d.t_admit_ns <= d.t_done_ns or tr.ns[k] == 0
    assert st.submitted == st.completed == len(tr.mats)


def test_server_alone_equals_in_mix():
    g = W.rng(42)
    big = g.integers(0, 3, (34, 34), dtype=np.uint8)
    smalls = [g.integers(0, 3, (n, n), dtype=np.uint8) for n in g.integers(8, 24, 60)]
    with P.Server(max_slots=16, quantum=1 << 31) as srv:
        assert srv.submit(big, 0)
        alone_big = drain(srv, 1)[0].result
        for k, M in enumerate(smalls):
            assert srv.submit(M, 1 + k)
        alone = drain(srv, len(smalls))
        # now the big one is in flight while the small ones arrive
        assert srv.submit(big, 1000)
        time.sleep(0.002)
        for k, M in enumerate(smalls):
            assert srv.submit(M, 2000 + k)
        mixed = drain(srv, 1 + len(smalls))
    assert mixed[1000].result == alone_big == P.perm_mod3(big)
    for k in range(len(smalls)):
        assert mixed[2000 + k].result == alone[1 + k].result
    want = oracle_perms(smalls)
    assert [alone[1 + k].result for k in range(len(smalls))] == want


def test_server_queue_full_and_errors():
    with P.Server(max_slots=1, queue_cap=2, quantum=1 << 20) as srv:
        A = W.uniform_matrix(30, 1)
        accepted = sum(1 for k in range(50) if srv.submit(A, k))
        assert 2 <= accepted < 50          # the queue pushes back instead of growing
        bad = A.copy()
        bad[0, 0] = 5
        with pytest.raises(P.PermError) as e:
            srv.submit(bad, 999)
        assert e.value.code == P.PERM_EDOMAIN
        got = drain(srv, accepted)
        r = P.perm_mod3(A)
        assert all(d.result == r for d in got.values())


def test_fast_lane_runs_beside_a_tick():
    """Small requests submitted while a 36x36 is being walked in ticks finish long before it,
    with results equal to the oracle's; the big one's result is unchanged."""
    g = W.rng(43)
    big = W.single_36()
    smalls = [g.integers(0, 3, (n, n), dtype=np.uint8) for n in g.integers(6, 19, 80)]
    want = oracle_perms(smalls)
    with P.Server(max_slots=8, quantum=1 << 30, fast_max_n=18) as srv:
        assert srv.submit(big, 0)
        time.sleep(0.002)                               # the ticks of the 36x36 are running
        for k, M in enumerate(smalls):
            assert srv.submit(M, 1 + k)
        got = drain(srv, 1 + len(smalls))
        st = srv.stats()
    assert got[0].result == P.perm_mod3(big)
    assert st.ticks > 1
    for k in range(len(smalls)):
        d = got[1 + k]
        assert d.status == 0 and d.result == want[k], k
        assert d.t_done_ns < got[0].t_done_ns, k         # not queued behind the big request


def test_server_config_errors():
    for bad in (-2, 29):
        with pytest.raises(P.PermError) as e:
            P.Server(max_slots=4, fast_max_n=bad)
        assert e.value.code == P.PERM_EINVAL
