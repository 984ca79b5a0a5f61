"""GPU parity for calls of up to 64 byte matrices (one launch plans, packs and, for at most 2^28
Gray indices in all, walks them), against the oracle.

Bar: exact equality.  The one-launch form keeps per-matrix accumulators that the wave completing a
matrix leaves at zero, so calls are repeated and interleaved with calls that take the longer path
(more work than one launch walks, a Gray range, packed planes) and each result is checked every time.
"""
import numpy as np
import pytest

import oracle
from gpu_util import flush_print, oracle_perms, require_gpu, to_dev
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu

ONE_LAUNCH_WORK = 1 << 28


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def run_dev(ns, mats, hist=False):
    """One device-input call; returns (results, histogram or None)."""
    import torch
    buf = np.concatenate([m.reshape(-1) for m in mats]) if mats else np.zeros(0, np.uint8)
    offs = np.zeros(len(mats), np.int64)
    offs[1:] = np.cumsum([m.size for m in mats[:-1]])
    out = torch.full((len(mats),), 0xEE, dtype=torch.uint8, device="cuda")
    h = torch.zeros(64 * 3, dtype=torch.int64, device="cuda") if hist else None
    P.perm_mod3_batch_dev(to_dev(buf, torch.uint8), to_dev(offs, torch.int64),
                          to_dev(np.asarray(ns, np.int32), torch.int32), out, h, None)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (h.cpu().numpy().reshape(64, 3) if hist else None)


def mixed(count, n_lo, n_hi, seed):
    g = W.rng(seed)
    ns = [int(n) for n in g.integers(n_lo, n_hi + 1, count)]
    return ns, [g.integers(0, 3, (n, n), dtype=np.uint8) for n in ns]


def test_repeated_and_interleaved_calls():
    cases = [mixed(1, 20, 20, 4000), mixed(3, 0, 12, 4001), mixed(64, 0, 18, 4002), mixed(17, 5, 21, 4003)]
    flush_print("oracle on", sum(len(c[0]) for c in cases), "matrices")
    wants = [np.array(oracle_perms(mats), np.uint8) for _, mats in cases]
    big_ns, big_mats = mixed(2, 28, 29, 4004)              # 2^28 + 2^29 indices: the longer path
    big_want = np.array(oracle_perms(big_mats), np.uint8)
    for rep in range(3):
        for (ns, mats), want in zip(cases, wants):
            got, _ = run_dev(ns, mats)
            assert np.array_equal(got, want), (rep, ns)
        if rep == 1:
            got, _ = run_dev(big_ns, big_mats)
            assert np.array_equal(got, big_want)
            A = cases[0][1][0]
            assert P.perm_mod3_range_tally(A, 5, 70000) == oracle.range_tally(A, 5, 70000)


def test_work_threshold_both_sides():
    """64 matrices of order 22 are exactly 2^28 indices (one launch); one of order 23 in their
    place goes over (plan and pack here, the walk in its own launch).  Host calls too."""
    g = W.rng(4010)
    mats = [g.integers(0, 3, (22, 22), dtype=np.uint8) for _ in range(64)]
    assert 64 * (1 << 22) == ONE_LAUNCH_WORK
    flush_print("oracle on 64 matrices of order 22 and one of order 23")
    want = np.array(oracle_perms(mats), np.uint8)
    over = list(mats)
    over[37] = g.integers(0, 3, (23, 23), dtype=np.uint8)
    want_over = want.copy()
    want_over[37] = oracle.perm_mod3(over[37])
    for ms, w in ((mats, want), (over, want_over), (mats, want)):
        got, _ = run_dev([m.shape[0] for m in ms], ms)
        assert np.array_equal(got, w)
        assert np.array_equal(P.perm_mod3_batch(ms), w)


def test_orders_zero_invalid_and_bad_entries_with_histogram():
    ns, mats = mixed(30, 0, 16, 4020)
    ns[4] = 0
    mats[4] = np.zeros((0, 0), np.uint8)
    want = np.array(oracle_perms(mats), np.uint8)
    mats[9] = mats[9].copy()
    mats[9][1, 2] = 7                                       # an entry outside {0, 1, 2}
    ns_in = list(ns)
    ns_in[13] = 64                                          # an order outside 0..63 (its bytes are ignored)
    got, hist = run_dev(ns_in, mats, hist=True)
    for k in range(len(ns)):
        if k in (9, 13):
            assert got[k] == P.PERM_RESULT_INVALID, k
        else:
            assert got[k] == want[k], k
    h = np.zeros((64, 3), np.int64)
    for k, (n, r) in enumerate(zip(ns, got)):
        if k not in (9, 13):
            h[n, r] += 1
    assert np.array_equal(hist, h)
    ok = [k for k in range(len(ns)) if k not in (9, 13)]   # later calls are unaffected
    got2, _ = run_dev([ns[k] for k in ok], [mats[k] for k in ok])
    assert np.array_equal(got2, want[ok])


@pytest.mark.parametrize("states", [1, 2, 4])
def test_states_per_lane(states):
    """The one-launch walk carries one chunk per lane whatever the tuning; the longer path (here a
    Gray range of a 26x26, planned by the same launch) follows the tuning."""
    ns, mats = mixed(8, 14, 26, 4030 + states)
    want = np.array(oracle_perms(mats), np.uint8)
    A = W.uniform_matrix(26, 4035)
    lo, hi = 12345, (1 << 25) + 777
    want_t = oracle.range_tally(A, lo, hi)
    base = P.tuning_get()
    try:
        t = P.tuning_get()
        t.states_per_lane = states
        P.tuning_set(t)
        for _ in range(2):
            got, _ = run_dev(ns, mats)
            assert np.array_equal(got, want)
            assert np.array_equal(P.perm_mod3_batch(mats), want)
            assert P.perm_mod3_range_tally(A, lo, hi) == want_t
    finally:
        P.tuning_set(base)


def test_launch_counts():
    A = W.single_20()
    P.timing_enable(True)
    try:
        assert P.perm_mod3(A) == oracle.perm_mod3(A)
        t = P.timing_last()
        assert t.launches == 1 and t.hot_kernel_ms > 0     # host call: plan, pack and walk in one launch
        got, _ = run_dev([20], [A])
        assert got[0] == oracle.perm_mod3(A)
        assert P.timing_last().launches == 2               # device input: k_walk follows, with no tasks
    finally:
        P.timing_enable(False)
