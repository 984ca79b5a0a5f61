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


def run_packed(ns, planes):
    """One call on caller-packed planes (uint64 words, mag then sgn per row); returns the results."""
    import torch
    row_off = np.zeros(len(ns), np.int64)
    row_off[1:] = np.cumsum(np.asarray(ns[:-1], np.int64))
    out = torch.full((len(ns),), 0xEE, dtype=torch.uint8, device="cuda")
    P.perm_mod3_batch_packed(to_dev(planes.view(np.int64), torch.int64), to_dev(row_off, torch.int64),
                             to_dev(np.asarray(ns, np.int32), torch.int32), out, None, None)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_packed_planes_one_launch_and_longer_path():
    """Caller-packed planes take the same two paths: packed into each wave's LDS and walked in the
    same launch, or (over 2^28 indices) packed into the work buffers for k_walk.  (0,1) zeros are
    accepted (Definition 2.1); a bit at or above n makes the matrix invalid."""
    ns, mats = mixed(20, 0, 20, 4040)
    want = np.array(oracle_perms(mats), np.uint8)
    flat = np.concatenate([P.perm_mod3_pack(M) for M in mats]).astype(np.uint64)
    g = W.rng(4041)
    r0 = 0
    for k, n in enumerate(ns):
        if k == 3 and n:
            for r in range(n):                            # sgn set where mag is clear: still zeros
                mag = int(flat[2 * (r0 + r)])
                flat[2 * (r0 + r) + 1] |= np.uint64(int(g.integers(0, 1 << n)) & ~mag)
        r0 += n
    bad = flat.copy()
    k7 = 7 if ns[7] else 8
    row7 = int(np.sum(ns[:k7]))
    bad[2 * row7] |= np.uint64(1) << np.uint64(ns[k7])      # a mag bit at column n
    big_ns, big_mats = mixed(2, 28, 29, 4004)
    big_want = np.array(oracle_perms(big_mats), np.uint8)
    big_flat = np.concatenate([P.perm_mod3_pack(M) for M in big_mats]).astype(np.uint64)
    for _ in range(2):
        assert np.array_equal(run_packed(ns, flat), want)
        got = run_packed(ns, bad)
        for k in range(len(ns)):
            assert got[k] == (P.PERM_RESULT_INVALID if k == k7 else want[k]), k
        assert np.array_equal(run_packed(big_ns, big_flat), big_want)


@pytest.mark.parametrize("states", [1, 2, 4])
def test_states_per_lane(states):
    """The one-launch walk carries one chunk per lane whatever the tuning; the longer path (here a
    Gray range of a 26x26, planned by the same launch) follows the tuning."""
    ns, mats = mixed(8, 14, 26, 4030 + states)
    want = np.array(oracle_perms(mats), np.uint8)
    A = W.uniform_matrix(26, 4035)
    lo, hi = 12345, (1 << 25) + 777
    want_t = oracle.range_tally(A, lo, hi)
    with P.saved_tunings():
        t = P.tuning_get()
        t.states_per_lane = states
        P.tuning_set(t)
        for _ in range(2):
            got, _ = run_dev(ns, mats)
            assert np.array_equal(got, want)
            assert np.array_equal(P.perm_mod3_batch(mats), want)
            assert P.perm_mod3_range_tally(A, lo, hi) == want_t


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
        run_packed([20], P.perm_mod3_pack(A).astype(np.uint64))
        assert P.timing_last().launches == 2               # caller-packed planes: the same two launches
    finally:
        P.timing_enable(False)
