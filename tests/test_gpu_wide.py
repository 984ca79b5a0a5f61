"""GPU parity for matrices of up to 128 columns (128-bit Gray indices) through the C ABI.

Bar: exact equality of the int64 tallies with the oracle, or with exact closed
forms built from oracle values.  The pins of the oracle's wide walk are in
test_oracle_wide.py.
"""
import math
import random
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from gpu_util import flush_print, host_threads, oracle_tallies, require_gpu
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def gray_inverse(x: int) -> int:
    i = 0
    while x:
        i ^= x
        x >>= 1
    return i


def cmod3(x: int) -> int:
    r = x % 3
    return -1 if r == 2 else r


def column_total_sign(D) -> int:
    d = 1
    for c in range(D.shape[1]):
        d *= cmod3(sum(-1 if int(x) == 2 else int(x) for x in D[:, c]))
    return d


def oracle_wide(A, ranges):
    with ThreadPoolExecutor(max_workers=host_threads()) as ex:
        return list(ex.map(lambda r: oracle.range_tally_wide(A, r[0], r[1]), ranges))


# ---------------------------------------------------------------- n <= 63: same sums as the narrow path

@pytest.mark.parametrize("n", [1, 2, 6, 7, 12, 16, 17, 20, 31, 32, 33, 36, 40, 63])
def test_wide_equals_narrow(n):
    g = W.rng(1000 + n)
    A = g.integers(0, 3, (n, n), dtype=np.uint8)
    total = 1 << n
    ranges = [(0, total)] if n <= 22 else [(0, 1 << 20)]
    ranges.append((total - min(total, 1 << 17), min(total, 1 << 17)))
    for _ in range(6):
        a = int(g.integers(0, total))
        ranges.append((a, min(int(g.integers(0, 1 << 19)), total - a)))
    flush_print(f"wide n={n}: {len(ranges)} ranges")
    want = oracle_tallies(A, [(a, a + c) for a, c in ranges])
    for (a, c), w in zip(ranges, want):
        assert P.perm_mod3_range_tally_wide(A, a, c) == w, (n, a, c)
        assert P.perm_mod3_range_tally(A, a, a + c) == w, (n, a, c)


# ---------------------------------------------------------------- n > 64 against the oracle

@pytest.mark.parametrize("n", [64, 65, 80, 96, 127, 128])
def test_wide_rank_one_ranges(n):
    """Two thirds of all terms are non-zero, so every block is re-walked and the
    words past the first are formed at almost every index."""
    A = W.rank_one_signs(n, 1100 + n)
    r = random.Random(1101 + n)
    L = 1 << 17
    total = 1 << n
    ranges = [(0, L), (total - L, L), ((1 << 63) - L // 3, L), (r.randrange(total - L), L + 13),
              (r.randrange(total - L) | 1, L - 7)]
    if n > 64:
        ranges.append(((1 << 64) - L // 2 - 5, L))
    flush_print(f"rank-one n={n}")
    want = oracle_wide(A, ranges)
    assert sum(w != 0 for w in want) >= len(want) // 2
    for (a, c), w in zip(ranges, want):
        assert P.perm_mod3_range_tally_wide(A, a, c) == w, (n, hex(a), c)


@pytest.mark.parametrize("n1,n2,pairs,shuffle", [(20, 108, 3, True), (24, 104, 2, False), (22, 77, 4, True),
                                                 (18, 47, 0, True), (26, 101, 3, True)])
def test_wide_block_closed_form(n1, n2, pairs, shuffle):
    A, M, D = W.wide_block(n1, n2, 1200 + n1 + n2, pairs=pairs, shuffle=shuffle)
    delta = column_total_sign(D)
    assert delta != 0
    h = gray_inverse((1 << n2) - 1)
    flush_print(f"block n1={n1} n2={n2}")
    T_M = oracle.range_tally(M, 0, 1 << n1, threads=host_threads())
    want = (-1) ** n2 * delta * T_M
    assert P.perm_mod3_range_tally_wide(A, h << n1, 1 << n1) == want
    # the same range in four pieces, cut off the chunk grid
    cuts = [0, (1 << n1) // 3 + 5, (1 << n1) // 2 + 1, (1 << n1) - 17, 1 << n1]
    parts = [P.perm_mod3_range_tally_wide(A, (h << n1) + cuts[k], cuts[k + 1] - cuts[k]) for k in range(4)]
    assert sum(parts) == want
    if pairs == 0:
        for hh in (h - 1, h + 1):
            assert P.perm_mod3_range_tally_wide(A, hh << n1, 1 << n1) == 0


# ---------------------------------------------------------------- the 128-column workload at full size

def test_wide_128_workload():
    """2^36 indices of the 128 x 128 workload, as the benchmark times them."""
    A, M, d, D = W.wide_128()
    delta = column_total_sign(D)
    begin = gray_inverse((1 << 92) - 1) << 36
    T = P.perm_mod3_range_tally_wide(A, begin, 1 << 36)
    # (-1)^n T = delta * perm(M) mod 3, and perm(M) is the product of M's hidden diagonal
    perm_M = math.prod(-1 if x == 2 else int(x) for x in d)
    assert (T - delta * perm_M) % 3 == 0
    # sixteen sampled pieces (aligned and not) against the oracle
    r = random.Random(7)
    pieces = [(begin + (k << 32) + (r.randrange(1 << 12) if k % 2 else 0), (1 << 18) + 3 * k) for k in range(16)]
    flush_print("oracle on 16 pieces of the 128-column workload")
    want = oracle_wide(A, pieces)
    for (a, c), w in zip(pieces, want):
        assert P.perm_mod3_range_tally_wide(A, a, c) == w, (hex(a), c)
    # four shards add up to the whole
    q = 1 << 34
    assert sum(P.perm_mod3_range_tally_wide(A, begin + k * q, q) for k in range(4)) == T


def test_wide_uniform_128_workload():
    """The uniform 128 x 128 matrix the benchmark times, 2^36 indices from 3 * 2^125: sampled pieces
    against the oracle, and shards that add up to the whole (T is 0 here: a non-zero term needs
    all 128 column sums non-zero, a (2/3)^128 event)."""
    U = W.uniform_matrix(128, W.SEED_WIDE)
    begin = 3 << 125
    T = P.perm_mod3_range_tally_wide(U, begin, 1 << 36)
    r = random.Random(11)
    pieces = [(begin + r.randrange(1 << 36), (1 << 17) + k) for k in range(8)]
    want = oracle_wide(U, pieces)
    for (a, c), w in zip(pieces, want):
        assert P.perm_mod3_range_tally_wide(U, a, c) == w, (hex(a), c)
    q = 1 << 33
    assert sum(P.perm_mod3_range_tally_wide(U, begin + k * q, q) for k in range(8)) == T


def test_wide_column_order_does_not_matter():
    """The library reorders columns for its filter; T is a product over all columns, so any
    permutation of the columns, and any range, gives the same tally."""
    A, M, D = W.wide_block(24, 90, 1400)
    h = gray_inverse((1 << 90) - 1)
    ref = P.perm_mod3_range_tally_wide(A, h << 24, 1 << 24)
    g = W.rng(1401)
    for _ in range(3):
        B = np.ascontiguousarray(A[:, g.permutation(114)])
        assert P.perm_mod3_range_tally_wide(B, h << 24, 1 << 24) == ref
    J = W.rank_one_signs(128, 1402)
    a = (1 << 127) + 999
    ref = P.perm_mod3_range_tally_wide(J, a, 1 << 15)
    assert ref == oracle.range_tally_wide(J, a, 1 << 15, threads=host_threads())
    assert P.perm_mod3_range_tally_wide(np.ascontiguousarray(J[:, ::-1]), a, 1 << 15) == ref


def test_wide_tuning_does_not_change_tallies():
    A = W.rank_one_signs(100, 1300)
    B, M, D = W.wide_block(20, 100, 1301)
    h = gray_inverse((1 << 100) - 1)
    a = (1 << 99) + 4321
    ref_a = P.perm_mod3_range_tally_wide(A, a, 1 << 16)
    ref_b = P.perm_mod3_range_tally_wide(B, h << 20, 1 << 20)
    with P.saved_tunings():
        for bl, cl, tpw, dm, wps in [(4, 8, 1, 10, 1), (6, 12, 4, 12, 2), (5, 24, 64, 40, 16), (4, 9, 2, 11, 4)]:
            t = P.tuning_get()
            t.body_log, t.chunk_log_max, t.tasks_per_wave, t.direct_max_n, t.waves_per_simd = bl, cl, tpw, dm, wps
            t.body_log_mid, t.mid_max_n = 4, 31
            P.tuning_set(t)
            assert P.perm_mod3_range_tally_wide(A, a, 1 << 16) == ref_a
            assert P.perm_mod3_range_tally_wide(B, h << 20, 1 << 20) == ref_b
    assert ref_a == oracle.range_tally_wide(A, a, 1 << 16, threads=host_threads())


def test_wide_argument_errors():
    A = W.uniform_matrix(10, 1)
    for args in [(A, (1 << 10) - 5, 6), (A, 0, (1 << 62) + 1)]:
        with pytest.raises(P.PermError) as e:
            P.perm_mod3_range_tally_wide(*args)
        assert e.value.code == P.PERM_EINVAL
    with pytest.raises(P.PermError) as e:
        P.perm_mod3_range_tally_wide(np.zeros((129, 129), np.uint8), 0, 1)
    assert e.value.code == P.PERM_EINVAL
    B = A.copy()
    B[3, 4] = 7
    with pytest.raises(P.PermError) as e:
        P.perm_mod3_range_tally_wide(B, 0, 1)
    assert e.value.code == P.PERM_EDOMAIN and e.value.index == 34
    assert P.perm_mod3_range_tally_wide(A, 5, 0) == 0
    # the top of the 128-bit index space
    J = W.rank_one_signs(128, 3)
    top = (1 << 128) - 1000
    assert P.perm_mod3_range_tally_wide(J, top, 1000) == oracle.range_tally_wide(J, top, 1000)
    with pytest.raises(P.PermError):
        P.perm_mod3_range_tally_wide(J, top, 1001)
