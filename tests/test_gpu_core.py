"""GPU parity: single matrices and Gray ranges through the C ABI, against the oracle.

Bar: exact equality (integer results and exact int64 partial tallies)."""
import math

import numpy as np
import pytest

import oracle
from conftest import read_golden
from gpu_util import flush_print, oracle_tallies, require_gpu
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


# ---------------------------------------------------------------- Theorem 2.1 device functions

def psi(m, s):
    return 0 if not m else (2 if s else 1)


def bits(word, b):
    return (int(word) >> b) & 1


def test_bipedal_ops_all_16_cases():
    # case c = (m1, s1, m2, s2) as 4 bits, one case per bit position, twice over the word
    w = np.zeros((1, 4), np.uint32)
    for b in range(32):
        c = b & 15
        for k in range(4):
            w[0, k] |= ((c >> (3 - k)) & 1) << b
    out = P.bipedal_ops(w)[0]
    for b in range(32):
        m1, s1, m2, s2 = (bits(w[0, k], b) for k in range(4))
        a, c = psi(m1, s1), psi(m2, s2)
        assert psi(bits(out[0], b), bits(out[1], b)) == (a + c) % 3
        assert psi(bits(out[2], b), bits(out[3], b)) == (a - c) % 3
        assert psi(bits(out[4], b), bits(out[5], b)) == (a * c) % 3
        assert psi(bits(out[6], b), bits(out[7], b)) == (a - c) % 3


def test_bipedal_add_matches_table1_bits():
    rows = read_golden("table1_addition_truth.txt")
    w = np.zeros((len(rows), 4), np.uint32)
    for i, r in enumerate(rows):
        w[i] = [int(x) for x in r[1:5]]
    out = P.bipedal_ops(w)
    for i, r in enumerate(rows):
        assert [int(out[i, 0]), int(out[i, 1])] == [int(r[5]), int(r[6])], r
        lhs, rhs = r[0].split("=")
        a, c = (int(x) for x in lhs.split("+"))
        assert psi(int(out[i, 0]), int(out[i, 1])) == int(rhs) == (a + c) % 3


def test_bipedal_ops_random_words():
    g = W.rng(9)
    w = g.integers(0, 1 << 32, size=(256, 4), dtype=np.uint64).astype(np.uint32)
    out = P.bipedal_ops(w)
    for i in range(0, 256, 7):
        for b in range(0, 32, 3):
            m1, s1, m2, s2 = (bits(w[i, k], b) for k in range(4))
            a, c = psi(m1, s1), psi(m2, s2)
            assert psi(bits(out[i, 0], b), bits(out[i, 1], b)) == (a + c) % 3
            assert psi(bits(out[i, 6], b), bits(out[i, 7], b)) == (a - c) % 3


# ---------------------------------------------------------------- whole matrices vs oracle

@pytest.mark.parametrize("n", list(range(0, 9)))
def test_small_vs_brute_force(n):
    for s in range(6 if n else 1):
        A = W.uniform_matrix(n, 7000 + 13 * n + s) if n else np.zeros((0, 0), np.uint8)
        want = oracle.brute_perm_mod3(A) if n else 1
        assert P.perm_mod3(A) == want, (n, s)


def test_empty_matrix_range_tally():
    # the 0 x 0 matrix has one subset, the empty one, whose term is +1
    Z = np.zeros((0, 0), np.uint8)
    for a, b in [(0, 1), (0, 0), (1, 1)]:
        want = oracle.range_tally(Z, a, b)
        assert want == (1 if (a, b) == (0, 1) else 0)
        assert P.perm_mod3_range_tally(Z, a, b) == want, (a, b)


@pytest.mark.parametrize("n", [9, 11, 12, 13, 15, 16, 17, 18, 19, 20, 21, 22, 24, 25, 26])
def test_random_vs_oracle(n):
    for s in range(3):
        A = W.uniform_matrix(n, 8000 + 31 * n + s)
        flush_print(f"n={n} seed={s}")
        assert P.perm_mod3(A) == oracle.perm_mod3(A), (n, s)
        T = oracle.range_tally(A, 0, 1 << n, threads=8)
        assert P.perm_mod3_range_tally(A, 0, 1 << n) == T


def test_single_20x20_workload():
    A = W.single_20()
    T = oracle.range_tally(A, 0, 1 << 20, threads=8)
    assert P.perm_mod3_range_tally(A, 0, 1 << 20) == T
    assert P.perm_mod3(A) == oracle.perm_mod3(A)


def test_closed_forms_on_gpu():
    for n in [1, 2, 3, 5, 13, 18, 24, 30, 33, 36]:
        assert P.perm_mod3(np.eye(n, dtype=np.uint8)) == 1
        assert P.perm_mod3(2 * np.eye(n, dtype=np.uint8)) == pow(2, n, 3)
        if n <= 30:
            assert P.perm_mod3(np.ones((n, n), np.uint8)) == math.factorial(n) % 3
        # T(0, 2^n) of I_n is (-1)^n: one non-zero term, the full subset
        assert P.perm_mod3_range_tally(np.eye(n, dtype=np.uint8), 0, 1 << n) == (-1) ** n


def test_all_ones_tally_closed_form():
    # J_n: every column sum of a k-subset is k, so T(0,2^n) = sum_k C(n,k) (-1)^k c(k)^n
    for n in [14, 20, 26, 28]:
        J = np.ones((n, n), np.uint8)
        want = sum(math.comb(n, k) * (-1) ** k * (((k + 1) % 3) - 1) ** n for k in range(n + 1))
        assert P.perm_mod3_range_tally(J, 0, 1 << n) == want, n


# ---------------------------------------------------------------- Gray ranges vs oracle

@pytest.mark.parametrize("n", [17, 23, 31, 32, 33, 36, 40, 44, 50, 63])
def test_ranges_vs_oracle(n):
    g = W.rng(600 + n)
    A = g.integers(0, 3, (n, n), dtype=np.uint8)
    total = 1 << n
    ranges = [(0, min(total, 1 << 18)), (total - min(total, 1 << 17), total)]
    for _ in range(10):
        a = int(g.integers(0, total))
        ln = int(g.integers(1, 1 << 18))
        ranges.append((a, min(total, a + ln)))
    ranges.append((5, 5))
    want = oracle_tallies(A, ranges)
    for (a, b), w in zip(ranges, want):
        assert P.perm_mod3_range_tally(A, a, b) == w, (n, a, b)


def hit_heavy(n, seed):
    """Ones in the columns held by the low word (bits 0..31, columns n-32..n-1), so a k-subset
    passes the low test whenever 3 does not divide k; random -1s in the other columns."""
    g = W.rng(seed)
    A = np.ones((n, n), np.uint8)
    hi_cols = max(0, n - 32)
    A[:, :hi_cols][g.random((n, hi_cols)) < 0.3] = 2
    return A


@pytest.mark.parametrize("n", [30, 33, 36, 40])
def test_hit_heavy_ranges(n):
    A = hit_heavy(n, 700 + n)
    g = W.rng(701 + n)
    ranges = [(0, 1 << 20), (1 << (n - 1), (1 << (n - 1)) + (1 << 20))]
    for _ in range(4):
        a = int(g.integers(0, (1 << n) - (1 << 21)))
        ranges.append((a, a + int(g.integers(1, 1 << 21))))
    want = oracle_tallies(A, ranges)
    # the ranges are full of non-zero terms (their sums may still cancel)
    sample = [a + k for a, b in ranges for k in range(0, b - a, max(1, (b - a) // 200))]
    assert sum(oracle.term(A, i) != 0 for i in sample) > len(sample) // 100
    for (a, b), w in zip(ranges, want):
        assert P.perm_mod3_range_tally(A, a, b) == w, (n, a, b)


def test_range_additivity_on_gpu():
    A = W.uniform_matrix(30, 99)
    total = P.perm_mod3_range_tally(A, 0, 1 << 30)
    g = W.rng(3)
    cuts = sorted(int(x) for x in g.integers(0, 1 << 30, 7))
    pts = [0] + cuts + [1 << 30]
    assert sum(P.perm_mod3_range_tally(A, pts[k], pts[k + 1]) for k in range(len(pts) - 1)) == total


# ---------------------------------------------------------------- the 36 x 36 workload

def test_single_36x36_sampled_chunks():
    A = W.single_36()
    chunks = W.sample_chunks(36, seed=W.SEED_SINGLE_36, count=64, log_len=24, unaligned=8)
    assert len(chunks) == 64
    flush_print("oracle on 64 chunks of the 36x36 matrix")
    want = oracle_tallies(A, chunks)
    for (a, b), w in zip(chunks, want):
        assert P.perm_mod3_range_tally(A, a, b) == w, (a, b)


def test_single_36x36_full_consistency():
    A = W.single_36()
    T = P.perm_mod3_range_tally(A, 0, 1 << 36)
    r = P.perm_mod3(A)
    assert r == ((T if 36 % 2 == 0 else -T) % 3)
    # sixteen shards, as sixteen devices would split the range, add up to the whole
    shards = [(k << 32, (k + 1) << 32) for k in range(16)]
    assert sum(P.perm_mod3_range_tally(A, a, b) for a, b in shards) == T
    # an independent traversal: the transpose has the same permanent
    assert P.perm_mod3(np.ascontiguousarray(A.T)) == r
    # scaling a row by 2 (= -1) multiplies the permanent by 2
    B = A.copy()
    B[7] = (2 * B[7].astype(np.int64) % 3).astype(np.uint8)
    assert P.perm_mod3(B) == (2 * r) % 3


# ---------------------------------------------------------------- structured large matrices

@pytest.mark.parametrize("n", [37, 40])
def test_hidden_triangular(n):
    M, d = W.hidden_triangular(n, 900 + n)
    want = math.prod(-1 if x == 2 else int(x) for x in d) % 3
    assert P.perm_mod3(M) == want


def test_hidden_block_diagonal_40():
    M, blocks = W.hidden_block_diagonal([14, 13, 13], 77)
    want = 1
    for B in blocks:
        want = want * oracle.perm_mod3(B) % 3
    assert P.perm_mod3(M) == want


def test_laplace_expansion_34():
    # perm(A) = sum_j a_{0j} perm(M_0j): 34 minors of size 33 through the GPU, in one batch
    A = W.uniform_matrix(34, 55)
    minors = [np.ascontiguousarray(np.delete(A[1:], j, axis=1)) for j in range(34)]
    pm = P.perm_mod3_batch(minors)
    want = sum((-1 if A[0, j] == 2 else int(A[0, j])) * int(pm[j]) for j in range(34)) % 3
    assert P.perm_mod3(A) == want


def test_tuning_does_not_change_tallies():
    A = W.uniform_matrix(33, 5)
    ref = P.perm_mod3_range_tally(A, 0, 1 << 33)
    with P.saved_tunings():
        for wps, bl, cl, tpw, dm, st in [(1, 4, 8, 1, 10, 1), (2, 6, 12, 4, 12, 2), (16, 5, 24, 64, 40, 4),
                                         (8, 4, 20, 8, 33, 2), (4, 5, 9, 2, 11, 4), (8, 6, 16, 16, 12, 1)]:
            t = P.perm_tuning()
            t.waves_per_simd, t.body_log, t.chunk_log_max, t.tasks_per_wave, t.direct_max_n = wps, bl, cl, tpw, dm
            t.states_per_lane = st
            t.body_log_mid, t.mid_max_n = (min(6, dm - 6), 40) if bl == 4 else (4, 20)
            P.tuning_set(t)
            assert P.perm_mod3_range_tally(A, 0, 1 << 33) == ref, (wps, bl, cl, tpw, dm, st)
            assert P.perm_mod3_range_tally(A, 12345, 1 << 22) == oracle.range_tally(A, 12345, 1 << 22)


def test_autotune_keeps_results():
    A = W.uniform_matrix(30, 123)
    ref = P.perm_mod3_range_tally(A, 0, 1 << 30)
    with P.saved_tunings():
        best = P.autotune(30, budget_ms=1500)
        now, src = P.tuning_get_class(P.PERM_TUNE_MID)     # n = 30: the class of 25..31
        assert best.as_dict() == now.as_dict()            # the winner becomes the class's tuning
        assert src == P.PERM_TUNE_SRC_AUTOTUNE
        assert 1 <= best.waves_per_simd <= 16 and best.body_log_mid in (4, 5, 6)
        assert P.perm_mod3_range_tally(A, 0, 1 << 30) == ref
        assert P.perm_mod3(A) == oracle.perm_mod3(A)


def test_from_tallies_finishes_shards():
    from paper_2407_20205_amd import longrun
    A = W.uniform_matrix(28, 91)
    shards = [P.perm_mod3_range_tally(A, *longrun.shard_bounds(28, 7, k)) for k in range(7)]
    assert P.perm_mod3_from_tallies(28, shards) == oracle.perm_mod3(A)
    # (-1)^n times the sum, mod 3, for arbitrary tallies and both parities of n
    g = W.rng(92)
    for n in (0, 1, 2, 33, 62, 63):
        for size in (1, 63, 64, 65, 1000):
            ts = g.integers(-(1 << 40), 1 << 40, size=size)
            assert P.perm_mod3_from_tallies(n, ts) == oracle.perm_from_tally(n, int(ts.sum())), (n, size)
    for bad in [(64, [1]), (-1, [1]), (5, [])]:
        with pytest.raises(P.PermError) as e:
            P.perm_mod3_from_tallies(*bad)
        assert e.value.code == P.PERM_EINVAL
