"""Pins for the CPU oracle against things fixed by the paper and by mathematics.

The oracle (Ryser + Gray code on unpacked residues) is checked against:
  * brute force eq. (1) over all permutations, itself pinned to closed forms;
  * Table 3's exact zero counts z(1..4) (and the 1 <-> -1 symmetry of Section 4);
  * the direct per-term definition of a Ryser term (no Gray walk);
  * invariants of the permanent (transpose, row/column permutations, scaling
    a row by 2, identity, all-ones, diagonal, zero row).
"""
import math

import numpy as np
import pytest

from conftest import read_golden
from paper_2407_20205_amd import workloads as W


def rand_mat(n, seed):
    return W.uniform_matrix(n, 1000 + 17 * n + seed)


# ---------------------------------------------------------------- brute force

def _signed_to_u8(M):
    return np.array([[2 if x == -1 else x for x in row] for row in M], dtype=np.uint8)


def test_brute_force_closed_forms(oracle_mod):
    for n in range(1, 8):
        J = np.ones((n, n), np.uint8)
        assert oracle_mod.brute_perm(J) == math.factorial(n)          # perm(J_n) = n!
        assert oracle_mod.brute_perm(np.eye(n, dtype=np.uint8)) == 1  # perm(I) = 1
        assert oracle_mod.brute_perm(np.zeros((n, n), np.uint8)) == 0
        # all -1: every product is (-1)^n
        assert oracle_mod.brute_perm(np.full((n, n), 2, np.uint8)) == (-1) ** n * math.factorial(n)
    # 2x2: ad + bc with a sign that a determinant would not have
    assert oracle_mod.brute_perm(_signed_to_u8([[1, 1], [-1, 1]])) == 0
    assert oracle_mod.brute_perm(_signed_to_u8([[1, -1], [1, 1]])) == 0
    assert oracle_mod.brute_perm(_signed_to_u8([[1, 1], [1, 1]])) == 2
    assert oracle_mod.brute_perm(_signed_to_u8([[0, 1], [1, 0]])) == 1
    # upper triangular: product of the diagonal
    g = W.rng(7)
    for n in range(1, 7):
        U = np.triu(g.integers(0, 3, (n, n), dtype=np.uint8))
        d = [(-1 if x == 2 else int(x)) for x in np.diag(U)]
        assert oracle_mod.brute_perm(U) == math.prod(d)


def test_brute_force_3x3_expansion(oracle_mod):
    # a 3x3 permanent expanded by hand along the first row
    g = W.rng(11)
    for _ in range(20):
        A = g.integers(0, 3, (3, 3), dtype=np.uint8)
        a = [[-1 if x == 2 else int(x) for x in r] for r in A]
        expect = (a[0][0] * (a[1][1] * a[2][2] + a[1][2] * a[2][1])
                  + a[0][1] * (a[1][0] * a[2][2] + a[1][2] * a[2][0])
                  + a[0][2] * (a[1][0] * a[2][1] + a[1][1] * a[2][0]))
        assert oracle_mod.brute_perm(A) == expect


# --------------------------------------------------------- oracle vs eq. (1)

@pytest.mark.parametrize("n", list(range(0, 9)))
def test_oracle_matches_brute_force(oracle_mod, n):
    trials = {0: 1, 1: 30, 2: 60, 3: 60, 4: 60, 5: 40, 6: 25, 7: 12, 8: 4}[n]
    for s in range(trials):
        A = rand_mat(n, s) if n else np.zeros((0, 0), np.uint8)
        expect = oracle_mod.brute_perm_mod3(A) if n else 1
        assert oracle_mod.perm_mod3(A, threads=1) == expect, (n, s)
    # structured: all -1, identity, all ones
    if n:
        for A in (np.full((n, n), 2, np.uint8), np.eye(n, dtype=np.uint8), np.ones((n, n), np.uint8)):
            assert oracle_mod.perm_mod3(A, threads=1) == oracle_mod.brute_perm_mod3(A)


def test_oracle_sparse_brute_force(oracle_mod):
    g = W.rng(21)
    for n in range(1, 8):
        for _ in range(10):
            A = W.sparse_matrix(n, g)
            assert oracle_mod.perm_mod3(A, threads=1) == oracle_mod.brute_perm_mod3(A)


# ------------------------------------------------------------ Table 3 pins

def test_table3_zero_counts_small(oracle_mod):
    z = {int(r[0]): int(r[1]) for r in read_golden("table3_zero_counts.txt")}
    for n in (1, 2, 3):
        c0, c1, c2 = oracle_mod.count_by_value(n)
        assert c0 == z[n]
        assert c0 + c1 + c2 == 3 ** (n * n)
        assert c1 == c2          # negating the first row swaps perm = 1 and perm = -1


@pytest.mark.slow
def test_table3_zero_count_n4(oracle_mod):
    z = {int(r[0]): int(r[1]) for r in read_golden("table3_zero_counts.txt")}
    c0, c1, c2 = oracle_mod.count_by_value(4)
    assert c0 == z[4] == 17116353
    assert c1 == c2 and c0 + c1 + c2 == 3 ** 16


# ------------------------------------------- Gray walk vs per-term definition

@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7])
def test_gray_walk_equals_direct_terms(oracle_mod, n):
    A = rand_mat(n, 3)
    terms = [oracle_mod.term(A, i) for i in range(1 << n)]
    for i in range(1 << n):
        assert oracle_mod.range_tally(A, i, i + 1) == terms[i], i
    g = W.rng(n)
    for _ in range(30):
        a, b = sorted(int(x) for x in g.integers(0, (1 << n) + 1, 2))
        assert oracle_mod.range_tally(A, a, b) == sum(terms[a:b])
    assert terms[0] == (1 if n == 0 else 0)      # empty subset: zero vector


def test_term_definition_small_case(oracle_mod):
    # 2x2, rows r0 = (1, -1), r1 = (1, 1).  Gray states 0, {0}, {0,1}, {1}.
    A = _signed_to_u8([[1, -1], [1, 1]])
    # S={0}: sums (1,-1) -> product -1, |S| = 1 -> +1
    # S={0,1}: sums (2,0) -> 0
    # S={1}: sums (1,1) -> 1, |S| = 1 -> -1
    assert [oracle_mod.term(A, i) for i in range(4)] == [0, 1, 0, -1]
    assert oracle_mod.range_tally(A, 0, 4) == 0
    assert oracle_mod.perm_mod3(A) == 0


def test_range_additivity_and_threads(oracle_mod):
    A = rand_mat(16, 0)
    full = oracle_mod.range_tally(A, 0, 1 << 16)
    g = W.rng(5)
    for _ in range(10):
        cuts = sorted(int(x) for x in g.integers(0, (1 << 16) + 1, 3))
        pts = [0] + cuts + [1 << 16]
        assert sum(oracle_mod.range_tally(A, pts[k], pts[k + 1]) for k in range(4)) == full
    assert oracle_mod.range_tally(A, 0, 1 << 16, threads=4) == full
    # |T| is at most the number of nonzero terms
    assert abs(full) <= 1 << 16


def test_range_edges(oracle_mod):
    A = rand_mat(10, 1)
    assert oracle_mod.range_tally(A, 0, 0) == 0
    assert oracle_mod.range_tally(A, 1024, 1024) == 0
    with pytest.raises(ValueError):
        oracle_mod.range_tally(A, 5, 4)
    with pytest.raises(ValueError):
        oracle_mod.range_tally(A, 0, 1025)
    bad = A.copy()
    bad[3, 4] = 3
    with pytest.raises(ValueError):
        oracle_mod.perm_mod3(bad)


# ------------------------------------------------------------- invariants

def _perm3(o, A):
    return o.perm_mod3(np.ascontiguousarray(A, dtype=np.uint8), threads=4)


@pytest.mark.parametrize("n", [9, 11, 13, 14])
def test_invariants(oracle_mod, n):
    g = W.rng(100 + n)
    A = g.integers(0, 3, (n, n), dtype=np.uint8)
    p = _perm3(oracle_mod, A)
    assert _perm3(oracle_mod, A.T) == p
    assert _perm3(oracle_mod, A[g.permutation(n)]) == p
    assert _perm3(oracle_mod, A[:, g.permutation(n)]) == p
    r = int(g.integers(0, n))
    B = A.copy()
    B[r] = (2 * B[r].astype(np.int64) % 3).astype(np.uint8)     # scale row r by 2 = -1
    assert _perm3(oracle_mod, B) == (2 * p) % 3
    Z = A.copy()
    Z[r] = 0
    assert _perm3(oracle_mod, Z) == 0
    assert _perm3(oracle_mod, Z.T) == 0


@pytest.mark.parametrize("n", list(range(1, 16)))
def test_closed_forms(oracle_mod, n):
    assert _perm3(oracle_mod, np.eye(n, dtype=np.uint8)) == 1
    assert _perm3(oracle_mod, np.ones((n, n), np.uint8)) == math.factorial(n) % 3
    assert _perm3(oracle_mod, 2 * np.eye(n, dtype=np.uint8)) == pow(2, n, 3)
    g = W.rng(300 + n)
    d = g.integers(0, 3, n).astype(np.uint8)
    expect = math.prod(-1 if x == 2 else int(x) for x in d) % 3
    assert _perm3(oracle_mod, np.diag(d)) == expect
    M, diag = W.hidden_triangular(n, 400 + n)
    assert _perm3(oracle_mod, M) == math.prod(-1 if x == 2 else int(x) for x in diag) % 3
