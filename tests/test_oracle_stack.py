"""Pins of the oracle's stacked permanent (eq. (1) grouped by the columns of the first rows).

It is pinned to Table 3's z(1..4), counted over every matrix of each order, to the oracle's
Ryser walk (eq. (2) in Gray-code order, a different formula) on random stacks, and to closed
forms: the identity, -I, the all-ones matrix (perm = n!), a zero row, row swaps.
"""
import math

import numpy as np
import pytest

from conftest import read_golden
from paper_2407_20205_amd import workloads as W


def _digits(count: int, nd: int) -> np.ndarray:
    """Base-3 digits (least significant first) of 0 .. count-1: every matrix of nd entries."""
    idx = np.arange(count, dtype=np.int64)
    D = np.empty((count, nd), np.uint8)
    for k in range(nd):
        D[:, k] = idx % 3
        idx //= 3
    return D


def test_table3_z1_to_z3_exhaustive(oracle_mod):
    z = {int(r[0]): int(r[1]) for r in read_golden("table3_zero_counts.txt")}
    for n in (1, 2, 3):
        M = _digits(3 ** (n * n), n * n).reshape(-1, n, n)
        r = oracle_mod.perm_mod3_stack(M)
        assert int(np.count_nonzero(r == 0)) == z[n], n


def test_table3_z4_exhaustive(oracle_mod):
    """All 3^16 matrices of order 4: rows 0-1 from the low 8 digits, rows 2-3 from the high 8."""
    z = {int(r[0]): int(r[1]) for r in read_golden("table3_zero_counts.txt")}
    half = _digits(3 ** 8, 8)
    counts = np.zeros(3, np.int64)
    for h0 in range(0, 3 ** 8, 256):
        h = half[h0:h0 + 256]
        M = np.concatenate([np.tile(half, (len(h), 1)), np.repeat(h, 3 ** 8, axis=0)], axis=1)
        r = oracle_mod.perm_mod3_stack(M.reshape(-1, 4, 4))
        counts += np.bincount(r, minlength=3)
    zeros = int(counts[0])
    assert zeros == z[4]
    assert int(counts.sum()) == 3 ** 16
    # negating the first row is a bijection that swaps permanents 1 and -1
    assert counts[1] == counts[2]


@pytest.mark.parametrize("n", list(range(0, 11)))
def test_agrees_with_the_ryser_walk(oracle_mod, n):
    g = W.rng(700 + n)
    count = 300 if n <= 8 else 40
    M = g.integers(0, 3, size=(count, n, n), dtype=np.uint8)
    got = oracle_mod.perm_mod3_stack(M)
    want = [oracle_mod.perm_mod3(A, threads=1) if n else 1 for A in M]
    assert got.tolist() == want


def test_closed_forms(oracle_mod):
    for n in range(0, 11):
        eye = np.eye(n, dtype=np.uint8)
        ones = np.ones((n, n), np.uint8)
        neg = (2 * eye).astype(np.uint8)
        stack = np.stack([eye, ones, neg]) if n else np.zeros((3, 0, 0), np.uint8)
        r = oracle_mod.perm_mod3_stack(stack).tolist()
        assert r[0] == 1, n                                   # one permutation, product 1
        assert r[1] == math.factorial(n) % 3, n               # every permutation contributes 1
        assert r[2] == (-1) ** n % 3, n                       # (-1)^n
    g = W.rng(711)
    A = g.integers(0, 3, size=(64, 7, 7), dtype=np.uint8)
    base = oracle_mod.perm_mod3_stack(A)
    Z = A.copy()
    Z[:, 3, :] = 0
    assert not oracle_mod.perm_mod3_stack(Z).any()
    # rows (or columns) in another order: same permanent
    P = A[:, [6, 0, 5, 1, 4, 2, 3], :]
    Q = A[:, :, [2, 4, 6, 0, 1, 3, 5]]
    assert np.array_equal(oracle_mod.perm_mod3_stack(P), base)
    assert np.array_equal(oracle_mod.perm_mod3_stack(Q), base)
    # one row negated: the permanent is negated
    N = A.copy()
    N[:, 2, :] = (3 - N[:, 2, :]) % 3
    assert np.array_equal(oracle_mod.perm_mod3_stack(N), (3 - base.astype(np.int32)) % 3)


def test_rejects_bad_stacks(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.perm_mod3_stack(np.zeros((2, 13, 13), np.uint8))
    with pytest.raises(ValueError):
        oracle_mod.perm_mod3_stack(np.full((2, 3, 3), 3, np.uint8))
    with pytest.raises(ValueError):
        oracle_mod.perm_mod3_stack(np.zeros((2, 3, 4), np.uint8))
    assert oracle_mod.perm_mod3_stack(np.zeros((0, 5, 5), np.uint8)).shape == (0,)
