"""CPU pins of the oracle's 128-bit Gray-index tallies (matrices of up to 128 columns).

Section 3 stops at n <= 64; past that, a row and a Gray index need two 64-bit
words, and the sums are the same sums.  What pins the wide walk:

* for n <= 63 it equals the narrow oracle (itself pinned by brute force eq. 1);
* on every range it equals the sum of the per-term definition, each term
  formed from scratch at its 128-bit index (no walk);
* a direct sum M (+) D with D's column totals non-zero has, on the Gray range
  whose high state holds every row of D, the exact closed form
      T = (-1)^n2 * prod_c cmod3(total of D's column c) * T_M(0, 2^n1),
  with T_M from the narrow oracle, and (-1)^n T = delta * perm(M) mod 3 with
  perm(M) by brute force eq. (1).
"""
import math
import random

import numpy as np
import pytest

import oracle
from paper_2407_20205_amd import workloads as W


def gray(i: int) -> int:
    return i ^ (i >> 1)


def gray_inverse(x: int) -> int:
    """The index whose Gray state is x (prefix xor of its bits from the top)."""
    i = 0
    while x:
        i ^= x
        x >>= 1
    return i


def cmod3(x: int) -> int:
    r = x % 3
    return -1 if r == 2 else r


def signed(v) -> int:
    return -1 if int(v) == 2 else int(v)


def column_total_sign(D) -> int:
    """prod over D's columns of cmod3(sum of the column), entries read in {-1, 0, 1}."""
    d = 1
    for c in range(D.shape[1]):
        d *= cmod3(sum(signed(x) for x in D[:, c]))
    return d


def test_gray_inverse():
    for x in list(range(300)) + [(1 << 100) - 1, (1 << 127) + 12345]:
        assert gray(gray_inverse(x)) == x


@pytest.mark.parametrize("n", [1, 5, 20, 40, 63])
def test_wide_equals_narrow_oracle(n):
    g = W.rng(900 + n)
    A = g.integers(0, 3, (n, n), dtype=np.uint8)
    total = 1 << n
    ranges = [(0, min(total, 5000)), (total - min(total, 3000), min(total, 3000))]
    for _ in range(6):
        a = int(g.integers(0, total))
        ranges.append((a, min(int(g.integers(0, 4000)), total - a)))
    for a, c in ranges:
        assert oracle.range_tally_wide(A, a, c) == oracle.range_tally(A, a, a + c), (n, a, c)


def wide_ranges(n: int, seed: int, length: int = 1500):
    r = random.Random(seed)
    total = 1 << n
    out = [(0, length), (total - length, length)]
    if n > 64:
        out.append(((1 << 64) - length // 2, length))          # across 2^64
    if n >= 64:
        out.append(((1 << 63) - length // 3, length))          # across 2^63
    for _ in range(2):
        out.append((r.randrange(0, total - length), length))
    return out


@pytest.mark.parametrize("n", [64, 65, 96, 127, 128])
def test_wide_walk_equals_definition(n):
    A = W.rank_one_signs(n, 910 + n)
    nonzero = 0
    seen = 0
    for a, c in wide_ranges(n, 911 + n):
        terms = [oracle.term_wide(A, i) for i in range(a, a + c)]
        nonzero += sum(t != 0 for t in terms)
        seen += c
        assert oracle.range_tally_wide(A, a, c) == sum(terms), (n, a, c)
    assert nonzero > 0.5 * seen            # the ranges are full of non-zero terms


def test_wide_definition_equals_narrow_definition():
    for n in [3, 17, 40, 63]:
        A = W.uniform_matrix(n, 920 + n)
        r = random.Random(n)
        for i in [r.randrange(1 << n) for _ in range(50)]:
            assert oracle.term_wide(A, i) == oracle.term(A, i)


@pytest.mark.parametrize("n1,n2,pairs,shuffle", [(6, 122, 3, True), (8, 119, 4, True), (12, 52, 2, False),
                                                 (10, 91, 0, True), (7, 57, 5, False), (16, 112, 3, True)])
def test_wide_block_closed_form(n1, n2, pairs, shuffle):
    A, M, D = W.wide_block(n1, n2, 930 + n1 + n2, pairs=pairs, shuffle=shuffle)
    n = n1 + n2
    delta = column_total_sign(D)
    assert delta != 0                                       # the construction's premise
    h = gray_inverse((1 << n2) - 1)
    T = oracle.range_tally_wide(A, h << n1, 1 << n1, threads=8)
    T_M = oracle.range_tally(M, 0, 1 << n1)
    assert T == (-1) ** n2 * delta * T_M
    if n1 <= 8:
        assert ((-1) ** n * T - delta * oracle.brute_perm(M)) % 3 == 0
    if pairs == 0:
        # D is a signed permutation: a row of D missing from the state zeroes a column
        for hh in (h - 1, h + 1):
            assert oracle.range_tally_wide(A, hh << n1, 1 << n1) == 0


def test_wide_threads_agree():
    A = W.rank_one_signs(100, 940)
    a = (1 << 99) + 777
    assert oracle.range_tally_wide(A, a, 50000, threads=8) == oracle.range_tally_wide(A, a, 50000)


def test_wide_additivity():
    A = W.rank_one_signs(128, 941)
    a = (1 << 64) - 20000
    cuts = [0, 7000, 19999, 20001, 33333, 40000]
    parts = [oracle.range_tally_wide(A, a + cuts[k], cuts[k + 1] - cuts[k]) for k in range(len(cuts) - 1)]
    assert sum(parts) == oracle.range_tally_wide(A, a, 40000)


def test_wide_rejects_bad_input():
    A = W.uniform_matrix(10, 1)
    with pytest.raises(ValueError):
        oracle.range_tally_wide(A, (1 << 10) - 5, 6)             # past 2^n
    with pytest.raises(ValueError):
        oracle.range_tally_wide(A, 0, (1 << 62) + 1)              # count too large
    with pytest.raises(ValueError):
        oracle.range_tally_wide(np.zeros((129, 129), np.uint8), 0, 1)
    B = A.copy()
    B[3, 4] = 3
    with pytest.raises(ValueError):
        oracle.range_tally_wide(B, 0, 1)
    # the top of the n = 128 range is legal and ends exactly at 2^128
    J = W.rank_one_signs(128, 2)
    top = (1 << 128) - 100
    assert oracle.range_tally_wide(J, top, 100) == sum(oracle.term_wide(J, i) for i in range(top, 1 << 128))
    with pytest.raises(ValueError):
        oracle.range_tally_wide(J, top, 101)


def test_rank_one_terms_closed_form():
    # a_kj = e_k f_j: every column of S sums to f_j * s with s = sum_{k in S} e_k, so
    # term(S) = (-1)^|S| * prod_j f_j * cmod3(s)^n
    n = 70
    A = W.rank_one_signs(n, 950)
    e = [signed(A[k, 0]) * signed(A[0, 0]) for k in range(n)]      # e_k up to a common sign
    f = [signed(A[0, j]) * e[0] for j in range(n)]
    for k in range(n):
        for j in range(n):
            assert signed(A[k, j]) == e[k] * f[j]
    fprod = math.prod(f)
    r = random.Random(5)
    for i in [r.randrange(1 << n) for _ in range(300)]:
        S = gray(i)
        s = sum(e[k] for k in range(n) if (S >> k) & 1)
        want = (-1) ** bin(S).count("1") * fprod * cmod3(s) ** n
        assert oracle.term_wide(A, i) == want
