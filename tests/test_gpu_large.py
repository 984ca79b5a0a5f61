"""GPU parity at sizes no full oracle run reaches: one 44 x 44 uniform matrix and
64 sparse 40 x 40 matrices (P(0) = 0.6).  Exact checks: sampled Gray chunks
against the oracle, shards that add up to the whole, independent traversals,
and closed forms of structured matrices."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import flush_print, oracle_tallies, require_gpu, to_dev
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


@pytest.fixture(scope="module")
def large():
    return W.large_sparse()


def test_44x44_sampled_chunks(large):
    big, _ = large
    chunks = W.sample_chunks(44, seed=W.SEED_LARGE, count=20, log_len=22, unaligned=4)
    flush_print("oracle on 20 chunks of the 44x44 matrix")
    want = oracle_tallies(big, chunks)
    for (a, b), w in zip(chunks, want):
        assert P.perm_mod3_range_tally(big, a, b) == w, (a, b)


def test_44x44_whole_equals_shards(large):
    big, _ = large
    flush_print("n=44: whole range, then 8 shards")
    T = P.perm_mod3_range_tally(big, 0, 1 << 44)
    assert abs(T) < 1 << 44
    shards = [(k << 41, (k + 1) << 41) for k in range(8)]
    assert sum(P.perm_mod3_range_tally(big, a, b) for a, b in shards) == T
    assert P.perm_mod3(big) == T % 3          # (-1)^44 = 1


def test_sparse40_batch_vs_single_and_oracle(large):
    import torch
    _, sp = large
    buf, offs = sp.flat()
    out = torch.zeros(sp.count, dtype=torch.uint8, device="cuda")
    flush_print("64 sparse 40x40 matrices in one launch")
    P.perm_mod3_batch_dev(to_dev(buf, torch.uint8), to_dev(offs[:-1], torch.int64), to_dev(sp.ns, torch.int32),
                          out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert set(np.unique(got)) <= {0, 1, 2}
    for k in (0, 17, 63):
        assert P.perm_mod3(sp.mats[k]) == got[k], k
    # the same matrices' Gray chunks against the oracle
    g = W.rng(51)
    for k in (5, 40):
        ranges = []
        for _ in range(3):
            a = int(g.integers(0, (1 << 40) - (1 << 22)))
            ranges.append((a, a + (1 << 22)))
        want = oracle_tallies(sp.mats[k], ranges)
        for (a, b), w in zip(ranges, want):
            assert P.perm_mod3_range_tally(sp.mats[k], a, b) == w, (k, a, b)


def test_sparse40_structured():
    g = W.rng(52)
    # sparse upper-triangular with a non-zero diagonal, hidden by row and column permutations
    U = W.sparse_matrix(40, g)
    U = np.triu(U)
    d = g.integers(1, 3, size=40).astype(np.uint8)
    U[np.arange(40), np.arange(40)] = d
    M = np.ascontiguousarray(U[g.permutation(40)][:, g.permutation(40)])
    assert P.perm_mod3(M) == math.prod(-1 if x == 2 else int(x) for x in d) % 3
    # block diagonal of sparse blocks, hidden
    blocks = [W.sparse_matrix(s, g) for s in (12, 14, 14)]
    B = np.zeros((40, 40), np.uint8)
    o = 0
    for blk in blocks:
        B[o:o + blk.shape[0], o:o + blk.shape[0]] = blk
        o += blk.shape[0]
    B = np.ascontiguousarray(B[g.permutation(40)][:, g.permutation(40)])
    want = 1
    for blk in blocks:
        want = want * oracle.perm_mod3(blk) % 3
    assert P.perm_mod3(B) == want
    # a zero column makes every column product vanish
    Z = W.sparse_matrix(40, g)
    Z[:, 7] = 0
    assert P.perm_mod3_range_tally(Z, 0, 1 << 40) == 0


@pytest.mark.parametrize("n", [38, 40])
def test_multilinear_in_a_row(n):
    """perm is linear in each row: with A and A2 equal but for row r, and A3 equal to them but
    with row r the entrywise sum of theirs over F_3, perm(A) + perm(A2) = perm(A3) mod 3.  Three
    independent whole-range walks per case, four cases per n, rows r spread over the low, middle
    and high Gray bits; and perm(A) = perm(A with row r replaced by its negation) * 2."""
    g = W.rng(900 + n)
    for r in (0, 5, n // 2, n - 1):
        flush_print(f"multilinearity n={n} row={r}")
        A = g.integers(0, 3, size=(n, n), dtype=np.uint8)
        A2 = A.copy()
        A2[r] = g.integers(0, 3, size=n, dtype=np.uint8)
        A3 = A.copy()
        A3[r] = (A[r].astype(np.int32) + A2[r]) % 3
        p, p2, p3 = P.perm_mod3(A), P.perm_mod3(A2), P.perm_mod3(A3)
        assert (p + p2) % 3 == p3, (n, r, p, p2, p3)
        N = A.copy()
        N[r] = (3 - N[r].astype(np.int32)) % 3
        assert P.perm_mod3(N) == (2 * p) % 3, (n, r)
