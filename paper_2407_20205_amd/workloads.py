"""Seeded synthetic inputs for perm(A) mod 3.

This module only draws random numbers and arranges them into matrices,
index lists and arrival times.  It holds none of the method's arithmetic and
imports nothing from the rest of the package, so the GPU path, the tests and
the CPU oracle can all take their inputs from it.

Every generator uses numpy ``Generator(PCG64(seed))``.  Matrices are n x n,
uint8, row-major, entries in {0, 1, 2} where 2 stands for -1 in F_3.  The
paper times random matrices with iid entries in {-1, 0, 1} (Section 3,
Table 2) and samples uniform random matrices for its Monte Carlo study
(Section 4); the uniform draws below are those distributions.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

# seeds of the five standard workloads
SEED_SINGLE_20 = 1
SEED_SINGLE_36 = 2
SEED_BATCH = 3
SEED_SERVE = 4
SEED_LARGE = 5


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_matrix(n: int, seed: int) -> np.ndarray:
    """One n x n matrix with iid entries uniform on {0, 1, 2}."""
    return rng(seed).integers(0, 3, size=(n, n), dtype=np.uint8)


def sparse_matrix(n: int, g: np.random.Generator, p=(0.6, 0.2, 0.2)) -> np.ndarray:
    """Entries iid with P(0), P(1), P(2) = p."""
    return g.choice(np.arange(3, dtype=np.uint8), size=(n, n), p=list(p)).astype(np.uint8)


def sha256(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def single_20() -> np.ndarray:
    """One 20 x 20 uniform matrix (2^20 Gray indices)."""
    return uniform_matrix(20, SEED_SINGLE_20)


def single_36() -> np.ndarray:
    """One 36 x 36 uniform matrix (2^36 Gray indices)."""
    return uniform_matrix(36, SEED_SINGLE_36)


def sample_chunks(n: int, seed: int, count: int = 64, log_len: int = 24,
                  unaligned: int = 8) -> list[tuple[int, int]]:
    """Seed-chosen Gray index ranges [a, b) of a 2^n range for spot checks.

    ``count - unaligned`` aligned chunks of length 2^log_len are drawn from the
    2^(n - log_len) chunk slots; the first and last slot are always among them
    and so is at least one odd slot.  ``unaligned`` further ranges start and
    end at arbitrary indices (length up to 2^log_len).
    """
    g = rng(seed)
    slots = 1 << (n - log_len)
    L = 1 << log_len
    n_al = max(0, count - unaligned)
    chosen = [0, slots - 1]
    if slots > 2:
        chosen.append(int(g.integers(0, slots // 2)) * 2 + 1)
    while len(chosen) < min(n_al, slots):
        c = int(g.integers(0, slots))
        if c not in chosen:
            chosen.append(c)
    out = [(c * L, (c + 1) * L) for c in chosen[:n_al]]
    total = 1 << n
    for _ in range(unaligned):
        a = int(g.integers(0, total - 1))
        ln = int(g.integers(1, L + 1))
        out.append((a, min(total, a + ln)))
    return out


@dataclass
class Batch:
    ns: np.ndarray                  # int32[count]
    mats: list                      # list of uint8 (n, n) arrays
    seed: int = SEED_BATCH

    @property
    def count(self) -> int:
        return len(self.mats)

    def flat(self) -> tuple[np.ndarray, np.ndarray]:
        """All matrices concatenated row-major, and the byte offset of each."""
        offs = np.zeros(self.count + 1, dtype=np.int64)
        offs[1:] = np.cumsum(self.ns.astype(np.int64) ** 2)
        buf = np.concatenate([m.reshape(-1) for m in self.mats]) if self.count else np.zeros(0, np.uint8)
        return buf, offs


def batch_uniform(count: int = 8192, n_lo: int = 12, n_hi: int = 28,
                  seed: int = SEED_BATCH) -> Batch:
    """``count`` matrices, n uniform on [n_lo, n_hi], entries uniform; n values drawn first."""
    g = rng(seed)
    ns = g.integers(n_lo, n_hi + 1, size=count).astype(np.int32)
    mats = [g.integers(0, 3, size=(int(n), int(n)), dtype=np.uint8) for n in ns]
    return Batch(ns=ns, mats=mats, seed=seed)


def batch_flat(count: int, n_lo: int, n_hi: int, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """``count`` matrices, n uniform on [n_lo, n_hi], entries uniform, drawn straight into one
    buffer (for batches of millions of matrices): returns (ns int32[count], offs int64[count + 1]
    byte offsets, buf uint8[offs[-1]]), matrix k row-major at buf[offs[k]:offs[k + 1]]."""
    g = rng(seed)
    ns = g.integers(n_lo, n_hi + 1, size=count).astype(np.int32)
    offs = np.zeros(count + 1, dtype=np.int64)
    offs[1:] = np.cumsum(ns.astype(np.int64) ** 2)
    buf = g.integers(0, 3, size=int(offs[-1]), dtype=np.uint8)
    return ns, offs, buf


def large_sparse(seed: int = SEED_LARGE, n_big: int = 44, n_sparse: int = 40,
                 count_sparse: int = 64) -> tuple[np.ndarray, Batch]:
    """One n_big x n_big uniform matrix plus ``count_sparse`` n_sparse matrices with P(0) = 0.6."""
    g = rng(seed)
    big = g.integers(0, 3, size=(n_big, n_big), dtype=np.uint8)
    mats = [sparse_matrix(n_sparse, g) for _ in range(count_sparse)]
    return big, Batch(ns=np.full(count_sparse, n_sparse, np.int32), mats=mats, seed=seed)


def serve_n_weights(n_lo: int = 8, n_hi: int = 40, ratio: float = 1.15) -> tuple[np.ndarray, np.ndarray]:
    ns = np.arange(n_lo, n_hi + 1)
    w = ratio ** (-(ns - n_lo).astype(np.float64))
    return ns, w / w.sum()


@dataclass
class ServeTrace:
    ns: np.ndarray                  # int32[count]
    mats: list
    arrival_s: np.ndarray           # float64[count], seconds from the start, nondecreasing
    rate: float
    seed: int = SEED_SERVE
    meta: dict = field(default_factory=dict)


def serve_trace(count: int = 20000, rate: float = 1000.0, seed: int = SEED_SERVE,
                n_lo: int = 8, n_hi: int = 40, ratio: float = 1.15) -> ServeTrace:
    """Open-loop request stream: n with P(n) proportional to ratio^-(n - n_lo),
    Poisson arrivals at ``rate`` per second (exponential gaps), uniform entries.
    Draw order: all n, then all gaps, then the matrices in arrival order."""
    g = rng(seed)
    support, p = serve_n_weights(n_lo, n_hi, ratio)
    ns = g.choice(support, size=count, p=p).astype(np.int32)
    gaps = g.exponential(1.0 / rate, size=count)
    arrival = np.cumsum(gaps) - gaps[0]
    mats = [g.integers(0, 3, size=(int(n), int(n)), dtype=np.uint8) for n in ns]
    return ServeTrace(ns=ns, mats=mats, arrival_s=arrival, rate=rate, seed=seed)


# ---- structured matrices for checks at sizes no enumeration reaches --------

def hidden_triangular(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """P U Q with U upper triangular, nonzero diagonal, random P, Q permutations.
    Returns the matrix and U's diagonal (entries in {1, 2})."""
    g = rng(seed)
    U = g.integers(0, 3, size=(n, n), dtype=np.uint8)
    U = np.triu(U)
    d = g.integers(1, 3, size=n, dtype=np.uint8)
    U[np.arange(n), np.arange(n)] = d
    P = g.permutation(n)
    Q = g.permutation(n)
    return np.ascontiguousarray(U[P][:, Q]), d


def hidden_block_diagonal(sizes, seed: int) -> tuple[np.ndarray, list]:
    """A direct sum of uniform blocks of the given sizes, rows and columns shuffled.
    Returns the matrix and the list of blocks."""
    g = rng(seed)
    n = int(sum(sizes))
    M = np.zeros((n, n), dtype=np.uint8)
    blocks = []
    o = 0
    for s in sizes:
        B = g.integers(0, 3, size=(s, s), dtype=np.uint8)
        M[o:o + s, o:o + s] = B
        blocks.append(B)
        o += s
    P = g.permutation(n)
    Q = g.permutation(n)
    return np.ascontiguousarray(M[P][:, Q]), blocks


# ---- the digits-of-pi matrix of Section 3.1 ---------------------------------

def wide_block(n1: int, n2: int, seed: int, pairs: int = 3, shuffle: bool = True, M=None):
    """A = M (+) D for matrices of up to 128 columns: M (n1 x n1, uniform unless given) in the
    first n1 rows and columns, D (n2 x n2) in the last n2.  Column c of D holds one +-1 in row
    p(c) (p a random permutation) and `pairs` further pairs of opposite entries (1 and 2, i.e. 1
    and -1) in other rows, so the entries of every D column over all n2 rows add up to that one
    +-1.  With `shuffle` the n columns of A are permuted at random (rows keep their order).
    Returns (A, M, D)."""
    g = rng(seed)
    n = n1 + n2
    M = g.integers(0, 3, size=(n1, n1), dtype=np.uint8) if M is None else np.asarray(M, dtype=np.uint8)
    assert M.shape == (n1, n1)
    D = np.zeros((n2, n2), dtype=np.uint8)
    piv = g.permutation(n2)
    for c in range(n2):
        D[piv[c], c] = g.integers(1, 3)
        others = [r for r in range(n2) if r != piv[c]]
        k = min(pairs, len(others) // 2)
        if k:
            rows = g.choice(others, size=2 * k, replace=False)
            for t in range(k):
                v = int(g.integers(1, 3))
                D[rows[2 * t], c] = v
                D[rows[2 * t + 1], c] = 3 - v
    A = np.zeros((n, n), dtype=np.uint8)
    A[:n1, :n1] = M
    A[n1:, n1:] = D
    if shuffle:
        A = A[:, g.permutation(n)]
    return np.ascontiguousarray(A), M, D


SEED_WIDE = 6


def wide_128():
    """The 128-column workload: M (+) D with M a hidden triangular 36 x 36 matrix (so perm(M) is
    the product of its diagonal) and D 92 x 92, columns shuffled.  Returns (A, M, d, D) with d
    the diagonal behind M."""
    M, d = hidden_triangular(36, SEED_WIDE)
    A, M, D = wide_block(36, 92, SEED_WIDE, pairs=3, shuffle=True, M=M)
    return A, M, d, D


def rank_one_signs(n: int, seed: int) -> np.ndarray:
    """a_kj = e_k * f_j with random signs e, f: every entry is +-1 (bytes 1 and 2) and all columns
    of a row subset have the same sum up to sign, so about two thirds of all Ryser terms are
    non-zero at any n."""
    g = rng(seed)
    e = g.integers(0, 2, size=n)
    f = g.integers(0, 2, size=n)
    return np.where(e[:, None] == f[None, :], 1, 2).astype(np.uint8)


def _arctan_inv(x: int, unity: int) -> int:
    """arctan(1/x) * unity by its alternating power series, in integers."""
    total = term = unity // x
    x2 = x * x
    k = 1
    while term:
        term //= x2
        k += 2
        total += -(term // k) if (k // 2) % 2 else term // k
    return total


def pi_digits(count: int) -> str:
    """The first ``count`` decimal digits of pi ("31415..."), from Machin's formula
    pi = 16 arctan(1/5) - 4 arctan(1/239), with 10 guard digits."""
    guard = 10
    unity = 10 ** (count + guard)
    pi = 16 * _arctan_inv(5, unity) - 4 * _arctan_inv(239, unity)
    return str(pi)[:count]


def pi_matrix(n: int, reading: str = "rows") -> np.ndarray:
    """Pi_n: an n x n matrix of decimal digits of pi reduced mod 3 (so entries are in
    {0, 1, 2}, 2 standing for -1).

    reading "rows": row i (0-based) holds digits n*i + 1 .. n*i + n (1-based digit
    positions), i.e. the first row is the first n digits, as the prose says.
    reading "formula": entry (i, j) (1-based) is digit (n-1)*i + j taken literally
    with i counted from 0, so consecutive rows share one digit.
    """
    if reading == "rows":
        d = pi_digits(n * n)
        idx = [[n * i + j for j in range(n)] for i in range(n)]
    elif reading == "formula":
        d = pi_digits((n - 1) * (n - 1) + n)
        idx = [[(n - 1) * i + j for j in range(n)] for i in range(n)]
    else:
        raise ValueError(reading)
    return np.array([[int(d[k]) % 3 for k in row] for row in idx], dtype=np.uint8)
