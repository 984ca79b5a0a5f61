"""CPU oracle for perm(A) mod 3 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2407_20205_amd``) and never imports it.

Two independent definitions live here:

* ``brute_perm`` -- the permanent by its definition, eq. (1): a sum over all
  n! permutations of products of entries, in exact Python integers.  Used for
  n <= 8.  ``perm_mod3_stack`` is the same sum mod 3 with the permutations
  grouped by the columns of the first rows, vectorised over stacks of up to
  millions of matrices of one order n <= 12.
* the C oracle (``perm3_oracle.c``) -- Ryser's identity, eq. (2), walked in
  reflected-binary Gray-code order with UNPACKED centred residues (Section 3
  with its cmod3 reduction), threaded over blocks of consecutive Gray indices
  as in Section 3.1.  It returns exact partial tallies T(a, b) and perm mod 3,
  and, for matrices of up to 128 columns, tallies over 128-bit Gray indices.
* vectors over F_3 (``f3_*``): phi and psi of Section 2 and elementwise
  arithmetic of F_3 on unpacked values, the definitions behind Theorem 2.1.

Inputs are n x n uint8 matrices with entries in {0, 1, 2}; 2 stands for -1.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perm3_oracle.c")
_LIB = os.path.join(_HERE, "libperm3_oracle.so")

MAX_N = 63
MAX_N_WIDE = 128


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/libperm3_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-Wall",
                        "-Wextra", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    """The loaded C oracle; built first only if no built copy exists."""
    global _lib
    if _lib is None:
        path = build(force=False)
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.oracle_term.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64]
        L.oracle_term.restype = ctypes.c_int
        L.oracle_range_tally.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
        L.oracle_range_tally.restype = ctypes.c_int64
        L.oracle_range_tally_mt.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64,
                                            ctypes.c_uint64, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int)]
        L.oracle_range_tally_mt.restype = ctypes.c_int64
        L.oracle_perm_mod3.argtypes = [u8p, ctypes.c_int, ctypes.c_int]
        L.oracle_perm_mod3.restype = ctypes.c_int
        L.oracle_count_by_value.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_count_by_value.restype = ctypes.c_int
        L.oracle_census.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_census.restype = ctypes.c_int
        L.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_splitmix64.restype = ctypes.c_uint64
        L.oracle_term_wide.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_term_wide.restype = ctypes.c_int
        L.oracle_range_tally_wide.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                              ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
        L.oracle_range_tally_wide.restype = ctypes.c_int64
        L.oracle_range_tally_wide_mt.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                                 ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.oracle_range_tally_wide_mt.restype = ctypes.c_int64
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_f3_phi.argtypes = [u8p, ctypes.c_int64, u64p]
        L.oracle_f3_phi.restype = ctypes.c_int64
        L.oracle_f3_psi.argtypes = [u64p, ctypes.c_int64, u8p]
        L.oracle_f3_psi.restype = None
        L.oracle_f3_op.argtypes = [ctypes.c_int, u8p, u8p, ctypes.c_int64, u8p]
        L.oracle_f3_op.restype = ctypes.c_int
        L.oracle_f3_dot.argtypes = [u8p, u8p, ctypes.c_int64]
        L.oracle_f3_dot.restype = ctypes.c_int64
        _lib = L
    return _lib


def _mat(A) -> tuple[np.ndarray, int]:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.uint8))
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    return A, A.shape[0]


def _ptr(A: np.ndarray):
    return A.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def term(A, i: int) -> int:
    """One Ryser term for Gray index i, formed from scratch: (-1)^|S| prod_col sum_{k in S} A[k][col], S = g(i)."""
    A, n = _mat(A)
    return lib().oracle_term(_ptr(A), n, i)


def range_tally(A, a: int, b: int, threads: int | None = None) -> int:
    """Exact T(a, b) = sum of Ryser terms over Gray indices a <= i < b."""
    A, n = _mat(A)
    ok = ctypes.c_int(0)
    if threads is None or threads <= 1:
        v = lib().oracle_range_tally(_ptr(A), n, a, b, ctypes.byref(ok))
    else:
        v = lib().oracle_range_tally_mt(_ptr(A), n, a, b, threads, ctypes.byref(ok))
    if not ok.value:
        raise ValueError("invalid matrix or range")
    return int(v)


def perm_from_tally(n: int, T: int) -> int:
    """perm(A) mod 3 in {0, 1, 2} from the whole Gray sum T = T(0, 2^n): eq. (2) carries the
    factor (-1)^n outside the sum over subsets."""
    return (-T if n % 2 else T) % 3


def perm_mod3(A, threads: int | None = None) -> int:
    """perm(A) mod 3 in {0, 1, 2} through Ryser + Gray code on unpacked residues."""
    A, n = _mat(A)
    r = lib().oracle_perm_mod3(_ptr(A), n, threads or default_threads())
    if r < 0:
        raise ValueError("invalid matrix")
    return r


def count_by_value(n: int) -> tuple[int, int, int]:
    """Over all 3^(n*n) matrices (n <= 4): how many have perm 0, 1 and -1."""
    c = (ctypes.c_uint64 * 3)()
    if lib().oracle_count_by_value(n, c) != 0:
        raise ValueError("n must be in 1..4")
    return int(c[0]), int(c[1]), int(c[2])


def census(n: int, generator: int, key: int, first: int, count: int) -> tuple[int, int, int]:
    """Counts of perm mod 3 = 0, 1, 2 over generated matrices (0: base-3 enumeration of the
    matrix index, 1: SplitMix64 draws), matrices first .. first + count - 1; n <= 63."""
    c = (ctypes.c_uint64 * 3)()
    if lib().oracle_census(n, generator, key, first, count, c) != 0:
        raise ValueError("bad census arguments")
    return int(c[0]), int(c[1]), int(c[2])


def splitmix64(key: int, q: int) -> int:
    """The q-th output (q >= 1) of SplitMix64 seeded with key."""
    return int(lib().oracle_splitmix64(key, q))


def term_wide(A, i: int) -> int:
    """One Ryser term by its definition at a Gray index of up to 128 bits (n <= 128)."""
    A, n = _mat(A)
    return lib().oracle_term_wide(_ptr(A), n, i >> 64, i & ((1 << 64) - 1))


def range_tally_wide(A, begin: int, count: int, threads: int | None = None) -> int:
    """Exact T(begin, begin + count) for n <= 128 with 128-bit Gray indices (count <= 2^62)."""
    A, n = _mat(A)
    ok = ctypes.c_int(0)
    hi, lo = begin >> 64, begin & ((1 << 64) - 1)
    if not 0 <= begin < (1 << 128) or not 0 <= count < (1 << 64):
        raise ValueError("begin must fit 128 bits and count 64 bits")
    if threads is None or threads <= 1:
        v = lib().oracle_range_tally_wide(_ptr(A), n, hi, lo, count, ctypes.byref(ok))
    else:
        v = lib().oracle_range_tally_wide_mt(_ptr(A), n, hi, lo, count, threads, ctypes.byref(ok))
    if not ok.value:
        raise ValueError("invalid matrix or range")
    return int(v)


def _vec(v) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(v, dtype=np.uint8))
    if v.ndim != 1:
        raise ValueError("vector expected")
    return v


def f3_phi(v) -> tuple[np.ndarray, int]:
    """phi of a vector: (planes uint64[2 * ceil(len/64)], count of bytes > 2); element e at bit e mod 64."""
    v = _vec(v)
    planes = np.zeros(2 * ((len(v) + 63) // 64), dtype=np.uint64)
    bad = lib().oracle_f3_phi(_ptr(v), len(v), planes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return planes, int(bad)


def f3_psi(planes, length: int) -> np.ndarray:
    """psi of bipedal planes back to bytes {0, 1, 2}."""
    planes = np.ascontiguousarray(np.asarray(planes, dtype=np.uint64))
    if planes.size < 2 * ((length + 63) // 64):
        raise ValueError("planes too short")
    out = np.zeros(length, dtype=np.uint8)
    lib().oracle_f3_psi(planes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), length, _ptr(out))
    return out


F3_ADD, F3_SUB, F3_MUL, F3_DIV, F3_NEG = range(5)


def f3_op(op: int, a, b=None) -> np.ndarray:
    """Elementwise a op b in F_3 on bytes (2 = -1); a quotient by 0 comes out as 0xFF."""
    a = _vec(a)
    b = a if b is None else _vec(b)
    if len(b) != len(a):
        raise ValueError("lengths differ")
    out = np.zeros(len(a), dtype=np.uint8)
    if lib().oracle_f3_op(op, _ptr(a), _ptr(b), len(a), _ptr(out)) != 0:
        raise ValueError("bad op or entry")
    return out


def f3_dot(a, b) -> int:
    """sum_e a_e b_e over the integers, entries read in {-1, 0, 1}."""
    a, b = _vec(a), _vec(b)
    if len(b) != len(a):
        raise ValueError("lengths differ")
    return int(lib().oracle_f3_dot(_ptr(a), _ptr(b), len(a)))


def signed(A) -> list[list[int]]:
    """Entries as integers in {-1, 0, 1} (2 read as -1)."""
    A, n = _mat(A)
    return [[-1 if int(x) == 2 else int(x) for x in row] for row in A]


def brute_perm(A) -> int:
    """perm(A) over the integers by eq. (1): sum over sigma in S_n of prod_i a_{i, sigma(i)}."""
    M = signed(A)
    n = len(M)
    total = 0
    for sigma in itertools.permutations(range(n)):
        p = 1
        for i in range(n):
            p *= M[i][sigma[i]]
            if p == 0:
                break
        total += p
    return total


def brute_perm_mod3(A) -> int:
    return brute_perm(A) % 3


def perm_mod3_stack(mats) -> np.ndarray:
    """perm mod 3 in {0, 1, 2} of every matrix of a stack of shape (m, n, n), n <= 12, by eq. (1)
    with its sum over permutations grouped by the set of columns that the first rows take.

    For a column set S let f(S) be the sum, over the bijections sigma from rows 0 .. |S|-1 onto S,
    of prod_i a_{i, sigma(i)}.  Then f(empty set) = 1 (the empty product), and splitting on the
    column j = sigma(|S| - 1) of the last of those rows gives
        f(S) = sum over j in S of a_{|S|-1, j} * f(S minus {j}),
    so perm(A) = f(all n columns).  Residues stay in {0, 1, 2} (2 is -1) and every step reduces
    mod 3.  Vectorised over the stack in chunks, so millions of small matrices take seconds."""
    M = np.asarray(mats, dtype=np.uint8)
    if M.ndim != 3 or M.shape[1] != M.shape[2]:
        raise ValueError("stack of square matrices expected")
    m, n = M.shape[0], M.shape[1]
    if n > 12:
        raise ValueError("n must be at most 12")
    if np.any(M > 2):
        raise ValueError("entries must be in {0, 1, 2}")
    out = np.empty(m, dtype=np.uint8)
    chunk = max(1, (1 << 24) >> n)
    for c0 in range(0, m, chunk):
        # column-major copy: A[row, j] is one contiguous vector over the chunk
        A = np.ascontiguousarray(M[c0:c0 + chunk].transpose(1, 2, 0))
        f = np.zeros((1 << n, A.shape[2]), dtype=np.uint8)
        f[0] = 1
        for S in range(1, 1 << n):
            row = bin(S).count("1") - 1
            acc = np.zeros(A.shape[2], dtype=np.uint8)     # at most 4 n <= 48: no overflow
            for j in range(n):
                if S >> j & 1:
                    acc += A[row, j] * f[S & ~(1 << j)]
            f[S] = acc % 3
        out[c0:c0 + chunk] = f[(1 << n) - 1]
    return out
