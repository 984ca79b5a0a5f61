"""Planted mistakes in a throwaway copy of the C oracle must be caught by the pins.

Each mutant is a small textual edit of ``oracle/perm3_oracle.c`` compiled with
gcc into a temporary directory (CPU only); the original oracle is untouched.
The pins used are the ones in test_oracle.py: brute force eq. (1), the direct
per-term definition, and closed forms of T(0, 2^n).
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2407_20205_amd import workloads as W

SRC = os.path.join(os.path.dirname(oracle.__file__), "perm3_oracle.c")

MUTANTS = {
    # the direction convention of the plain-integer listing (add when the row is already in)
    "direction_swapped": ("leaving ? v[col] - E[t][col] : v[col] + E[t][col]",
                          "leaving ? v[col] + E[t][col] : v[col] - E[t][col]"),
    "drop_minus_one_to_the_n": ("int64_t p = (n & 1) ? -T : T;", "int64_t p = T;"),
    "drop_subset_sign": ("if (popcount64(x) & 1) s -= prod; else s += prod;", "s += prod;"),
    "sign_from_index_not_state": ("if (popcount64(x) & 1) s -= prod; else s += prod;",
                                  "if (i & 2) s -= prod; else s += prod;"),
    "seed_without_gray": ("uint64_t x = a ^ (a >> 1);", "uint64_t x = a;"),
    "row_off_by_one": ("v[col] - E[t][col] : v[col] + E[t][col]",
                       "v[col] - E[(t + 1) % n][col] : v[col] + E[(t + 1) % n][col]"),
    "seed_transposed": ("if ((x >> k) & 1u) sum += E[k][col];", "if ((x >> k) & 1u) sum += E[col][k];"),
    "skip_first_term": ("        int prod = 1;\n        for (int col = 0; col < n; ++col) prod *= v[col];",
                        "        int prod = (i == a) ? 0 : 1;\n        for (int col = 0; col < n; ++col) prod *= v[col];"),
    # (reading 2 as +2 would be no mistake at all: 2 = -1 in F_3)
    "minus_one_read_as_one": ("return A[row * n + col] == 2 ? -1 : (int)A[row * n + col];",
                              "return A[row * n + col] == 2 ? 1 : (int)A[row * n + col];"),
    "product_skips_last_column": ("for (int col = 0; col < n; ++col) prod *= v[col];",
                                  "for (int col = 0; col + 1 < n; ++col) prod *= v[col];"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-o", str(so), str(c)], check=True)
    L = ctypes.CDLL(str(so))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.oracle_perm_mod3.argtypes = [u8p, ctypes.c_int, ctypes.c_int]
    L.oracle_perm_mod3.restype = ctypes.c_int
    L.oracle_term.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64]
    L.oracle_term.restype = ctypes.c_int
    L.oracle_range_tally.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.POINTER(ctypes.c_int)]
    L.oracle_range_tally.restype = ctypes.c_int64
    return L


def _p(A):
    A = np.ascontiguousarray(A, dtype=np.uint8)
    return A, A.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def pins_pass(L) -> bool:
    ok = ctypes.c_int(0)
    # brute force eq. (1)
    for n in range(1, 7):
        for s in range(6):
            A, p = _p(W.uniform_matrix(n, 5000 + 10 * n + s))
            if L.oracle_perm_mod3(p, n, 1) != oracle.brute_perm_mod3(A):
                return False
    # Gray walk vs per-term definition on every range start
    A, p = _p(W.uniform_matrix(5, 77))
    terms = [0] * 32
    for i in range(32):
        terms[i] = L.oracle_term(p, 5, i)
    for a in range(32):
        if L.oracle_range_tally(p, 5, a, 32, ctypes.byref(ok)) != sum(terms[a:]):
            return False
    # closed forms: T(0,2^n) of I_n is (-1)^n; of J_n is sum_k C(n,k) (-1)^k c(k)^n
    for n in range(1, 9):
        _, pI = _p(np.eye(n))
        if L.oracle_range_tally(pI, n, 0, 1 << n, ctypes.byref(ok)) != (-1) ** n:
            return False
        _, pJ = _p(np.ones((n, n)))
        expect = sum(math.comb(n, k) * (-1) ** k * (((k + 1) % 3) - 1) ** n for k in range(n + 1))
        if L.oracle_range_tally(pJ, n, 0, 1 << n, ctypes.byref(ok)) != expect:
            return False
    return True


def test_unmutated_oracle_passes_pins(tmp_path):
    L = _build(tmp_path, "original", "#include <stdint.h>", "#include <stdint.h>")
    assert pins_pass(L)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    L = _build(tmp_path, name, old, new)
    assert not pins_pass(L), f"planted mistake {name} slipped through the pins"


# ---------------------------------------------------------------- 128-bit Gray indices

WIDE_MUTANTS = {
    "wide_state_low_half": ("oracle_u128 state = a ^ (a >> 1);",
                            "oracle_u128 state = (uint64_t)(a ^ (a >> 1));"),
    "wide_popcount_low_half": ("return popcount64((uint64_t)x) + popcount64((uint64_t)(x >> 64));",
                               "return popcount64((uint64_t)x);"),
    "wide_seed_drops_high_rows": ("if ((state >> k) & 1u) sum += E[k][col];",
                                  "if (k < 64 && ((state >> k) & 1u)) sum += E[k][col];"),
    "wide_step_ctz_low_word": ("int t = trailing_zeros128(i);",
                               "int t = trailing_zeros64((uint64_t)i | ((uint64_t)1 << 63));"),
    "wide_term_gray_low_half": ("oracle_u128 S = i ^ (i >> 1);",
                                "oracle_u128 S = (uint64_t)i ^ ((uint64_t)i >> 1);"),
    "wide_range_one_too_many": ("for (uint64_t step = 0; step < count; ++step) {",
                                "for (uint64_t step = 0; step <= count; ++step) {"),
}


def _wide(L):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.oracle_term_wide.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    L.oracle_term_wide.restype = ctypes.c_int
    L.oracle_range_tally_wide.argtypes = [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    L.oracle_range_tally_wide.restype = ctypes.c_int64
    return L


def wide_pins_pass(L) -> bool:
    """The pins of test_oracle_wide.py, on a mutated copy: narrow equality, per-term
    definition on ranges across 2^63, 2^64 and at the top, and the block closed form."""
    ok = ctypes.c_int(0)
    M64 = (1 << 64) - 1

    def tally(p, n, a, c):
        return L.oracle_range_tally_wide(p, n, a >> 64, a & M64, c, ctypes.byref(ok))

    def term(p, n, i):
        return L.oracle_term_wide(p, n, i >> 64, i & M64)

    A, p = _p(W.uniform_matrix(20, 960))
    for a, c in [(0, 3000), (123456, 2000), ((1 << 20) - 900, 900)]:
        if tally(p, 20, a, c) != oracle.range_tally(A, a, a + c):
            return False
    for n in (65, 128):
        J, pJ = _p(W.rank_one_signs(n, 961 + n))
        for a in (0, (1 << 63) - 300, (1 << 64) - 300, (1 << n) - 600, (1 << (n - 1)) + 12345):
            if tally(pJ, n, a, 600) != sum(term(pJ, n, i) for i in range(a, a + 600)):
                return False
    for n1, n2 in ((6, 57), (8, 119), (6, 122)):
        B, Mb, Db = W.wide_block(n1, n2, 962 + n2)
        _, pB = _p(B)
        delta = 1
        for c in range(n2):
            r = sum(-1 if int(x) == 2 else int(x) for x in Db[:, c]) % 3
            delta *= -1 if r == 2 else r
        h, x = 0, (1 << n2) - 1
        while x:
            h ^= x
            x >>= 1
        if tally(pB, n1 + n2, h << n1, 1 << n1) != (-1) ** n2 * delta * oracle.range_tally(Mb, 0, 1 << n1):
            return False
    return True


def test_unmutated_oracle_passes_wide_pins(tmp_path):
    L = _wide(_build(tmp_path, "original_wide", "#include <stdint.h>", "#include <stdint.h>"))
    assert wide_pins_pass(L)


@pytest.mark.parametrize("name", sorted(WIDE_MUTANTS))
def test_wide_mutant_is_caught(tmp_path, name):
    old, new = WIDE_MUTANTS[name]
    L = _wide(_build(tmp_path, name, old, new))
    assert not wide_pins_pass(L), f"planted mistake {name} slipped through the wide pins"


# ---------------------------------------------------------------- vectors over F_3

F3_MUTANTS = {
    "f3_phi_sign_on_one": ("if (v[e] == 2) planes[2 * (e / 64) + 1] |= bit;",
                           "if (v[e] != 0) planes[2 * (e / 64) + 1] |= bit;"),
    "f3_phi_msb_first": ("uint64_t bit = (uint64_t)1 << (e % 64);",
                         "uint64_t bit = (uint64_t)1 << (63 - e % 64);"),
    "f3_sub_reversed": ("case 1: out[e] = f3_byte(x - y); break;", "case 1: out[e] = f3_byte(y - x); break;"),
    "f3_div_negated": ("out[e] = inv ? f3_byte(x * inv) : 0xFF;", "out[e] = inv ? f3_byte(-x * inv) : 0xFF;"),
    "f3_psi_second_zero_as_minus_one": ("v[e] = m ? (s ? 2 : 1) : 0;", "v[e] = m ? (s ? 2 : 1) : (s ? 2 : 0);"),
    "f3_dot_ignores_sign": ("s += (int64_t)f3_value(a[e]) * f3_value(b[e]);",
                            "s += (int64_t)(a[e] != 0) * (b[e] != 0);"),
}


def _f3(L):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.oracle_f3_phi.argtypes = [u8p, ctypes.c_int64, u64p]
    L.oracle_f3_phi.restype = ctypes.c_int64
    L.oracle_f3_psi.argtypes = [u64p, ctypes.c_int64, u8p]
    L.oracle_f3_psi.restype = None
    L.oracle_f3_op.argtypes = [ctypes.c_int, u8p, u8p, ctypes.c_int64, u8p]
    L.oracle_f3_op.restype = ctypes.c_int
    L.oracle_f3_dot.argtypes = [u8p, u8p, ctypes.c_int64]
    L.oracle_f3_dot.restype = ctypes.c_int64
    return L


def f3_pins_pass(L) -> bool:
    """The pins of test_oracle_f3.py on a mutated copy: the hand-written tables, the worked
    example of Section 2, psi after phi (with the second zero), the dot product's closed forms."""
    from conftest import read_golden
    u64p = ctypes.POINTER(ctypes.c_uint64)
    ops = {"add": 0, "sub": 1, "mul": 2, "div": 3}
    byte = lambda x: 2 if x == -1 else x
    out = np.zeros(1, np.uint8)
    for op, a, b, r in read_golden("f3_tables.txt"):
        va, pa = _p(np.array([byte(int(a))]))
        vb, pb = _p(np.array([byte(int(b))]))
        L.oracle_f3_op(ops[op], pa, pb, 1, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        if out[0] != byte(int(r)):
            return False
    (vec, mag, sgn, _), = read_golden("phi_worked_example.txt")
    v, pv = _p(np.array([int(x) for x in vec.split(",")]))
    planes = np.zeros(2, np.uint64)
    L.oracle_f3_phi(pv, 4, planes.ctypes.data_as(u64p))
    rev = lambda x: int(format(x, "04b")[::-1], 2)
    if planes.tolist() != [rev(int(mag, 16)), rev(int(sgn, 16))]:
        return False
    back = np.zeros(4, np.uint8)
    second_zero = np.array([0b0110, 0b1100], np.uint64)
    L.oracle_f3_psi(second_zero.ctypes.data_as(u64p), 4, back.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if back.tolist() != [0, 1, 2, 0]:
        return False
    g = W.rng(977)
    a, pa = _p(g.integers(0, 3, 300))
    b, pb = _p(g.integers(0, 3, 300))
    if L.oracle_f3_dot(pa, pa, 300) != int((a != 0).sum()):
        return False
    ones, po = _p(np.ones(300))
    if L.oracle_f3_dot(pa, po, 300) != int((a == 1).sum()) - int((a == 2).sum()):
        return False
    return True


def test_unmutated_oracle_passes_f3_pins(tmp_path):
    L = _f3(_build(tmp_path, "original_f3", "#include <stdint.h>", "#include <stdint.h>"))
    assert f3_pins_pass(L)


@pytest.mark.parametrize("name", sorted(F3_MUTANTS))
def test_f3_mutant_is_caught(tmp_path, name):
    old, new = F3_MUTANTS[name]
    L = _f3(_build(tmp_path, name, old, new))
    assert not f3_pins_pass(L), f"planted mistake {name} slipped through the F_3 pins"
