"""CPU pins of the oracle's vectors over F_3 (Section 2's phi and psi, the arithmetic behind
Theorem 2.1).  The elementwise operations are pinned to the field's tables written out by hand
(tests/golden/f3_tables.txt), phi to the worked example of Section 2, the dot product to closed
forms."""
import numpy as np
import pytest

import oracle
from conftest import read_golden
from paper_2407_20205_amd import workloads as W

OPS = {"add": oracle.F3_ADD, "sub": oracle.F3_SUB, "mul": oracle.F3_MUL, "div": oracle.F3_DIV}


def byte(x: int) -> int:
    return 2 if x == -1 else x


def test_tables():
    rows = read_golden("f3_tables.txt")
    assert len(rows) == 9 * 3 + 6
    for op, a, b, r in rows:
        got = oracle.f3_op(OPS[op], [byte(int(a))], [byte(int(b))])
        assert got[0] == byte(int(r)), (op, a, b)
    for x in (-1, 0, 1):
        assert oracle.f3_op(oracle.F3_NEG, [byte(x)])[0] == byte(-x)


def test_division_by_zero_is_flagged():
    assert list(oracle.f3_op(oracle.F3_DIV, [0, 1, 2], [0, 0, 0])) == [0xFF] * 3


def test_phi_worked_example():
    # Section 2 stores (1, 1, 0, -1) as (0xd, 0x1) with element i (1-based) at bit n - i; the vector
    # layout puts element e (0-based) at bit e, i.e. the same bits reversed over the 4 positions
    (vec, mag, sgn, _), = read_golden("phi_worked_example.txt")
    v = [int(x) for x in vec.split(",")]
    planes, bad = oracle.f3_phi(v)
    rev = lambda x: int(format(x, "04b")[::-1], 2)
    assert bad == 0 and planes.tolist() == [rev(int(mag, 16)), rev(int(sgn, 16))]


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 200, 1000])
def test_psi_inverts_phi(n):
    v = W.rng(20 + n).integers(0, 3, n, dtype=np.uint8)
    planes, bad = oracle.f3_phi(v)
    assert bad == 0 and len(planes) == 2 * ((n + 63) // 64)
    assert (oracle.f3_psi(planes, n) == v).all()
    # bits at and above n stay zero
    if n % 64:
        assert int(planes[-2]) >> (n % 64) == 0 and int(planes[-1]) >> (n % 64) == 0


def test_phi_counts_invalid_bytes():
    v = np.array([0, 1, 2, 3, 255, 1, 7], dtype=np.uint8)
    planes, bad = oracle.f3_phi(v)
    assert bad == 3
    assert list(oracle.f3_psi(planes, 7)) == [0, 1, 2, 0, 0, 1, 0]


def test_psi_reads_the_second_zero():
    # (0, 1) is also 0 (Definition 2.1)
    planes = np.array([0b0110, 0b1100], dtype=np.uint64)
    assert list(oracle.f3_psi(planes, 4)) == [0, 1, 2, 0]


def test_field_laws_on_vectors():
    g = W.rng(30)
    a, b, c = (g.integers(0, 3, 500, dtype=np.uint8) for _ in range(3))
    add = lambda x, y: oracle.f3_op(oracle.F3_ADD, x, y)
    mul = lambda x, y: oracle.f3_op(oracle.F3_MUL, x, y)
    assert (add(a, b) == add(b, a)).all() and (mul(a, b) == mul(b, a)).all()
    assert (add(add(a, b), c) == add(a, add(b, c))).all()
    assert (mul(a, add(b, c)) == add(mul(a, b), mul(a, c))).all()
    assert (oracle.f3_op(oracle.F3_SUB, a, b) == add(a, oracle.f3_op(oracle.F3_NEG, b))).all()
    nz = b != 0
    q = oracle.f3_op(oracle.F3_DIV, a, b)
    assert (mul(q[nz], b[nz]) == a[nz]).all() and (q[~nz] == 0xFF).all()


def test_dot_closed_forms():
    g = W.rng(31)
    for n in (0, 1, 77, 1000):
        a = g.integers(0, 3, n, dtype=np.uint8)
        b = g.integers(0, 3, n, dtype=np.uint8)
        assert oracle.f3_dot(a, a) == int((a != 0).sum())                 # x^2 = 1 for x = +-1
        ones = np.ones(n, dtype=np.uint8)
        assert oracle.f3_dot(a, ones) == int((a == 1).sum()) - int((a == 2).sum())
        assert oracle.f3_dot(a, b) == oracle.f3_dot(b, a)
        assert oracle.f3_dot(a, oracle.f3_op(oracle.F3_NEG, b)) == -oracle.f3_dot(a, b)
