"""GPU census (matrices made on the device) against the oracle, exactly, and the
published exact counts of Table 3."""
import pytest

import oracle
from conftest import read_golden
from gpu_util import flush_print, require_gpu
from paper_2407_20205_amd import perm3 as P

pytestmark = pytest.mark.gpu

ENUM, SPLIT = P.PERM_GEN_ENUMERATE, P.PERM_GEN_SPLITMIX


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def z_table():
    return {int(r[0]): int(r[1]) for r in read_golden("table3_zero_counts.txt")}


def test_enumeration_small_n_exact():
    z = z_table()
    for n in (1, 2, 3, 4):
        c = P.perm_mod3_census(n, ENUM, 0, 0, 3 ** (n * n))
        assert c[0] == z[n] and c[1] == c[2] and sum(c) == 3 ** (n * n), (n, c)
    assert P.perm_mod3_census(3, ENUM, 0, 0, 3 ** 9) == oracle.census(3, 0, 0, 0, 3 ** 9)


def test_enumeration_n5_ranges_vs_oracle():
    for a, cnt in [(0, 200000), (123456789, 300000), (3 ** 25 - 100000, 100000)]:
        assert P.perm_mod3_census(5, ENUM, 0, a, cnt) == oracle.census(5, 0, 0, a, cnt), a


def test_enumeration_ranges_every_order_vs_oracle():
    """Enumeration is walked 27 consecutive matrices a lane: ranges that start and end inside a
    group of 27, single matrices, one group exactly, ranges up to the last matrix, every n."""
    for n in range(1, 7):
        total = 3 ** (n * n)
        ranges = [(0, min(total, 1)), (0, min(total, 27)), (min(total - 1, 26), 1)]
        if total > 100:
            ranges += [(5, 50), (27 * 11 + 13, 40), (total // 2 + 7, min(20000, total // 3)),
                       (total - 61, 61), (total - 27, 27)]
        for a, cnt in ranges:
            got = P.perm_mod3_census(n, ENUM, 0, a, cnt)
            assert sum(got) == cnt
            assert got == oracle.census(n, 0, 0, a, cnt), (n, a, cnt)


def test_random_matrices_vs_oracle():
    for n, cnt in [(1, 1000), (2, 5000), (5, 50000), (8, 50000), (11, 20000), (14, 5000), (17, 600), (20, 100)]:
        assert P.perm_mod3_census(n, SPLIT, 77 + n, 1000, cnt) == oracle.census(n, 1, 77 + n, 1000, cnt), n
    # sizes that go through device generation and the batch walk
    for n, cnt in [(21, 60), (22, 40)]:
        flush_print(f"census n={n}")
        assert P.perm_mod3_census(n, SPLIT, 5 + n, 0, cnt) == oracle.census(n, 1, 5 + n, 0, cnt), n


def test_random_matrices_every_lane_order_vs_oracle():
    """Every order the lanes walk: up to 8 with every index tested, from 9 on through the
    block filter and the wave's re-walk lists; counts over thousands of matrices."""
    sizes = {3: 20000, 4: 20000, 6: 20000, 7: 20000, 8: 20000, 9: 20000, 10: 20000,
             12: 8000, 13: 4000, 15: 1500, 16: 800, 18: 200, 19: 120}
    for n, cnt in sizes.items():
        assert P.perm_mod3_census(n, SPLIT, 300 + n, 17, cnt) == oracle.census(n, 1, 300 + n, 17, cnt), n


def test_single_matrices_vs_oracle():
    """One matrix per call, so each count is that matrix's own perm mod 3."""
    for n in (8, 9, 10, 14, 17, 20):
        for t in (0, 1, 5, 1000003):
            got = P.perm_mod3_census(n, SPLIT, 9000 + n, t, 1)
            assert sum(got) == 1
            assert got == oracle.census(n, 1, 9000 + n, t, 1), (n, t)


def test_exact_z5_table3():
    """All 3^25 = 847,288,609,443 matrices 5 x 5 over F_3, walked on the device."""
    z = z_table()
    flush_print("census of all 5x5 matrices")
    c = P.perm_mod3_census(5, ENUM, 0, 0, 3 ** 25)
    assert c[0] == z[5] == 317193401763
    assert c[1] == c[2] and sum(c) == 3 ** 25
