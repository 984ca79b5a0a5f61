"""Pins for the oracle's census generators (CPU only)."""
import math

import pytest

import oracle
from conftest import read_golden


def test_enumeration_reproduces_table3():
    z = {int(r[0]): int(r[1]) for r in read_golden("table3_zero_counts.txt")}
    for n in (1, 2, 3):
        c = oracle.census(n, 0, 0, 0, 3 ** (n * n))
        assert c[0] == z[n] and c[1] == c[2] and sum(c) == 3 ** (n * n)
        assert c == oracle.count_by_value(n)


def test_enumeration_ranges_add_up():
    whole = oracle.census(3, 0, 0, 0, 3 ** 9)
    parts = [oracle.census(3, 0, 0, a, b - a) for a, b in [(0, 5000), (5000, 5001), (5001, 3 ** 9)]]
    assert tuple(map(sum, zip(*parts))) == whole


def test_splitmix64_reference_output():
    # the first output of the reference SplitMix64 generator from state 0
    assert oracle.splitmix64(0, 1) == 0xE220A8397B1DCDAF
    # consecutive outputs advance the state by the golden-ratio increment
    assert oracle.splitmix64(0x9E3779B97F4A7C15, 1) == oracle.splitmix64(0, 2)


def test_random_trits_are_uniform_and_match_table4_n6():
    # 10^5 uniform 6 x 6 matrices: the zero fraction agrees with Table 4's 0.35456
    # (10^11 trials) within 4 standard errors
    c = oracle.census(6, 1, 2024, 0, 100000)
    p = c[0] / sum(c)
    assert abs(p - 35456365448 / 1e11) < 4 * math.sqrt(0.3546 * 0.6454 / 1e5)
    assert abs(c[1] - c[2]) < 4 * math.sqrt(c[1] + c[2])          # 1 and -1 equally likely
