"""Host logic of long runs (CPU only): the digits of pi behind the Pi_n matrix,
and sharded tallies with checkpoint / resume, using the oracle as the tally."""
import json

import numpy as np
import pytest

import oracle
from paper_2407_20205_amd import longrun
from paper_2407_20205_amd import workloads as W


def _atan_inv_series(q, scale):
    # arctan(1/q) * scale, summed term by term with explicit signs
    s, power, k, sign = 0, scale // q, 1, 1
    while power:
        s += sign * (power // k)
        power //= q * q
        k += 2
        sign = -sign
    return s


def test_pi_digits_agree_with_stormer_formula():
    # Stormer: pi/4 = 44 atan(1/57) + 7 atan(1/239) - 12 atan(1/682) + 24 atan(1/12943)
    count = 2600
    scale = 10 ** (count + 12)
    pi = 4 * (44 * _atan_inv_series(57, scale) + 7 * _atan_inv_series(239, scale)
              - 12 * _atan_inv_series(682, scale) + 24 * _atan_inv_series(12943, scale))
    assert W.pi_digits(count) == str(pi)[:count]
    assert W.pi_digits(count).startswith("3")


def test_pi_matrix_readings():
    d = W.pi_digits(2600)
    A = W.pi_matrix(50, "rows")
    B = W.pi_matrix(50, "formula")
    assert A.shape == B.shape == (50, 50)
    # first row: the first 50 digits, reduced mod 3, in both readings
    assert [int(x) for x in A[0]] == [int(c) % 3 for c in d[:50]]
    assert np.array_equal(A[0], B[0])
    # "rows": row i starts at digit 50 i + 1; "formula": at digit 49 i + 1
    assert [int(x) for x in A[7]] == [int(c) % 3 for c in d[350:400]]
    assert [int(x) for x in B[7]] == [int(c) % 3 for c in d[343:393]]


def oracle_finish(n, tallies):
    return oracle.perm_from_tally(n, sum(tallies))


def test_sharded_tallies_match_whole_range(tmp_path):
    A = W.uniform_matrix(14, 8)
    whole = oracle.range_tally(A, 0, 1 << 14)
    for shards in (1, 3, 16, 100):
        ts = longrun.sharded_tallies(A, shards, tally_fn=oracle.range_tally)
        assert len(ts) == shards and sum(ts) == whole
        assert ts == [oracle.range_tally(A, *longrun.shard_bounds(14, shards, k)) for k in range(shards)]
    got = longrun.perm_mod3_sharded(A, 7, tally_fn=oracle.range_tally, finish_fn=oracle_finish)
    assert got == oracle.perm_mod3(A)


def test_checkpoint_resume_after_interruption(tmp_path):
    A = W.uniform_matrix(13, 9)
    ck = str(tmp_path / "ck.json")
    calls = []

    class Interrupted(Exception):
        pass

    def flaky(M, a, b):
        calls.append((a, b))
        if len(calls) == 5:
            raise Interrupted()
        return oracle.range_tally(M, a, b)

    with pytest.raises(Interrupted):
        longrun.sharded_tallies(A, 12, tally_fn=flaky, checkpoint=ck)
    state = json.load(open(ck))
    assert len(state["done"]) == 4                # four shards were saved before the failure
    calls.clear()
    ts = longrun.sharded_tallies(A, 12, tally_fn=lambda M, a, b: (calls.append((a, b)), oracle.range_tally(M, a, b))[1],
                                 checkpoint=ck)
    assert len(calls) == 8                         # only the missing shards ran again
    assert sum(ts) == oracle.range_tally(A, 0, 1 << 13)
    # a checkpoint of another matrix or sharding is refused
    with pytest.raises(ValueError):
        longrun.sharded_tallies(W.uniform_matrix(13, 10), 12, tally_fn=oracle.range_tally, checkpoint=ck)
    with pytest.raises(ValueError):
        longrun.sharded_tallies(A, 11, tally_fn=oracle.range_tally, checkpoint=ck)


def test_shard_bounds_cover_the_range():
    for n, s in [(5, 1), (5, 3), (10, 7), (40, 64)]:
        pts = [longrun.shard_bounds(n, s, k) for k in range(s)]
        assert pts[0][0] == 0 and pts[-1][1] == 1 << n
        assert all(pts[k][1] == pts[k + 1][0] for k in range(s - 1))


def test_checkpoint_directory_is_made(tmp_path):
    A = W.uniform_matrix(10, 64)
    ck = str(tmp_path / "not" / "yet" / "ck.json")
    tallies = longrun.sharded_tallies(A, 4, tally_fn=oracle.range_tally, checkpoint=ck)
    assert sum(tallies) == oracle.range_tally(A, 0, 1 << 10)

    def never(*args):
        raise AssertionError("a resumed run walked a shard again")

    assert longrun.sharded_tallies(A, 4, tally_fn=never, checkpoint=ck) == tallies
