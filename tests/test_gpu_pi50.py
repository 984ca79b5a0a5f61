"""perm(Pi_50) mod 3 on the GPU against the value Section 3.1 reports, as a sharded
run of 64 Gray ranges of 2^44 indices (about 85 s on one MI355X), plus sampled
ranges of the same matrix against the oracle."""
import pytest

import oracle
from conftest import read_golden
from gpu_util import flush_print, oracle_tallies, require_gpu
from paper_2407_20205_amd import longrun
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def test_pi50_sampled_ranges_vs_oracle():
    A = W.pi_matrix(50, "rows")
    ranges = W.sample_chunks(50, seed=50, count=12, log_len=22, unaligned=4)
    want = oracle_tallies(A, ranges)
    for (a, b), w in zip(ranges, want):
        assert P.perm_mod3_range_tally(A, a, b) == w, (a, b)


def test_pi50_published_value(tmp_path):
    n, want = (int(x) for x in read_golden("pi50_mod3.txt")[0])
    A = W.pi_matrix(n, "rows")
    got = longrun.perm_mod3_sharded(A, 64, checkpoint=str(tmp_path / "pi50.json"), log=flush_print)
    assert got == want
