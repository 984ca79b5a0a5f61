"""The full-size expected values under tests/golden/ (written by make_full_goldens.py from the CPU
oracle alone) checked without a GPU: their inputs are still the ones the workloads generate (input
SHA-256), the batch histogram is the count of its own results by n, the serving file marks exactly
the requests of order above 28, and a sample of the stored results is recomputed by the oracle
here: every batch matrix and serving request of order up to 16, and a few larger ones."""
import numpy as np
import pytest

import oracle
from conftest import read_golden
from paper_2407_20205_amd import workloads as W


def kv(name):
    out = {}
    for row in read_golden(name):
        key, vals = row[0], row[1:]
        if key in ("results", "hist"):
            out.setdefault(key, []).append(vals)
        else:
            out[key] = vals[0]
    return out


def test_single36_golden_input():
    g = kv("full_single36.txt")
    A = W.single_36()
    assert g["input_sha256"] == W.sha256(A) and int(g["n"]) == 36
    T = int(g["tally"])
    assert abs(T) < 1 << 36
    assert int(g["perm_mod3"]) == oracle.perm_from_tally(36, T)


def test_batch_golden_consistent_and_sampled():
    g = kv("full_batch8192.txt")
    b = W.batch_uniform()
    assert g["input_sha256"] == W.sha256(b.ns, *b.mats)
    res = np.array([int(c) for c in "".join(r[0] for r in g["results"])], np.uint8)
    assert res.size == b.count == int(g["count"]) and set(np.unique(res)) <= {0, 1, 2}
    hist = {int(r[0]): [int(x) for x in r[1:]] for r in g["hist"]}
    for n in range(12, 29):
        got = [int(np.count_nonzero((b.ns == n) & (res == v))) for v in range(3)]
        assert hist[n] == got, n
    rng = W.rng(77)
    sample = [k for k in range(b.count) if b.ns[k] <= 16]
    sample += [int(k) for k in rng.choice(np.flatnonzero(b.ns >= 17), size=6, replace=False)]
    for k in sample:
        assert res[k] == oracle.perm_mod3(b.mats[k], threads=4), (k, int(b.ns[k]))


def test_serve_golden_consistent_and_sampled():
    g = kv("full_serve_le28.txt")
    tr = W.serve_trace(count=int(g["count"]))
    assert g["input_sha256"] == W.sha256(tr.ns, *tr.mats)
    digits = "".join(r[0] for r in g["results"])
    assert len(digits) == len(tr.ns)
    for k, n in enumerate(tr.ns.tolist()):
        assert (digits[k] == "-") == (n > int(g["n_max"])), k
    assert sum(ch != "-" for ch in digits) == int(g["checked"])
    small = [k for k, n in enumerate(tr.ns.tolist()) if n <= 16]
    for k in small[:: max(1, len(small) // 2000)]:
        assert int(digits[k]) == oracle.perm_mod3(tr.mats[k], threads=1), k
