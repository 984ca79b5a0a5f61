"""perm_mod3_batch_packed_noalloc through the C ABI: the same results as perm_mod3_batch_packed
(the entry point it is a variant of) and as the oracle, on consecutive calls that share the
library's static work set, each smaller than the one before; at the size limit; and recorded
into a caller's graph."""
import numpy as np
import pytest

from gpu_util import flush_print, oracle_perms, require_gpu, to_dev
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def packed(b):
    import torch
    planes = np.concatenate([P.perm_mod3_pack(M) for M in b.mats]).view(np.int64)
    row_off = np.zeros(b.count, np.int64)
    row_off[1:] = np.cumsum(b.ns[:-1].astype(np.int64))
    return to_dev(planes, torch.int64), to_dev(row_off, torch.int64), to_dev(b.ns, torch.int32)


def hist_of(results, ns):
    h = np.zeros((64, 3), np.int64)
    for r, n in zip(results, ns):
        h[int(n), int(r)] += 1
    return h


def both(b, stream):
    """(existing entry point's out, hist), (allocation-free out, hist) on the same inputs."""
    import torch
    planes, row_off, ns = packed(b)
    res = []
    for fn in (P.perm_mod3_batch_packed, P.perm_mod3_batch_packed_noalloc):
        out = torch.full((b.count,), 0xEE, dtype=torch.uint8, device="cuda")
        hist = torch.zeros(64 * 3, dtype=torch.int64, device="cuda")
        fn(planes, row_off, ns, out, hist, stream)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), hist.cpu().numpy().reshape(64, 3)))
    return res


# (count, n_lo, n_hi, seed): plan, pack and walk kernels; then up to 64 matrices walked by one
# launch; then one matrix of 2^29 Gray indices (one-launch plan and pack, then the walk)
CALLS = [(1000, 0, 24, 9101), (40, 10, 22, 9102), (1, 29, 29, 9103)]


def test_consecutive_calls_shrinking():
    import torch
    stream = torch.cuda.current_stream()
    for count, lo, hi, seed in CALLS:
        b = W.batch_uniform(count=count, n_lo=lo, n_hi=hi, seed=seed)
        flush_print(f"no-alloc call: {count} matrices, n in {lo}..{hi}")
        want = np.array(oracle_perms(b.mats), np.uint8)
        (oa, ha), (ob, hb) = both(b, stream)
        assert np.array_equal(oa, want)
        assert np.array_equal(ob, oa)
        assert np.array_equal(hb, ha) and np.array_equal(hb, hist_of(want, b.ns))


def test_at_the_limit_then_small():
    import torch
    stream = torch.cuda.current_stream()
    b = W.batch_uniform(count=P.PERM_NOALLOC_MAX_COUNT, n_lo=12, n_hi=22, seed=9104)
    flush_print(f"no-alloc call at the limit: {b.count} matrices")
    (oa, ha), (ob, hb) = both(b, stream)
    assert np.array_equal(ob, oa) and np.array_equal(hb, ha)
    small = [k for k in range(b.count) if b.ns[k] <= 16]
    want = np.array(oracle_perms([b.mats[k] for k in small]), np.uint8)
    assert np.array_equal(ob[small], want)
    c = W.batch_uniform(count=7, n_lo=5, n_hi=20, seed=9105)
    (oa, _), (ob, _) = both(c, None)          # NULL stream
    assert np.array_equal(ob, oa) and np.array_equal(oa, np.array(oracle_perms(c.mats), np.uint8))


def test_over_the_limit_is_refused():
    import torch
    n = P.PERM_NOALLOC_MAX_COUNT + 1
    planes = torch.zeros(2 * n, dtype=torch.int64, device="cuda")
    row_off = torch.zeros(n, dtype=torch.int64, device="cuda")
    ns = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PermError) as e:
        P.perm_mod3_batch_packed_noalloc(planes, row_off, ns, out)
    assert e.value.code == P.PERM_EINVAL


@pytest.mark.parametrize("count,n_lo,n_hi,seed", [(200, 8, 21, 9106), (30, 12, 20, 9107)])
def test_recorded_into_a_graph(count, n_lo, n_hi, seed):
    import torch
    b = W.batch_uniform(count=count, n_lo=n_lo, n_hi=n_hi, seed=seed)
    planes, row_off, ns = packed(b)
    out = torch.zeros(count, dtype=torch.uint8, device="cuda")
    hist = torch.zeros(64 * 3, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.perm_mod3_batch_packed_noalloc(planes, row_off, ns, out, hist, side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out.fill_(0xEE)
        hist.zero_()
        P.perm_mod3_batch_packed_noalloc(planes, row_off, ns, out, hist, torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = W.rng(seed + 1)
    for rep in range(3):
        mats = [g.integers(0, 3, size=(int(n), int(n)), dtype=np.uint8) for n in b.ns]
        want = np.array(oracle_perms(mats), np.uint8)
        planes.copy_(to_dev(np.concatenate([P.perm_mod3_pack(M) for M in mats]).view(np.int64), torch.int64))
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), rep
        assert np.array_equal(hist.cpu().numpy().reshape(64, 3), hist_of(want, b.ns)), rep
        # an eager call between replays uses the same static work set, in stream order
        o2 = torch.zeros(count, dtype=torch.uint8, device="cuda")
        P.perm_mod3_batch_packed_noalloc(planes, row_off, ns, o2, None, torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert np.array_equal(o2.cpu().numpy(), want), rep
    del graph
