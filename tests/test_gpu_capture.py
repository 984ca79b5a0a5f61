"""perm_mod3_batch_packed recorded into a caller's graph (torch.cuda.graph): the call adds its
kernels to the caller's capture, and every replay recomputes the results from whatever the input
buffers then hold.  Checked against the oracle on replays with new inputs copied in, with eager
calls into the library and other device work between the replays."""
import numpy as np
import pytest

from gpu_util import flush_print, oracle_perms, require_gpu, to_dev
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def planes_of(mats):
    return np.concatenate([P.perm_mod3_pack(M) for M in mats]).view(np.int64)


def same_orders(b, seed):
    """New uniform matrices with the orders of batch b (the captured call's layout)."""
    g = W.rng(seed)
    return [g.integers(0, 3, size=(int(n), int(n)), dtype=np.uint8) for n in b.ns]


def hist_of(results, ns):
    h = np.zeros((64, 3), np.int64)
    for r, n in zip(results, ns):
        h[int(n), int(r)] += 1
    return h


# (count, n_lo, n_hi): more than 64 matrices (plan, pack and walk kernels); up to 64 walked by
# one launch; up to 64 with more than 2^28 Gray indices (one-launch plan and pack, then the walk)
CASES = [(300, 6, 21, 81), (40, 10, 22, 82), (5, 26, 26, 83)]


@pytest.mark.parametrize("count,n_lo,n_hi,seed", CASES)
def test_packed_batch_in_a_captured_graph(count, n_lo, n_hi, seed):
    import torch
    b = W.batch_uniform(count=count, n_lo=n_lo, n_hi=n_hi, seed=seed)
    planes = to_dev(planes_of(b.mats), torch.int64)
    row_off = np.zeros(count, np.int64)
    row_off[1:] = np.cumsum(b.ns[:-1].astype(np.int64))
    row_off = to_dev(row_off, torch.int64)
    ns = to_dev(b.ns, torch.int32)
    out = torch.zeros(count, dtype=torch.uint8, device="cuda")
    hist = torch.zeros(64 * 3, dtype=torch.int64, device="cuda")
    # an eager call first on a side stream, as torch asks before a capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.perm_mod3_batch_packed(planes, row_off, ns, out, hist, side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.array(oracle_perms(b.mats), np.uint8))

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out.fill_(0xEE)
        hist.zero_()
        P.perm_mod3_batch_packed(planes, row_off, ns, out, hist, torch.cuda.current_stream())
    torch.cuda.synchronize()

    other = W.batch_uniform(count=70, n_lo=4, n_hi=18, seed=seed + 100)
    other_want = np.array(oracle_perms(other.mats), np.uint8)
    for rep in range(3):
        mats = same_orders(b, seed * 10 + rep)
        flush_print(f"replay {rep}: oracle on {count} matrices")
        want = np.array(oracle_perms(mats), np.uint8)
        planes.copy_(to_dev(planes_of(mats), torch.int64))
        graph.replay()
        # eager work beside the replay: another library call and a torch reduction
        o2 = torch.zeros(other.count, dtype=torch.uint8, device="cuda")
        P.perm_mod3_batch_dev(*_bytes_inputs(other), o2, None, torch.cuda.current_stream())
        _ = (torch.arange(1 << 16, device="cuda") * 3).sum().item()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), rep
        assert np.array_equal(hist.cpu().numpy().reshape(64, 3), hist_of(want, b.ns)), rep
        assert np.array_equal(o2.cpu().numpy(), other_want), rep
    del graph


def _bytes_inputs(b):
    import torch
    buf, offs = b.flat()
    return to_dev(buf, torch.uint8), to_dev(offs[:-1], torch.int64), to_dev(b.ns, torch.int32)
