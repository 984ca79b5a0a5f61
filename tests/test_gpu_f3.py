"""GPU parity for bitsliced vectors over F_3 (perm_f3_*) against the oracle's definitions.

Bar: bit-exact.  Packed planes equal the oracle's phi word for word; unpacked bytes equal its psi;
every operation's result read back through psi equals the F_3 arithmetic of the oracle (a quotient
by zero excepted); the addition's raw bits equal Table 1; dot products are equal integers.
"""
import numpy as np
import pytest

import oracle
from conftest import read_golden
from gpu_util import flush_print, require_gpu
from paper_2407_20205_amd import perm3 as P
from paper_2407_20205_amd import workloads as W

pytestmark = pytest.mark.gpu

LENGTHS = [1, 2, 63, 64, 65, 127, 1000, 1023, 1024, 1025, 4113, 65536, (1 << 20) + 3]
OPS = [P.PERM_F3_ADD, P.PERM_F3_SUB, P.PERM_F3_MUL, P.PERM_F3_DIV, P.PERM_F3_NEG]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    return require_gpu()


def torch():
    import torch as t
    return t


def to_dev(arr):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(arr)).to("cuda")


def planes_dev(words):
    return torch().zeros(2 * words, dtype=torch().int64, device="cuda")


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


def gpu_pack(v):
    p = planes_dev(P.f3_words(len(v)))
    bad = torch().zeros(1, dtype=torch().int64, device="cuda")
    P.f3_pack(to_dev(v), p, bad)
    torch().cuda.synchronize()
    return p, int(bad.item())


def with_second_zeros(planes, seed):
    """Set the sgn bit of some zero elements: (0, 1) is also 0 (Definition 2.1)."""
    g = W.rng(seed)
    p = planes.copy()
    noise = g.integers(0, 1 << 63, size=len(p) // 2, dtype=np.uint64) * np.uint64(2) + \
        g.integers(0, 2, size=len(p) // 2, dtype=np.uint64)
    p[1::2] |= noise & ~p[0::2]
    return p


@pytest.mark.parametrize("n", LENGTHS)
def test_pack_matches_phi(n):
    v = W.rng(3000 + n).integers(0, 3, n, dtype=np.uint8)
    p, bad = gpu_pack(v)
    want, wbad = oracle.f3_phi(v)
    assert bad == wbad == 0
    assert (host_u64(p) == want).all()


def test_pack_unaligned_with_invalid_bytes():
    g = W.rng(3100)
    base = g.integers(0, 3, 5000, dtype=np.uint8)
    base[[7, 100, 4096]] = [3, 200, 9]
    for off, n in [(3, 4000), (1, 1025), (5, 17)]:
        v = base[off:off + n]
        dv = to_dev(base)[off:off + n]                       # data_ptr not 16-byte aligned
        p = planes_dev(P.f3_words(n))
        bad = torch().zeros(1, dtype=torch().int64, device="cuda")
        P.f3_pack(dv, p, bad)
        torch().cuda.synchronize()
        want, wbad = oracle.f3_phi(v)
        assert int(bad.item()) == wbad and (host_u64(p) == want).all(), (off, n)


@pytest.mark.parametrize("n", LENGTHS)
def test_unpack_matches_psi(n):
    g = W.rng(3200 + n)
    words = P.f3_words(n)
    planes = g.integers(0, 1 << 63, size=2 * words, dtype=np.uint64) * np.uint64(2) + \
        g.integers(0, 2, size=2 * words, dtype=np.uint64)                     # every bit pattern
    t = torch()
    want = oracle.f3_psi(planes, n)
    for off in (5, 16):                                   # an unaligned and an aligned target
        out = t.full((n + 32,), 77, dtype=t.uint8, device="cuda")
        P.f3_unpack(to_dev(planes.view(np.int64)), n, out[off:off + n])
        got = out.cpu().numpy()
        assert (got[off:off + n] == want).all(), off
        assert (got[:off] == 77).all() and (got[off + n:] == 77).all()       # nothing outside written


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", [1, 64, 1000, 4113, (1 << 20) + 3])
def test_ops_match_definition(op, n):
    g = W.rng(3300 + 7 * op + n)
    a = g.integers(0, 3, n, dtype=np.uint8)
    b = g.integers(0, 3, n, dtype=np.uint8)
    pa = with_second_zeros(oracle.f3_phi(a)[0], 1 + n)
    pb = with_second_zeros(oracle.f3_phi(b)[0], 2 + n)
    t = torch()
    da, db = to_dev(pa.view(np.int64)), to_dev(pb.view(np.int64))
    out = planes_dev(P.f3_words(n))
    P.f3_op(op, da, db, out)
    back = t.zeros(n, dtype=t.uint8, device="cuda")
    P.f3_unpack(out, n, back)
    t.cuda.synchronize()
    want = oracle.f3_op(op, a, b)
    keep = want != 0xFF                                  # a quotient by 0 is unspecified
    got_gpu_psi = back.cpu().numpy()
    got_oracle_psi = oracle.f3_psi(host_u64(out), n)
    assert (got_gpu_psi[keep] == want[keep]).all()
    assert (got_oracle_psi[keep] == want[keep]).all()


def test_op_in_place():
    g = W.rng(3400)
    a = g.integers(0, 3, 3000, dtype=np.uint8)
    b = g.integers(0, 3, 3000, dtype=np.uint8)
    da = to_dev(oracle.f3_phi(a)[0].view(np.int64))
    db = to_dev(oracle.f3_phi(b)[0].view(np.int64))
    P.f3_op(P.PERM_F3_MUL, da, db, da)
    P.f3_op(P.PERM_F3_SUB, da, db, db)
    torch().cuda.synchronize()
    ab = oracle.f3_op(oracle.F3_MUL, a, b)
    assert (oracle.f3_psi(host_u64(da), 3000) == ab).all()
    assert (oracle.f3_psi(host_u64(db), 3000) == oracle.f3_op(oracle.F3_SUB, ab, b)).all()


def test_add_bits_match_table1():
    rows = read_golden("table1_addition_truth.txt")
    pa = np.zeros(2, np.uint64)
    pb = np.zeros(2, np.uint64)
    for i, r in enumerate(rows):
        m1, s1, m2, s2 = (int(x) for x in r[1:5])
        pa[0] |= np.uint64(m1 << i); pa[1] |= np.uint64(s1 << i)
        pb[0] |= np.uint64(m2 << i); pb[1] |= np.uint64(s2 << i)
    out = planes_dev(1)
    P.f3_op(P.PERM_F3_ADD, to_dev(pa.view(np.int64)), to_dev(pb.view(np.int64)), out)
    o = host_u64(out)
    for i, r in enumerate(rows):
        assert [int(o[0] >> np.uint64(i)) & 1, int(o[1] >> np.uint64(i)) & 1] == [int(r[5]), int(r[6])], r


@pytest.mark.parametrize("n", [0, 1, 63, 65, 1000, 4113, (1 << 20) + 3, (1 << 26) + 5])
def test_dot_matches_definition(n):
    g = W.rng(3500 + n)
    a = g.integers(0, 3, n, dtype=np.uint8)
    b = g.integers(0, 3, n, dtype=np.uint8)
    t = torch()
    s = t.full((1,), 12345, dtype=t.int64, device="cuda")   # overwritten, not added to
    pa, _ = gpu_pack(a) if n else (planes_dev(0), 0)
    pb, _ = gpu_pack(b) if n else (planes_dev(0), 0)
    P.f3_dot(pa, pb, s)
    assert int(s.item()) == oracle.f3_dot(a, b)


def test_full_size_sampled():
    """2^32 elements, the size the benchmark times: sampled elements of every result against
    the oracle, the dot product against the oracle in full."""
    t = torch()
    n = 1 << 32
    gen = t.Generator(device="cuda")
    gen.manual_seed(3600)
    flush_print("drawing two vectors of 2^32 bytes on the device")
    va = t.randint(0, 3, (n,), dtype=t.uint8, device="cuda", generator=gen)
    vb = t.randint(0, 3, (n,), dtype=t.uint8, device="cuda", generator=gen)
    words = P.f3_words(n)
    pa, pb, po = planes_dev(words), planes_dev(words), planes_dev(words)
    bad = t.zeros(1, dtype=t.int64, device="cuda")
    P.f3_pack(va, pa, bad)
    P.f3_pack(vb, pb, bad)
    s = t.zeros(1, dtype=t.int64, device="cuda")
    P.f3_dot(pa, pb, s)
    back = t.empty(n, dtype=t.uint8, device="cuda")
    idx = t.from_numpy(W.rng(3601).integers(0, n, 4096)).to("cuda")
    a_s, b_s = va[idx].cpu().numpy(), vb[idx].cpu().numpy()
    for op in OPS:
        P.f3_op(op, pa, pb, po)
        P.f3_unpack(po, n, back)
        got = back[idx].cpu().numpy()
        want = oracle.f3_op(op, a_s, b_s)
        keep = want != 0xFF
        assert (got[keep] == want[keep]).all(), op
    assert int(bad.item()) == 0
    flush_print("oracle dot product over 2^32 elements")
    assert int(s.item()) == oracle.f3_dot(va.cpu().numpy(), vb.cpu().numpy())


def test_argument_errors():
    t = torch()
    p = planes_dev(4)
    with pytest.raises(P.PermError) as e:
        P.f3_op(9, p, p, p)
    assert e.value.code == P.PERM_EINVAL
    with pytest.raises(P.PermError) as e:
        P.f3_op(P.PERM_F3_ADD, p[1:], p[1:], p[1:], words=1)      # 8-byte aligned only
    assert e.value.code == P.PERM_EINVAL
    with pytest.raises(P.PermError) as e:
        P.f3_unpack(p, -1, t.zeros(4, dtype=t.uint8, device="cuda"))
    assert e.value.code == P.PERM_EINVAL
    P.f3_op(P.PERM_F3_NEG, p, None, p)                             # b may be null for negation
    P.f3_op(P.PERM_F3_ADD, p, p, p, words=0)                       # nothing to do
