"""The binding refuses device-call arguments that would send the kernels outside their buffers
(CPU only: every check fires before any C call, so no GPU is needed)."""
import numpy as np
import pytest
import torch

from paper_2407_20205_amd import perm3 as P


def batch_args(count=5, ns_dtype=torch.int32, out_len=None, hist_len=192, hist_dtype=torch.int64):
    ns = torch.full((count,), 12, dtype=ns_dtype)
    offs = torch.zeros(count, dtype=torch.int64)
    mats = torch.zeros(count * 144, dtype=torch.uint8)
    out = torch.zeros(count if out_len is None else out_len, dtype=torch.uint8)
    hist = None if hist_len is None else torch.zeros(hist_len, dtype=hist_dtype)
    return mats, offs, ns, out, hist


@pytest.mark.parametrize("call", [P.perm_mod3_batch_dev, P.perm_mod3_batch_packed])
def test_batch_calls_check_their_tensors(call):
    packed = call is not P.perm_mod3_batch_dev
    mats, offs, ns, out, hist = batch_args()
    first = torch.zeros(2 * 60, dtype=torch.int64) if packed else mats
    # torch's default int64 for the orders would be read as pairs of int32
    with pytest.raises(ValueError, match="ns_dev must have dtype"):
        call(first, offs, ns.to(torch.int64), out, hist)
    with pytest.raises(ValueError, match="(mats_dev|planes_dev) must have dtype"):
        call(first.to(torch.int32), offs, ns, out, hist)
    with pytest.raises(ValueError, match="(offs_dev|row_off_dev) must have dtype"):
        call(first, offs.to(torch.int32), ns, out, hist)
    with pytest.raises(ValueError, match="(offs_dev|row_off_dev) holds 4 elements"):
        call(first, offs[:4], ns, out, hist)
    with pytest.raises(ValueError, match="out_dev holds 3 elements"):
        call(first, offs, ns, out[:3], hist)
    with pytest.raises(ValueError, match="out_dev must have dtype"):
        call(first, offs, ns, out.to(torch.int32), hist)
    with pytest.raises(ValueError, match="hist_dev holds 191 elements"):
        call(first, offs, ns, out, hist[:191])
    with pytest.raises(ValueError, match="hist_dev must have dtype"):
        call(first, offs, ns, out, hist.to(torch.int32))
    with pytest.raises(ValueError, match="must be contiguous"):
        call(first, torch.zeros(10, dtype=torch.int64)[::2], ns, out, hist)
    # well-formed tensors that are not on a GPU
    with pytest.raises(ValueError, match="must be on a CUDA device"):
        call(first, offs, ns, out, hist)
    with pytest.raises(ValueError, match="must be on a CUDA device"):
        call(first, offs, ns, out, None)
    with pytest.raises(ValueError, match="must be a torch tensor"):
        call(first, np.zeros(5, np.int64), ns, out, None)


def test_vector_calls_check_their_tensors():
    v = torch.zeros(130, dtype=torch.uint8)
    planes = torch.zeros(2 * P.f3_words(130), dtype=torch.int64)
    with pytest.raises(ValueError, match="planes_dev holds 4 elements"):
        P.f3_pack(v, planes[:4])
    with pytest.raises(ValueError, match="v_dev must have dtype"):
        P.f3_pack(v.to(torch.int32), planes)
    with pytest.raises(ValueError, match="invalid_dev holds 0 elements"):
        P.f3_pack(v, planes, torch.zeros(0, dtype=torch.int64))
    with pytest.raises(ValueError, match="must be on a CUDA device"):
        P.f3_pack(v, planes)
    with pytest.raises(ValueError, match="v_dev holds 130 elements; the call needs at least 131"):
        P.f3_unpack(planes, 131, v)
    with pytest.raises(ValueError, match="planes_dev holds 6 elements; the call needs at least 8"):
        P.f3_unpack(planes, 193, torch.zeros(200, dtype=torch.uint8))
    a = torch.zeros(8, dtype=torch.int64)
    with pytest.raises(ValueError, match="b_dev holds 6 elements"):
        P.f3_op(P.PERM_F3_ADD, a, a[:6], a)
    with pytest.raises(ValueError, match="out_dev must have dtype"):
        P.f3_op(P.PERM_F3_MUL, a, a, a.to(torch.float32))
    with pytest.raises(ValueError, match="a_dev holds 8 elements; the call needs at least 10"):
        P.f3_op(P.PERM_F3_ADD, a, a, a, words=5)
    with pytest.raises(ValueError, match="must be on a CUDA device"):
        P.f3_op(P.PERM_F3_NEG, a, None, a)
    with pytest.raises(ValueError, match="sum_dev must have dtype"):
        P.f3_dot(a, a, torch.zeros(1, dtype=torch.int32))
    with pytest.raises(ValueError, match="sum_dev holds 0 elements"):
        P.f3_dot(a, a, torch.zeros(0, dtype=torch.int64))
