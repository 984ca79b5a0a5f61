"""Helpers for the GPU parity tests (inputs and oracle fan-out; no method arithmetic)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def host_threads() -> int:
    # the GPU machines give one GPU's share of the host: 16 cores
    return max(1, min(16, oracle.default_threads()))


def oracle_tallies(A, ranges):
    """Oracle T(a, b) for each range, ranges spread over host threads (ctypes releases the GIL)."""
    with ThreadPoolExecutor(max_workers=host_threads()) as ex:
        return list(ex.map(lambda r: oracle.range_tally(A, r[0], r[1]), ranges))


def oracle_perms(mats):
    with ThreadPoolExecutor(max_workers=host_threads()) as ex:
        return list(ex.map(lambda M: oracle.perm_mod3(M, threads=1), mats))


def require_gpu():
    import torch
    from paper_2407_20205_amd import perm3 as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    info = P.device_info()
    assert info.arch.decode().startswith("gfx950"), info.arch
    return info


def flush_print(*a):
    print(*a, flush=True)


def to_dev(arr, torch_dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device="cuda", dtype=torch_dtype)
