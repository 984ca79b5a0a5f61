"""Long runs: one matrix's Gray range split into shards, with a checkpoint file.

The range [0, 2^n) is cut into equal shards; each shard's exact partial
tally T(a, b) is computed by ``tally_fn`` (by default the library's
``perm_mod3_range_tally``) and recorded in a JSON checkpoint together with
the matrix hash, so an interrupted run resumes where it stopped and a
checkpoint of another matrix is refused.  This module only does that
bookkeeping: the shard tallies are summed and reduced, (-1)^n times their
sum mod 3 (Section 3.1's blocks of consecutive Gray states, eq. (2)), by
``finish_fn``, by default the library's ``perm_mod3_from_tallies``, which
does it on the device.  A shard is also exactly what one GPU of several
would take.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Callable

import numpy as np


def matrix_hash(A: np.ndarray) -> str:
    A = np.ascontiguousarray(A, dtype=np.uint8)
    return hashlib.sha256(A.tobytes() + str(A.shape).encode()).hexdigest()


def shard_bounds(n: int, shards: int, k: int) -> tuple[int, int]:
    total = 1 << n
    return total * k // shards, total * (k + 1) // shards


def _save(path: str, state: dict) -> None:
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(state, f)
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def sharded_tallies(A, shards: int, tally_fn: Callable | None = None, checkpoint: str | None = None,
                    log: Callable | None = None) -> list[int]:
    """The tally of every shard of A, in shard order; resumes from ``checkpoint`` if it exists."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    n = A.shape[0]
    if shards < 1 or shards > (1 << n):
        raise ValueError("shards must be in [1, 2^n]")
    if tally_fn is None:
        from . import perm3
        tally_fn = perm3.perm_mod3_range_tally
    h = matrix_hash(A)
    state = {"sha256": h, "n": n, "shards": shards, "done": {}}
    if checkpoint and os.path.exists(checkpoint):
        with open(checkpoint) as f:
            old = json.load(f)
        if old.get("sha256") != h or old.get("n") != n or old.get("shards") != shards:
            raise ValueError(f"checkpoint {checkpoint} belongs to another matrix or sharding")
        state = old
    for k in range(shards):
        if str(k) in state["done"]:
            continue
        a, b = shard_bounds(n, shards, k)
        t0 = time.perf_counter()
        state["done"][str(k)] = int(tally_fn(A, a, b))
        if checkpoint:
            _save(checkpoint, state)
        if log:
            log(f"shard {k + 1}/{shards} [{a}, {b}) tally {state['done'][str(k)]} "
                f"in {time.perf_counter() - t0:.2f} s")
    return [int(state["done"][str(k)]) for k in range(shards)]


def perm_mod3_sharded(A, shards: int, finish_fn: Callable | None = None, **kw) -> int:
    """perm(A) mod 3 in {0, 1, 2} from a sharded, checkpointed run; ``finish_fn(n, tallies)``
    reduces the shard tallies (default: the library's perm_mod3_from_tallies)."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    tallies = sharded_tallies(A, shards, **kw)
    if finish_fn is None:
        from . import perm3
        finish_fn = perm3.perm_mod3_from_tallies
    return int(finish_fn(A.shape[0], tallies))
