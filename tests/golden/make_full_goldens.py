"""Write the full-size expected values of the standard workloads, from the CPU oracle alone.

    python tests/golden/make_full_goldens.py [--only single36|batch|serve] [--threads N]

Inputs come from ``paper_2407_20205_amd/workloads.py`` (seeded random draws, none of the
method's arithmetic); every value written comes from ``oracle/`` (Ryser's identity, eq. (2),
walked in Gray-code order over unpacked residues, Section 3).  Nothing here loads the GPU
library.  Each file records the SHA-256 of the input bytes it was computed from, so a test can
tell a stale golden from a wrong result.

Files (all under tests/golden/):
  full_single36.txt   the 36 x 36 matrix of seed 2: T(0, 2^36) and perm mod 3 = (-1)^36 T mod 3
  full_batch8192.txt  the 8192 matrices of seed 3 (n uniform on 12..28): perm mod 3 of each,
                      and the count of results 0 / 1 / 2 for every n
  full_serve_le28.txt the 20000-request serving trace of seed 4: perm mod 3 of every request
                      with n <= 28 (19157 of them; '-' marks the larger ones)

About 4.4e11 Gray indices in all: under an hour on 8 host cores.
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2407_20205_amd import workloads as W  # noqa: E402


def _write(name: str, lines: list[str]) -> None:
    path = os.path.join(HERE, name)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, path)
    print(f"wrote {path}", flush=True)


def _results_many(mats, threads: int, label: str) -> list[int]:
    """perm mod 3 of every matrix, one single-threaded oracle call per matrix, largest first."""
    order = sorted(range(len(mats)), key=lambda k: -mats[k].shape[0])
    res = [None] * len(mats)
    t0 = time.time()
    done = 0

    def one(k):
        return k, oracle.perm_mod3(mats[k], threads=1)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        for k, r in ex.map(one, order):
            res[k] = r
            done += 1
            if done % 256 == 0 or done == len(order):
                print(f"{label}: {done}/{len(order)} matrices, {time.time() - t0:.0f} s", flush=True)
    return res


def single36(threads: int) -> None:
    A = W.single_36()
    n = A.shape[0]
    t0 = time.time()
    T = oracle.range_tally(A, 0, 1 << n, threads=threads)
    r = oracle.perm_from_tally(n, T)
    print(f"single36: T = {T}, perm mod 3 = {r}, {time.time() - t0:.0f} s", flush=True)
    _write("full_single36.txt", [
        "# The 36 x 36 workload (uniform entries, seed 2, workloads.single_36()) walked over all",
        "# 2^36 Gray indices by the CPU oracle: T(0, 2^36) of Section 3 and perm mod 3 =",
        "# (-1)^n T mod 3 (eq. (2)).  Written by tests/golden/make_full_goldens.py.",
        f"input_sha256 {W.sha256(A)}",
        f"n {n}",
        f"tally {T}",
        f"perm_mod3 {r}",
    ])


def batch(threads: int) -> None:
    b = W.batch_uniform()
    res = _results_many(b.mats, threads, "batch")
    hist = {}
    for n, r in zip(b.ns.tolist(), res):
        hist.setdefault(int(n), [0, 0, 0])[r] += 1
    lines = [
        "# The 8192-matrix workload (seed 3, workloads.batch_uniform(): n uniform on 12..28 drawn",
        "# first, then uniform entries): perm mod 3 of every matrix by the CPU oracle (eq. (2),",
        "# Section 3), and per n the number of results equal to 0, 1 and 2.  Written by",
        "# tests/golden/make_full_goldens.py.",
        f"input_sha256 {W.sha256(b.ns, *b.mats)}",
        f"count {b.count}",
    ]
    digits = "".join(str(r) for r in res)
    for k in range(0, len(digits), 128):
        lines.append(f"results {digits[k:k + 128]}")
    for n in sorted(hist):
        h = hist[n]
        lines.append(f"hist {n} {h[0]} {h[1]} {h[2]}")
    _write("full_batch8192.txt", lines)


def serve(threads: int, n_max: int = 28) -> None:
    tr = W.serve_trace(count=20000)
    idx = [k for k, n in enumerate(tr.ns.tolist()) if n <= n_max]
    res = _results_many([tr.mats[k] for k in idx], threads, "serve")
    chars = ["-"] * len(tr.ns)
    for k, r in zip(idx, res):
        chars[k] = str(r)
    digits = "".join(chars)
    lines = [
        "# The 20000-request serving trace (seed 4, workloads.serve_trace(count=20000); the arrival",
        "# rate changes only the gaps, not n or the matrices): perm mod 3 by the CPU oracle (eq. (2),",
        f"# Section 3) of every request with n <= {n_max}; '-' marks a larger request.  Written by",
        "# tests/golden/make_full_goldens.py.",
        f"input_sha256 {W.sha256(tr.ns, *tr.mats)}",
        f"count {len(tr.ns)}",
        f"n_max {n_max}",
        f"checked {len(idx)}",
    ]
    for k in range(0, len(digits), 128):
        lines.append(f"results {digits[k:k + 128]}")
    _write("full_serve_le28.txt", lines)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["single36", "batch", "serve"], action="append")
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    args = ap.parse_args()
    todo = args.only or ["single36", "batch", "serve"]
    oracle.build(force=False)
    for name in todo:
        {"single36": single36, "batch": batch, "serve": serve}[name](args.threads)


if __name__ == "__main__":
    main()
