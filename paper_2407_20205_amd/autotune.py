"""Tune every class of call on this GPU and write the tuning cache.

    python -m paper_2407_20205_amd.autotune [--out PATH] [--budget-ms MS]

Runs perm_autotune for one matrix of each single-matrix class (n = 20, 28 and 36:
the classes small, mid and large) and perm_autotune_batch on the Monte Carlo batch
(8192 matrices, n uniform on 12..28, packed planes), starting every class from the
library's defaults, then saves the result with perm_tuning_cache_save.  The library
reads ``perm3_tuning.txt`` beside ``libperm3.so`` whenever it makes a device context
(or the file named by PERM3_TUNING_CACHE).  Prints one JSON line per class with
the winner and the search time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "perm3_tuning.txt"))
    ap.add_argument("--budget-ms", type=int, default=20000)
    args = ap.parse_args()

    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2407_20205_amd import perm3 as P
    from paper_2407_20205_amd import workloads as W

    torch.cuda.set_device(0)
    info = P.device_info()
    P.tuning_reset()
    for n, cls in ((20, P.PERM_TUNE_SMALL), (28, P.PERM_TUNE_MID), (36, P.PERM_TUNE_LARGE)):
        t0 = time.perf_counter()
        best = P.autotune(n, args.budget_ms)
        print(json.dumps({"class": P.TUNE_CLASS_NAMES[cls], "n": n, "seconds": time.perf_counter() - t0,
                          "tuning": best.as_dict()}), flush=True)
    b = W.batch_uniform()
    planes = np.concatenate([P.perm_mod3_pack(M) for M in b.mats]).view(np.int64)
    row_off = np.zeros(b.count, np.int64)
    row_off[1:] = np.cumsum(b.ns[:-1].astype(np.int64))
    dev = torch.device("cuda", 0)
    planes_d = torch.from_numpy(planes).to(dev)
    row_off_d = torch.from_numpy(row_off).to(dev)
    ns_d = torch.from_numpy(b.ns.copy()).to(dev)
    out = torch.zeros(b.count, dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    best = P.autotune_batch(planes_d, row_off_d, ns_d, out, 3 * args.budget_ms)
    print(json.dumps({"class": "batch", "workload": "8192 matrices, n uniform on 12..28",
                      "seconds": time.perf_counter() - t0, "tuning": best.as_dict()}), flush=True)
    P.tuning_cache_save(args.out)
    print(f"wrote {args.out} for {info.arch.decode()} with {info.compute_units} CUs", flush=True)


if __name__ == "__main__":
    main()
