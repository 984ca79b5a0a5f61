"""Benchmark: perm(A) mod 3 by the bipedal Gray-code Ryser sum on one MI355X.

Headline (one step = one whole pass of the method over one 36 x 36 matrix
already resident in HBM: validate + pack, plan, Gray walk, reduce, mod 3):
Ryser subset-terms per second, 2^36 - 1 terms per step.  The same JSON line
carries the walk kernel's roofline position (integer VALU bound), the CPU
oracle timed on this host, the batched Monte Carlo workload (8192 matrices,
n = 12..28, one persistent launch) against one launch per matrix, and the
serving stream (20000 requests, n = 8..40, Poisson arrivals) with p50/p99
latency against FIFO one-launch-per-request.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only headline|batch|serve|large|wide|...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np


def input_sha256(*arrays) -> str:
    """SHA-256 of the generated uint8 matrices, in order, so any run can be matched to the oracle's inputs."""
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.uint8).tobytes())
    return h.hexdigest()

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vector ALU: 128 32-bit lane-ops per clock per CU (the lane rate behind the
# published 157.3 TFLOP/s fp32 vector figure: 157.3e12 / 2 flops / 256 CUs / 2.4 GHz),
# 256 CUs, 2.4 GHz
PEAK_LANE_OPS = 256 * 128 * 2.4e9
# lane-ops the walk needs per Gray index on gfx950, in blocks of 16 indices whose subset
# sums are H + L_k (H the block's sum over rows 4 .. n-1, L_k fixed sums of rows 0 .. 3):
# the 32-bit low mag word of each of the 15 states with k >= 1 in two 3-input bitwise
# ops, one 3-input max per two of the block's 16 mag words to find candidates, and one
# Gray step (three 3-input ops) moving H to the next block; the sign and the high word
# only for candidates
OPS_PER_TERM = (2 * 15 + 15 / 2 + 3) / 16
# a chained Gray step's count (three 3-input ops carry mag and sgn of the low word from
# one index to the next, plus half a max): the walk's count before it was cut into
# blocks of independent states, reported beside as gray_step_frac
GRAY_STEP_OPS_PER_TERM = 3.5
# the paper's count for a two-word (n = 33..64 on 32-bit lanes) step: 6 bitwise ops
# per word for the add/sub plus one compare per word
PAPER_OPS_PER_TERM_2W = 14


def walk_counters():
    """The committed counter passes of the 36x36 walk (profiles/k_walk_36x36_counters.json), or None
    once the kernel source differs from the profiled one."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_walk_36x36_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    h = hashlib.sha256()
    for name in ("perm3_walk.hpp", "perm3_kernels.hip"):
        with open(os.path.join(ROOT, "paper_2407_20205_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return d if h.hexdigest() == d.get("source_sha256") else None


def measured_traffic():
    """HBM bytes per walk launch (FETCH_SIZE and WRITE_SIZE, each scaled by a 256 MiB copy)."""
    d = walk_counters()
    return d["traffic_bytes_per_launch"] if d else None


GOLDEN = os.path.join(ROOT, "tests", "golden")
GOLDEN_MISMATCH = []   # names of workloads whose results differ from the oracle's stored ones


def read_golden(name):
    """A stored expected-value file (written by tests/golden/make_full_goldens.py from the CPU oracle
    alone): 'key value' lines, the repeated 'results' and 'hist' keys collected in lists."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition(" ")
            if key in ("results", "hist"):
                out.setdefault(key, []).append(val)
            else:
                out[key] = val
    return out


def check_golden(name, same, detail):
    """Record whether a workload's results equal the oracle's stored ones."""
    if not same:
        GOLDEN_MISMATCH.append(name)
        log(f"ERROR: {name} differs from the oracle's expected values in tests/golden/")
    return {"file": "tests/golden/" + name, "match": bool(same), **detail}


def tuning_info(P, cls):
    """Which tuning a class of call runs with: its source (default, cache, set, autotune) and values."""
    t, src = P.tuning_get_class(cls)
    return {"class": P.TUNE_CLASS_NAMES[cls], "source": P.TUNE_SOURCE_NAMES[src], "values": t.as_dict()}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(x, q):
    return float(np.percentile(np.asarray(x, dtype=np.float64), q)) if len(x) else float("nan")


# ------------------------------------------------------------------ headline

def bench_headline(P, W, torch, steps, warmup):
    A = W.single_36()
    n = 36
    terms = (1 << n) - 1
    dev = torch.device("cuda", 0)
    mats = torch.from_numpy(A.reshape(-1).copy()).to(dev)
    offs = torch.zeros(1, dtype=torch.int64, device=dev)
    ns = torch.full((1,), n, dtype=torch.int32, device=dev)
    out = torch.zeros(1, dtype=torch.uint8, device=dev)
    P.timing_enable(True)
    for _ in range(warmup):
        P.perm_mod3_batch_dev(mats, offs, ns, out)
    torch.cuda.synchronize()
    hot = []
    total = []
    t0 = time.perf_counter()
    for _ in range(steps):
        P.perm_mod3_batch_dev(mats, offs, ns, out)
        t = P.timing_last()           # waits for this step's events on the library stream
        hot.append(t.hot_kernel_ms)
        total.append(t.total_ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.timing_enable(False)
    result = int(out.item())
    g = read_golden("full_single36.txt")
    golden = check_golden("full_single36.txt",
                          g["input_sha256"] == W.sha256(A) and result == int(g["perm_mod3"]),
                          {"oracle_tally": int(g["tally"]), "oracle_perm_mod3": int(g["perm_mod3"])})
    sec = t1 - t0
    hot_s = float(np.mean(hot)) * 1e-3
    achieved = OPS_PER_TERM * terms / hot_s
    res = {
        "terms_per_s": steps * terms / sec,
        "ms_per_step": 1e3 * sec / steps,
        "hot_kernel_ms_mean": float(np.mean(hot)),
        "hot_kernel_ms_median": float(np.median(hot)),
        "hot_kernel_ms_min": float(np.min(hot)),
        "input_sha256": input_sha256(A),
        "launches_ms_mean": float(np.mean(total)),
        "result": result,
        "oracle_golden": golden,
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "T int32 lane-ops/s",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": measured_traffic(),
            "ops_per_term": OPS_PER_TERM,
            "terms_per_launch": terms,
            "kernel": "k_walk<1> (16-index blocks)",
        },
        "gray_step_frac": GRAY_STEP_OPS_PER_TERM * terms / hot_s / PEAK_LANE_OPS,
        "paper_ops_frac": PAPER_OPS_PER_TERM_2W * terms / hot_s / PEAK_LANE_OPS,
    }
    d = walk_counters()
    # traffic, executed_frac and valu_utilization_pct are not measured in this run: they come from
    # the committed counter passes, used only while the kernel sources hash to the profiled ones
    res["roofline"]["counters_source"] = (
        {"file": "profiles/k_walk_36x36_counters.json", "source_sha256": d["source_sha256"],
         "fields": ["traffic", "executed_frac", "valu_utilization_pct"]} if d else None)
    if d:
        # executed VALU lane-ops (SQ_INSTS_VALU x 64 per index, from the counter pass) over the peak,
        # and rocprof's VALUUtilization
        res["roofline"]["executed_frac"] = d["valu_lane_ops_per_term"] * terms / hot_s / PEAK_LANE_OPS
        if "valu_utilization_pct" in d:
            res["roofline"]["valu_utilization_pct"] = d["valu_utilization_pct"]
    return res


def with_default_tuning(P, cls, fn):
    """Run fn() with every class at the library's defaults (None when class cls already runs them)."""
    if P.tuning_get_class(cls)[1] == P.PERM_TUNE_SRC_DEFAULT:
        return None
    with P.saved_tunings():
        P.tuning_reset()
        return fn()


# ------------------------------------------------------------------ batch

def packed_batch(P, W, torch, b):
    planes = np.concatenate([P.perm_mod3_pack(M) for M in b.mats])
    row_off = np.zeros(b.count, np.int64)
    row_off[1:] = np.cumsum(b.ns[:-1].astype(np.int64))
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(planes.view(np.int64)).to(dev), torch.from_numpy(row_off).to(dev),
            torch.from_numpy(b.ns.copy()).to(dev))


def bench_batch(P, W, torch, reps, baseline=True):
    b = W.batch_uniform()
    terms = int(sum((1 << int(n)) - 1 for n in b.ns))
    planes, row_off, ns = packed_batch(P, W, torch, b)
    dev = torch.device("cuda", 0)
    out = torch.zeros(b.count, dtype=torch.uint8, device=dev)
    hist = torch.zeros(64 * 3, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    P.perm_mod3_batch_packed(planes, row_off, ns, out, hist, stream)   # captures the graph
    torch.cuda.synchronize()
    hist.zero_()
    t0 = time.perf_counter()
    for _ in range(reps):
        P.perm_mod3_batch_packed(planes, row_off, ns, out, hist, stream)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    res = out.cpu().numpy()
    h = hist.cpu().numpy().reshape(64, 3) // reps
    per_n = {int(n): [int(x) for x in h[n]] for n in range(12, 29)}
    g = read_golden("full_batch8192.txt")
    want = np.array([int(ch) for ch in "".join(g["results"])], np.uint8)
    want_hist = {int(row.split()[0]): [int(x) for x in row.split()[1:]] for row in g["hist"]}
    bad = int(np.count_nonzero(res != want)) if want.size == res.size else -1
    golden = check_golden("full_batch8192.txt",
                          g["input_sha256"] == W.sha256(b.ns, *b.mats) and bad == 0 and per_n == want_hist,
                          {"results_differing": bad, "hist_equal": per_n == want_hist})

    achieved = OPS_PER_TERM * terms / sec
    states = int(P.tuning_get_class(P.PERM_TUNE_BATCH)[0].states_per_lane)
    result = {
        "workload": "8192 matrices, n uniform on 12..28, uniform entries, packed (mag, sgn) uint64 planes",
        "matrices_per_s": b.count / sec,
        "terms_per_s": terms / sec,
        # the whole call per batch (plan, pack, walk) by the host clock over graph replays
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "T int32 lane-ops/s", "frac": achieved / PEAK_LANE_OPS, "ops_per_term": OPS_PER_TERM,
                     "kernel": f"k_walk<{states}, true> ({states} chunk(s) a lane per task, candidate blocks "
                               "re-walked one lane each)"},
        "ms_per_batch": 1e3 * sec,
        "hist_per_n": per_n,
        "zero_fraction": float(np.mean(res == 0)),
        "input_sha256": input_sha256(*b.mats),
        "oracle_golden": golden,
    }
    if not baseline:
        return result
    # baseline: one launch sequence per matrix on the same GPU, no graphs
    L = P.lib()
    saved = P.tuning_get()
    t = P.tuning_get()
    t.use_graphs = 0
    P.tuning_set(t)
    out1 = torch.zeros(b.count, dtype=torch.uint8, device=dev)
    base_ptr = planes.data_ptr()
    roff = row_off.cpu().numpy()
    ns_ptr = ns.data_ptr()
    zero_off = torch.zeros(1, dtype=torch.int64, device=dev)
    sh = int(stream.cuda_stream)
    t0 = time.perf_counter()
    for k in range(b.count):
        rc = L.perm_mod3_batch_packed(base_ptr + 16 * int(roff[k]), zero_off.data_ptr(), ns_ptr + 4 * k, 1,
                                      out1.data_ptr() + k, None, sh)
        assert rc == 0, P.lib().perm_last_error()
    torch.cuda.synchronize()
    sec1 = time.perf_counter() - t0
    P.tuning_set(saved)
    same = bool(np.array_equal(out1.cpu().numpy(), res))
    result["baseline_one_launch_per_matrix"] = {"matrices_per_s": b.count / sec1, "ms": 1e3 * sec1,
                                                "results_identical": same}
    result["speedup_vs_baseline"] = sec1 / sec
    return result


def bench_batch_classes(P, W, torch, reps=5):
    """The batch workload split by order: the matrices of each n (12..28) as a batch of their own,
    timed by the library's HIP events (walk kernel, and all launches of the call), median of reps."""
    b = W.batch_uniform()
    dev = torch.device("cuda", 0)
    rows = []
    P.timing_enable(True)
    try:
        for n in range(12, 29):
            mats = [M for M, k in zip(b.mats, b.ns) if int(k) == n]
            planes = np.concatenate([P.perm_mod3_pack(M) for M in mats]).view(np.int64)
            row_off = (np.arange(len(mats), dtype=np.int64) * n)
            pl = torch.from_numpy(planes).to(dev)
            ro = torch.from_numpy(row_off).to(dev)
            ns = torch.full((len(mats),), n, dtype=torch.int32, device=dev)
            out = torch.zeros(len(mats), dtype=torch.uint8, device=dev)
            hot, tot = [], []
            for _ in range(reps + 1):
                P.perm_mod3_batch_packed(pl, ro, ns, out, None, None)
                t = P.timing_last()
                hot.append(t.hot_kernel_ms)
                tot.append(t.total_ms)
            terms = len(mats) * ((1 << n) - 1)
            walk_ms = float(np.median(hot[1:]))
            rows.append({"n": n, "count": len(mats), "walk_ms": walk_ms, "call_ms": float(np.median(tot[1:])),
                         "terms_per_s": terms / walk_ms * 1e3})
            log(f"batch class n={n}: {len(mats)} matrices, walk {walk_ms:.3f} ms, {rows[-1]['terms_per_s']:.3e} terms/s")
    finally:
        P.timing_enable(False)
    return {"workload": "the 8192-matrix batch split by n, each order as its own batch", "rows": rows}


# ------------------------------------------------------------------ single 20 x 20 (latency)

def bench_single20(P, W, torch, reps=200):
    """End-to-end latency of one 20x20 matrix resident in HBM (2^20 terms: launch-bound)."""
    A = W.single_20()
    dev = torch.device("cuda", 0)
    mats = torch.from_numpy(A.reshape(-1).copy()).to(dev)
    offs = torch.zeros(1, dtype=torch.int64, device=dev)
    ns = torch.full((1,), 20, dtype=torch.int32, device=dev)
    out = torch.zeros(1, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(5):
        P.perm_mod3_batch_dev(mats, offs, ns, out, None, stream)
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        P.perm_mod3_batch_dev(mats, offs, ns, out, None, stream)
        stream.synchronize()
        lat.append(time.perf_counter() - t0)
    # the same matrix through perm_mod3(A, n) from host memory: staging copy in, result copy out
    for _ in range(5):
        P.perm_mod3(A)
    hl = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = P.perm_mod3(A)
        hl.append(time.perf_counter() - t0)
    return {"workload": "one 20x20 uniform matrix resident in HBM, device-input call on the NULL stream, "
                        "synchronised each call",
            "p50_us": 1e6 * pct(lat, 50), "p99_us": 1e6 * pct(lat, 99),
            "terms_per_s": ((1 << 20) - 1) / pct(lat, 50), "result": int(out.item()),
            "input_sha256": input_sha256(A),
            "host_call": {"workload": "perm_mod3(A, 20) from host memory, result to host",
                          "p50_us": 1e6 * pct(hl, 50), "p99_us": 1e6 * pct(hl, 99), "result": int(r)}}


# ------------------------------------------------------------------ large and sparse

def bench_large(P, W, torch):
    """One 44x44 uniform matrix, then 64 matrices 40x40 with P(0) = 0.6 in one launch."""
    big, sp = W.large_sparse()
    dev = torch.device("cuda", 0)
    mats = torch.from_numpy(big.reshape(-1).copy()).to(dev)
    offs = torch.zeros(1, dtype=torch.int64, device=dev)
    ns = torch.full((1,), 44, dtype=torch.int32, device=dev)
    out = torch.zeros(1, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.perm_mod3_batch_dev(mats, offs, ns, out)
    torch.cuda.synchronize()
    t44 = time.perf_counter() - t0
    r44 = int(out.item())
    buf, o = sp.flat()
    smats = torch.from_numpy(buf).to(dev)
    soffs = torch.from_numpy(o[:-1].copy()).to(dev)
    sns = torch.from_numpy(sp.ns.copy()).to(dev)
    sout = torch.zeros(sp.count, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.perm_mod3_batch_dev(smats, soffs, sns, sout)
    torch.cuda.synchronize()
    t40 = time.perf_counter() - t0
    terms44 = (1 << 44) - 1
    terms40 = sp.count * ((1 << 40) - 1)
    return {"workload": "one 44x44 uniform matrix; 64 matrices 40x40 with P(0)=0.6, P(1)=P(2)=0.2",
            "input_sha256": input_sha256(big, *sp.mats),
            "n44_s": t44, "n44_terms_per_s": terms44 / t44, "n44_result": r44,
            "sparse40_s": t40, "sparse40_terms_per_s": terms40 / t40,
            "sparse40_matrices_per_s": sp.count / t40,
            "sparse40_result_counts": [int((sout == v).sum().item()) for v in range(3)]}


# ------------------------------------------------------------------ 128 columns

def gray_inverse(x: int) -> int:
    """The Gray index whose state is x."""
    i = 0
    while x:
        i ^= x
        x >>= 1
    return i


def _time_wide(P, A, begin, count, steps, warmup):
    P.timing_enable(True)
    for _ in range(warmup):
        P.perm_mod3_range_tally_wide(A, begin, count)
    hot, wall = [], []
    T = None
    for _ in range(steps):
        t0 = time.perf_counter()
        T = P.perm_mod3_range_tally_wide(A, begin, count)
        wall.append(time.perf_counter() - t0)
        hot.append(P.timing_last().hot_kernel_ms)
    P.timing_enable(False)
    hot_s = float(np.mean(hot)) * 1e-3
    achieved = OPS_PER_TERM * count / hot_s
    return {"indices": count, "tally": T,
            "hot_kernel_ms_mean": float(np.mean(hot)), "hot_kernel_ms_min": float(np.min(hot)),
            "call_ms_mean": 1e3 * float(np.mean(wall)), "terms_per_s": count / hot_s,
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "T int32 lane-ops/s", "frac": achieved / PEAK_LANE_OPS, "kernel": "k_walk_wide"}}


def bench_wide(P, W, steps=6, warmup=2):
    """Matrices of 128 columns, 2^36 Gray indices per call (the headline's count) at indices near 2^127:
    a uniform 128 x 128 matrix, and the block matrix M (+) D (M 36 x 36 hidden triangular, D 92 x 92)
    on the range whose state holds every row of D, where T has a closed form."""
    count = 1 << 36
    U = W.uniform_matrix(128, W.SEED_WIDE)
    uni = _time_wide(P, U, 3 << 125, count, steps, warmup)
    uni["workload"] = "uniform 128x128 over F_3, 2^36 Gray indices from 3 * 2^125"
    A, M, d, D = W.wide_128()
    blk = _time_wide(P, A, gray_inverse((1 << 92) - 1) << 36, count, steps, warmup)
    blk["workload"] = ("128x128 M (+) D: M hidden triangular 36x36, D 92x92, columns shuffled; 2^36 Gray "
                       "indices from g^-1(all rows of D) * 2^36")
    return {"n": 128, "uniform": uni, "block": blk}


# ------------------------------------------------------------------ vectors over F_3

HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s


def bench_vec(P, torch, log2_len=32, reps=10):
    """Bitsliced F_3 vectors of 2^32 elements in HBM: phi, Theorem 2.1's add and mul, the dot
    product and psi, each timed by HIP events on one stream, against the HBM peak."""
    n = 1 << log2_len
    words = P.f3_words(n)
    t = torch
    gen = t.Generator(device="cuda")
    gen.manual_seed(7)
    va = t.randint(0, 3, (n,), dtype=t.uint8, device="cuda", generator=gen)
    vb = t.randint(0, 3, (n,), dtype=t.uint8, device="cuda", generator=gen)
    pa = t.empty(2 * words, dtype=t.int64, device="cuda")
    pb = t.empty_like(pa)
    po = t.empty_like(pa)
    back = t.empty(n, dtype=t.uint8, device="cuda")
    s = t.zeros(1, dtype=t.int64, device="cuda")
    st = t.cuda.current_stream()
    plane_bytes = 16 * words
    cases = {
        # name: (call, algorithmic HBM bytes: each operand read once, each result written once)
        "pack": (lambda: P.f3_pack(va, pa, None, st), n + plane_bytes),
        "add": (lambda: P.f3_op(P.PERM_F3_ADD, pa, pb, po, stream=st), 3 * plane_bytes),
        "mul": (lambda: P.f3_op(P.PERM_F3_MUL, pa, pb, po, stream=st), 3 * plane_bytes),
        "dot": (lambda: P.f3_dot(pa, pb, s, stream=st), 2 * plane_bytes),
        "unpack": (lambda: P.f3_unpack(po, n, back, stream=st), plane_bytes + n),
    }
    P.f3_pack(vb, pb, None, st)
    out = {"workload": f"two uniform vectors of 2^{log2_len} elements over F_3 (bytes), "
                       f"bipedal planes of {plane_bytes} bytes each"}
    for name, (call, nbytes) in cases.items():
        for _ in range(2):
            call()
        e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            call()
        e1.record(st)
        e1.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        out[name] = {"ms": sec * 1e3, "bytes": nbytes, "GB_per_s": nbytes / sec / 1e9,
                     "roofline": {"bound": "hbm", "achieved": nbytes / sec / 1e9, "peak": HBM_PEAK / 1e9,
                                  "unit": "GB/s", "frac": nbytes / sec / HBM_PEAK}}
    out["dot_value"] = int(s.item())
    del pa, pb, po, back
    # what a plain device-to-device copy of the same 2^32 bytes reaches on this GPU (read + write)
    for _ in range(2):
        vb.copy_(va)
    e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        vb.copy_(va)
    e1.record(st)
    e1.synchronize()
    out["device_copy_GB_per_s"] = 2 * n / (e0.elapsed_time(e1) * 1e-3 / reps) / 1e9
    del va, vb
    return out


# ------------------------------------------------------------------ Pi_50 (Section 3.1)

def bench_pi50(P, W, shards=64, ckdir=None):
    """perm(Pi_50) mod 3, both readings of the matrix, as a sharded and checkpointed run."""
    from paper_2407_20205_amd import longrun
    out = {}
    for reading in ("rows", "formula"):
        A = W.pi_matrix(50, reading)
        ck = os.path.join(ckdir, f"pi50_{reading}.json") if ckdir else None
        t0 = time.perf_counter()
        r = longrun.perm_mod3_sharded(A, shards, checkpoint=ck, log=log)
        sec = time.perf_counter() - t0
        out[reading] = {"perm_mod3": int(r), "as_centred": {0: 0, 1: 1, 2: -1}[int(r)], "seconds": sec,
                        "terms_per_s": ((1 << 50) - 1) / sec, "matrix_sha256": longrun.matrix_hash(A)}
        log(f"Pi_50 ({reading}): perm = {r} (mod 3) in {sec:.1f} s")
    out["paper"] = "perm(Pi_50) = -1 (mod 3) after 832 hours of parallel computation (Section 3.1)"
    return out


# ------------------------------------------------------------------ exact census (Section 4, Table 3)

def read_table3():
    with open(os.path.join(ROOT, "tests", "golden", "table3_zero_counts.txt")) as f:
        return [tuple(int(x) for x in line.split()) for line in f if line.strip() and not line.startswith("#")]


def bench_census(P):
    """Table 3's exact counts: every n x n matrix over F_3 (n = 1..5) enumerated on the device."""
    out = {"rows": []}
    for n, z_paper in read_table3():
        total = 3 ** (n * n)
        t0 = time.perf_counter()
        c = P.perm_mod3_census(n, P.PERM_GEN_ENUMERATE, 0, 0, total)
        sec = time.perf_counter() - t0
        out["rows"].append({"n": n, "matrices": total, "z": c[0], "ones": c[1], "minus_ones": c[2],
                            "z_table3": z_paper, "equal": c[0] == z_paper, "seconds": sec,
                            "matrices_per_s": total / sec})
        log(f"z({n}) = {c[0]} (Table 3: {z_paper}), {total} matrices in {sec:.2f} s")
    return out


# ------------------------------------------------------------------ Monte Carlo (Section 4, Table 4)

def read_table4():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "table4_montecarlo.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, z, lg = line.split()
                rows.append((int(n), int(z), 10 ** int(lg)))
    return rows


def bench_montecarlo(P, scale, n_min=6, n_max=30):
    """Table 4's study: for each n, uniform random matrices (SplitMix64 draws made on the
    device) and the fraction with perm = 0, at `scale` times the paper's trial counts."""
    import math
    out = {"scale": scale, "rows": [], "paper": "Table 4: about one day on 128 processors at scale 1"}
    total_s = 0.0
    for n, z_paper, trials_paper in read_table4():
        if n > n_max or n < n_min:
            continue
        trials = max(1000, int(trials_paper * scale))
        t0 = time.perf_counter()
        c = P.perm_mod3_census(n, P.PERM_GEN_SPLITMIX, 4_000_000 + n, 0, trials)
        sec = time.perf_counter() - t0
        total_s += sec
        p_ours = c[0] / trials
        p_paper = z_paper / trials_paper
        se = math.sqrt(p_ours * (1 - p_ours) / trials + p_paper * (1 - p_paper) / trials_paper)
        row = {"n": n, "trials": trials, "zeros": c[0], "ones": c[1], "minus_ones": c[2],
               "p0": p_ours, "p0_paper": p_paper, "z_score": (p_ours - p_paper) / se if se else 0.0,
               "seconds": sec, "terms_per_s": trials * ((1 << n) - 1) / sec}
        out["rows"].append(row)
        log(f"n={n}: {trials} trials, P(perm=0) {p_ours:.5f} vs Table 4 {p_paper:.5f} "
            f"(z = {row['z_score']:+.2f}), {sec:.2f} s")
    out["seconds"] = total_s
    return out


# ------------------------------------------------------------------ serving

def expected_work(W):
    support, p = W.serve_n_weights()
    return float(sum(pi * (2.0 ** int(n)) for n, pi in zip(support, p)))


def replay_server(P, tr, policy, quantum, work_budget=1 << 44):
    """Open-loop replay: requests are submitted at their arrival times; latency = done - arrival."""
    count = len(tr.mats)
    done = {}
    srv = P.Server(max_slots=4096, queue_cap=1 << 16, work_budget=work_budget, quantum=quantum, policy=policy)
    start = time.monotonic_ns()
    stop = threading.Event()

    def collect():
        while len(done) < count and not stop.is_set():
            for d in srv.poll(4096, 2000):
                done[int(d.tag)] = (int(d.t_done_ns), int(d.result), int(d.t_admit_ns))

    th = threading.Thread(target=collect, daemon=True)
    th.start()
    for k in range(count):
        at = start + int(tr.arrival_s[k] * 1e9)
        while True:
            now = time.monotonic_ns()
            if now >= at:
                break
            time.sleep(min(0.0005, (at - now) / 1e9))
        while not srv.submit(tr.mats[k], k):
            time.sleep(0.0002)
    th.join(timeout=600)
    stop.set()
    st = srv.stats()
    srv.close()
    lat = [(done[k][0] - (start + int(tr.arrival_s[k] * 1e9))) / 1e6 for k in range(count)]
    end = max(v[0] for v in done.values())
    return lat, [done[k][1] for k in range(count)], (end - start) / 1e9, st


def replay_fifo_baseline(P, tr):
    """One launch sequence per request, in arrival order, synchronously."""
    count = len(tr.mats)
    start = time.monotonic_ns()
    lat, res = [], []
    for k in range(count):
        at = start + int(tr.arrival_s[k] * 1e9)
        now = time.monotonic_ns()
        if now < at:
            time.sleep((at - now) / 1e9)
        res.append(P.perm_mod3(tr.mats[k]))
        lat.append((time.monotonic_ns() - at) / 1e6)
    return lat, res, (time.monotonic_ns() - start) / 1e9


def bench_serve(P, W, torch, rate, count, batched_terms_per_s, quantum=1 << 33, baseline=True):
    ew = expected_work(W)
    if rate is None:
        rate = 0.7 * batched_terms_per_s / ew
    tr = W.serve_trace(count=count, rate=rate)
    terms = float(sum((1 << int(n)) - 1 for n in tr.ns))
    # untimed warm-up: a short replay of another trace, so that loading the server's kernels and
    # first-use allocations are not counted in the measured tail
    replay_server(P, W.serve_trace(count=max(count // 10, 1), rate=rate, seed=W.SEED_SERVE + 1),
                  P.PERM_POLICY_SRPT, quantum)
    log(f"serve: {count} requests at {rate:.1f}/s, {terms:.3e} terms")
    lat, res, span, st = replay_server(P, tr, P.PERM_POLICY_SRPT, quantum)
    log(f"serve: continuous batching done in {span:.2f} s, p50 {pct(lat, 50):.3f} ms, p99 {pct(lat, 99):.3f} ms")
    if not baseline:
        return {"rate_per_s": rate, "quantum": quantum, "requests_per_s": count / span, "p50_ms": pct(lat, 50),
                "p99_ms": pct(lat, 99), "ticks": int(st.ticks)}
    # the same trace with a work budget that binds: at most 2^36 Gray indices admitted at once
    # (one 36 x 36 request's work), so larger requests run alone and later ones wait in the queue
    budget = 1 << 36
    qlat, qres, qspan, qst = replay_server(P, tr, P.PERM_POLICY_SRPT, quantum, work_budget=budget)
    log(f"serve: budget 2^36 done in {qspan:.2f} s, p50 {pct(qlat, 50):.3f} ms, p99 {pct(qlat, 99):.3f} ms")
    blat, bres, bspan = replay_fifo_baseline(P, tr)
    log(f"serve: FIFO baseline done in {bspan:.2f} s")
    g = read_golden("full_serve_le28.txt")
    if int(g["count"]) == count:
        want = "".join(g["results"])
        checked = [k for k in range(count) if want[k] != "-"]
        bad = sum(1 for k in checked if res[k] != int(want[k]))
        golden = check_golden("full_serve_le28.txt",
                              g["input_sha256"] == W.sha256(tr.ns, *tr.mats) and bad == 0 and len(checked) > 0,
                              {"checked": len(checked), "results_differing": bad})
    else:
        golden = {"file": "tests/golden/full_serve_le28.txt", "match": None,
                  "skipped": f"the stored values are for the {g['count']}-request trace, this one has {count}"}
    return {
        "workload": f"{count} requests, n in 8..40 with P(n) ~ 1.15^-(n-8), Poisson arrivals at {rate:.1f}/s "
                    "(0.7 x batched capacity / E[2^n]), uniform entries",
        "rate_per_s": rate,
        "requests_per_s": count / span,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(np.mean(lat)),
        "terms_per_s": terms / span,
        "ticks": int(st.ticks),
        "quantum": quantum,
        "input_sha256": input_sha256(*tr.mats),
        "baseline_fifo_one_launch_per_request": {"p50_ms": pct(blat, 50), "p99_ms": pct(blat, 99),
                                                 "requests_per_s": count / bspan},
        "results_identical_to_baseline": bool(res == bres),
        "oracle_golden": golden,
        "work_budget": 1 << 44,
        "budgeted_2pow36": {"work_budget": budget, "requests_per_s": count / qspan, "p50_ms": pct(qlat, 50),
                            "p99_ms": pct(qlat, 99), "mean_ms": float(np.mean(qlat)), "ticks": int(qst.ticks),
                            "results_identical": bool(qres == res)},
    }


# ------------------------------------------------------------------ CPU oracle baseline

def bench_cpu(W, seconds=12.0):
    import oracle
    threads = oracle.default_threads()
    A = W.single_36()
    calib = 1 << 21
    t0 = time.perf_counter()
    oracle.range_tally(A, 0, calib * threads, threads=threads)
    rate = calib * threads / (time.perf_counter() - t0)
    length = int(min(1 << 36, max(calib * threads, rate * seconds)))
    a = (1 << 35) - length // 2
    t0 = time.perf_counter()
    oracle.range_tally(A, a, a + length, threads=threads)
    sec = time.perf_counter() - t0
    # one core, over a short range of the same matrix
    one = 1 << 24
    t0 = time.perf_counter()
    oracle.range_tally(A, a, a + one, threads=1)
    one_s = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((line.split(":", 1)[1].strip() for line in f if line.startswith("model name")), "")
    except OSError:
        pass
    return {"value": length / sec, "unit": "subset-terms/s", "cores": threads, "kind": "oracle",
            "single_core_terms_per_s": one / one_s, "cpu_model": model, "os_cpu_count": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "sample": f"Gray indices [{a}, {a + length}) of the 36x36 matrix ({length} of 2^36 terms), "
                      f"{sec:.1f} s on {threads} threads; full matrix extrapolates to "
                      f"{(1 << 36) / (length / sec):.0f} s"}


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", choices=["headline", "single20", "batch", "batch-classes", "serve", "large", "wide",
                                       "vec", "pi50", "montecarlo", "census"],
                    default=None)
    ap.add_argument("--mc-scale", type=float, default=0.01, help="fraction of Table 4's trial counts")
    ap.add_argument("--mc-n", default="6-30", help="range of n for the Monte Carlo study, e.g. 6-17")
    ap.add_argument("--checkpoint-dir", default=None, help="checkpoint files of the sharded Pi_50 run")
    ap.add_argument("--serve-count", type=int, default=20000)
    ap.add_argument("--serve-rate", type=float, default=None)
    ap.add_argument("--serve-quantum-log", type=int, default=33, help="log2 of the Gray indices per tick")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-baselines", action="store_true",
                    help="skip the one-launch-per-matrix and FIFO baselines (for profiling)")
    ap.add_argument("--no-default-tuning", action="store_true",
                    help="skip the second run of the headline and the batch with the built-in tuning "
                         "(so that a kernel trace holds only the tuned launches)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a known-size kernel for "
                         "calibrating the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (every box here has one GPU; "
              "a single matrix would shard its Gray range across GPUs with one int64 sum at the end)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_20205_amd import perm3 as P
    from paper_2407_20205_amd import workloads as W
    torch.cuda.set_device(0)
    info = P.device_info()
    log(f"device {info.arch.decode()} CUs {info.compute_units} clock {info.max_clock_khz} kHz")

    line = {"metric": "Ryser subset-terms/s at n=36 (% int VALU peak); batch matrices/s + p50/p99 latency",
            "value": None, "unit": "subset-terms/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32 bitwise / i64 tally", "data": "synthetic (seeded uniform matrices over F_3)",
            "config": {"workload": "one 36x36 matrix over F_3, iid uniform {0,1,2}, uint8 row-major, "
                                   "2^36 - 1 Gray-code Ryser terms per step", "n": 36, "global_batch": 1,
                       "parallelism": "1 GPU, persistent waves over Gray chunks"}}

    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes device to device")
        del src, dst
    if args.only in (None, "headline"):
        tune = tuning_info(P, P.PERM_TUNE_LARGE)
        h = bench_headline(P, W, torch, args.steps, args.warmup)
        log(f"headline: {h['terms_per_s']:.4e} terms/s, walk {h['hot_kernel_ms_mean']:.3f} ms, "
            f"frac {h['roofline']['frac']:.3f} (tuning: {tune['source']})")
        line["value"] = h["terms_per_s"]
        line["ms_per_step"] = h["ms_per_step"]
        line["roofline"] = h["roofline"]
        line["roofline"]["tuning_source"] = tune["source"]
        line["headline_detail"] = {k: v for k, v in h.items() if k != "roofline"}
        line["headline_detail"]["tuning"] = tune
        hd = None if args.no_default_tuning else with_default_tuning(
            P, P.PERM_TUNE_LARGE, lambda: bench_headline(P, W, torch, max(5, args.steps // 2), args.warmup))
        if hd is not None:
            line["headline_default_tuning"] = {
                "terms_per_s": hd["terms_per_s"], "hot_kernel_ms_mean": hd["hot_kernel_ms_mean"],
                "frac": hd["roofline"]["frac"], "result": hd["result"], "steps": max(5, args.steps // 2)}
            log(f"headline with default tuning: {hd['terms_per_s']:.4e} terms/s, "
                f"walk {hd['hot_kernel_ms_mean']:.3f} ms")
        line["vs_paper_one_core"] = h["terms_per_s"] / ((1 << 36) / 101.9)
    if args.only in (None, "single20"):
        s20 = bench_single20(P, W, torch)
        log(f"single 20x20: p50 {s20['p50_us']:.1f} us, p99 {s20['p99_us']:.1f} us "
            f"(host call: p50 {s20['host_call']['p50_us']:.1f} us, p99 {s20['host_call']['p99_us']:.1f} us)")
        line["single20"] = s20
    if args.only in (None, "batch"):
        tune = tuning_info(P, P.PERM_TUNE_BATCH)
        bt = bench_batch(P, W, torch, reps=max(3, args.steps // 4), baseline=not args.no_baselines)
        bt["tuning"] = tune
        log(f"batch: {bt['matrices_per_s']:.1f} matrices/s ({bt.get('speedup_vs_baseline', 0):.1f}x one-launch, "
            f"tuning: {tune['source']})")
        bd = None if args.no_default_tuning else with_default_tuning(
            P, P.PERM_TUNE_BATCH, lambda: bench_batch(P, W, torch, reps=max(3, args.steps // 4), baseline=False))
        if bd is not None:
            bt["default_tuning"] = {"matrices_per_s": bd["matrices_per_s"], "terms_per_s": bd["terms_per_s"],
                                    "ms_per_batch": bd["ms_per_batch"],
                                    "hist_identical": bd["hist_per_n"] == bt["hist_per_n"]}
            log(f"batch with default tuning: {bd['matrices_per_s']:.1f} matrices/s")
        line["batch"] = bt
    if args.only in (None, "serve"):
        cap = line.get("batch", {}).get("terms_per_s") or 8e12
        line["serve"] = bench_serve(P, W, torch, args.serve_rate, args.serve_count, cap,
                                    quantum=1 << args.serve_quantum_log, baseline=not args.no_baselines)
    if args.only in (None, "large"):
        lg = bench_large(P, W, torch)
        log(f"large: n=44 {lg['n44_s']:.3f} s ({lg['n44_terms_per_s']:.3e} terms/s), 64 sparse n=40 "
            f"{lg['sparse40_s']:.3f} s ({lg['sparse40_terms_per_s']:.3e} terms/s)")
        line["large"] = lg
    if args.only in (None, "wide"):
        wd = bench_wide(P, W)
        for k in ("uniform", "block"):
            log(f"wide {k}: n=128, 2^36 indices, walk {wd[k]['hot_kernel_ms_mean']:.3f} ms "
                f"({wd[k]['terms_per_s']:.3e} indices/s, frac {wd[k]['roofline']['frac']:.3f})")
        line["wide"] = wd
    if args.only in (None, "vec"):
        vc = bench_vec(P, torch)
        log("vec: " + ", ".join(f"{k} {vc[k]['GB_per_s']:.0f} GB/s" for k in ("pack", "add", "mul", "dot", "unpack")) +
            f"; device copy {vc['device_copy_GB_per_s']:.0f} GB/s")
        line["vec"] = vc
    if args.only == "batch-classes":
        line["batch_classes"] = bench_batch_classes(P, W, torch)
    if args.only == "montecarlo":
        lo, hi = (int(x) for x in args.mc_n.split("-"))
        line["montecarlo"] = bench_montecarlo(P, args.mc_scale, lo, hi)
    if args.only == "census":
        line["census"] = bench_census(P)
    if args.only == "pi50":
        line["pi50"] = bench_pi50(P, W, ckdir=args.checkpoint_dir)
    if args.only is None and not args.no_cpu:
        line["cpu_baseline"] = bench_cpu(W)
        log(f"cpu oracle: {line['cpu_baseline']['value']:.3e} terms/s on {line['cpu_baseline']['cores']} threads")
    if GOLDEN_MISMATCH:
        line["oracle_golden_mismatch"] = GOLDEN_MISMATCH
    print(json.dumps(line), flush=True)
    if GOLDEN_MISMATCH:
        sys.exit(3)


if __name__ == "__main__":
    main()
