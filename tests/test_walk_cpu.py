"""The device walk templates and the planning helpers built for the CPU under AddressSanitizer and
UndefinedBehaviorSanitizer (tests/walk_cpu.cpp), against the oracle: whole fast-walk chunks for
every block length and chunks per lane, direct chunks, arbitrary ranges, forward re-walks and
whole-block re-walks, 128-bit ranges of matrices with up to 128 columns, the plan's cover of a
Gray range, and the one-launch decision of small calls, whose work sum must not wrap (two orders
of 63 add up to 2^64).  Bar: exact equality."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2407_20205_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_20205_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "walk_cpu.cpp")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("walk_cpu") / "walk_cpu")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-Wall", "-Wextra",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan",
                    "-I", CSRC, "-o", exe, SRC], check=True)

    def run(lines):
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                           timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr, r.stderr[-4000:]
        out = r.stdout.strip().split("\n")
        assert len(out) == len(lines) and "error" not in out, out
        return out

    return run


def below(g, bound):
    """A draw from [0, bound) for bounds past int64 (2^63 and 2^64 included)."""
    x = (int(g.integers(0, 1 << 32)) << 32) | int(g.integers(0, 1 << 32))
    return x % bound


def digits(A):
    return "".join(str(int(x)) for x in np.asarray(A).reshape(-1))


def hit_heavy(n, seed):
    """Every entry +-1 as a rank-one sign pattern: two thirds of all terms are non-zero."""
    return W.rank_one_signs(n, seed)


# ---------------------------------------------------------------- one-launch decision of small calls

def test_small_call_decision_does_not_wrap(harness):
    cap = 1 << 28
    cases = [[63, 63], [58] * 64, [63] * 64, [28], [29], [27, 27], [28, 0], [0] * 64, [0] * 65, [],
             [-1, 64, 20], [64, 64], [62, 62, 62, 62], [20] * 64, [22] * 64, [22] * 65, [63, 1]]
    g = W.rng(7)
    for _ in range(40):
        cases.append([int(x) for x in g.integers(0, 64, size=int(g.integers(1, 70)))])
    out = harness([f"fused {len(c)} " + " ".join(map(str, c)) for c in cases])
    for c, line in zip(cases, out):
        fused, work = (int(x) for x in line.split())
        total = sum(1 << n for n in c if 0 <= n <= 63)
        assert work == min(total, cap + 1), c
        assert fused == int(1 <= len(c) <= 64 and total <= cap), c


# ---------------------------------------------------------------- plan

def test_target_chunk_log_and_queue_floor(harness):
    """A task (64 lanes x 2^m indices x S chunks) holds the call's work over waves x tasks_per_wave
    tasks, but at least 2^queue_task_log indices while the work still gives every wave one such task
    (else the work over the waves): the chunk log is the floor of log2 of that, less 6 and log2 S."""
    g = W.rng(9)
    cases = []
    for _ in range(400):
        work = float(int(g.integers(1, 1 << 40)))
        waves = int(g.choice([1, 64, 1024, 6144, 8192]))
        tpw = int(g.integers(1, 65))
        slog = int(g.integers(0, 3))
        q = int(g.choice([0, 12, 18, 20]))
        cases.append((work, waves, tpw, slog, q))
    cases += [(2.0 ** 36, 8192, 16, 0, 18), (2.0 ** 36, 6144, 32, 0, 18), (2.567e11, 8192, 32, 0, 18),
              (8.1e9, 8192, 32, 0, 18), (8.1e9, 8192, 32, 0, 0), (100.0, 8192, 16, 0, 18)]
    out = harness([f"target {w!r} {wv} {t} {s} {q}" for w, wv, t, s, q in cases])
    for (work, waves, tpw, slog, q), line in zip(cases, out):
        per_task = work / (waves * tpw)
        if q:
            per_task = max(per_task, min(2.0 ** q, work / waves))
        want = 0 if per_task < 128 else int(np.floor(np.log2(np.floor(per_task)))) - 6 - slog
        assert int(line) == want, (work, waves, tpw, slog, q)
    # the 36x36 and the Monte Carlo batch are not changed by the floor; an order-24 batch alone is
    by_case = dict(zip(cases, out))
    assert int(by_case[(2.0 ** 36, 8192, 16, 0, 18)]) == 13
    assert int(by_case[(2.567e11, 8192, 32, 0, 18)]) == 13
    assert int(by_case[(8.1e9, 8192, 32, 0, 18)]) == 12 and int(by_case[(8.1e9, 8192, 32, 0, 0)]) == 8


def test_plan_covers_the_range(harness):
    g = W.rng(8)
    cases, meta = [], []
    for _ in range(600):
        n = int(g.integers(1, 64))
        lo = below(g, 1 << n)
        hi = lo + below(g, (1 << n) - lo + 1)
        if g.integers(0, 4) == 0:
            lo, hi = 0, 1 << n
        bl, blm = int(g.integers(4, 7)), int(g.integers(4, 7))
        dmx = int(g.integers(max(bl, blm) + 6, 40))
        tun = [bl, int(g.integers(8, 25)), dmx, 10, blm, int(g.integers(0, 64)), int(g.integers(0, 3)),
               int(g.integers(0, 41)), int(g.integers(0, 31)), int(g.integers(1, 65))]
        tm = int(g.integers(0, 31))
        cases.append(f"plan {n} {lo} {hi} {tm} " + " ".join(map(str, tun)))
        meta.append((n, lo, hi, tun))
    for (n, lo, hi, tun), line in zip(meta, harness(cases)):
        mode, m, ul, c_first, ntasks = (int(x) for x in line.split())
        slog = tun[6]
        if hi <= lo:
            assert mode == 2 and ntasks == 0
            continue
        assert mode in (0, 1)
        per = 64 << slog
        assert c_first == lo >> m
        assert (c_first << m) <= lo
        assert ((c_first + ntasks * per) << m) >= hi            # the tasks cover [lo, hi)
        assert ((c_first + (ntasks - 1) * per) << m) < hi       # and none starts past it
        if mode == 0:                                           # fast walk: whole blocks, int32 lane tallies
            assert ul + 1 <= m <= min(n - 6 - slog, 24 - slog), (n, m, ul, tun)
            assert ul == (tun[4] if n <= tun[5] else tun[0])
        else:
            assert 0 <= m <= min(max(n - 6, 0), 10)


# ---------------------------------------------------------------- walks

def chunk_cases(g, count):
    cases, want = [], []
    for _ in range(count):
        ul = int(g.choice([4, 5, 6]))
        s = int(g.choice([1, 2, 4]))
        slog = {1: 0, 2: 1, 4: 2}[s]
        n = int(g.integers(ul + 8 + slog, 64))
        m = int(g.integers(ul + 1, min(n - 6 - slog, 14) + 1))
        nchunks = 1 << (n - m)
        c = below(g, nchunks - 64 * (s - 1))
        A = hit_heavy(n, int(g.integers(1 << 30))) if g.integers(0, 2) else W.uniform_matrix(n, int(g.integers(1 << 30)))
        cases.append(f"chunks {ul} {s} {n} {m} {c} {digits(A)}")
        want.append([(A, (c + 64 * q) << m, (c + 64 * q + 1) << m) for q in range(s)])
    return cases, want


def test_fast_walk_chunks_vs_oracle(harness):
    g = W.rng(9)
    cases, want = chunk_cases(g, 90)
    for line, parts in zip(harness(cases), want):
        assert int(line) == sum(oracle.range_tally(A, a, b) for A, a, b in parts), parts[0][1:]


def test_candidate_list_and_its_overflow_vs_oracle(harness):
    """Blocks holding a candidate are noted (up to 128 per wave) and re-walked after the chunk; past
    that the rest are re-walked at once.  A hit-heavy matrix makes nearly every block a candidate:
    2^(m - UL) blocks below, at and far above the list's size, for every block length."""
    cases, want = [], []
    for ul in (4, 5, 6):
        for blocks_log in (1, 6, 7, 8, 10):
            m = ul + blocks_log
            n = m + 8
            for k, A in enumerate((hit_heavy(n, 900 + ul * 10 + blocks_log), W.uniform_matrix(n, 950 + ul))):
                c = 3 + k
                cases.append(f"chunks {ul} 1 {n} {m} {c} {digits(A)}")
                want.append((A, c << m, (c + 1) << m))
    for line, (A, a, b) in zip(harness(cases), want):
        assert int(line) == oracle.range_tally(A, a, b), (A.shape[0], a, b)


def test_direct_chunks_and_ranges_vs_oracle(harness):
    g = W.rng(10)
    cases, want = [], []
    for _ in range(120):
        n = int(g.integers(1, 64))
        A = hit_heavy(n, int(g.integers(1 << 30))) if g.integers(0, 2) else W.uniform_matrix(n, int(g.integers(1 << 30)))
        if g.integers(0, 2):
            m = int(g.integers(0, min(n, 11)))
            c = below(g, 1 << (n - m))
            cases.append(f"direct {n} {m} {c} {digits(A)}")
            want.append((A, c << m, (c + 1) << m))
        else:
            a = below(g, 1 << n)
            e = min(1 << n, a + int(g.integers(0, 1 << 12)))
            cases.append(f"range {n} {a} {e} {digits(A)}")
            want.append((A, a, e))
    for line, (A, a, b) in zip(harness(cases), want):
        assert int(line) == oracle.range_tally(A, a, b), (A.shape[0], a, b)


def test_rewalks_vs_oracle(harness):
    """A forward exact re-walk of a range inside an aligned block, and the exact walk of whole aligned
    blocks of 2^4, 2^5 and 2^6 indices (one lane's re-walk of a candidate block)."""
    g = W.rng(11)
    cases, want = [], []
    for _ in range(150):
        n = int(g.integers(3, 64))
        A = hit_heavy(n, int(g.integers(1 << 30))) if g.integers(0, 3) else W.uniform_matrix(n, int(g.integers(1 << 30)))
        k = int(g.integers(1, min(n, 9)))             # a block of 2^k indices aligned to its length
        base = below(g, 1 << (n - k)) << k
        a = base
        e = base + int(g.integers(1, 1 << k))
        cases.append(f"rewalk {n} {a} {e} {digits(A)}")
        want.append((A, a, e + 1))
    for line, (A, a, b) in zip(harness(cases), want):
        fwd, *blocks = (int(x) for x in line.split())
        w = oracle.range_tally(A, a, b)
        assert fwd == w, (A.shape[0], a, b, fwd, w)
        n = A.shape[0]
        for ul, got in zip((4, 5, 6), blocks):
            if n > ul:
                lo = a & ~((1 << ul) - 1)
                assert got == oracle.range_tally(A, lo, lo + (1 << ul)), (n, ul, lo)


def test_wide_lanes_vs_oracle(harness):
    g = W.rng(12)
    cases, want = [], []
    for _ in range(60):
        ul = int(g.choice([4, 5, 6]))
        n = int(g.integers(40, 129))
        A = hit_heavy(n, int(g.integers(1 << 30))) if g.integers(0, 3) else W.uniform_matrix(n, int(g.integers(1 << 30)))
        m = int(g.integers(ul + 1, 13))
        c0 = below(g, 1 << (n - m - 4))
        cr = int(g.integers(0, 8))
        fast = int(g.integers(0, 2))
        # the range relative to B = c0 2^m: sometimes the whole chunk, sometimes ragged ends
        oa0, oe0 = cr << m, (cr + 1) << m
        if g.integers(0, 2):
            off_lo, off_hi = oa0, oe0
        else:
            off_lo = oa0 + int(g.integers(0, 1 << m))
            off_hi = int(g.integers(off_lo, oe0 + 1))
        lim = 1 << n
        B = c0 << m
        if B + oe0 > lim:
            continue
        cases.append(f"wide {ul} {n} {c0 >> 64} {c0 & ((1 << 64) - 1)} {m} {fast} {off_lo} {off_hi} {cr} {digits(A)}")
        oa, oe = max(oa0, off_lo), min(oe0, off_hi)
        want.append((A, B + oa, max(oe - oa, 0)))
    out = harness(cases)
    for line, (A, begin, count) in zip(out, want):
        w = oracle.range_tally_wide(A, begin, count) if count else 0
        assert int(line) == w, (A.shape[0], begin, count)
