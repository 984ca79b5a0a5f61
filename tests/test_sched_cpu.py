"""The serving scheduler (csrc/perm3_sched.hpp) on the CPU under ThreadSanitizer, driven by a mock
executor whose "device" thread walks each tick's tasks with the oracle (tests/sched_cpu.cpp):
every result must equal the oracle's perm mod 3, every slot's Gray range must be covered once and
in order by its tasks, admission must respect the slots and the work budget, and injected faults
(a failed launch, a failed fast-lane call, a tick that never finishes and trips the watchdog) must
complete every accepted request with PERM_EDEVICE instead of hanging.  Several submitter threads
and a polling thread run against the worker, so TSan sees the real concurrency.

libstdc++'s condition variables wait through pthread_cond_clockwait, which GCC 11's TSan runtime
does not intercept (it then reports false double locks); the test uses the LLVM toolchain that
ships with ROCm, whose runtime does."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_20205_amd", "csrc")
LLVM = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin")
CLANG = os.path.join(LLVM, "clang")
CLANGXX = os.path.join(LLVM, "clang++")


@pytest.fixture(scope="module")
def sched_exe(tmp_path_factory):
    if not (os.path.exists(CLANG) and os.path.exists(CLANGXX)):
        pytest.skip("needs the ROCm LLVM toolchain for ThreadSanitizer")
    d = tmp_path_factory.mktemp("sched_cpu")
    obj = str(d / "oracle.o")
    exe = str(d / "sched_cpu")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=thread"]
    subprocess.run([CLANG, *flags, "-c", os.path.join(ROOT, "oracle", "perm3_oracle.c"), "-o", obj], check=True)
    subprocess.run([CLANGXX, "-std=c++17", *flags, "-Wall", "-Wextra", "-Werror", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"), "-o", exe, os.path.join(ROOT, "tests", "sched_cpu.cpp"),
                    obj, "-lpthread"], check=True)
    return exe


def run(exe, seed, count, policy, slots, budget_log, quantum_log, fast_n, submitters, queue_cap,
        fault="none", fault_at=-1, n_lo=1, n_hi=16, timeout_ms=0):
    args = [str(x) for x in (seed, count, policy, slots, budget_log, quantum_log, fast_n, submitters,
                             queue_cap, fault, fault_at, n_lo, n_hi, timeout_ms)]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66:second_deadlock_stack=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-4000:])
    line = r.stdout.strip().splitlines()[-1]
    assert line.startswith("ok "), line
    return dict(kv.split("=") for kv in line.split()[1:])


@pytest.mark.parametrize("policy", [0, 1])
def test_every_result_equals_the_oracle(sched_exe, policy):
    out = run(sched_exe, 11 + policy, 500, policy, 8, 0, 13, 10, 3, 64)
    assert int(out["ok"]) == 500 and int(out["failed"]) == 0
    assert int(out["ticks"]) > 10 and int(out["fast_calls"]) > 0


def test_binding_work_budget_and_few_slots(sched_exe):
    # budget 2^14 with orders up to 18: larger requests run alone, the rest wait in the queue
    out = run(sched_exe, 21, 400, 0, 3, 14, 12, 9, 4, 16, n_hi=18)
    assert int(out["ok"]) == 400


def test_no_fast_lane_tiny_quantum(sched_exe):
    # every request through the slots, ticks of 2^9 indices: ranges split over many ticks
    out = run(sched_exe, 31, 200, 1, 16, 0, 9, -1, 2, 1000, n_lo=0, n_hi=14)
    assert int(out["ok"]) == 200 and int(out["fast_calls"]) == 0
    assert int(out["ticks"]) > 50


@pytest.mark.parametrize("fault,at", [("launch", 3), ("fast", 2), ("hang", 2)])
def test_faults_fail_every_request_without_hanging(sched_exe, fault, at):
    out = run(sched_exe, 41, 300, 0, 8, 0, 12, 10, 3, 64, fault=fault, fault_at=at,
              timeout_ms=200 if fault == "hang" else 0)
    assert int(out["failed"]) > 0 and int(out["fatal"]) == -4   # PERM_EDEVICE


def test_gcc_build_without_sanitizer(tmp_path):
    """The header also builds with the host compiler alone (warnings as errors)."""
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path / "sched_plain")
    obj = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", "-O2", "-c", os.path.join(ROOT, "oracle", "perm3_oracle.c"), "-o", obj], check=True)
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", "-I", CSRC, "-I",
                    os.path.join(ROOT, "include"), "-o", exe, os.path.join(ROOT, "tests", "sched_cpu.cpp"), obj,
                    "-lpthread"], check=True)
    r = subprocess.run([exe, "51", "300", "0", "8", "0", "12", "10", "3", "64", "none", "-1", "1", "16", "0"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok "), r.stdout + r.stderr[-2000:]
