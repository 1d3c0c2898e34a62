"""Host code under the sanitizers (CPU only): the scheduler against its
simulated executor and the threaded server front under AddressSanitizer +
UndefinedBehaviorSanitizer, the threaded server front under ThreadSanitizer
with client threads submitting, polling, cancelling and forgetting while the
worker runs rounds, and the FP64 oracle's own tests against an oracle built
with AddressSanitizer + UndefinedBehaviorSanitizer.

ThreadSanitizer uses ROCm's clang: the runtime of the system gcc does not
intercept pthread_cond_clockwait (which std::condition_variable::wait_for
calls), so it reports lock-order and race errors that are not there."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
SCENARIOS = ["fifo_budget", "slots", "reject", "mixed_steps", "cancel", "nan", "add_fail", "hol", "latency",
             "arrivals", "work_cap", "cap_latency_uncapped", "cap_latency_capped"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build(tmp, name, src, flags, cxx="g++"):
    exe = str(tmp / name)
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-pthread", *flags, "-o", exe,
                    os.path.join(HOST, src)], check=True)
    return exe


def _run(exe, *args):
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=ENV, timeout=120)
    assert r.returncode == 0 and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_scheduler_under_asan_ubsan(tmp_path):
    plain = _build(tmp_path, "sched_plain", "sched_sim.cpp", [])
    san = _build(tmp_path, "sched_san", "sched_sim.cpp", SAN)
    for sc in SCENARIOS:
        assert json.loads(_run(san, sc)) == json.loads(_run(plain, sc)), sc


def _check_threads(d):
    assert d["bad"] == 0 and d["waited"] and d["inited"] and d["shut"] and d["jobs_left"] == 0
    assert d["total"] == 96 and d["done"] + d["cancelled"] == 96 and d["steps_ok"] == d["done"]
    assert d["forgotten"] == 96 and d["stats_completed"] == d["done"] and d["stats_submitted"] == 96
    assert 1 <= d["max_active"] <= 6


def test_threaded_server_under_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "threads_san", "server_threads.cpp", SAN)
    for _ in range(3):
        _check_threads(json.loads(_run(exe)))


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang (ThreadSanitizer runtime) not installed")
def test_threaded_server_under_tsan(tmp_path):
    exe = _build(tmp_path, "threads_tsan", "server_threads.cpp", ["-fsanitize=thread", "-g"], cxx=CLANG)
    for _ in range(3):
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                             env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1"))
        assert out.returncode == 0 and "ThreadSanitizer" not in out.stderr, out.stderr[-4000:]
        _check_threads(json.loads(out.stdout))


def test_oracle_tests_under_asan_ubsan(tmp_path):
    """The oracle's own CPU tests (all but the two long unfrozen-difference
    runs) against an oracle built with the address and undefined-behaviour
    sanitizers; the runtimes are preloaded into the Python process."""
    so = str(tmp_path / "liboracle_san.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-pthread", *SAN,
                    os.path.join(ROOT, "oracle", "oracle.cpp"), "-o", so], check=True)
    pre = [subprocess.run(["g++", f"-print-file-name={n}"], capture_output=True, text=True, check=True).stdout.strip()
           for n in ("libasan.so", "libubsan.so")]
    assert all(os.path.isabs(p) for p in pre), pre
    env = dict(os.environ, LD_PRELOAD=":".join(pre), ASAN_OPTIONS="detect_leaks=0", ORACLE_LIB=so,
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    tests = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))
    args = [sys.executable, "-m", "pytest", *tests, "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
            "-k", "not unfrozen"] + (["-n", "4"] if _has_xdist() else [])
    r = subprocess.run(args,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0 and "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail


def _has_xdist():
    try:
        import xdist  # noqa: F401
        return True
    except ImportError:
        return False
