"""Host logic of the serving loop (server.cpp) under ThreadSanitizer and
AddressSanitizer + UndefinedBehaviorSanitizer, on the CPU.

server.cpp is compiled with the host compiler against a CPU stand-in for the
few HIP runtime calls it makes (tests/server_host/hip/hip_runtime.h) and a
fake engine (tests/server_host/fake_engine.cpp) that steps simulations and
writes outputs like the real one; tests/server_host/stress.cpp drives it from
several client threads (submit, cancel while queued, admitting or running,
wait with and without time-outs, poll, destroy with work outstanding) and
checks every request's end state and outputs and the counters.  Any
sanitizer report fails the test.  (LLVM's ThreadSanitizer is used: it
intercepts the timed condition-variable waits that std::condition_variable
makes, which GCC 11's runtime does not, and without which it reports races
between threads that hold the same mutex.)
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "server_host")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"


def _build_and_run(tmp_path, sanitize):
    if not os.path.exists(CLANG):
        pytest.skip("LLVM clang++ not found")
    exe = str(tmp_path / "stress")
    cmd = [CLANG, "-std=c++17", "-g", "-O1", f"-fsanitize={sanitize}", "-fno-sanitize-recover=all",
           "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1905_07622_amd", "csrc"),
           os.path.join(ROOT, "paper_1905_07622_amd", "csrc", "server.cpp"), os.path.join(HERE, "fake_engine.cpp"),
           os.path.join(HERE, "stress.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1 print_stacktrace=1")
    for _ in range(3):
        run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
        out = run.stdout + run.stderr
        assert run.returncode == 0 and "Sanitizer" not in out and "runtime error" not in out, out[-6000:]
        assert "0 failures" in out, out[-2000:]


def test_server_host_logic_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, "thread")


def test_server_host_logic_address_and_ub_sanitizers(tmp_path):
    _build_and_run(tmp_path, "address,undefined")
