"""Host logic of the serving scheduler (csrc/serve.cpp) under sanitizers, no GPU.

serve.cpp is compiled for the CPU against a test-only fake executor
(tests/native/fake_device.cpp: HIP runtime calls and batched kernels on host
memory, with a device thread that runs the enqueued work asynchronously) and
driven by tests/native/serve_stress.cpp: concurrent submitters, a poller that
checks every result exactly and releases it, fetches, a canceller and a
statistics reader race with the scheduler thread; then a cancel-while-queued
budget check, injected allocation failures at admission (every third model
creation fails: those requests return PF_ERR_NOMEM, the others stay exact,
nothing leaks), and destroys with requests queued, running and unreleased.

Builds: g++ with AddressSanitizer + UndefinedBehaviorSanitizer, and clang++
(ROCm's LLVM) with ThreadSanitizer -- GCC 11's ThreadSanitizer runtime does
not intercept pthread_cond_clockwait (what libstdc++'s steady-clock waits
call), so it reports every wait_for as a double lock; clang's runtime does.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRCS = [os.path.join(ROOT, "paper_2511_10508_amd", "csrc", "serve.cpp"),
        os.path.join(ROOT, "tests", "native", "fake_device.cpp"),
        os.path.join(ROOT, "tests", "native", "serve_stress.cpp")]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
         "-I" + os.path.join(ROCM, "include")]


def _build(tmp_path, cxx, san, name):
    exe = str(tmp_path / name)
    cmd = [cxx] + FLAGS + san + SRCS + ["-o", exe, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


def _run(exe, args, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    res = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True,
                         timeout=240, env=env)
    out = res.stdout + res.stderr
    assert res.returncode == 0 and "serve_stress: ok" in out, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert "WARNING: ThreadSanitizer" not in out, out[-6000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "g++", ["-fsanitize=address,undefined"], "stress_asan")
    for seed in (1, 2, 3):
        _run(exe, [500, seed], {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
                                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})


CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")


@pytest.mark.skipif(not os.path.exists(CLANG), reason="needs ROCm's clang++ for ThreadSanitizer")
def test_scheduler_tsan(tmp_path):
    exe = _build(tmp_path, CLANG, ["-fsanitize=thread"], "stress_tsan")
    for seed in (1, 2, 3):
        _run(exe, [500, seed], {"TSAN_OPTIONS": "halt_on_error=1"})
