"""The request loop (csrc/serve.hip) on the CPU: compiled with g++ against stand-ins of the library
(tests/serve_harness/), run under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer. Covers concurrent clients, admission by device footprint (the bytes reserved by
resident jobs never exceed the budget), the slot limit, the bounded queue (WFQ_EAGAIN), unknown and
already-retrieved tickets (WFQ_ENOTFOUND), a job that can never fit (WFQ_ENOMEM) and stop with work
pending. No GPU is used."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "serve_harness")
SERVE = os.path.join(ROOT, "paper_2103_00438_amd", "csrc", "serve.hip")


def _build_and_run(tmp_path, flags, name):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    # compile the loop's own source as C++ beside the stand-in headers
    src = tmp_path / "serve.cpp"
    shutil.copyfile(SERVE, src)
    exe = tmp_path / name
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, f"-I{HARNESS}",
           f"-I{os.path.join(ROOT, 'include')}", str(src), os.path.join(HARNESS, "stub_lib.cpp"),
           os.path.join(HARNESS, "driver.cpp"), "-o", str(exe), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               TSAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe), "5"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK: 0 failed checks" in r.stdout


def test_serve_loop_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined"], "serve_asan")


def test_serve_loop_tsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], "serve_tsan")
