"""Host-side runtime tests, no GPU: the server's scheduling core (serve_core.h,
against a fake device, a fake clock and a mock memory budget) and the weight
packing (pack.cpp), each compiled with g++ and run under the address and
undefined-behaviour sanitizers, and the server core under the thread
sanitizer too (concurrent submitters, a poller and the worker thread).
The C++ test programs are under tests/host/."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2304_09439_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
INCLUDE = os.path.join(ROOT, "include")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
TSAN = ["-fsanitize=thread"]

PROGRAMS = {
    "serve_core": (["serve_core_test.cpp"], []),
    "pack": (["pack_test.cpp"], [os.path.join(CSRC, "pack.cpp")]),
}


def _gxx():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    return gxx


def _build_and_run(tmp_path, name, sanitizer, args=()):
    tests, extra = PROGRAMS[name]
    exe = tmp_path / f"{name}_{'tsan' if sanitizer is TSAN else 'asan'}"
    cmd = [_gxx(), "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", *sanitizer, "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(HOST, t) for t in tests], *extra, "-o", str(exe), "-pthread"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, f"compile failed:\n{res.stderr[-4000:]}"
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    run = subprocess.run([str(exe), *args], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, f"{name} failed:\n{run.stdout[-3000:]}\n{run.stderr[-6000:]}"
    assert "all tests passed" in run.stdout
    return run.stdout


def test_serve_core_under_address_and_ub_sanitizers(tmp_path):
    _build_and_run(tmp_path, "serve_core", ASAN, ["4"])


def test_serve_core_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, "serve_core", TSAN, ["3"])


def test_packing_under_address_and_ub_sanitizers(tmp_path):
    _build_and_run(tmp_path, "pack", ASAN)
