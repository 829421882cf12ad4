"""The library's host-only logic (csrc/lb_host.cpp: parameter validation, the
tuning-cache parser, checkpoint header checks) built with g++ and
AddressSanitizer + UndefinedBehaviorSanitizer (host code only, no GPU) and
run against valid and malformed inputs (tests/sanitize/host_fuzz.cpp): any
invalid access, leak or undefined behaviour aborts the harness.  A second
build with ThreadSanitizer covers the initial-field checks' host threads."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1004_5058_amd", "csrc")


def test_host_logic_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "host_fuzz")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Werror",
           "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize", "host_fuzz.cpp"), os.path.join(CSRC, "lb_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout


def test_host_logic_under_tsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "host_fuzz_tsan")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-Wall", "-Werror",
           "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize", "host_fuzz.cpp"), os.path.join(CSRC, "lb_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    if "FATAL: ThreadSanitizer" in r.stderr:
        # the runtime could not start here (its shadow memory layout); a race
        # found is reported as a WARNING and fails below
        pytest.skip("ThreadSanitizer's runtime cannot start on this host: " + r.stderr.strip()[-200:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
