"""The library's host-only code under AddressSanitizer, UndefinedBehaviorSanitizer
and ThreadSanitizer.

The tearing planner (plan.cpp, with its refresh; its passes over large circuits
run on several host threads) and the host-only C ABI calls (host_api.cpp) are
compiled for the CPU with g++ and the sanitizers, linked with
tests/host_abi_check.cpp, and run: every check must hold and no sanitizer may
report (each report aborts the run).  No device code is involved.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0910_0663_amd", "csrc")


def build(tmp_path, name, flags):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "host_api.cpp"),
           os.path.join(ROOT, "tests", "host_abi_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = build(tmp_path, "host_abi_check_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    # verify_asan_link_order=0: the environment may preload a library ahead of ASan's runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host ABI checks passed" in r.stdout
    assert "Sanitizer" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_threaded_planner_under_thread_sanitizer(tmp_path):
    exe = build(tmp_path, "host_abi_check_tsan", ["-fsanitize=thread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:abort_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host ABI checks passed" in r.stdout
    assert "ThreadSanitizer" not in r.stderr, r.stderr
