"""The CPU oracle and the library's host bookkeeping (symmetric-heap
allocator, serving admission budget) built with AddressSanitizer and
UndefinedBehaviorSanitizer by the host compiler and driven by small test
programs; any sanitizer report or failed check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd_build, exe):
    r = subprocess.run(cmd_build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout, r.stderr)
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_allocator_and_admission_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_logic")
    _run(["g++", "-std=c++17", *SAN, "-pthread", "-I", os.path.join(ROOT, "paper_2607_08006_amd", "csrc"),
          os.path.join(HOST, "host_logic_test.cpp"), os.path.join(ROOT, "paper_2607_08006_amd", "csrc", "hostalloc.cpp"),
          "-o", exe], exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", os.path.join(HOST, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "vshmem_oracle.c"), "-o", exe], exe)
