"""The host drivers (registration library and warm-start network) under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): regnk_host.hip (net_host.hip) is compiled with g++ for the
host, against the range-checking launch functions of tests/regmock/ (tests/netmock/), into a
standalone program (asan_driver.cpp there) that calls every entry point for a few grids and models.
Heap and stack misuse, leaks and undefined behaviour in the host code end the program with a report;
every launch is range-checked as in test_reg_host_cpu.py and test_net_host_cpu.py."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_driver_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "asan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "tests", "regmock"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1503_00757_amd", "csrc"),
           "-x", "c++", os.path.join(ROOT, "paper_1503_00757_amd", "csrc", "regnk_host.hip"),
           "-x", "c++", os.path.join(ROOT, "tests", "regmock", "regmock_kernels.cpp"),
           "-x", "c++", os.path.join(ROOT, "tests", "regmock", "asan_driver.cpp"), "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_network_host_driver_is_clean_under_sanitizers(tmp_path):
    """The same for the warm-start network's host driver (net_host.hip) against tests/netmock/."""
    exe = str(tmp_path / "net_asan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "tests", "netmock"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1503_00757_amd", "csrc"),
           "-x", "c++", os.path.join(ROOT, "paper_1503_00757_amd", "csrc", "net_host.hip"),
           "-x", "c++", os.path.join(ROOT, "tests", "netmock", "netmock_kernels.cpp"),
           "-x", "c++", os.path.join(ROOT, "tests", "netmock", "asan_driver.cpp"), "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
