"""The library's mixed-radix FFT (device_common.hpp: the planner mr_plan and the LDS Stockham transform
fft_mr, radices 2, 3, 4, 5, 8) compiled for the host with one emulated thread and checked against
numpy's FFT on every even length of the form 2^a 3^b 5^c up to 2048 that is not a power of two, in
double and single precision, forward and inverse.  No GPU involved."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("devmock") / "libmrfft.so")
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-I", os.path.join(ROOT, "tests", "devmock"),
           "-I", os.path.join(ROOT, "paper_1503_00757_amd", "csrc"), "-x", "c++",
           os.path.join(ROOT, "tests", "devmock", "mr_fft_cpu.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    L = ctypes.CDLL(out)
    dp = ctypes.POINTER(ctypes.c_double)
    L.mr_fft.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
    L.mr_plan_radices.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    return L


def smooth_lengths():
    out = []
    for n in range(8, 2049, 2):
        m = n
        for q in (2, 3, 5):
            while m % q == 0:
                m //= q
        if m == 1 and n & (n - 1):
            out.append(n)
    return out


def run(L, x, inv, single):
    n = len(x)
    xi = np.ascontiguousarray(np.stack([x.real, x.imag], -1).ravel())
    w = np.exp(-2j * np.pi * np.arange(n) / n)
    wi = np.ascontiguousarray(np.stack([w.real, w.imag], -1).ravel())
    out = np.zeros(2 * n)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = L.mr_fft(n, inv, single, xi.ctypes.data_as(dp), wi.ctypes.data_as(dp), out.ctypes.data_as(dp))
    assert rc == 0
    return out[0::2] + 1j * out[1::2]


def test_planner_factors_smooth_lengths_only(lib):
    r = (ctypes.c_int * 16)()
    for n in smooth_lengths():
        k = lib.mr_plan_radices(n, r)
        assert k > 0 and int(np.prod([r[i] for i in range(k)])) == n and all(r[i] in (2, 3, 4, 5, 8) for i in range(k))
    for n in (14, 22, 2046, 998):          # a prime factor other than 2, 3, 5
        assert lib.mr_plan_radices(n, r) == 0


@pytest.mark.parametrize("single", [0, 1])
def test_mixed_radix_fft_matches_numpy(lib, single):
    rng = np.random.default_rng(11)
    tol = 1e-13 if not single else 2e-6
    lengths = smooth_lengths()
    assert {96, 150, 1000, 250, 2000, 1536} <= set(lengths)
    for n in lengths:
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        ref = np.fft.fft(x)
        assert np.linalg.norm(run(lib, x, 0, single) - ref) <= tol * np.linalg.norm(ref) * np.log2(n), n
        refi = np.fft.ifft(x) * n
        assert np.linalg.norm(run(lib, x, 1, single) - refi) <= tol * np.linalg.norm(refi) * np.log2(n), n
