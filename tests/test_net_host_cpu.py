"""The warm-start network's host driver (net_host.hip, compiled with g++) run on the CPU against
bounds-checked CPU versions of its kernels (tests/netmock): every operand range of every launch is
checked against the caller's buffers, and forward, reverse pass, loss, Adam and predict are
compared with the FP64 oracle evaluated with bfloat16 multiplicands.  No GPU involved."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import synthdata
from oracle import fno

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("netmock") / "libnetmock.so")
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared",
           "-I", os.path.join(ROOT, "tests", "netmock"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1503_00757_amd", "csrc"),
           "-x", "c++", os.path.join(ROOT, "paper_1503_00757_amd", "csrc", "net_host.hip"),
           "-x", "c++", os.path.join(ROOT, "tests", "netmock", "netmock_kernels.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    L = ctypes.CDLL(out)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.mock_register.argtypes = [vp, sz]
    L.mock_last_error.restype = ctypes.c_char_p
    L.reg_fno_workspace_bytes.argtypes = [i32, i32, ctypes.POINTER(sz)]
    L.reg_fno_create.argtypes = [i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    L.reg_fno_destroy.argtypes = [vp]
    L.reg_fno_features.argtypes = [vp, vp, vp, vp, vp]
    L.reg_fno_target.argtypes = [vp, vp, vp, vp, vp]
    L.reg_fno_gather.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    L.reg_fno_forward.argtypes = [vp, vp, vp, vp]
    L.reg_fno_backward.argtypes = [vp, vp, vp, vp, vp]
    L.reg_fno_adam.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
    L.reg_fno_predict.argtypes = [vp, vp, vp, vp, vp, vp]
    return L


class Net:
    def __init__(self, L, n, B):
        self.L, self.n, self.B = L, n, B
        L.mock_reset()
        nb = ctypes.c_size_t()
        assert L.reg_fno_workspace_bytes(n, B, ctypes.byref(nb)) == 0
        self.raw = np.zeros(nb.value + 256, dtype=np.uint8)
        base = self.raw.ctypes.data
        self.ws = (base + 255) // 256 * 256
        L.mock_register(ctypes.c_void_p(self.ws), nb.value)   # only the aligned part
        self.h = ctypes.c_void_p()
        rc = L.reg_fno_create(n, B, ctypes.c_void_p(self.ws), nb.value, None, ctypes.byref(self.h))
        assert rc == 0, L.mock_last_error()

    def buf(self, a):
        a = np.ascontiguousarray(a)
        self.L.mock_register(ctypes.c_void_p(a.ctypes.data), a.nbytes)
        return a

    def check(self, rc):
        assert rc == 0, self.L.mock_last_error()
        assert self.L.mock_violations() == 0


def _pairs(B, n):
    mTs, mRs = [], []
    for b in range(B):
        w = synthdata.make_workload(5, pair=b, n=n)
        mTs.append(w.mT)
        mRs.append(np.roll(w.mT, (1 + b, -2), axis=(0, 1)) * 0.9 + 0.05)
    return mTs, mRs


def _theta_test():
    """Initial weights with the output bias removed: with it, the untrained output is a near-constant
    field whose bfloat16 rounding in the band limit sits on one rounding boundary, which turns
    FP32-versus-FP64 differences of 1e-8 into whole-ulp flips of many values at once."""
    th = synthdata.network_init().copy()
    th[-fno.OUT_CH:] = 0.0
    return th


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _assert_forward_parity(y, theta, a):
    """The HIP output against the oracle network with bfloat16 multiplicands.  Differences come
    from bfloat16 rounding decisions that flip where FP32 and FP64 intermediates straddle a rounding
    boundary (small DFT coefficients next to a large mean), so the bound is stated against the
    size of the bfloat16 effect itself: within 1e-3, and within a fifth of the distance between
    the bfloat16 and the exact network (a wrong rounding mode, index or sign exceeds it)."""
    y_bf, cache = fno.forward(theta, a, bf16=True)
    y_ex, _ = fno.forward(theta, a, bf16=False)
    err, eff = _rel(y, y_bf), _rel(y_bf, y_ex)
    assert err < 1e-3 and err < 0.2 * eff, (err, eff)
    return y_bf, cache


@pytest.mark.parametrize("n,B", [(32, 2), (64, 3)])
def test_forward_backward_adam_match_oracle(lib, n, B):
    net = Net(lib, n, B)
    theta = _theta_test().astype(np.float64)
    mTs, mRs = _pairs(B, n)
    a = np.stack([fno.features(t, r)[0] for t, r in zip(mTs, mRs)])            # (B, 4, n, n)
    rng = np.random.default_rng(11)
    t = rng.standard_normal((B, fno.OUT_CH, n, n)) * 0.05
    t[0, 4:6] = 0.0                                                            # a slot without a target
    th32 = net.buf(theta.astype(np.float32))
    a_dev = net.buf(np.transpose(a, (1, 0, 2, 3)).astype(np.float32))       # [9][B][n][n]
    t_dev = net.buf(np.transpose(t, (1, 0, 2, 3)).astype(np.float32))
    out = net.buf(np.zeros((fno.OUT_CH, B, n, n), np.float32))
    grad = net.buf(np.zeros(fno.param_count(), np.float32))
    loss = net.buf(np.zeros(1))
    vp = lambda x: ctypes.c_void_p(x.ctypes.data)   # noqa: E731
    assert lib.reg_fno_backward(net.h, vp(th32), vp(t_dev), vp(grad), vp(loss)) == -6   # no forward yet
    net.check(lib.reg_fno_forward(net.h, vp(th32), vp(a_dev), vp(out)))
    y = np.transpose(out, (1, 0, 2, 3)).astype(np.float64)
    y_or, cache = _assert_forward_parity(y, th32.astype(np.float64), a)
    net.check(lib.reg_fno_backward(net.h, vp(th32), vp(t_dev), vp(grad), vp(loss)))
    t32 = t.astype(np.float32).astype(np.float64)
    L_own = fno.loss(y, t32)[0]          # the loss kernel on the library's own output
    assert abs(loss[0] - L_own) < 1e-9 * L_own
    L_or, dy = fno.loss(y_or, t32)
    g_or = fno.backward(cache, dy)
    off = 0
    for name, shp in fno.param_shapes():
        k = int(np.prod(shp))
        # Spectral-weight gradients are batch-size sums of bfloat16 products whose real and
        # imaginary terms largely cancel (bfloat16 vs exact arithmetic differs by up to 1e-1 on
        # them), so the rare rounding flips between FP32 and FP64 intermediates show up at 1e-3;
        # a wrong index, sign or transpose gives O(1).
        tol = 1e-2 if name[0] == "R" else 1e-3
        assert _rel(grad[off:off + k].astype(np.float64), g_or[off:off + k]) < tol, name
        off += k
    m = net.buf(np.zeros(fno.param_count(), np.float32))
    v = net.buf(np.zeros(fno.param_count(), np.float32))
    p0 = th32.copy()
    net.check(lib.reg_fno_adam(net.h, vp(th32), vp(grad), vp(m), vp(v), 1, 1e-3, 0.9, 0.999, 1e-8))
    p_or, _, _ = fno.adam_step(p0.astype(np.float64), grad.astype(np.float64), 0.0, 0.0, 1, 1e-3)
    assert np.abs(th32 - p_or).max() < 1e-6


def test_gather_and_predict(lib):
    n = 32
    net = Net(lib, n, 3)
    rng = np.random.default_rng(12)
    vp = lambda x: ctypes.c_void_p(x.ctypes.data)   # noqa: E731
    data = net.buf(rng.standard_normal((5, 4, n, n)).astype(np.float32))
    idx = net.buf(np.array([4, 0, 9], np.int32))   # 9 is outside the set: zeros
    out = net.buf(np.full((4, 3, n, n), 7.0, np.float32))
    net.check(lib.reg_fno_gather(net.h, vp(data), 5, 4, vp(idx), None, vp(out)))
    np.testing.assert_array_equal(out[:, 0], data[4])
    np.testing.assert_array_equal(out[:, 1], data[0])
    assert not out[:, 2].any()

    one = Net(lib, n, 1)
    theta = one.buf(_theta_test())
    mTs, mRs = _pairs(1, n)
    mT, mR = one.buf(mTs[0]), one.buf(mRs[0])
    feat = one.buf(np.zeros((9, n, n), np.float32))
    scale = one.buf(np.zeros(1))
    one.check(lib.reg_fno_features(one.h, vp(mT), vp(mR), vp(feat), vp(scale)))
    a_or, s_or = fno.features(mT, mR)
    np.testing.assert_allclose(feat, a_or, rtol=1e-6, atol=1e-6 * np.abs(a_or).max())
    assert abs(scale[0] - s_or) < 1e-14 * s_or
    v = one.buf(np.random.default_rng(3).standard_normal((2, n, n)))
    dirs_in = one.buf(np.random.default_rng(5).standard_normal((fno.RANK, 2, n, n)))
    tgt = one.buf(np.full((fno.OUT_CH, n, n), 7.0, np.float32))
    one.check(lib.reg_fno_target(one.h, vp(v), vp(scale), None, vp(tgt)))
    np.testing.assert_allclose(tgt[:2], v / s_or, rtol=1e-6)
    assert not tgt[2:].any()                                     # no directions: zero targets
    one.check(lib.reg_fno_target(one.h, vp(v), vp(scale), vp(dirs_in), vp(tgt)))
    np.testing.assert_allclose(tgt[2:], dirs_in.reshape(-1, n, n), rtol=1e-6)
    v0 = one.buf(np.zeros((2, n, n)))
    dirs = one.buf(np.zeros((fno.RANK, 2, n, n)))
    one.check(lib.reg_fno_predict(one.h, vp(theta), vp(mT), vp(mR), vp(v0), vp(dirs)))
    y = np.concatenate([v0 / s_or, dirs.reshape(-1, n, n)])[None]
    _assert_forward_parity(y, theta.astype(np.float64), a_or[None])
    v0b = one.buf(np.zeros((2, n, n)))
    one.check(lib.reg_fno_predict(one.h, vp(theta), vp(mT), vp(mR), vp(v0b), None))   # directions not wanted
    np.testing.assert_array_equal(v0b, v0)
    assert lib.reg_fno_predict(net.h, vp(theta), vp(mT), vp(mR), vp(v0), None) == -1   # batch 3 handle


def transform_scalar(m, code):
    """Image under the grid symmetry `code` (bit 0 swap axes, bits 1 / 2 flip axis 1 / 2):
    out(i) = m(P(F(i))), flips i -> (n - i) mod n."""
    t = m.T if code & 1 else m
    for ax, bit in ((0, 2), (1, 4)):
        if code & bit:
            t = np.roll(np.flip(t, ax), 1, ax)
    return t


def transform_vector(v, code):
    w = [transform_scalar(v[0], code), transform_scalar(v[1], code)]
    if code & 1:
        w = w[::-1]
    return np.stack([w[0] * (-1 if code & 2 else 1), w[1] * (-1 if code & 4 else 1)])


def test_gather_symmetries_match_transformed_images(lib):
    """Features gathered under each of the 8 grid symmetries equal the features of the transformed
    image pair; velocities transform as vectors."""
    n, B = 32, 8
    net = Net(lib, n, B)
    vp = lambda x: ctypes.c_void_p(x.ctypes.data)   # noqa: E731
    mTs, mRs = _pairs(2, n)
    feats = net.buf(np.stack([fno.features(t, r)[0] for t, r in zip(mTs, mRs)]).astype(np.float32))
    vel = net.buf(np.random.default_rng(4).standard_normal((2, 2, n, n)).astype(np.float32))
    idx = net.buf(np.array([1, 0, 1, 0, 1, 0, 1, 1], np.int32))
    sym = net.buf(np.arange(8, dtype=np.int32))
    out = net.buf(np.zeros((9, B, n, n), np.float32))
    outv = net.buf(np.zeros((2, B, n, n), np.float32))
    net.check(lib.reg_fno_gather(net.h, vp(feats), 2, 9, vp(idx), vp(sym), vp(out)))
    net.check(lib.reg_fno_gather(net.h, vp(vel), 2, 2, vp(idx), vp(sym), vp(outv)))
    for b in range(B):
        p, code = idx[b], sym[b]
        want, _ = fno.features(transform_scalar(mTs[p], code), transform_scalar(mRs[p], code))
        np.testing.assert_allclose(out[:, b], want, rtol=1e-6, atol=1e-6 * np.abs(want).max())
        np.testing.assert_array_equal(outv[:, b], transform_vector(vel[p], code))
    # the target layout (velocity, then the direction fields): every channel pair is a vector
    tg = net.buf(np.random.default_rng(6).standard_normal((2, fno.OUT_CH, n, n)).astype(np.float32))
    outt = net.buf(np.zeros((fno.OUT_CH, B, n, n), np.float32))
    net.check(lib.reg_fno_gather(net.h, vp(tg), 2, fno.OUT_CH, vp(idx), vp(sym), vp(outt)))
    for b in range(B):
        p, code = idx[b], sym[b]
        for c in range(0, fno.OUT_CH, 2):
            np.testing.assert_array_equal(outt[c:c + 2, b], transform_vector(tg[p, c:c + 2], code))
    bad = net.buf(np.zeros((3, 2, n, n), np.float32))
    assert lib.reg_fno_gather(net.h, vp(bad), 3, 2, vp(idx), vp(sym), vp(outv)) == 0   # velocity layout
    assert lib.reg_fno_gather(net.h, vp(feats), 2, 3, vp(idx), vp(sym), vp(out)) == -1  # unknown layout


def test_argument_checks(lib):
    nb = ctypes.c_size_t()
    for n, B in [(16, 1), (48, 1), (2048, 1), (64, 0), (64, 65)]:
        assert lib.reg_fno_workspace_bytes(n, B, ctypes.byref(nb)) == -1
    assert lib.reg_fno_workspace_bytes(1024, 64, ctypes.byref(nb)) == 0
