"""Pins of the FP64 warm-start network oracle against closed forms, library routines and finite
differences (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import fno


def _theta(seed, scale=0.05):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(fno.param_count()) * scale


def _grid(n):
    x = 2.0 * np.pi * np.arange(n) / n
    return np.meshgrid(x, x, indexing="ij")


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        # exact ties between two bfloat16 values: round to even
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, -0.0])])
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(fno.to_bf16(x), want)
    assert fno.to_bf16(1.0 + 2.0 ** -8) == 1.0
    assert fno.to_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_param_count():
    C, M = 32, 16
    per_layer = 2 * (2 * M * M * C * C) + C * C + C
    assert fno.OUT_CH == 2 + 2 * fno.RANK == 10
    assert fno.param_count() == C * 9 + C + 4 * per_layer + 64 * C + 64 + 10 * 64 + 10 == 4201610
    th = _theta(0)
    np.testing.assert_array_equal(fno.pack(fno.unpack(th)), th)


@pytest.mark.parametrize("n", [32, 64])
def test_gemm_formulation_equals_fft_formulation(n):
    rng = np.random.default_rng(2)
    th = _theta(3)
    a = rng.standard_normal((2, 9, n, n))
    y_fft, _ = fno.forward(th, a, spectral="fft")
    y_gemm, _ = fno.forward(th, a, spectral="gemm")
    assert np.abs(y_fft - y_gemm).max() <= 1e-12 * np.abs(y_fft).max()


def _single_channel_weights(entries):
    Rr = np.zeros((32, 16, 1, 1))
    Ri = np.zeros((32, 16, 1, 1))
    for (j, k2), r in entries.items():
        Rr[j, k2, 0, 0] = r.real
        Ri[j, k2, 0, 0] = r.imag
    return Rr, Ri


@pytest.mark.parametrize("form", ["fft", "gemm"])
def test_spectral_layer_on_single_modes(form):
    """cos(k.x) with k2 > 0 maps to Re(r e^{ik.x}); on the k2 = 0 column, cos(k1 x1) has the two
    coefficients 1/2 at +-k1 and maps to (1/2) Re(r+ e^{i k1 x1} + r- e^{-i k1 x1}); modes that are
    not retained map to zero."""
    n = 64
    X1, X2 = _grid(n)
    rp, rm, rk = 0.7 - 0.4j, -0.3 + 0.9j, 1.3 + 0.25j
    Rr, Ri = _single_channel_weights({(4, 0): rp, (32 - 4, 0): rm, (32 - 3, 5): rk})

    def S(h):
        h = h[None, None]
        if form == "fft":
            return fno.spectral_conv_fft(h, Rr, Ri)[0, 0]
        return fno._spectral_gemm(fno._Mul(False), fno.dft_bases(n), h, Rr, Ri)[0][0, 0]

    th = -3 * X1 + 5 * X2
    np.testing.assert_allclose(S(np.cos(th)), rk.real * np.cos(th) - rk.imag * np.sin(th), atol=1e-13)
    th0 = 4 * X1
    want0 = 0.5 * np.real(rp * np.exp(1j * th0) + rm * np.exp(-1j * th0))
    np.testing.assert_allclose(S(np.cos(th0)), want0, atol=1e-13)
    for k1, k2 in [(20, 3), (3, 16), (-17, 2), (0, 31)]:
        assert np.abs(S(np.cos(k1 * X1 + k2 * X2))).max() < 1e-13


@pytest.mark.parametrize("form", ["fft", "gemm"])
def test_band_limit_closed_forms(form):
    """B keeps the retained modes with |k| <= 12 and removes all others; it is symmetric."""
    n = 64
    X1, X2 = _grid(n)

    def Bop(u):
        u = u[None, None]
        if form == "fft":
            return fno.band_limit_fft(u)[0, 0]
        return fno._band_limit_gemm(fno._Mul(False), fno.dft_bases(n), u)[0, 0]

    for k1, k2 in [(0, 0), (3, 0), (-7, 5), (12, 0), (-8, 8), (0, 12), (5, -10), (-10, -6)]:
        for f in (np.cos, np.sin):
            u = f(k1 * X1 + k2 * X2)
            np.testing.assert_allclose(Bop(u), u, atol=1e-13)
    for k1, k2 in [(16, 3), (20, 0), (2, 16), (-17, 1), (9, 9), (-13, 0), (12, 1), (5, -11), (15, 15), (-16, 0)]:
        assert np.abs(Bop(np.cos(k1 * X1 + k2 * X2))).max() < 1e-13, (k1, k2)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, n, n))
    assert abs((Bop(a) * b).sum() - (a * Bop(b)).sum()) < 1e-10 * np.abs(a).sum()
    if form == "gemm":
        mul, bases = fno._Mul(False), fno.dft_bases(n)
        np.testing.assert_allclose(fno._band_limit_gemm_T(mul, bases, b[None, None])[0, 0], Bop(b), atol=1e-12)


def test_dft_bases_closed_forms():
    n = 64
    b = fno.dft_bases(n)
    # forward then inverse on the retained band is the identity on band-limited fields
    X1, X2 = _grid(n)
    rng = np.random.default_rng(4)
    h = sum(rng.standard_normal() * np.cos(k1 * X1 + k2 * X2 + rng.uniform(0, 6))
            for k1, k2 in [(0, 0), (3, 2), (-5, 7), (15, 0), (-16, 15), (2, 15)])
    Y = h @ b["F2"]
    T = b["CS"] @ Y
    M = 16
    Zr = T[:2 * M, :M] + T[2 * M:, M:]
    Zi = T[:2 * M, M:] - T[2 * M:, :M]
    Hk = np.fft.rfft2(h) / n ** 2
    rows = [k % n for k in fno.kept_k1(n)]
    np.testing.assert_allclose(Zr + 1j * Zi, Hk[rows, :M], atol=1e-14)


def test_gelu_closed_forms():
    assert fno.gelu(np.array(0.0)) == 0.0
    assert abs(fno.gelu(np.array(10.0)) - 10.0) < 1e-20
    assert abs(fno.gelu(np.array(-10.0))) < 1e-20
    assert abs(fno.gelu_grad(np.array(0.0)) - 0.5) < 1e-16
    x = np.linspace(-4, 4, 41)
    e = 1e-6
    np.testing.assert_allclose(fno.gelu_grad(x), (fno.gelu(x + e) - fno.gelu(x - e)) / (2 * e), atol=1e-9)
    want = np.array([xi * 0.5 * (1.0 + math.erf(xi / math.sqrt(2.0))) for xi in x])
    np.testing.assert_allclose(fno.gelu(x), want, rtol=1e-15, atol=1e-300)


def test_features_closed_form():
    n = 64
    X1, X2 = _grid(n)
    h = 2 * np.pi / n
    mT = np.sin(X1) + np.cos(2 * X2)
    mR = mT + 0.5 * np.cos(X2)                      # misfit cos(x2) / 2: rms 1 / (2 sqrt 2)
    a, s = fno.features(mT, mR)
    assert abs(s - 0.5 / np.sqrt(2.0)) < 1e-15
    d1 = np.cos(X1) * np.sin(h) / h                   # central differences of sin, cos
    d2 = -2 * np.sin(2 * X2) * np.sin(2 * h) / (2 * h)
    r = np.sqrt(2.0) * np.cos(X2)
    want = [mT, d1, d2, d1 * d1, d1 * d2, d2 * d2, r, r * d1, r * d2]
    for c in range(9):
        np.testing.assert_allclose(a[c], want[c], atol=1e-14)
    a0, s0 = fno.features(mT, mT)                     # identical images: no misfit channels
    assert s0 == 0.0 and not a0[6:].any()
    th = _theta(2)
    assert not fno.predict(th, mT, mT)[0].any()
    v1, z1 = fno.predict(th, mT, mR)
    v2, z2 = fno.predict(th, mT, mT + 3.0 * (mR - mT))    # the warm start scales with the misfit,
    np.testing.assert_allclose(v2, 3.0 * v1, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(z2, z1, rtol=1e-12, atol=1e-15)    # the directions do not
    assert z1.shape == (fno.RANK, 2) + mT.shape and np.abs(z1).max() > 0


def test_loss_closed_form():
    """Velocity channels: relative squared error.  Directions: 0 for any multiple of the target
    (either sign), 1 for a field orthogonal to it, nothing for a zero target."""
    rng = np.random.default_rng(5)
    R = fno.RANK
    t = rng.standard_normal((3, fno.OUT_CH, 8, 8))
    t[2, 2:] = 0.0                                               # sample 2: no direction targets
    y = rng.standard_normal(t.shape)
    y[:, :2] = t[:, :2] * np.array([1.1, 0.8, 1.0])[:, None, None, None]
    y[0, 2:] = -2.0 * t[0, 2:]                                    # sample 0: parallel
    for k in range(R):                                           # sample 1: orthogonal
        ch = slice(2 + 2 * k, 4 + 2 * k)
        u = y[1, ch]
        y[1, ch] = u - (u * t[1, ch]).sum() / (t[1, ch] ** 2).sum() * t[1, ch]
    L, dy = fno.loss(y, t)
    assert abs(L - ((0.01 + 0.04 + 0.0) + fno.DIR_WEIGHT) / 3) < 1e-14
    assert not dy[2, 2:].any()
    # scale and sign of either side do not matter
    t2, y2 = t.copy(), y.copy()
    t2[:, 2:4] *= -3.0
    y2[:, 4:6] *= 0.25
    assert abs(fno.loss(y2, t2)[0] - L) < 1e-14


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(15)
    t = rng.standard_normal((3, fno.OUT_CH, 8, 8))
    t[1, 4:6] = 0.0                                              # one slot without a target
    y = rng.standard_normal(t.shape)
    L, dy = fno.loss(y, t)
    for seed in range(3):
        d = np.random.default_rng(100 + seed).standard_normal(y.shape)
        e = 1e-6
        fd = (fno.loss(y + e * d, t)[0] - fno.loss(y - e * d, t)[0]) / (2 * e)
        assert abs(fd - (dy * d).sum()) < 1e-8 * max(1.0, abs(fd))
    # the direction part alone (velocity channels held fixed), near alignment where the angle
    # terms have a sizeable slope
    y[:, 2:] = t[:, 2:] + 0.7 * rng.standard_normal(t[:, 2:].shape)
    L, dy = fno.loss(y, t)
    d = np.zeros_like(y)
    d[:, 2:] = rng.standard_normal(d[:, 2:].shape)
    e = 1e-5
    fd = (fno.loss(y + e * d, t)[0] - fno.loss(y - e * d, t)[0]) / (2 * e)
    an = (dy * d).sum()
    assert abs(fd - an) < 1e-6 * abs(an) and abs(an) > 1e-3


def test_gradient_matches_finite_differences_per_block():
    """Every parameter block: directional derivative of the loss against central differences of
    the FFT-formulation forward (exact arithmetic)."""
    n = 32
    rng = np.random.default_rng(6)
    th = _theta(7, 0.08)
    a = rng.standard_normal((2, 9, n, n))
    t = rng.standard_normal((2, fno.OUT_CH, n, n))
    y, cache = fno.forward(th, a)
    _, dy = fno.loss(y, t)
    g = fno.backward(cache, dy)
    f = lambda p: fno.loss(fno.forward(p, a, spectral="fft")[0], t)[0]   # noqa: E731
    L0 = f(th)
    off = 0
    for name, shp in fno.param_shapes():
        k = int(np.prod(shp))
        d = np.zeros_like(th)
        d[off:off + k] = rng.standard_normal(k)
        eps = 3e-5 * np.linalg.norm(th[off:off + k]) / np.linalg.norm(d)   # relative to the block
        fd = (f(th + eps * d) - f(th - eps * d)) / (2 * eps)
        an = float(g @ d)
        # truncation O(eps^2) plus the rounding of L in the difference quotient
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-14 * L0 / eps, (name, fd, an)
        assert abs(an) > 1e3 * 1e-14 * L0 / eps, (name, an)   # the check has room to fail
        off += k


def test_bf16_network_stays_close_to_exact():
    n = 32
    rng = np.random.default_rng(8)
    th = _theta(9)
    a = rng.standard_normal((2, 9, n, n))
    t = rng.standard_normal((2, fno.OUT_CH, n, n))
    y, c = fno.forward(th, a)
    yb, cb = fno.forward(th, a, bf16=True)
    assert 1e-5 < np.linalg.norm(yb - y) / np.linalg.norm(y) < 1e-2
    g = fno.backward(c, fno.loss(y, t)[1])
    gb = fno.backward(cb, fno.loss(yb, t)[1])
    assert np.linalg.norm(gb - g) / np.linalg.norm(g) < 3e-2


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(10)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    th1, m, v = fno.adam_step(th, g, z, z, 1, 1e-3, eps=1e-8)
    np.testing.assert_allclose(th1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    # a constant gradient keeps the bias-corrected moments equal to it
    th2, m2, v2 = fno.adam_step(th1, g, m, v, 2, 1e-3, eps=0.0)
    np.testing.assert_allclose(th2, th1 - 1e-3 * np.sign(g), rtol=1e-12)
