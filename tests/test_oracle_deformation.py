"""Pins of the oracle's deformation diagnostics (CPU only).

Closed forms: a constant velocity gives u_1 = v and F_1 = I; a shear flow v = (a sin x2, 0) gives
u_1 = v and F_1 = [[1, a cos x2], [0, 1]] (both linear in t, which Heun integrates exactly); the
compressible flow v = (a sin x1, 0) has the characteristic solution tan(x/2) = tan(x0/2) e^{a t},
with F_11 = sin(x) / sin(x0) and u_1 = x - x0, approached at second order in n_t.  For a
divergence-free velocity det F_1 approaches 1, and det F_1 approaches 1 / det(I - grad u_1) (the
Eulerian relation of the two diagnostics) as n_t grows.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, Params
from oracle.deformation import deformation, det2, summary


def coords(n):
    x = np.arange(n) * 2 * np.pi / n
    return x[:, None] + 0 * x[None, :], 0 * x[:, None] + x[None, :]


def params(n, nt):
    return Params(n, n, nt, "H1", "none", 1e-2, 0.0)


def test_constant_velocity():
    n = 16
    g = Grid(n, n)
    v = np.stack([np.full((n, n), 0.3), np.full((n, n), -0.2)])
    u, F = deformation(g, params(n, 4), v)
    assert np.allclose(u, v, atol=1e-14)
    assert np.allclose(F[0, 0], 1) and np.allclose(F[1, 1], 1)
    assert np.abs(F[0, 1]).max() < 1e-14 and np.abs(F[1, 0]).max() < 1e-14


def test_shear_flow_exact():
    n, a = 32, 0.4
    g = Grid(n, n)
    x1, x2 = coords(n)
    v = np.stack([a * np.sin(x2), 0 * x2])
    u, F = deformation(g, params(n, 3), v)
    assert np.allclose(u, v, atol=1e-13)
    assert np.allclose(F[0, 1], a * np.cos(x2), atol=1e-13)      # F_12 = d_2 v_1 t
    assert np.abs(F[1, 0]).max() < 1e-13                         # not F_21: the index order is pinned
    assert np.allclose(F[0, 0], 1, atol=1e-13) and np.allclose(F[1, 1], 1, atol=1e-13)
    assert np.allclose(det2(F), 1.0, atol=1e-13)


def compressible_exact(n, a):
    x1, _ = coords(n)
    xc = np.where(x1 > np.pi, x1 - 2 * np.pi, x1)                 # (-pi, pi]
    x0 = 2 * np.arctan(np.tan(xc / 2) * np.exp(-a))
    with np.errstate(invalid="ignore", divide="ignore"):
        f11 = np.sin(xc) / np.sin(x0)
    f11 = np.where(np.isclose(xc, 0), np.exp(a), f11)             # fixed points: linearised flow
    f11 = np.where(np.isclose(np.abs(xc), np.pi), np.exp(-a), f11)
    return xc - x0, f11


def test_compressible_flow_second_order():
    n, a = 64, 0.5
    g = Grid(n, n)
    x1, _ = coords(n)
    v = np.stack([a * np.sin(x1), 0 * x1])
    u_ex, f_ex = compressible_exact(n, a)
    errs = []
    for nt in (16, 32, 64):
        u, F = deformation(g, params(n, nt), v)
        assert np.abs(F[0, 1]).max() < 1e-13 and np.abs(F[1, 0]).max() < 1e-13
        assert np.allclose(F[1, 1], 1, atol=1e-13) and np.abs(u[1]).max() < 1e-13
        errs.append((np.abs(F[0, 0] - f_ex).max(), np.abs(u[0] - u_ex).max()))
    for k in range(2):
        for j in range(2):
            assert 3.0 < errs[k][j] / errs[k + 1][j] < 5.0, errs      # O(h_t^2)
    assert errs[-1][0] < 1e-3 and errs[-1][1] < 1e-3
    d = det2(F)
    assert np.allclose(d, F[0, 0] * F[1, 1])


def test_divergence_free_keeps_volume_and_eulerian_relation():
    n = 32
    g = Grid(n, n)
    rng = np.random.default_rng(3)
    v = sd.scale_to_max(sd.random_velocity(n, n, 3, rng, True, False), 0.5)
    errs, rel = [], []
    for nt in (8, 16, 32):
        u, F = deformation(g, params(n, nt), v)
        dF = det2(F)
        errs.append(np.abs(dF - 1).max())
        gu = [[np.real(np.fft.ifft2(1j * (np.fft.fftfreq(n, 1 / n)[:, None] if l == 0 else np.fft.fftfreq(n, 1 / n)[None, :]) * np.fft.fft2(u[i]))) for l in range(2)] for i in range(2)]
        dety = (1 - gu[0][0]) * (1 - gu[1][1]) - gu[0][1] * gu[1][0]
        rel.append(np.abs(dF - 1 / dety).max())
        mn, mx, mean = summary(dF)
        assert mn <= mean <= mx and mn > 0
    assert errs[-1] < 1e-3 and errs[0] / errs[-1] > 10
    assert rel[-1] < 1e-2 and rel[0] > rel[-1]
