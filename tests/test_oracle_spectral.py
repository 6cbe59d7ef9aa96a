"""Pins of the oracle's spectral operators against closed forms and invariants (CPU only).

Q1 exact spectral derivatives of band-limited sinusoids; Q2 skew symmetry of the derivative and of
the transport operator; Q6 properties of the projection K (Sec. 3.3, eq. (project-body-force));
the regularisation operator A against the seminorm definitions of eq. (reg-v); the preconditioner
of App. E.2.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, Params, spectral, transport, reduced


def sinus(n1, n2, a, b, phase=0.3):
    x1, x2 = sd.grid_coords(n1, n2)
    X1, X2 = np.meshgrid(x1, x2, indexing="ij")
    return X1, X2, np.sin(a * X1 + b * X2 + phase)


@pytest.mark.parametrize("n1,n2", [(8, 8), (16, 12), (32, 64)])
def test_q1_derivative_of_sinusoid_is_exact(n1, n2):
    g = Grid(n1, n2)
    for a in range(-(n1 // 2) + 1, n1 // 2):
        for b in (-(n2 // 2) + 1, 0, 1, n2 // 2 - 1):
            X1, X2, u = sinus(n1, n2, a, b)
            c = np.cos(a * X1 + b * X2 + 0.3)
            assert np.abs(spectral.d(g, u, 0) - a * c).max() < 1e-12 * max(1, abs(a)) * n1
            assert np.abs(spectral.d(g, u, 1) - b * c).max() < 1e-12 * max(1, abs(b)) * n2
            w = np.stack([u, 2 * u])
            assert np.abs(spectral.div(g, w) - (a + 2 * b) * c).max() < 1e-11 * (n1 + n2)


def test_q1_nyquist_mode_has_zero_derivative():
    g = Grid(8, 8)
    x1, x2 = sd.grid_coords(8, 8)
    u = np.cos(4 * x1)[:, None] * np.ones(8)[None, :]          # pure Nyquist in x1
    assert np.abs(spectral.d(g, u, 0)).max() < 1e-14


@pytest.mark.parametrize("n1,n2", [(8, 8), (16, 10)])
def test_q2_skew_symmetry(n1, n2):
    g = Grid(n1, n2)
    rng = np.random.default_rng(7)
    u, w = rng.standard_normal((2, n1, n2))                   # full spectrum incl. Nyquist
    for ax in (0, 1):
        lhs = g.inner(spectral.d(g, u, ax), w)
        rhs = -g.inner(u, spectral.d(g, w, ax))
        assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + 1)
    v = rng.standard_normal((2, n1, n2))
    lhs = g.inner(transport.L(g, v, u), w)
    rhs = g.inner(u, transport.LT(g, v, w))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def _params(constraint, norm="H1", beta_w=None, n=16):
    bw = (1e-3 if beta_w is None else beta_w) if constraint == "mass_source" else 0.0
    return Params(n, n, 2, norm, constraint, 1e-2, bw)


def test_q6_leray_projection():
    g = Grid(16, 16)
    p = _params("divfree")
    b = np.random.default_rng(1).standard_normal((2, 16, 16))
    Kb = spectral.apply_K(g, p, b)
    assert np.abs(spectral.div(g, Kb)).max() < 1e-12
    assert np.abs(spectral.apply_K(g, p, Kb) - Kb).max() < 1e-12           # K^2 = K
    c = np.random.default_rng(2).standard_normal((2, 16, 16))
    assert abs(g.inner(Kb, c) - g.inner(b, spectral.apply_K(g, p, c))) < 1e-12   # K = K^T
    # divergence-free fields are left alone; gradients (k != 0) are removed
    psi = sd.random_field(16, 16, 5, 3)
    rot = np.stack([-spectral.d(g, psi, 1), spectral.d(g, psi, 0)])
    assert np.abs(spectral.apply_K(g, p, rot) - rot).max() < 1e-12
    gr = spectral.grad(g, psi)
    assert np.abs(spectral.apply_K(g, p, gr)).max() < 1e-12


@pytest.mark.parametrize("norm", ["H1", "H2"])
def test_q6_mass_source_eigenvalues_and_limits(norm):
    g = Grid(16, 16)
    p = _params("mass_source", norm)
    X1, X2, u = sinus(16, 16, 3, 2)
    grad_mode = np.stack([3 * np.cos(3 * X1 + 2 * X2 + 0.3), 2 * np.cos(3 * X1 + 2 * X2 + 0.3)])
    ksq = 13.0
    Ahat = ksq if norm == "H1" else ksq ** 2
    Mhat = 1.0 + p.beta_v * Ahat / (p.beta_w * ksq * (ksq + 1))
    assert np.abs(spectral.apply_K(g, p, grad_mode) - (1 - 1 / Mhat) * grad_mode).max() < 1e-12
    rot_mode = np.stack([-2 * np.cos(3 * X1 + 2 * X2 + 0.3), 3 * np.cos(3 * X1 + 2 * X2 + 0.3)])
    assert np.abs(spectral.apply_K(g, p, rot_mode) - rot_mode).max() < 1e-12
    if norm == "H1":   # the printed M of eq. (project-body-force): beta_v (beta_w(|k|^2+1))^{-1} + 1
        assert abs(Mhat - (p.beta_v / (p.beta_w * (ksq + 1)) + 1)) < 1e-14
    b = np.random.default_rng(3).standard_normal((2, 16, 16))
    big = spectral.apply_K(g, _params("mass_source", norm, beta_w=1e12), b)
    assert np.abs(big - spectral.apply_K(g, _params("divfree", norm), b)).max() < 1e-8
    small = spectral.apply_K(g, _params("mass_source", norm, beta_w=1e-14), b)
    assert np.abs(small - b).max() < 1e-8
    # K^{-1} K = I
    assert np.abs(spectral.apply_Kinv(g, p, spectral.apply_K(g, p, b)) - b).max() < 1e-10


@pytest.mark.parametrize("norm", ["H1", "H2", "H3"])
def test_regulariser_matches_seminorm_definition(norm):
    """<v, A v> equals |v|^2_{H1} = int grad v : grad v, |v|^2_{H2} = int Lap v . Lap v (eq. (reg-v)), or
    |v|^2_{H3} = int grad Lap v : grad Lap v, all written with the (pinned) spectral derivative."""
    g = Grid(16, 16)
    p = _params("none", norm)
    v = sd.random_vec(16, 16, 6, 4)
    lhs = g.inner(v, spectral.apply_A(g, p, v))
    if norm == "H1":
        rhs = sum(g.inner(spectral.d(g, v[c], a), spectral.d(g, v[c], a)) for c in (0, 1) for a in (0, 1))
    else:
        lap = [spectral.d(g, spectral.d(g, v[c], 0), 0) + spectral.d(g, spectral.d(g, v[c], 1), 1) for c in (0, 1)]
        if norm == "H2":
            rhs = sum(g.inner(l, l) for l in lap)
        else:
            rhs = sum(g.inner(spectral.d(g, l, a), spectral.d(g, l, a)) for l in lap for a in (0, 1))
    assert abs(lhs - rhs) < 1e-12 * rhs
    X1, X2, u = sinus(16, 16, 3, -2)
    w = np.stack([u, 0 * u])
    fac = {"H1": 13.0, "H2": 169.0, "H3": 2197.0}[norm]
    assert np.abs(spectral.apply_A(g, p, w) - fac * w).max() < 1e-12 * fac


@pytest.mark.parametrize("norm", ["H1", "H2", "H3"])
def test_preconditioner_inverts_beta_A_and_fixes_kernel(norm):
    g = Grid(16, 16)
    p = Params(16, 16, 2, norm, "none", 3e-3, 0.0)
    r = spectral.nyquist_project(g, np.random.default_rng(5).standard_normal((2, 16, 16)))
    z = reduced.precond(g, p, r)
    mean_r = r.mean(axis=(1, 2))
    assert np.allclose(z.mean(axis=(1, 2)), mean_r / p.beta_v, atol=1e-12)
    back = p.beta_v * spectral.apply_A(g, p, z)
    r0 = r - mean_r[:, None, None]
    assert np.abs(back - r0).max() < 1e-9 * np.abs(r0).max()


def test_nyquist_projection_removes_only_nyquist():
    g = Grid(8, 8)
    x1, x2 = sd.grid_coords(8, 8)
    ny = np.cos(4 * x1)[:, None] + np.cos(4 * x2)[None, :]
    low = np.sin(x1)[:, None] * np.cos(3 * x2)[None, :]
    v = np.stack([ny + low, low])
    out = spectral.nyquist_project(g, v)
    assert np.abs(out - np.stack([low, low])).max() < 1e-14


@pytest.mark.parametrize("n1,n2", [(8, 8), (10, 12), (96, 150), (64, 32)])
def test_nyquist_projection_real_space_form(n1, n2):
    """The device path removes the Nyquist modes in real space: with the alternating sums
    a(i1) = mean over i2 of (-1)^i2 v, b(i2) = mean over i1 of (-1)^i1 v and the corner
    c = mean of (-1)^(i1+i2) v, the projection is v - (-1)^i2 a - (-1)^i1 b + (-1)^(i1+i2) c.
    Check that identity against the oracle's FFT form."""
    g = Grid(n1, n2)
    v = np.random.default_rng(n1 * n2).standard_normal((2, n1, n2))
    s1 = (-1.0) ** np.arange(n1)[:, None]
    s2 = (-1.0) ** np.arange(n2)[None, :]
    out = np.empty_like(v)
    for c in range(2):
        a = (v[c] * s2).mean(axis=1, keepdims=True)
        b = (v[c] * s1).mean(axis=0, keepdims=True)
        cc = (v[c] * s1 * s2).mean()
        out[c] = v[c] - s2 * a - s1 * b + s1 * s2 * cc
    assert np.abs(out - spectral.nyquist_project(g, v)).max() < 1e-13
