"""Pins of the oracle's nonlinear Stokes (shear-control) regulariser (CPU only).

nu = 1 reduces to the linear model, whose first variation is the closed-form operator
-Lap v - grad div v (Fourier symbol |k|^2 I + k k^T) and whose value on divergence-free fields is
1/2 |v|^2_{H1}; for nu != 1 the first variation is the derivative of the value and the second
variation the derivative of the first (central differences, second-order error decay); the second
variation is symmetric and positive semidefinite (convex model); the viscosity falls with strain for
nu > 1 (shear thinning) and rises for nu < 1 (thickening).
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, spectral
from oracle import stokes


def field(n, seed, divfree=False, amp=0.3):
    return amp * sd.random_vec(n, n, 4, seed, divfree=divfree) / np.abs(sd.random_vec(n, n, 4, seed, divfree=divfree)).max()


def test_linear_model_closed_form():
    n = 16
    g = Grid(n, n)
    v = field(n, 1)
    A = stokes.first_variation(g, 1.0, 1e-6, v)
    v1h, v2h = g.fft(v[0]), g.fft(v[1])
    kv = g.k1 * v1h + g.k2 * v2h
    ref = np.stack([g.ifft(g.ksq * v1h + g.k1 * kv), g.ifft(g.ksq * v2h + g.k2 * kv)])
    assert np.abs(A - ref).max() < 1e-11 * np.abs(ref).max()
    w = field(n, 2)
    assert np.allclose(stokes.second_variation(g, 1.0, 1e-6, v, w), stokes.first_variation(g, 1.0, 1e-6, w),
                       atol=1e-12)
    vd = field(n, 3, divfree=True)
    h1 = sum(g.inner(spectral.d(g, vd[c], a), spectral.d(g, vd[c], a)) for c in (0, 1) for a in (0, 1))
    assert abs(stokes.value(g, 1.0, 1e-6, vd) - (0.5 * h1 + 1e-6 * g.n1 * g.n2 * g.h1 * g.h2)) < 1e-12 * h1


@pytest.mark.parametrize("nu", [0.5, 1.7, 3.0])
def test_variations_are_derivatives(nu):
    n, eps = 16, 1e-4
    g = Grid(n, n)
    v, w = field(n, 4), field(n, 5)
    A = stokes.first_variation(g, nu, eps, v)
    B = stokes.second_variation(g, nu, eps, v, w)
    errs_a, errs_b = [], []
    for h in (1e-3, 1e-4):
        fd = (stokes.value(g, nu, eps, v + h * w) - stokes.value(g, nu, eps, v - h * w)) / (2 * h)
        errs_a.append(abs(fd - g.inner(A, w)) / abs(g.inner(A, w)))
        fdb = (stokes.first_variation(g, nu, eps, v + h * w) - stokes.first_variation(g, nu, eps, v - h * w)) / (2 * h)
        errs_b.append(np.abs(fdb - B).max() / np.abs(B).max())
    assert errs_a[1] < 1e-7 and errs_a[0] / errs_a[1] > 50
    assert errs_b[1] < 1e-6 and errs_b[0] / errs_b[1] > 50


@pytest.mark.parametrize("nu", [0.5, 1.7])
def test_second_variation_symmetric_positive(nu):
    n = 16
    g = Grid(n, n)
    v, x, y = field(n, 6), field(n, 7), field(n, 8)
    Bx, By = stokes.second_variation(g, nu, 1e-4, v, x), stokes.second_variation(g, nu, 1e-4, v, y)
    assert abs(g.inner(Bx, y) - g.inner(x, By)) < 1e-12 * abs(g.inner(Bx, y))
    assert g.inner(Bx, x) > 0 and g.inner(By, y) > 0


def test_viscosity_thins_and_thickens():
    small = (np.full(4, 0.01), np.zeros(4), np.zeros(4))
    big = (np.full(4, 1.0), np.zeros(4), np.zeros(4))
    assert np.all(stokes.viscosity(2.0, 1e-8, big) < stokes.viscosity(2.0, 1e-8, small))   # nu > 1 thins
    assert np.all(stokes.viscosity(0.5, 1e-8, big) > stokes.viscosity(0.5, 1e-8, small))   # nu < 1 thickens
    assert np.allclose(stokes.viscosity(1.0, 1e-8, big), 1.0)


@pytest.mark.parametrize("constraint", ["divfree", "none"])
def test_reduced_problem_with_shear_control(constraint):
    """The full-Newton matvec with the shear-control model is the derivative of the reduced gradient,
    and Alg. 1 converges with the vector-Laplacian preconditioner."""
    from oracle import Params, reduced, solver, transport
    n = 16
    p = Params(n, n, 4, "stokes", constraint, 1e-2, 0.0, nu=1.7, eps=1e-4)
    g = Grid(n, n)
    rng = np.random.default_rng(5)
    mT = sd.template_image(n, n, 5, 0, rng)
    vs = sd.scale_to_max(sd.random_velocity(n, n, 3, rng, True, constraint != "divfree"), 0.3)
    mR = transport.state_forward(g, p, mT, vs).m[-1]
    v = 0.6 * vs
    lin = reduced.gradient(g, p, mT, mR, v)
    vt = sd.random_vec(n, n, 5, 9, divfree=(constraint == "divfree"))
    H = reduced.hessian_matvec_full(g, p, lin, vt)
    errs = []
    for e in (1e-3, 1e-4):
        fd = (reduced.gradient(g, p, mT, mR, v + e * vt).g - reduced.gradient(g, p, mT, mR, v - e * vt).g) / (2 * e)
        errs.append(np.linalg.norm(fd - H) / np.linalg.norm(H))
    assert errs[1] < 1e-6 and errs[0] / errs[1] > 50
    _, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=30, gtol_rel=1e-6, max_pcg=300))
    assert st.status == solver.OK and st.g_rel <= 1e-6
