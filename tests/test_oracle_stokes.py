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


# ---- shear-control model with a mass source (relaxed incompressibility; App. A, eq. for K[b, v]) ----
def ms_problem(nu=1.7, n=16, nt=4, beta_v=1e-2, beta_w=1e-2, seed=5):
    from oracle import Params, transport
    p = Params(n, n, nt, "stokes", "mass_source", beta_v, beta_w, nu=nu, eps=1e-4)
    g = Grid(n, n)
    rng = np.random.default_rng(seed)
    mT = sd.template_image(n, n, 5, 0, rng)
    vs = sd.scale_to_max(sd.random_velocity(n, n, 3, rng, True, True), 0.3)
    mR = transport.state_forward(g, p, mT, vs).m[-1]
    return g, p, mT, mR, vs


@pytest.mark.parametrize("nu", [0.5, 1.0, 3.0])
def test_mass_source_gradient_is_the_printed_elimination(nu):
    """The gradient equals the printed form -div(2 beta_v eta E[v]) + K[b, v] with
    K[b, v] = grad M^{-1} Lap^{-1} div(div(2 beta_v eta_hat E[v]) - b) + b, M = 2 beta_v eta_bar
    (beta_w(-Lap + I))^{-1} + I, eta = eta_hat + eta_bar (eta_bar its mean), written out here with
    Fourier symbols (grad Lap^{-1} div = k k^T / |k|^2)."""
    from oracle import reduced
    g, p, mT, mR, vs = ms_problem(nu)
    v = 0.6 * vs
    lin = reduced.gradient(g, p, mT, mR, v)
    v = spectral.nyquist_project(g, v)
    E = stokes.strain(g, v)
    eta = stokes.viscosity(nu, p.eps, E)
    eta_bar = eta.mean()
    eta_hat = eta - eta_bar
    d = spectral.d

    def div_stress(w):   # div(2 beta_v w E), w a scalar field
        s11, s12, s22 = (2 * p.beta_v * w * E[k] for k in range(3))
        return np.stack([d(g, s11, 0) + d(g, s12, 1), d(g, s12, 0) + d(g, s22, 1)])

    f = div_stress(eta_hat) - lin.b
    fh = [g.fft(f[0]), g.fft(f[1])]
    kf = g.k1 * fh[0] + g.k2 * fh[1]
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(g.ksq > 0, 1.0 / (g.ksq * (1.0 + 2 * p.beta_v * eta_bar / (p.beta_w * (g.ksq + 1.0)))), 0.0)
    proj = np.stack([g.ifft(w * g.k1 * kf), g.ifft(w * g.k2 * kf)])
    g_printed = spectral.nyquist_project(g, -div_stress(eta) + proj + lin.b)
    assert np.abs(lin.g - g_printed).max() < 1e-12 * np.abs(g_printed).max()
    assert lin.p.eta_bar == pytest.approx(eta_bar, rel=1e-14)


def test_mass_source_gradient_and_hessian_are_derivatives_of_the_objective():
    """K_v^{-1} g is the gradient of the discrete objective (central differences of J), and K_v^{-1}
    times the full-Newton matvec is the derivative of that gradient (second-order error decay); the
    Gauss-Newton matvec is W-symmetric and positive."""
    from oracle import reduced
    g, p, mT, mR, vs = ms_problem(1.7)
    v = 0.6 * vs
    dvec = sd.random_vec(16, 16, 4, 11)
    lin = reduced.gradient(g, p, mT, mR, v)
    gJ = lambda x: spectral.apply_Kinv(g, reduced.gradient(g, p, mT, mR, x).p, reduced.gradient(g, p, mT, mR, x).g)  # noqa: E731
    slope = g.inner(gJ(v), dvec)
    e1, e2 = [], []
    Hf = spectral.apply_Kinv(g, lin.p, reduced.hessian_matvec_full(g, p, lin, dvec))
    for h in (1e-3, 1e-4):
        fd = (reduced.objective(g, p, mT, mR, v + h * dvec)[0] - reduced.objective(g, p, mT, mR, v - h * dvec)[0]) / (2 * h)
        e1.append(abs(fd - slope) / abs(slope))
        fdg = (gJ(v + h * dvec) - gJ(v - h * dvec)) / (2 * h)
        e2.append(np.linalg.norm(fdg - Hf) / np.linalg.norm(Hf))
    assert e1[1] < 1e-7 and e1[0] / e1[1] > 50
    assert e2[1] < 1e-6 and e2[0] / e2[1] > 50
    x, y = sd.random_vec(16, 16, 4, 12), sd.random_vec(16, 16, 4, 13)
    Hx, Hy = reduced.hessian_matvec(g, p, lin, x), reduced.hessian_matvec(g, p, lin, y)
    a, b = reduced.w_inner(g, lin.p, Hx, y), reduced.w_inner(g, lin.p, x, Hy)
    assert abs(a - b) < 1e-11 * abs(a) and reduced.w_inner(g, lin.p, x, Hx) > 0


def test_mass_source_limits():
    """beta_w -> infinity: on a divergence-free v the gradient tends to the incompressible model's;
    beta_w -> 0: it tends to the unconstrained model's (K -> I, the penalty vanishes)."""
    from dataclasses import replace
    from oracle import reduced
    g, p, mT, mR, vs = ms_problem(3.0)
    vd = 0.3 * sd.random_vec(16, 16, 3, 14, divfree=True)
    g_inc = reduced.gradient(g, replace(p, constraint="divfree", beta_w=0.0), mT, mR, vd).g
    g_big = reduced.gradient(g, replace(p, beta_w=1e10), mT, mR, vd).g
    assert np.linalg.norm(g_big - g_inc) < 1e-7 * np.linalg.norm(g_inc)
    v = 0.6 * vs
    g_none = reduced.gradient(g, replace(p, constraint="none", beta_w=0.0), mT, mR, v).g
    g_small = reduced.gradient(g, replace(p, beta_w=1e-12), mT, mR, v).g
    assert np.linalg.norm(g_small - g_none) < 1e-8 * np.linalg.norm(g_none)


def test_mass_source_solve_converges():
    from oracle import solver
    g, p, mT, mR, vs = ms_problem(1.7)
    _, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=30, gtol_rel=1e-6, max_pcg=300))
    assert st.status == solver.OK and st.g_rel <= 1e-6
    Js = [h["J"] for h in st.history] + [st.J]
    assert all(Js[i + 1] <= Js[i] for i in range(len(Js) - 1))
    with pytest.raises(ValueError):
        solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=1, recycle=2))
