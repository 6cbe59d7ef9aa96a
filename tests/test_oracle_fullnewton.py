"""Pins of the oracle's full-Newton Hessian (CPU only).

The full-Newton matvec claims to be the exact Hessian of the discrete reduced objective in the
'dto' discretisation.  It is pinned against central differences of the oracle's gradient (an
independent computation: two complete state/adjoint solves), whose error must fall as eps^2; against
symmetry in <., .>_W; against the Gauss-Newton matvec where the residual vanishes (every term that
full Newton adds carries lam, and lam = 0 there); and against quadratic convergence of the solve.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, Params, reduced, solver, spectral, transport


def problem(constraint, norm="H2", n=16, nt=4, beta_v=1e-3, adjoint="dto"):
    bw = 1e-3 if constraint == "mass_source" else 0.0
    p = Params(n, n, nt, norm, constraint, beta_v, bw, adjoint)
    g = Grid(n, n)
    rng = np.random.default_rng(5)
    mT = sd.template_image(n, n, 5, 0, rng)
    vs = sd.scale_to_max(sd.random_velocity(n, n, 3, rng, True, constraint != "divfree"), 0.3)
    mR = transport.state_forward(g, p, mT, vs).m[-1]
    return g, p, mT, mR, vs


def direction(g, p, seed):
    u = spectral.nyquist_project(g, np.random.default_rng(seed).standard_normal((2, g.n1, g.n2)))
    return spectral.apply_K(g, p, u) if p.constraint == "divfree" else u


@pytest.mark.parametrize("constraint,norm", [("mass_source", "H2"), ("divfree", "H1"), ("none", "H2"), ("none", "H1")])
def test_full_hessian_is_the_derivative_of_the_gradient(constraint, norm):
    g, p, mT, mR, vs = problem(constraint, norm)
    v = 0.6 * vs
    lin = reduced.gradient(g, p, mT, mR, v)
    vt = direction(g, p, 2)
    H = reduced.hessian_matvec_full(g, p, lin, vt)
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (reduced.gradient(g, p, mT, mR, v + eps * vt).g - reduced.gradient(g, p, mT, mR, v - eps * vt).g) / (2 * eps)
        errs.append(np.linalg.norm(fd - H) / np.linalg.norm(H))
    assert errs[1] < 1e-6
    assert 50 < errs[0] / errs[1] < 200          # second-order convergence of the central difference
    # the Gauss-Newton matvec misses the lam terms by far more than that
    Hg = reduced.hessian_matvec(g, p, lin, vt)
    assert np.linalg.norm(Hg - H) / np.linalg.norm(H) > 100 * errs[1]


@pytest.mark.parametrize("constraint", ["mass_source", "divfree", "none"])
def test_full_hessian_is_symmetric(constraint):
    g, p, mT, mR, vs = problem(constraint)
    lin = reduced.gradient(g, p, mT, mR, 0.5 * vs)
    x, y = direction(g, p, 3), direction(g, p, 4)
    Hx, Hy = reduced.hessian_matvec_full(g, p, lin, x), reduced.hessian_matvec_full(g, p, lin, y)
    a, b = reduced.w_inner(g, p, y, Hx), reduced.w_inner(g, p, Hy, x)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_full_equals_gauss_newton_where_the_residual_vanishes():
    g, p, mT, mR, vs = problem("mass_source")
    lin = reduced.gradient(g, p, mT, mR, vs)       # m_R is the transport of m_T by v*: lam = 0
    assert max(np.abs(l).max() for l in lin.lam) < 1e-14     # round-off of the input projection only
    vt = direction(g, p, 6)
    H, Hg = reduced.hessian_matvec_full(g, p, lin, vt), reduced.hessian_matvec(g, p, lin, vt)
    assert np.linalg.norm(H - Hg) <= 1e-12 * np.linalg.norm(Hg)
    # away from it the two differ
    lin2 = reduced.gradient(g, p, mT, mR, 0.5 * vs)
    H2, Hg2 = reduced.hessian_matvec_full(g, p, lin2, vt), reduced.hessian_matvec(g, p, lin2, vt)
    assert np.linalg.norm(H2 - Hg2) > 1e-4 * np.linalg.norm(Hg2)


def test_full_hessian_needs_the_exact_discrete_adjoint():
    g, p, mT, mR, vs = problem("none", adjoint="paper")
    lin = reduced.gradient(g, p, mT, mR, 0.5 * vs)
    with pytest.raises(ValueError):
        reduced.hessian_matvec_full(g, p, lin, direction(g, p, 1))


@pytest.mark.parametrize("constraint", ["mass_source", "divfree"])
def test_full_newton_converges_quadratically(constraint):
    g, p, mT, mR, vs = problem(constraint)
    opts = dict(max_newton=40, gtol_rel=1e-9, max_pcg=300)
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(**opts))
    vf, sf = solver.solve(g, p, mT, mR, solver.SolveOpts(hessian="full", **opts))
    assert st.status == sf.status == solver.OK
    assert sf.newton_iters < st.newton_iters and sf.pcg_iters < st.pcg_iters
    assert g.norm(vf - v) <= 1e-5 * g.norm(v)
    # once in the fast regime each step at least squares the relative gradient (up to a constant)
    gr = [h["g_rel"] for h in sf.history] + [sf.g_rel]
    fast = [k for k in range(len(gr) - 1) if gr[k] < 2e-3]
    assert fast and all(gr[k + 1] <= 10 * gr[k] ** 1.5 for k in fast)
    with pytest.raises(ValueError):
        solver.solve(g, p, mT, mR, solver.SolveOpts(hessian="exact", **opts))
