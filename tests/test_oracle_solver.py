"""Pins of the oracle's PCG (Alg. 2) and Newton loop (Alg. 1) (CPU only).

Q13 PCG on a dense SPD system matches a direct solve after n steps and its energy-norm error
decreases monotonically; Q14 solve invariants (Armijo keeps J non-increasing, a tight tolerance is
reachable, the spectral preconditioner of App. E.2 reduces the iteration count).
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, Params, spectral, transport, reduced, solver


def test_q13_pcg_dense_spd():
    rng = np.random.default_rng(0)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    Minv = np.diag(1.0 / np.diag(A))
    b = rng.standard_normal(n)
    x, its, _ = solver.pcg(lambda s: A @ s, lambda r: Minv @ r, lambda a, c: float(a @ c),
                        lambda a: float(np.linalg.norm(a)), b, 0.0, 100, fixed_iters=n)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)
    xs = np.linalg.solve(A, b)
    errs = []
    for k in range(1, n + 1):
        xk, _, _ = solver.pcg(lambda s: A @ s, lambda r: Minv @ r, lambda a, c: float(a @ c),
                           lambda a: float(np.linalg.norm(a)), b, 0.0, 100, fixed_iters=k)
        e = xk - xs
        errs.append(e @ A @ e)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def test_q13_pcg_relative_stop():
    rng = np.random.default_rng(1)
    n = 30
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + 0.5 * np.eye(n)
    b = rng.standard_normal(n)
    x, its, rr = solver.pcg(lambda s: A @ s, lambda r: r, lambda a, c: float(a @ c),
                        lambda a: float(np.linalg.norm(a)), b, 1e-3, 1000)
    assert np.linalg.norm(b - A @ x) <= 1e-3 * np.linalg.norm(b) * (1 + 1e-9)
    assert its < n + 5


def small_problem(constraint="divfree", norm="H1", n=16, nt=4, beta_v=1e-2):
    bw = 1e-3 if constraint == "mass_source" else 0.0
    p = Params(n, n, nt, norm, constraint, beta_v, bw)
    g = Grid(n, n)
    rng = np.random.default_rng(5)
    mT = sd.template_image(n, n, 5, 0, rng)
    vs = sd.scale_to_max(sd.random_velocity(n, n, 3, rng, True, constraint != "divfree"), 0.3)
    mR = transport.state_forward(g, p, mT, vs).m[-1]
    return g, p, mT, mR


@pytest.mark.parametrize("constraint,norm", [("divfree", "H1"), ("mass_source", "H2"), ("none", "H1")])
def test_q14_solve_invariants(constraint, norm):
    g, p, mT, mR = small_problem(constraint, norm)
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=30, gtol_rel=1e-6, max_pcg=200))
    assert st.status == solver.OK
    assert st.g_rel <= 1e-6
    Js = [h["J"] for h in st.history] + [st.J]
    assert all(Js[i + 1] <= Js[i] for i in range(len(Js) - 1))
    lin = reduced.gradient(g, p, mT, mR, v)
    assert g.norm(lin.g) / st.g0_norm <= 1e-6 * (1 + 1e-9)
    if constraint == "divfree":
        assert np.abs(spectral.div(g, v)).max() < 1e-10
    # inexact Newton: each PCG solve ends at the forcing term of Alg. 2, eta_k = min(1/2, sqrt(g_rel))
    for h in st.history:
        assert h["pcg_relres"] <= min(0.5, np.sqrt(h["g_rel"])) * (1 + 1e-12)
        assert h["pcg_relres"] > 1e-3 * min(0.5, np.sqrt(h["g_rel"]))


def test_q14_preconditioner_reduces_iterations():
    g, p, mT, mR = small_problem("none", "H1", beta_v=1e-3)
    lin = reduced.gradient(g, p, mT, mR, np.zeros((2, 16, 16)))
    mv = lambda s: reduced.hessian_matvec(g, p, lin, s)
    wi = lambda a, b: g.inner(a, b)
    _, it_p, _ = solver.pcg(mv, lambda r: reduced.precond(g, p, r), wi, g.norm, -lin.g, 1e-6, 500)
    _, it_u, _ = solver.pcg(mv, lambda r: r.copy(), wi, g.norm, -lin.g, 1e-6, 500)
    assert it_p < it_u


def test_q14_fixed_schedule_counts():
    g, p, mT, mR = small_problem()
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=2, fixed_pcg_iters=3, gtol_rel=0.0))
    assert st.newton_iters == 2 and st.pcg_iters == 6 and st.n_matvec == 6


def test_warm_start_uses_gradient_at_zero_for_relative_norm():
    g, p, mT, mR = small_problem()
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=20, gtol_rel=1e-3))
    _, st2 = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=20, gtol_rel=1e-3, v0=v))
    assert abs(st2.g0_norm - st.g0_norm) < 1e-12 * st.g0_norm
    assert st2.newton_iters == 0 and st2.g_rel <= 1e-3


def test_q14_pcg_stops_at_first_iterate_below_forcing_term():
    """Alg. 2: PCG leaves at the first l with ||r_l|| <= eta_k ||r_0||, eta_k = min(1/2, sqrt(g_rel))."""
    g, p, mT, mR = small_problem(beta_v=1e-3)
    checked = 0
    for k in range(1, 4):
        v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=k, gtol_rel=0.0))
        h = st.history[-1]
        eta = min(0.5, np.sqrt(h["g_rel"]))
        v_prev, _ = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=k - 1, gtol_rel=0.0))
        lin = reduced.gradient(g, p, mT, mR, v_prev)
        assert abs(g.norm(lin.g) / st.g0_norm - h["g_rel"]) < 1e-12
        if h["pcg"] >= 2:
            _, _, rr = solver.pcg(lambda s: reduced.hessian_matvec(g, p, lin, s),
                                  lambda r: reduced.precond(g, p, r), lambda a, b: g.inner(a, b),
                                  g.norm, -lin.g, eta, 100, fixed_iters=h["pcg"] - 1)
            assert rr > eta
            checked += 1
        assert h["pcg_relres"] <= eta
    assert checked >= 2
