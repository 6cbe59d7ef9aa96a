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


# ---- CFL number (Sec. 4: n_t is chosen by monitoring the CFL condition of the explicit RK2 steps) ---
def test_cfl_number_hand_values():
    """C = h_t (max|v_1| n1/2 + max|v_2| n2/2), values worked out by hand for fields whose maxima are
    exact on the grid."""
    n1, n2 = 16, 32
    g = Grid(n1, n2)
    x1 = 2 * np.pi * np.arange(n1)[:, None] / n1
    x2 = 2 * np.pi * np.arange(n2)[None, :] / n2
    one = np.ones((n1, n2))
    # constant velocity (0.3, -0.2), n_t = 4: (0.3 * 8 + 0.2 * 16) / 4 = 1.4
    p4 = Params(n1, n2, 4, "H1", "none", 1e-2, 0.0)
    assert solver.cfl_number(g, p4, np.stack([0.3 * one, -0.2 * one])) == pytest.approx(1.4, rel=1e-13)
    # v = (0.25 sin x2, -0.1 cos 3 x1), n_t = 2: sin reaches 1 at x2 = pi/2, |cos| reaches 1 at x1 = 0:
    # (0.25 * 8 + 0.1 * 16) / 2 = 1.8
    p2 = Params(n1, n2, 2, "H1", "none", 1e-2, 0.0)
    v = np.stack([0.25 * np.sin(x2) * one, -0.1 * np.cos(3 * x1) * one])
    assert solver.cfl_number(g, p2, v) == pytest.approx(1.8, rel=1e-13)
    # a Nyquist mode is not resolved and does not count: 0.1 + 0.5 (-1)^i2 in v_1 leaves 0.1,
    # (0.1 * 8 + 0) / 2 = 0.4
    alt = np.where(np.arange(n2)[None, :] % 2 == 0, 1.0, -1.0) * one
    v = np.stack([0.1 * one + 0.5 * alt, 0 * one])
    assert solver.cfl_number(g, p2, v) == pytest.approx(0.4, rel=1e-12)


def test_cfl_number_bounds_spectral_radius_of_the_step_operator():
    """For a constant velocity, h_t L_v (L_v u = -v . grad u, built here from explicit DFT matrices)
    has eigenvalues -i h_t k~ . v; its spectral radius h_t (|v1|(n1/2 - 1) + |v2|(n2/2 - 1)) (the
    largest resolved wavenumbers) is below C and approaches it as the grid grows."""
    from dense_reference import Dense
    for (n1, n2, nt, a, b) in [(8, 8, 3, 0.7, -0.4), (8, 12, 2, -0.25, 0.9), (12, 8, 5, 1.1, 0.3)]:
        d = Dense(n1, n2, nt, "H1", "none", 1e-2, 0.0)
        L = -(a * d.D1 + b * d.D2) / nt
        rho = np.abs(np.linalg.eigvals(L)).max()
        assert rho == pytest.approx((abs(a) * (n1 / 2 - 1) + abs(b) * (n2 / 2 - 1)) / nt, rel=1e-10)
        p = Params(n1, n2, nt, "H1", "none", 1e-2, 0.0)
        C = solver.cfl_number(Grid(n1, n2), p, np.stack([a * np.ones((n1, n2)), b * np.ones((n1, n2))]))
        assert rho < C <= rho * min(n1, n2) / (min(n1, n2) - 2) * (1 + 1e-12)


# ---- Armijo backtracking (Sec. 4: Armijo condition with default parameters, N&W Alg. 3.1) --------
def translated_sinusoids(n=16, nt=64, shift=1.5, kf=2, beta_v=1e-4):
    """A pair whose reference is the template shifted by (shift, shift/2): the Gauss-Newton model of a
    shift this large overshoots, so full steps are rejected (the defaults keep the CFL number of every
    iterate below 0.9, where the RK2 transport is stable)."""
    p = Params(n, n, nt, "H1", "none", beta_v, 0.0)
    g = Grid(n, n)
    x1 = 2 * np.pi * np.arange(n)[:, None] / n
    x2 = 2 * np.pi * np.arange(n)[None, :] / n
    mT = 0.5 + 0.25 * np.sin(kf * x1) + 0.2 * np.cos(x2) + 0 * x1 * x2
    mR = 0.5 + 0.25 * np.sin(kf * (x1 - shift)) + 0.2 * np.cos(x2 - 0.5 * shift) + 0 * x1 * x2
    return g, p, mT, mR


# the schedule under which the default pair backtracks in its first two Newton steps (alpha = 1/2)
BACKTRACK_OPTS = dict(max_newton=4, fixed_pcg_iters=6, gtol_rel=0.0)


def test_armijo_backtracking_accepts_first_halving_that_decreases_enough():
    """Default line search (reading: alpha_0 = 1, rho = 1/2, c_1 = 1e-4): every accepted step is
    alpha = (1/2)^k after k rejections, satisfies J(v + alpha v~) <= J(v) + c_1 alpha dJ(v)[v~], and
    the previous trial alpha / rho = 2 alpha does not."""
    g, p, mT, mR = translated_sinusoids()
    opts = solver.SolveOpts(**BACKTRACK_OPTS)
    assert opts.armijo_c1 == 1e-4 and opts.max_backtracks == 10
    v, st = solver.solve(g, p, mT, mR, opts)
    assert st.status == solver.OK and st.backtracks >= 2
    assert max(solver.cfl_number(g, p, h["v"]) for h in st.history) < 0.9
    for h in st.history:
        a, k = h["alpha"], h["backtracks"]
        assert a == 0.5 ** k
        J = lambda t: reduced.objective(g, p, mT, mR, h["v"] + t * h["step"])[0]   # noqa: E731
        slope = g.inner(reduced.gradient(g, p, mT, mR, h["v"]).g, h["step"])
        assert slope == pytest.approx(h["slope"], rel=1e-12)
        assert slope < 0
        assert J(a) <= h["J"] + 1e-4 * a * slope
        if k > 0:
            assert J(2 * a) > h["J"] + 1e-4 * 2 * a * slope
    assert st.backtracks == sum(h["backtracks"] for h in st.history)


# ---- CFL-adapted n_t (Sec. 4 monitors the CFL condition and adapts n_t; Sec. 5 starts at 2 max(n)) --
def test_cfl_adaptation_raises_nt_to_the_smallest_admissible_value():
    from dataclasses import replace
    g, p, mT, mR = small_problem(nt=2)
    opts = solver.SolveOpts(max_newton=8, gtol_rel=1e-4, cfl_max=0.5, nt_max=64)
    v, st = solver.solve(g, p, mT, mR, opts)
    assert st.status == solver.OK and st.g_rel <= 1e-4
    assert st.nt_changes >= 1 and st.nt > 2
    assert st.cfl <= 0.5
    nts = [h["nt"] for h in st.history] + [st.nt]
    assert nts == sorted(nts)
    iterates = [h["v"] for h in st.history] + [v]
    for k in range(1, len(nts)):
        if nts[k] != nts[k - 1]:       # raised after step k-1, at iterate k
            c = lambda nt: solver.cfl_number(g, replace(p, nt=nt), iterates[k])   # noqa: E731
            assert c(nts[k - 1]) > 0.5 >= c(nts[k]) and c(nts[k] - 1) > 0.5
    # a limit never reached changes nothing
    v0, st0 = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=3, gtol_rel=1e-4))
    v1, st1 = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=3, gtol_rel=1e-4, cfl_max=1e3, nt_max=64))
    assert st1.nt_changes == 0 and st1.nt == 2 and np.array_equal(v0, v1)
    # the relative gradient's reference g(0) is the same at every n_t (the state is m_T at v = 0)
    _, st8 = solver.solve(g, replace(p, nt=8), mT, mR, solver.SolveOpts(max_newton=0))
    assert st8.g0_norm == pytest.approx(st0.g0_norm, rel=1e-13)


def test_cfl_adaptation_stops_at_nt_max():
    g, p, mT, mR = small_problem(nt=2)
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=6, gtol_rel=1e-4, cfl_max=0.05, nt_max=5))
    assert st.nt == 5 and st.cfl > 0.05
