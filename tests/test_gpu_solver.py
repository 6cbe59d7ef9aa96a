"""GPU parity of PCG (Alg. 2) and of the Gauss-Newton-Krylov solve (Alg. 1) with the oracle, plus
properties that hold at any size (adjoint symmetry, positivity) checked at the full 1024^2 workload
in the launch configuration the benchmark times.

Solve parity follows the fixed-schedule reading: same Newton count, exactly ``fixed_pcg_iters`` PCG
steps per Newton step, and the line search must accept the same step lengths; the final velocities
are then compared (1e-10 FP64, 1e-4 FP32 -- the final-velocity bound of the precision plan)."""
import numpy as np
import pytest

from gpu_cases import Case, dev, gpu_problem, host, inputs, params, rel
from oracle import Grid, reduced, solver

pytestmark = pytest.mark.gpu

C1_64 = Case(64, 64, 4, "H1", "divfree", 1e-2, 0.0, "fp64", config=1)
C1_32 = Case(64, 64, 4, "H1", "divfree", 1e-2, 0.0, "fp32", config=1)
MS_64 = Case(32, 128, 5, "H2", "mass_source", 1e-3, 1e-4, "fp64", "dto", 1)
C2 = Case(256, 256, 16, "H2", "mass_source", 1e-3, 1e-4, "fp32", config=2)
C3 = Case(1024, 1024, 32, "H1", "divfree", 1e-4, 0.0, "fp32", config=3)
NP2_64 = Case(150, 96, 4, "H2", "mass_source", 1e-3, 1e-4, "fp64", seed=21)     # not powers of two
NP2_32 = Case(96, 150, 4, "H1", "divfree", 1e-2, 0.0, "fp32", seed=22)


@pytest.mark.parametrize("case,tol", [(C1_64, 1e-10), (MS_64, 1e-9), (C1_32, 1e-5)])
def test_pcg_fixed_iterations_parity(case, tol):
    print(f"[case] pcg {case}", flush=True)
    mT, mR, vlin, vt, vtr = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    lin = reduced.gradient(g, p, mT, mR, vlin)
    x_ref, it_ref, rr_ref = solver.pcg(lambda s: reduced.hessian_matvec(g, p, lin, s),
                                       lambda r: reduced.precond(g, p, r),
                                       lambda a, b: reduced.w_inner(g, p, a, b), g.norm, -lin.g, 0.0, 100,
                                       fixed_iters=6)
    P = gpu_problem(case)
    try:
        gg, _ = P.gradient(dev(vlin), want_J=False)
        x, it, rr = P.pcg(dev(-lin.g), eta=0.0, max_iters=100, fixed_iters=6)
        assert it == 6
        assert rel(host(x), x_ref) < tol
        assert abs(rr - rr_ref) <= 10 * tol * max(rr_ref, 1e-3)
        # adaptive stop: ||r|| <= eta ||r_0|| at the first iterate below eta (same count as the oracle)
        x2, it2, rr2 = P.pcg(dev(-lin.g), eta=0.05, max_iters=100)
        _, it_o, rr_o = solver.pcg(lambda s: reduced.hessian_matvec(g, p, lin, s),
                                   lambda r: reduced.precond(g, p, r),
                                   lambda a, b: reduced.w_inner(g, p, a, b), g.norm, -lin.g, 0.05, 100)
        assert rr2 <= 0.05 and it2 == it_o
    finally:
        P.close()


@pytest.mark.parametrize("case,newton,pcg,tol", [(C1_64, 5, 10, 1e-10), (MS_64, 3, 6, 1e-9), (C2, 3, 8, 1e-4),
                                                  (NP2_64, 3, 6, 1e-9), (NP2_32, 3, 6, 1e-4)])
def test_solve_fixed_schedule_parity(case, newton, pcg, tol):
    print(f"[case] solve {case}", flush=True)
    mT, mR, *_ = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    v_ref, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=newton, fixed_pcg_iters=pcg, gtol_rel=0.0))
    assert st.status == solver.OK and st.newton_iters == newton
    P = gpu_problem(case)
    try:
        v, s = P.solve(max_newton=newton, fixed_pcg_iters=pcg, gtol_rel=0.0)
        assert s["status"] == 0 and s["newton_iters"] == newton
        assert s["pcg_iters"] == st.pcg_iters and s["n_matvec"] == st.n_matvec
        assert s["backtracks"] == st.backtracks       # same accepted step lengths
        assert rel(host(v), v_ref) < tol
        assert abs(s["g_rel"] - st.g_rel) <= 100 * tol * st.g_rel + 1e-12
        assert abs(s["J"] - st.J) <= 100 * tol * abs(st.J)
    finally:
        P.close()


def test_solve_adaptive_c2_reaches_tolerance_like_oracle():
    """Both paths run Alg. 1 with the forcing term to ||g||/||g(0)|| <= 1e-2 on the 256^2 workload."""
    case = C2
    mT, mR, *_ = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    v_ref, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=50, gtol_rel=1e-2))
    P = gpu_problem(case)
    try:
        v, s = P.solve(max_newton=50, gtol_rel=1e-2)
        assert s["status"] == 0 and s["g_rel"] <= 1e-2
        assert s["newton_iters"] == st.newton_iters
        assert abs(s["pcg_iters"] - st.pcg_iters) <= 2
        assert rel(host(v), v_ref) < 1e-3
    finally:
        P.close()


def test_warm_start_keeps_gradient_at_zero_as_reference():
    case = C1_64
    P = gpu_problem(case)
    try:
        v, s = P.solve(max_newton=20, gtol_rel=1e-3)
        v2, s2 = P.solve(max_newton=20, gtol_rel=1e-3, v0=v)
        assert abs(s2["g0_norm"] - s["g0_norm"]) <= 1e-12 * s["g0_norm"]
        assert s2["newton_iters"] == 0 and s2["g_rel"] <= 1e-3
    finally:
        P.close()


def test_line_search_failure_reports_enotconv():
    """Forced from the host: an Armijo constant c1 close to 1 rejects every step (max_backtracks = 0)."""
    case = C1_64
    P = gpu_problem(case)
    try:
        v, s = P.solve(max_newton=3, gtol_rel=1e-6, max_backtracks=0, armijo_c1=0.999999, raise_on_error=False)
        assert s["return_status"] == -4 and s["status"] == -4
    finally:
        P.close()


def test_c3_full_size_matvec_parity_symmetry_positivity():
    """1024^2, n_t = 32, FP32 transport: matvec parity (1e-5), <Hx,y> = <x,Hy>, <x,Hx> >= beta_v <x,Ax>."""
    case = C3
    print(f"[case] {case}", flush=True)
    mT, mR, vlin, vt, vtr = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    lin = reduced.gradient(g, p, mT, mR, vlin)
    H_ref = reduced.hessian_matvec(g, p, lin, vt)
    P = gpu_problem(case)
    try:
        gg, J = P.gradient(dev(vlin))
        assert rel(host(gg), lin.g) < 1e-5
        Hx = P.hessian_matvec(dev(vt))
        assert rel(host(Hx), H_ref) < 1e-5
        import synthdata as sd
        y = sd.random_vec(case.n1, case.n2, 12, 99, divfree=True)
        Hy = P.hessian_matvec(dev(y))
        a = float((host(Hx) * y).sum())
        b = float((vt * host(Hy)).sum())
        assert abs(a - b) <= 1e-5 * abs(a)
        from oracle import spectral
        xAx = float((vt * spectral.apply_A(g, p, vt)).sum())
        assert float((vt * host(Hx)).sum()) >= p.beta_v * xAx * (1 - 1e-6)
    finally:
        P.close()


def test_c1_fixed_schedule_every_newton_step():
    """Config 1 as specified: 5 GN steps of exactly 10 PCG iterations in FP64; after every step the
    objective, the relative gradient and the iterate match the oracle's to 1e-10."""
    case = C1_64
    mT, mR, *_ = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    P = gpu_problem(case)
    try:
        for k in range(1, 6):
            v_ref, st = solver.solve(g, p, mT, mR, solver.SolveOpts(max_newton=k, fixed_pcg_iters=10, gtol_rel=0.0))
            v, s = P.solve(max_newton=k, fixed_pcg_iters=10, gtol_rel=0.0)
            assert s["newton_iters"] == k and s["pcg_iters"] == 10 * k
            assert rel(host(v), v_ref) < 1e-10, k
            assert abs(s["J"] - st.J) <= 1e-10 * abs(st.J), k
            # g shrinks while its rounding stays at the scale of g(0): compare relative to ||g(0)||
            assert abs(s["g_rel"] - st.g_rel) <= 1e-10, k
            gk, _ = P.gradient(v, want_J=False)
            g_ref = reduced.gradient(g, p, mT, mR, v_ref).g
            assert np.linalg.norm(host(gk) - g_ref) <= 1e-10 * st.g0_norm / np.sqrt(g.h1 * g.h2), k
    finally:
        P.close()
