"""GPU parity of the H3 seminorm (REG_H3) and of the CFL monitoring (reg_cfl, stats.cfl) with the
oracle, and the adaptive-n_t driver built on it."""
import numpy as np
import pytest

from gpu_cases import Case, dev, gpu_problem, host, inputs, params, rel, oracle_results
from oracle import Grid, reduced, solver

pytestmark = pytest.mark.gpu

H3_64 = Case(64, 64, 4, "H3", "mass_source", 1e-4, 1e-4, "fp64", seed=5)
H3_64F = Case(64, 64, 4, "H3", "none", 1e-4, 0.0, "fp32", seed=5)
C1_64 = Case(64, 64, 4, "H1", "divfree", 1e-2, 0.0, "fp64", config=1)


@pytest.mark.parametrize("case", [H3_64, H3_64F], ids=["H3_mass_fp64", "H3_none_fp32"])
def test_h3_gradient_matvec_and_solve_parity(case):
    print(f"[case] H3 {case}", flush=True)
    mT, mR, vlin, vt, _ = inputs(case)
    ref = oracle_results(case)
    tol = max(case.tol, 10 * ref["sens_H"])
    P = gpu_problem(case)
    try:
        g, J = P.gradient(dev(vlin))
        assert rel(host(g), ref["g"]) < max(tol, ref["sens_g"] / np.linalg.norm(ref["g"]) * 10)
        assert abs(J - ref["J"]) <= 1e-8 * abs(ref["J"]) + 10 * ref["Jscale"] * case.eps
        assert rel(host(P.hessian_matvec(dev(vt))), ref["H"]) < tol
        gg = Grid(case.n1, case.n2)
        v_ref, st = solver.solve(gg, params(case), mT, mR, solver.SolveOpts(max_newton=3, fixed_pcg_iters=6, gtol_rel=0.0))
        v, s = P.solve(max_newton=3, fixed_pcg_iters=6, gtol_rel=0.0)
        assert s["pcg_iters"] == st.pcg_iters and s["backtracks"] == st.backtracks
        assert rel(host(v), v_ref) < (1e-9 if case.precision == "fp64" else 1e-4)
        assert abs(s["cfl"] - st.cfl) <= (1e-9 if case.precision == "fp64" else 1e-4) * st.cfl
    finally:
        P.close()


def test_cfl_number_matches_oracle():
    case = C1_64
    mT, mR, vlin, vt, _ = inputs(case)
    P = gpu_problem(case)
    try:
        gg = Grid(case.n1, case.n2)
        for v in (vlin, 3.0 * vt):
            assert abs(P.cfl(dev(v)) - solver.cfl_number(gg, params(case), v)) <= 1e-12 * solver.cfl_number(gg, params(case), v)
        v_ref, st = solver.solve(gg, params(case), mT, mR, solver.SolveOpts(max_newton=20, gtol_rel=1e-3))
        v, s = P.solve(max_newton=20, gtol_rel=1e-3)
        assert abs(s["cfl"] - st.cfl) <= 1e-8 * st.cfl and s["newton_iters"] == st.newton_iters
    finally:
        P.close()


def test_adaptive_nt_raises_nt_until_the_cfl_limit_holds():
    import torch
    from paper_1503_00757_amd import solve_adaptive_nt
    case = C1_64
    mT, mR, *_ = inputs(case)
    kw = dict(norm=case.norm, constraint=case.constraint, beta_v=case.beta_v, beta_w=case.beta_w,
              precision=case.precision)
    v, st, tried = solve_adaptive_nt(dev(mT), dev(mR), 4, cfl_max=0.5, problem_kw=kw, max_newton=20, gtol_rel=1e-3)
    print(tried, st)
    assert tried[0] == 4 and len(tried) >= 2 and tried[-1] > 4
    assert st["status"] == 0 and st["cfl"] <= 0.5 and st["g_rel"] <= 1e-3
