"""GPU parity of the H3 seminorm (REG_H3), of the CFL monitoring (reg_cfl, stats.cfl) and of the
CFL-adapted n_t of reg_solve with the oracle."""
import numpy as np
import pytest

from gpu_cases import Case, dev, gpu_problem, host, inputs, params, rel, close, oracle_results
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
        assert close(host(g), ref["g"], max(tol, ref["sens_g"] / np.linalg.norm(ref["g"]) * 10))
        assert abs(J - ref["J"]) <= 1e-8 * abs(ref["J"]) + 10 * ref["Jscale"] * case.eps
        assert close(host(P.hessian_matvec(dev(vt))), ref["H"], tol)
        gg = Grid(case.n1, case.n2)
        v_ref, st = solver.solve(gg, params(case), mT, mR, solver.SolveOpts(max_newton=3, fixed_pcg_iters=6, gtol_rel=0.0))
        v, s = P.solve(max_newton=3, fixed_pcg_iters=6, gtol_rel=0.0)
        assert s["pcg_iters"] == st.pcg_iters and s["backtracks"] == st.backtracks
        assert close(host(v), v_ref, (1e-9 if case.precision == "fp64" else 1e-4))
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


def test_cfl_adapted_nt_matches_oracle():
    """CFL-adapted n_t inside reg_solve (Sec. 4; reg_solve_opts.cfl_max, params.nt_max): starting from
    n_t = 2 the solve raises n_t whenever the iterate's CFL number exceeds 0.5, exactly as the oracle
    does (same n_t at the end, same number of raises, same Newton and PCG counts and iterate, FP64)."""
    from test_oracle_solver import small_problem
    from paper_1503_00757_amd import Problem
    g, p, mT, mR = small_problem(nt=2)
    o = dict(max_newton=8, gtol_rel=1e-4)
    v_ref, st = solver.solve(g, p, mT, mR, solver.SolveOpts(cfl_max=0.5, nt_max=64, **o))
    assert st.nt_changes >= 1
    P = Problem(dev(mT), dev(mR), p.nt, p.norm, p.constraint, p.beta_v, p.beta_w, "fp64", nt_max=64)
    try:
        v, s = P.solve(cfl_max=0.5, **o)
        print(s, {"oracle_nt": st.nt, "oracle_changes": st.nt_changes})
        assert s["status"] == 0 and s["nt"] == st.nt and s["nt_changes"] == st.nt_changes
        assert s["newton_iters"] == st.newton_iters and s["pcg_iters"] == st.pcg_iters
        assert close(host(v), v_ref, 1e-9)
        assert s["cfl"] <= 0.5 and abs(s["cfl"] - st.cfl) <= 1e-9 * st.cfl
        # the handle keeps the raised n_t: a gradient now matches the oracle's at that n_t
        from dataclasses import replace
        gk, Jk = P.gradient(v)
        lin = reduced.gradient(g, replace(p, nt=st.nt), mT, mR, v_ref)
        assert close(host(gk), lin.g, 1e-8)
    finally:
        P.close()


def test_cfl_adapted_nt_fp32_from_the_paper_start():
    """FP32 transport on the 64^2 workload: from n_t = 4 the adaptation reaches a CFL-admissible n_t
    and converges; from the paper's start n_t = 2 max(n) = 128 nothing needs to change."""
    from paper_1503_00757_amd import Problem, paper_nt
    case = C1_64
    mT, mR, *_ = inputs(case)
    for nt0 in (4, paper_nt(case.n1, case.n2)):
        P = Problem(dev(mT), dev(mR), nt0, case.norm, case.constraint, case.beta_v, case.beta_w, "fp32", nt_max=256)
        try:
            v, s = P.solve(max_newton=20, gtol_rel=1e-3, cfl_max=0.5)
            print(nt0, s)
            assert s["status"] == 0 and s["g_rel"] <= 1e-3 and s["cfl"] <= 0.5
            assert (s["nt"] > nt0 and s["nt_changes"] >= 1) if nt0 == 4 else (s["nt"] == nt0 and s["nt_changes"] == 0)
            assert abs(P.cfl(v) - s["cfl"]) <= 1e-12 * s["cfl"]
        finally:
            P.close()
