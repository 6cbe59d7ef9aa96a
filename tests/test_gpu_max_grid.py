"""The largest supported grid, 2048 x 2048 (FP32 transport, n_t = 2 so that the oracle stays cheap):
gradient and Gauss-Newton matvec against the oracle (1e-5, the per-matvec bound of the precision
plan), <Hx, y> = <x, Hy> and <x, Hx> >= beta_v <x, A x>, before and after autotuning (whose candidate
shapes must fit the 2048-point lines).  Every kernel runs at its largest shape:
the 2048-point fused stages, the two-column FP64 spectral pass and the real-space projection."""
import numpy as np
import pytest

import synthdata as sd
from gpu_cases import Case, dev, gpu_problem, host, inputs, params, rel, close
from oracle import Grid, reduced, spectral

pytestmark = pytest.mark.gpu

MAX = Case(2048, 2048, 2, "H1", "divfree", 1e-2, 0.0, "fp32", seed=31)


def test_2048sq_gradient_matvec_parity_symmetry_positivity():
    case = MAX
    print(f"[case] {case}", flush=True)
    mT, mR, vlin, vt, vtr = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    lin = reduced.gradient(g, p, mT, mR, vlin)
    H_ref = reduced.hessian_matvec(g, p, lin, vt)
    P = gpu_problem(case)
    try:
        gg, J = P.gradient(dev(vlin))
        assert close(host(gg), lin.g, 1e-5)
        assert abs(J - lin.J) <= 1e-5 * abs(lin.J)
        Hx = host(P.hessian_matvec(dev(vt)))
        assert close(Hx, H_ref, 1e-5)
        y = sd.random_vec(case.n1, case.n2, 12, 98, divfree=True)
        Hy = host(P.hessian_matvec(dev(y)))
        a, b = float((Hx * y).sum()), float((vt * Hy).sum())
        assert abs(a - b) <= 1e-5 * abs(a)
        xAx = float((vt * spectral.apply_A(g, p, vt)).sum())
        assert float((vt * Hx).sum()) >= p.beta_v * xAx * (1 - 1e-6)
        # the autotuner only times shapes that fit 2048-point lines (256+ threads per transform), and
        # the tuned matvec is the same operator
        from test_gpu_parity import expected_shapes
        rep = P.autotune(reps=3)
        fits = expected_shapes(2048, 2048)
        assert fits == {4, 6, 7, 8, 18}
        for op in ("A1", "A2", "I1", "I2"):
            assert {v for v, _ in rep[op]} <= fits, rep[op]
        assert set(rep["chosen"][2:6]) <= fits
        assert close(host(P.hessian_matvec(dev(vt))), H_ref, 1e-5)
    finally:
        P.close()


def test_2048sq_fp64_gradient_matvec_parity():
    """FP64 transport at the largest grid.  Floor: 10x the oracle's own response to FP64 round-off in
    its input (beta_v A with |k| up to 1024 amplifies it), measured from the oracle."""
    case = Case(2048, 2048, 2, "H2", "none", 1e-3, 0.0, "fp64", seed=32)
    print(f"[case] {case}", flush=True)
    mT, mR, vlin, vt, vtr = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    lin = reduced.gradient(g, p, mT, mR, vlin)
    H_ref = reduced.hessian_matvec(g, p, lin, vt)
    rng = np.random.default_rng(1234)
    H_n = reduced.hessian_matvec(g, p, lin, vt + 2.2e-16 * np.abs(vt).max() * rng.standard_normal(vt.shape))
    g_n = reduced.gradient(g, p, mT, mR, vlin + 2.2e-16 * np.abs(vlin).max() * rng.standard_normal(vlin.shape)).g
    P = gpu_problem(case)
    try:
        gg, J = P.gradient(dev(vlin))
        assert close(host(gg), lin.g, max(1e-10, 10 * rel(g_n, lin.g)))
        Hx = host(P.hessian_matvec(dev(vt)))
        assert close(Hx, H_ref, max(1e-10, 10 * rel(H_n, H_ref)))
    finally:
        P.close()


def test_2048sq_deformation_shear_flow_closed_form():
    """Deformation diagnostics at the largest grid: the shear flow v = (a sin x2, 0) has u_1 = v,
    F_1 = [[1, a cos x2], [0, 1]] and det F_1 = 1 exactly (n_t = 512 keeps the time-step CFL at 0.8)."""
    import torch
    from paper_1503_00757_amd import Problem
    n, nt, amp = 2048, 512, 0.4
    img = torch.full((n, n), 0.5, dtype=torch.float64, device="cuda:0")
    P = Problem(img, img.clone(), nt, "H1", "divfree", 1e-2, 0.0, "fp32")
    try:
        x2 = np.arange(n)[None, :] * 2 * np.pi / n + np.zeros((n, 1))
        v = np.stack([amp * np.sin(x2), 0 * x2])
        u1, F1, det, (mn, mx, mean) = P.deformation(dev(v))
        assert np.abs(host(u1) - v).max() < 1e-11
        F = host(F1)
        assert np.abs(F[0, 0] - 1).max() < 1e-11 and np.abs(F[1, 1] - 1).max() < 1e-11
        assert np.abs(F[0, 1] - amp * np.cos(x2)).max() < 1e-11 and np.abs(F[1, 0]).max() < 1e-11
        assert np.abs(host(det) - 1).max() < 1e-11 and abs(mn - 1) < 1e-11 and abs(mx - 1) < 1e-11
    finally:
        P.close()


def test_2048sq_full_newton_matvec_parity():
    """Full-Newton stages (the lam v~ flux terms) at the largest grid, FP32 transport."""
    case = MAX
    mT, mR, vlin, vt, vtr = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    lin = reduced.gradient(g, p, mT, mR, vlin)
    H_ref = reduced.hessian_matvec_full(g, p, lin, vt)
    P = gpu_problem(case, hessian="full")
    try:
        P.gradient(dev(vlin), want_J=False)
        assert close(host(P.hessian_matvec(dev(vt))), H_ref, 1e-5)
    finally:
        P.close()
