"""GPU parity of the deformation diagnostics (reg_deformation) with the oracle.

Closed form first (the shear flow v = (a sin x2, 0): u_1 = v, F_1 = [[1, a cos x2], [0, 1]], det = 1
exactly), then element-wise parity of u_1, F_1 and det F_1 with the oracle on square and non-square
grids for divergence-free and compressible velocities (1e-10: both are FP64), and det F_1 of a
solved 256^2 registration.
"""
import numpy as np
import pytest

import synthdata as sd
from gpu_cases import Case, dev, gpu_problem, host, inputs, params, rel, close
from oracle import Grid
from oracle.deformation import deformation, det2, summary

pytestmark = pytest.mark.gpu

C1_64 = Case(64, 64, 4, "H1", "divfree", 1e-2, 0.0, "fp64", config=1)
MS_64 = Case(32, 128, 5, "H2", "mass_source", 1e-3, 1e-4, "fp32", "dto", 1)
C2 = Case(256, 256, 16, "H2", "mass_source", 1e-3, 1e-4, "fp32", config=2)
# not powers of two; v* (time-step CFL 0.8): the fixed |v| = 0.5 field runs at CFL ~9 on this grid,
# where the oracle's own det F_1 moves by 2e-10 under round-off in v
NP2 = Case(96, 150, 4, "H1", "none", 1e-2, 0.0, "fp64", seed=23)


def test_shear_flow_closed_form():
    case = C1_64
    P = gpu_problem(case)
    try:
        x2 = np.arange(64)[None, :] * 2 * np.pi / 64 + np.zeros((64, 1))
        v = np.stack([0.4 * np.sin(x2), 0 * x2])
        u1, F1, det, (mn, mx, mean) = P.deformation(dev(v))
        assert np.abs(host(u1) - v).max() < 1e-12
        F = host(F1)
        assert np.abs(F[0, 1] - 0.4 * np.cos(x2)).max() < 1e-12 and np.abs(F[1, 0]).max() < 1e-12
        assert np.abs(host(det) - 1).max() < 1e-12 and abs(mn - 1) < 1e-12 and abs(mx - 1) < 1e-12
    finally:
        P.close()


@pytest.mark.parametrize("case,which", [(C1_64, "vstar"), (MS_64, "vstar"), (MS_64, "compressible"),
                                        (NP2, "vstar")],
                         ids=["64sq_divfree", "32x128_vstar", "32x128_compressible", "96x150_vstar"])
def test_deformation_parity(case, which):
    print(f"[case] deformation {case} {which}", flush=True)
    mT, mR, vlin, vt, vtr = inputs(case)
    v = 2.0 * vlin if which == "vstar" else 0.5 * sd.random_vec(case.n1, case.n2, 3, 11) / \
        np.abs(sd.random_vec(case.n1, case.n2, 3, 11)).max()
    g = Grid(case.n1, case.n2)
    u_ref, F_ref = deformation(g, params(case), v)
    d_ref = det2(F_ref)
    P = gpu_problem(case)
    try:
        u1, F1, det, stats = P.deformation(dev(v))
        assert close(host(u1), u_ref, 1e-10)
        assert close(host(F1), F_ref, 1e-10)
        assert np.abs(host(det) - d_ref).max() < 1e-10
        assert np.allclose(stats, summary(d_ref), rtol=1e-10, atol=1e-12)
        # the linearisation point is untouched: a matvec after the diagnostics needs a gradient first
        P.gradient(dev(vlin), want_J=False)
        H1 = host(P.hessian_matvec(dev(vt)))
        P.deformation(dev(v))
        assert np.array_equal(H1, host(P.hessian_matvec(dev(vt))))
    finally:
        P.close()


def test_deformation_of_a_solved_registration():
    case = C2
    P = gpu_problem(case)
    try:
        v, s = P.solve(max_newton=50, gtol_rel=1e-2)
        u1, F1, det, (mn, mx, mean) = P.deformation(v)
        d_ref = det2(deformation(Grid(256, 256), params(case), host(v))[1])
        assert np.abs(host(det) - d_ref).max() < 1e-10
        assert 0 < mn <= mean <= mx and abs(mean - 1) < 0.05
        print({"det_min": mn, "det_max": mx, "det_mean": mean})
        from paper_1503_00757_amd import ffi
        nb = ffi.reg_deformation_workspace_bytes(P.params)
        with pytest.raises(ffi.RegError) as e:
            ffi.reg_deformation(P.h, v.data_ptr(), P._dws.data_ptr(), nb - 8, None, None, None)
        assert e.value.status == ffi.REG_ENOMEM
    finally:
        P.close()
