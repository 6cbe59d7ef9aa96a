"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element by element (rel-L2 over
whole vectors) on seeded inputs.  Tolerances: 1e-10 with FP64 transport; with FP32 transport 1e-5 per
Hessian matvec (the per-matvec bound of the precision plan) and the same for gradient, objective,
deformed template and preconditioner.  Two floors, both measured from the oracle, never from the GPU:
the gradient and data term carry an absolute floor of 32 eps times the body force of an O(1) misfit
(they are formed from m_R - m_1), and every bound is at least 10x the oracle's own response to FP64
round-off in its input (beta_v A amplifies that by up to beta_v (n/2)^4 on a 2048-point H2 axis).  Sizes span several workgroup tiles, non-square grids, the
smallest (8) and largest (2048) supported axis lengths, 512-point lines, the full 64^2 / 256^2 / 1024^2
workloads, and even axis lengths that are not powers of two: 2^a 3^b 5^c lengths (10, 90, 96, 150, 250,
600, 1200: mixed-radix transforms) and 2046 = 2 * 3 * 11 * 31 (direct sums) on one or both axes."""
import numpy as np
import pytest

from gpu_cases import Case, dev, gpu_problem, host, inputs, oracle_results, rel, close

pytestmark = pytest.mark.gpu

CASES = {
    "c1_64sq_nt4_H1_divfree_fp64": Case(64, 64, 4, "H1", "divfree", 1e-2, 0.0, "fp64", config=1),
    "c1_64sq_nt4_H1_divfree_fp32": Case(64, 64, 4, "H1", "divfree", 1e-2, 0.0, "fp32", config=1),
    "32x128_nt5_H2_mass_fp64_paper": Case(32, 128, 5, "H2", "mass_source", 1e-3, 1e-4, "fp64", "paper", 1),
    "128x32_nt3_H1_none_fp32": Case(128, 32, 3, "H1", "none", 1e-2, 0.0, "fp32", "dto", 2),
    "8x8_nt2_H1_divfree_fp64": Case(8, 8, 2, "H1", "divfree", 1e-2, 0.0, "fp64", "dto", 3),
    "16x8_nt1_H2_none_fp64_paper": Case(16, 8, 1, "H2", "none", 1e-2, 0.0, "fp64", "paper", 4),
    "8x64_nt3_H1_mass_fp32": Case(8, 64, 3, "H1", "mass_source", 1e-2, 1e-3, "fp32", "dto", 5),
    "2048x16_nt128_H1_none_fp32": Case(2048, 16, 128, "H1", "none", 1e-2, 0.0, "fp32", "dto", 6, vmax=0.1),
    "16x2048_nt128_H2_divfree_fp64": Case(16, 2048, 128, "H2", "divfree", 1e-2, 0.0, "fp64", "dto", 7, vmax=0.1),
    "c2_256sq_nt16_H2_mass_fp32": Case(256, 256, 16, "H2", "mass_source", 1e-3, 1e-4, "fp32", config=2),
    "8sq_nt2_H1_divfree_fp32": Case(8, 8, 2, "H1", "divfree", 1e-2, 0.0, "fp32", seed=22),
    "16sq_nt2_H2_mass_fp32": Case(16, 16, 2, "H2", "mass_source", 1e-2, 1e-3, "fp32", seed=23),
    "32sq_nt2_H1_none_fp32": Case(32, 32, 2, "H1", "none", 1e-2, 0.0, "fp32", seed=20),
    "128sq_nt3_H2_divfree_fp32": Case(128, 128, 3, "H2", "divfree", 1e-3, 0.0, "fp32", seed=21),
    "512sq_nt4_H1_none_fp32": Case(512, 512, 4, "H1", "none", 1e-2, 0.0, "fp32", seed=17),
    "512x32_nt4_H2_mass_fp32": Case(512, 32, 4, "H2", "mass_source", 1e-3, 1e-4, "fp32", seed=18),
    "64x512_nt4_H1_divfree_fp64": Case(64, 512, 4, "H1", "divfree", 1e-2, 0.0, "fp64", seed=19),
    # axis lengths that are not powers of two (direct-sum spectral passes, circulant stage derivatives)
    "96x96_nt4_H1_divfree_fp64": Case(96, 96, 4, "H1", "divfree", 1e-2, 0.0, "fp64", seed=11),
    "150x128_nt6_H2_mass_fp32": Case(150, 128, 6, "H2", "mass_source", 1e-3, 1e-4, "fp32", seed=12),
    "128x150_nt5_H1_none_fp64_paper": Case(128, 150, 5, "H1", "none", 1e-2, 0.0, "fp64", "paper", seed=13),
    "10x8_nt2_H2_none_fp64": Case(10, 8, 2, "H2", "none", 1e-2, 0.0, "fp64", seed=14),
    "16x2046_nt128_H2_divfree_fp64": Case(16, 2046, 128, "H2", "divfree", 1e-2, 0.0, "fp64", seed=15, vmax=0.1),
    "2046x16_nt128_H1_none_fp32": Case(2046, 16, 128, "H1", "none", 1e-2, 0.0, "fp32", seed=16, vmax=0.1),
    # square lengths 2^a 3^b 5^c (one launch per stage, mixed-radix transforms of up to 8 and 4 elements
    # per thread in the row and column parts)
    "250sq_nt4_H2_mass_fp32": Case(250, 250, 4, "H2", "mass_source", 1e-3, 1e-4, "fp32", seed=24),
    "600sq_nt3_H1_divfree_fp32": Case(600, 600, 3, "H1", "divfree", 1e-3, 0.0, "fp32", seed=25),
    "1200sq_nt2_H1_none_fp32": Case(1200, 1200, 2, "H1", "none", 1e-3, 0.0, "fp32", seed=26),
    "90sq_nt3_H1_divfree_fp64": Case(90, 90, 3, "H1", "divfree", 1e-2, 0.0, "fp64", seed=27),
    # one time step with the exact-transpose quadrature: the only adjoint step is both the first and
    # the last, so the assembly's row pass completes the body force from nothing (power-of-two rows)
    # and the pointwise last-step pass does it before a mixed-radix row pass (24 points)
    "32sq_nt1_H1_divfree_fp32": Case(32, 32, 1, "H1", "divfree", 1e-2, 0.0, "fp32", seed=28),
    "32x24_nt1_H2_mass_fp64": Case(32, 24, 1, "H2", "mass_source", 1e-2, 1e-3, "fp64", seed=29),
}


@pytest.fixture(scope="module")
def problems():
    cache = {}
    yield cache
    for p in cache.values():
        p.close()


def get(problems, name):
    if name not in problems:
        print(f"[case] {name} {CASES[name]}", flush=True)
        problems[name] = gpu_problem(CASES[name])
    return problems[name]


@pytest.mark.parametrize("name", list(CASES))
def test_gradient_and_objective_parity(problems, name):
    case = CASES[name]
    P = get(problems, name)
    mT, mR, vlin, vt, vtr = inputs(case)
    ref = oracle_results(case)
    g, J = P.gradient(dev(vlin))
    # relative bound, plus an absolute floor of 32 eps times the body force of an O(1) misfit
    err = np.linalg.norm(host(g) - ref["g"])
    assert err <= case.tol * np.linalg.norm(ref["g"]) + 32 * case.eps * ref["bscale"] + 10 * ref["sens_g"], err
    floor = 32 * case.eps * ref["Jscale"]
    assert abs(J - ref["J"]) <= case.tol * abs(ref["J"]) + floor
    Jt, terms = P.objective(dev(vtr))
    assert abs(Jt - ref["Jt"]) <= case.tol * abs(ref["Jt"]) + floor
    for a, b in zip(terms, ref["terms"]):
        assert abs(a - b) <= case.tol * abs(ref["Jt"]) + floor


@pytest.mark.parametrize("name", list(CASES))
def test_hessian_matvec_parity(problems, name):
    case = CASES[name]
    P = get(problems, name)
    mT, mR, vlin, vt, vtr = inputs(case)
    ref = oracle_results(case)
    P.gradient(dev(vlin), want_J=False)
    H = P.hessian_matvec(dev(vt))
    assert close(host(H), ref["H"], max(case.tol, 10 * ref["sens_H"]))


@pytest.mark.parametrize("name", list(CASES))
def test_state_forward_and_preconditioner_parity(problems, name):
    case = CASES[name]
    P = get(problems, name)
    mT, mR, vlin, vt, vtr = inputs(case)
    ref = oracle_results(case)
    m1 = P.state_forward(dev(vtr))
    assert close(host(m1), ref["m1"], case.tol)
    z = P.precond(dev(ref["g"]))
    assert close(host(z), ref["z"], 1e-12)   # FP64 spectral path in both precisions


def test_matvec_is_bitwise_repeatable(problems):
    """Deterministic kernels: a race in LDS or in the reductions would show up as run-to-run noise."""
    name = "c2_256sq_nt16_H2_mass_fp32"
    case = CASES[name]
    P = get(problems, name)
    mT, mR, vlin, vt, vtr = inputs(case)
    P.gradient(dev(vlin), want_J=False)
    a = host(P.hessian_matvec(dev(vt)))
    b = host(P.hessian_matvec(dev(vt)))
    assert np.array_equal(a, b)
    J1, _ = P.objective(dev(vtr))
    J2, _ = P.objective(dev(vtr))
    assert J1 == J2


def test_matvec_edge_inputs(problems):
    import paper_1503_00757_amd as R
    name = "c1_64sq_nt4_H1_divfree_fp64"
    case = CASES[name]
    mT, mR, vlin, vt, vtr = inputs(case)
    P = gpu_problem(case)
    try:
        with pytest.raises(R.RegError) as e:      # no linearisation point yet
            P.hessian_matvec(dev(vt))
        assert e.value.status == R.ffi.REG_ESTATE
        P.gradient(dev(vlin), want_J=False)
        zero = np.zeros((2, 64, 64))
        assert np.abs(host(P.hessian_matvec(dev(zero)))).max() == 0.0
        x1 = np.arange(64) * 2 * np.pi / 64
        nyq = np.stack([np.cos(32 * x1)[:, None] * np.ones((1, 64)), np.cos(32 * x1)[None, :] * np.ones((64, 1))])
        assert np.abs(host(P.hessian_matvec(dev(nyq)))).max() < 1e-12
    finally:
        P.close()


def test_nonfinite_template_rejected():
    import torch
    import paper_1503_00757_amd as R
    mT = torch.zeros((16, 16), dtype=torch.float64, device="cuda:0")
    mT[3, 4] = float("nan")
    with pytest.raises(R.RegError) as e:
        R.Problem(mT, torch.zeros_like(mT), 2)
    assert e.value.status == R.ffi.REG_EINVAL


def test_constant_template_hessian_is_regulariser(problems):
    """m_T constant: b~ = 0, so H v~ = beta_v A v~ exactly (closed form, no oracle)."""
    import torch
    from paper_1503_00757_amd import Problem
    n = 32
    mT = torch.full((n, n), 0.37, dtype=torch.float64, device="cuda:0")
    P = Problem(mT, mT.clone(), 3, "H2", "none", 2e-3, 0.0, "fp32")
    try:
        x = np.arange(n) * 2 * np.pi / n
        X1, X2 = np.meshgrid(x, x, indexing="ij")
        vt = np.stack([np.sin(3 * X1 + 2 * X2), np.cos(X1 - 5 * X2)])
        P.gradient(dev(0.1 * vt), want_J=False)
        H = host(P.hessian_matvec(dev(vt)))
        expect = 2e-3 * np.stack([13.0 ** 2 * vt[0], 26.0 ** 2 * vt[1]])
        assert close(H, expect, 1e-9)   # b~ is FP32 round-off of the derivative of a constant
    finally:
        P.close()


# Launch shapes of the FP32 fused stages: (elements per thread of the row transform, of the column
# transform, threads per block).  A shape exists on a square power-of-two grid of N >= 64 points when
# both transforms fit (E <= N/2, a block holds at least one transform of each kind, at most 1024
# threads) and the transforms' LDS fits in 160 KiB; smaller or other grids have one fixed shape.
SHAPES = [(8, 16, 128), (4, 16, 256), (4, 8, 256), (8, 8, 128), (8, 8, 256), (4, 4, 256), (8, 16, 256),
          (16, 16, 128), (4, 4, 512), (4, 4, 64), (8, 8, 64), (16, 16, 64),
          (2, 2, 128), (2, 4, 128), (2, 2, 256), (2, 4, 256), (2, 4, 512), (2, 8, 512), (2, 4, 1024), (4, 2, 128)]


def expected_shapes(n1, n2):
    if n1 != n2 or n1 & (n1 - 1) or n1 < 64:
        return {0}
    n, lds = n1, (n1 + n1 // 16) * 8
    ok = set()
    for v, (er, ec, bs) in enumerate(SHAPES):
        if er <= n // 2 and ec <= n // 2 and n // er <= bs <= 1024 and n // ec <= bs and \
                (bs // (n // er)) * 2 * lds <= 160 * 1024 and (bs // (n // ec)) * 2 * lds <= 160 * 1024:
            ok.add(v)
    return ok


@pytest.mark.parametrize("name", ["c2_256sq_nt16_H2_mass_fp32", "c1_64sq_nt4_H1_divfree_fp32", "128x32_nt3_H1_none_fp32",
                                  "128sq_nt3_H2_divfree_fp32", "512sq_nt4_H1_none_fp32"])
def test_every_launch_shape_matches_oracle(problems, name):
    """The autotuner may pick any launch shape (elements per thread, transforms per block): it must time
    exactly the shapes that fit the grid, every one must give an oracle-parity matvec, and so must the
    tuned choice."""
    import paper_1503_00757_amd as R
    case = CASES[name]
    P = get(problems, name)
    mT, mR, vlin, vt, vtr = inputs(case)
    ref = oracle_results(case)
    P.gradient(dev(vlin), want_J=False)
    tol = max(case.tol, 10 * ref["sens_H"])
    want = expected_shapes(case.n1, case.n2)
    P.set_pass_variants([0] * 7)
    P.hessian_matvec(dev(vt))
    rep = P.autotune(reps=5)
    for op in ("A2", "I2", "A1", "I1"):
        assert {v for v, _ in rep[op]} == want, (op, rep[op])
    assert all(c in want for c in rep["chosen"][2:6])
    # the whole-matvec pass only keeps a change that made the matvec faster
    assert 0 < rep["matvec_ms"] <= rep["matvec_ms_isolated_choice"], rep
    H = P.hessian_matvec(dev(vt))
    assert close(host(H), ref["H"], tol)
    for v in sorted(want):
        P.set_pass_variants([v] * 7)
        H = P.hessian_matvec(dev(vt))   # a shape that fits must launch (no fallback is expected here)
        assert close(host(H), ref["H"], tol), v
    P.set_pass_variants([0] * 7)
    with pytest.raises(R.RegError):
        P.set_pass_variants([len(SHAPES)] * 7)


@pytest.mark.parametrize("name", ["c2_256sq_nt16_H2_mass_fp32", "250sq_nt4_H2_mass_fp32", "128x32_nt3_H1_none_fp32"])
def test_timing_hooks(problems, name):
    """reg_time_pass and the phase mode of reg_time_phases on real matvecs: positive intervals, the
    phase stamps only from the one-launch stages of square power-of-two FP32 grids, and the timed
    matvecs leave the matvec's result bitwise unchanged."""
    case = CASES[name]
    P = get(problems, name)
    mT, mR, vlin, vt, vtr = inputs(case)
    P.gradient(dev(vlin), want_J=False)
    before = host(P.hessian_matvec(dev(vt)))
    stamped = case.n1 == case.n2 and case.n1 & (case.n1 - 1) == 0 and case.n1 >= 64 and case.precision == "fp32"
    for which in range(4):
        ms, by, ex = P.time_pass(which, 2)
        assert ms > 0 and ex > 0 and by > 0, (which, ms, ex, by)
        ph = P.time_phases(which, 2)
        assert ph["dispatch"] > 0 and ph["exec"] > 0 and ph["start_spread"] >= 0, ph
        parts = [ph["loads"], ph["transforms"], ph["stores"]]
        if stamped:
            assert all(p > 0 for p in parts), ph
            # a block's phases follow one another inside the launch's execution interval
            assert sum(parts) <= ph["exec"] * 1.001, ph
        else:
            assert parts == [0.0, 0.0, 0.0], ph
    assert np.array_equal(host(P.hessian_matvec(dev(vt))), before)
