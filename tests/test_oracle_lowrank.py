"""Pins of the oracle's low-rank preconditioner correction and warm-start fallback (CPU only).

The correction is checked on operators whose generalised eigenpairs with the spectral
preconditioner M are known in closed form: H = M S with S a scalar Fourier multiplier s(k), so
every single Fourier mode is an eigenvector of M^{-1} H with eigenvalue s(k).  Rayleigh-Ritz on a
span of such modes must return exactly those s(k); the corrected preconditioner must map H to the
identity on that span and leave M^{-1} H alone on modes outside it; PCG must then converge in as
many steps as the corrected operator has distinct eigenvalues.  On the real Gauss-Newton Hessian
and arbitrary directions the balancing form must still give P H = I on the span, be symmetric
positive definite in <., .>_W, and the corrected solve must reach the same minimiser.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, Params, spectral, transport, reduced, solver


def mode(g, k1, k2, comp, phase=0.0):
    x1 = np.arange(g.n1)[:, None] * g.h1
    x2 = np.arange(g.n2)[None, :] * g.h2
    u = np.zeros((2, g.n1, g.n2))
    u[comp] = np.cos(k1 * x1 + k2 * x2 + phase)
    return u



def multiplier_operator(g, p, table):
    """H = M S: S multiplies the Fourier coefficients of (|k1|, |k2|) by table.get(., 1)."""
    s = np.ones_like(g.ksq)
    K1 = np.abs(np.rint(g.k1)).astype(int) + 0 * g.k2.astype(int)
    K2 = np.abs(np.rint(g.k2)).astype(int) + 0 * g.k1.astype(int)
    for (a, b), val in table.items():
        s[(K1 == a) & (K2 == b)] = val

    def H(u):
        su = np.stack([g.ifft(g.keep * s * g.fft(u[c])) for c in range(2)])
        return solver.precond_op(g, p, su)
    return H


TABLE = {(1, 2): 7.0, (3, 1): 0.25, (2, 2): 40.0}


@pytest.mark.parametrize("constraint", ["none", "mass_source", "divfree"])
def test_ritz_values_of_exact_invariant_span(constraint):
    g = Grid(16, 16)
    bw = 1e-3 if constraint == "mass_source" else 0.0
    p = Params(16, 16, 4, "H2", constraint, 1e-2, bw)
    H = multiplier_operator(g, p, TABLE)
    U = [mode(g, 1, 2, 0), mode(g, 3, 1, 1, 0.3), mode(g, 2, 2, 0, 1.1) + mode(g, 1, 2, 0)]
    theta, Z, HZ = solver.lowrank_setup(g, p, H, U)
    assert np.allclose(np.sort(theta), [0.25, 7.0, 40.0], rtol=1e-10)
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    for i, zi in enumerate(Z):
        if constraint == "divfree":
            assert np.abs(spectral.div(g, zi)).max() < 1e-10
        for j, zj in enumerate(Z):
            assert abs(W(zi, solver.precond_op(g, p, zj)) - (i == j)) < 1e-10
            assert abs(W(zi, H(zj)) - (theta[i] if i == j else 0.0)) < 1e-9 * max(theta)
        assert np.allclose(HZ[i], H(zi), atol=1e-12 * np.abs(HZ[i]).max())
    P = solver.corrected_precond(g, p, theta, Z, HZ)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(3)
    x = sum(ci * u for ci, u in zip(c, U))
    x = solver.admissible(g, p, x)
    assert np.allclose(P(H(x)), x, atol=1e-10 * np.abs(x).max())
    # outside the span the corrected preconditioner is the plain one
    y = solver.admissible(g, p, mode(g, 2, 2, 1, 0.7) + mode(g, 4, 1, 0))
    y_out = y - sum(W(z, solver.precond_op(g, p, y)) * z for z in Z)
    assert np.allclose(P(H(y_out)), reduced.precond(g, p, H(y_out)), atol=1e-10 * np.abs(y_out).max())


@pytest.mark.parametrize("constraint", ["none", "mass_source"])
def test_corrected_pcg_converges_in_distinct_eigenvalue_count(constraint):
    """With every outlier mode in the span, P_c H = I on the admissible space: one PCG step."""
    g = Grid(16, 16)
    bw = 1e-3 if constraint == "mass_source" else 0.0
    p = Params(16, 16, 4, "H1", constraint, 1e-2, bw)
    table = {(1, 2): 7.0, (3, 1): 0.25}
    H = multiplier_operator(g, p, table)
    U = []
    for (a, b) in table:
        for kk in [(a, b), (a, -b)]:
            for comp in range(2):
                for ph in (0.0, np.pi / 2):
                    U.append(mode(g, kk[0], kk[1], comp, ph))
    theta, Z, HZ = solver.lowrank_setup(g, p, H, U)
    assert len(Z) == 16      # 2 components x 2 phases x 2 sign patterns x 2 modes, all independent
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    rng = np.random.default_rng(4)
    rhs = solver.admissible(g, p, rng.standard_normal((2, 16, 16)))
    plain = lambda r: reduced.precond(g, p, r)     # noqa: E731
    _, it_p, rr_p = solver.pcg(H, plain, W, g.norm, rhs, 1e-10, 50)
    _, it_c, rr_c = solver.pcg(H, solver.corrected_precond(g, p, theta, Z, HZ), W, g.norm, rhs, 1e-10, 50)
    assert it_p == 3 and rr_p <= 1e-10         # eigenvalues {1, 7, 0.25}
    assert it_c == 1 and rr_c <= 1e-10


def test_dependent_and_nonpositive_directions_are_dropped():
    g = Grid(16, 16)
    p = Params(16, 16, 4, "H1", "none", 1e-2, 0.0)
    H = multiplier_operator(g, p, TABLE)
    u = mode(g, 1, 2, 0)
    theta, Z, HZ = solver.lowrank_setup(g, p, H, [u, 2.0 * u, mode(g, 3, 1, 1)])
    assert len(Z) == len(HZ) == 2 and np.allclose(np.sort(theta), [0.25, 7.0], rtol=1e-10)
    # a Nyquist-only direction is not admissible and vanishes
    nyq = np.zeros((2, 16, 16))
    nyq[0] = (-1.0) ** np.arange(16)[:, None]
    assert solver.lowrank_setup(g, p, H, [nyq])[1] == []
    assert solver.lowrank_setup(g, p, H, [])[1] == []
    # a direction of negative curvature cannot be inverted on: it is dropped
    Hneg = multiplier_operator(g, p, {(1, 2): -3.0, (3, 1): 0.25})
    theta, Z, HZ = solver.lowrank_setup(g, p, Hneg, [mode(g, 1, 2, 0), mode(g, 3, 1, 1)])
    assert len(Z) == 1 and np.allclose(theta, [0.25], rtol=1e-10)


def test_corrected_preconditioner_is_spd():
    g = Grid(16, 16)
    p = Params(16, 16, 4, "H2", "mass_source", 1e-2, 1e-3)
    H = multiplier_operator(g, p, TABLE)
    U = [mode(g, 1, 2, 0), mode(g, 3, 1, 1, 0.3), mode(g, 2, 2, 0, 1.1)]
    theta, Z, HZ = solver.lowrank_setup(g, p, H, U)
    P = solver.corrected_precond(g, p, theta, Z, HZ)
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    rng = np.random.default_rng(9)
    for _ in range(4):
        a = solver.admissible(g, p, rng.standard_normal((2, 16, 16)))
        b = solver.admissible(g, p, rng.standard_normal((2, 16, 16)))
        assert abs(W(a, P(b)) - W(P(a), b)) < 1e-10 * abs(W(a, P(a)))
        assert W(a, P(a)) > 0
    for zi in Z:
        assert W(zi, P(zi)) > 0


@pytest.mark.parametrize("constraint", ["mass_source", "divfree", "none"])
def test_balancing_identity_on_span_of_arbitrary_directions(constraint):
    """P H s = s for every s in span(U) (U random, not invariant), and P symmetric positive definite in
    <., .>_W, on the Gauss-Newton Hessian of a small registration problem."""
    g, p, mT, mR, vs = small_problem(constraint)
    lin = reduced.gradient(g, p, mT, mR, 0.5 * vs)
    H = lambda u: reduced.hessian_matvec(g, p, lin, u)   # noqa: E731
    rng = np.random.default_rng(11)
    U = [rng.standard_normal((2, 16, 16)) for _ in range(3)]
    theta, Z, HZ = solver.lowrank_setup(g, p, H, U)
    assert len(Z) == 3 and np.all(theta > 0)
    P = solver.corrected_precond(g, p, theta, Z, HZ)
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    x = solver.admissible(g, p, 0.3 * U[0] - 1.2 * U[1] + 0.7 * U[2])
    assert np.allclose(P(H(x)), x, atol=1e-9 * np.abs(x).max())
    for _ in range(3):
        a = solver.admissible(g, p, rng.standard_normal((2, 16, 16)))
        b = solver.admissible(g, p, rng.standard_normal((2, 16, 16)))
        assert abs(W(a, P(b)) - W(P(a), b)) < 1e-10 * abs(W(a, P(a)))
        assert W(a, P(a)) > 0
    # with a Hessian from another linearisation point (stale H Z) P stays SPD
    lin2 = reduced.gradient(g, p, mT, mR, vs)
    H2 = lambda u: reduced.hessian_matvec(g, p, lin2, u)   # noqa: E731
    a = solver.admissible(g, p, rng.standard_normal((2, 16, 16)))
    assert W(a, P(a)) > 0 and W(P(H2(a)), H2(a)) > 0


def small_problem(constraint="mass_source", norm="H2", n=16, nt=4, beta_v=1e-3):
    bw = 1e-3 if constraint == "mass_source" else 0.0
    p = Params(n, n, nt, norm, constraint, beta_v, bw)
    g = Grid(n, n)
    rng = np.random.default_rng(5)
    mT = sd.template_image(n, n, 5, 0, rng)
    vs = sd.scale_to_max(sd.random_velocity(n, n, 3, rng, True, constraint != "divfree"), 0.3)
    mR = transport.state_forward(g, p, mT, vs).m[-1]
    return g, p, mT, mR, vs


@pytest.mark.parametrize("constraint", ["mass_source", "divfree"])
def test_corrected_solve_reaches_the_same_minimiser(constraint):
    g, p, mT, mR, vs = small_problem(constraint)
    opts = dict(max_newton=30, gtol_rel=1e-6, max_pcg=300)
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(**opts))
    lin0 = reduced.gradient(g, p, mT, mR, np.zeros_like(vs))
    U = np.stack([v, lin0.g, vs])
    vc, stc = solver.solve(g, p, mT, mR, solver.SolveOpts(precond_U=U, **opts))
    assert st.status == stc.status == solver.OK
    assert stc.lowrank is not None and np.all(stc.lowrank[0] > 0) and stc.lowrank_dim == 3
    assert stc.n_matvec == stc.pcg_iters + 3          # Rayleigh-Ritz costs one matvec per direction
    assert g.norm(vc - v) <= 1e-3 * g.norm(v)
    # the first PCG solve to a tight tolerance needs fewer iterations with the correction
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    mv = lambda s: reduced.hessian_matvec(g, p, lin0, s)   # noqa: E731
    theta, Z, HZ = solver.lowrank_setup(g, p, mv, list(U))
    _, it_p, _ = solver.pcg(mv, lambda r: reduced.precond(g, p, r), W, g.norm, -lin0.g, 1e-6, 300)
    _, it_c, _ = solver.pcg(mv, solver.corrected_precond(g, p, theta, Z, HZ), W, g.norm, -lin0.g, 1e-6, 300)
    assert it_c < it_p


@pytest.mark.parametrize("constraint", ["mass_source", "divfree", "none"])
def test_recorded_pcg_directions_are_conjugate_and_deflate(constraint):
    """CG search directions are mutually H-conjugate in <., .>_W, so the balancing correction built
    from the ones a solve recorded (e = <s, H s>_W) maps each of them to itself: P H s = s."""
    g, p, mT, mR, vs = small_problem(constraint)
    lin = reduced.gradient(g, p, mT, mR, np.zeros_like(vs))
    mv = lambda s: reduced.hessian_matvec(g, p, lin, s)   # noqa: E731
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    rec = []
    _, its, _ = solver.pcg(mv, lambda r: reduced.precond(g, p, r), W, g.norm, -lin.g, 1e-8, 300,
                           record=rec, record_max=4)
    assert its > 4 and len(rec) == 4
    for i, (si, hsi, ei) in enumerate(rec):
        assert np.allclose(hsi, mv(si), rtol=0, atol=1e-13 * np.abs(hsi).max())
        assert abs(ei - W(si, hsi)) < 1e-12 * ei and ei > 0
        for j in range(i):
            assert abs(W(rec[j][0], hsi)) < 1e-8 * np.sqrt(ei * rec[j][2])
    E = [e for _, _, e in rec]
    P = solver.corrected_precond(g, p, E, [r[0] for r in rec], [r[1] for r in rec])
    for si, hsi, _ in rec:
        assert np.allclose(P(hsi), si, atol=1e-7 * np.abs(si).max())


@pytest.mark.parametrize("constraint", ["mass_source", "divfree"])
def test_recycled_directions_cut_pcg_iterations(constraint):
    g, p, mT, mR, vs = small_problem(constraint)
    opts = dict(max_newton=30, gtol_rel=1e-6, max_pcg=300)
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(**opts))
    vr, str_ = solver.solve(g, p, mT, mR, solver.SolveOpts(recycle=4, lowrank_capacity=16, **opts))
    assert st.status == str_.status == solver.OK
    assert str_.lowrank_dim == 16 and st.lowrank_dim == 0
    assert str_.n_matvec == str_.pcg_iters            # recycling costs no extra matvecs
    assert str_.pcg_iters < 0.75 * st.pcg_iters, (str_.pcg_iters, st.pcg_iters)
    assert g.norm(vr - v) <= 1e-3 * g.norm(v)
    # the first Newton step sees no correction yet: identical to the plain one
    assert str_.history[0]["pcg"] == st.history[0]["pcg"]
    # capacity bounds the set; recycle = 0 adds nothing
    _, s2 = solver.solve(g, p, mT, mR, solver.SolveOpts(recycle=4, lowrank_capacity=6, **opts))
    assert s2.lowrank_dim == 6
    _, s3 = solver.solve(g, p, mT, mR, solver.SolveOpts(recycle=0, lowrank_capacity=6, **opts))
    assert s3.lowrank_dim == 0 and s3.pcg_iters == st.pcg_iters


def test_warm_start_fallback_restarts_from_zero():
    g, p, mT, mR, vs = small_problem()
    opts = dict(max_newton=20, gtol_rel=1e-3)
    v, st = solver.solve(g, p, mT, mR, solver.SolveOpts(**opts))
    bad = 40.0 * sd.scale_to_max(sd.random_velocity(16, 16, 3, np.random.default_rng(1), True, True), 0.3)
    assert reduced.objective(g, p, mT, mR, bad)[0] > reduced.objective(g, p, mT, mR, np.zeros_like(bad))[0]
    vb, stb = solver.solve(g, p, mT, mR, solver.SolveOpts(v0=bad, **opts))
    assert stb.fallback_used == 1 and st.fallback_used == 0
    assert np.array_equal(vb, v)
    assert stb.n_pde == st.n_pde + 2 and stb.newton_iters == st.newton_iters
    _, stg = solver.solve(g, p, mT, mR, solver.SolveOpts(v0=v, **opts))
    assert stg.fallback_used == 0 and stg.newton_iters == 0


@pytest.mark.parametrize("constraint", ["none", "mass_source"])
def test_subspace_iteration_finds_the_leading_eigenspaces(constraint):
    """H = M S: the leading generalised eigenvectors are the Fourier modes with the largest s(k).
    The (2, 2) class spans 8 real vector fields (cos and sin of 2x1 +- 2x2, two components) with
    s = 40, the (1, 2) class another 8 with s = 7, everything else s <= 1.  Ten directions from
    random fields must converge to all 8 of the first class and 2 of the second, in that order."""
    g = Grid(16, 16)
    bw = 1e-3 if constraint == "mass_source" else 0.0
    p = Params(16, 16, 4, "H2", constraint, 1e-2, bw)
    H = multiplier_operator(g, p, {(2, 2): 40.0, (1, 2): 7.0, (3, 1): 0.25})
    rng = np.random.default_rng(11)
    U = [rng.standard_normal((2, 16, 16)) for _ in range(10)]
    theta, Z = solver.ritz_directions(g, p, H, U, iters=30)
    assert np.allclose(theta[:8], 40.0, rtol=1e-9)
    assert np.allclose(theta[8:], 7.0, rtol=1e-6)
    assert np.all(np.diff(theta) <= 1e-9 * theta[0])
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    for t, z in zip(theta, Z):
        assert np.allclose(H(z), t * solver.precond_op(g, p, z), atol=1e-6 * t * np.abs(z).max())
        assert abs(W(z, solver.precond_op(g, p, z)) - 1.0) < 1e-9
    # no iteration: plain Rayleigh-Ritz on the random span, values sorted the same way
    theta0, _ = solver.ritz_directions(g, p, H, U, iters=0)
    ref, _, _ = solver.lowrank_setup(g, p, H, U)
    assert np.allclose(theta0, np.sort(ref)[::-1], rtol=1e-12)
    assert theta0[0] < 40.0 - 1e-3   # a random span is not invariant
