"""Pins of the oracle's reduced-space operators (CPU only).

Q5 linearisation at v = 0 (closed form); Q7 constant template; Q8 adjoint symmetry <Hx,y> = <x,Hy>;
Q9 gradient against central differences of the objective; Q10 Taylor test at the true velocity
(lam = 0 there, so GN equals Newton); Q11 positivity; Q12 brute force against an independent
dense-matrix construction; Z5 the mass-source projection satisfies g = K grad J_pen.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, Params, spectral, transport, reduced
from dense_reference import Dense

CASES = [("none", "H1"), ("divfree", "H1"), ("mass_source", "H2"), ("mass_source", "H1"), ("none", "H2"),
         ("mass_source", "H3"), ("divfree", "stokes"), ("none", "stokes")]


def problem(constraint, norm, n=16, nt=3, mode="dto", amp=0.5, seed=1, n2=None):
    n2 = n2 or n
    bw = 1e-3 if constraint == "mass_source" else 0.0
    p = Params(n, n2, nt, norm, constraint, 1e-2, bw, mode, nu=1.7 if norm == "stokes" else 1.0)
    g = Grid(n, n2)
    rng = np.random.default_rng(seed)
    mT = sd.template_image(n, n2, 4, 3, rng)
    vs = sd.scale_to_max(sd.random_velocity(n, n2, 3, rng, True, constraint != "divfree"), amp)
    mR = transport.state_forward(g, p, mT, vs).m[-1]
    return g, p, mT, mR, vs


def dirs(n, constraint, seeds=(3, 4), n2=None):
    n2 = n2 or n
    return [sd.random_vec(n, n2, min(5, n // 2 - 1, n2 // 2 - 1), s, divfree=(constraint == "divfree"))
            for s in seeds]


@pytest.mark.parametrize("constraint,norm", CASES)
@pytest.mark.parametrize("mode", ["dto", "paper"])
def test_q5_linearisation_at_zero(constraint, norm, mode):
    g, p, mT, mR, _ = problem(constraint, norm, mode=mode)
    lin = reduced.gradient(g, p, mT, mR, np.zeros((2, 16, 16)))
    Gm = spectral.grad(g, mT)
    g_expect = spectral.nyquist_project(g, spectral.apply_K(g, p, (mR - mT) * Gm))
    assert np.abs(lin.g - g_expect).max() < 1e-12 * np.abs(g_expect).max()
    vt, _ = dirs(16, constraint)
    H = reduced.hessian_matvec(g, p, lin, vt)
    vtp = spectral.nyquist_project(g, vt)
    gn = (vtp[0] * Gm[0] + vtp[1] * Gm[1]) * Gm
    if norm == "stokes":
        # E(0) = 0: constant viscosity eps^{(1-nu)/(2nu)} times -Lap - grad div (symbol |k|^2 I + k k^T),
        # projected together with the body force
        eta0 = p.eps ** ((1 - p.nu) / (2 * p.nu))
        v1h, v2h = g.fft(vtp[0]), g.fft(vtp[1])
        kv = g.k1 * v1h + g.k2 * v2h
        B = eta0 * np.stack([g.ifft(g.ksq * v1h + g.k1 * kv), g.ifft(g.ksq * v2h + g.k2 * kv)])
        expect = spectral.nyquist_project(g, spectral.apply_K(g, p, p.beta_v * B + gn))
    else:
        expect = spectral.nyquist_project(g, p.beta_v * spectral.apply_A(g, p, vtp) + spectral.apply_K(g, p, gn))
    assert np.abs(H - expect).max() < 1e-12 * np.abs(expect).max()


@pytest.mark.parametrize("constraint,norm", CASES[:3])
def test_q7_constant_template(constraint, norm):
    g, p, _, _, vs = problem(constraint, norm)
    mT = np.full((16, 16), 0.37)
    lin = reduced.gradient(g, p, mT, mT.copy(), 0.5 * spectral.nyquist_project(g, vs))
    assert np.abs(lin.b).max() < 1e-13
    vt, _ = dirs(16, constraint)
    vtp = spectral.nyquist_project(g, vt)
    H = reduced.hessian_matvec(g, p, lin, vt)
    expect = spectral.nyquist_project(g, p.beta_v * spectral.apply_A(g, p, vtp))
    assert np.abs(H - expect).max() < 1e-12 * np.abs(expect).max()


@pytest.mark.parametrize("constraint,norm", CASES)
def test_q8_symmetry_dto(constraint, norm):
    g, p, mT, mR, vs = problem(constraint, norm)
    lin = reduced.gradient(g, p, mT, mR, 0.5 * vs)
    x, y = dirs(16, constraint)
    a = reduced.w_inner(g, p, reduced.hessian_matvec(g, p, lin, x), y)
    b = reduced.w_inner(g, p, x, reduced.hessian_matvec(g, p, lin, y))
    assert abs(a - b) < 1e-13 * abs(a)


def test_q8_paper_mode_asymmetry_shrinks_second_order():
    asym = []
    for nt in (4, 8, 16):
        g, p, mT, mR, vs = problem("none", "H1", nt=nt, mode="paper", amp=0.8)
        lin = reduced.gradient(g, p, mT, mR, 0.5 * vs)
        x, y = dirs(16, "none")
        a = g.inner(reduced.hessian_matvec(g, p, lin, x), y)
        b = g.inner(x, reduced.hessian_matvec(g, p, lin, y))
        asym.append(abs(a - b) / abs(a))
    assert asym[0] / asym[1] > 3.0 and asym[1] / asym[2] > 3.0


@pytest.mark.parametrize("constraint,norm", CASES)
def test_q9_gradient_finite_differences(constraint, norm):
    g, p, mT, mR, vs = problem(constraint, norm)
    v = 0.5 * spectral.nyquist_project(g, vs)
    lin = reduced.gradient(g, p, mT, mR, v)
    dd = spectral.nyquist_project(g, dirs(16, constraint)[0])
    eps = 1e-5
    Jp, _ = reduced.objective(g, p, mT, mR, v + eps * dd)
    Jm, _ = reduced.objective(g, p, mT, mR, v - eps * dd)
    fd = (Jp - Jm) / (2 * eps)
    an = reduced.directional_derivative(g, p, lin.g, dd)
    assert abs(fd - an) < 1e-8 * abs(an)


@pytest.mark.parametrize("constraint,norm", CASES[:3])
def test_q10_taylor_at_true_velocity(constraint, norm):
    g, p, mT, mR, vs = problem(constraint, norm)
    lin = reduced.gradient(g, p, mT, mR, vs)
    assert lin.terms[0] < 1e-26                              # m_1 = m_R exactly (inverse crime)
    assert np.abs(lin.b).max() < 1e-14                       # lam = 0
    dd = spectral.nyquist_project(g, dirs(16, constraint)[0])
    Hd = reduced.hessian_matvec(g, p, lin, dd)
    rem = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        J, _ = reduced.objective(g, p, mT, mR, lin.v + eps * dd)
        lin_part = reduced.directional_derivative(g, p, lin.g, dd)
        rem.append(abs(J - lin.J - eps * lin_part - 0.5 * eps ** 2 * reduced.w_inner(g, p, Hd, dd)))
    assert rem[0] / rem[1] > 6.0 and rem[1] / rem[2] > 6.0     # O(eps^3)


@pytest.mark.parametrize("constraint,norm", CASES[:3])
def test_q11_positivity(constraint, norm):
    g, p, mT, mR, vs = problem(constraint, norm)
    lin = reduced.gradient(g, p, mT, mR, 0.7 * vs)
    for x in dirs(16, constraint, seeds=(5, 6, 7)):
        x = spectral.nyquist_project(g, x)
        xHx = reduced.w_inner(g, p, x, reduced.hessian_matvec(g, p, lin, x))
        assert xHx >= p.beta_v * g.inner(x, spectral.apply_A(g, p, x)) * (1 - 1e-12)


@pytest.mark.parametrize("constraint,norm,n1,n2,nt", [
    ("none", "H1", 8, 8, 3), ("divfree", "H1", 8, 6, 2), ("mass_source", "H2", 8, 8, 2),
    ("none", "H2", 6, 8, 4)])
def test_q12_dense_brute_force(constraint, norm, n1, n2, nt):
    g, p, mT, mR, vs = problem(constraint, norm, n=n1, n2=n2, nt=nt, amp=0.6)
    D = Dense(n1, n2, nt, norm, constraint, p.beta_v, p.beta_w)
    v = 0.8 * spectral.nyquist_project(g, vs)
    lin = reduced.gradient(g, p, mT, mR, v)
    Hd = D.hessian_gn(v.reshape(-1), mT.reshape(-1))
    N2 = 2 * n1 * n2
    Ho = np.zeros((N2, N2))
    for i in range(N2):
        e = np.zeros(N2)
        e[i] = 1.0
        Ho[:, i] = reduced.hessian_matvec(g, p, lin, e.reshape(2, n1, n2)).reshape(-1)
    assert np.abs(Ho - Hd).max() < 1e-11 * np.abs(Hd).max()
    gd = D.gradient(v.reshape(-1), mT.reshape(-1), mR.reshape(-1))
    assert np.abs(lin.g.reshape(-1) - gd).max() < 1e-12 * np.abs(gd).max()
    m1 = D.forward(v.reshape(-1), mT.reshape(-1))
    assert np.abs(lin.traj.m[-1].reshape(-1) - m1).max() < 1e-13


@pytest.mark.parametrize("norm", ["H1", "H2", "H3"])
def test_z5_mass_source_gradient_is_projected_penalty_gradient(norm):
    g, p, mT, mR, vs = problem("mass_source", norm)
    lin = reduced.gradient(g, p, mT, mR, 0.5 * vs)
    gp = spectral.nyquist_project(g, spectral.apply_K(g, p, reduced.penalised_gradient(g, p, lin)))
    assert np.abs(gp - lin.g).max() < 1e-12 * np.abs(lin.g).max()


def test_paper_mode_equals_dto_to_second_order():
    diffs = []
    for nt in (4, 8, 16):
        out = {}
        for mode in ("dto", "paper"):
            g, p, mT, mR, vs = problem("none", "H1", nt=nt, mode=mode, amp=0.8)
            lin = reduced.gradient(g, p, mT, mR, 0.5 * vs)
            out[mode] = reduced.hessian_matvec(g, p, lin, dirs(16, "none")[0])
        diffs.append(np.abs(out["dto"] - out["paper"]).max())
    assert diffs[0] / diffs[1] > 3.0 and diffs[1] / diffs[2] > 3.0
