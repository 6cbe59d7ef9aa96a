"""Pins of the oracle's transport solves (CPU only).

Q3 constant velocity: each Fourier mode is multiplied by Heun's amplification factor
R(z) = 1 + z + z^2/2, z = -i h_t k.c, per step (state) and by R(conj z) (adjoint); and it converges to
the exact shift m_T(x - c).  Q4 constant v and v~: the incremental state obeys a closed per-mode
recurrence.  Q15 second-order convergence in time.  Trapezoid quadrature of a time-constant integrand.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import Grid, Params, transport


def _R(z):
    return 1 + z + 0.5 * z * z


def _setup(n1, n2, nt, mode="dto"):
    g = Grid(n1, n2)
    p = Params(n1, n2, nt, "H1", "none", 1e-2, 0.0, mode)
    mT = sd.random_field(n1, n2, min(n1, n2) // 2 - 1, 11)
    return g, p, mT


@pytest.mark.parametrize("n1,n2,nt", [(16, 16, 3), (12, 20, 5)])
def test_q3_constant_velocity_modes(n1, n2, nt):
    g, p, mT = _setup(n1, n2, nt)
    c = np.array([0.7, -0.4])
    v = np.stack([np.full((n1, n2), c[0]), np.full((n1, n2), c[1])])
    traj = transport.state_forward(g, p, mT, v)
    z = -1j * (1.0 / nt) * (g.k1 * c[0] + g.k2 * c[1])
    expect = g.fft(mT) * _R(z) ** nt
    assert np.abs(g.fft(traj.m[-1]) - expect).max() < 1e-11 * np.abs(expect).max()
    lam, _ = transport.adjoint_backward(g, p, v, mT)
    expect_adj = g.fft(mT) * _R(np.conj(z)) ** nt
    assert np.abs(g.fft(lam[0]) - expect_adj).max() < 1e-11 * np.abs(expect_adj).max()


def test_q3_converges_to_exact_shift():
    """m(1) -> m_T(x - c) as n_t grows, at second order (Heun truncation)."""
    n = 32
    x1, x2 = sd.grid_coords(n, n)
    X1, X2 = np.meshgrid(x1, x2, indexing="ij")
    c = np.array([0.6, 0.3])
    mT = np.sin(X1) * np.cos(2 * X2)
    exact = np.sin(X1 - c[0]) * np.cos(2 * (X2 - c[1]))
    errs = []
    for nt in (8, 16, 32):
        g, p, _ = _setup(n, n, nt)
        v = np.stack([np.full((n, n), c[0]), np.full((n, n), c[1])])
        errs.append(np.abs(transport.state_forward(g, p, mT, v).m[-1] - exact).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("mode", ["dto", "paper"])
def test_q4_incremental_state_constant_fields(mode):
    n1, n2, nt = 16, 12, 4
    g, p, mT = _setup(n1, n2, nt, mode)
    c = np.array([0.5, 0.8])
    dd = np.array([-0.3, 0.45])
    v = np.stack([np.full((n1, n2), c[0]), np.full((n1, n2), c[1])])
    vt = np.stack([np.full((n1, n2), dd[0]), np.full((n1, n2), dd[1])])
    traj = transport.state_forward(g, p, mT, v)
    mt = transport.inc_state_forward(g, p, v, traj, vt)
    h = 1.0 / nt
    z = -1j * h * (g.k1 * c[0] + g.k2 * c[1])
    kd = g.k1 * dd[0] + g.k2 * dd[1]
    mTh = g.fft(mT)
    u = np.zeros_like(mTh)
    R = _R(z)
    for j in range(nt):
        s = -1j * kd * R ** j * mTh
        ss = -1j * kd * (1 + z) * R ** j * mTh if mode == "dto" else -1j * kd * R ** (j + 1) * mTh
        u = R * u + 0.5 * h * ((1 + z) * s + ss)
    assert np.abs(g.fft(mt) - u).max() < 1e-11 * np.abs(u).max()


def test_q4_incremental_state_continuous_limit():
    """m~(1) -> -d . grad m_T(x - c) for constant v = c, v~ = d."""
    n = 32
    x1, x2 = sd.grid_coords(n, n)
    X1, X2 = np.meshgrid(x1, x2, indexing="ij")
    c, dd = np.array([0.4, -0.2]), np.array([0.3, 0.5])
    mT = np.cos(X1 + X2)
    exact = (dd[0] + dd[1]) * np.sin((X1 - c[0]) + (X2 - c[1]))
    errs = []
    for nt in (8, 16, 32):
        g, p, _ = _setup(n, n, nt)
        v = np.stack([np.full((n, n), c[0]), np.full((n, n), c[1])])
        vt = np.stack([np.full((n, n), dd[0]), np.full((n, n), dd[1])])
        traj = transport.state_forward(g, p, mT, v)
        errs.append(np.abs(transport.inc_state_forward(g, p, v, traj, vt) - exact).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_q15_second_order_in_time_variable_velocity():
    n = 16
    g = Grid(n, n)
    mT = sd.random_field(n, n, 4, 21)
    v = 0.3 * sd.random_vec(n, n, 3, 22)
    ref = transport.state_forward(g, Params(n, n, 256, "H1", "none", 1e-2), mT, v).m[-1]
    e = [np.abs(transport.state_forward(g, Params(n, n, nt, "H1", "none", 1e-2), mT, v).m[-1] - ref).max()
         for nt in (16, 32)]
    assert 3.3 < e[0] / e[1] < 4.7


def test_trapezoid_quadrature_of_time_constant_integrand():
    """With v = 0 every lam_j and G_j is constant in time, so both quadratures give lam grad m_T."""
    n, nt = 12, 5
    for mode in ("dto", "paper"):
        g, p, mT = _setup(n, n, nt, mode)
        v = np.zeros((2, n, n))
        traj = transport.state_forward(g, p, mT, v)
        lamT = sd.random_field(n, n, 4, 5)
        lam, lam_s = transport.adjoint_backward(g, p, v, lamT)
        b = transport.body_force(p, traj, lam, lam_s)
        Gm = np.stack([transport.d(g, mT, 0), transport.d(g, mT, 1)])
        assert np.abs(b - lamT * Gm).max() < 1e-13
