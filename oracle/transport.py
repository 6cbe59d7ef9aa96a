"""State, adjoint and incremental transport solves (oracle; test infrastructure only).

Paper: Sec. 3.1, eqs. (state-eq), (adj-eq), (terminal-adj-eq) and the body force b = int_0^1 lam grad m dt;
Sec. 3.2, eq. (newton-step) and the incremental body force; Sec. 3.3, eqs. (state-eq-elim),
(adj-eq-elim), (inc-state-eq-elim), (inc-adj-eq-elim); Sec. 4 (explicit second-order Runge-Kutta
in time, trapezoidal quadrature, Gauss-Newton approximation: every term that carries lam is dropped
from the incremental system).

Full Newton (an extension; the paper uses Gauss-Newton): for the 'dto' discretisation the
incremental system is differentiated exactly, keeping the terms that carry lam, so that the matvec is
the exact Hessian of the discrete reduced objective (``inc_adjoint_backward_full``,
``inc_body_force_full``).

Discretisation (readings listed in the design notes):
  * h_t = 1/n_t, t_j = j h_t; the RK2 scheme is Heun's method (explicit trapezoid).  For the
    autonomous state and adjoint equations every two-stage RK2 gives I + h L + h^2 L^2 / 2.
  * Transport operator L_v u = -(v1 d1 u + v2 d2 u) (non-conservative form of eq. (state-eq)) and
    its L2 transpose L_v^T q = d1(v1 q) + d2(v2 q) (conservative form of eq. (adj-eq)).  With the
    Nyquist wavenumber zeroed the spectral derivative is exactly skew, so L_v^T is the exact
    transpose of L_v.
  * Two quadratures for the body-force time integrals:
      'dto'   b = sum_{j<n_t} (h_t/2) [lam*_j G_j + lam_{j+1} G*_j]  and the second incremental-state
              stage samples the source at the state predictor m*_j.  This is the exact transpose of
              the discrete forward map, so the gradient is exact for the discrete objective and the
              GN Hessian is exactly symmetric.
      'paper' b = sum_{j=0}^{n_t} w_j h_t lam_j G_j with trapezoid weights w_0 = w_{n_t} = 1/2, and
              the second stage samples the source at m_{j+1} (Sec. 4 as printed).
  Here G_j = grad m_j, G*_j = grad m*_j, and lam*_j is the adjoint Heun predictor.
"""
from __future__ import annotations

import numpy as np

from .spectral import Grid, Params, d, grad


def L(g: Grid, v, u):
    """L_v u = -(v . grad u)."""
    return -(v[0] * d(g, u, 0) + v[1] * d(g, u, 1))


def LT(g: Grid, v, q):
    """L_v^T q = div(v q)."""
    return d(g, v[0] * q, 0) + d(g, v[1] * q, 1)


class StateTrajectory:
    """Stored state trajectory: m_j (j = 0..n_t), the Heun predictors m*_j (j < n_t) and the
    gradients G_j = grad m_j, G*_j = grad m*_j that the adjoint and incremental solves need."""

    def __init__(self, m, ms, G, Gs):
        self.m, self.ms, self.G, self.Gs = m, ms, G, Gs


def state_forward(g: Grid, p: Params, mT, v) -> StateTrajectory:
    """Solve d_t m + grad m . v = 0, m(0) = m_T forward in time by Heun (eq. (state-eq-elim))."""
    h = 1.0 / p.nt
    m = [mT.copy()]
    ms, G, Gs = [], [], []
    for _ in range(p.nt):
        mj = m[-1]
        Gj = grad(g, mj)
        k1 = -(v[0] * Gj[0] + v[1] * Gj[1])
        mstar = mj + h * k1
        Gsj = grad(g, mstar)
        k2 = -(v[0] * Gsj[0] + v[1] * Gsj[1])
        m.append(mj + 0.5 * h * (k1 + k2))
        ms.append(mstar)
        G.append(Gj)
        Gs.append(Gsj)
    G.append(grad(g, m[-1]))                      # G_{n_t}, used by the trapezoid quadrature only
    return StateTrajectory(m, ms, G, Gs)


def adjoint_backward(g: Grid, p: Params, v, lam_T):
    """Solve -d_t lam - div(v lam) = 0 backward from lam(1) = lam_T by Heun (eq. (adj-eq-elim)).

    Returns (lam, lam_star) with lam[j] for j = 0..n_t and lam_star[j] for j < n_t.
    """
    h = 1.0 / p.nt
    lam = [None] * (p.nt + 1)
    lam_star = [None] * p.nt
    lam[p.nt] = lam_T.copy()
    for j in range(p.nt - 1, -1, -1):
        k1 = LT(g, v, lam[j + 1])
        lam_star[j] = lam[j + 1] + h * k1
        k2 = LT(g, v, lam_star[j])
        lam[j] = lam[j + 1] + 0.5 * h * (k1 + k2)
    return lam, lam_star


def body_force(p: Params, traj: StateTrajectory, lam, lam_star):
    """Time integral b = int_0^1 lam grad m dt (Sec. 3.1) in the chosen quadrature."""
    h = 1.0 / p.nt
    b = np.zeros_like(traj.G[0])
    if p.adjoint == "dto":
        for j in range(p.nt):
            b += 0.5 * h * (lam_star[j] * traj.G[j] + lam[j + 1] * traj.Gs[j])
    else:
        for j in range(p.nt + 1):
            w = 0.5 if j in (0, p.nt) else 1.0
            b += w * h * lam[j] * traj.G[j]
    return b


def inc_state_forward(g: Grid, p: Params, v, traj: StateTrajectory, vt):
    """Incremental state, eq. (inc-state-eq-elim): d_t m~ + grad m~ . v + grad m . v~ = 0, m~(0) = 0.

    Heun with source S = -v~ . grad m sampled at m_j (first stage) and at m*_j ('dto') or m_{j+1}
    ('paper') in the second stage.  Returns m~_{n_t}.
    """
    h = 1.0 / p.nt
    mt = np.zeros_like(traj.m[0])
    for j in range(p.nt):
        Sj = -(vt[0] * traj.G[j][0] + vt[1] * traj.G[j][1])
        Gnext = traj.Gs[j] if p.adjoint == "dto" else traj.G[j + 1]
        Ss = -(vt[0] * Gnext[0] + vt[1] * Gnext[1])
        k1 = L(g, v, mt) + Sj
        mstar = mt + h * k1
        mt = mt + 0.5 * h * (k1 + L(g, v, mstar) + Ss)
    return mt


def inc_adjoint_backward_gn(g: Grid, p: Params, v, traj: StateTrajectory, mt_final):
    """Gauss-Newton incremental adjoint, eq. (inc-adj-eq-elim) with the div(lam v~) term dropped
    (Sec. 4): -d_t lam~ - div(lam~ v) = 0, lam~(1) = -m~(1) (terminal condition of eq. (second-order-elim)).

    Returns the incremental body force b~ = int_0^1 lam~ grad m dt (the lam grad m~ term is dropped
    under Gauss-Newton) in the chosen quadrature.
    """
    lam, lam_star = adjoint_backward(g, p, v, -mt_final)
    return body_force(p, traj, lam, lam_star)


# ---- full Newton (second-order) incremental system, exact for the 'dto' discretisation ---------------
def inc_state_forward_stages(g: Grid, p: Params, v, traj: StateTrajectory, vt):
    """The incremental state of ``inc_state_forward`` with its stage values kept: returns
    (mt, mt_star) with m~_j for j = 0..n_t and the predictors m~*_j for j < n_t."""
    h = 1.0 / p.nt
    mt = [np.zeros_like(traj.m[0])]
    mts = []
    for j in range(p.nt):
        Sj = -(vt[0] * traj.G[j][0] + vt[1] * traj.G[j][1])
        Gnext = traj.Gs[j] if p.adjoint == "dto" else traj.G[j + 1]
        Ss = -(vt[0] * Gnext[0] + vt[1] * Gnext[1])
        k1 = L(g, v, mt[-1]) + Sj
        mstar = mt[-1] + h * k1
        mts.append(mstar)
        mt.append(mt[-1] + 0.5 * h * (k1 + L(g, v, mstar) + Ss))
    return mt, mts


def inc_adjoint_backward_full(g: Grid, p: Params, v, vt, lam, lam_star, mt_final):
    """Full-Newton incremental adjoint: the derivative along v~ of the discrete adjoint recursion
    (Heun on eq. (adj-eq-elim)), i.e. eq. (inc-adj-eq-elim) with the div(lam v~) term kept:

        lam~*_j = lam~_{j+1} + h (L_v^T lam~_{j+1} + L_v~^T lam_{j+1}),
        lam~_j  = (lam~_{j+1} + lam~*_j)/2 + (h/2)(L_v^T lam~*_j + L_v~^T lam*_j),

    from lam~_{n_t} = -m~_{n_t}.  Returns (lam~, lam~*) like ``adjoint_backward``."""
    h = 1.0 / p.nt
    lt = [None] * (p.nt + 1)
    lts = [None] * p.nt
    lt[p.nt] = -mt_final
    for j in range(p.nt - 1, -1, -1):
        k1 = LT(g, v, lt[j + 1]) + LT(g, vt, lam[j + 1])
        lts[j] = lt[j + 1] + h * k1
        k2 = LT(g, v, lts[j]) + LT(g, vt, lam_star[j])
        lt[j] = lt[j + 1] + 0.5 * h * (k1 + k2)
    return lt, lts


def inc_body_force_full(g: Grid, p: Params, traj: StateTrajectory, lam, lam_star, mt, mts, lt, lts):
    """Derivative along v~ of the 'dto' body force sum (h/2)(lam*_j G_j + lam_{j+1} G*_j):
    b~ = sum (h/2)(lam~*_j G_j + lam*_j grad m~_j + lam~_{j+1} G*_j + lam_{j+1} grad m~*_j)."""
    h = 1.0 / p.nt
    b = np.zeros_like(traj.G[0])
    for j in range(p.nt):
        b += 0.5 * h * (lts[j] * traj.G[j] + lam_star[j] * grad(g, mt[j])
                        + lt[j + 1] * traj.Gs[j] + lam[j + 1] * grad(g, mts[j]))
    return b
