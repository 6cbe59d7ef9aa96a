"""Reduced-space objective, gradient, Gauss-Newton Hessian matvec and preconditioner
(oracle; test infrastructure only).

Paper: Sec. 2, eq. (objective) with eqs. (reg-v), (reg-w); Sec. 3.3, eq. (control-eq-elim)
g = beta_v A[v] + K[b]; eq. (inc-control-eq-elim) H v~ = beta_v B[v~] + L[b~] with B = A and L = K for
the quadratic seminorms; Sec. 4 (Gauss-Newton: every term carrying lam is dropped, which keeps H
positive definite); App. E.2 (preconditioner (beta_v A)^{-1}).  ``hessian_matvec_full`` keeps the lam
terms (full Newton, an extension).

Readings (listed in the design notes):
  * every velocity-like input (v, v~) and output (g, H v~) has its Nyquist modes removed (F_Nyq);
  * J = 1/2 <m_R - m_1, m_R - m_1> + 1/2 beta_v <v, A v> + [mass source] 1/2 beta_w <div v, (1-Lap) div v>:
    the last term is gamma/2 beta_w ||w||^2_{H1} of eq. (objective) with w = div v, exact after the
    elimination of w; it vanishes identically for w = 0;
  * the inner product that makes H self-adjoint is <a, b>_W = <K^{-1} a, b> for the mass-source
    model (H = K * Hessian of the penalised objective) and the plain L2 product otherwise.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .spectral import (Grid, Params, apply_A, apply_K, apply_Kinv, apply_precond, nyquist_project,
                       div, penalty_grad_w)
from . import stokes
from .transport import (state_forward, adjoint_backward, body_force, inc_state_forward,
                        inc_adjoint_backward_gn, inc_state_forward_stages, inc_adjoint_backward_full,
                        inc_body_force_full)


def objective_terms(g: Grid, p: Params, mT, mR, v, traj=None):
    """(J, [data, reg_v, reg_w], traj) at v (Nyquist-projected first)."""
    v = nyquist_project(g, v)
    if traj is None:
        traj = state_forward(g, p, mT, v)
    r = mR - traj.m[-1]
    data = 0.5 * g.inner(r, r)
    if p.norm == "stokes":
        reg_v = p.beta_v * stokes.value(g, p.nu, p.eps, v)
    else:
        reg_v = 0.5 * p.beta_v * g.inner(v, apply_A(g, p, v))
    reg_w = 0.0
    if p.constraint == "mass_source":
        dv = div(g, v)
        reg_w = 0.5 * p.beta_w * g.inner(dv, g.ifft((1.0 + g.ksq) * g.fft(dv)))
    return data + reg_v + reg_w, [data, reg_v, reg_w], traj


def objective(g: Grid, p: Params, mT, mR, v):
    J, terms, _ = objective_terms(g, p, mT, mR, v)
    return J, terms


class Linearization:
    """Everything the GN matvec needs at a linearisation point v: the state trajectory (with the
    stored gradients G_j, G*_j), plus J and g at v."""

    def __init__(self, v, traj, lam, lam_star, b, g, J, terms, p=None):
        self.v, self.traj, self.lam, self.lam_star = v, traj, lam, lam_star
        self.b, self.g, self.J, self.terms = b, g, J, terms
        self.p = p   # the parameters at this point (with eta_bar for the shear-control mass-source K)


def gradient(g: Grid, p: Params, mT, mR, v) -> Linearization:
    """Reduced gradient g = F_Nyq[beta_v A v + K b], b = int lam grad m dt (eq. (control-eq-elim)).

    State forward (eq. (state-eq-elim)), adjoint backward from lam(1) = m_R - m(1)
    (eq. (init-adj-eq-elim)), body-force quadrature, then the control equation.
    """
    v = nyquist_project(g, v)
    J, terms, traj = objective_terms(g, p, mT, mR, v)
    lam, lam_star = adjoint_backward(g, p, v, mR - traj.m[-1])
    b = body_force(p, traj, lam, lam_star)
    if p.norm == "stokes":   # K (the Leray projection, I, or K_v with a mass source) of grad J_pen
        p = at_point(g, p, v)
        gr = nyquist_project(g, apply_K(g, p, p.beta_v * stokes.first_variation(g, p.nu, p.eps, v) + b
                                        + penalty_grad_w(g, p, v)))
    else:
        gr = nyquist_project(g, p.beta_v * apply_A(g, p, v) + apply_K(g, p, b))
    return Linearization(v, traj, lam, lam_star, b, gr, J, terms, p)


def at_point(g: Grid, p: Params, v):
    """Parameters with the mean viscosity of v (used by K_v of the shear-control model with a mass
    source; unchanged otherwise)."""
    if p.norm == "stokes" and p.constraint == "mass_source":
        return replace(p, eta_bar=stokes.mean_viscosity(g, p.nu, p.eps, v))
    return p


def hessian_matvec(g: Grid, p: Params, lin: Linearization, vt):
    """Gauss-Newton reduced Hessian matvec H v~ = F_Nyq[beta_v A v~ + K b~] (eq. (inc-control-eq-elim)).

    One incremental state solve forward (eq. (inc-state-eq-elim)) and one GN incremental adjoint solve
    backward (eq. (inc-adj-eq-elim) without div(lam v~)), then the incremental body force b~.
    """
    vt = nyquist_project(g, vt)
    mt1 = inc_state_forward(g, p, lin.v, lin.traj, vt)
    bt = inc_adjoint_backward_gn(g, p, lin.v, lin.traj, mt1)
    return _assemble(g, p, lin, vt, bt)


def _assemble(g: Grid, p: Params, lin, vt, bt):
    """F_Nyq[beta_v B v~ + K b~] (quadratic seminorms: B = A) or F_Nyq K[beta_v B(v)[v~] + b~]
    (shear-control model)."""
    if p.norm == "stokes":
        p = lin.p if lin.p is not None else at_point(g, p, lin.v)
        return nyquist_project(g, apply_K(g, p, p.beta_v * stokes.second_variation(g, p.nu, p.eps, lin.v, vt) + bt
                                          + penalty_grad_w(g, p, vt)))
    return nyquist_project(g, p.beta_v * apply_A(g, p, vt) + apply_K(g, p, bt))


def hessian_matvec_full(g: Grid, p: Params, lin: Linearization, vt):
    """Full-Newton reduced Hessian matvec (an extension of the paper's Gauss-Newton step): eq.
    (inc-control-eq-elim) with every lam term of eqs. (inc-adj-eq-elim) and the incremental body force
    kept, H v~ = F_Nyq[beta_v A v~ + K b~], b~ = int lam~ grad m + lam grad m~ dt.  Implemented as the
    exact derivative of the 'dto' discrete gradient, so it is the Hessian of the discrete objective
    (symmetric in <., .>_W, possibly indefinite away from a minimiser)."""
    if p.adjoint != "dto":
        raise ValueError("the full-Newton Hessian is defined for the 'dto' discretisation")
    vt = nyquist_project(g, vt)
    mt, mts = inc_state_forward_stages(g, p, lin.v, lin.traj, vt)
    lt, lts = inc_adjoint_backward_full(g, p, lin.v, vt, lin.lam, lin.lam_star, mt[-1])
    bt = inc_body_force_full(g, p, lin.traj, lin.lam, lin.lam_star, mt, mts, lt, lts)
    return _assemble(g, p, lin, vt, bt)


def precond(g: Grid, p: Params, r):
    """z = (beta_v A)^{-1} r with the modified kernel (App. E.2)."""
    return apply_precond(g, p, r)


def w_inner(g: Grid, p: Params, a, b):
    """<a, b>_W: <K^{-1} a, b> for the mass-source model, <a, b> otherwise."""
    if p.constraint == "mass_source":
        return g.inner(apply_Kinv(g, p, a), b)
    return g.inner(a, b)


def directional_derivative(g: Grid, p: Params, gr, d):
    """dJ(v)[d] = <grad_v J_pen, d> = <K^{-1} g, d> for the mass-source model and <g, d> otherwise
    (d admissible)."""
    return w_inner(g, p, gr, d)


def penalised_gradient(g: Grid, p: Params, lin: Linearization):
    """grad J_pen = b + beta_v A v + beta_w(-grad (1-Lap) div v) (without the projection K)."""
    return lin.b + p.beta_v * apply_A(g, p, lin.v) + penalty_grad_w(g, p, lin.v)
