"""Nonlinear Stokes (shear-control) regularisation of the velocity (oracle; test infrastructure only).

Paper: Sec. 2, eq. (shear-control-reg-v): R(v) = 2nu/(nu+1) int (E:E)^{(1+nu)/(2nu)} with the strain
rate E = (grad v + grad v^T)/2; eq. (1st-var-reg-v-nls): first variation A[v] = -div(2 eta E) with the
effective viscosity eta = (E:E)^{(1-nu)/(2nu)}; eq. (2nd-var-reg-v-nls): second variation
B(v)[v~] = -div(2 eta (I + (1-nu)/nu E (x) E / E:E) E[v~]).  nu in (0, 1) thickens, nu > 1 thins under
shear; nu = 1 is the linear model (eta = 1).

Readings (listed in the design notes):
  * E:E is replaced by E:E + eps (eps > 0) everywhere, so that eta stays finite where the strain
    vanishes (for nu > 1 the exponent of eta is negative); R, A and B are the exact first and second
    variations of the regularised R;
  * the objective carries beta_v R(v), whose first variation beta_v A[v] is the regularisation term of
    the control equation; for nu = 1 and divergence-free v this is 1/2 beta_v |v|^2_{H1} (+ beta_v eps |Omega|);
  * with the incompressibility constraint the reduced gradient is the Leray projection of
    beta_v A[v] + b (the elimination of the pressure), and the Hessian that of beta_v B[v~] + b~;
  * with a mass source (relaxed incompressibility, App. A) the pressure elimination splits eta into
    its mean eta_bar and the rest eta_hat and gives K[b, v] = grad M^{-1} Lap^{-1} div(div(2 beta_v
    eta_hat E[v]) - b) + b with M = 2 beta_v eta_bar (beta_w(-Lap + I))^{-1} + I.  Since eta_bar is a
    constant, M is a Fourier multiplier, and -div(2 beta_v eta E[v]) + K[b, v] equals
    K_v[b + beta_v A[v] - beta_w grad (1 - Lap) div v] with K_v = I - grad M^{-1} Lap^{-1} div: the
    projection of the gradient of the penalised objective (data + beta_v R + 1/2 beta_w
    <div v, (1 - Lap) div v>), as for the quadratic seminorms.  The Hessian is K_v applied to beta_v
    B(v)[v~] + b~ + the penalty's Hessian, with eta_bar of the linearisation point; the PCG inner
    product is <K_v^{-1} ., .>;
  * the preconditioner is the inverse of beta_v times the vector Laplacian (App. E.2).
"""
from __future__ import annotations

import numpy as np

from .spectral import Grid, d


def strain(g: Grid, v):
    """(E11, E12, E22) of E = sym grad v with spectral derivatives."""
    return d(g, v[0], 0), 0.5 * (d(g, v[0], 1) + d(g, v[1], 0)), d(g, v[1], 1)


def _EE(E):
    e11, e12, e22 = E
    return e11 * e11 + 2.0 * e12 * e12 + e22 * e22


def value(g: Grid, nu: float, eps: float, v):
    """R(v) = 2nu/(nu+1) int (E:E + eps)^{(1+nu)/(2nu)} dx (trapezoidal rule on the periodic grid)."""
    p = (1.0 + nu) / (2.0 * nu)
    return 2.0 * nu / (nu + 1.0) * g.h1 * g.h2 * float(np.sum((_EE(strain(g, v)) + eps) ** p))


def viscosity(nu: float, eps: float, E):
    return (_EE(E) + eps) ** ((1.0 - nu) / (2.0 * nu))


def mean_viscosity(g: Grid, nu: float, eps: float, v):
    """eta_bar[v] = (1/#Omega) int eta[v]: the constant part of the decomposition eta = eta_hat + eta_bar
    that App. A uses to eliminate the pressure (the grid mean on the periodic grid)."""
    return float(np.mean(viscosity(nu, eps, strain(g, v))))


def _div_sym(g: Grid, s11, s12, s22):
    """div of a symmetric tensor field: (d1 s11 + d2 s12, d1 s12 + d2 s22)."""
    return np.stack([d(g, s11, 0) + d(g, s12, 1), d(g, s12, 0) + d(g, s22, 1)])


def first_variation(g: Grid, nu: float, eps: float, v):
    """A[v] = -div(2 eta E)."""
    E = strain(g, v)
    eta = viscosity(nu, eps, E)
    return -_div_sym(g, 2 * eta * E[0], 2 * eta * E[1], 2 * eta * E[2])


def second_variation(g: Grid, nu: float, eps: float, v, vt):
    """B(v)[v~] = -div(2 eta (E~ + (1-nu)/nu (E:E~)/(E:E + eps) E))."""
    E = strain(g, v)
    Et = strain(g, vt)
    eta = viscosity(nu, eps, E)
    c = (1.0 - nu) / nu * (E[0] * Et[0] + 2 * E[1] * Et[1] + E[2] * Et[2]) / (_EE(E) + eps)
    return -_div_sym(g, *(2 * eta * (Et[k] + c * E[k]) for k in range(3)))
