"""Deformation diagnostics of a stationary velocity: displacement, deformation gradient and its
determinant (oracle; test infrastructure only).

Paper: appendix "Illustration of Deformation Map": eq. (displacement), the displacement u with
u(0) = 0 transported by v with source v (the Eulerian map is y = x - u_1), and eq. (def-grad), the
deformation gradient F with F(0) = I transported by v with source (grad v) F, i.e.
dF_ik/dt + v . grad F_ik = sum_l (d_l v_i) F_lk; det F_1 is reported as the local volume change.

Readings (listed in the design notes): both equations are integrated with the same explicit RK2
(Heun) and the same n_t as the state equation, with spectral derivatives whose Nyquist wavenumber is
zeroed, for the Nyquist-projected velocity.
"""
from __future__ import annotations

import numpy as np

from .spectral import Grid, Params, d, nyquist_project


def _rhs(g: Grid, v, dv, u, F):
    """Right-hand sides: du_i = -v . grad u_i + v_i, dF_ik = -v . grad F_ik + sum_l dv[i, l] F_lk."""
    adv = lambda q: -(v[0] * d(g, q, 0) + v[1] * d(g, q, 1))   # noqa: E731
    du = np.stack([adv(u[i]) + v[i] for i in range(2)])
    dF = np.empty_like(F)
    for i in range(2):
        for k in range(2):
            dF[i, k] = adv(F[i, k]) + dv[i, 0] * F[0, k] + dv[i, 1] * F[1, k]
    return du, dF


def deformation(g: Grid, p: Params, v):
    """(u_1, F_1) after n_t Heun steps on [0, 1]; u_1 is (2, n1, n2), F_1 is (2, 2, n1, n2) with
    F_1[i, k] = F_ik."""
    v = nyquist_project(g, v)
    dv = np.stack([np.stack([d(g, v[i], l) for l in range(2)]) for i in range(2)])   # dv[i, l] = d_l v_i
    h = 1.0 / p.nt
    u = np.zeros((2, g.n1, g.n2))
    F = np.zeros((2, 2, g.n1, g.n2))
    F[0, 0] = 1.0
    F[1, 1] = 1.0
    for _ in range(p.nt):
        ku, kF = _rhs(g, v, dv, u, F)
        us, Fs = u + h * ku, F + h * kF
        ku2, kF2 = _rhs(g, v, dv, us, Fs)
        u = u + 0.5 * h * (ku + ku2)
        F = F + 0.5 * h * (kF + kF2)
    return u, F


def det2(F):
    """det F = F_11 F_22 - F_12 F_21 pointwise."""
    return F[0, 0] * F[1, 1] - F[0, 1] * F[1, 0]


def summary(detF):
    """(min, max, mean) of det F_1 over the grid."""
    return float(detF.min()), float(detF.max()), float(detF.mean())
