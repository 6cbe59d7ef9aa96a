"""PCG inner iteration, Armijo backtracking and the outer Gauss-Newton-Krylov loop
(oracle; test infrastructure only).

Paper: Sec. 4, eq. (reduced-space-kkt-system) (H_k v~_k = -g_k, v_{k+1} = v_k + alpha_k v~_k);
App. E.1, Alg. 1 (outer iteration, v_0 = 0) and Alg. 2 (PCG Newton step with forcing term
eta_k = min(0.5, (||g_k|| / ||g_0||)^{1/2})); Sec. 4 (backtracking line search subject to the Armijo
condition with default parameters, Nocedal & Wright Alg. 3.1).

Readings (listed in the design notes):
  * PCG stops when ||r_{l+1}|| <= eta_k ||r_0|| (relative test of the cited inexact-Newton forcing);
    Alg. 2 applies H to the search direction s_l; ``fixed_pcg_iters`` runs exactly that many steps;
  * the PCG inner product is <.,.>_W (the plain L2 product unless the mass-source model is used);
  * if <s, H s>_W <= 0 PCG stops (on its first step it returns the preconditioned steepest-descent
    direction);
  * Armijo: alpha_0 = 1, rho = 1/2, c_1 = 1e-4, at most ``max_backtracks`` halvings; slope = dJ[v~];
  * the relative gradient is ||g(v_k)|| / ||g(0)||, with g(0) taken at v = 0 even for a warm start.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

from .spectral import Grid, Params
from . import reduced

OK, ENOTCONV, ENONFINITE = 0, -4, -5


@dataclass
class SolveOpts:
    max_newton: int = 50
    max_pcg: int = 100
    fixed_pcg_iters: int = 0
    max_backtracks: int = 10
    gtol_rel: float = 1e-2
    armijo_c1: float = 1e-4
    armijo_rho: float = 0.5
    v0: np.ndarray | None = None


@dataclass
class SolveStats:
    newton_iters: int = 0
    pcg_iters: int = 0
    n_matvec: int = 0
    n_pde: int = 0
    backtracks: int = 0
    status: int = OK
    g0_norm: float = 0.0
    g_rel: float = 1.0
    J: float = 0.0
    history: list = field(default_factory=list)


def pcg(matvec, prec, winner, norm, rhs, eta, max_pcg, fixed_iters=0):
    """Alg. 2: preconditioned CG on H x = rhs (rhs = -g_k), x_0 = 0.

    Returns (x, iterations, ||r|| / ||r_0||).  ``winner`` is the inner product that makes H and the
    preconditioner self-adjoint; ``norm`` is the residual norm of the stopping test.
    """
    x = np.zeros_like(rhs)
    r = rhs.copy()
    z = prec(r)
    s = z.copy()
    rz = winner(r, z)
    r0 = norm(r)
    nit = fixed_iters if fixed_iters > 0 else max_pcg
    l = 0
    rn = r0
    while l < nit:
        st = matvec(s)
        sHs = winner(s, st)
        l += 1
        if not sHs > 0.0:
            if l == 1:
                x = s.copy()
            break
        kappa = rz / sHs
        x = x + kappa * s
        r = r - kappa * st
        rn = norm(r)
        if fixed_iters == 0 and rn <= eta * r0:
            break
        z = prec(r)
        rz_new = winner(r, z)
        mu = rz_new / rz
        rz = rz_new
        s = z + mu * s
    return x, l, (rn / r0 if r0 > 0 else 0.0)


def solve(g: Grid, p: Params, mT, mR, opts: SolveOpts):
    """Alg. 1: inexact reduced-space Gauss-Newton-Krylov with Armijo line search.

    Returns (v, stats).
    """
    st = SolveStats()
    lin0 = reduced.gradient(g, p, mT, mR, np.zeros((2, p.n1, p.n2)))
    st.n_pde += 2
    g0 = g.norm(lin0.g)
    st.g0_norm = g0
    if opts.v0 is not None:
        lin = reduced.gradient(g, p, mT, mR, opts.v0)
        st.n_pde += 2
    else:
        lin = lin0
    v = lin.v
    k = 0
    while True:
        grel = g.norm(lin.g) / g0 if g0 > 0 else 0.0
        st.g_rel, st.J = grel, lin.J
        if not np.isfinite(grel) or not np.isfinite(lin.J):
            st.status = ENONFINITE
            break
        if grel <= opts.gtol_rel or k >= opts.max_newton:
            break
        eta = min(0.5, math.sqrt(grel))

        def mv(s, _lin=lin):
            st.n_matvec += 1
            st.n_pde += 2
            return reduced.hessian_matvec(g, p, _lin, s)

        vt, its, relres = pcg(mv, lambda r: reduced.precond(g, p, r),
                      lambda a, b: reduced.w_inner(g, p, a, b), g.norm,
                      -lin.g, eta, opts.max_pcg, opts.fixed_pcg_iters)
        st.pcg_iters += its
        slope = reduced.directional_derivative(g, p, lin.g, vt)
        alpha = 1.0
        accepted = False
        nbt = 0
        if slope < 0.0:
            for nbt in range(opts.max_backtracks + 1):
                Jt, _ = reduced.objective(g, p, mT, mR, v + alpha * vt)
                st.n_pde += 1
                if Jt <= lin.J + opts.armijo_c1 * alpha * slope:
                    accepted = True
                    break
                alpha *= opts.armijo_rho
        st.backtracks += nbt
        st.history.append(dict(k=k, J=lin.J, g_rel=grel, pcg=its, eta=eta, pcg_relres=relres,
                               alpha=alpha if accepted else 0.0, slope=slope))
        if not accepted:
            st.status = ENOTCONV
            break
        v = v + alpha * vt
        lin = reduced.gradient(g, p, mT, mR, v)
        st.n_pde += 2
        k += 1
    st.newton_iters = k
    return lin.v, st
