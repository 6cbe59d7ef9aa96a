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
  * the relative gradient is ||g(v_k)|| / ||g(0)||, with g(0) taken at v = 0 even for a warm start;
  * ``hessian="full"`` replaces the Gauss-Newton matvec by the exact Hessian of the discrete objective
    (an extension); where it is not positive along a search direction PCG stops as above;
  * a warm start is kept only if J(v_0) < J(0) (the globalisation needs descent from the plain
    start), otherwise the solve starts from v = 0;
  * optional low-rank correction of the preconditioner (not in the paper): a deflation set of
    directions z_i with H z_i and e_i > 0 feeds the balancing (deflation) preconditioner
    (``corrected_precond``), which stays SPD for any such set.  The set starts with the
    Rayleigh-Ritz pairs (theta_i, z_i) of the GN Hessian on span(U) relative to M (z_i orthonormal
    in <., M .>_W, M = beta_v A with the modified kernel, e_i = theta_i), computed at the point
    where the first Newton step is taken, for caller directions U; with ``recycle`` = q > 0 the
    first q search directions of every PCG solve (with H s and e = <s, H s>_W, mutually
    H-conjugate within that solve) are appended, until ``lowrank_capacity`` directions are held.
    The plain spectral form M^{-1} + sum (1/theta - 1) z z^* was tried first and made PCG slower
    whenever span(U) is not an invariant subspace.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

from .spectral import Grid, Params
from . import reduced, spectral

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
    precond_U: np.ndarray | None = None   # (r, 2, n1, n2) directions of the low-rank correction
    recycle: int = 0                      # PCG directions of each Newton step kept for the next ones
    hessian: str = "gn"                   # "gn" (the paper's Gauss-Newton) or "full" (exact Hessian)
    lowrank_capacity: int = 16            # most directions the correction holds
    cfl_max: float = 0.0                  # > 0: n_t adapted to keep the CFL number of the iterate below
    nt_max: int = 0                       # largest n_t the adaptation may reach (0: p.nt)


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
    fallback_used: int = 0
    lowrank_dim: int = 0                  # directions in the correction at the end of the solve
    cfl: float = 0.0                      # CFL number of the final velocity (``cfl_number``), final n_t
    nt: int = 0                           # n_t at the end (raised by the CFL adaptation)
    nt_changes: int = 0
    lowrank: tuple | None = None          # (Ritz values theta, Ritz vectors z) from precond_U
    history: list = field(default_factory=list)


def pcg(matvec, prec, winner, norm, rhs, eta, max_pcg, fixed_iters=0, record=None, record_max=0):
    """Alg. 2: preconditioned CG on H x = rhs (rhs = -g_k), x_0 = 0.

    Returns (x, iterations, ||r|| / ||r_0||).  ``winner`` is the inner product that makes H and the
    preconditioner self-adjoint; ``norm`` is the residual norm of the stopping test.  If ``record`` is
    a list, the first ``record_max`` search directions that complete a step are appended to it as
    (s, H s, <s, H s>_W).
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
        if record is not None and l <= record_max:
            record.append((s.copy(), st.copy(), sHs))
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


def cfl_number(g: Grid, p: Params, v):
    """C(v) = h_t (max|v_1| n1/2 + max|v_2| n2/2): the largest |h_t k . v| over the resolved modes, the
    quantity the explicit RK2 step has to keep below about one (Sec. 4 monitors the CFL condition)."""
    v = spectral.nyquist_project(g, v)
    return (np.abs(v[0]).max() * (g.n1 / 2) + np.abs(v[1]).max() * (g.n2 / 2)) / p.nt


def admissible(g: Grid, p: Params, u):
    """A direction in the space PCG works in: Nyquist-free, and Leray-projected (K) for w = 0."""
    u = spectral.nyquist_project(g, u)
    return spectral.apply_K(g, p, u) if p.constraint == "divfree" else u


def precond_op(g: Grid, p: Params, u):
    """M u = F_Nyq (beta_v A with the modified kernel) u, the operator whose inverse PCG applies."""
    sym = spectral.precond_symbol(g, p)
    return np.stack([g.ifft(g.keep * sym * g.fft(u[c])) for c in range(2)])


def lowrank_setup(g: Grid, p: Params, matvec, U, rel_tol=1e-10):
    """Rayleigh-Ritz on span(U): returns (theta, Z, HZ) with Z^T W M Z = I, Z^T W H Z = diag(theta)
    and HZ = H Z.

    Directions are made admissible, then orthonormalised in <., M .>_W through the eigenvectors of
    their Gram matrix (directions whose Gram eigenvalue is at most rel_tol times the largest are
    dropped); H is applied to the orthonormal basis, the projected Hessian is diagonalised, and
    Ritz pairs with non-positive (or non-finite) theta are dropped, so that E = Z^T W H Z is SPD."""
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731
    U = [admissible(g, p, u) for u in U]
    r = len(U)
    if r == 0:
        return np.zeros(0), [], []
    MU = [precond_op(g, p, u) for u in U]
    G = np.array([[W(U[i], MU[j]) for j in range(r)] for i in range(r)])
    G = 0.5 * (G + G.T)
    lam, E = np.linalg.eigh(G)
    keep = lam > rel_tol * max(lam.max(), 0.0)
    if not keep.any():
        return np.zeros(0), [], []
    C = E[:, keep] / np.sqrt(lam[keep])                       # Q = U C is M-orthonormal
    Q = [sum(C[j, i] * U[j] for j in range(r)) for i in range(C.shape[1])]
    HQ = [matvec(q) for q in Q]
    T = np.array([[W(Q[i], HQ[j]) for j in range(len(Q))] for i in range(len(Q))])
    T = 0.5 * (T + T.T)
    theta, V = np.linalg.eigh(T)
    ok = np.isfinite(theta) & (theta > 0.0)
    theta, V = theta[ok], V[:, ok]
    Z = [sum(V[j, i] * Q[j] for j in range(len(Q))) for i in range(V.shape[1])]
    HZ = [sum(V[j, i] * HQ[j] for j in range(len(Q))) for i in range(V.shape[1])]
    return theta, Z, HZ


def ritz_directions(g: Grid, p: Params, matvec, U, iters: int):
    """Leading generalised eigenpairs of (H, M) by subspace iteration (an extension: the targets of
    the learned low-rank correction).  Rayleigh-Ritz on span(U) (``lowrank_setup``), then
    U <- M^{-1} H Z with the preconditioner PCG applies, repeated ``iters`` times; each step damps
    the components along eigenvectors with smaller theta by their ratio to the kept ones.  Returns
    (theta, Z) with theta descending and Z orthonormal in <., M .>_W."""
    theta, Z, HZ = lowrank_setup(g, p, matvec, U)
    for _ in range(iters):
        U = [reduced.precond(g, p, hz) for hz in HZ]
        theta, Z, HZ = lowrank_setup(g, p, matvec, U)
    order = np.argsort(-theta, kind="stable")
    return theta[order], [Z[i] for i in order]


def corrected_precond(g: Grid, p: Params, theta, Z, HZ):
    """Balancing (deflation) correction of M^{-1} on span(Z), with E = Z^T W H Z = diag(theta):

        P r = Pi M^{-1} Pi^* r + Z E^{-1} Z^* r,   Pi = I - Z E^{-1} (H Z)^*,

    adjoints taken in <., .>_W.  P H is the identity on span(Z); P is SPD whenever M and E are (also
    when H has moved on from the point where HZ was taken)."""
    W = lambda a, b: reduced.w_inner(g, p, a, b)   # noqa: E731

    def prec(r):
        a = [W(zi, r) / th for zi, th in zip(Z, theta)]
        rt = r - sum((ai * hz for ai, hz in zip(a, HZ)), np.zeros_like(r))
        y = reduced.precond(g, p, rt)
        b = [W(hz, y) / th for hz, th in zip(HZ, theta)]
        return y + sum(((ai - bi) * zi for ai, bi, zi in zip(a, b, Z)), np.zeros_like(r))
    return prec


def adapt_nt(g: Grid, p: Params, v, cfl_max: float, nt_max: int):
    """Sec. 4 adapts the number of time steps by monitoring the CFL condition (Sec. 5 starts from
    n_t = 2 max(n)).  Reading: when C(v) > cfl_max at the current n_t, n_t becomes the smallest value
    with C(v) <= cfl_max, at most max(p.nt, nt_max); n_t never decreases.  Returns (params, changed)."""
    if not cfl_max > 0:
        return p, False
    c = cfl_number(g, p, v)
    cap = max(p.nt, nt_max)
    if c <= cfl_max or p.nt >= cap:
        return p, False
    nt_new = min(cap, math.ceil(p.nt * (c / cfl_max) - 1e-9))
    if nt_new <= p.nt:
        return p, False
    return replace(p, nt=nt_new), True


def solve(g: Grid, p: Params, mT, mR, opts: SolveOpts):
    """Alg. 1: inexact reduced-space Gauss-Newton-Krylov with Armijo line search.

    Returns (v, stats).  With opts.cfl_max > 0 the number of time steps follows ``adapt_nt`` before the
    first Newton step and after every accepted one; the problem is then linearised again at the same
    v (J and g depend on n_t; g(0) does not).
    """
    st = SolveStats()
    lin0 = reduced.gradient(g, p, mT, mR, np.zeros((2, p.n1, p.n2)))
    st.n_pde += 2
    g0 = g.norm(lin0.g)
    st.g0_norm = g0
    lin = lin0
    if opts.v0 is not None:
        lin_ws = reduced.gradient(g, p, mT, mR, opts.v0)
        st.n_pde += 2
        if np.isfinite(lin_ws.J) and lin_ws.J < lin0.J:
            lin = lin_ws
        else:
            st.fallback_used = 1
    v = lin.v
    p, changed = adapt_nt(g, p, v, opts.cfl_max, opts.nt_max)
    if changed:
        st.nt_changes += 1
        lin = reduced.gradient(g, p, mT, mR, v)
        st.n_pde += 2
    if opts.hessian not in ("gn", "full"):
        raise ValueError("hessian must be 'gn' or 'full'")
    hess = reduced.hessian_matvec_full if opts.hessian == "full" else reduced.hessian_matvec
    if p.norm == "stokes" and p.constraint == "mass_source" and (opts.recycle > 0 or opts.precond_U is not None):
        # the W-product of this model moves with the point (K_v); a stored correction would be stale
        raise ValueError("no preconditioner correction for the shear-control model with a mass source")
    # deflation set of the preconditioner correction: directions z, H z and e = <z, H z>_W
    E, Zs, HZs = [], [], []
    cap = opts.lowrank_capacity
    if opts.precond_U is not None and len(opts.precond_U) > 0:
        if len(opts.precond_U) > cap:
            raise ValueError("more directions than the correction holds")

        def mv0(s, _lin=lin):
            st.n_matvec += 1
            st.n_pde += 2
            return hess(g, p, _lin, s)
        theta, Z, HZ = lowrank_setup(g, lin.p or p, mv0, list(opts.precond_U))
        st.lowrank = (theta, Z)
        E, Zs, HZs = list(theta), list(Z), list(HZ)
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
            return hess(g, p, _lin, s)

        if Zs:
            prec = corrected_precond(g, lin.p or p, E, Zs, HZs)
        else:
            prec = lambda r: reduced.precond(g, p, r)   # noqa: E731
        rec = []
        vt, its, relres = pcg(mv, prec,
                      lambda a, b: reduced.w_inner(g, lin.p or p, a, b), g.norm,
                      -lin.g, eta, opts.max_pcg, opts.fixed_pcg_iters,
                      record=rec, record_max=min(opts.recycle, cap - len(Zs)))
        for s_, hs_, e_ in rec:
            Zs.append(s_)
            HZs.append(hs_)
            E.append(e_)
        st.pcg_iters += its
        slope = reduced.directional_derivative(g, lin.p or p, lin.g, vt)
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
                               alpha=alpha if accepted else 0.0, slope=slope, backtracks=nbt,
                               v=v.copy(), step=vt.copy(), nt=p.nt))
        if not accepted:
            st.status = ENOTCONV
            break
        v = v + alpha * vt
        p, changed = adapt_nt(g, p, v, opts.cfl_max, opts.nt_max)
        st.nt_changes += int(changed)
        lin = reduced.gradient(g, p, mT, mR, v)
        st.n_pde += 2
        k += 1
    st.newton_iters = k
    st.lowrank_dim = len(Zs)
    st.cfl = cfl_number(g, p, lin.v)
    st.nt = p.nt
    return lin.v, st
