"""Pseudospectral operators on the periodic grid (oracle; test infrastructure only).

Paper: Sec. 4 (pseudospectral Fourier discretisation in space); Sec. 2, eqs. (reg-v), (reg-w)
(H1/H2 seminorms of v, H1 norm of the mass source w); Sec. 3.1, eq. (var-reg-v) (A = -Lap or Lap^2);
Sec. 3.3, eq. (project-body-force) (the projection K and the operator M); App. E.2 (preconditioner
(beta_v A)^{-1} with its kernel modified so it is invertible).

Readings where the paper is silent (listed in the design notes):
  * domain [0, 2pi)^2 with nodes 2 pi i/n (equivalent to (-pi, pi)^2 under periodicity);
  * wavenumbers are integers; every operator uses k~ = k with the Nyquist wavenumber set to 0,
    and velocity-like inputs/outputs have their Nyquist row and column projected out (F_Nyq);
  * K for H2 with a mass source: M^ = 1 + beta_v A^ / (beta_w |k|^2 (|k|^2 + 1)), obtained by redoing
    the elimination of App. A.1 with A = Lap^2; it reduces to the printed M for A = -Lap;
  * the preconditioner symbol is beta_v A^ where A^ > 0 and beta_v on the kernel (k = 0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

NORMS = ("H1", "H2", "H3", "stokes")
CONSTRAINTS = ("none", "divfree", "mass_source")
ADJOINT_MODES = ("dto", "paper")


@dataclass(frozen=True)
class Params:
    """Problem parameters.

    norm        'H1' or 'H2' seminorm on v (eq. (reg-v)); 'H3' (triharmonic A) is the variant the paper
                names with the Stokes model; 'stokes' is the nonlinear shear-control model of eq.
                (shear-control-reg-v) with exponent nu and strain regularisation eps (oracle/stokes.py)
    constraint  'none'        gamma = 0 (no constraint on div v)
                'divfree'     gamma = 1, w = 0 (incompressible)
                'mass_source' gamma = 1, beta_w > 0 (near-incompressible, eq. (reg-w))
    adjoint     'dto'   time quadrature that is the exact transpose of the discrete forward map
                'paper' trapezoidal rule in time, as printed in Sec. 4
    """
    n1: int
    n2: int
    nt: int
    norm: str = "H1"
    constraint: str = "divfree"
    beta_v: float = 1e-2
    beta_w: float = 0.0
    adjoint: str = "dto"
    nu: float = 1.0
    eps: float = 1e-6
    eta_bar: float = 0.0   # shear-control model with a mass source: mean viscosity at the point of K

    def __post_init__(self):
        if self.norm not in NORMS or self.constraint not in CONSTRAINTS or self.adjoint not in ADJOINT_MODES:
            raise ValueError("bad parameter choice")
        if self.n1 % 2 or self.n2 % 2 or self.n1 < 4 or self.n2 < 4 or self.nt < 1 or self.beta_v <= 0:
            raise ValueError("bad sizes or weights")
        if (self.constraint == "mass_source") != (self.beta_w > 0):
            raise ValueError("beta_w > 0 exactly when constraint == 'mass_source'")
        if self.norm == "stokes" and not (self.nu > 0 and self.eps > 0):
            raise ValueError("the shear-control model takes nu > 0 and eps > 0")


WORKERS = -1


def set_workers(w: int):
    """Number of threads scipy.fft may use (-1 = all cores)."""
    global WORKERS
    WORKERS = w


class Grid:
    """Periodic n1 x n2 grid on [0, 2pi)^2 with its integer wavenumbers (rfft2 layout)."""

    def __init__(self, n1: int, n2: int):
        self.n1, self.n2 = n1, n2
        self.h1, self.h2 = 2 * np.pi / n1, 2 * np.pi / n2
        k1 = np.fft.fftfreq(n1, d=1.0 / n1)               # 0..n1/2-1, -n1/2..-1
        k2 = np.fft.rfftfreq(n2, d=1.0 / n2)              # 0..n2/2
        self.nyq1 = np.zeros(n1, dtype=bool)
        self.nyq1[n1 // 2] = True
        self.nyq2 = np.zeros(k2.size, dtype=bool)
        self.nyq2[n2 // 2] = True
        k1t = k1.copy()
        k1t[n1 // 2] = 0.0
        k2t = k2.copy()
        k2t[n2 // 2] = 0.0
        self.k1 = k1t[:, None]                            # k~1, shape (n1, 1)
        self.k2 = k2t[None, :]                            # k~2, shape (1, n2/2+1)
        self.ksq = self.k1 ** 2 + self.k2 ** 2            # |k~|^2
        # F_Nyq keeps modes whose k1 and k2 are both below Nyquist.
        self.keep = (~self.nyq1)[:, None] & (~self.nyq2)[None, :]

    # ---- transforms ---------------------------------------------------------------------------
    def fft(self, u):
        return sfft.rfft2(u, workers=WORKERS)

    def ifft(self, uh):
        return sfft.irfft2(uh, s=(self.n1, self.n2), workers=WORKERS)

    # ---- inner product <a, b> = h1 h2 sum a.b (Sec. 4, trapezoidal rule on a periodic grid) ---
    def inner(self, a, b):
        return self.h1 * self.h2 * float(np.sum(a * b))

    def norm(self, a):
        return np.sqrt(self.inner(a, a))


def d(g: Grid, u, axis: int):
    """Spectral partial derivative d/dx_axis of a real field (Sec. 4): symbol i k~_axis."""
    k = g.k1 if axis == 0 else g.k2
    return g.ifft(1j * k * g.fft(u))


def grad(g: Grid, u):
    return np.stack([d(g, u, 0), d(g, u, 1)])


def div(g: Grid, w):
    return d(g, w[0], 0) + d(g, w[1], 1)


def nyquist_project(g: Grid, v):
    """F_Nyq: remove the Nyquist row and column from each component of a vector field."""
    out = np.empty_like(v)
    for c in range(v.shape[0]):
        out[c] = g.ifft(g.fft(v[c]) * g.keep)
    return out


# ---- Fourier symbols (all diagonal in k; K mixes the two vector components) -----------------

def A_symbol(g: Grid, p: Params):
    """First variation of the v-seminorm, eq. (var-reg-v): A = -Lap (H1) -> |k|^2, A = Lap^2 (H2) -> |k|^4;
    the H3 seminorm (triharmonic reduced gradient, App. A) gives A = -Lap^3 -> |k|^6.  For the
    shear-control model this is the vector Laplacian of its preconditioner (App. E.2); its own
    variations are not Fourier multipliers (oracle/stokes.py)."""
    return {"H1": g.ksq, "H2": g.ksq ** 2, "H3": g.ksq ** 3, "stokes": g.ksq}[p.norm]


def M_symbol(g: Grid, p: Params):
    """M of eq. (project-body-force) for the mass-source model, generalised to A (see module header).
    For the shear-control model with a mass source (App. A, nonlinear Stokes with a relaxed
    incompressibility constraint) M = 2 beta_v eta_bar (beta_w (-Lap + I))^{-1} + I with the mean
    viscosity eta_bar of the point where K is taken (p.eta_bar).

    Defined where |k~| > 0; returns +inf at k~ = 0 (where the projection part vanishes anyway).
    """
    with np.errstate(divide="ignore", invalid="ignore"):
        if p.norm == "stokes":
            m = 1.0 + 2.0 * p.beta_v * p.eta_bar / (p.beta_w * (g.ksq + 1.0))
        else:
            m = 1.0 + p.beta_v * A_symbol(g, p) / (p.beta_w * g.ksq * (g.ksq + 1.0))
    return np.where(g.ksq > 0, m, np.inf)


def projection_weight(g: Grid, p: Params):
    """Scalar c(k) with K(k) = I - c(k) k~ k~^T / |k~|^2 (c = 0 at k~ = 0).

    gamma = 0: c = 0 (K = I); w = 0: c = 1 (Leray projection, M = I); mass source: c = 1/M^.
    """
    if p.constraint == "none":
        return np.zeros_like(g.ksq)
    if p.constraint == "divfree":
        return np.where(g.ksq > 0, 1.0, 0.0)
    return np.where(g.ksq > 0, 1.0 / M_symbol(g, p), 0.0)


def _kk_over_ksq(g: Grid):
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(g.ksq > 0, 1.0 / g.ksq, 0.0)
    return g.k1 * g.k1 * inv, g.k1 * g.k2 * inv, g.k2 * g.k2 * inv


def apply_K(g: Grid, p: Params, b, c=None):
    """K[b] = b - grad M^{-1} Lap^{-1} div b  (eq. (project-body-force)), as a Fourier multiplier.

    In Fourier space -grad M^-1 Lap^-1 div acts as -(1/M^) k k^T / |k|^2.
    ``c`` overrides the weight c(k) (used for K^{-1}).
    """
    if c is None:
        c = projection_weight(g, p)
    b1, b2 = g.fft(b[0]), g.fft(b[1])
    p11, p12, p22 = _kk_over_ksq(g)
    o1 = b1 - c * (p11 * b1 + p12 * b2)
    o2 = b2 - c * (p12 * b1 + p22 * b2)
    return np.stack([g.ifft(o1), g.ifft(o2)])


def apply_Kinv(g: Grid, p: Params, b):
    """K^{-1} for the mass-source model: K = I - P/M^ has eigenvalues 1 and 1 - 1/M^ on the range of
    P = k k^T/|k|^2, so K^{-1} = I + P / (M^ - 1).  Only defined when beta_w > 0."""
    if p.constraint != "mass_source":
        raise ValueError("K is invertible only for the mass-source model")
    m = M_symbol(g, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(g.ksq > 0, -1.0 / (m - 1.0), 0.0)
    return apply_K(g, p, b, c=c)


def apply_A(g: Grid, p: Params, v):
    """A v componentwise (eq. (var-reg-v))."""
    a = A_symbol(g, p)
    return np.stack([g.ifft(a * g.fft(v[0])), g.ifft(a * g.fft(v[1]))])


def precond_symbol(g: Grid, p: Params):
    """beta_v A^ with the kernel of A replaced by 1 (App. E.2: the kernel is modified so that the
    preconditioner is invertible)."""
    a = A_symbol(g, p)
    return p.beta_v * np.where(a > 0, a, 1.0)


def apply_precond(g: Grid, p: Params, r):
    """z = F_Nyq (beta_v A)^{-1} r  (App. E.2: a diagonal scaling in Fourier space)."""
    s = precond_symbol(g, p)
    return np.stack([g.ifft(g.keep * g.fft(r[c]) / s) for c in range(2)])


def penalty_grad_w(g: Grid, p: Params, v):
    """Gradient of 1/2 beta_w <div v, (1 - Lap) div v>: -beta_w grad (1 - Lap) div v.

    This is the gamma * 1/2 beta_w ||w||^2_H1 term of eq. (objective) with w = div v
    (eq. (constraint-divv)), i.e. the mass-source penalty after w is eliminated.
    """
    if p.constraint != "mass_source":
        return np.zeros_like(v)
    dv = div(g, v)
    q = g.ifft((1.0 + g.ksq) * g.fft(dv))
    return -p.beta_w * grad(g, q)
