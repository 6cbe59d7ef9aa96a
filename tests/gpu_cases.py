"""Seeded parity cases shared by the GPU tests: inputs from ``synthdata``, expected values from the
oracle (computed on the host), results from the HIP library through its C ABI."""
from __future__ import annotations

from dataclasses import dataclass
import functools

import numpy as np

import synthdata as sd
from oracle import Grid, Params, reduced, transport


@dataclass(frozen=True)
class Case:
    n1: int
    n2: int
    nt: int
    norm: str
    constraint: str
    beta_v: float
    beta_w: float
    precision: str
    adjoint: str = "dto"
    seed: int = 0
    config: int = 0          # 1..5: the seeded workload of that configuration (full size)
    ktex: int = 8
    vmax: float = 0.0        # > 0: scale v* to this max |v| instead of CFL 0.8 (nt chosen to keep CFL < 1)
    nu: float = 1.0          # shear-control model (norm "stokes"): exponent and strain regularisation
    stokes_eps: float = 1e-6

    @property
    def tol(self):
        # FP64 transport: round-off of O(10^2..10^3) FFT passes; FP32 transport: the per-matvec bound
        return 1e-10 if self.precision == "fp64" else 1e-5

    @property
    def eps(self):
        return 2.2e-16 if self.precision == "fp64" else 1.2e-7


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def elem(a, b):
    """Largest pointwise error relative to the largest reference value."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if b.size else 0.0


# A localised error (one wrong tile of a large field) can hide in a relative L2 norm, so every parity
# check also bounds the pointwise error: max|a - b| <= ELEM_FACTOR * tol * max|b|.
ELEM_FACTOR = 10.0


class Close:
    """Outcome of a parity comparison; true when both bounds hold, printed with the measured errors."""

    def __init__(self, r, e, tol):
        self.r, self.e, self.tol = r, e, tol

    def __bool__(self):
        return bool(self.r < self.tol and self.e <= ELEM_FACTOR * self.tol)

    def __repr__(self):
        return f"Close(rel_l2={self.r:.3e}, pointwise={self.e:.3e}, tol={self.tol:.1e})"


def close(a, b, tol):
    """rel-L2 below tol and the pointwise error below ELEM_FACTOR * tol of the reference's maximum."""
    return Close(rel(a, b), elem(a, b), tol)


@functools.lru_cache(maxsize=None)
def inputs(case: Case):
    """(mT, mR, v_lin, vtilde, v_trial) for a case; mR is the oracle's transport of mT by v*."""
    if case.config:
        w = sd.make_workload(case.config)
        mT, vs, vt = w.mT, w.vstar, w.vtilde
    else:
        rng = np.random.Generator(np.random.PCG64(sd.BASE_SEED + 77 + case.seed))
        nmin = min(case.n1, case.n2)
        if nmin >= 32:
            mT = sd.template_image(case.n1, case.n2, 6, min(case.ktex, nmin // 4), rng)
        else:   # blobs would be under-resolved on a short axis: band-limited texture only
            mT = sd.minmax01(sd.texture(case.n1, case.n2, max(1, nmin // 4), rng))
        kv = max(1, min(4, case.n1 // 2 - 1, case.n2 // 2 - 1))
        vs = sd.random_velocity(case.n1, case.n2, kv, rng, divfree=True,
                                compressible=case.constraint != "divfree")
        vs = sd.scale_to_max(vs, case.vmax) if case.vmax > 0 else sd.scale_to_cfl(vs, case.nt, 0.8)
        vt = sd.unit_l2(sd.random_velocity(case.n1, case.n2, kv, rng, divfree=True,
                                           compressible=case.constraint != "divfree"))
    p = params(case)
    g = Grid(case.n1, case.n2)
    mR = transport.state_forward(g, p, mT, vs).m[-1]
    return mT, mR, 0.5 * vs, vt, 0.7 * vs


def params(case: Case) -> Params:
    return Params(case.n1, case.n2, case.nt, case.norm, case.constraint, case.beta_v, case.beta_w, case.adjoint,
                  nu=case.nu, eps=case.stokes_eps)


@functools.lru_cache(maxsize=None)
def oracle_results(case: Case):
    mT, mR, vlin, vt, vtr = inputs(case)
    p = params(case)
    g = Grid(case.n1, case.n2)
    lin = reduced.gradient(g, p, mT, mR, vlin)
    H = reduced.hessian_matvec(g, p, lin, vt)
    Jt, terms = reduced.objective(g, p, mT, mR, vtr)
    m1 = transport.state_forward(g, p, mT, reduced.nyquist_project(g, vtr)).m[-1]
    z = reduced.precond(g, p, lin.g)
    # Size the body force would have for an O(1) misfit: the gradient and the data term are formed
    # from m_R - m_1, so rounding of m_1 (a few eps |m| per step) enters them with this weight even
    # when the misfit itself is small.
    from oracle import spectral
    bscale = float(np.linalg.norm(mT * spectral.grad(g, mT)))
    Jscale = float(g.norm(mR - lin.traj.m[-1]) * g.norm(mT)) + float(g.norm(mR - m1) * g.norm(mT))
    # Conditioning floor: both paths Nyquist-project their FP64 input with an FFT round trip, which
    # leaves white round-off of size eps64 |v|; beta_v A^ (up to beta_v (n/2)^4 for H2) amplifies it.
    # Measured here as the oracle's own response to such noise.
    rng = np.random.default_rng(1234)
    H_n = reduced.hessian_matvec(g, p, lin, vt + 2.2e-16 * np.abs(vt).max() * rng.standard_normal(vt.shape))
    g_n = reduced.gradient(g, p, mT, mR, vlin + 2.2e-16 * np.abs(vlin).max() * rng.standard_normal(vlin.shape)).g
    return dict(g=lin.g, J=lin.J, H=H, Jt=Jt, terms=terms, m1=m1, z=z, bscale=bscale, Jscale=Jscale,
                sens_H=rel(H_n, H), sens_g=float(np.linalg.norm(g_n - lin.g)))


@functools.lru_cache(maxsize=None)
def tight_solution(case: Case, gtol: float):
    """The oracle's Alg. 1 solve of a case to ||g||/||g(0)|| <= gtol: the converged velocity that
    run-to-tolerance GPU solves (plain, recycled, full Newton, batched) are compared with."""
    from oracle import solver
    mT, mR, *_ = inputs(case)
    return solver.solve(Grid(case.n1, case.n2), params(case), mT, mR,
                        solver.SolveOpts(max_newton=50, max_pcg=300, gtol_rel=gtol))


def gpu_problem(case: Case, lowrank_capacity=0, hessian="gn"):
    import torch
    from paper_1503_00757_amd import Problem
    mT, mR, *_ = inputs(case)
    dev = torch.device("cuda:0")
    return Problem(torch.tensor(mT, device=dev), torch.tensor(mR, device=dev), case.nt, case.norm,
                   case.constraint, case.beta_v, case.beta_w, case.precision, case.adjoint,
                   lowrank_capacity=lowrank_capacity, hessian=hessian, nu=case.nu, eps=case.stokes_eps)


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def host(t):
    return t.detach().cpu().numpy()
