"""Convenience wrapper: one registration problem whose workspace and vectors live in torch tensors.

All arithmetic happens in the HIP library; this class allocates device memory through torch, passes
pointers and the current stream, and returns tensors.
"""
from __future__ import annotations

from . import ffi

_NORMS = {"H1": ffi.REG_H1, "H2": ffi.REG_H2, "H3": ffi.REG_H3, "stokes": ffi.REG_STOKES}
_CONS = {"none": ffi.REG_UNCONSTRAINED, "divfree": ffi.REG_DIVFREE, "mass_source": ffi.REG_MASS_SOURCE}
_PREC = {"fp64": ffi.REG_FP64, "fp32": ffi.REG_FP32_TRANSPORT}
_ADJ = {"dto": ffi.REG_ADJ_DISCRETE, "paper": ffi.REG_ADJ_PAPER}


_HESS = {"gn": ffi.REG_HESS_GN, "full": ffi.REG_HESS_FULL}


def make_params(n1, n2, nt, norm="H1", constraint="divfree", beta_v=1e-2, beta_w=0.0, precision="fp32",
                adjoint="dto", lowrank_capacity=0, hessian="gn", nu=1.0, eps=1e-6, nt_max=0) -> ffi.RegParams:
    """reg_params; nu and eps are the shear-control model's exponent and strain regularisation (used
    for norm="stokes" only); nt_max is the largest n_t the solve's CFL adaptation may reach."""
    st = norm == "stokes"
    return ffi.RegParams(n1, n2, nt, _NORMS[norm], _CONS[constraint], _PREC[precision], _ADJ[adjoint],
                         _HESS[hessian], int(lowrank_capacity), int(nt_max), float(beta_v), float(beta_w),
                         float(nu) if st else 0.0, float(eps) if st else 0.0)


def paper_nt(n1, n2):
    """The number of time steps the paper starts from before adapting it to the CFL condition:
    n_t = 2 max(n1, n2) (Sec. 5)."""
    return 2 * max(n1, n2)


class Problem:
    def __init__(self, mT, mR, nt, norm="H1", constraint="divfree", beta_v=1e-2, beta_w=0.0,
                 precision="fp32", adjoint="dto", stream=None, lowrank_capacity=0, hessian="gn", nu=1.0,
                 eps=1e-6, nt_max=0):
        import torch
        self.torch = torch
        if mT.dtype != torch.float64 or mR.dtype != torch.float64 or not mT.is_cuda or not mR.is_cuda:
            raise ValueError("m_T and m_R must be float64 device tensors")
        n1, n2 = mT.shape
        self.n1, self.n2, self.nt = n1, n2, nt
        self.device = mT.device
        self.params = make_params(n1, n2, nt, norm, constraint, beta_v, beta_w, precision, adjoint,
                                  lowrank_capacity, hessian, nu, eps, nt_max)
        self.ws_bytes = ffi.reg_workspace_bytes(self.params)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.mT = mT.contiguous()
        self.mR = mR.contiguous()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = ffi.reg_create(self.params, self.mT.data_ptr(), self.mR.data_ptr(), self.ws_ptr,
                                self.ws_bytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            ffi.reg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_images(self, mT, mR):
        """Load a new image pair (same grid and settings) into this handle (reg_set_images)."""
        if mT.dtype != self.torch.float64 or mR.dtype != self.torch.float64 or tuple(mT.shape) != (self.n1, self.n2) \
                or tuple(mR.shape) != (self.n1, self.n2):
            raise ValueError("m_T and m_R must be float64 device tensors of the problem's grid size")
        self.mT = mT.contiguous()
        self.mR = mR.contiguous()
        ffi.reg_set_images(self.h, self.mT.data_ptr(), self.mR.data_ptr())

    def vec(self):
        return self.torch.empty((2, self.n1, self.n2), dtype=self.torch.float64, device=self.device)

    @staticmethod
    def _c(x):
        return x.contiguous()

    def state_forward(self, v):
        v = self._c(v)
        m1 = self.torch.empty((self.n1, self.n2), dtype=self.torch.float64, device=self.device)
        ffi.reg_state_forward(self.h, v.data_ptr(), m1.data_ptr())
        return m1

    def objective(self, v):
        v = self._c(v)
        return ffi.reg_objective(self.h, v.data_ptr())

    def gradient(self, v, want_J=True):
        v = self._c(v)
        g = self.vec()
        J = ffi.reg_gradient(self.h, v.data_ptr(), g.data_ptr(), want_J)
        return g, J

    def hessian_matvec(self, vt, out=None):
        vt = self._c(vt)
        out = self.vec() if out is None else out
        ffi.reg_hessian_matvec(self.h, vt.data_ptr(), out.data_ptr())
        return out

    def precond(self, r):
        r = self._c(r)
        z = self.vec()
        ffi.reg_precond_apply(self.h, r.data_ptr(), z.data_ptr())
        return z

    def pcg(self, rhs, eta=1e-3, max_iters=100, fixed_iters=0):
        rhs = self._c(rhs)
        x = self.vec()
        it, rr = ffi.reg_pcg(self.h, rhs.data_ptr(), eta, max_iters, fixed_iters, x.data_ptr())
        return x, it, rr

    def solve_opts(self, max_newton=50, max_pcg=100, fixed_pcg_iters=0, max_backtracks=10, gtol_rel=1e-2,
                   armijo_c1=1e-4, armijo_rho=0.5, v0=None, precond_U=None, recycle=0, ritz_out=None,
                   cfl_max=0.0, steps=None):
        """reg_solve_opts; v0 / precond_U must be contiguous float64 device tensors kept alive by the
        caller, ritz_out a ctypes double array of len(precond_U) (or None), steps a ctypes array of
        RegStepRecord (or None)."""
        import ctypes
        rank = 0 if precond_U is None else int(precond_U.shape[0])
        rec = ctypes.cast(steps, ctypes.POINTER(ffi.RegStepRecord)) if steps is not None else None
        return ffi.RegSolveOpts(max_newton, max_pcg, fixed_pcg_iters, max_backtracks, gtol_rel, armijo_c1,
                                armijo_rho, v0.data_ptr() if v0 is not None else None,
                                precond_U.data_ptr() if precond_U is not None else None, ritz_out, rank,
                                int(recycle), float(cfl_max), rec, len(steps) if steps is not None else 0)

    def solve(self, max_newton=50, max_pcg=100, fixed_pcg_iters=0, max_backtracks=10, gtol_rel=1e-2,
              armijo_c1=1e-4, armijo_rho=0.5, v0=None, raise_on_error=True, precond_U=None, recycle=0,
              cfl_max=0.0, log=None):
        """Alg. 1 (reg_solve).  precond_U: (r, 2, n1, n2) float64 directions of the preconditioner
        correction; recycle: PCG directions kept per Newton step (both need lowrank_capacity > 0);
        cfl_max > 0: n_t raised (up to nt_max) whenever the iterate's CFL number exceeds it.
        The stats dict carries the Ritz values of precond_U as "ritz" and, with `log`, the
        per-Newton-step records as "steps" (J, ||g||_rel, PCG iterations, step length, C(v), n_t and
        the step's wall time; reg_step_record).  log: a path (one JSON line per step is appended,
        with the grid and the step) or a callable taking each record."""
        import ctypes
        v0c = self._c(v0) if v0 is not None else None
        Uc = self._c(precond_U) if precond_U is not None else None
        ritz = (ctypes.c_double * int(Uc.shape[0]))() if Uc is not None and Uc.shape[0] > 0 else None
        steps = (ffi.RegStepRecord * max(1, min(max_newton + 1, 4096)))() if log is not None else None
        opts = self.solve_opts(max_newton, max_pcg, fixed_pcg_iters, max_backtracks, gtol_rel, armijo_c1,
                               armijo_rho, v0c, Uc, recycle, ritz, cfl_max, steps)
        v = self.vec()
        status, st = ffi.reg_solve(self.h, opts, v.data_ptr(), raise_on_error)
        d = st.as_dict()
        d["return_status"] = status
        if ritz is not None:
            d["ritz"] = list(ritz)
        self.nt = d["nt"]
        if steps is not None:
            # the failed step of a line search that gave up also has a record
            n_rec = min(len(steps), d["newton_iters"] + (1 if status == ffi.REG_ENOTCONV else 0))
            d["steps"] = [steps[k].as_dict() for k in range(n_rec)]
            write_step_log(log, d["steps"], {"n1": self.n1, "n2": self.n2})
        return v, d

    def ritz_directions(self, U, iters=8):
        """Leading generalised eigenpairs of (H, M) at the current linearisation point by subspace
        iteration from the directions U [r][2][n1][n2] (reg_ritz_directions): (Ritz vectors, values)."""
        U = self._c(U).clone()
        theta = ffi.reg_ritz_directions(self.h, U.data_ptr(), int(U.shape[0]), iters)
        return U, theta

    def cfl(self, v):
        """CFL number of v for this problem's n_t (reg_cfl)."""
        return ffi.reg_cfl(self.h, self._c(v).data_ptr())

    def deformation(self, v):
        """Deformation diagnostics of v (reg_deformation): (u_1, F_1, det F_1, (min, max, mean) of det F_1);
        the diagnostics workspace is allocated through torch on first use and kept."""
        v = self._c(v)
        nb = ffi.reg_deformation_workspace_bytes(self.params)
        if getattr(self, "_dws", None) is None:
            self._dws = self.torch.empty(nb + 256, dtype=self.torch.uint8, device=self.device)
        ptr = (self._dws.data_ptr() + 255) // 256 * 256
        u1 = self.vec()
        F1 = self.torch.empty((2, 2, self.n1, self.n2), dtype=self.torch.float64, device=self.device)
        det = self.torch.empty((self.n1, self.n2), dtype=self.torch.float64, device=self.device)
        stats = ffi.reg_deformation(self.h, v.data_ptr(), ptr, nb, u1.data_ptr(), F1.data_ptr(), det.data_ptr())
        return u1, F1, det, stats

    def time_pass(self, which, reps=100):
        return ffi.reg_time_pass(self.h, which, reps)

    def time_phases(self, which, reps=8):
        """reg_time_phases as a dict (microseconds per launch)."""
        keys = ("dispatch", "exec", "start_spread", "loads", "transforms", "stores")
        return dict(zip(keys, ffi.reg_time_phases(self.h, which, reps)))

    def autotune(self, reps=50):
        """Pick the fastest launch shape of each FP32 transport pass; returns the JSON timing report."""
        import json
        return json.loads(ffi.reg_autotune(self.h, reps))

    def set_pass_variants(self, variants):
        ffi.reg_set_pass_variants(self.h, list(variants))


def batch_solve(problems, raise_on_error=True, v0s=None, **opts):
    """Solve many problems concurrently (reg_batch_solve); returns ([v], [stats dict])."""
    outs = [p.vec() for p in problems]
    v0s = [v0.contiguous() if v0 is not None else None for v0 in (v0s or [None] * len(problems))]
    o = [p.solve_opts(v0=v0, **opts) for p, v0 in zip(problems, v0s)]
    status, st = ffi.reg_batch_solve([p.h for p in problems], o, [v.data_ptr() for v in outs], raise_on_error)
    return outs, [s.as_dict() for s in st]


def write_step_log(log, records, context):
    """Per-Newton-step records: appended to the file `log` as JSON lines ({**context, **record}), or
    passed one by one to the callable `log`."""
    import json
    if callable(log):
        for r in records:
            log(dict(context, **r))
        return
    with open(log, "a") as fh:
        for r in records:
            fh.write(json.dumps(dict(context, **r)) + "\n")
