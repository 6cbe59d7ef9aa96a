"""ctypes declarations of the C ABI in ``include/regnk.h`` (argument marshalling only).

Every ``reg_*`` function here has the name and argument order of the C function; device arrays are
passed as integer addresses (``tensor.data_ptr()``), host outputs are returned.  A non-zero status
raises ``RegError`` carrying the status code and ``reg_last_error()``.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))

REG_OK, REG_EINVAL, REG_ENOMEM, REG_EDEVICE, REG_ENOTCONV, REG_ENONFINITE, REG_ESTATE = 0, -1, -2, -3, -4, -5, -6
REG_H1, REG_H2, REG_H3, REG_STOKES = 1, 2, 3, 4
REG_UNCONSTRAINED, REG_DIVFREE, REG_MASS_SOURCE = 0, 1, 2
REG_FP64, REG_FP32_TRANSPORT = 0, 1
REG_ADJ_DISCRETE, REG_ADJ_PAPER = 0, 1
REG_HESS_GN, REG_HESS_FULL = 0, 1

STATUS_NAMES = {0: "REG_OK", -1: "REG_EINVAL", -2: "REG_ENOMEM", -3: "REG_EDEVICE", -4: "REG_ENOTCONV",
                -5: "REG_ENONFINITE", -6: "REG_ESTATE"}


class RegParams(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("nt", C.c_int32), ("norm", C.c_int32),
                ("constraint", C.c_int32), ("precision", C.c_int32), ("adjoint", C.c_int32),
                ("hessian", C.c_int32), ("lowrank_capacity", C.c_int32), ("nt_max", C.c_int32),
                ("beta_v", C.c_double), ("beta_w", C.c_double), ("stokes_nu", C.c_double),
                ("stokes_eps", C.c_double)]


class RegStepRecord(C.Structure):
    _fields_ = [("newton_iter", C.c_int32), ("pcg_iters", C.c_int32), ("backtracks", C.c_int32),
                ("nt", C.c_int32), ("J", C.c_double), ("g_rel", C.c_double), ("alpha", C.c_double),
                ("cfl", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RegSolveOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("max_pcg", C.c_int32), ("fixed_pcg_iters", C.c_int32),
                ("max_backtracks", C.c_int32), ("gtol_rel", C.c_double), ("armijo_c1", C.c_double),
                ("armijo_rho", C.c_double), ("v0", C.c_void_p), ("precond_U", C.c_void_p),
                ("precond_d", C.POINTER(C.c_double)), ("rank", C.c_int32), ("recycle", C.c_int32),
                ("cfl_max", C.c_double), ("steps", C.POINTER(RegStepRecord)), ("max_steps", C.c_int32)]


class RegSolveStats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters", C.c_int32), ("n_matvec", C.c_int32),
                ("n_pde", C.c_int32), ("backtracks", C.c_int32), ("status", C.c_int32),
                ("fallback_used", C.c_int32), ("lowrank_dim", C.c_int32),
                ("g0_norm", C.c_double), ("g_rel", C.c_double), ("J", C.c_double), ("cfl", C.c_double),
                ("nt", C.c_int32), ("nt_changes", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RegError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def library_path() -> str:
    return os.path.join(HERE, "libregnk.so")


def lib():
    """Load the HIP library (no fallback: raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_1503_00757_amd.build`")
        L = C.CDLL(path)
        vp, dp, i32, d, sz = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_size_t
        L.reg_workspace_bytes.argtypes = [C.POINTER(RegParams), C.POINTER(sz)]
        L.reg_create.argtypes = [C.POINTER(RegParams), vp, vp, vp, sz, vp, C.POINTER(vp)]
        L.reg_destroy.argtypes = [vp]
        L.reg_set_images.argtypes = [vp, vp, vp]
        f32, i64 = C.c_float, C.c_int64
        L.reg_fno_param_count.argtypes = [C.POINTER(i64)]
        L.reg_fno_workspace_bytes.argtypes = [i32, i32, C.POINTER(sz)]
        L.reg_fno_create.argtypes = [i32, i32, vp, sz, vp, C.POINTER(vp)]
        L.reg_fno_destroy.argtypes = [vp]
        L.reg_fno_features.argtypes = [vp, vp, vp, vp, vp]
        L.reg_fno_target.argtypes = [vp, vp, vp, vp, vp]
        L.reg_fno_gather.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.reg_fno_forward.argtypes = [vp, vp, vp, vp]
        L.reg_fno_backward.argtypes = [vp, vp, vp, vp, vp]
        L.reg_fno_adam.argtypes = [vp, vp, vp, vp, vp, i32, f32, f32, f32, f32]
        L.reg_fno_train_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, f32, vp]
        L.reg_fno_predict.argtypes = [vp, vp, vp, vp, vp, vp]
        L.reg_set_stream.argtypes = [vp, vp]
        L.reg_state_forward.argtypes = [vp, vp, vp]
        L.reg_objective.argtypes = [vp, vp, dp, dp]
        L.reg_gradient.argtypes = [vp, vp, vp, dp]
        L.reg_hessian_matvec.argtypes = [vp, vp, vp]
        L.reg_precond_apply.argtypes = [vp, vp, vp]
        L.reg_pcg.argtypes = [vp, vp, d, i32, i32, vp, C.POINTER(i32), dp]
        L.reg_solve.argtypes = [vp, C.POINTER(RegSolveOpts), vp, C.POINTER(RegSolveStats)]
        L.reg_time_pass.argtypes = [vp, i32, i32, dp, dp, dp]
        L.reg_time_phases.argtypes = [vp, i32, i32, dp]
        L.reg_autotune.argtypes = [vp, i32, C.c_char_p, sz]
        L.reg_batch_solve.argtypes = [i32, C.POINTER(vp), C.POINTER(RegSolveOpts), C.POINTER(vp),
                                      C.POINTER(RegSolveStats)]
        L.reg_set_pass_variants.argtypes = [vp, C.POINTER(i32), i32]
        L.reg_deformation_workspace_bytes.argtypes = [C.POINTER(RegParams), C.POINTER(sz)]
        L.reg_cfl.argtypes = [vp, vp, dp]
        L.reg_ritz_directions.argtypes = [vp, vp, i32, i32, dp]
        L.reg_deformation.argtypes = [vp, vp, vp, sz, vp, vp, vp, dp]
        L.reg_deformation_static.argtypes = [vp, vp, vp, vp, vp, dp]
        L.reg_last_error.argtypes = []
        L.reg_last_error.restype = C.c_char_p
        for name in ("reg_workspace_bytes", "reg_create", "reg_destroy", "reg_set_stream", "reg_state_forward",
                     "reg_objective", "reg_gradient", "reg_hessian_matvec", "reg_precond_apply", "reg_pcg",
                     "reg_solve", "reg_time_pass", "reg_time_phases", "reg_autotune", "reg_set_pass_variants", "reg_batch_solve",
                     "reg_deformation_workspace_bytes", "reg_deformation", "reg_cfl", "reg_deformation_static",
                     "reg_ritz_directions"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def reg_last_error() -> str:
    return lib().reg_last_error().decode()


def _check(status: int):
    if status != REG_OK:
        raise RegError(status, reg_last_error())


def reg_workspace_bytes(params: RegParams) -> int:
    out = C.c_size_t(0)
    _check(lib().reg_workspace_bytes(C.byref(params), C.byref(out)))
    return out.value


def reg_create(params: RegParams, m_T: int, m_R: int, workspace: int, workspace_bytes: int, stream: int):
    h = C.c_void_p(0)
    _check(lib().reg_create(C.byref(params), m_T, m_R, workspace, workspace_bytes, stream, C.byref(h)))
    return h


def reg_destroy(h):
    _check(lib().reg_destroy(h))


def reg_set_stream(h, stream: int):
    _check(lib().reg_set_stream(h, stream))


def reg_state_forward(h, v: int, m1: int):
    _check(lib().reg_state_forward(h, v, m1))


def reg_objective(h, v: int):
    J = C.c_double(0)
    terms = (C.c_double * 3)()
    _check(lib().reg_objective(h, v, C.byref(J), terms))
    return J.value, list(terms)


def reg_gradient(h, v: int, g: int, want_J: bool = True):
    J = C.c_double(0)
    _check(lib().reg_gradient(h, v, g, C.byref(J) if want_J else None))
    return J.value if want_J else None


def reg_hessian_matvec(h, vtilde: int, Hvtilde: int):
    _check(lib().reg_hessian_matvec(h, vtilde, Hvtilde))


def reg_precond_apply(h, r: int, z: int):
    _check(lib().reg_precond_apply(h, r, z))


def reg_pcg(h, rhs: int, eta: float, max_iters: int, fixed_iters: int, x: int):
    it = C.c_int32(0)
    rr = C.c_double(0)
    _check(lib().reg_pcg(h, rhs, eta, max_iters, fixed_iters, x, C.byref(it), C.byref(rr)))
    return it.value, rr.value


def reg_solve(h, opts: RegSolveOpts, v_out: int, raise_on_error: bool = True):
    st = RegSolveStats()
    status = lib().reg_solve(h, C.byref(opts), v_out, C.byref(st))
    if raise_on_error:
        _check(status)
    return status, st


def reg_time_pass(h, which: int, reps: int):
    """(dispatch ms per launch, bytes per launch, execution ms per launch)"""
    ms = C.c_double(0)
    by = C.c_double(0)
    ex = C.c_double(0)
    _check(lib().reg_time_pass(h, which, reps, C.byref(ms), C.byref(by), C.byref(ex)))
    return ms.value, by.value, ex.value


def reg_time_phases(h, which: int, reps: int):
    """Phase-mode stage timing (microseconds per launch): dispatch, block execution, start spread,
    loads, transforms, stores."""
    out = (C.c_double * 6)()
    _check(lib().reg_time_phases(h, which, reps, out))
    return list(out)


def reg_autotune(h, reps: int = 50) -> str:
    buf = C.create_string_buffer(8192)
    _check(lib().reg_autotune(h, reps, buf, len(buf)))
    return buf.value.decode()


def reg_set_pass_variants(h, variants):
    arr = (C.c_int32 * len(variants))(*variants)
    _check(lib().reg_set_pass_variants(h, arr, len(variants)))


def reg_batch_solve(handles, opts, v_outs, raise_on_error: bool = True):
    n = len(handles)
    H = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    O = (RegSolveOpts * n)(*opts)
    V = (C.c_void_p * n)(*v_outs)
    S = (RegSolveStats * n)()
    status = lib().reg_batch_solve(n, H, O, V, S)
    if raise_on_error:
        _check(status)
    return status, [S[i] for i in range(n)]


def reg_ritz_directions(h, U: int, rank: int, iters: int):
    """Subspace iteration in place on the device directions U; returns the Ritz values (descending)."""
    th = (C.c_double * rank)()
    _check(lib().reg_ritz_directions(h, U, rank, iters, th))
    return list(th)


def reg_cfl(h, v: int) -> float:
    c = C.c_double(0)
    _check(lib().reg_cfl(h, v, C.byref(c)))
    return c.value


def reg_deformation_workspace_bytes(params: RegParams) -> int:
    out = C.c_size_t(0)
    _check(lib().reg_deformation_workspace_bytes(C.byref(params), C.byref(out)))
    return out.value


def reg_deformation(h, v: int, workspace: int, workspace_bytes: int, u1, F1, detF1, want_stats=True):
    """Returns (min, max, mean) of det F_1 (or None)."""
    st = (C.c_double * 3)()
    _check(lib().reg_deformation(h, v, workspace, workspace_bytes, u1, F1, detF1, st if want_stats else None))
    return tuple(st) if want_stats else None


def reg_deformation_static(h, v: int, u1, F1, detF1, want_stats=True):
    """reg_deformation with the library's static scratch (no workspace); (min, max, mean) of det F_1."""
    st = (C.c_double * 3)()
    _check(lib().reg_deformation_static(h, v, u1, F1, detF1, st if want_stats else None))
    return tuple(st) if want_stats else None


def reg_set_images(h, m_T: int, m_R: int):
    _check(lib().reg_set_images(h, m_T, m_R))


# ---- learned warm start (include/regnet.h) -------------------------------------------------------
REG_FNO_PARAMS = 4201610
REG_FNO_RANK = 4
REG_FNO_DIR_WEIGHT = 0.1
REG_FNO_OUT = 2 + 2 * REG_FNO_RANK
REG_FNO_SYMMETRIES = 8


def reg_fno_param_count() -> int:
    c = C.c_int64()
    _check(lib().reg_fno_param_count(C.byref(c)))
    return c.value


def reg_fno_workspace_bytes(n: int, batch: int) -> int:
    b = C.c_size_t()
    _check(lib().reg_fno_workspace_bytes(n, batch, C.byref(b)))
    return b.value


def reg_fno_create(n: int, batch: int, workspace: int, workspace_bytes: int, stream: int):
    h = C.c_void_p()
    _check(lib().reg_fno_create(n, batch, workspace, workspace_bytes, stream, C.byref(h)))
    return h


def reg_fno_destroy(h):
    _check(lib().reg_fno_destroy(h))


def reg_fno_features(h, m_T: int, m_R: int, out: int, scale=None):
    _check(lib().reg_fno_features(h, m_T, m_R, out, scale))


def reg_fno_target(h, v: int, scale: int, dirs, out: int):
    _check(lib().reg_fno_target(h, v, scale, dirs, out))


def reg_fno_gather(h, data_set: int, nset: int, channels: int, idx: int, sym, out: int):
    _check(lib().reg_fno_gather(h, data_set, nset, channels, idx, sym, out))


def reg_fno_forward(h, params: int, inp: int, out):
    _check(lib().reg_fno_forward(h, params, inp, out))


def reg_fno_backward(h, params: int, target: int, grad: int, loss):
    _check(lib().reg_fno_backward(h, params, target, grad, loss))


def reg_fno_adam(h, params: int, grad: int, m: int, v: int, step: int, lr: float, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8):
    _check(lib().reg_fno_adam(h, params, grad, m, v, step, lr, beta1, beta2, eps))


def reg_fno_train_step(h, params: int, inp: int, target: int, grad: int, m: int, v: int, step: int, lr: float,
                       loss):
    _check(lib().reg_fno_train_step(h, params, inp, target, grad, m, v, step, lr, loss))


def reg_fno_predict(h, params: int, m_T: int, m_R: int, v0: int, dirs=None):
    _check(lib().reg_fno_predict(h, params, m_T, m_R, v0, dirs))
