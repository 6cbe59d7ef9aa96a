"""The registration library's host driver (regnk_host.hip, compiled with g++) run on the CPU against
range-checking CPU versions of every kernel launch (tests/regmock): each launch checks that every
array it would read or write lies inside a buffer the caller registered (workspace, images,
velocities, outputs) or the library's static scratch, so a workspace carve-out, an offset or a size
that runs past its buffer fails the call.  Kernels compute nothing here (they return placeholder
scalars), so these tests cover addressing and control flow of every entry point, not values; the
values are covered by the GPU parity tests.  No GPU involved."""
import ctypes as C
import json
import os
import subprocess

import numpy as np
import pytest

from paper_1503_00757_amd.ffi import (REG_DIVFREE, REG_EDEVICE, REG_FP32_TRANSPORT, REG_FP64, REG_H1, REG_H2,
                                      REG_H3, REG_HESS_FULL, REG_HESS_GN, REG_MASS_SOURCE, REG_STOKES,
                                      REG_UNCONSTRAINED, RegParams, RegSolveOpts, RegSolveStats,
                                      RegStepRecord)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEF_STATIC_MAX_POINTS = 65536


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    return build_mock(str(tmp_path_factory.mktemp("regmock") / "libregmock.so"))


def build_mock(out):
    cmd = ["g++", "-std=c++17", "-O1", "-fPIC", "-shared",
           "-I", os.path.join(ROOT, "tests", "regmock"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1503_00757_amd", "csrc"),
           "-x", "c++", os.path.join(ROOT, "paper_1503_00757_amd", "csrc", "regnk_host.hip"),
           "-x", "c++", os.path.join(ROOT, "tests", "regmock", "regmock_kernels.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    L = C.CDLL(out)
    vp, dp, i32, d, sz = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_size_t
    L.mock_register.argtypes = [vp, sz]
    L.mock_last_error.restype = C.c_char_p
    L.mock_launches.restype = C.c_long
    L.mock_pcg_updates.restype = C.c_long
    L.mock_pcg_updates.argtypes = [C.c_int]
    L.reg_workspace_bytes.argtypes = [C.POINTER(RegParams), C.POINTER(sz)]
    L.reg_create.argtypes = [C.POINTER(RegParams), vp, vp, vp, sz, vp, C.POINTER(vp)]
    L.reg_destroy.argtypes = [vp]
    L.reg_set_images.argtypes = [vp, vp, vp]
    L.reg_state_forward.argtypes = [vp, vp, vp]
    L.reg_objective.argtypes = [vp, vp, dp, dp]
    L.reg_gradient.argtypes = [vp, vp, vp, dp]
    L.reg_hessian_matvec.argtypes = [vp, vp, vp]
    L.reg_precond_apply.argtypes = [vp, vp, vp]
    L.reg_pcg.argtypes = [vp, vp, d, i32, i32, vp, C.POINTER(i32), dp]
    L.reg_solve.argtypes = [vp, C.POINTER(RegSolveOpts), vp, C.POINTER(RegSolveStats)]
    L.reg_batch_solve.argtypes = [i32, C.POINTER(vp), C.POINTER(RegSolveOpts), C.POINTER(vp),
                                  C.POINTER(RegSolveStats)]
    L.reg_cfl.argtypes = [vp, vp, dp]
    L.reg_deformation_workspace_bytes.argtypes = [C.POINTER(RegParams), C.POINTER(sz)]
    L.reg_deformation.argtypes = [vp, vp, vp, sz, vp, vp, vp, dp]
    L.reg_deformation_static.argtypes = [vp, vp, vp, vp, vp, dp]
    L.reg_time_pass.argtypes = [vp, i32, i32, dp, dp, dp]
    L.reg_time_phases.argtypes = [vp, i32, i32, dp]
    L.reg_autotune.argtypes = [vp, i32, C.c_char_p, sz]
    L.reg_set_pass_variants.argtypes = [vp, C.POINTER(i32), i32]
    L.reg_ritz_directions.argtypes = [vp, vp, i32, i32, dp]
    L.reg_last_error.restype = C.c_char_p
    return L


def params(n1, n2, nt=2, norm=REG_H1, constraint=REG_UNCONSTRAINED, precision=REG_FP32_TRANSPORT,
           hessian=REG_HESS_GN, lowrank=0, nt_max=0):
    p = RegParams()
    p.n1, p.n2, p.nt, p.norm, p.constraint, p.precision = n1, n2, nt, norm, constraint, precision
    p.adjoint, p.hessian, p.lowrank_capacity, p.nt_max = 0, hessian, lowrank, nt_max
    p.beta_v = 1e-2
    p.beta_w = 1e-3 if constraint == REG_MASS_SOURCE else 0.0
    p.stokes_nu, p.stokes_eps = (0.5, 1e-2) if norm == REG_STOKES else (0.0, 0.0)
    return p


def aligned(L, n, dtype, keep):
    """A zeroed, registered array of n elements starting on a 256-byte boundary (device allocations
    are at least that aligned)."""
    isz = np.dtype(dtype).itemsize
    raw = np.zeros(n * isz + 256, dtype=np.uint8)
    off = (-raw.ctypes.data) % 256
    a = raw[off:off + n * isz].view(dtype)
    L.mock_register(C.c_void_p(a.ctypes.data), a.nbytes)
    keep.append(raw)
    return a


class Host:
    """Registered host buffers standing in for device memory, and the problem handle."""

    def __init__(self, L, p):
        self.L, self.p = L, p
        self.nn = p.n1 * p.n2
        L.mock_reset()
        self.keep = []
        nb = C.c_size_t()
        assert L.reg_workspace_bytes(C.byref(p), C.byref(nb)) == 0, L.reg_last_error()
        self.ws = self.buf(nb.value, np.uint8)   # zeroed pages are only touched where written
        self.mT = self.buf(self.nn)
        self.mR = self.buf(self.nn)
        self.h = C.c_void_p()
        self.check(L.reg_create(C.byref(p), self.ptr(self.mT), self.ptr(self.mR), self.ptr(self.ws), nb.value, None,
                                C.byref(self.h)))

    def buf(self, n, dtype=np.float64):
        return aligned(self.L, n, dtype, self.keep)

    @staticmethod
    def ptr(a):
        return C.c_void_p(a.ctypes.data)

    def check(self, rc, ok=(0,)):
        err = self.L.mock_last_error().decode()
        assert err == "", err
        assert rc != REG_EDEVICE and rc in ok, (rc, self.L.reg_last_error().decode())

    def close(self):
        self.check(self.L.reg_destroy(self.h))


def run_all(L, p, solve=True):
    """Every single-problem entry point once, in a valid order."""
    H = Host(L, p)
    nn, dbl = H.nn, C.c_double
    v, m1, g = H.buf(2 * nn), H.buf(nn), H.buf(2 * nn)
    J, terms = dbl(), (dbl * 3)()
    H.check(L.reg_set_images(H.h, H.ptr(H.mT), H.ptr(H.mR)))
    H.check(L.reg_state_forward(H.h, H.ptr(v), H.ptr(m1)))
    H.check(L.reg_objective(H.h, H.ptr(v), C.byref(J), terms))
    H.check(L.reg_gradient(H.h, H.ptr(v), H.ptr(g), C.byref(J)))
    vt, Hv, z, x = H.buf(2 * nn), H.buf(2 * nn), H.buf(2 * nn), H.buf(2 * nn)
    H.check(L.reg_hessian_matvec(H.h, H.ptr(vt), H.ptr(Hv)))
    H.check(L.reg_hessian_matvec(H.h, H.ptr(vt), H.ptr(Hv)))   # replay (graph slot reuse on a GPU)
    H.check(L.reg_precond_apply(H.h, H.ptr(g), H.ptr(z)))
    it, rel = C.c_int32(), dbl()
    H.check(L.reg_pcg(H.h, H.ptr(g), 0.5, 4, 0, H.ptr(x), C.byref(it), C.byref(rel)), ok=(0, -4, -5))
    H.check(L.reg_pcg(H.h, H.ptr(g), 0.5, 8, 3, H.ptr(x), C.byref(it), C.byref(rel)), ok=(0, -4, -5))
    cfl = dbl()
    H.check(L.reg_cfl(H.h, H.ptr(v), C.byref(cfl)))
    ms, by, ex = dbl(), dbl(), dbl()
    for which in range(4):   # the timing hook covers the Gauss-Newton stages only
        H.check(L.reg_time_pass(H.h, which, 2, C.byref(ms), C.byref(by), C.byref(ex)),
                ok=(0,) if p.hessian == REG_HESS_GN else (-1,))
        ph = (dbl * 6)()
        H.check(L.reg_time_phases(H.h, which, 2, ph), ok=(0,) if p.hessian == REG_HESS_GN else (-1,))
    rep = C.create_string_buffer(4096)
    H.check(L.reg_autotune(H.h, 1, rep, len(rep)))
    if p.precision == REG_FP32_TRANSPORT:   # both rounds ran (isolated stage launches, whole matvecs)
        r = json.loads(rep.value.decode())
        assert len(r["chosen"]) == 7 and "matvec_ms" in r and "matvec_ms_isolated_choice" in r, r
    var = (C.c_int32 * 7)(*[k % 12 for k in range(7)])
    H.check(L.reg_set_pass_variants(H.h, var, 7))
    H.check(L.reg_hessian_matvec(H.h, H.ptr(vt), H.ptr(Hv)))
    if p.lowrank_capacity:
        rank = min(p.lowrank_capacity, 8)
        U = H.buf(rank * 2 * nn)
        th = (dbl * rank)()
        ok = (-1,) if p.norm == REG_STOKES and p.constraint == REG_MASS_SOURCE else (0,)
        H.check(L.reg_ritz_directions(H.h, H.ptr(U), rank, 3, th), ok=ok)
    else:
        H.check(L.reg_ritz_directions(H.h, H.ptr(v), 1, 3, None), ok=(-1,))   # no correction slots
    u1, F1, det = H.buf(2 * nn), H.buf(4 * nn), H.buf(nn)
    stats = (dbl * 8)()
    nb = C.c_size_t()
    H.check(L.reg_deformation_workspace_bytes(C.byref(p), C.byref(nb)))
    dws = H.buf(nb.value, np.uint8)
    H.check(L.reg_deformation(H.h, H.ptr(v), H.ptr(dws), nb.value, H.ptr(u1), H.ptr(F1), H.ptr(det), stats))
    rc = L.reg_deformation_static(H.h, H.ptr(v), H.ptr(u1), H.ptr(F1), H.ptr(det), stats)
    H.check(rc, ok=(0,) if nn <= DEF_STATIC_MAX_POINTS else (-1,))
    if solve:
        o = RegSolveOpts()
        o.max_newton, o.max_pcg, o.fixed_pcg_iters, o.max_backtracks = 4, 6, 0, 3
        o.gtol_rel, o.armijo_c1, o.armijo_rho = 1e-3, 1e-4, 0.5
        o.cfl_max = 0.5 if p.nt_max > p.nt else 0.0
        o.recycle = 1 if p.lowrank_capacity else 0
        st = RegSolveStats()
        vout = H.buf(2 * nn)
        recs = (RegStepRecord * 3)()   # fewer records than steps: the first three are kept
        o.steps, o.max_steps = C.cast(recs, C.POINTER(RegStepRecord)), 3
        H.check(L.reg_solve(H.h, C.byref(o), H.ptr(vout), C.byref(st)), ok=(0, -4, -5))
        assert st.newton_iters == 4   # the placeholder scalars let every line search succeed
        assert [r.newton_iter for r in recs] == [0, 1, 2] and all(r.alpha > 0 and r.nt >= p.nt for r in recs)
        o.steps, o.max_steps = None, 0
        if p.lowrank_capacity:
            assert st.lowrank_dim == p.lowrank_capacity
        o.fixed_pcg_iters = 3
        o.v0 = C.c_void_p(vout.ctypes.data)
        H.check(L.reg_solve(H.h, C.byref(o), H.ptr(vout), C.byref(st)), ok=(0, -4, -5))
    assert L.mock_launches() > 0
    H.close()
    return H


GRIDS = [
    (8, 8), (16, 16), (64, 64), (256, 256), (2048, 2048),            # powers of two (register FFTs)
    (64, 96), (128, 150), (30, 30), (250, 250), (1000, 1000),          # 2^a 3^b 5^c (mixed radix)
    (14, 22), (2046, 8), (8, 2046), (96, 14),                          # other even lengths (direct sums)
]


@pytest.mark.parametrize("n1,n2", GRIDS)
@pytest.mark.parametrize("precision", [REG_FP32_TRANSPORT, REG_FP64])
def test_every_entry_point_stays_in_bounds(lib, n1, n2, precision):
    big = n1 * n2 > 1 << 20
    run_all(lib, params(n1, n2, nt=2 if big else 4, precision=precision))


@pytest.mark.parametrize("case", [
    dict(norm=REG_H2, constraint=REG_DIVFREE),
    dict(norm=REG_H3, constraint=REG_MASS_SOURCE),
    dict(norm=REG_STOKES, constraint=REG_UNCONSTRAINED),
    dict(norm=REG_STOKES, constraint=REG_DIVFREE),
    dict(norm=REG_STOKES, constraint=REG_MASS_SOURCE),
    dict(hessian=REG_HESS_FULL, precision=REG_FP64),
    dict(hessian=REG_HESS_FULL, constraint=REG_DIVFREE),
    dict(lowrank=4),
    dict(lowrank=4, constraint=REG_MASS_SOURCE),
    dict(nt_max=24),
])
@pytest.mark.parametrize("n1,n2", [(64, 64), (96, 80), (22, 14)])
def test_models_and_options_stay_in_bounds(lib, case, n1, n2):
    run_all(lib, params(n1, n2, **case))


def test_batch_solve_stays_in_bounds(lib):
    p = params(64, 64, constraint=REG_DIVFREE)
    lib.mock_reset()
    keep, handles, outs = [], [], []
    for _ in range(3):
        nb = C.c_size_t()
        lib.reg_workspace_bytes(C.byref(p), C.byref(nb))
        ws = aligned(lib, nb.value, np.uint8, keep)
        mT, mR, vo = aligned(lib, 4096, np.float64, keep), aligned(lib, 4096, np.float64, keep), \
            aligned(lib, 8192, np.float64, keep)
        h = C.c_void_p()
        assert lib.reg_create(C.byref(p), Host.ptr(mT), Host.ptr(mR), Host.ptr(ws), nb.value, None, C.byref(h)) == 0
        handles.append(h.value)
        outs.append(vo.ctypes.data)
    o = RegSolveOpts()
    o.max_newton, o.max_pcg, o.max_backtracks, o.gtol_rel, o.armijo_c1, o.armijo_rho = 2, 5, 2, 1e-3, 1e-4, 0.5
    st = (RegSolveStats * 3)()
    rc = lib.reg_batch_solve(3, (C.c_void_p * 3)(*handles), C.byref(o), (C.c_void_p * 3)(*outs), st)
    assert lib.mock_last_error().decode() == ""
    assert rc != REG_EDEVICE
    for h in handles:
        assert lib.reg_destroy(C.c_void_p(h)) == 0


def test_harness_catches_a_short_buffer(lib):
    """The harness itself: an output one element too short is reported, and the call fails."""
    p = params(16, 16)
    H = Host(lib, p)
    v = H.buf(2 * H.nn)
    short = H.buf(H.nn - 1)
    rc = lib.reg_state_forward(H.h, H.ptr(v), H.ptr(short))
    assert rc == REG_EDEVICE
    assert "outside every registered buffer" in lib.mock_last_error().decode() or \
        "hipMemcpyAsync" in lib.mock_last_error().decode()


def test_static_scratch_limit_on_the_host(lib):
    """reg_deformation_static takes grids up to its static size and refuses larger ones without
    touching device memory."""
    for n1, n2, want in [(256, 256, 0), (128, 512, 0), (256, 264, -1), (512, 512, -1)]:
        H = Host(lib, params(n1, n2))
        nn = H.nn
        v, u1, F1, det = H.buf(2 * nn), H.buf(2 * nn), H.buf(4 * nn), H.buf(nn)
        launches = lib.mock_launches()
        rc = lib.reg_deformation_static(H.h, H.ptr(v), H.ptr(u1), H.ptr(F1), H.ptr(det), None)
        H.check(rc, ok=(want,))
        if want:
            assert lib.mock_launches() == launches
        H.close()


@pytest.mark.parametrize("n1,n2,lowrank,recurrence", [
    (64, 64, 0, True), (512, 256, 0, True), (256, 256, 4, True),    # column pass forms P^{-1} H s
    (1024, 1024, 0, False), (32, 128, 0, False), (64, 96, 0, False),   # no such column pass
    (256, 256, 4, None),                                              # recycling solve
])
def test_pcg_preconditioned_residual_schedule(lib, n1, n2, lowrank, recurrence):
    """Which update each PCG iteration launches: with the recurrence every iteration but each eighth
    updates z (and K^{-1} r) from P^{-1} H s, and each eighth forms them from r (the refresh); without
    it (no such column pass, or the low-rank-corrected preconditioner of a solve with caller
    directions) every iteration applies the preconditioner to r.  A recycling solve runs its first
    Newton step, before any direction is held, with the plain preconditioner and the recurrence."""
    p = params(n1, n2, constraint=REG_MASS_SOURCE, lowrank=lowrank)
    H = Host(lib, p)
    nn = H.nn
    v, g, x = H.buf(2 * nn), H.buf(2 * nn), H.buf(2 * nn)
    H.check(lib.reg_gradient(H.h, H.ptr(v), H.ptr(g), None))
    before = (lib.mock_pcg_updates(0), lib.mock_pcg_updates(1))
    if recurrence is None:
        # two Newton steps of 20 PCG iterations, recycling directions: the first step with the plain
        # preconditioner by recurrence, the second with the correction its directions switched on
        o = RegSolveOpts()
        o.max_newton, o.max_pcg, o.fixed_pcg_iters, o.max_backtracks = 2, 20, 20, 3
        o.gtol_rel, o.armijo_c1, o.armijo_rho, o.recycle = 0.0, 1e-4, 0.5, 2
        st = RegSolveStats()
        H.check(lib.reg_solve(H.h, C.byref(o), H.ptr(x), C.byref(st)), ok=(0, -4, -5))
        assert st.newton_iters == 2 and st.pcg_iters == 40 and st.lowrank_dim > 0
    else:
        it, rel = C.c_int32(), C.c_double()
        H.check(lib.reg_pcg(H.h, H.ptr(g), 0.0, 20, 20, H.ptr(x), C.byref(it), C.byref(rel)))
    plain = lib.mock_pcg_updates(0) - before[0]
    rec = lib.mock_pcg_updates(1) - before[1]
    want = {True: (2, 18), False: (20, 0), None: (2 + 20, 18)}[recurrence]
    assert (plain, rec) == want
    H.close()
