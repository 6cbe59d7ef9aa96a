"""The C-ABI library loads and exports every symbol declared in include/regnk.h; host-side argument
checking (no device work).  CPU only."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1503_00757_amd as R
from paper_1503_00757_amd.problem import make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:reg_status|const char\*)\s+(reg_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("reg_create", "reg_objective", "reg_gradient", "reg_hessian_matvec", "reg_solve",
                 "reg_precond_apply", "reg_pcg", "reg_workspace_bytes", "reg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = R.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", R.library_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (reg_\w+)", out))
    assert set(declared_functions()) <= exported


def test_struct_layouts_match_header():
    assert ctypes.sizeof(R.RegParams) == 10 * 4 + 4 * 8
    assert ctypes.sizeof(R.RegSolveOpts) == 4 * 4 + 3 * 8 + 3 * 8 + 2 * 4 + 8 + 8 + 8   # steps, max_steps (padded)
    assert ctypes.sizeof(R.RegStepRecord) == 4 * 4 + 5 * 8
    assert ctypes.sizeof(R.RegSolveStats) == 8 * 4 + 4 * 8 + 2 * 4


def test_workspace_bytes_scales_with_grid_and_steps():
    a = R.reg_workspace_bytes(make_params(64, 64, 4))
    b = R.reg_workspace_bytes(make_params(64, 64, 8))
    c = R.reg_workspace_bytes(make_params(128, 64, 4))
    d = R.reg_workspace_bytes(make_params(64, 64, 4, precision="fp64"))
    assert b > a and c > a and d > a
    # the stored trajectory (2 nt + 1 vector fields in transport precision) dominates the growth in nt
    assert b - a >= 8 * 2 * 64 * 64 * 4


@pytest.mark.parametrize("kw", [
    dict(n1=61), dict(n2=4), dict(n1=4096), dict(n2=2050), dict(nt=0), dict(beta_v=0.0), dict(beta_v=-1.0),
    dict(constraint="mass_source", beta_w=0.0), dict(constraint="divfree", beta_w=1e-3),
])
def test_invalid_parameters_are_rejected(kw):
    args = dict(n1=64, n2=64, nt=4, norm="H1", constraint="divfree", beta_v=1e-2, beta_w=0.0)
    args.update(kw)
    p = make_params(args["n1"], args["n2"], args["nt"], args["norm"], args["constraint"], args["beta_v"],
                    args["beta_w"])
    with pytest.raises(R.RegError) as e:
        R.reg_workspace_bytes(p)
    assert e.value.status == -1
    assert len(R.reg_last_error()) > 0


def test_bad_enum_and_lowrank_capacity_rejected():
    p = make_params(64, 64, 4)
    p.norm = 5
    with pytest.raises(R.RegError):
        R.reg_workspace_bytes(p)
    for cap in (-1, 65):
        p = make_params(64, 64, 4, lowrank_capacity=cap)
        with pytest.raises(R.RegError) as e:
            R.reg_workspace_bytes(p)
        assert e.value.status == -1


@pytest.mark.parametrize("constraint,beta_w,sets", [("divfree", 0.0, 2), ("mass_source", 1e-3, 4)])
def test_workspace_grows_with_lowrank_capacity(constraint, beta_w, sets):
    """Each direction of the correction holds z and H z (and their K^-1 images for the mass-source
    model) as FP64 vector fields."""
    n = 64
    ws = [R.reg_workspace_bytes(make_params(n, n, 4, "H1", constraint, 1e-2, beta_w, lowrank_capacity=c))
          for c in (0, 4, 8)]
    field = 2 * n * n * 8
    assert ws[1] - ws[0] >= sets * 4 * field
    assert ws[2] - ws[1] == sets * 4 * field


def test_create_rejects_null_and_small_workspace_without_device_work():
    p = make_params(64, 64, 4)
    need = R.reg_workspace_bytes(p)
    with pytest.raises(R.RegError) as e:
        R.reg_create(p, 0, 0, 0, need, 0)
    assert e.value.status == -1
    with pytest.raises(R.RegError) as e:
        R.reg_create(p, 256, 256, 256, need - 1, 0)   # never dereferenced: size is checked first
    assert e.value.status == -2


def test_hessian_mode_checked_and_full_newton_workspace():
    p = make_params(64, 64, 4)
    p.hessian = 2
    with pytest.raises(R.RegError):
        R.reg_workspace_bytes(p)
    p = make_params(64, 64, 4)
    p.nt_max = 3          # below nt
    with pytest.raises(R.RegError):
        R.reg_workspace_bytes(p)
    p.nt_max = 4097
    with pytest.raises(R.RegError):
        R.reg_workspace_bytes(p)
    # room for the CFL adaptation: the trajectory of nt_max steps (2 nt_max + 1 vector fields)
    p.nt_max = 16
    assert R.reg_workspace_bytes(p) - R.reg_workspace_bytes(make_params(64, 64, 4)) == 2 * 12 * 2 * 64 * 64 * 4
    with pytest.raises(R.RegError) as e:   # full Newton is the derivative of the exact discrete adjoint
        R.reg_workspace_bytes(make_params(64, 64, 4, adjoint="paper", hessian="full"))
    assert e.value.status == -1
    # full Newton stores lam_{j+1}, lam*_j (2 n_t fields) and grad m~_j, grad m~*_j (2 n_t vector fields)
    for prec, ts in (("fp32", 4), ("fp64", 8)):
        gn = R.reg_workspace_bytes(make_params(64, 64, 4, precision=prec))
        full = R.reg_workspace_bytes(make_params(64, 64, 4, precision=prec, hessian="full"))
        assert full - gn == 2 * 4 * 64 * 64 * ts + 2 * 4 * 2 * 64 * 64 * ts


def test_deformation_workspace_and_null_checks():
    assert R.reg_deformation_workspace_bytes(make_params(64, 32, 4)) == 37 * 64 * 32 * 8
    with pytest.raises(R.RegError):
        R.reg_deformation_workspace_bytes(make_params(64, 31, 4))
    with pytest.raises(R.RegError) as e:
        R.reg_deformation(None, 256, 256, 1 << 20, None, None, None)
    assert e.value.status == -1


def test_shear_control_parameters_checked():
    assert R.reg_workspace_bytes(make_params(64, 64, 4, norm="stokes", nu=1.7, eps=1e-4)) > \
        R.reg_workspace_bytes(make_params(64, 64, 4))
    for kw in (dict(nu=0.0), dict(eps=0.0), dict(nu=float("nan"))):
        with pytest.raises(R.RegError):
            R.reg_workspace_bytes(make_params(64, 64, 4, norm="stokes", **kw))
    # with a mass source (relaxed incompressibility): two more FP64 fields for the penalty's gradient
    ms = R.reg_workspace_bytes(make_params(64, 64, 4, norm="stokes", constraint="mass_source", beta_w=1e-3, nu=1.7,
                                           eps=1e-4))
    assert ms > R.reg_workspace_bytes(make_params(64, 64, 4, constraint="mass_source", beta_w=1e-3))
    p = make_params(64, 64, 4)
    p.stokes_nu = 1.0                      # only meaningful for the shear-control model
    with pytest.raises(R.RegError):
        R.reg_workspace_bytes(p)


def test_even_grids_that_are_not_powers_of_two_are_accepted():
    """The paper's 128 x 150 slice (and 96^2 = 2^5 3 squared) take the mixed-radix transforms."""
    for n1, n2 in ((128, 150), (96, 96), (150, 128)):
        assert R.reg_workspace_bytes(make_params(n1, n2, 4)) > 0


def test_struct_offsets_match_header(tmp_path):
    """Every field of the ctypes mirrors sits where a C compiler puts it (gcc on include/regnk.h)."""
    structs = {"reg_params": R.RegParams, "reg_solve_opts": R.RegSolveOpts, "reg_solve_stats": R.RegSolveStats,
               "reg_step_record": R.RegStepRecord}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "regnk.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "offsets.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "offsets"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
