"""Per-Newton-step records, and checkpoint / resume of the solve and of the network training (GPU).

* The step records of reg_solve agree with the solve's own statistics (one per Newton step, the last
  ||g||_rel and J are the final ones, the PCG and backtrack counts add up) and with the oracle's
  per-step gradient norms on a fixed-schedule solve; the C(v) of the last record is reg_cfl's.
* A solve stopped after two Newton steps, saved, loaded and resumed ends where the uninterrupted
  solve ends (same step counts, same iterate up to the rounding of re-projecting the saved iterate).
* Training stopped after one epoch, saved, loaded into a fresh network and resumed gives bitwise the
  parameters and Adam moments of the uninterrupted run.
"""
import numpy as np
import pytest

from gpu_cases import Case, dev, gpu_problem, host, inputs, params, close
from oracle import Grid, solver

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

C1_64 = Case(64, 64, 4, "H1", "divfree", 1e-2, 0.0, "fp64", config=1)
C2_32 = Case(256, 256, 16, "H2", "mass_source", 1e-3, 1e-4, "fp32", config=2)


def test_step_records_match_stats_and_oracle():
    case = C1_64
    print(f"[case] step records {case}", flush=True)
    mT, mR, *_ = inputs(case)
    g = Grid(case.n1, case.n2)
    v_ref, st_ref = solver.solve(g, params(case), mT, mR,
                                 solver.SolveOpts(max_newton=3, fixed_pcg_iters=4, gtol_rel=0.0))
    P = gpu_problem(case)
    try:
        seen = []
        v, st = P.solve(max_newton=3, fixed_pcg_iters=4, gtol_rel=0.0, log=seen.append)
        recs = st["steps"]
        assert len(recs) == len(seen) == st["newton_iters"] == 3
        assert [r["newton_iter"] for r in recs] == [0, 1, 2]
        assert sum(r["pcg_iters"] for r in recs) == st["pcg_iters"]
        assert sum(r["backtracks"] for r in recs) == st["backtracks"]
        assert recs[-1]["g_rel"] == st["g_rel"] and recs[-1]["J"] == st["J"]
        assert all(0 < r["alpha"] <= 1 and r["ms"] > 0 and r["nt"] == case.nt for r in recs)
        assert abs(recs[-1]["cfl"] - P.cfl(v)) <= 1e-12 * max(1.0, recs[-1]["cfl"])
        assert abs(st["g_rel"] - st_ref.g_rel) <= 1e-8 * st_ref.g_rel
        assert close(host(v), v_ref, 1e-10)
    finally:
        P.close()


@pytest.mark.parametrize("case", [C1_64, C2_32])
def test_solve_resumes_from_checkpoint(case, tmp_path):
    from paper_1503_00757_amd import checkpoint
    print(f"[case] resume {case}", flush=True)
    P = gpu_problem(case)
    try:
        v_full, st_full = P.solve(max_newton=50, gtol_rel=1e-3)
        assert st_full["status"] == 0 and st_full["newton_iters"] > 2
        v2, st2 = P.solve(max_newton=2, gtol_rel=1e-3)
        assert st2["newton_iters"] == 2
        path = tmp_path / "newton.npz"
        checkpoint.save_newton(path, v2, st2["newton_iters"], P.nt, st2["g0_norm"])
        state = checkpoint.load_newton(path)
        v_res, st_res = checkpoint.resume_solve(P, state, max_newton=50, gtol_rel=1e-3)
        assert st_res["status"] == 0 and st_res["fallback_used"] == 0
        assert st_res["newton_iters"] == st_full["newton_iters"]
        assert st_res["g0_norm"] == st2["g0_norm"] == st_full["g0_norm"]
        tol = 1e-10 if case.precision == "fp64" else 1e-5
        assert close(host(v_res), host(v_full), tol)
    finally:
        P.close()


def test_training_resumes_from_checkpoint(tmp_path):
    import synthdata
    from paper_1503_00757_amd import checkpoint
    from paper_1503_00757_amd import warmstart as W
    dev0 = torch.device("cuda:0")
    g = torch.Generator().manual_seed(3)
    n, N = 64, 32
    feats = torch.randn(N, 9, n, n, generator=g).to(dev0)
    targets = (0.1 * torch.randn(N, W.ffi.REG_FNO_OUT, n, n, generator=g)).to(dev0)
    a = W.WarmStart(synthdata.network_init(), dev0)
    a.train(feats, targets, 3, batch=16)
    b = W.WarmStart(synthdata.network_init(), dev0)
    b.train(feats, targets, 3, batch=16, end_epoch=1)
    path = tmp_path / "train.npz"
    checkpoint.save_training(path, b, epoch=1)
    c = W.WarmStart(np.zeros(W.N_PARAMS, dtype=np.float32), dev0)
    start = checkpoint.load_training(path, c)
    c.train(feats, targets, 3, batch=16, start_epoch=start)
    for name in ("params", "m", "v"):
        assert torch.equal(getattr(a, name), getattr(c, name)), name
    assert a.step == c.step
