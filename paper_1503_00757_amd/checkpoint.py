"""Checkpoint and resume of the two iterative processes around the hot path.

* Newton (Alg. 1): the state of a solve is its iterate v_k, the step count k and n_t (which a
  CFL-adapted solve may have raised); ||g(0)|| needs no storing, since reg_solve recomputes it at
  v = 0.  Resuming is a warm-started solve from v_k with the remaining step budget: the library
  re-linearises at v_k, keeps it (it lowers J below J(0)) and takes the same steps the uninterrupted
  solve would have taken (without recycled PCG directions, which live in the handle).
* Network training: the parameters, the two Adam moments and the Adam step count; the epoch
  reached resumes the same shuffling and learning-rate schedule (WarmStart.train, start_epoch).

Files are NumPy .npz archives written and read without pickling.
"""
from __future__ import annotations

import numpy as np


def save_newton(path, v, newton_iters: int, nt: int, g0_norm: float | None = None) -> None:
    """v: the iterate (device or host array [2][n1][n2], float64)."""
    vh = v.detach().cpu().numpy() if hasattr(v, "detach") else np.asarray(v)
    np.savez(path, v=np.ascontiguousarray(vh, dtype=np.float64), newton_iters=np.int64(newton_iters),
             nt=np.int64(nt), g0_norm=np.float64(np.nan if g0_norm is None else g0_norm))


def load_newton(path) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {"v": z["v"], "newton_iters": int(z["newton_iters"]), "nt": int(z["nt"]),
                "g0_norm": float(z["g0_norm"])}


def resume_solve(P, state: dict, max_newton: int = 50, **solve_kw):
    """Continue a solve from a save_newton state on the problem handle P (same images, parameters and
    n_t = state["nt"]): at most max_newton - k more Newton steps.  Returns (v, stats) with the step
    counts of the whole solve."""
    import torch
    if P.nt != state["nt"]:
        raise ValueError(f"the handle runs n_t = {P.nt}, the checkpoint n_t = {state['nt']}")
    k = state["newton_iters"]
    v0 = torch.as_tensor(state["v"], dtype=torch.float64, device=P.device).contiguous()
    v, st = P.solve(max_newton=max(0, max_newton - k), v0=v0, **solve_kw)
    st = dict(st)
    st["newton_iters"] += k
    st["resumed_from"] = k
    return v, st


def save_training(path, ws, epoch: int) -> None:
    """WarmStart ws after `epoch` completed epochs."""
    np.savez(path, params=ws.params.cpu().numpy(), m=ws.m.cpu().numpy(), v=ws.v.cpu().numpy(),
             step=np.int64(ws.step), epoch=np.int64(epoch))


def load_training(path, ws) -> int:
    """Restore parameters, Adam moments and step into ws; returns the epoch to resume from."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        for name in ("params", "m", "v"):
            t = torch.as_tensor(z[name], dtype=torch.float32)
            if t.numel() != getattr(ws, name).numel():
                raise ValueError(f"{name}: {t.numel()} values, expected {getattr(ws, name).numel()}")
            getattr(ws, name).copy_(t.to(ws.device))
        ws.step = int(z["step"])
        return int(z["epoch"])
