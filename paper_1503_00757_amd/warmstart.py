"""Learned warm start (``include/regnet.h``): a Fourier neural operator predicts the initial velocity of
the Gauss-Newton solve (Alg. 1) from (m_T, m_R), and directions for the low-rank correction of its
PCG preconditioner.  It is trained on the GPU by the library's own
forward, reverse-pass and Adam kernels on registrations that the plain solver produced, and the
plain solver has the last word: ``reg_solve`` drops a warm start that does not lower the objective.

This module only holds device buffers (torch tensors), the training schedule (batch order, learning
rate) and host timing; every arithmetic step runs in ``libregnk.so``.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import ffi
from .problem import Problem, batch_solve

N_PARAMS = ffi.REG_FNO_PARAMS


class Network:
    """One network handle for an n x n grid and a fixed batch size."""

    def __init__(self, n: int, batch: int, device, stream=None):
        import torch
        self.torch = torch
        self.n, self.batch, self.device = n, batch, device
        self.ws_bytes = ffi.reg_fno_workspace_bytes(n, batch)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.h = ffi.reg_fno_create(n, batch, ptr, self.ws_bytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            ffi.reg_fno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, *shape):
        return self.torch.empty(shape, dtype=self.torch.float32, device=self.device)

    def features(self, mT, mR, out=None, scale=None):
        """[9][n][n] float32 input features of one pair (FP64 device fields); the misfit scale s goes
        to `scale` (a device float64 tensor of one element) when given."""
        out = self._f32(9, self.n, self.n) if out is None else out
        ffi.reg_fno_features(self.h, mT.contiguous().data_ptr(), mR.contiguous().data_ptr(), out.data_ptr(),
                             scale.data_ptr() if scale is not None else None)
        return out

    def target(self, v, scale, dirs=None, out=None):
        """[REG_FNO_OUT][n][n] float32 training target: v / s of a solved velocity (FP64) and its pair's
        scale, then the direction targets dirs [REG_FNO_RANK][2][n][n] (FP64; None: zeros, not trained)."""
        out = self._f32(ffi.REG_FNO_OUT, self.n, self.n) if out is None else out
        ffi.reg_fno_target(self.h, v.contiguous().data_ptr(), scale.data_ptr(),
                           dirs.contiguous().data_ptr() if dirs is not None else None, out.data_ptr())
        return out

    def gather(self, data_set, idx, out=None, sym=None):
        """out[c][b] = data_set[idx[b]][c] mapped by the grid symmetry sym[b] (nullable), for a
        sample-major data set [N][C][n][n]."""
        nset, ch = data_set.shape[0], data_set.shape[1]
        for t in (idx,) if sym is None else (idx, sym):
            if t.dtype != self.torch.int32 or t.numel() < self.batch or not t.is_cuda:
                raise ValueError("idx / sym must be device int32 tensors with at least `batch` entries")
        out = self._f32(ch, self.batch, self.n, self.n) if out is None else out
        ffi.reg_fno_gather(self.h, data_set.data_ptr(), nset, ch, idx.data_ptr(),
                           sym.data_ptr() if sym is not None else None, out.data_ptr())
        return out

    def forward(self, params, inp, out=None):
        out = self._f32(ffi.REG_FNO_OUT, self.batch, self.n, self.n) if out is None else out
        ffi.reg_fno_forward(self.h, params.data_ptr(), inp.contiguous().data_ptr(), out.data_ptr())
        return out

    def backward(self, params, target, grad=None, loss=None):
        grad = self._f32(N_PARAMS) if grad is None else grad
        ffi.reg_fno_backward(self.h, params.data_ptr(), target.contiguous().data_ptr(), grad.data_ptr(),
                             loss.data_ptr() if loss is not None else None)
        return grad

    def adam(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        ffi.reg_fno_adam(self.h, params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), step, lr, beta1,
                         beta2, eps)

    def train_step(self, params, inp, target, grad, m, v, step, lr, loss=None):
        ffi.reg_fno_train_step(self.h, params.data_ptr(), inp.data_ptr(), target.data_ptr(), grad.data_ptr(),
                               m.data_ptr(), v.data_ptr(), step, lr, loss.data_ptr() if loss is not None else None)

    def predict(self, params, mT, mR):
        """(v0 FP64 [2][n][n], directions FP64 [REG_FNO_RANK][2][n][n]) for one pair (batch-1 handle)."""
        t = self.torch
        v0 = t.empty((2, self.n, self.n), dtype=t.float64, device=self.device)
        dirs = t.empty((ffi.REG_FNO_RANK, 2, self.n, self.n), dtype=t.float64, device=self.device)
        ffi.reg_fno_predict(self.h, params.data_ptr(), mT.contiguous().data_ptr(), mR.contiguous().data_ptr(),
                            v0.data_ptr(), dirs.data_ptr())
        return v0, dirs


class WarmStart:
    """Network parameters (float32 master copy on the device), Adam state and the training loop."""

    def __init__(self, params, device):
        import torch
        self.torch = torch
        self.device = device
        p = torch.as_tensor(params, dtype=torch.float32)
        if p.numel() != N_PARAMS:
            raise ValueError(f"expected {N_PARAMS} parameters, got {p.numel()}")
        self.params = p.to(device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0
        self._pred = {}

    def train(self, feats, targets, epochs, batch=16, lr=1e-3, lr_final=5e-5, seed=0, log=None, augment=True,
              start_epoch=0, end_epoch=None):
        """Adam on the network loss (regnet.h) over shuffled batches; cosine learning-rate decay from
        lr to lr_final.  feats: [N][9][n][n], targets: [N][REG_FNO_OUT][n][n] (normalised velocities
        v / s, then the direction targets; float32, device).  With augment, every sample of a batch is mapped by a random one of the 8
        symmetries of the periodic square grid (exact for the discrete problem).  Runs epochs
        [start_epoch, end_epoch) of an `epochs`-long schedule (same shuffling and learning rates as
        one uninterrupted run; resume from a checkpoint.save_training state).  Returns the mean
        training loss of every epoch run."""
        torch = self.torch
        N, n = feats.shape[0], feats.shape[-1]
        if N < batch:
            raise ValueError("fewer samples than one batch")
        net = Network(n, batch, self.device)
        inp = net._f32(feats.shape[1], batch, n, n)
        tgt = net._f32(targets.shape[1], batch, n, n)
        steps_per_epoch = N // batch
        total = epochs * steps_per_epoch
        losses = torch.zeros(steps_per_epoch, dtype=torch.float64, device=self.device)
        rng = np.random.Generator(np.random.PCG64(seed))
        history = []
        end_epoch = epochs if end_epoch is None else end_epoch
        if not 0 <= start_epoch <= end_epoch <= epochs:
            raise ValueError("need 0 <= start_epoch <= end_epoch <= epochs")
        done = start_epoch * steps_per_epoch
        for ep in range(end_epoch):
            perm = rng.permutation(N)[:steps_per_epoch * batch].astype(np.int32)
            sy = rng.integers(0, ffi.REG_FNO_SYMMETRIES, steps_per_epoch * batch).astype(np.int32) if augment else None
            if ep < start_epoch:   # the draws of the epochs already run
                continue
            order = torch.tensor(perm, device=self.device)
            syms = torch.tensor(sy, device=self.device) if augment else None
            for i in range(steps_per_epoch):
                idx = order[i * batch:(i + 1) * batch]
                sym = syms[i * batch:(i + 1) * batch] if augment else None
                net.gather(feats, idx, inp, sym)
                net.gather(targets, idx, tgt, sym)
                self.step += 1
                frac = done / max(1, total - 1)
                lr_i = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
                ffi.reg_fno_train_step(net.h, self.params.data_ptr(), inp.data_ptr(), tgt.data_ptr(),
                                       self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.step,
                                       lr_i, losses.data_ptr() + 8 * i)
                done += 1
            history.append(float(losses.mean().item()))
            if log:
                log(f"epoch {ep + 1}/{epochs}: training loss {history[-1]:.4f}")
        net.close()
        return history

    def evaluate(self, feats, targets, batch=16):
        """Mean relative squared error over a data set (no parameter change)."""
        torch = self.torch
        N, n = feats.shape[0], feats.shape[-1]
        b = min(batch, N)
        net = Network(n, b, self.device)
        inp, tgt = net._f32(feats.shape[1], b, n, n), net._f32(targets.shape[1], b, n, n)
        grad = torch.empty_like(self.params)
        nb = N // b
        losses = torch.zeros(nb, dtype=torch.float64, device=self.device)
        for i in range(nb):
            idx = torch.arange(i * b, (i + 1) * b, dtype=torch.int32, device=self.device)
            net.gather(feats, idx, inp)
            net.gather(targets, idx, tgt)
            net.forward(self.params, inp)
            net.backward(self.params, tgt, grad, losses[i:i + 1])
        out = float(losses.mean().item())
        net.close()
        return out

    def predict(self, mT, mR):
        """(v0, directions) for one pair."""
        n = mT.shape[-1]
        if n not in self._pred:
            self._pred[n] = Network(n, 1, self.device)
        return self._pred[n].predict(self.params, mT, mR)


# ---- data set and evaluation helpers ---------------------------------------------------------------
SOLVER = dict(norm="H2", constraint="mass_source", beta_v=1e-3, beta_w=1e-4, precision="fp32")


def transport_reference(mT, vstar, nt, device, **settings):
    """m_R = m_T transported by v* (the library's FP64 state solve)."""
    import torch
    s = dict(SOLVER, **settings)
    P = Problem(mT, mT, nt, **s)
    m1 = P.state_forward(torch.as_tensor(vstar, dtype=torch.float64, device=device))
    P.close()
    return m1


def tune_shapes(P, device):
    """Pick the launch shapes of a problem with the library's autotuner (at v = 0) and return them."""
    import torch
    v0 = torch.zeros((2, P.n1, P.n2), dtype=torch.float64, device=device)
    P.gradient(v0, want_J=False)
    P.hessian_matvec(v0 + 1e-3)
    return P.autotune(reps=20)["chosen"]


RITZ_BLOCK = 8     # subspace-iteration block for the direction targets (the leading 4 are kept)
RITZ_ITERS = 6


def direction_targets(P, v, seed):
    """Leading REG_FNO_RANK generalised eigenvectors of (H, M) at v (reg_ritz_directions, block of
    RITZ_BLOCK from seeded white noise, RITZ_ITERS steps), FP64 [REG_FNO_RANK][2][n1][n2]."""
    import torch
    P.gradient(v, want_J=False)
    rng = np.random.Generator(np.random.PCG64(seed))
    U0 = torch.as_tensor(rng.standard_normal((RITZ_BLOCK, 2, P.n1, P.n2)), device=v.device)
    U, _ = P.ritz_directions(U0, RITZ_ITERS)
    return U[:ffi.REG_FNO_RANK]


def build_dataset(pairs, nt, device, label_gtol=1e-2, pool=8, log=None, directions=True, seed=0, **settings):
    """Features and plain-solver labels for a list of (m_T, v*) numpy pairs of one grid size.

    Returns (feats [N][9][n][n], labels [N][REG_FNO_OUT][n][n], stats list); the labels are the
    velocities of the plain solves (v0 = 0) to ||g|| / ||g(0)|| <= label_gtol divided by each pair's
    misfit scale, solved `pool` at a time with reg_batch_solve on handles reused through
    reg_set_images (pool 1: one after another on the calling thread), then (with directions) the
    leading generalised eigenvectors of (H, M) at that velocity (``direction_targets``)."""
    import torch
    s = dict(SOLVER, **settings)
    s["lowrank_capacity"] = max(s.get("lowrank_capacity", 0), RITZ_BLOCK)
    N = len(pairs)
    n = pairs[0][0].shape[0]
    feats = torch.empty((N, 9, n, n), dtype=torch.float32, device=device)
    scale = torch.empty(1, dtype=torch.float64, device=device)
    labels = torch.empty((N, ffi.REG_FNO_OUT, n, n), dtype=torch.float32, device=device)
    net = Network(n, 1, device)
    gen = None
    probs = []
    all_stats = []
    t0 = time.perf_counter()
    for c0 in range(0, N, pool):
        chunk = pairs[c0:c0 + pool]
        imgs = []
        for mT_np, vs in chunk:
            mT = torch.as_tensor(mT_np, dtype=torch.float64, device=device)
            if gen is None:
                gen = Problem(mT, mT, nt, **s)
            gen.set_images(mT, mT)
            mR = gen.state_forward(torch.as_tensor(vs, dtype=torch.float64, device=device))
            imgs.append((mT, mR))
        while len(probs) < len(chunk):
            probs.append(Problem(imgs[len(probs)][0], imgs[len(probs)][1], nt, **s))
            if len(probs) == 1:
                shapes = tune_shapes(probs[0], device)
            probs[-1].set_pass_variants(shapes)
        for p, (mT, mR) in zip(probs, imgs):
            p.set_images(mT, mR)
        if pool > 1:
            vs_out, st = batch_solve(probs[:len(chunk)], raise_on_error=False, gtol_rel=label_gtol)
        else:
            vs_out, st = [], []
            for p in probs[:len(chunk)]:
                v, s_ = p.solve(gtol_rel=label_gtol, raise_on_error=False)
                vs_out.append(v)
                st.append(s_)
        for i, (v, (mT, mR)) in enumerate(zip(vs_out, imgs)):
            net.features(mT, mR, feats[c0 + i], scale)
            dirs = direction_targets(probs[i], v, seed + c0 + i) if directions else None
            net.target(v, scale, dirs, labels[c0 + i])
        all_stats += st
        if log and (c0 // pool) % max(1, 1024 // pool) == 0:
            log(f"labels {c0 + len(chunk)}/{N} ({time.perf_counter() - t0:.1f} s)")
    for p in probs:
        p.close()
    if gen is not None:
        gen.close()
    net.close()
    return feats, labels, all_stats


def compare_plain_vs_learned(pairs, nt, ws: WarmStart, device, gtol=1e-2, warmup=1, log=None, recycle=0,
                             **settings):
    """Time to ||g|| / ||g(0)|| <= gtol for every (m_T, v*) pair on one problem handle: the plain solve
    (v0 = 0), the learned warm start (network inference + solve from its v0, which includes g(0) and
    g(v0)) and the learned warm start with the network's directions in the low-rank correction of
    the preconditioner (precond_U).  recycle > 0 also times all three with that many PCG directions
    of each Newton step recycled into the correction.  Returns per-pair records."""
    import torch
    s = dict(SOLVER, **settings)
    s["lowrank_capacity"] = max(s.get("lowrank_capacity", 0), ffi.REG_FNO_RANK + (16 if recycle > 0 else 0))
    recs = []
    P = None
    gen = None

    def timed(**kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kw.pop("learned", False):
            v0, dirs = ws.predict(mT, mR)
            if kw.pop("dirs", False):
                kw["precond_U"] = dirs
            kw["v0"] = v0
        _, st = P.solve(gtol_rel=gtol, raise_on_error=False, **kw)
        return time.perf_counter() - t0, st

    for i, (mT_np, vs) in enumerate(pairs):
        mT = torch.as_tensor(mT_np, dtype=torch.float64, device=device)
        if gen is None:
            gen = Problem(mT, mT, nt, **s)
        gen.set_images(mT, mT)
        mR = gen.state_forward(torch.as_tensor(vs, dtype=torch.float64, device=device))
        if P is None:
            P = Problem(mT, mR, nt, **s)
            tune_shapes(P, device)   # launch shapes for this grid (untimed; kept by the handle)
            for _ in range(warmup):   # graph capture and first-touch costs, not timed
                timed()
                timed(learned=True, dirs=True)
                if recycle > 0:
                    timed(recycle=recycle)
                    timed(learned=True, dirs=True, recycle=recycle)
        P.set_images(mT, mR)
        tp, sp = timed()
        tl, sl = timed(learned=True)
        td, sd = timed(learned=True, dirs=True)
        rec = {"plain_s": tp, "learned_s": tl, "learned_dirs_s": td, "plain": sp, "learned": sl, "learned_dirs": sd}
        if recycle > 0:
            tp, spr = timed(recycle=recycle)
            tl, slr = timed(learned=True, recycle=recycle)
            td, sdr = timed(learned=True, dirs=True, recycle=recycle)
            rec.update({"plain_rc_s": tp, "learned_rc_s": tl, "learned_dirs_rc_s": td, "plain_rc": spr,
                        "learned_rc": slr, "learned_dirs_rc": sdr})
        recs.append(rec)
        if log and i % 32 == 0:
            log(f"pair {i}: plain {1e3 * rec['plain_s']:.1f} ms ({sp['newton_iters']} GN, {sp['pcg_iters']} PCG), "
                f"learned {1e3 * rec['learned_s']:.1f} ms ({sl['newton_iters']} GN, {sl['pcg_iters']} PCG, "
                f"fallback {sl['fallback_used']}), with directions {1e3 * rec['learned_dirs_s']:.1f} ms "
                f"({sd['newton_iters']} GN, {sd['pcg_iters']} PCG)")
    if P is not None:
        P.close()
    if gen is not None:
        gen.close()
    return recs


def summarize(recs):
    """Means over the pairs for every variant in the records (plain, learned, learned with
    directions; with and without recycling), and how often the learned variants beat the plain one."""
    import statistics as stt
    out = {"pairs": len(recs)}
    variants = [k for k in ("plain", "learned", "learned_dirs", "plain_rc", "learned_rc", "learned_dirs_rc")
                if recs and k in recs[0]]
    for k in variants:
        sts = [r[k] for r in recs]
        out[k] = {
            "ms_mean": round(1e3 * stt.mean(r[k + "_s"] for r in recs), 3),
            "ms_median": round(1e3 * stt.median(r[k + "_s"] for r in recs), 3),
            "newton_mean": stt.mean(st["newton_iters"] for st in sts),
            "pcg_mean": stt.mean(st["pcg_iters"] for st in sts),
            "converged": sum(1 for st in sts if st["g_rel"] <= 1e-2 and st["status"] == 0),
            "fallback_rate": stt.mean(st["fallback_used"] for st in sts),
        }
    for k in variants:
        if k.startswith("learned"):
            base = "plain_rc" if k.endswith("_rc") else "plain"
            out[k]["faster_than_" + base] = sum(1 for r in recs if r[k + "_s"] < r[base + "_s"]) / len(recs)
    return out
