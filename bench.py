"""Benchmark: Gauss-Newton Hessian matvecs per second on one MI355X.

Workload (the headline configuration): one image pair on a 256 x 256 periodic grid, n_t = 16 RK2
steps, H2 seminorm with the mass-source constraint (beta_v = 1e-3, beta_w = 1e-4), FP32 transport and
FFTs, FP64 spectral assembly and Krylov vectors.  Synthetic inputs (seeded blob-plus-texture template,
band-limited velocity scaled to CFL 0.8); the reference image is the template transported by that
velocity, computed on the GPU.

A step is one PCG iteration of Alg. 2 at a fixed linearisation point: one GN Hessian matvec
(incremental state solve forward, GN incremental adjoint solve backward, body-force quadrature,
regularisation + projection assembly), one preconditioner application and the FP64 PCG inner
products and vector updates.  ``value`` = steps per second = matvecs per second.

Also reported: the dominant kernel's achieved HBM bandwidth against the 8 TB/s peak (hipEvents around
its launches inside real matvecs on the library's stream), the time to ||g||/||g(0)|| <= 1e-2 of the
plain solver on the same workload, matvec throughput and roofline fraction at 1024^2 / n_t = 32, the
learned warm start (config 5: a Fourier network trained on the GPU by the library's kernels on 4096
plain-solver registrations at 128^2, then plain vs learned time to ||g||/||g(0)|| <= 1e-2 on 256
unseen pairs at 256^2), and the FP64 CPU oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources of the dominant kernel; counter-derived traffic is reported only while these are unchanged
KERNEL_SOURCES = ["paper_1503_00757_amd/csrc/transport_kernels.hpp", "paper_1503_00757_amd/csrc/device_common.hpp",
                  "paper_1503_00757_amd/csrc/transport_op_a2.hip", "paper_1503_00757_amd/csrc/kernels.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by its plain-copy calibration factor), or None when the
    kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or t.get("source_sha256") != kernel_source_hash():
        return None
    return e["fetch_bytes"] + e["write_bytes"]


def tune(P, cache: str | None):
    """Pick launch shapes (untimed): reuse a cached choice when given, else run the autotuner."""
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            chosen = json.load(fh)["chosen"]
        P.set_pass_variants(chosen)
        return chosen
    rep = P.autotune(reps=50)
    if cache:
        with open(cache, "w") as fh:
            json.dump(rep, fh)
    return rep["chosen"]


def setup(config: int, precision: str = "fp32", tune_cache: str | None = None):
    import numpy as np
    import torch
    import synthdata as sd
    from paper_1503_00757_amd import Problem

    w = sd.make_workload(config)
    dev = torch.device("cuda:0")
    mT = torch.tensor(w.mT, device=dev)
    # reference image: the template transported by v* (state solve on the GPU)
    P0 = Problem(mT, mT.clone(), w.nt, w.norm, w.constraint, w.beta_v, w.beta_w, precision)
    mR = P0.state_forward(torch.tensor(w.vstar, device=dev))
    P0.close()
    P = Problem(mT, mR, w.nt, w.norm, w.constraint, w.beta_v, w.beta_w, precision,
                lowrank_capacity=LOWRANK_CAPACITY)
    vlin = torch.tensor(0.5 * w.vstar, device=dev)
    vt = torch.tensor(w.vtilde, device=dev)
    P.gradient(vlin, want_J=False)
    P.hessian_matvec(vt)
    P.tuned = tune(P, tune_cache)
    return w, P, vlin, vt


def bench_pcg(P, vlin, steps, warmup, windows=5):
    """`warmup` untimed PCG iterations, then `windows` timed windows of exactly `steps` iterations
    each (fixed schedule: no host round trip inside a window), every window bracketed by device
    synchronisation.  Returns the median window's seconds and all window times."""
    import torch
    g, _ = P.gradient(vlin, want_J=False)
    rhs = -g
    if warmup > 0:
        P.pcg(rhs, eta=0.0, max_iters=warmup, fixed_iters=warmup)
    times = []
    for _ in range(windows):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, it, _ = P.pcg(rhs, eta=0.0, max_iters=steps, fixed_iters=steps)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        assert it == steps
    return sorted(times)[len(times) // 2], times


def bench_matvec(P, vt, reps):
    import torch
    out = P.vec()
    P.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def copy_bandwidth(mib=1024, reps=10):
    """Measured device-to-device copy bandwidth (read + write bytes / time) of a plain torch copy of
    `mib` MiB, timed with events on the current stream: the practical HBM ceiling next to the 8 TB/s
    specification."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)


def roofline(P, reps=None, workload="c2"):
    """Dominant kernel: the fused GN incremental-adjoint stage-2 launch (stage_fused_kernel<..., OP_A2>):
    row blocks read 10 and write 3 fields (incl. the body-force accumulation), column blocks read 3
    and write 1.  Its launches are timed inside real matvecs on the library's stream with events the
    dispatch stamps (reg_time_pass)."""
    ms, by, ex = P.time_pass(0, reps or max(1, 256 // P.nt))   # ~256 timed launches
    achieved = by / (ms * 1e-3) / 1e9
    # phase mode (reg_time_phases): every block stamps its loads' arrival and the end of its
    # transforms after waiting for them, so the phases run one after another; their lengths, not
    # the overlapped launch above
    phases = {k: round(v, 3) for k, v in P.time_phases(0, max(1, 128 // P.nt)).items()}
    return {"kernel": "stage_fused_kernel<float, N, ..., OP_A2> (GN incremental adjoint, RK2 stage 2)",
            "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(workload),
            "bytes_per_launch": by, "us_per_launch": round(ms * 1e3, 3),
            # the blocks' own execution interval (device clock), without the dispatch ramp and the
            # end-of-kernel completion that the launch duration above includes
            "exec_us_per_launch": round(ex * 1e3, 3),
            "exec_achieved": round(by / (ex * 1e-3) / 1e9, 2),
            "phase_mode_us_per_launch": phases}


LOWRANK_CAPACITY = 16   # directions of the preconditioner correction the bench problems can hold


def moved_bytes_per_matvec(nt, nn):
    """Compulsory bytes the implemented GN matvec moves (each operand read once, each result written
    once), incompressible H1 case, in FP32 fields of 4 N bytes: incremental state stage 1 13 fields
    (none at j = 0, where m~_0 = 0 makes it pointwise), stage 2 13 (14 at j = 0, which forms m~*_0
    from v~ . grad m_0), GN adjoint stage 1 9 and stage 2 17 (none at j = 0: its body-force term is
    folded into the assembly): 52 n_t - 29 fields.  The real-space Nyquist projection of the input
    (two FP64 reads, FP64 and FP32 writes: 56 N) and the FP64 assembly (row forward: v~ 16 N and
    the nine FP32 fields of the last body-force term 36 N in, 32 N out; column pass 32 N in, 16 N out;
    row inverse 16 N in, 16 N out: 164 N)."""
    return (4 * (52 * nt - 29) + 56 + 164) * nn


def bench_solve(P, recycle=0, diagnostics=False):
    """Alg. 1 to ||g||/||g(0)|| <= 1e-2 from v = 0; recycle > 0 keeps that many PCG directions of each
    Newton step in the low-rank correction of the preconditioner (one untimed run first: graph
    capture).  diagnostics: also det F_1 of the solution (reg_deformation) and its time."""
    import torch
    P.solve(max_newton=50, max_pcg=100, gtol_rel=1e-2, recycle=recycle)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v, st = P.solve(max_newton=50, max_pcg=100, gtol_rel=1e-2, recycle=recycle)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"seconds": round(dt, 4), "newton_iters": st["newton_iters"], "pcg_iters": st["pcg_iters"],
           "n_matvec": st["n_matvec"], "n_pde": st["n_pde"], "g_rel": st["g_rel"], "status": st["status"]}
    if diagnostics:
        P.deformation(v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, (mn, mx, mean) = P.deformation(v)
        out["det_F1"] = {"min": round(mn, 5), "max": round(mx, 5), "mean": round(mean, 6),
                         "diagnostics_ms": round(1e3 * (time.perf_counter() - t0), 3)}
    return out


def bench_hessians(config=2):
    """Alg. 1 on one workload with the Gauss-Newton Hessian of the paper and with the full-Newton
    Hessian (REG_HESS_FULL), to ||g||/||g(0)|| <= 1e-2 and 1e-4 (one untimed solve first each), for
    the reference m_T(v*) and for that reference plus an intensity change no velocity explains."""
    import torch
    import synthdata as sd
    from paper_1503_00757_amd import Problem
    w = sd.make_workload(config)
    dev = torch.device("cuda:0")
    mT = torch.tensor(w.mT, device=dev)
    P0 = Problem(mT, mT.clone(), w.nt, w.norm, w.constraint, w.beta_v, w.beta_w, "fp32")
    mR = P0.state_forward(torch.tensor(w.vstar, device=dev))
    P0.close()
    out = {}
    refs = {"exact_reference": mR,
            "changed_reference": mR + torch.tensor(sd.reference_change(w.n1, w.n2), device=dev)}
    for name, ref in refs.items():
        for hess in ("gn", "full"):
            P = Problem(mT, ref, w.nt, w.norm, w.constraint, w.beta_v, w.beta_w, "fp32", hessian=hess)
            for gtol in (1e-2, 1e-4):
                P.solve(max_newton=50, max_pcg=100, gtol_rel=gtol, raise_on_error=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = P.solve(max_newton=50, max_pcg=100, gtol_rel=gtol, raise_on_error=False)
                torch.cuda.synchronize()
                out.setdefault(name, {})[f"{hess}_to_{gtol:g}"] = {
                    "seconds": round(time.perf_counter() - t0, 4), "newton_iters": st["newton_iters"],
                    "pcg_iters": st["pcg_iters"], "n_pde": st["n_pde"], "g_rel": st["g_rel"],
                    "status": st["status"]}
            P.close()
    return out


def bench_shear_control(n=256, nt=16, beta_v=1e-4):
    """The shear-control model on a self-made sliding-interface pair (two bands sliding past each other,
    divergence-free; synthdata.sliding_pair): Alg. 1 to ||g||/||g(0)|| <= 1e-2 with the linear H1 model
    and the nonlinear model at the paper's exponents nu = 1/2, 3, 5 (eps = 1e-4), incompressible.  Reports
    time, iterations, the remaining misfit ||m_R - m_1|| / ||m_R - m_T||, the largest shear strain
    |E_12| of the solution (v*: the generating one) and the range of det F_1."""
    import numpy as np
    import torch
    import synthdata as sd
    from paper_1503_00757_amd import Problem
    w = sd.sliding_pair(n, nt)
    dev = torch.device("cuda:0")
    mT = torch.tensor(w.mT, device=dev)
    P0 = Problem(mT, mT.clone(), nt, "H1", "divfree", beta_v, 0.0, "fp32")
    mR = P0.state_forward(torch.tensor(w.vstar, device=dev))
    P0.close()
    mis0 = float(torch.linalg.norm(mR - mT))
    k = np.fft.fftfreq(n, 1.0 / n)
    k[n // 2] = 0.0

    def shear(v):   # max |E_12| = max |(d2 v1 + d1 v2)/2| (analysis of the result, host FFT)
        d = lambda u, ax: np.real(np.fft.ifft(1j * k * np.fft.fft(u, axis=ax), axis=ax))   # noqa: E731
        return float(np.abs(0.5 * (d(v[0], 1) + d(v[1], 0))).max())

    out = {"workload": f"sliding interfaces {n}^2, n_t={nt}, beta_v={beta_v:g}; divergence-free unless named "
                       "mass_source (relaxed incompressibility, beta_w=1e-3)",
           "vstar_max_shear": round(shear(w.vstar), 4)}
    divfree = dict(constraint="divfree", beta_w=0.0)
    for name, kw in (("H1", dict(norm="H1", **divfree)), ("stokes_nu0.5", dict(norm="stokes", nu=0.5, eps=1e-4, **divfree)),
                     ("stokes_nu3", dict(norm="stokes", nu=3.0, eps=1e-4, **divfree)),
                     ("stokes_nu5", dict(norm="stokes", nu=5.0, eps=1e-4, **divfree)),
                     ("stokes_nu3_mass_source", dict(norm="stokes", nu=3.0, eps=1e-4, constraint="mass_source",
                                                     beta_w=1e-3))):
        P = Problem(mT, mR, nt, beta_v=beta_v, precision="fp32", **kw)
        P.solve(max_newton=50, max_pcg=100, gtol_rel=1e-2, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v, st = P.solve(max_newton=50, max_pcg=100, gtol_rel=1e-2, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        m1 = P.state_forward(v)
        _, _, _, (mn, mx, mean) = P.deformation(v)
        out[name] = {"seconds": round(dt, 4), "newton_iters": st["newton_iters"], "pcg_iters": st["pcg_iters"],
                     "status": st["status"], "misfit_rel": round(float(torch.linalg.norm(mR - m1)) / mis0, 5),
                     "max_shear": round(shear(v.cpu().numpy()), 4), "det_F1_min_max": [round(mn, 5), round(mx, 5)]}
        P.close()
    return out


def bench_grid_sizes():
    """Grids that are not powers of two (mixed-radix 2/3/5 transforms) against the nearest power of
    two: GN matvec time per grid point at 128 x 150 vs 128 x 128 (n_t = 16) and 1000^2 vs 1024^2
    (n_t = 32), H1 + divergence-free, FP32 transport, seeded blob-plus-texture images, default launch
    shapes on both sides (median of 5 timed batches of graph-replayed matvecs)."""
    import numpy as np
    import torch
    import synthdata as sd
    from paper_1503_00757_amd import Problem
    dev = torch.device("cuda:0")
    out = {}
    for (n1, n2, nt, ref) in ((128, 150, 16, (128, 128)), (1000, 1000, 32, (1024, 1024))):
        per_point = {}
        for (a, b) in ((n1, n2), ref):
            rng = np.random.Generator(np.random.PCG64(sd.BASE_SEED + 600 + a + b))
            mT = sd.template_image(a, b, 16, 16, rng)
            vs = sd.scale_to_cfl(sd.random_velocity(a, b, 8, rng, divfree=True), nt, 0.8)
            vt = sd.unit_l2(sd.random_velocity(a, b, 8, rng, divfree=True))
            mTd = torch.tensor(mT, device=dev)
            P0 = Problem(mTd, mTd.clone(), nt, "H1", "divfree", 1e-3, 0.0, "fp32")
            mR = P0.state_forward(torch.tensor(vs, device=dev))
            P0.close()
            P = Problem(mTd, mR, nt, "H1", "divfree", 1e-3, 0.0, "fp32")
            P.gradient(torch.tensor(0.5 * vs, device=dev), want_J=False)
            reps = 20 if a * b > 500000 else 100
            ts = sorted(bench_matvec(P, torch.tensor(vt, device=dev), reps) for _ in range(5))
            P.close()
            per_point[f"{a}x{b}"] = {"ms_per_matvec": round(ts[2] * 1e3, 4),
                                     "ns_per_point": round(ts[2] * 1e9 / (a * b), 4)}
        k0, k1 = f"{n1}x{n2}", f"{ref[0]}x{ref[1]}"
        per_point["per_point_ratio"] = round(per_point[k0]["ns_per_point"] / per_point[k1]["ns_per_point"], 3)
        out[f"{k0}_vs_{k1}_nt{nt}"] = per_point
    return out


def bench_batch(npairs=96):
    """Config 4: 96 pairs (32 each at 128^2, 256^2, 512^2; beta_v log-uniform in [1e-4, 1e-2]; n_t in
    {8, 16, 32}; H1 + divergence-free), all solved to ||g||/||g(0)|| <= 1e-2 by reg_batch_solve.
    Reports wall time (inputs resident, problems created, untimed tuning excluded) and aggregate
    matvecs/s, next to the same pairs solved one after another."""
    import torch
    import synthdata as sd
    from paper_1503_00757_amd import Problem, batch_solve
    dev = torch.device("cuda:0")
    probs = []
    for i in range(npairs):
        w = sd.make_workload(4, pair=i)
        mT = torch.tensor(w.mT, device=dev)
        P0 = Problem(mT, mT.clone(), w.nt, w.norm, w.constraint, w.beta_v, w.beta_w, "fp32")
        mR = P0.state_forward(torch.tensor(w.vstar, device=dev))
        P0.close()
        probs.append((w, Problem(mT, mR, w.nt, w.norm, w.constraint, w.beta_v, w.beta_w, "fp32",
                                 lowrank_capacity=LOWRANK_CAPACITY)))
    torch.cuda.synchronize()
    print(f"[bench] c4: {npairs} problems created", file=sys.stderr, flush=True)
    Ps = [P for _, P in probs]
    # launch shapes: tune one problem per grid size (untimed) and give the choice to the others
    chosen = {}
    for w, P in probs:
        if w.n1 not in chosen:
            v0 = torch.zeros((2, w.n1, w.n2), dtype=torch.float64, device=dev)
            P.gradient(v0, want_J=False)
            P.hessian_matvec(v0 + 1e-3)
            chosen[w.n1] = P.autotune(reps=20)["chosen"]
        P.set_pass_variants(chosen[w.n1])
    t0 = time.perf_counter()
    vs, stats = batch_solve(Ps, max_newton=50, max_pcg=100, gtol_rel=1e-2, raise_on_error=False)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    nmv = sum(s["n_matvec"] for s in stats)
    ok = sum(1 for s in stats if s["status"] == 0 and s["g_rel"] <= 1e-2)
    print(f"[bench] c4 batched {t_batch:.2f}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for P in Ps:
        P.solve(max_newton=50, max_pcg=100, gtol_rel=1e-2, raise_on_error=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    sizes = {}
    for (w, _), s in zip(probs, stats):
        d = sizes.setdefault(w.n1, {"pairs": 0, "matvecs": 0, "newton": 0})
        d["pairs"] += 1
        d["matvecs"] += s["n_matvec"]
        d["newton"] += s["newton_iters"]
    # the same batch with 4 recycled PCG directions per Newton step in the preconditioner correction
    batch_solve(Ps, max_newton=50, max_pcg=100, gtol_rel=1e-2, raise_on_error=False, recycle=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats_rc = batch_solve(Ps, max_newton=50, max_pcg=100, gtol_rel=1e-2, raise_on_error=False, recycle=4)
    torch.cuda.synchronize()
    t_rc = time.perf_counter() - t0
    recycled = {"seconds": round(t_rc, 3), "total_matvecs": sum(s_["n_matvec"] for s_ in stats_rc),
                "converged": sum(1 for s_ in stats_rc if s_["status"] == 0 and s_["g_rel"] <= 1e-2)}
    for P in Ps:
        P.close()
    return {"metric": "96-pair batched solve to ||g||/||g(0)|| <= 1e-2 (config 4)", "value": round(t_batch, 3),
            "unit": "s", "higher_is_better": False, "pairs": npairs, "converged": ok, "total_matvecs": nmv,
            "matvecs_per_s": round(nmv / t_batch, 1), "sequential_seconds": round(t_seq, 3),
            "speedup_vs_sequential": round(t_seq / t_batch, 2), "per_size": sizes, "launch_shapes": chosen,
            "with_recycled_directions": recycled,
            "data": "synthetic"}


def c3_matvec(w3, P3, vlin3, vt3, copy_gbs):
    """GN matvec throughput at 1024^2, n_t = 32 (reg_hessian_matvec: the Nyquist projection of the
    input and the graph-replayed matvec), as the median of 5 timed batches of 20, against the per-step
    byte model of the matvec (248 N per step + 112 N) and against the bytes the kernels move."""
    P3.gradient(vlin3, want_J=False)
    reps3 = sorted(bench_matvec(P3, vt3, 20) for _ in range(5))
    t3 = reps3[2]
    nn = w3.n1 * w3.n2
    bmodel = (248 * w3.nt + 112) * nn
    bmoved = moved_bytes_per_matvec(w3.nt, nn)
    rl3 = roofline(P3, workload="c3")
    return {"matvecs_per_s": round(1.0 / t3, 2), "ms_per_matvec": round(t3 * 1e3, 3),
            "ms_per_matvec_min_max_of_5": [round(reps3[0] * 1e3, 3), round(reps3[-1] * 1e3, 3)],
            "model_bytes_per_matvec": bmodel,
            "model_frac_of_8TBs": round(bmodel / t3 / 8e12, 4),
            "model_frac_of_measured_copy": round(bmodel / t3 / (copy_gbs * 1e9), 4),
            "moved_bytes_per_matvec": bmoved,
            "moved_frac_of_8TBs": round(bmoved / t3 / 8e12, 4),
            "launch_shapes": P3.tuned,
            "dominant_kernel": rl3}


def _single_thread():
    """Pool-worker initialiser: one BLAS / OpenMP thread per worker (set before numpy loads in the
    worker, which is when its thread pools are sized)."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    import numpy  # noqa: F401
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _warmstart_pair(args):
    import synthdata as sd
    p, n = args
    w = sd.warmstart_pair(p, n)
    return w.mT, w.vstar


def warmstart_pairs(ntrain, ntest, ntr=128, nte=256, nval=256):
    """Seeded pairs of the warm-start data set, drawn on the host cores before the GPU is touched:
    training pairs 0..ntrain-1 at ntr^2, a separate held-out set from index 50000 on at ntr^2, unseen
    test pairs from index 100000 on at nte^2."""
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 4))
    with ProcessPoolExecutor(workers, initializer=_single_thread) as ex:
        train = list(ex.map(_warmstart_pair, [(p, ntr) for p in range(ntrain)], chunksize=32))
        val = list(ex.map(_warmstart_pair, [(50000 + p, ntr) for p in range(nval)], chunksize=16))
        test = list(ex.map(_warmstart_pair, [(100000 + p, nte) for p in range(ntest)], chunksize=4))
    return train, val, test


def bench_warmstart(train, val, test, epochs=60, label_gtol=1e-3, label_pool=16):
    """Config 5: label the training pairs with the plain solver, train the warm-start network with the
    library's kernels (Adam, batch 16, grid-symmetry augmentation), then time the plain and the
    learned solve (network inference + solve from its v0, which includes g(0) and g(v0)) to
    ||g||/||g(0)|| <= 1e-2 on every unseen test pair, on one problem handle."""
    import torch
    import synthdata as sd
    from paper_1503_00757_amd import warmstart as W
    dev = torch.device("cuda:0")
    log = lambda m: print(f"[bench] c5 {m}", file=sys.stderr, flush=True)   # noqa: E731
    t0 = time.perf_counter()
    feats, labels, st = W.build_dataset(train, 16, dev, label_gtol=label_gtol, pool=label_pool, log=log)
    vfeats, vlabels, _ = W.build_dataset(val, 16, dev, label_gtol=label_gtol, pool=label_pool)
    torch.cuda.synchronize()
    t_labels = time.perf_counter() - t0
    ws = W.WarmStart(sd.network_init(), dev)
    nval = len(val)
    t0 = time.perf_counter()
    hist = ws.train(feats, labels, epochs, batch=16,
                    log=lambda m: log(m) if m.startswith("epoch") and int(m.split()[1].split("/")[0]) % 10 == 0 else None)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = epochs * (len(train) // 16)
    val = ws.evaluate(vfeats, vlabels)
    vlabels[:, 2:] = 0.0   # without direction targets the loss is the velocity term alone
    val_v = ws.evaluate(vfeats, vlabels)
    del feats, labels, vfeats, vlabels
    # inference latency at the test size (features + network + rescale), events on the current stream
    mT = torch.tensor(test[0][0], device=dev)
    ws.predict(mT, mT)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        ws.predict(mT, mT)
    e1.record()
    torch.cuda.synchronize()
    t_inf = e0.elapsed_time(e1) / 20
    log(f"comparing plain vs learned on {len(test)} unseen pairs")
    recs = W.compare_plain_vs_learned(test, 16, ws, dev, log=log, recycle=4)
    s = W.summarize(recs)
    # tighter solves (more PCG iterations per Newton step, the same fixed set-up cost of the directions)
    log("tight tolerance 1e-3 on 64 of the test pairs")
    tight = W.summarize(W.compare_plain_vs_learned(test[:64], 16, ws, dev, gtol=1e-3))
    ratio = lambda a, b: round(s[b]["ms_mean"] / s[a]["ms_mean"], 3)   # noqa: E731  (speed-up of a over b)
    return {
        "protocol": f"train {len(train)} pairs at {train[0][0].shape[0]}^2 (a separate {nval} held out), "
                    f"{epochs} epochs; test {len(test)} unseen pairs at {test[0][0].shape[0]}^2; "
                    "H2 + mass source, beta_v=1e-3, beta_w=1e-4, n_t=16, FP32 transport; targets: v/s and the "
                    f"leading {W.ffi.REG_FNO_RANK} generalised eigenvectors of (H, M) at the label solution",
        # means over the test pairs: plain (v0 = 0), learned v0, learned v0 + learned directions in
        # the preconditioner correction; *_rc: the same with 4 recycled PCG directions per Newton step
        "variants": {k: s[k] for k in ("plain", "learned", "learned_dirs", "plain_rc", "learned_rc",
                                       "learned_dirs_rc")},
        "speedup_mean": {"learned_vs_plain": ratio("learned", "plain"),
                         "learned_dirs_vs_learned": ratio("learned_dirs", "learned"),
                         "learned_dirs_vs_plain": ratio("learned_dirs", "plain"),
                         "learned_rc_vs_plain_rc": ratio("learned_rc", "plain_rc"),
                         "learned_dirs_rc_vs_learned_rc": ratio("learned_dirs_rc", "learned_rc"),
                         "learned_dirs_rc_vs_plain_rc": ratio("learned_dirs_rc", "plain_rc")},
        "tight_grel_1e-3_64_pairs": {k: {"ms_mean": tight[k]["ms_mean"], "pcg_mean": tight[k]["pcg_mean"],
                                         "newton_mean": tight[k]["newton_mean"]}
                                     for k in ("plain", "learned", "learned_dirs")},
        "label_seconds": round(t_labels, 2), "train_seconds": round(t_train, 2), "train_steps": steps,
        "train_ms_per_step_batch16": round(t_train / steps * 1e3, 3),
        "train_loss_last_epoch": round(hist[-1], 5), "heldout_loss": round(val, 5),
        # split of the held-out loss: velocity relative squared error, and the mean cos^2 between a
        # predicted direction and its target (angle terms = DIR_WEIGHT (1 - mean cos^2))
        "heldout_velocity_rel_sq_error": round(val_v, 5),
        "heldout_direction_mean_cos2": round(1.0 - (val - val_v) / W.ffi.REG_FNO_DIR_WEIGHT, 4),
        "inference_ms": round(t_inf, 3),
    }


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle's GN matvec on the host cores (bounded sample of the same workload)."""
    import numpy as np
    import synthdata as sd
    from oracle import Grid, Params, reduced, transport, spectral
    w = sd.make_workload(2)
    p = Params(w.n1, w.n2, w.nt, w.norm, w.constraint, w.beta_v, w.beta_w)
    g = Grid(w.n1, w.n2)
    spectral.set_workers(-1)
    mR = transport.state_forward(g, p, w.mT, w.vstar).m[-1]
    lin = reduced.gradient(g, p, w.mT, mR, 0.5 * w.vstar)
    reduced.hessian_matvec(g, p, lin, w.vtilde)   # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        reduced.hessian_matvec(g, p, lin, w.vtilde)
        n += 1
        dt = time.perf_counter() - t0
        if dt > budget_s or n >= 200:
            break
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    all_cores = n / dt
    # the same matvec with one scipy.fft worker (faster on small transforms: no thread hand-off)
    spectral.set_workers(1)
    n1 = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 6.0 and n1 < 80:
        reduced.hessian_matvec(g, p, lin, w.vtilde)
        n1 += 1
    dt1 = time.perf_counter() - t0
    one = n1 / dt1
    spectral.set_workers(-1)
    # the baseline is the faster of the two setups, with the threads that setup used
    if one >= all_cores:
        out = {"value": round(one, 3), "unit": "matvecs/s", "cores": 1, "kind": "oracle",
               "sample": f"{n1} FP64 oracle GN matvecs (numpy/scipy.fft, one worker) on the 256^2, n_t=16 "
                         f"workload at its linearisation point, {dt1:.1f} s"}
    else:
        out = {"value": round(all_cores, 3), "unit": "matvecs/s", "cores": cores, "kind": "oracle",
               "sample": f"{n} FP64 oracle GN matvecs (numpy/scipy.fft, all cores) on the 256^2, n_t=16 "
                         f"workload at its linearisation point, {dt:.1f} s"}
    out["all_cores_matvecs_per_s"] = round(all_cores, 3)
    out["all_cores_threads"] = cores
    out["single_worker_matvecs_per_s"] = round(one, 3)
    # the oracle's full solves of configs 1 and 2
    from oracle import solver
    w1 = sd.make_workload(1)
    p1 = Params(w1.n1, w1.n2, w1.nt, w1.norm, w1.constraint, w1.beta_v, w1.beta_w)
    g1 = Grid(w1.n1, w1.n2)
    mR1 = transport.state_forward(g1, p1, w1.mT, w1.vstar).m[-1]
    t0 = time.perf_counter()
    solver.solve(g1, p1, w1.mT, mR1, solver.SolveOpts(max_newton=5, fixed_pcg_iters=10, gtol_rel=0.0))
    out["solve_c1_5x10_seconds"] = round(time.perf_counter() - t0, 3)
    t0 = time.perf_counter()
    _, st = solver.solve(g, p, w.mT, mR, solver.SolveOpts(max_newton=50, gtol_rel=1e-2))
    out["solve_c2_to_grel_1e-2_seconds"] = round(time.perf_counter() - t0, 3)
    out["solve_c2_pcg_iters"] = st.pcg_iters
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the solve and 1024^2 measurements")
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5", "grids"], default="c2",
                    help="c2: 256^2 headline workload (default); c3: 1024^2, n_t=32 (profiling); "
                         "c4: 96-pair batched solve; c5: learned warm start alone")
    ap.add_argument("--no-warmstart", action="store_true", help="skip the learned warm-start leg (config 5)")
    ap.add_argument("--warmstart-train", type=int, default=4096)
    ap.add_argument("--warmstart-test", type=int, default=256)
    ap.add_argument("--warmstart-epochs", type=int, default=60)
    ap.add_argument("--warmstart-label-pool", type=int, default=16,
                    help="pairs labelled concurrently (reg_batch_solve); 1 = one after another")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file with launch shapes chosen by an earlier run (written if missing)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (HBM-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the single-pair path "
              "does not shard across GPUs; see the design notes for how it would)", file=sys.stderr)
        sys.exit(2)
    ws_pairs = None
    if args.workload == "c5" or (args.workload == "c2" and not args.no_extras and not args.no_warmstart):
        t0 = time.perf_counter()
        ws_pairs = warmstart_pairs(args.warmstart_train, args.warmstart_test)
        print(f"[bench] c5 pairs drawn in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    import torch
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: 3 copies of {args.copy_probe_mib} MiB (read + write each)", file=sys.stderr,
              flush=True)
        del a, b
    if args.workload == "c4":
        print(json.dumps(bench_batch()))
        return
    if args.workload == "grids":
        print(json.dumps(bench_grid_sizes()))
        return
    if args.workload == "c5":
        r = bench_warmstart(*ws_pairs, epochs=args.warmstart_epochs, label_pool=args.warmstart_label_pool)
        t = r["variants"]
        print(json.dumps({"metric": "time to ||g||/||g(0)|| <= 1e-2 at 256^2, learned warm start and directions "
                                    "(config 5)",
                          "value": t["learned_dirs"]["ms_mean"], "unit": "ms", "higher_is_better": False,
                          "plain_value": t["plain"]["ms_mean"], "n_gpus": 1, "dtype": "f32 transport, bf16 network",
                          "data": "synthetic", **r}))
        return
    cfg = 2 if args.workload == "c2" else 3
    print(f"[bench] workload {args.workload} setup", file=sys.stderr, flush=True)
    w, P, vlin, vt = setup(cfg, tune_cache=args.tune_cache)
    dt, windows = bench_pcg(P, vlin, args.steps, args.warmup)
    print(f"[bench] pcg {len(windows)} windows of {args.steps} steps, median {dt:.4f}s", file=sys.stderr, flush=True)
    rl = roofline(P, workload=args.workload)
    copy_gbs = copy_bandwidth()
    rl["measured_copy_GBs"] = copy_gbs
    rl["frac_of_measured_copy"] = round(rl["achieved"] / copy_gbs, 4)
    tuned = P.tuned
    extras = {}
    if not args.no_extras:
        extras["matvec_only_per_s"] = round(1.0 / bench_matvec(P, vt, 50), 2)
        print("[bench] solve", file=sys.stderr, flush=True)
        extras["solve_to_grel_1e-2_plain"] = bench_solve(P, diagnostics=True)
        extras["solve_to_grel_1e-2_recycle4"] = bench_solve(P, recycle=4)
        print("[bench] Gauss-Newton vs full-Newton solves", file=sys.stderr, flush=True)
        extras["gauss_newton_vs_full_newton"] = bench_hessians(cfg)
        print("[bench] shear-control regularisation", file=sys.stderr, flush=True)
        extras["shear_control_sliding"] = bench_shear_control()
        extras["shear_control_sliding_512"] = bench_shear_control(n=512, nt=16)
        print("[bench] grids that are not powers of two", file=sys.stderr, flush=True)
        extras["non_power_of_two_grids"] = bench_grid_sizes()
    if cfg == 3:
        extras["c3_1024sq_nt32"] = c3_matvec(w, P, vlin, vt, copy_gbs)
    P.close()
    if not args.no_extras and cfg == 2:
        print("[bench] 1024^2 nt=32", file=sys.stderr, flush=True)
        w3, P3, vlin3, vt3 = setup(3)
        extras["c3_1024sq_nt32"] = c3_matvec(w3, P3, vlin3, vt3, copy_gbs)
        P3.close()
        print("[bench] c4 batched solve of 96 pairs", file=sys.stderr, flush=True)
        extras["c4_batched_96_pairs"] = bench_batch()
    if ws_pairs is not None:
        print("[bench] c5 learned warm start", file=sys.stderr, flush=True)
        extras["c5_warm_start"] = bench_warmstart(*ws_pairs, epochs=args.warmstart_epochs,
                                                  label_pool=args.warmstart_label_pool)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    if cfg == 3:
        wl = ("c3: one pair, 1024x1024 periodic grid, n_t=32, H1 + divergence-free, beta_v=1e-4; FP32 "
              "transport/FFT, FP64 assembly and PCG; step = one PCG iteration")
    else:
        wl = ("c2: one pair, 256x256 periodic grid, n_t=16, H2 + mass source, beta_v=1e-3, "
              "beta_w=1e-4; FP32 transport/FFT, FP64 assembly and PCG; step = one PCG "
              "iteration (1 GN matvec + preconditioner + FP64 PCG updates)")
    out = {
        "metric": f"GN Hessian matvecs/s at {w.n1}^2", "value": round(args.steps / dt, 2), "unit": "matvecs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl, "n1": w.n1, "n2": w.n2, "nt": w.nt},
        "roofline": rl,
        "cpu_baseline": cpu,
        "launch_shapes": tuned,
        # the timed region: 5 windows of exactly `steps` PCG iterations; `value` is from the median one
        "window_ms": [round(t * 1e3, 4) for t in windows],
    }
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
