"""What the trained warm-start network gains over the plain solver (GPU).

A network is trained by the library's own kernels on plain-solver registrations of 512 seeded pairs
at 64^2 (the warm-start data generator, labels solved to ||g|| / ||g(0)|| <= 1e-3, direction
targets from reg_ritz_directions at the label), then the plain solver, the learned warm start and
the learned warm start with the learned directions in the preconditioner correction run on 12
unseen pairs at 128^2 to ||g|| / ||g(0)|| <= 1e-2 on one handle.  The learned solve pays for the
network inference and the extra gradient at v0, and must still need fewer PDE solves and less time
than the plain one; the learned directions must not add PCG iterations.
"""
import numpy as np
import pytest

import synthdata

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_trained_network_beats_plain_solver(dev):
    from paper_1503_00757_amd import warmstart as W
    train = [(w.mT, w.vstar) for w in (synthdata.warmstart_pair(p, 64) for p in range(512))]
    feats, labels, st = W.build_dataset(train, 16, dev, label_gtol=1e-3, pool=16)
    assert all(s["status"] == 0 for s in st)
    ws = W.WarmStart(synthdata.network_init(), dev)
    hist = ws.train(feats[:480], labels[:480], 40, batch=16)
    assert hist[-1] < 0.2 * hist[0], hist
    val = ws.evaluate(feats[480:], labels[480:])
    assert val < 0.2, val      # held-out relative squared error of v / s
    test = [(w.mT, w.vstar) for w in (synthdata.warmstart_pair(100000 + p, 128) for p in range(12))]
    recs = W.compare_plain_vs_learned(test, 16, ws, dev)
    s = W.summarize(recs)
    print(s)
    assert s["plain"]["converged"] == s["learned"]["converged"] == s["learned_dirs"]["converged"] == len(test)
    assert s["learned"]["newton_mean"] < s["plain"]["newton_mean"]
    assert sum(r["learned"]["n_pde"] for r in recs) < sum(r["plain"]["n_pde"] for r in recs)
    ratio = np.mean([r["learned_s"] / r["plain_s"] for r in recs])
    assert ratio < 1.0, ratio
    # the learned directions feed the preconditioner correction: no more PCG iterations than the
    # learned warm start alone (the correction is SPD for any directions; trained ones deflate)
    assert s["learned_dirs"]["pcg_mean"] <= s["learned"]["pcg_mean"], s
