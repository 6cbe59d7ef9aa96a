"""Checkpoint files and the per-Newton-step log, on the host (no device work): the Newton state and
the training state survive a save / load round trip exactly, files load without unpickling, and
the step log writes one JSON line per record."""
import json

import numpy as np
import pytest

from paper_1503_00757_amd import checkpoint
from paper_1503_00757_amd.problem import write_step_log

torch = pytest.importorskip("torch")


def test_newton_state_round_trip(tmp_path):
    rng = np.random.Generator(np.random.PCG64(7))
    v = rng.standard_normal((2, 16, 12))
    path = tmp_path / "newton.npz"
    checkpoint.save_newton(path, torch.tensor(v), newton_iters=3, nt=24, g0_norm=0.5)
    st = checkpoint.load_newton(path)
    assert np.array_equal(st["v"], v) and st["v"].dtype == np.float64
    assert (st["newton_iters"], st["nt"], st["g0_norm"]) == (3, 24, 0.5)
    with np.load(path, allow_pickle=False) as z:   # plain arrays only
        assert sorted(z.files) == ["g0_norm", "newton_iters", "nt", "v"]


class _FakeWarmStart:
    def __init__(self, n, seed):
        g = torch.Generator().manual_seed(seed)
        self.device = torch.device("cpu")
        self.params, self.m, self.v = (torch.randn(n, generator=g) for _ in range(3))
        self.step = 5 * seed


def test_training_state_round_trip(tmp_path):
    a, b = _FakeWarmStart(100, 1), _FakeWarmStart(100, 2)
    path = tmp_path / "train.npz"
    checkpoint.save_training(path, a, epoch=4)
    assert checkpoint.load_training(path, b) == 4
    for name in ("params", "m", "v"):
        assert torch.equal(getattr(a, name), getattr(b, name))
    assert b.step == a.step
    with pytest.raises(ValueError):
        checkpoint.load_training(path, _FakeWarmStart(99, 3))


def test_step_log_lines(tmp_path):
    recs = [{"newton_iter": k, "g_rel": 0.5 ** k, "alpha": 1.0} for k in range(3)]
    path = tmp_path / "steps.jsonl"
    write_step_log(str(path), recs, {"n1": 8, "n2": 8})
    write_step_log(str(path), recs[:1], {"n1": 8, "n2": 8})   # appends
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    assert len(lines) == 4 and lines[2] == {"n1": 8, "n2": 8, **recs[2]}
    seen = []
    write_step_log(seen.append, recs, {"n1": 8})
    assert [s["newton_iter"] for s in seen] == [0, 1, 2] and seen[0]["n1"] == 8
