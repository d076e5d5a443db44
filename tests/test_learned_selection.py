"""Checkpoint selection and learning-rate schedule of the learned correction (host logic, not
gpu): the GMRES iteration counts and the training step are replaced by scripted stand-ins, so
only the rules are tested."""
import pytest
import torch

from paper_0809_4802_amd import binding as B
from paper_0809_4802_amd import learned


class _Ctx:
    device = "cpu"


def _select(monkeypatch, scores, **kw):
    it = iter(scores)
    monkeypatch.setattr(learned, "gmres_iterations", lambda ctx, A, b, w, **k: next(it))
    monkeypatch.setattr(B, "vms_pc_train_step", lambda *a, **k: None)
    data = [(None, torch.zeros((4, 3, 4)))]
    return learned.train_validated(_Ctx(), data, [(None, None)], steps=len(scores) - 1, check_every=1, **kw)


def test_a_checkpoint_must_save_a_fifth(monkeypatch):
    # block-Jacobi 1000; checkpoints 950, 780, 960, 700: 780 is the first to save 20%, 700 the best
    w, rep = _select(monkeypatch, [1000, 950, 780, 960, 700])
    assert rep["selected"] == "learned" and rep["val_iters_selected"] == 700 and w is not None
    assert [c["val_iters"] for c in rep["checkpoints"]] == [950, 780, 960, 700]


def test_small_gains_keep_block_jacobi(monkeypatch):
    # 10.5% (a gain that turned into a loss on a finer mesh) is not enough
    w, rep = _select(monkeypatch, [1000, 950, 895, 801])
    assert rep["selected"] == "bj" and rep["val_iters_selected"] == 1000 and w is None


def test_min_gain_zero_takes_any_improvement(monkeypatch):
    w, rep = _select(monkeypatch, [1000, 999, 1200], min_gain=0.0)
    assert rep["selected"] == "learned" and rep["val_iters_selected"] == 999


def _rates(monkeypatch, steps, **kw):
    """The learning rate handed to each training step."""
    seen = []
    monkeypatch.setattr(learned, "gmres_iterations", lambda ctx, A, b, w, **k: 1000)
    monkeypatch.setattr(B, "vms_pc_train_step", lambda ctx, A, S, w, state, step, lr, *a: seen.append((step, lr)))
    data = [(None, torch.zeros((4, 3, 4)))]
    learned.train_validated(_Ctx(), data, [(None, None)], steps=steps, check_every=steps, lr=1e-3, **kw)
    return seen


def test_cosine_decay_of_the_learning_rate(monkeypatch):
    steps = 100
    seen = _rates(monkeypatch, steps, lr_decay="cosine")
    assert [s for s, _ in seen] == list(range(1, steps + 1))
    lrs = [lr for _, lr in seen]
    assert lrs[0] == 1e-3                                   # full rate at the first step
    assert abs(lrs[steps // 2] - 0.5e-3) < 1e-12            # half way (step 51: cos(pi / 2) = 0)
    assert 0.0 < lrs[-1] < 1e-6                             # close to zero at the last step
    assert all(a >= b for a, b in zip(lrs, lrs[1:]))        # never rises


def test_constant_rate_without_decay_and_unknown_decay_rejected(monkeypatch):
    assert {lr for _, lr in _rates(monkeypatch, 10)} == {1e-3}
    with pytest.raises(ValueError):
        _rates(monkeypatch, 10, lr_decay="linear")
