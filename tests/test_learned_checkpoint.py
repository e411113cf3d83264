"""Checkpoint and resume of the predictor's training (CPU).

The training loop of paper_2506_03266_amd.learned is driven here by the
oracle's float64 step (oracle/cnn_oracle.py: loss gradient and Adam,
Kingma & Ba Algorithm 1) instead of the library's kernels.  A run
interrupted after one epoch and resumed from its checkpoint must end with
exactly the parameters, moments and losses of the run that was not
interrupted: the checkpoint holds the master weights, the Adam moments, the
update count and the data-order generator's state."""
from __future__ import annotations

import os

import numpy as np
import torch

import oracle
from oracle import cnn_oracle as co
from paper_2506_03266_amd import learned


class OracleOps:
    """The training step of the CPU oracle (float64)."""

    def init(self, seed):
        p = torch.from_numpy(co.init_params(seed, oracle.philox4x32_10).astype(np.float64))
        return p, torch.zeros_like(p), torch.zeros_like(p)

    def loss_grad(self, c, params, y):
        loss, grad, _ = co.loss_and_grad(c.numpy(), params.numpy(), y.numpy(), mode="f64")
        return loss, torch.from_numpy(grad)

    def adam(self, params, grad, m, v, step, lr):
        p, m2, v2 = co.adam_step(params.numpy(), grad.numpy(), m.numpy(), v.numpy(), step, lr)
        return torch.from_numpy(p), torch.from_numpy(m2), torch.from_numpy(v2)

    def to_device(self, t):
        return t.to(torch.float64)


def _data(n=48, M=4):
    rng = np.random.default_rng(77)
    counts = torch.from_numpy(rng.integers(0, 9, size=(n, M, M)).astype(np.uint8))
    target = torch.from_numpy(rng.uniform(1.0, 2.0, n))
    return counts, target


def test_resume_equals_uninterrupted(tmp_path):
    counts, target = _data()
    kw = dict(epochs=3, batch=16, lr=5e-3, lr_final=5e-4, seed=3)
    p_full, h_full = learned.train(counts, target, ops=OracleOps(), **kw)
    ck = os.path.join(tmp_path, "train.safetensors")
    p_cut, h_cut = learned.train(counts, target, ops=OracleOps(), checkpoint=ck, stop_after=1, **kw)
    assert len(h_cut) == 1
    st = learned.load_checkpoint(ck)
    assert int(st["step"][0]) == 3 and int(st["epoch"][0]) == 1
    assert torch.equal(st["params"], p_cut)
    p_res, h_res = learned.train(counts, target, ops=OracleOps(), resume=ck, **kw)
    assert torch.equal(p_res, p_full)
    assert h_res == h_full
    # the interrupted run really stopped early: its parameters differ
    assert not torch.equal(p_cut, p_full)


def test_resume_from_later_epoch_and_moments(tmp_path):
    """Resuming after two of three epochs; the saved moments are those of the
    uninterrupted run at that point."""
    counts, target = _data()
    kw = dict(epochs=3, batch=16, lr=5e-3, lr_final=5e-4, seed=5)
    ck2 = os.path.join(tmp_path, "after2.safetensors")
    learned.train(counts, target, ops=OracleOps(), checkpoint=ck2, stop_after=2, **kw)
    ck_full = os.path.join(tmp_path, "full.safetensors")
    p_full, _ = learned.train(counts, target, ops=OracleOps(), checkpoint=ck_full, **kw)
    p_res, _ = learned.train(counts, target, ops=OracleOps(), resume=ck2, **kw)
    assert torch.equal(p_res, p_full)
    a, b = learned.load_checkpoint(ck2), learned.load_checkpoint(ck_full)
    assert int(a["step"][0]) == 6 and int(b["step"][0]) == 9
    assert not torch.equal(a["m"], b["m"])
