"""Surrogate checkpoints on the host: a save / load round trip restores every
array and counter, and a checkpoint of another shape is refused."""
import numpy as np
import pytest
import torch

from paper_2011_04736_amd import MlpTrain, Surrogate
from paper_2011_04736_amd import surrogate as sg


def _state(seed, n_in=6, n_out=2, p=50):
    g = torch.Generator().manual_seed(seed)
    r = lambda *s: torch.rand(*s, generator=g)
    sur = Surrogate(params=r(p), in_scale=r(n_in), out_scale=r(n_out), lin=r(n_out, n_in), cell_hi=float(seed))
    train = MlpTrain(params=sur.params, adam_m=r(p), adam_v=r(p), step=seed * 10)
    rep = sg.TrainReport(1, 1, 4, 8, 0.0, epoch_loss=[0.5 * seed, 0.25 * seed])
    return train, sur, rep


def test_round_trip(tmp_path):
    path = str(tmp_path / "ck.npz")
    t1, s1, r1 = _state(3)
    sg._save_checkpoint(path, 1, t1, s1, r1)
    t2, s2, r2 = _state(7)
    nxt = sg._load_checkpoint(path, t2, s2, r2)
    assert nxt == 2
    for a, b in ((t1.params, t2.params), (t1.adam_m, t2.adam_m), (t1.adam_v, t2.adam_v),
                 (s1.in_scale, s2.in_scale), (s1.out_scale, s2.out_scale), (s1.lin, s2.lin)):
        np.testing.assert_array_equal(a.numpy(), b.numpy())
    assert t2.step == t1.step and s2.cell_hi == s1.cell_hi and r2.epoch_loss == r1.epoch_loss
    assert s2.params is t2.params


def test_shape_mismatch_is_refused(tmp_path):
    path = str(tmp_path / "ck.npz")
    t1, s1, r1 = _state(3)
    sg._save_checkpoint(path, 0, t1, s1, r1)
    t2, s2, r2 = _state(4, p=60)
    with pytest.raises(ValueError, match="params"):
        sg._load_checkpoint(path, t2, s2, r2)
