"""Training and set-up of the learned surrogate (host orchestration).

Every computation runs in libfcat.so: path lengths of the training rays
(``fcat_pathlengths``), their exact primary group signals (``fcat_spectral``),
the linear term (``fcat_mlp_linear_term``), the input/output scales and the
optical-depth range of the cells (``fcat_mlp_setup``), forward/backward/Adam
(``fcat_mlp_train_epoch``) and the held-out validation that decides where
the network may replace the exact sum (``fcat_mlp_validate``).  This module
only draws the seeded samples and initial weights (inputs to those kernels),
slices tensors, loops over epochs and sets the learning-rate schedule.

Checkpoints: with ``checkpoint=path`` the weights, the Adam moments and step,
the scales and the loss history are written to ``path`` (NumPy ``.npz``,
arrays only, replaced atomically) after every epoch; with ``resume=True`` a
run continues after the last epoch the file holds.  Sampling, the epoch
orders and the schedule are seeded by epoch, so a resumed run reproduces
the uninterrupted one.
"""
from __future__ import annotations

import math
import os
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import (MlpTrain, Problem, Surrogate, fcat_mlp_linear_term, fcat_mlp_param_count, fcat_mlp_setup,
               fcat_mlp_train_epoch, fcat_mlp_validate, fcat_pathlengths, fcat_spectral)

HIDDEN = 64


def init_params(n_in: int, n_out: int, seed: int) -> np.ndarray:
    """Seeded initial weights: uniform(+-sqrt(6 / (fan_in + fan_out))), zero biases, small last layer."""
    rng = np.random.default_rng(seed)

    def glorot(fan_out, fan_in, gain=1.0):
        lim = gain * math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_out, fan_in))
    parts = [glorot(HIDDEN, n_in), np.zeros(HIDDEN), glorot(HIDDEN, HIDDEN), np.zeros(HIDDEN),
             glorot(n_out, HIDDEN, 0.1), np.zeros(n_out)]
    p = np.concatenate([a.ravel() for a in parts]).astype(np.float32)
    assert p.size == fcat_mlp_param_count(n_in, n_out)
    return p


def sample_rays(pb: Problem, n_mat: int, n_samples: int, angles, seed: int, chunk: int = 4):
    """Path lengths L[n][n_mat] (device) of n_samples rays drawn without replacement
    from the rays of the given angles that cross the phantom."""
    import torch
    rng = np.random.default_rng(seed)
    angles = np.asarray(angles, dtype=np.int64)
    picked = []
    per_angle = pb.geometry.nu * pb.geometry.nv
    # draw the share of each angle chunk in proportion to its hit count
    chunks = [angles[i:i + chunk] for i in range(0, len(angles), chunk)]
    want = [n_samples * len(c) // len(angles) for c in chunks]
    want[-1] += n_samples - sum(want)
    for c, k in zip(chunks, want):
        rows = []
        for a in c:
            La = fcat_pathlengths(pb, n_mat, int(a), int(a) + 1).reshape(per_angle, n_mat)
            rows.append(La.cpu().numpy())
        La = np.concatenate(rows)
        hit = np.nonzero(La.sum(1) > 0)[0]
        sel = rng.choice(hit, size=min(k, hit.size), replace=False)
        picked.append(La[np.sort(sel)])
    L = np.concatenate(picked)
    L = L[rng.permutation(L.shape[0])]
    return torch.as_tensor(L, device=pb.phantom.labels.device)


@dataclass
class TrainReport:
    n_train: int
    n_holdout: int
    epochs: int
    batch: int
    seconds: float
    epoch_loss: list = field(default_factory=list)
    cell_err: Optional[np.ndarray] = None
    cell_ok: Optional[np.ndarray] = None
    cell_count: Optional[np.ndarray] = None
    holdout_in_ok_cells: float = 0.0


def _save_checkpoint(path: str, epoch: int, train: MlpTrain, sur: Surrogate, report: "TrainReport") -> None:
    tmp = path + ".tmp.npz"
    np.savez(tmp, epoch=np.int64(epoch), step=np.int64(train.step), params=train.params.cpu().numpy(),
             adam_m=train.adam_m.cpu().numpy(), adam_v=train.adam_v.cpu().numpy(),
             in_scale=sur.in_scale.cpu().numpy(), out_scale=sur.out_scale.cpu().numpy(), lin=sur.lin.cpu().numpy(),
             cell_hi=np.float64(sur.cell_hi), epoch_loss=np.asarray(report.epoch_loss, np.float64))
    os.replace(tmp, path)


def _load_checkpoint(path: str, train: MlpTrain, sur: Surrogate, report: "TrainReport") -> int:
    """Restore the state of ``path`` into train / sur / report; returns the next epoch."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        for name, dst in (("params", train.params), ("adam_m", train.adam_m), ("adam_v", train.adam_v),
                          ("in_scale", sur.in_scale), ("out_scale", sur.out_scale), ("lin", sur.lin)):
            src = z[name]
            if tuple(src.shape) != tuple(dst.shape):
                raise ValueError(f"checkpoint {path}: {name} has shape {src.shape}, expected {tuple(dst.shape)}")
            dst.copy_(torch.as_tensor(src, device=dst.device))
        train.step = int(z["step"])
        sur.cell_hi = float(z["cell_hi"])
        report.epoch_loss = [float(x) for x in z["epoch_loss"]]
        return int(z["epoch"]) + 1


def build_surrogate(pb: Problem, n_samples: int = 4_000_000, holdout: float = 0.1, epochs: int = 120,
                    batch: int = 4096, lr: float = 2e-3, lr_final: float = 2e-5, threshold: float = 1e-3,
                    min_count: int = 16, angles=None, seed: int = 47365, verbose: bool = False,
                    checkpoint: Optional[str] = None, resume: bool = False, stop_after: Optional[int] = None):
    """Train the surrogate on rays of ``pb`` and validate it; returns (Surrogate, TrainReport).

    ``checkpoint`` / ``resume``: see the module notes.  ``stop_after`` ends
    the run after that many epochs of this call (the checkpoint then holds a
    resumable state); the returned surrogate is validated either way."""
    import torch
    sp = pb.spectral
    M, _E = (int(x) for x in sp.mu.shape)
    G = int(sp.n_groups)
    dev = pb.phantom.labels.device
    A = pb.geometry.n_angles
    if angles is None:
        angles = np.arange(0, A, max(1, A // 36))
    L = sample_rays(pb, M, n_samples, angles, seed)
    Y = fcat_spectral(L, sp)                                   # exact primary group signals
    n = int(L.shape[0])
    n_hold = int(round(n * holdout))
    n_train = n - n_hold
    Lt, Lh = L[:n_train].contiguous(), L[n_train:].contiguous()
    Yt, Yh = Y[:, :n_train].contiguous(), Y[:, n_train:].contiguous()

    lin = fcat_mlp_linear_term(sp)
    in_scale, out_scale, tau_max = fcat_mlp_setup(sp, lin, Lt, Yt)
    params = torch.as_tensor(init_params(M, G, seed), device=dev)
    sur = Surrogate(params=params, in_scale=in_scale, out_scale=out_scale, lin=lin, cell_ok=None,
                    cell_lo=0.0, cell_hi=float(tau_max.item()) * (1.0 + 1e-6))
    train = MlpTrain(params=params, adam_m=torch.zeros_like(params), adam_v=torch.zeros_like(params), lr=lr)
    nb = (n_train + batch - 1) // batch
    batch_loss = torch.empty(nb, dtype=torch.float32, device=dev)
    report = TrainReport(n_train, n_hold, epochs, batch, 0.0)
    first = 0
    if checkpoint and resume and os.path.exists(checkpoint):
        first = _load_checkpoint(checkpoint, train, sur, report)
    last = epochs if stop_after is None else min(epochs, first + stop_after)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(first, last):
        train.lr = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * ep / max(epochs - 1, 1)))
        # the epoch's sample order, drawn on the device (a host permutation of
        # millions of samples took longer than the epoch's training)
        g = torch.Generator(device=dev).manual_seed(seed * 1000 + ep)
        order = torch.randperm(n_train, generator=g, device=dev).to(torch.int32)
        fcat_mlp_train_epoch(train, sur, sp, Lt, Yt, order, batch, batch_loss=batch_loss)
        report.epoch_loss.append(float(batch_loss.mean().item()))
        if checkpoint:
            _save_checkpoint(checkpoint, ep, train, sur, report)
        if verbose:
            print(f"epoch {ep}: lr {train.lr:.2e} loss {report.epoch_loss[-1]:.3e}", flush=True)
    torch.cuda.synchronize()
    report.seconds = time.perf_counter() - t0
    cell_err, cell_ok, cell_count = fcat_mlp_validate(sur, sp, Lh, Yh, threshold=threshold, min_count=min_count)
    report.cell_err = cell_err.cpu().numpy()
    report.cell_ok = cell_ok.cpu().numpy()
    report.cell_count = cell_count.cpu().numpy()
    # share of held-out rays that fall in validated cells
    report.holdout_in_ok_cells = float(report.cell_count[report.cell_ok == 1].sum()) / max(n_hold, 1)
    return sur, report
