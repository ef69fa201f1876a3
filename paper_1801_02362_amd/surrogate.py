"""Training pipeline of the learned surrogate (exact labels -> aligned BF16
inputs -> Adam steps), all compute on the GPU through the C ABI.

* ``exact_labels``: (s, z) of every training frame from the exact path
  (Eq. 2 and Eq. 3 through the batched-walker launch, all walkers sharing the
  landmark set);
* ``aligned_inputs``: the frames superposed onto the surrogate's reference
  (BF16 bit patterns, int16 tensor);
* ``train``: minibatch Adam steps with a geometric learning-rate decay.

Host code here only slices tensors, moves them between host and device and
computes the two label means and deviations used for standardisation.
"""
from __future__ import annotations

import math

import numpy as np

from . import BatchPathCV, Surrogate

__all__ = ["exact_labels", "aligned_inputs", "standardise", "train", "test_loss"]


def exact_labels(landmarks, lam: float, frames, *, batch: int = 256):
    """Exact (s, z) [F][2] float64 (device) of frames ``[F][n][3]`` (device
    float32) against ``landmarks`` ``[L][n][3]`` (device float32)."""
    import torch
    F, n = int(frames.shape[0]), int(frames.shape[1])
    out = torch.empty(F, 2, dtype=torch.float64, device=frames.device)
    t0 = 0
    while t0 < F:
        W = min(batch, F - t0)
        b = BatchPathCV([landmarks] * W, [lam] * W, use_graph=False)
        while t0 + W <= F:
            sz, _, _ = b.eval(frames[t0:t0 + W].reshape(W * n, 3), grad=False)
            out[t0:t0 + W].copy_(sz)
            t0 += W
        b.close()
    return out


def aligned_inputs(sur: Surrogate, frames):
    """BF16 aligned inputs [F][3n] (int16 bit patterns) of device frames."""
    import torch
    F = int(frames.shape[0])
    out = torch.empty(F, 3 * sur.n, dtype=torch.int16, device=frames.device)
    for t0 in range(0, F, sur.max_batch):
        t1 = min(F, t0 + sur.max_batch)
        ob, _ = sur.align(frames[t0:t1])
        out[t0:t1].copy_(ob)
    return out


def standardise(labels):
    """Mean and deviation of s and z over the training labels (host)."""
    lab = labels.detach().cpu().numpy()
    mean = lab.mean(axis=0)
    sd = lab.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mean, sd


def train(sur: Surrogate, inputs, targets, *, epochs: int, batch: int, lr: float, lr_final: float | None = None,
          log=None):
    """Minibatch Adam over contiguous slices (rows pre-shuffled by the
    caller); the learning rate decays geometrically from ``lr`` to
    ``lr_final`` over all steps.  Returns the loss after each epoch."""
    import torch
    F = int(inputs.shape[0])
    per_epoch = max(1, F // batch)
    total = epochs * per_epoch
    lr_final = lr if lr_final is None else lr_final
    decay = (lr_final / lr) ** (1.0 / max(1, total - 1))
    loss = torch.zeros(1, dtype=torch.float32, device=inputs.device)
    hist = []
    k = 0
    for e in range(epochs):
        acc = torch.zeros(1, dtype=torch.float64, device=inputs.device)
        for s0 in range(0, per_epoch * batch, batch):
            sur.train_step(inputs[s0:s0 + batch], targets[s0:s0 + batch], lr * decay ** k, loss)
            acc += loss
            k += 1
        hist.append(float(acc.item()) / per_epoch)
        if log:
            log(f"[surrogate] epoch {e + 1}/{epochs} loss {hist[-1]:.3e} lr {lr * decay ** (k - 1):.2e}")
    return hist


def test_loss(sur: Surrogate, inputs, targets) -> float:
    """Mean squared error (standardised units) of the network on a set."""
    F = int(inputs.shape[0])
    tot = 0.0
    for t0 in range(0, F, sur.max_batch):
        t1 = min(F, t0 + sur.max_batch)
        y = sur.forward(inputs[t0:t1])
        tot += float(((y - targets[t0:t1]) ** 2).sum().item())
    return tot / F
