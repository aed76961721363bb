"""Training and calibration of the search-radius model (host side).

Everything numerical runs in the library's kernels (features, targets,
forward, backward, Adam, BF16 inference); this module draws the seeded
random numbers the training consumes (initial weights, sample order),
loops over training chunks and picks the margin from the residuals.

Typical use (see the design notes for the workload):

    feats, target = ctx.radius_dataset(pos, params, cell_bits, nbr=nbr)
    w, losses = train(ctx, feats, target)
    margin = calibrate(ctx, w, feats, target, miss_rate=0.01)
    ctx.radius_load(HOP_RADIUS_MLP, w, margin)
    ctx.density(pos, HopParams(..., learned_radius=True))
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import HOP_MLP_PARAMS, HOP_RADIUS_ANALYTIC, HOP_RADIUS_MLP, load

__all__ = ["cell_bits_for", "init_weights", "train", "calibrate", "OCCUPANCY"]

# mean particles per cell that the features are defined for
OCCUPANCY = 8.0


def cell_bits_for(n: int, grid_bits: int = 21, occupancy: float = OCCUPANCY) -> int:
    """The cell side bits the library uses for n particles."""
    cb = load().hop_radius_cell_bits(int(n), C.c_uint32(grid_bits), C.c_float(occupancy))
    if cb < 0:
        raise ValueError("bad arguments to hop_radius_cell_bits")
    return int(cb)


def init_weights(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (layout W1, b1, W2, b2, W3, b3)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(HOP_MLP_PARAMS, np.float32)
    o = 0
    w[o:o + 27 * 64] = rng.normal(0.0, np.sqrt(2.0 / 27), 27 * 64)
    o += 27 * 64 + 64
    w[o:o + 64 * 64] = rng.normal(0.0, np.sqrt(2.0 / 64), 64 * 64)
    o += 64 * 64 + 64
    w[o:o + 64] = rng.normal(0.0, np.sqrt(1.0 / 64), 64)
    return w


def train(ctx, feats, target, steps: int = 3000, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0, chunk: int = 500, log=None):
    """Adam on the mean squared error with uniformly drawn batches.

    Returns (weights as a device float32 tensor, numpy array of step losses).
    """
    import torch
    dev = feats.device
    n = feats.shape[0]
    rng = np.random.default_rng(seed + 1)
    w = torch.from_numpy(init_weights(seed)).to(dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    losses = []
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        idx = torch.from_numpy(rng.integers(0, n, size=k * batch).astype(np.int32)).to(dev)
        l = ctx.mlp_train(feats, target, w, m, v, idx, k, batch, first_step=done + 1, lr=lr)
        losses.append(l.cpu().numpy())
        done += k
        if log:
            log(f"step {done}: loss {float(losses[-1][-1]):.4f}")
    return w, np.concatenate(losses) if losses else np.zeros(0, np.float32)


def calibrate(ctx, w, feats, target, miss_rate: float = 0.01, kind: int = HOP_RADIUS_MLP,
              n_dens: int = 64, occupancy: float = OCCUPANCY, sample: int = 4_000_000,
              seed: int = 0) -> float:
    """Margin m such that a fraction miss_rate of the (sampled) particles
    have log(r / side) above prediction + m; loads the model with it."""
    import torch
    ctx.radius_load(kind, w if kind == HOP_RADIUS_MLP else None, 0.0, occupancy)
    n = feats.shape[0]
    if n > sample:
        sel = torch.from_numpy(np.random.default_rng(seed).choice(n, sample, replace=False)
                               .astype(np.int64)).to(feats.device)
        feats, target = feats[sel].contiguous(), target[sel].contiguous()
    pred = ctx.radius_predict(feats, n_dens)
    res = (target - pred).cpu().numpy().astype(np.float64)
    margin = float(np.quantile(res, 1.0 - miss_rate))
    ctx.radius_load(kind, w if kind == HOP_RADIUS_MLP else None, margin, occupancy)
    return margin
