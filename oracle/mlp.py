"""FP64 reference for the learned search radius (test infrastructure only).

TEST INFRASTRUCTURE ONLY: loaded by the test suite and nothing else.  It
shares no code with the GPU library.

The paper searches a fixed number of nearest neighbours per particle (its
section 2); it motivates but does not define a predicted search radius.  The
model here is this project's: a 27 -> 64 -> 64 -> 1 ReLU network that maps
the log counts of the 3x3x3 cells around a particle's cell to the log of
its N_dens-th neighbour distance in cell units.  This module writes out, in
plain NumPy FP64:

* the cell counts and the 27 features per particle, f_k = log(1 + n_k) over
  the cells (cz+dz, cy+dy, cx+dx), dz outermost, each of dz, dy, dx running
  -1, 0, 1, periodic or (non-periodic) zero outside the box;
* the training target y = log(r / side), r the distance to the last entry
  of the particle's neighbour list, side = 2^cell_bits;
* the network's forward pass, mean-squared-error loss and its gradient by
  the chain rule;
* one Adam step (Kingma & Ba, bias-corrected moments).

Parameters are one flat vector in this order: W1 [27][64] (input-major),
b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1] -- 6017 numbers.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 27, 64
N_PARAMS = N_IN * N_H + N_H + N_H * N_H + N_H + N_H + 1  # 6017


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == N_PARAMS
    o = 0
    W1 = w[o:o + N_IN * N_H].reshape(N_IN, N_H); o += N_IN * N_H
    b1 = w[o:o + N_H]; o += N_H
    W2 = w[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = w[o:o + N_H]; o += N_H
    W3 = w[o:o + N_H]; o += N_H
    b3 = w[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2),
                           np.ravel(W3), np.ravel(b3)]).astype(np.float64)


def cell_counts(pos, cell_bits, grid_bits=21):
    """counts[cz, cy, cx] of particles per cell of side 2^cell_bits."""
    pos = np.asarray(pos, dtype=np.int64)
    g = 1 << (grid_bits - cell_bits)
    c = pos >> cell_bits
    flat = (c[:, 2] * g + c[:, 1]) * g + c[:, 0]
    return np.bincount(flat, minlength=g ** 3).reshape(g, g, g)


def features(pos, cell_bits, periodic=True, grid_bits=21):
    """[n, 27] log(1 + count) of the 3x3x3 cells around each particle's cell."""
    counts = cell_counts(pos, cell_bits, grid_bits).astype(np.float64)
    g = counts.shape[0]
    pos = np.asarray(pos, dtype=np.int64)
    c = pos >> cell_bits
    out = np.empty((pos.shape[0], 27), dtype=np.float64)
    k = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                z, y, x = c[:, 2] + dz, c[:, 1] + dy, c[:, 0] + dx
                if periodic:
                    n = counts[z % g, y % g, x % g]
                else:
                    inside = (z >= 0) & (z < g) & (y >= 0) & (y < g) & (x >= 0) & (x < g)
                    n = np.where(inside, counts[np.clip(z, 0, g - 1), np.clip(y, 0, g - 1),
                                                np.clip(x, 0, g - 1)], 0.0)
                out[:, k] = np.log1p(n)
                k += 1
    return out


def targets(d2_last, cell_bits):
    """log(r / side) with r^2 = d2_last (exact integers)."""
    d2 = np.asarray(d2_last, dtype=np.float64)
    return 0.5 * np.log(d2) - cell_bits * np.log(2.0)


def forward(w, X):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3 + b3[0]
    return y, (X, a1, h1, a2, h2)


def loss_and_grad(w, X, t):
    """Mean squared error over the rows and its gradient (flat, FP64)."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    y, (X, a1, h1, a2, h2) = forward(w, X)
    t = np.asarray(t, dtype=np.float64)
    B = y.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    gW3 = h2.T @ dy
    gb3 = np.array([dy.sum()])
    dh2 = np.outer(dy, W3) * (a2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (a1 > 0)
    gW1 = X.T @ dh1
    gb1 = dh1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(w, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    w = np.asarray(w, np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return w, m, v
