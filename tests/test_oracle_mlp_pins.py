"""Pins of the FP64 learned-radius reference (oracle/mlp.py).

The gradient is checked against central finite differences and against the
closed form of the all-active (linear) regime; the Adam step against its
first-step closed form; the features against brute-force cell counting and
lattices; the target against the lattice closed form r^2 = 6 a^2.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import mlp


def rand_net(rng, scale=0.3):
    return rng.normal(0.0, scale, mlp.N_PARAMS)


def test_param_layout_roundtrip():
    rng = np.random.default_rng(0)
    w = rand_net(rng)
    assert mlp.N_PARAMS == 6017
    assert np.array_equal(mlp.pack(*mlp.unpack(w)), w)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    w = rand_net(rng)
    X = rng.uniform(0.0, 3.0, (24, 27))
    t = rng.normal(0.0, 1.0, 24)
    loss, g = mlp.loss_and_grad(w, X, t)
    _, (_, a1, _, a2, _) = mlp.forward(w, X)
    h = 1e-6
    # keep away from ReLU kinks: a step of h moves pre-activations by far less
    assert min(np.abs(a1).min(), np.abs(a2).min()) > 1e-4
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False),
                          np.arange(mlp.N_PARAMS - 65, mlp.N_PARAMS)])
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss_and_grad(wp, X, t)[0] - mlp.loss_and_grad(wm, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_linear_regime_closed_form():
    # positive weights and inputs: every unit is active, the net is linear
    rng = np.random.default_rng(2)
    W1 = rng.uniform(0.01, 0.1, (27, 64))
    b1 = rng.uniform(0.01, 0.1, 64)
    W2 = rng.uniform(0.01, 0.1, (64, 64))
    b2 = rng.uniform(0.01, 0.1, 64)
    W3 = rng.uniform(0.01, 0.1, 64)
    b3 = np.array([0.3])
    w = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = rng.uniform(0.0, 2.0, (10, 27))
    t = rng.normal(0.0, 1.0, 10)
    a = W1 @ W2 @ W3
    c = b1 @ W2 @ W3 + b2 @ W3 + b3[0]
    y, _ = mlp.forward(w, X)
    assert np.allclose(y, X @ a + c, rtol=1e-13, atol=0)
    loss, g = mlp.loss_and_grad(w, X, t)
    r = X @ a + c - t
    assert np.isclose(loss, np.mean(r * r), rtol=1e-13)
    dy = 2 * r / 10
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unpack(g)
    assert np.isclose(gb3[0], dy.sum(), rtol=1e-12)
    assert np.allclose(gb1, dy.sum() * (W2 @ W3), rtol=1e-12)
    assert np.allclose(gW1, np.outer(X.T @ dy, W2 @ W3), rtol=1e-12)
    assert np.allclose(gb2, dy.sum() * W3, rtol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    w1, m1, v1 = mlp.adam_step(w, np.zeros(50), np.zeros(50), g, 1, lr=1e-3, eps=1e-8)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_features_bruteforce_counts():
    rng = np.random.default_rng(4)
    pos = rng.integers(0, 1 << 21, (300, 3)).astype(np.uint32)
    cb = 19  # 4 cells per axis
    for periodic in (True, False):
        f = mlp.features(pos, cb, periodic=periodic)
        cells = pos.astype(np.int64) >> cb
        for i in rng.choice(300, 25, replace=False):
            k = 0
            for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
                want = np.array([cells[i, 0] + dx, cells[i, 1] + dy, cells[i, 2] + dz])
                if periodic:
                    want %= 4
                    n = int(np.all(cells == want, axis=1).sum())
                elif np.any(want < 0) or np.any(want > 3):
                    n = 0
                else:
                    n = int(np.all(cells == want, axis=1).sum())
                assert f[i, k] == np.log1p(n), (i, k)
                k += 1


def test_features_lattice_one_per_cell():
    p = synth.lattice_box(16)          # spacing 2^17 = one particle per cell
    f = mlp.features(p.pos, 17, periodic=True)
    assert np.all(f == np.log(2.0))
    fn = mlp.features(p.pos, 17, periodic=False)
    corner = np.flatnonzero(np.all(p.pos == 0, axis=1))[0]
    assert np.count_nonzero(fn[corner] == 0.0) == 27 - 8


def test_target_lattice_closed_form(orc):
    p = synth.lattice_box(16)          # a = 2^17: the 64-list ends in the d^2 = 6 a^2 shell
    _, d2 = orc.knn(p.pos, 64, periodic=True)
    y = mlp.targets(d2[:, -1], 17)
    assert np.allclose(y, 0.5 * np.log(6.0), rtol=0, atol=1e-14)
