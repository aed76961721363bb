"""Host-side decomposition front end (paper_1001_3411_amd/decompose.py).

The prime-factor cutting rounds, the load balance on a 3% subsample, the
padding of Eq. (1) in closed form on a lattice, directional padding on an
anisotropic density, and the layout of the padded batch (every particle in
exactly one core, every particle of a padded box present, frames shifted
by the padded low corner with the periodic wrap).
"""
import numpy as np
import pytest

import synth
from paper_1001_3411_amd import decompose as dc

G = 1 << 21


def test_prime_factors():
    assert dc.prime_factors(1) == []
    assert dc.prime_factors(8) == [2, 2, 2]
    assert dc.prime_factors(12) == [3, 2, 2]
    assert dc.prime_factors(7) == [7]
    assert dc.prime_factors(360) == [5, 3, 3, 2, 2, 2]
    with pytest.raises(ValueError):
        dc.prime_factors(0)


@pytest.mark.parametrize("tasks", [1, 2, 8, 12, 27])
def test_cuts_partition_the_box(tasks):
    rng = np.random.default_rng(tasks)
    pts = rng.integers(0, G, (20000, 3))
    boxes = dc.cut_boxes(pts, tasks)
    assert len(boxes) == tasks
    vol = np.prod((boxes[:, 1] - boxes[:, 0]).astype(np.float64), axis=1).sum()
    assert vol == float(G) ** 3
    probe = rng.integers(0, G, (5000, 3))
    inside = np.stack([np.all((probe >= b[0]) & (probe < b[1]), axis=1) for b in boxes])
    assert np.all(inside.sum(axis=0) == 1)      # disjoint and covering


def test_power_of_two_is_bisection():
    pts = np.random.default_rng(3).integers(0, G, (4000, 3))
    boxes = dc.cut_boxes(pts, 2)
    assert np.array_equal(boxes[0][1][1:], [G, G]) and boxes[0][1][0] == boxes[1][0][0]


def test_load_balance_on_a_subsample():
    p = synth.config(2)                          # clustered, 2M particles
    d = dc.decompose(p.pos, 12, sample_frac=0.03, seed=1)
    core = np.bincount(d.index[d.padded == 0], minlength=p.n)
    assert np.all(core == 1)                     # every particle in exactly one core
    counts = np.array([np.count_nonzero(d.padded[a:b] == 0)
                       for a, b in zip(d.offsets[:-1], d.offsets[1:])])
    assert counts.max() / counts.min() < 1.10    # the paper's 10% spread


def test_padding_closed_form_on_a_lattice():
    p = synth.lattice_box(32)                    # spacing a = 2^16
    a = G // 32
    boxes = np.array([[[0, 0, 0], [G // 2, G, G]], [[G // 2, 0, 0], [G, G, G]]], np.int64)
    pads = dc.paddings(p.pos, boxes, n_dens=64, safety=1.5, directional=False)
    # V / N = a^3, so L_p = s * (64 a^3)^(1/3) = 1.5 * 4 a
    assert np.all(pads == int(np.ceil(1.5 * 4 * a)))
    dpads = dc.paddings(p.pos, boxes, n_dens=64, safety=1.5, directional=True)
    # a face slab of a uniform lattice has the same spacing: within one lattice plane
    assert np.all(np.abs(dpads - pads) <= np.ceil(1.5 * 4 * a * 0.2))


def test_directional_padding_follows_the_local_density():
    rng = np.random.default_rng(5)
    n = 200000
    x = (rng.random(n) ** 3 * G).astype(np.int64)      # dense near x = 0, sparse near x = G
    pos = np.stack([x, rng.integers(0, G, n), rng.integers(0, G, n)], axis=1)
    boxes = np.array([[[0, 0, 0], [G, G, G]]], np.int64)
    pads = dc.paddings(pos, boxes, directional=True)
    assert pads[0, 1, 0] > 2 * pads[0, 0, 0]            # sparse face gets the wider padding
    flat = dc.paddings(pos, boxes, directional=False)
    assert pads[0, 0, 0] < flat[0, 0, 0] < pads[0, 1, 0]


def test_batch_layout():
    rng = np.random.default_rng(8)
    pos = rng.integers(0, G, (60000, 3)).astype(np.uint32)
    d = dc.decompose(pos, 8, seed=2)
    p64 = pos.astype(np.int64)
    for t in range(8):
        a, b = d.offsets[t], d.offsets[t + 1]
        lo, hi = d.boxes[t]
        org = d.origin[t]
        span = (hi - lo) + d.pads[t, 0] + d.pads[t, 1]
        rel = np.mod(p64 - org, G)
        want = np.flatnonzero(np.all(rel < span, axis=1))
        assert np.array_equal(np.sort(d.index[a:b]), want)         # the whole padded box
        assert np.array_equal(d.pos[a:b].astype(np.int64), rel[d.index[a:b]])
        assert np.all(d.pos[a:b].astype(np.int64) < span)
        core = np.all((p64[d.index[a:b]] >= lo) & (p64[d.index[a:b]] < hi), axis=1)
        assert np.array_equal(d.padded[a:b] == 0, core)
