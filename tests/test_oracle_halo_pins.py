"""Pins of the per-halo statistics reference (oracle/halo.py).

Closed forms (a cube's corners), the periodic unwrapping of a halo that
straddles the box edge, invariance under translation, a constant velocity
field, a plain-Python evaluation of the same definition member by member,
and the FP64 summation bound of the bulk velocity against an exact sum.
"""
import math

import numpy as np

from oracle import halo

G = 1 << 21


def test_cube_corners_closed_form():
    pos = np.array([[x, y, z] for x in (10, 12) for y in (20, 22) for z in (30, 32)], np.uint32)
    for peak in range(8):
        o = halo.halo_stats(pos, np.zeros(8, np.int32), np.array([peak]))
        assert o["count"][0] == 8
        assert np.array_equal(o["com"][0], [11.0, 21.0, 31.0])
        assert o["rmax"][0] == math.sqrt(3.0)


def test_periodic_halo_straddling_the_edge():
    xs = [G - 2, G - 1, 0, 1]
    pos = np.array([[x, 100, 200] for x in xs], np.uint32)
    for peak in range(4):
        o = halo.halo_stats(pos, np.zeros(4, np.int32), np.array([peak]), periodic=True)
        assert o["com"][0, 0] == G - 0.5, peak      # unwrapped, not the box middle
        assert o["rmax"][0] == 1.5                  # the ends are 1.5 from the centre
    o = halo.halo_stats(pos, np.zeros(4, np.int32), np.array([0]), periodic=False)
    assert o["com"][0, 0] == (2 * G - 2) / 4.0       # plain mean without wrapping


def _clumps(seed, n=600, k=4):
    rng = np.random.default_rng(seed)
    centres = rng.integers(0, G, (k, 3))
    lab = rng.integers(0, k, n)
    pos = (centres[lab] + rng.integers(-3000, 3000, (n, 3))) % G
    lab[rng.random(n) < 0.1] = -1                    # some particles belong to no halo
    peak = np.array([np.flatnonzero(lab == g)[0] for g in range(k)])
    return pos.astype(np.uint32), lab.astype(np.int32), peak


def test_translation_invariance():
    pos, lab, peak = _clumps(1)
    t = np.array([12345, 678, (1 << 20) + 5], np.int64)
    a = halo.halo_stats(pos, lab, peak)
    b = halo.halo_stats(((pos.astype(np.int64) + t) % G).astype(np.uint32), lab, peak)
    assert np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["rmax"], b["rmax"])      # offsets are the same integers
    dc = np.mod(b["com"] - a["com"] - t, G)
    dc = np.where(dc > G / 2, dc - G, dc)
    assert np.all(np.abs(dc) <= 4 * np.spacing(float(G)))


def test_constant_velocity():
    pos, lab, peak = _clumps(2)
    vel = np.tile(np.array([0.375, -2.5, 1.25], np.float32), (pos.shape[0], 1))
    o = halo.halo_stats(pos, lab, peak, vel=vel)
    assert np.array_equal(o["vbulk"], np.tile([0.375, -2.5, 1.25], (peak.size, 1)))


def test_member_by_member_python():
    pos, lab, peak = _clumps(3, n=300, k=3)
    o = halo.halo_stats(pos, lab, peak)
    for g in range(3):
        mem = [i for i in range(pos.shape[0]) if lab[i] == g]
        p = [int(c) for c in pos[peak[g]]]
        offs = []
        for i in mem:
            d = []
            for k in range(3):
                x = (int(pos[i][k]) - p[k]) % G
                d.append(x - G if x >= G // 2 else x)
            offs.append(d)
        m = [float(sum(o_[k] for o_ in offs)) / float(len(mem)) for k in range(3)]
        com = [p[k] + m[k] for k in range(3)]
        com = [c + G if c < 0 else (c - G if c >= G else c) for c in com]
        r = 0.0
        for d in offs:
            ex, ey, ez = (d[0] - m[0]), (d[1] - m[1]), (d[2] - m[2])
            r = max(r, math.sqrt((ex * ex + ey * ey) + ez * ez))
        assert o["count"][g] == len(mem)
        assert list(o["com"][g]) == com
        assert o["rmax"][g] == r


def test_bulk_velocity_within_fp64_bound():
    pos, lab, peak = _clumps(4, n=5000, k=5)
    vel = np.random.default_rng(9).normal(0, 300, (pos.shape[0], 3)).astype(np.float32)
    o = halo.halo_stats(pos, lab, peak, vel=vel)
    u = 2.0 ** -53
    for g in range(5):
        mem = np.flatnonzero(lab == g)
        c = mem.size
        for k in range(3):
            exact = math.fsum(float(v) for v in vel[mem, k]) / c
            bound = 2 * (c - 1) * u * float(np.abs(vel[mem, k].astype(np.float64)).sum()) / c \
                + 2 * u * abs(exact)
            assert abs(o["vbulk"][g, k] - exact) <= bound
