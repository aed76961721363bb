"""Pins of the oracle's subhalo extension (the ADAPTAHOP-style variant the
paper sketches in its section on subhalos; the readings are stated in the
oracle source and the design notes).

A hand-built five-chain case whose symmetric boundaries, levels, members,
numbering and parents are worked out by hand below; the special case of a
level at zero, where the structures must be the connected components of
the symmetric chain graph (a textbook routine); and the nesting of the
hierarchy on a clustered box.
"""
import numpy as np
import pytest

import synth

# chains A..E = 0..4 (two particles each), particle 10 unchained;
# rows: self first, then the 3 neighbours searched for boundaries
NBR = np.array([[0, 1, 6, 10], [1, 0, 3, 10], [2, 3, 4, 10], [3, 2, 1, 10],
                [4, 5, 7, 10], [5, 4, 3, 10], [6, 7, 1, 10], [7, 6, 9, 10],
                [8, 9, 10, 10], [9, 8, 7, 10], [10, 0, 1, 2]], np.int32)
DENS = np.array([500.0, 300.0, 450.0, 320.0, 260.0, 150.0, 230.0, 210.0, 480.0, 330.0, 50.0])
CHAIN = np.array([0, 0, 1, 1, 2, 2, 3, 3, 4, 4, -1], np.int32)
# directed maxima: A->B 310, B->A 310; B->C 355, C->B 235; C->D 235 (no
# D->C); D->E 270, E->D 270; A->D 365, D->A 265.  Symmetric boundaries
# (both directions, the smaller maximum): AB 310, BC 235, DE 270, AD 265.


def test_hand_worked_hierarchy(orc):
    s = orc.subhalos(NBR, DENS, CHAIN, 5, [260.0, 300.0, 400.0], n_merge=4, alpha=0.0)
    assert s.n_sym == 4
    # level 260: links AB, DE, AD kept -> {A, B, D, E} with members >= 260
    # {0, 1, 2, 3, 8, 9} (peak 0), and {C} with member 4 (peak 260 >= 260)
    assert s.sub[0].tolist() == [0, 0, 0, 0, 1, -1, -1, -1, 0, 0, -1]
    a, b = s.t_off[0], s.t_off[1]
    assert s.count[a:b].tolist() == [6, 1] and s.peak[a:b].tolist() == [0, 4]
    assert s.peak_dens[a:b].tolist() == [500.0, 260.0] and s.parent[a:b].tolist() == [-1, -1]
    # level 300: only AB kept -> {A, B} (members 0-3) and {E} (8, 9); C and D
    # have no member >= 300
    assert s.sub[1].tolist() == [0, 0, 0, 0, -1, -1, -1, -1, 1, 1, -1]
    a, b = s.t_off[1], s.t_off[2]
    assert s.count[a:b].tolist() == [4, 2] and s.peak[a:b].tolist() == [0, 8]
    assert s.parent[a:b].tolist() == [0, 0]
    # level 400: no link kept; single members 0 (500), 8 (480), 2 (450),
    # numbered by peak density among equal counts
    assert s.sub[2].tolist() == [0, -1, 2, -1, -1, -1, -1, -1, 1, -1, -1]
    a, b = s.t_off[2], s.t_off[3]
    assert s.peak[a:b].tolist() == [0, 8, 2] and s.parent[a:b].tolist() == [0, 1, 0]


def test_hand_worked_significance(orc):
    # alpha = 0.5 at level 260: {A,B,D,E} (6 members) needs a peak of at
    # least 260 (1 + 0.5 / sqrt 6) = 313.07 (it has 500); {C} (1 member)
    # needs 390 and has 260, so it is rejected
    s = orc.subhalos(NBR, DENS, CHAIN, 5, [260.0], n_merge=4, alpha=0.5)
    assert s.sub[0].tolist() == [0, 0, 0, 0, -1, -1, -1, -1, 0, 0, -1]
    # alpha = 3 at level 260: the 6-member structure would need
    # 260 (1 + 3 / sqrt 6) = 578.4 > 500 -- rejected (a 1 / N rule would keep it)
    s = orc.subhalos(NBR, DENS, CHAIN, 5, [260.0], n_merge=4, alpha=3.0)
    assert s.t_off[-1] == 0
    # alpha = 1 at level 400: single members would need 800
    s = orc.subhalos(NBR, DENS, CHAIN, 5, [400.0], n_merge=4, alpha=1.0)
    assert s.t_off[-1] == 0 and np.all(s.sub[0] == -1)


def test_levels_must_ascend(orc):
    with pytest.raises(RuntimeError):
        orc.subhalos(NBR, DENS, CHAIN, 5, [300.0, 260.0])


def _symmetric_components(nbr, chain_of, n_chains, n_merge):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    i = np.repeat(np.arange(nbr.shape[0]), n_merge - 1)
    j = nbr[:, 1:n_merge].reshape(-1)
    a, b = chain_of[i], chain_of[j]
    keep = (a >= 0) & (b >= 0) & (a != b)
    d = coo_matrix((np.ones(keep.sum()), (a[keep], b[keep])), shape=(n_chains, n_chains)).tocsr()
    sym = d.minimum(d.T)  # an edge only where both directions exist
    return connected_components(sym, directed=False)[1]


def test_level_zero_gives_symmetric_components(orc):
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    s = orc.subhalos(r.nbr, r.density, r.chain_of, r.n_chains, [0.0], n_merge=4)
    comp = _symmetric_components(r.nbr, r.chain_of, r.n_chains, 4)
    alive = r.chain_of >= 0
    lab = s.sub[0][alive]
    ref = comp[r.chain_of[alive]]
    # the same partition of the chained particles
    pairs = set(zip(lab.tolist(), ref.tolist()))
    assert len(pairs) == len(set(lab.tolist())) == len(set(ref.tolist()))
    assert np.all(s.sub[0][~alive] == -1)


def test_hierarchy_nests_on_a_clustered_box(orc):
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    levels = [200.0, 400.0, 800.0, 1600.0]
    s = orc.subhalos(r.nbr, r.density, r.chain_of, r.n_chains, levels, n_merge=4, alpha=1.0)
    assert s.t_off[1] > 5
    for l in range(1, len(levels)):
        a, b = s.t_off[l], s.t_off[l + 1]
        for t in range(b - a):
            members = np.flatnonzero(s.sub[l] == t)
            par = s.parent[a + t]
            assert members.size == s.count[a + t]
            assert r.density[members].min() >= levels[l]
            # every member of a structure lies in its parent (when it has one)
            if par >= 0:
                assert np.all(s.sub[l - 1][members] == par)
