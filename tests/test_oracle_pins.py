"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Nothing here compares the oracle with itself: each check is a brute-force
definition written independently in NumPy, a closed form, an invariance of
the method, or a worked example printed in the paper.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = 1 << 21


# --------------------------------------------------------------------------
# brute-force kNN in NumPy: sort every other particle by (d^2, id, index)
# --------------------------------------------------------------------------

def np_knn(pos, k, periodic=True, ids=None):
    pos = pos.astype(np.int64)
    n = pos.shape[0]
    ids = np.arange(n, dtype=np.int64) if ids is None else ids.astype(np.int64)
    out = np.empty((n, k), np.int64)
    d2out = np.empty((n, k), np.int64)
    for i in range(n):
        d = np.abs(pos - pos[i])
        if periodic:
            d = np.minimum(d, G - d)
        d2 = (d * d).sum(axis=1)
        d2[i] = -1  # self first
        order = np.lexsort((np.arange(n), ids, d2))
        out[i] = order[:k]
        d2out[i] = np.maximum(d2[order[:k]], 0)
    return out, d2out


TINY = [("uniform", 64, 1), ("uniform", 100, 2), ("uniform", 1000, 3),
        ("clustered", 1000, 4), ("lattice", 4096, 5), ("plattice", 1000, 6)]


@pytest.mark.parametrize("kind,n,seed", TINY)
@pytest.mark.parametrize("periodic", [True, False])
def test_knn_brute_matches_numpy_definition(orc, kind, n, seed, periodic):
    p = synth.tiny_case(kind, n, seed)
    k = min(64, p.n)
    ref, ref_d2 = np_knn(p.pos, k, periodic)
    for method in ("brute", "kdtree"):
        nbr, d2 = orc.knn(p.pos, k, periodic=periodic, method=method)
        assert np.array_equal(nbr, ref), method
        assert np.array_equal(d2, ref_d2), method


def test_knn_ties_follow_ids(orc):
    # perfect lattice: the 64th neighbour sits in the 24-fold d^2 = 6a^2 shell,
    # so which 7 of the 24 are kept is decided by the ids
    p = synth.lattice_box(16)
    rng = np.random.default_rng(11)
    ids = rng.permutation(p.n).astype(np.int64) * 3 + 5
    ref, _ = np_knn(p.pos, 64, True, ids)
    nbr, _ = orc.knn(p.pos, 64, ids=ids)
    assert np.array_equal(nbr, ref)


def test_kdtree_equals_brute_on_clustered_box(orc):
    p = synth.config(1)
    sub = np.arange(0, p.n, 7)
    a, da = orc.knn(p.pos, 64, queries=sub, method="brute")
    b, db = orc.knn(p.pos, 64, queries=sub, method="kdtree")
    assert np.array_equal(a, b) and np.array_equal(da, db)


def test_knn_coincident_points(orc):
    rng = np.random.default_rng(3)
    pos = synth.quantise(rng.random((300, 3)))
    pos[10:40] = pos[10]  # 30 coincident particles
    ref, _ = np_knn(pos, 64, True)
    nbr, _ = orc.knn(pos, 64)
    assert np.array_equal(nbr, ref)


# --------------------------------------------------------------------------
# density
# --------------------------------------------------------------------------

def _m4_textbook(q):
    """M4 cubic spline (Monaghan & Lattanzio 1985), 3-D normalisation 1/(pi h^3)."""
    if q < 1:
        return 1.0 - 1.5 * q * q + 0.75 * q ** 3
    if q < 2:
        return 0.25 * (2.0 - q) ** 3
    return 0.0


def test_m4_is_normalised():
    # integral of W over space = 1: 4 pi int_0^2 w(q) q^2 dq / pi = 1
    from scipy.integrate import quad
    val = 4.0 * quad(lambda q: _m4_textbook(q) * q * q, 0, 2, points=[1.0])[0]
    assert abs(val - 1.0) < 1e-12


def test_density_perfect_lattice_closed_form(orc):
    # simple cubic lattice, spacing a: with 64 neighbours (self included) the
    # farthest lies in the d^2 = 6 a^2 shell, so h^2 = 1.5 a^2 and the shells
    # m = 0..5 with multiplicities r3(m) = 1, 6, 12, 8, 6, 24 contribute.
    shells = {0: 1, 1: 6, 2: 12, 3: 8, 4: 6, 5: 24}
    # r3 multiplicities counted here independently
    cnt = {}
    r = range(-3, 4)
    for v in itertools.product(r, r, r):
        m = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
        cnt[m] = cnt.get(m, 0) + 1
    assert all(cnt[m] == c for m, c in shells.items())
    assert sum(shells.values()) + cnt[6] > 64 > sum(shells.values())
    h = math.sqrt(1.5)
    S = sum(c * _m4_textbook(math.sqrt(m) / h) for m, c in shells.items())
    closed = S / (math.pi * h ** 3)          # rho_bar = 1 / a^3
    assert abs(closed - 0.99963851) < 5e-9
    p = synth.lattice_box(16)
    _, d2 = orc.knn(p.pos, 64)
    dens = orc.density(d2, p.mean_density)
    assert np.all(dens == dens[0])           # every particle bit-identical
    assert abs(dens[0] - closed) <= 4e-16 * closed


def test_density_perturbed_lattice_near_one(orc):
    p = synth.perturbed_lattice_box(32, 9)
    _, d2 = orc.knn(p.pos, 64)
    dens = orc.density(d2, p.mean_density)
    assert abs(dens.mean() - 1.0) < 0.01


def test_density_only_uses_ndens_neighbours(orc):
    # the density depends only on the N_dens nearest neighbours (section 3):
    # moving a far particle does not change a particle's density
    p = synth.uniform_box(2000, 5)
    nbr, d2 = orc.knn(p.pos, 64)
    dens = orc.density(d2, p.mean_density)
    i = 17
    far = np.setdiff1d(np.arange(p.n), nbr[i])
    pos2 = p.pos.copy()
    far_d2 = ((np.minimum(np.abs(p.pos[far].astype(np.int64) - p.pos[i]),
                          G - np.abs(p.pos[far].astype(np.int64) - p.pos[i]))) ** 2).sum(1)
    j = far[np.argmax(far_d2)]
    pos2[j] = (pos2[j] + 12345) % G
    _, d2b = orc.knn(pos2, 64, queries=np.array([i]))
    if np.array_equal(d2b[0], d2[i]):
        assert orc.density(d2b, p.mean_density)[0] == dens[i]


def test_density_scale_invariance_bit_exact(orc):
    # doubling every coordinate (grid 2^20 -> 2^21) and dividing the mean
    # density by 8 scales h^3 and the normalisation by exact powers of two
    rng = np.random.default_rng(8)
    pos = (rng.random((3000, 3)) * (1 << 20)).astype(np.uint32)
    md = 3000 / float(1 << 60)
    _, d2a = orc.knn(pos, 64, grid_bits=20)
    _, d2b = orc.knn(pos * 2, 64, grid_bits=21)
    a = orc.density(d2a, md)
    b = orc.density(d2b, md / 8)
    assert np.array_equal(a, b)


def test_degenerate_coincident_raises(orc):
    pos = np.zeros((100, 3), np.uint32)
    pos[80:] = 5000
    with pytest.raises(RuntimeError):
        orc.run(pos)


# --------------------------------------------------------------------------
# hop and chains: invariants stated in the paper
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cfg1(orc):
    p = synth.config(1)
    return p, orc.run(p.pos)


def _key(d, i):
    return (d, -i)


def test_hop_goes_uphill_and_roots_are_local_maxima(cfg1):
    p, r = cfg1
    d = r.density
    for i in range(p.n):
        h = r.hop[i]
        assert h in r.nbr[i, :16]
        assert _key(d[h], h) >= _key(d[i], i)
        assert (h == i) == (_key(d[h], h) == _key(d[i], i))
        best = max(r.nbr[i, :16], key=lambda j: _key(d[j], j))
        assert best == h
    roots = np.flatnonzero(r.hop == np.arange(p.n))
    for rt in roots:
        assert all(_key(d[rt], rt) >= _key(d[j], j) for j in r.nbr[rt, :16])


def test_chains_idempotent_and_acyclic(cfg1):
    p, r = cfg1
    assert np.array_equal(r.root[r.root], r.root)
    assert np.all(r.hop[r.root] == r.root)
    alive = r.density >= 80.0
    assert np.array_equal(r.chain_of >= 0, alive)
    # chain numbers follow the root index
    roots = np.unique(r.root[alive])
    assert np.all(r.chain_of[alive] == np.searchsorted(roots, r.root[alive]))
    assert r.n_chains == roots.size


def test_run_is_deterministic(orc, cfg1):
    p, r = cfg1
    r2 = orc.run(p.pos)
    assert np.array_equal(r.group, r2.group) and np.array_equal(r.density, r2.density)


def test_groups_sorted_by_size_and_consistent(cfg1):
    p, r = cfg1
    assert np.all(np.diff(r.g_count) <= 0)
    cnt = np.bincount(r.group[r.group >= 0], minlength=r.n_groups)
    assert np.array_equal(cnt, r.g_count)
    assert np.all(r.density[r.g_peak] == r.g_peak_dens)
    # every group holds a particle at or above delta_peak
    for g in range(r.n_groups):
        assert r.density[r.group == g].max() >= 240.0


def _invariance_check(orc, pos, r0):
    r1 = orc.run(pos)
    assert np.array_equal(r1.group, r0.group)
    assert np.array_equal(r1.density, r0.density)
    assert np.array_equal(r1.nbr, r0.nbr)


def test_translation_reflection_axis_swap_invariance(orc, cfg1):
    p, r = cfg1
    pos = p.pos.astype(np.int64)
    _invariance_check(orc, ((pos + np.array([123457, 999999, 2 ** 20 + 3])) % G).astype(np.uint32), r)
    _invariance_check(orc, ((G - pos) % G).astype(np.uint32), r)
    _invariance_check(orc, np.ascontiguousarray(p.pos[:, [2, 0, 1]]), r)


def test_permutation_invariance_with_carried_ids(orc):
    p = synth.tiny_case("clustered", 4096, 21)
    r0 = orc.run(p.pos, mean_density=p.mean_density)
    perm = np.random.default_rng(2).permutation(p.n)
    ids = perm.astype(np.int64)  # original index of each stored particle
    r1 = orc.run(p.pos[perm], mean_density=p.mean_density, ids=ids)
    assert np.array_equal(r1.density, r0.density[perm])
    assert np.array_equal(perm[r1.nbr], r0.nbr[perm])
    assert np.array_equal(perm[r1.hop], r0.hop[perm])
    assert np.array_equal(r1.group, r0.group[perm])
    assert np.array_equal(perm[r1.g_peak], r0.g_peak)


def test_lattice_permutation_invariance_with_ids(orc):
    # heavy ties: results only agree when ties follow the carried ids
    p = synth.lattice_box(16)
    r0 = orc.run(p.pos, params=orc.HopParams(delta_outer=0.5, delta_saddle=0.6,
                                              delta_peak=0.7))
    perm = np.random.default_rng(5).permutation(p.n)
    r1 = orc.run(p.pos[perm], ids=perm.astype(np.int64),
                 params=orc.HopParams(delta_outer=0.5, delta_saddle=0.6, delta_peak=0.7))
    assert np.array_equal(perm[r1.nbr], r0.nbr[perm])
    assert np.array_equal(perm[r1.hop], r0.hop[perm])
    assert np.array_equal(r1.group, r0.group[perm])


# --------------------------------------------------------------------------
# boundary table: a hand-worked case
# --------------------------------------------------------------------------

def test_saddles_hand_worked(orc):
    # 7 particles, N_merge = 3 (ranks 1 and 2 searched); rows: self first
    nbr = np.array([[0, 1, 2], [1, 0, 3], [2, 3, 0], [3, 2, 4],
                    [4, 3, 5], [5, 4, 6], [6, 5, 4]], np.int32)
    dens = np.array([100.0, 90.0, 150.0, 120.0, 85.0, 300.0, 50.0])
    chain_of = np.array([0, 0, 1, 1, 2, 2, -1], np.int32)
    padded = np.array([0, 0, 0, 1, 1, 0, 0], np.uint8)
    lo, hi, s = orc.saddles(nbr, dens, chain_of, 3)
    # pairs: 0->2 (0,1) 125 ; 1->3 (0,1) 105 ; 2->0 (0,1) 125 ;
    # 3->4 (1,2) 102.5 ; 4->3 (1,2) 102.5 ; 6 is not in a chain
    assert lo.tolist() == [0, 1] and hi.tolist() == [1, 2]
    assert s.tolist() == [125.0, 102.5]
    # padded rule: 3 and 4 are both padded, so the (1,2) boundary vanishes
    lo, hi, s = orc.saddles(nbr, dens, chain_of, 3, padded=padded, padded_rules=True)
    assert lo.tolist() == [0] and hi.tolist() == [1] and s.tolist() == [125.0]


# --------------------------------------------------------------------------
# merge: the paper's worked example, textbook special cases, brute force
# --------------------------------------------------------------------------

def _halos_from(chain_halo, names):
    groups = {}
    for c, h in enumerate(chain_halo):
        if h >= 0:
            groups.setdefault(int(h), []).append(names[c])
    return sorted(sorted(g) for g in groups.values())


def test_merge_figure1_worked_example(orc):
    with open(os.path.join(GOLDEN, "fig1_merge.json")) as f:
        fx = json.load(f)
    names = fx["chains"]
    ix = {c: i for i, c in enumerate(names)}
    for edges, expect in ((fx["edges"], fx["expected_halos"]),
                          (fx["variant_de_wins"]["edges"],
                           fx["variant_de_wins"]["expected_halos"])):
        lo = np.array([min(ix[a], ix[b]) for a, b, _ in edges], np.int32)
        hi = np.array([max(ix[a], ix[b]) for a, b, _ in edges], np.int32)
        s = np.array([w for _, _, w in edges])
        ch = orc.merge(np.array(fx["chain_peak"]), lo, hi, s, fx["delta_saddle"],
                       fx["delta_peak"])
        assert _halos_from(ch, names) == sorted(sorted(g) for g in expect)


def test_merge_large_saddle_keeps_protohalos_apart(orc, cfg1):
    p, _ = cfg1
    r = orc.run(p.pos, params=orc.HopParams(delta_saddle=1e30))
    root_dens = r.density[r.root]
    for g in range(r.n_groups):
        members = r.group == g
        proto_roots = np.unique(r.root[members & (root_dens >= 240.0)])
        assert proto_roots.size == 1


def test_fof_special_case(orc):
    # delta_outer = delta_saddle = delta_peak = 0: every chain is a proto-halo
    # and every boundary merges, so groups are the connected components of
    # the graph {hop links} U {N_merge neighbour links} over all particles
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    p = synth.tiny_case("clustered", 4096, 33)
    prm = orc.HopParams(delta_outer=0.0, delta_saddle=0.0, delta_peak=0.0)
    r = orc.run(p.pos, params=prm)
    n = p.n
    rows = np.concatenate([np.arange(n), np.repeat(np.arange(n), 3)])
    cols = np.concatenate([r.hop, r.nbr[:, 1:4].reshape(-1)])
    A = coo_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n))
    nc, lab = connected_components(A, directed=False)
    assert r.n_groups == nc
    # same partition: a bijection between labels
    pairs = set(zip(lab.tolist(), r.group.tolist()))
    assert len(pairs) == nc


def _brute_msf_halos(n, peaks, edges, d_saddle, d_peak):
    """Enumerate every edge subset; the unique maximum-weight spanning forest
    of the chain graph plus a virtual root tied to every proto-halo (weights
    are distinct powers of two, so the maximum is unique)."""
    proto = [pk >= d_peak for pk in peaks]
    V = n
    order = sorted(range(len(edges)), key=lambda e: (edges[e][2], -edges[e][0], -edges[e][1]))
    w = {e: 2 ** r for r, e in enumerate(order)}
    best, best_set = -1, None
    for mask in range(1 << len(edges)):
        par = list(range(n + 1))

        def f(x):
            while par[x] != x:
                x = par[x]
            return x
        ok = True
        for c in range(n):  # virtual-root edges are always present
            if proto[c]:
                a, b = f(c), f(V)
                if a == b:
                    ok = False
                    break
                par[a] = b
        if not ok:
            continue
        tot = 0
        for e in range(len(edges)):
            if mask >> e & 1:
                a, b = f(edges[e][0]), f(edges[e][1])
                if a == b:
                    ok = False
                    break
                par[a] = b
                tot += w[e]
        if ok and tot > best:
            # must be spanning: every component of the graph is connected
            best, best_set = tot, mask
    # halos: forest edges plus proto pairs with a boundary >= d_saddle
    par = list(range(n))

    def f2(x):
        while par[x] != x:
            x = par[x]
        return x
    for e in range(len(edges)):
        a, b, s = edges[e]
        if (best_set >> e & 1) or (proto[a] and proto[b] and s >= d_saddle):
            ra, rb = f2(a), f2(b)
            if ra != rb:
                par[max(ra, rb)] = min(ra, rb)
    comp = [f2(c) for c in range(n)]
    rooted = {comp[c] for c in range(n) if proto[c]}
    return [min(x for x in range(n) if comp[x] == comp[c]) if comp[c] in rooted else -1
            for c in range(n)]


def test_merge_matches_bruteforce_spanning_forest(orc):
    rng = np.random.default_rng(17)
    for trial in range(60):
        n = int(rng.integers(2, 7))
        peaks = rng.choice([150.0, 230.0, 250.0, 400.0], size=n)
        pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
        m = int(rng.integers(1, min(len(pairs), 8) + 1))
        sel = rng.choice(len(pairs), size=m, replace=False)
        svals = rng.permutation(np.linspace(90, 260, m))
        edges = [(pairs[s][0], pairs[s][1], float(v)) for s, v in zip(sel, svals)]
        expect = _brute_msf_halos(n, peaks, edges, 200.0, 240.0)
        got = orc.merge(peaks, np.array([e[0] for e in edges], np.int32),
                        np.array([e[1] for e in edges], np.int32),
                        np.array([e[2] for e in edges]), 200.0, 240.0)
        assert got.tolist() == expect, (trial, peaks, edges)


def _clump(center, n, rng, scale):
    x = center + rng.normal(0, scale, size=(n, 3))
    return synth.quantise(x)


def test_isolated_clumps_give_one_halo_each(orc):
    rng = np.random.default_rng(4)
    one = np.concatenate([_clump(np.array([0.3, 0.3, 0.3]), 1500, rng, 0.01),
                          synth.quantise(rng.random((1500, 3)))])
    r1 = orc.run(one)
    assert r1.n_groups == 1
    two = np.concatenate([_clump(np.array([0.25, 0.25, 0.25]), 1500, rng, 0.01),
                          _clump(np.array([0.75, 0.75, 0.75]), 1500, rng, 0.01),
                          synth.quantise(rng.random((1500, 3)))])
    r2 = orc.run(two)
    assert r2.n_groups == 2


def test_padded_particles_get_no_group(orc):
    p = synth.padded_subvolume(6000, 77)
    r = orc.run(p.pos, periodic=False, mean_density=p.mean_density, padded=p.padded,
                padded_rules=True)
    pad = p.padded.astype(bool)
    assert np.all(r.group[pad] == -1)
    assert np.all(r.hop[pad] == np.flatnonzero(pad))


# --------------------------------------------------------------------------
# labels: the group order (count desc, peak density desc, peak id asc) and
# the padded-only rule, on hand-built chain tables whose expected numbering
# is written out by hand
# --------------------------------------------------------------------------

def test_labels_equal_counts_order_by_peak_density(orc):
    # three one-chain halos of two particles each; chain peaks 300, 500, 400
    chain_of = np.array([0, 0, 1, 1, 2, 2], np.int32)
    chain_root = np.array([0, 2, 4], np.int32)
    chain_peak = np.array([300.0, 500.0, 400.0])
    chain_halo = np.array([0, 1, 2], np.int32)
    group, gc, gp, gd = orc.labels(chain_of, chain_root, chain_peak, chain_halo)
    # densest peak first: chain 1 -> 0, chain 2 -> 1, chain 0 -> 2
    assert group.tolist() == [2, 2, 0, 0, 1, 1]
    assert gc.tolist() == [2, 2, 2]
    assert gp.tolist() == [2, 4, 0]
    assert gd.tolist() == [500.0, 400.0, 300.0]


def test_labels_count_comes_before_peak_density(orc):
    # halo of chain 0: 3 particles, peak 250; halo of chain 1: 2 particles,
    # peak 900 -- the larger halo is number 0 although its peak is lower
    chain_of = np.array([0, 0, 0, 1, 1], np.int32)
    group, gc, gp, gd = orc.labels(chain_of, np.array([1, 3], np.int32),
                                   np.array([250.0, 900.0]), np.array([0, 1], np.int32))
    assert group.tolist() == [0, 0, 0, 1, 1]
    assert gc.tolist() == [3, 2] and gp.tolist() == [1, 3]


def test_labels_equal_counts_and_peaks_order_by_peak_id(orc):
    # equal counts and equal peak densities: the peak with the smaller id
    # comes first; without ids the index decides, with ids the ids decide
    chain_of = np.array([0, 1, 2, 0, 1, 2], np.int32)
    chain_root = np.array([3, 1, 5], np.int32)
    chain_peak = np.array([300.0, 300.0, 300.0])
    chain_halo = np.array([0, 1, 2], np.int32)
    group, _, gp, _ = orc.labels(chain_of, chain_root, chain_peak, chain_halo)
    # peaks by index: 1 (chain 1) -> 0, 3 (chain 0) -> 1, 5 (chain 2) -> 2
    assert gp.tolist() == [1, 3, 5]
    assert group.tolist() == [1, 0, 2, 1, 0, 2]
    ids = np.array([60, 50, 40, 30, 20, 10], np.int64)
    group, _, gp, _ = orc.labels(chain_of, chain_root, chain_peak, chain_halo, ids=ids)
    # ids of the peaks: 5 -> 10, 3 -> 30, 1 -> 50, so chain 2 -> 0,
    # chain 0 -> 1, chain 1 -> 2
    assert gp.tolist() == [5, 3, 1]
    assert group.tolist() == [1, 2, 0, 1, 2, 0]


def test_labels_halo_peak_is_its_densest_chain(orc):
    # one halo of chains 0 and 1 (peaks 250 and 600), one halo of chain 2
    # (peak 450); equal counts, so the first halo's peak (600) puts it first
    chain_of = np.array([0, 1, 2, 2], np.int32)
    chain_root = np.array([0, 1, 3], np.int32)
    chain_peak = np.array([250.0, 600.0, 450.0])
    chain_halo = np.array([0, 0, 2], np.int32)
    group, gc, gp, gd = orc.labels(chain_of, chain_root, chain_peak, chain_halo)
    assert group.tolist() == [0, 0, 1, 1]
    assert gp.tolist() == [1, 3] and gd.tolist() == [600.0, 450.0]


def test_labels_padded_only_halo_gets_no_number(orc):
    # halo of chain 0: particles 0, 1 (both padded); halo of chain 1:
    # particles 2, 3, 4 with 3 and 4 padded (one labelled member); halo of
    # chain 2: particles 5, 6 (two labelled members); particle 7 unchained
    chain_of = np.array([0, 0, 1, 1, 1, 2, 2, -1], np.int32)
    chain_root = np.array([0, 2, 5], np.int32)
    chain_peak = np.array([900.0, 800.0, 300.0])
    chain_halo = np.array([0, 1, 2], np.int32)
    padded = np.array([1, 1, 0, 1, 1, 0, 0, 0], np.uint8)
    group, gc, gp, _ = orc.labels(chain_of, chain_root, chain_peak, chain_halo,
                                  padded=padded, padded_rules=True)
    # chain 0's halo has no unpadded member: no number; chain 2's halo (2
    # members) precedes chain 1's (1 member) despite the lower peak
    assert group.tolist() == [-1, -1, 1, -1, -1, 0, 0, -1]
    assert gc.tolist() == [2, 1] and gp.tolist() == [5, 2]
    # without the padded rules every halo counts all its members
    group, gc, _, _ = orc.labels(chain_of, chain_root, chain_peak, chain_halo, padded=padded)
    assert group.tolist() == [1, 1, 0, 0, 0, 2, 2, -1]
    assert gc.tolist() == [3, 2, 2]
