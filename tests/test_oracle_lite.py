"""The bounded-memory oracle pipeline (orc_run_lite) against the plain one.

orc_run_lite keeps only the first list columns and a fingerprint of each
whole row, so that a 134M-particle box fits host memory; every output it
does keep must equal orc_run's, on boxes where orc_run still fits.
"""
import numpy as np
import pytest

import synth
from listhash import row_fnv1a


def _same(orc, p, prm=None, ids=None, padded_rules=False, k_keep=16, chunk=5000):
    prm = prm or orc.HopParams()
    kw = dict(periodic=p.periodic, mean_density=p.mean_density, params=prm, ids=ids,
              padded=p.padded, padded_rules=padded_rules)
    r = orc.run(p.pos, **kw)
    l = orc.run_lite(p.pos, k_keep=k_keep, chunk=chunk, **kw)
    assert np.array_equal(l.density, r.density)
    assert np.array_equal(l.nbr, r.nbr[:, :k_keep])
    assert np.array_equal(l.row_hash, row_fnv1a(r.nbr, prm.k_store))
    for k in ("hop", "root", "chain_of", "group", "g_count", "g_peak", "g_peak_dens"):
        assert np.array_equal(getattr(l, k), getattr(r, k)), k
    assert (l.n_chains, l.n_edges, l.n_groups) == (r.n_chains, r.n_edges, r.n_groups)
    return r, l


def test_fingerprint_separates_swapped_columns():
    a = np.array([[5, 1, 2, 3], [5, 2, 1, 3]], np.int32)
    h = row_fnv1a(a)
    assert h[0] != h[1]
    assert row_fnv1a(a[:1])[0] == h[0]


def test_lite_equals_full_on_config1(orc):
    p = synth.config(1)
    r, l = _same(orc, p)
    # the kept d^2 of the last list entry is that of the brute-force list
    sub = np.arange(0, p.n, 97)
    _, d2 = orc.knn(p.pos, 64, queries=sub, method="brute")
    assert np.array_equal(l.r2max[sub], d2[:, -1])
    assert r.n_groups > 5


def test_lite_equals_full_padded_ids_ndens65(orc):
    p = synth.padded_subvolume(9000, 52)
    ids = np.random.default_rng(3).permutation(p.n).astype(np.int64) * 3 + 1
    _same(orc, p, prm=orc.HopParams(n_dens=65, k_store=65), ids=ids, padded_rules=True,
          k_keep=20, chunk=777)


@pytest.mark.slow
def test_lite_equals_full_on_config2(orc):
    _same(orc, synth.config(2), chunk=300_000)


def test_incremental_pieces_equal_full(orc):
    p = synth.tiny_case("clustered", 4096, 14)
    r = orc.run(p.pos, mean_density=p.mean_density)
    L = orc.Lite(p.pos, mean_density=p.mean_density, k_keep=16)
    for c0 in range(0, p.n, 1000):  # ragged last piece
        L.query(c0, min(c0 + 1000, p.n))
    hop, root, chain_of, group, gc, gp, gd, nc, ne, ng = L.finish()
    assert np.array_equal(L.density, r.density) and np.array_equal(L.nbr, r.nbr[:, :16])
    assert np.array_equal(L.row_hash, row_fnv1a(r.nbr))
    for a, b in ((hop, r.hop), (root, r.root), (chain_of, r.chain_of), (group, r.group),
                 (gc, r.g_count), (gp, r.g_peak), (gd, r.g_peak_dens)):
        assert np.array_equal(a, b)
    assert (nc, ne, ng) == (r.n_chains, r.n_edges, r.n_groups)
