"""hop_density_link: the search and the links in one call, the links formed
in Morton order from the sorted copy the search keeps.  Its outputs must be
the outputs of hop_density followed by hop_link, bit for bit, and the
oracle's (the other parity tests run it through HopContext.run as well);
here both paths are compared directly, on the cases where the sorted copy
is shorter than the list (n_hop < 16 < n_dens), as long as it (n_dens = 16),
absent (n_hop > 16 falls back to the two calls), with ids, padded rules, no
list output, ragged last buckets, and the learned-radius search whose
missed buckets are searched again by a second kernel.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1001_3411_amd import HopContext
    c = HopContext(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def _both(ctx, pos, prm, ids=None, padded=None):
    d1, n1 = ctx.density(pos, prm, ids=ids)
    h1 = ctx.link(n1, d1, prm, ids=ids, padded=padded)
    d2, n2, h2 = ctx.density_link(pos, prm, ids=ids, padded=padded)
    # no device error bit may be left set (regression: the binding once
    # freed its device copy of ids before the call, and the padded flags'
    # copy landed in the same memory, so the ids read as duplicates)
    ctx.sync()
    return (_np(d1), _np(n1), _np(h1)), (_np(d2), _np(n2), _np(h2))


def _same(a, b, label):
    print(f"[density_link] {label}", flush=True)
    assert np.array_equal(a[0], b[0]), f"{label}: density"
    assert np.array_equal(a[1], b[1]), f"{label}: nbr"
    assert np.array_equal(a[2], b[2]), f"{label}: hop"


@pytest.mark.parametrize("kind,n,seed,kw", [
    ("clustered", 4096, 11, {}),
    ("uniform", 4097, 12, {}),                                   # ragged last bucket
    ("uniform", 65, 13, {}),                                     # one full + one 1-particle bucket
    ("clustered", 3000, 14, dict(n_dens=16, k_store=16, n_hop=16, n_merge=4)),
    ("clustered", 3000, 15, dict(n_dens=32, k_store=16, n_hop=8, n_merge=3)),
    ("clustered", 3000, 16, dict(n_dens=32, k_store=32, n_hop=24, n_merge=4)),  # two calls
])
def test_fused_equals_two_calls(ctx, kind, n, seed, kw):
    from paper_1001_3411_amd import HopParams
    p = synth.tiny_case(kind, n, seed)
    prm = HopParams(mean_density=p.mean_density, **kw)
    a, b = _both(ctx, p.pos, prm)
    _same(a, b, f"{kind}-{n}-{seed}-{kw}")


def test_fused_with_ids_and_padded_rules(ctx):
    from paper_1001_3411_amd import HopParams
    p = synth.padded_subvolume(20000, 33)
    ids = np.random.default_rng(3).permutation(p.n).astype(np.int64) * 5 + 11
    prm = HopParams(periodic=False, mean_density=p.mean_density, padded_rules=True)
    a, b = _both(ctx, p.pos, prm, ids=ids, padded=p.padded)
    _same(a, b, "subvolume-ids-padded")


def test_fused_matches_oracle_with_n_hop_above_16(ctx, orc):
    p = synth.tiny_case("clustered", 4096, 17)
    prm = orc.HopParams(n_dens=32, n_hop=24, n_merge=4, k_store=32)
    r = orc.run(p.pos, mean_density=p.mean_density, params=prm)
    from paper_1001_3411_amd import HopParams
    d, nb, h = ctx.density_link(p.pos, HopParams(mean_density=p.mean_density, n_dens=32, n_hop=24,
                                                 n_merge=4, k_store=32))
    assert np.array_equal(_np(nb), r.nbr) and np.array_equal(_np(d), r.density)
    assert np.array_equal(_np(h), r.hop)


def test_fused_without_list_output(ctx, orc):
    from paper_1001_3411_amd import HopParams
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    d, nb, h = ctx.density_link(p.pos, HopParams(mean_density=p.mean_density), want_nbr=False)
    assert nb is None
    assert np.array_equal(_np(d), r.density)
    assert np.array_equal(_np(h), r.hop)


def test_fused_config2(ctx):
    from paper_1001_3411_amd import HopParams
    p = synth.config(2)
    a, b = _both(ctx, p.pos, HopParams(mean_density=p.mean_density))
    _same(a, b, "config2")


def test_fused_with_learned_radius(ctx):
    """Buckets that miss the predicted radius are searched again by a second
    kernel, which writes their sorted copies too."""
    from paper_1001_3411_amd import HOP_RADIUS_ANALYTIC, HopParams
    p = synth.config(1)
    prm = HopParams(mean_density=p.mean_density)
    d0, n0 = ctx.density(p.pos, prm)
    h0 = ctx.link(n0, d0, prm)
    # a radius far too small: every bucket goes through the second search
    ctx.radius_load(HOP_RADIUS_ANALYTIC, None, -6.0)
    try:
        from dataclasses import replace
        d1, n1, h1 = ctx.density_link(p.pos, replace(prm, learned_radius=True))
        st = ctx.stats()
    finally:
        ctx.radius_load(0)
    assert st["misses"] == p.n
    _same((_np(d0), _np(n0), _np(h0)), (_np(d1), _np(n1), _np(h1)), "learned-all-miss")


def test_abi_rejects_null_nbr_for_long_links(ctx):
    from paper_1001_3411_amd import HopError, HopParams
    p = synth.tiny_case("uniform", 1000, 18)
    with pytest.raises(HopError):
        ctx.density_link(p.pos, HopParams(mean_density=p.mean_density, n_dens=32, n_hop=24,
                                          n_merge=4, k_store=32), want_nbr=False)


def test_work_counters(ctx):
    """Profiling bit 2 counts the kNN kernel's work on the device: tree
    nodes tested, leaves streamed, heap-insertion loop iterations (each for
    the whole wave) and candidates offered to a lane's heap (each costs that
    lane one iteration, so a bucket's lanes together are offered at most 64
    per iteration).  Counting leaves the outputs unchanged; one bucket of 64
    particles with N_dens = 64 fills every heap with its 63 others
    directly, so nothing is offered."""
    from paper_1001_3411_amd import HopParams
    p = synth.config(1)
    prm = HopParams(mean_density=p.mean_density)
    ctx.set_profiling(0)
    d0, n0 = ctx.density(p.pos, prm)
    ctx.set_profiling(3)
    d1, n1 = ctx.density(p.pos, prm)
    st = ctx.stats()
    ctx.set_profiling(0)
    assert np.array_equal(_np(d0), _np(d1)) and np.array_equal(_np(n0), _np(n1))
    it, off = st["insert_iterations"], st["offered"]
    print(f"[counters] {p.name}: {it / ((p.n + 63) // 64):.1f} insertion iterations per bucket, "
          f"{off / p.n:.1f} offered per query, {st['nodes_visited'] / p.n:.1f} nodes per query",
          flush=True)
    assert 0 < off <= 64 * it and st["nodes_visited"] > 0 and st["leaves_scanned"] > 0
    q = synth.tiny_case("uniform", 64, 3)
    ctx.set_profiling(3)
    ctx.density(q.pos, HopParams(mean_density=q.mean_density, periodic=q.periodic))
    st = ctx.stats()
    ctx.set_profiling(0)
    assert st["insert_iterations"] == 0 and st["offered"] == 0
