"""GPU parity: every stage of the HIP path against the CPU oracle, element by
element, on the same seeded inputs.  Integer outputs (neighbour lists, links,
roots, chains, groups) must match exactly; FP64 densities must match bit for
bit because both sides run the same operation sequence (exact integer d^2,
correctly rounded division and square root, no contraction, pairwise sum).
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


def gpu_run(ctx, p, params, ids=None):
    out = ctx.run(p.pos, params, ids=ids, padded=p.padded)
    return {k: (_np(v) if hasattr(v, "detach") else v) for k, v in out.items()}


def _params(p, **kw):
    from paper_1001_3411_amd import HopParams
    return HopParams(periodic=p.periodic, mean_density=p.mean_density, **kw)


def assert_parity(g, r, label=""):
    print(f"[parity] {label}", flush=True)
    assert np.array_equal(g["nbr"], r.nbr), f"{label}: nbr"
    bad = np.flatnonzero(g["density"] != r.density)
    assert bad.size == 0, f"{label}: density differs at {bad[:5]} " \
                          f"{g['density'][bad[:3]]} vs {r.density[bad[:3]]}"
    assert np.array_equal(g["hop"], r.hop), f"{label}: hop"
    assert np.array_equal(g["root"], r.root), f"{label}: root"
    assert np.array_equal(g["chain_of"], r.chain_of), f"{label}: chain_of"
    assert g["n_chains"] == r.n_chains, label
    assert g["n_groups"] == r.n_groups, f"{label}: n_groups {g['n_groups']} vs {r.n_groups}"
    assert np.array_equal(g["group"], r.group), f"{label}: group"
    assert np.array_equal(g["g_count"], r.g_count), f"{label}: g_count"
    assert np.array_equal(g["g_peak"], r.g_peak), f"{label}: g_peak"
    assert np.array_equal(g["g_peak_dens"], r.g_peak_dens), f"{label}: g_peak_dens"


CASES = [("uniform", 64, 1), ("uniform", 100, 2), ("uniform", 1000, 3), ("clustered", 1000, 4),
         ("clustered", 4096, 5), ("lattice", 4096, 6), ("plattice", 4096, 7),
         ("uniform", 4097, 8)]


@pytest.mark.parametrize("kind,n,seed", CASES)
def test_tiny_cases_full_pipeline(ctx, orc, kind, n, seed):
    p = synth.tiny_case(kind, n, seed)
    prm = orc.HopParams()
    if kind in ("uniform", "lattice", "plattice"):
        # uniform-ish sets never reach 80x the mean: lower the thresholds so
        # that chains, boundaries and merges all occur
        prm = orc.HopParams(delta_outer=0.9, delta_saddle=1.2, delta_peak=1.4)
    r = orc.run(p.pos, mean_density=p.mean_density, params=prm)
    g = gpu_run(ctx, p, _params(p, delta_outer=prm.delta_outer, delta_saddle=prm.delta_saddle,
                                delta_peak=prm.delta_peak))
    assert_parity(g, r, f"{kind}-{n}-{seed}")


def test_config1_full_pipeline(ctx, orc):
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    g = gpu_run(ctx, p, _params(p))
    assert r.n_groups > 5
    assert_parity(g, r, "config1")


def test_nonperiodic_padded_subvolume(ctx, orc):
    p = synth.padded_subvolume(20000, 31)
    r = orc.run(p.pos, periodic=False, mean_density=p.mean_density, padded=p.padded,
                padded_rules=True)
    g = gpu_run(ctx, p, _params(p, padded_rules=True))
    assert_parity(g, r, "subvolume-padded")


def test_nonperiodic_without_padded_rules(ctx, orc):
    p = synth.padded_subvolume(12000, 32)
    r = orc.run(p.pos, periodic=False, mean_density=p.mean_density)
    p.padded = None
    g = gpu_run(ctx, p, _params(p))
    assert_parity(g, r, "subvolume-plain")


def test_ids_permutation(ctx, orc):
    p = synth.lattice_box(16)
    perm = np.random.default_rng(5).permutation(p.n)
    ids = (perm.astype(np.int64) * 7 - 3000)
    prm = orc.HopParams(delta_outer=0.5, delta_saddle=0.6, delta_peak=0.7)
    r = orc.run(p.pos[perm], ids=ids, params=prm)
    q = synth.Particles(pos=np.ascontiguousarray(p.pos[perm]), periodic=True,
                        mean_density=p.mean_density)
    g = gpu_run(ctx, q, _params(q, delta_outer=0.5, delta_saddle=0.6, delta_peak=0.7), ids=ids)
    assert_parity(g, r, "lattice-ids")


def test_small_kstore_and_ndens(ctx, orc):
    p = synth.tiny_case("clustered", 4096, 9)
    prm = orc.HopParams(n_dens=32, n_hop=8, n_merge=3, k_store=16)
    r = orc.run(p.pos, mean_density=p.mean_density, params=prm)
    g = gpu_run(ctx, p, _params(p, n_dens=32, n_hop=8, n_merge=3, k_store=16))
    assert_parity(g, r, "ndens32")


def test_stages_on_oracle_inputs(ctx, orc):
    """Each GPU stage fed with the oracle's own upstream outputs."""
    import torch
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    prm = _params(p)
    dev = "cuda:0"
    nbr = torch.from_numpy(r.nbr).to(dev)
    dens = torch.from_numpy(r.density).to(dev)
    hop = ctx.link(nbr, dens, prm)
    assert np.array_equal(_np(hop), r.hop)
    root, chain_of, nc = ctx.groups(torch.from_numpy(r.hop).to(dev), dens, prm)
    assert np.array_equal(_np(root), r.root) and np.array_equal(_np(chain_of), r.chain_of)
    out = ctx.merge(nbr, dens, torch.from_numpy(r.root).to(dev),
                    torch.from_numpy(r.chain_of).to(dev), r.n_chains, prm)
    assert out["n_groups"] == r.n_groups
    assert np.array_equal(_np(out["group"]), r.group)


def test_determinism_two_runs(ctx):
    p = synth.config(1)
    a = gpu_run(ctx, p, _params(p))
    b = gpu_run(ctx, p, _params(p))
    for k in ("nbr", "density", "hop", "group"):
        assert np.array_equal(a[k], b[k]), k


@pytest.fixture(scope="module")
def cfg2(orc):
    p = synth.config(2)
    return p, orc.run(p.pos, mean_density=p.mean_density)


def test_config2_full_pipeline(ctx, cfg2):
    p, r = cfg2
    g = gpu_run(ctx, p, _params(p))
    assert_parity(g, r, "config2")


# FP32 density: r_max^2 and 4 d^2 round once to FP32 (2^-24 relative), the
# division, square roots, 64-term pairwise sum, h^3 and the final product and
# quotient add a few ulps each; the largest error seen on 2M particles is
# below 5e-7 = 8.4 ulp(FP32), so 1e-6 leaves a factor of two.
FP32_REL_TOL = 1e-6


def test_fp32_density_variant(ctx, cfg2):
    from paper_1001_3411_amd.report import group_change_fraction, max_rel_error
    p, r = cfg2
    g = gpu_run(ctx, p, _params(p, density_fp32=True))
    assert np.array_equal(g["nbr"], r.nbr), "the neighbour search must not change"
    err = max_rel_error(r.density, g["density"])
    chg = group_change_fraction(r.group, g["group"])
    print(f"[fp32] max rel err {err:.3e}, group change fraction {chg:.3e}, "
          f"groups {g['n_groups']} vs {r.n_groups}", flush=True)
    assert 0.0 < err <= FP32_REL_TOL
    assert chg < 1e-3


def test_range_error_reported(ctx):
    from paper_1001_3411_amd import HopError
    p = synth.uniform_box(500, 3)
    pos = p.pos.copy()
    pos[7, 1] = 1 << 21
    with pytest.raises(HopError) as e:
        gpu_run(ctx, synth.Particles(pos=pos, periodic=True, mean_density=p.mean_density),
                _params(p))
    assert e.value.code == -2


def test_degenerate_reported(ctx):
    from paper_1001_3411_amd import HopError
    pos = np.zeros((200, 3), np.uint32)
    pos[100:] = 777
    with pytest.raises(HopError) as e:
        gpu_run(ctx, synth.Particles(pos=pos, periodic=True, mean_density=200 / 2.0 ** 63),
                _params(synth.Particles(pos=pos, periodic=True, mean_density=200 / 2.0 ** 63)))
    assert e.value.code == -3


def test_coarse_leaf_ranges_parity(orc):
    """A tiny frontier capacity stops the breadth-first walk near the root,
    so every bucket streams whole subtrees; results must not change."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1001_3411_amd import HopContext
    c = HopContext(0)
    c.set_tuning(front_cap=2)
    try:
        for p in (synth.config(1), synth.padded_subvolume(9000, 41)):
            pr = p.padded is not None
            r = orc.run(p.pos, periodic=p.periodic, mean_density=p.mean_density,
                        padded=p.padded, padded_rules=pr)
            g = gpu_run(c, p, _params(p, padded_rules=pr))
            assert_parity(g, r, f"coarse-{p.name}")
    finally:
        c.close()


@pytest.mark.parametrize("waves", [8, 37, 5000])
def test_persistent_waves_parity(orc, waves):
    """The one-box kNN kernel is a persistent launch whose workgroups take
    buckets from 8 per-XCD queues and move on to the other queues when
    theirs is empty: with the fewest waves allowed, a count that divides
    nothing evenly, and more waves than buckets (capped), every output
    equals the oracle's, for the 63-key heap and the 127-key heap."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1001_3411_amd import HopContext
    c = HopContext(0)
    c.set_tuning(persistent_waves=waves)
    try:
        p = synth.config(1)
        r = orc.run(p.pos, periodic=p.periodic, mean_density=p.mean_density)
        assert_parity(gpu_run(c, p, _params(p)), r, f"waves{waves}-{p.name}")
        q = synth.tiny_case("clustered", 4097, 31)
        prm = orc.HopParams(n_dens=128, n_hop=32, n_merge=8, k_store=100)
        r = orc.run(q.pos, mean_density=q.mean_density, params=prm)
        g = gpu_run(c, q, _params(q, n_dens=128, n_hop=32, n_merge=8, k_store=100))
        assert_parity(g, r, f"waves{waves}-ndens128")
    finally:
        c.close()


def test_dense_cells_parity(ctx, orc):
    """The Morton sort orders particles by the top 48 code bits only (cells
    of 32 grid units); particles sharing such a cell keep their input
    order.  Half of this box lies in a 48^3 cube, so many share cells, in
    shuffled input order, with coincident positions among them: every
    output still equals the oracle's."""
    rng = np.random.default_rng(77)
    blob = rng.integers(1_000_000, 1_000_048, size=(3000, 3), dtype=np.uint32)
    blob[:40] = blob[40:80]  # some coincident pairs
    back = rng.integers(0, 1 << 21, size=(3000, 3), dtype=np.uint32)
    pos = np.concatenate([blob, back])[rng.permutation(6000)]
    p = synth.Particles(pos=pos, periodic=True, mean_density=6000 / float(1 << 21) ** 3,
                        name="dense_cells")
    r = orc.run(p.pos, mean_density=p.mean_density)
    g = gpu_run(ctx, p, _params(p))
    assert r.n_groups >= 1
    assert_parity(g, r, "dense-cells")


@pytest.mark.parametrize("gb", [12, 16])
def test_smaller_grids_parity(ctx, orc, gb):
    """Periodic boxes of side 2^12 and 2^16: the Morton codes have 36 and 48
    bits (all of them sorted) and the sorted coordinates are decoded from
    them; a clustered set with coincident points, every output equal to the
    oracle's."""
    rng = np.random.default_rng(100 + gb)
    side = 1 << gb
    n = 5000
    centre = rng.integers(0, side, size=3)
    blob = (centre + rng.normal(0, side / 200, size=(n // 2, 3))).astype(np.int64) % side
    back = rng.integers(0, side, size=(n - n // 2, 3))
    pos = np.concatenate([blob, back]).astype(np.uint32)[rng.permutation(n)]
    prm = orc.HopParams(grid_bits=gb, delta_outer=10.0, delta_saddle=25.0, delta_peak=30.0)
    r = orc.run(pos, mean_density=n / float(side) ** 3, params=prm)
    p = synth.Particles(pos=pos, periodic=True, mean_density=n / float(side) ** 3, name=f"grid{gb}")
    g = gpu_run(ctx, p, _params(p, grid_bits=gb, delta_outer=10.0, delta_saddle=25.0, delta_peak=30.0))
    assert r.n_groups >= 1
    assert_parity(g, r, f"grid-{gb}")
