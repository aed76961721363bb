"""Per-halo statistics on the GPU against the oracle (oracle/halo.py).

Centres of mass and maximum radii are exact functions of the inputs on
both sides (integer offset sums, one FP64 division, a fixed FP64 operation
sequence per member, a maximum), so they must match bit for bit.  Bulk
velocities are FP64 sums in different orders: each component must lie
within the FP64 summation bound of the other,
|a - b| <= 2 (count - 1) u sum|v| / count + 2 u |b|, u = 2^-53 (the bound
for either order against the exact sum, applied to the pair).
"""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


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


def _check(ctx, p, params, r, label, vel=None, stats_ctx=None):
    from oracle import halo
    out = ctx.run(p.pos, params, padded=p.padded)
    assert np.array_equal(_np(out["group"]), r.group), label
    sc = stats_ctx or ctx
    g = sc.halo_stats(p.pos, out["group"], out["table"], params, vel=vel)
    sc.sync()
    ref = halo.halo_stats(p.pos, r.group, r.g_peak, periodic=params.periodic, vel=vel)
    print(f"[halo] {label}: {r.n_groups} halos", flush=True)
    assert np.array_equal(ref["count"], r.g_count)
    assert np.array_equal(_np(g["com"]), ref["com"]), f"{label}: com"
    assert np.array_equal(_np(g["rmax"]), ref["rmax"]), f"{label}: rmax"
    if vel is not None:
        a, b = _np(g["vbulk"]), ref["vbulk"]
        c = ref["count"][:, None].astype(np.float64)
        bound = 2 * (c - 1) * U * ref["vabs"] / c + 2 * U * np.abs(b)
        assert np.all(np.abs(a - b) <= bound), f"{label}: vbulk"


def test_tiny_periodic_clustered(ctx, orc):
    from paper_1001_3411_amd import HopParams
    p = synth.tiny_case("clustered", 4096, 21)
    prm = HopParams(mean_density=p.mean_density, delta_outer=5.0, delta_saddle=12.5, delta_peak=15.0)
    r = orc.run(p.pos, mean_density=p.mean_density,
                params=orc.HopParams(delta_outer=5.0, delta_saddle=12.5, delta_peak=15.0))
    assert r.n_groups > 1
    vel = np.random.default_rng(4).normal(0, 200, (p.n, 3)).astype(np.float32)
    _check(ctx, p, prm, r, "tiny", vel=vel)


def test_config1_with_velocities(ctx, orc):
    from paper_1001_3411_amd import HopParams
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    vel = np.random.default_rng(5).normal(0, 300, (p.n, 3)).astype(np.float32)
    _check(ctx, p, HopParams(mean_density=p.mean_density), r, "config1", vel=vel)


def test_input_order_on_a_fresh_context(ctx, orc):
    """A context whose last kNN call sorted these particles takes the members
    in that Morton order (the other tests); one that has sorted nothing
    takes them in input order: the same exact centres and radii, the bulk
    velocities within the same bound."""
    from paper_1001_3411_amd import HopContext, HopParams
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    vel = np.random.default_rng(6).normal(0, 300, (p.n, 3)).astype(np.float32)
    fresh = HopContext(0)
    try:
        _check(ctx, p, HopParams(mean_density=p.mean_density), r, "config1-input-order", vel=vel,
               stats_ctx=fresh)
    finally:
        fresh.close()


def test_halo_across_the_box_edge(ctx, orc):
    """A clump centred on a corner of the periodic box: its members sit at
    both ends of every axis and its centre must come out near the corner."""
    from paper_1001_3411_amd import HopParams
    G = 1 << 21
    rng = np.random.default_rng(6)
    clump = np.mod(rng.normal(0, 4000, (3000, 3)).astype(np.int64), G)
    back = rng.integers(0, G, (3000, 3))
    pos = np.concatenate([clump, back]).astype(np.uint32)
    p = synth.Particles(pos=pos, periodic=True, mean_density=pos.shape[0] / float(1 << 63))
    r = orc.run(p.pos, mean_density=p.mean_density)
    assert r.n_groups >= 1
    _check(ctx, p, HopParams(mean_density=p.mean_density), r, "edge")
    from oracle import halo
    ref = halo.halo_stats(p.pos, r.group, r.g_peak)
    c = ref["com"][0]
    dist = np.minimum(c, G - c)
    assert np.all(dist < 2000), c     # the biggest halo is the corner clump


def test_padded_subvolume_nonperiodic(ctx, orc):
    from paper_1001_3411_amd import HopParams
    p = synth.padded_subvolume(20000, 35)
    r = orc.run(p.pos, periodic=False, mean_density=p.mean_density, padded=p.padded,
                padded_rules=True)
    _check(ctx, p, HopParams(periodic=False, mean_density=p.mean_density, padded_rules=True), r,
           "subvolume")


def test_config3_timing(ctx):
    import torch
    from paper_1001_3411_amd import HopParams
    p = synth.config(3)
    prm = HopParams(mean_density=p.mean_density)
    out = ctx.run(p.pos, prm)
    pos = torch.from_numpy(p.pos.view(np.int32)).cuda()
    vel = torch.zeros((p.n, 3), dtype=torch.float32, device="cuda")
    ctx.halo_stats(pos, out["group"], out["table"], prm, vel=vel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        g = ctx.halo_stats(pos, out["group"], out["table"], prm, vel=vel)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 3 * 1e3
    print(f"[halo] config 3: {p.n} particles, {out['n_groups']} halos, {ms:.2f} ms", flush=True)
    assert np.all(_np(g["vbulk"]) == 0.0)
    assert np.all(_np(g["rmax"]) >= 0.0)
