"""The decomposition front end and the stitching end to end, against the
oracle's whole-box run of the 2,097,152-particle box.  Cut into 8
load-balanced, directionally padded subvolumes and run through the batched
call, every core particle whose whole-box neighbour sphere lies inside its
padded subvolume gets exactly the whole-box density (same neighbours at the
same exact distances, same global mean density, same operation sequence);
particles nearer the padded box's edge than their 64th neighbour are only
counted: how many there are is what the safety factor s of Eq. (1)
controls.  Stitched (chains rebuilt through padded particles, one boundary
table, one merge), every whole-box output is reproduced.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def box2(orc):
    p = synth.config(2)
    return p, orc.run(p.pos, mean_density=p.mean_density)


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1001_3411_amd import HopContext
    c = HopContext(0)
    yield c
    c.close()


def test_padded_subvolumes_reproduce_box_densities(ctx, box2):
    from paper_1001_3411_amd import HopParams
    from paper_1001_3411_amd.decompose import decompose
    G = 1 << 21
    p, r = box2
    dens_full = r.density
    far = r.nbr[:, -1]
    d = decompose(p.pos, 8, seed=3)
    sub = HopParams(periodic=False, padded_rules=True, mean_density=p.mean_density)
    out = ctx.run_batch(d.pos, d.offsets, sub, padded=d.padded,
                        mean_density=np.full(8, p.mean_density))
    dens_b = out["density"].cpu().numpy()
    p64 = p.pos.astype(np.int64)
    checked = 0
    for t in range(8):
        a, b = int(d.offsets[t]), int(d.offsets[t + 1])
        rows = np.arange(a, b)[d.padded[a:b] == 0]
        gi = d.index[rows]
        dx = np.abs(p64[gi] - p64[far[gi]])
        dx = np.minimum(dx, G - dx)
        r = np.sqrt((dx.astype(np.float64) ** 2).sum(axis=1))
        span = (d.boxes[t, 1] - d.boxes[t, 0]) + d.pads[t, 0] + d.pads[t, 1]
        loc = d.pos[rows].astype(np.int64)
        room = np.minimum(loc, span - 1 - loc).min(axis=1)
        fits = room > r + 1.0
        bad = np.flatnonzero(dens_b[rows[fits]] != dens_full[gi[fits]])
        assert bad.size == 0, f"subvolume {t}: {bad.size} densities differ"
        checked += int(fits.sum())
        print(f"[decompose] subvolume {t}: {rows.size} core, {int(fits.sum())} checked, "
              f"{int(np.count_nonzero(dens_b[rows[~fits]] != dens_full[gi[~fits]]))} of the "
              f"{int((~fits).sum())} near the edge differ", flush=True)
    assert checked > 0.9 * p.n


def _stitched(ctx, p, premerge, task_densities=False):
    import time

    import torch

    from paper_1001_3411_amd import HopParams
    from paper_1001_3411_amd.decompose import decompose
    d = decompose(p.pos, 8, seed=3, safety=1.5)
    sub = HopParams(periodic=False, padded_rules=True, mean_density=p.mean_density)
    box = HopParams(periodic=False, padded_rules=True, mean_density=p.mean_density)
    pos_b = torch.from_numpy(d.pos.view(np.int32)).cuda()
    pad_b = torch.from_numpy(d.padded).cuda()
    idx_b = torch.from_numpy(d.index).cuda()
    md = np.full(8, p.mean_density)
    for rep in range(2):   # the second pass is timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = ctx.run_batch(pos_b, d.offsets, sub, padded=pad_b, mean_density=md)
        out = ctx.stitch(d.offsets, idx_b, pad_b, b, p.n, box, premerge=premerge,
                         task_densities=task_densities)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    print(f"[stitch] premerge={premerge} task_densities={task_densities}: {p.n} particles, 8 subvolumes "
          f"({d.pos.shape[0]} rows with padding): {dt * 1e3:.1f} ms; {out['n_chains']} chains, "
          f"{out['n_groups']} groups, {ctx.stats()['premerged']} premerged pairs", flush=True)
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def test_stitched_chains_equal_whole_box(ctx, box2):
    """Decompose (s = 1.5), run the subvolumes in one batched call, then
    rebuild the chains through the padded particles they end on, give
    padded particles their owners' chains, build one boundary table from
    every subvolume's rows and merge (hop_stitch, no premerge): every output
    equals the oracle's whole-box run."""
    p, r = box2
    g = _stitched(ctx, p, premerge=False)
    for k in ("density", "hop", "root", "chain_of", "group", "g_count", "g_peak", "g_peak_dens"):
        assert np.array_equal(g[k], getattr(r, k)), k
    assert g["n_chains"] == r.n_chains and g["n_groups"] == r.n_groups


def test_stitched_with_premerge(ctx, box2):
    """The premerge joins proto-halos inside each subvolume before the
    chains are reconnected; a join the whole box would not make can only
    come from a padded particle's density, so the labels should barely
    change: the fraction of particles whose group changes is reported."""
    from paper_1001_3411_amd.report import group_change_fraction
    p, r = box2
    g = _stitched(ctx, p, premerge=True)
    for k in ("density", "hop", "root", "chain_of"):
        assert np.array_equal(g[k], getattr(r, k)), k
    chg = group_change_fraction(r.group, g["group"])
    print(f"[stitch] premerge group change fraction {chg:.3e} "
          f"({g['n_groups']} vs {r.n_groups} groups)", flush=True)
    assert chg < 1e-3


def test_stitched_with_task_densities(ctx, box2):
    """The paper's own form: padded particles keep the densities their
    subvolume gave them and local links are the subvolume's.  A padded
    particle whose list the padding cut short can then carry a wrong density
    into a local particle's link or a boundary; the chains are still rebuilt
    and merged, and the fractions of changed links and groups are reported."""
    from paper_1001_3411_amd.report import group_change_fraction
    p, r = box2
    g = _stitched(ctx, p, premerge=False, task_densities=True)
    assert np.array_equal(g["density"], r.density)
    link_chg = float(np.mean(g["hop"] != r.hop))
    chg = group_change_fraction(r.group, g["group"])
    print(f"[stitch] task densities: link change fraction {link_chg:.3e}, group change "
          f"fraction {chg:.3e} ({g['n_groups']} vs {r.n_groups} groups)", flush=True)
    assert link_chg < 1e-3 and chg < 1e-2
