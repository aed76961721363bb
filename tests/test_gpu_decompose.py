"""The decomposition front end end to end: a periodic box cut into 8
load-balanced, directionally padded subvolumes and run through the batched
call must give every core particle whose whole-box neighbour sphere lies
inside its padded subvolume exactly the whole-box density (same neighbours
at the same exact distances, same global mean density, same operation
sequence).  Particles nearer the padded box's edge than their 64th
neighbour are only counted: how many there are is what the safety factor
s of Eq. (1) controls.
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


def test_padded_subvolumes_reproduce_box_densities(ctx):
    from paper_1001_3411_amd import HopParams
    from paper_1001_3411_amd.decompose import decompose
    G = 1 << 21
    p = synth.config(2)
    full = HopParams(mean_density=p.mean_density)
    dens_full, nbr_full = ctx.density(p.pos, full)
    dens_full = dens_full.cpu().numpy()
    far = nbr_full[:, -1].cpu().numpy()
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
