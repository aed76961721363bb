"""Subhalos on the GPU (hop_subhalos) against the oracle's subhalo function:
structure numbers at every level, and the table (members, peak, peak
density, parent), element by element.
"""
import numpy as np
import pytest

import synth
from test_gpu_parity import _params

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


def _check(ctx, orc, p, levels, alpha, ids=None, label=""):
    import torch
    r = orc.run(p.pos, mean_density=p.mean_density, ids=ids)
    ref = orc.subhalos(r.nbr, r.density, r.chain_of, r.n_chains, levels, n_merge=4, alpha=alpha,
                       ids=ids)
    dev = "cuda:0"
    g = ctx.subhalos(torch.from_numpy(r.nbr).to(dev), torch.from_numpy(r.density).to(dev),
                     torch.from_numpy(r.chain_of).to(dev), r.n_chains, levels, _params(p),
                     alpha=alpha, ids=ids)
    print(f"[subhalos] {label}: {r.n_chains} chains, {ref.n_sym} symmetric boundaries, "
          f"structures per level {np.diff(ref.t_off).tolist()}", flush=True)
    assert g["t_off"] == ref.t_off.tolist(), label
    assert np.array_equal(g["sub"].cpu().numpy(), ref.sub), label
    assert np.array_equal(g["count"].cpu().numpy(), ref.count), label
    assert np.array_equal(g["peak"].cpu().numpy(), ref.peak), label
    assert np.array_equal(g["peak_dens"].cpu().numpy(), ref.peak_dens), label
    assert np.array_equal(g["parent"].cpu().numpy(), ref.parent), label
    assert ctx.stats()["premerged"] == ref.n_sym
    return ref


def test_config1_levels(ctx, orc):
    ref = _check(ctx, orc, synth.config(1), [200.0, 400.0, 800.0, 1600.0, 3200.0], 1.0,
                 label="config1")
    assert ref.t_off[1] > 5


def test_config1_all_structures_and_ties_by_id(ctx, orc):
    p = synth.config(1)
    ids = np.random.default_rng(4).permutation(p.n).astype(np.int64) * 2 + 9
    _check(ctx, orc, p, [80.0, 250.0], 0.0, ids=ids, label="config1-ids")


def test_config2_levels(ctx, orc):
    _check(ctx, orc, synth.config(2), [240.0, 1000.0, 5000.0], 2.0, label="config2")
