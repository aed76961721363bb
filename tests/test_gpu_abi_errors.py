"""Argument validation and the error paths of the C ABI (include/hop.h):
each bad input returns its documented code, and the capacity paths either
recover (the boundary table regrows) or report HOP_ERR_CAPACITY.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from test_gpu_parity import _params, assert_parity, gpu_run

pytestmark = pytest.mark.gpu

ARG, RANGE, CAPACITY = -1, -2, -4


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1001_3411_amd import HopContext
    c = HopContext(0)
    yield c
    c.close()


def _density_rc(ctx, pos, prm):
    """Raw return code of hop_density (no exception)."""
    import torch
    from paper_1001_3411_amd import _ptr
    pos_d = torch.from_numpy(pos.view(np.int32)).cuda()
    n = pos.shape[0]
    dens = torch.empty(n, dtype=torch.float64, device="cuda")
    nbr = torch.empty((n, max(prm.k_store, 1)), dtype=torch.int32, device="cuda")
    cp = prm.c()
    rc = ctx.lib.hop_density(ctx.h, n, _ptr(pos_d), None, C.byref(cp), _ptr(dens), _ptr(nbr),
                             ctx._stream(None))
    torch.cuda.synchronize()
    return rc, ctx.lib.hop_last_error(ctx.h).decode()


BAD_PARAMS = [
    dict(n_dens=129, k_store=64),                    # above the compile-time maximum
    dict(n_dens=1, n_hop=1, n_merge=1, k_store=1),   # n_dens < 2
    dict(n_merge=0),                                 # n_merge < 1
    dict(n_merge=17),                                # n_merge > n_hop
    dict(n_hop=65),                                  # n_hop > k_store
    dict(k_store=80),                                # k_store > n_dens
    dict(delta_outer=float("nan")),
    dict(delta_saddle=float("inf")),
    dict(delta_peak=-1.0),
    dict(mean_density=float("nan")),
    dict(mean_density=-2.0),
    dict(grid_bits=0),
    dict(grid_bits=22),
]


@pytest.mark.parametrize("kw", BAD_PARAMS, ids=[str(k) for k in BAD_PARAMS])
def test_bad_parameters_are_rejected(ctx, kw):
    from paper_1001_3411_amd import HopParams
    p = synth.uniform_box(500, 1)
    rc, msg = _density_rc(ctx, p.pos, HopParams(**kw))
    assert rc == ARG, (kw, rc, msg)
    assert msg


def test_fewer_particles_than_ndens(ctx):
    from paper_1001_3411_amd import HopParams
    p = synth.uniform_box(63, 2)
    rc, msg = _density_rc(ctx, p.pos, HopParams())
    assert rc == ARG and "n_dens" in msg
    # exactly n_dens particles is allowed
    q = synth.uniform_box(64, 2)
    assert _density_rc(ctx, q.pos, HopParams(mean_density=q.mean_density))[0] == 0


def test_unknown_flag_is_rejected(ctx):
    from paper_1001_3411_amd import HopParams
    p = synth.uniform_box(500, 3)
    prm = HopParams()
    cp = prm.c()
    cp.flags |= 0x100
    import torch
    from paper_1001_3411_amd import _ptr
    pos_d = torch.from_numpy(p.pos.view(np.int32)).cuda()
    dens = torch.empty(p.n, dtype=torch.float64, device="cuda")
    rc = ctx.lib.hop_density(ctx.h, p.n, _ptr(pos_d), None, C.byref(cp), _ptr(dens), None,
                             ctx._stream(None))
    assert rc == ARG


def test_one_slot_boundary_table_regrows_to_oracle_parity(ctx, orc):
    # a one-slot initial table overflows at the first chain pair; it must be
    # doubled and rebuilt until every pair fits, with unchanged results
    p = synth.config(1)
    r = orc.run(p.pos, mean_density=p.mean_density)
    ctx.set_tuning(hash_slots=1)
    try:
        g = gpu_run(ctx, p, _params(p))
    finally:
        ctx.set_tuning(hash_slots=0)
    assert_parity(g, r, "config1-hash1")


def test_links_that_close_a_cycle_are_reported(ctx):
    import torch
    from paper_1001_3411_amd import HopError, HopParams
    n = 200
    hop = torch.arange(n, dtype=torch.int32, device="cuda")
    hop[10], hop[11] = 11, 10  # a two-cycle
    dens = torch.full((n,), 100.0, dtype=torch.float64, device="cuda")
    with pytest.raises(HopError) as e:
        ctx.groups(hop, dens, HopParams())
    assert e.value.code == ARG and "self-linked" in str(e.value)
    # the context stays usable
    hop[10], hop[11] = 10, 11
    root, chain_of, nc = ctx.groups(hop, dens, HopParams())
    assert nc == n


def test_link_outside_range_is_reported(ctx):
    import torch
    from paper_1001_3411_amd import HopError, HopParams
    n = 100
    hop = torch.arange(n, dtype=torch.int32, device="cuda")
    hop[3] = n + 7
    dens = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(HopError) as e:
        ctx.groups(hop, dens, HopParams())
    assert e.value.code == RANGE


def test_halo_stats_rejects_a_peak_outside_range(ctx):
    import torch
    from paper_1001_3411_amd import HopError
    p = synth.config(1)
    out = ctx.run(p.pos, _params(p))
    table = out["table"].clone()
    assert table.shape[0] > 1
    table[1, 1] = p.n + 5  # peak index of group 1 (the low word)
    with pytest.raises(HopError) as e:
        ctx.halo_stats(p.pos, out["group"], table, _params(p))
    assert e.value.code == RANGE
    # the intact table still works on the same context
    st = ctx.halo_stats(p.pos, out["group"], out["table"], _params(p))
    assert torch.isfinite(st["rmax"]).all()


def test_packed_key_width_error(ctx):
    # n > 2^22 leaves 64 - 23 = 41 bits for d^2 in the packed (d^2, tie) key;
    # one particle 1.8e6 grid units (min image) from all the others needs
    # more, which is reported as HOP_ERR_CAPACITY instead of a wrong list
    from paper_1001_3411_amd import HopError, HopParams
    rng = np.random.default_rng(9)
    n = (1 << 22) + 1
    pos = np.empty((n, 3), np.uint32)
    pos[:-1] = rng.integers(0, 1 << 14, size=(n - 1, 3), dtype=np.uint32)
    pos[-1] = 1 << 20
    print(f"[abi] key width case n={n}", flush=True)
    with pytest.raises(HopError) as e:
        ctx.run(pos, HopParams())
    assert e.value.code == CAPACITY and "key" in str(e.value)
