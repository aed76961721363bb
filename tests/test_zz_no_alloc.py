"""hop_halo_stats_noalloc: the statistics of hop_halo_stats from a static
device scratch array, no allocation.  Called through the C ABI twice in a
row (the second time on a smaller input, so stale contents of the shared
array would show) and compared with hop_halo_stats on the same inputs:
centres and radii bit for bit, bulk velocities within the FP64 summation
bound of the two orders.  Sizes beyond the array are rejected.
"""
import ctypes as C

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


def _noalloc(ctx, pos_d, vel_d, group, table, params):
    import torch
    from paper_1001_3411_amd import _ptr
    n, ng = pos_d.shape[0], table.shape[0]
    dev = pos_d.device
    com = torch.full((ng, 3), float("nan"), dtype=torch.float64, device=dev)
    rmax = torch.full((ng,), float("nan"), dtype=torch.float64, device=dev)
    vbulk = torch.full((ng, 3), float("nan"), dtype=torch.float64, device=dev)
    cp = params.c()
    rc = ctx.lib.hop_halo_stats_noalloc(ctx.h, n, _ptr(pos_d), _ptr(vel_d), _ptr(group), ng,
                                        _ptr(table), C.byref(cp), _ptr(com), _ptr(rmax),
                                        _ptr(vbulk), ctx._stream(None))
    assert rc == 0, ctx.lib.hop_last_error(ctx.h)
    ctx.sync()
    return com.cpu().numpy(), rmax.cpu().numpy(), vbulk.cpu().numpy()


def _case(ctx, p, params, seed):
    import torch
    out = ctx.run(p.pos, params, padded=p.padded)
    pos_d = torch.from_numpy(p.pos.view(np.int32)).cuda()
    rng = np.random.default_rng(seed)
    vel = (rng.standard_normal((p.n, 3)) * 300.0).astype(np.float32)
    vel_d = torch.from_numpy(vel).cuda()
    ref = ctx.halo_stats(p.pos, out["group"], out["table"], params, vel=vel)
    ctx.sync()
    got = _noalloc(ctx, pos_d, vel_d, out["group"], out["table"], params)
    print(f"[noalloc] n={p.n}: {out['n_groups']} halos", flush=True)
    assert out["n_groups"] > 0
    assert np.array_equal(got[0], ref["com"].cpu().numpy()), "com"
    assert np.array_equal(got[1], ref["rmax"].cpu().numpy()), "rmax"
    b = ref["vbulk"].cpu().numpy()
    grp = out["group"].cpu().numpy()
    cnt = np.bincount(grp[grp >= 0], minlength=out["n_groups"]).astype(np.float64)[:, None]
    vabs = np.zeros((out["n_groups"], 3))
    np.add.at(vabs, grp[grp >= 0], np.abs(vel[grp >= 0].astype(np.float64)))
    bound = 2 * (cnt - 1) * U * vabs / cnt + 2 * U * np.abs(b)
    assert np.all(np.abs(got[2] - b) <= bound), "vbulk"


def test_two_calls_second_smaller(ctx):
    from paper_1001_3411_amd import HopParams
    p1 = synth.config(1)
    _case(ctx, p1, HopParams(mean_density=p1.mean_density), 1)
    p2 = synth.padded_subvolume(9000, 61)
    _case(ctx, p2, HopParams(periodic=False, padded_rules=True, mean_density=p2.mean_density), 2)


def test_too_many_groups_is_rejected(ctx):
    import torch
    from paper_1001_3411_amd import HopParams, _ptr
    n = 100
    pos = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
    group = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    cp = HopParams().c()
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = ctx.lib.hop_halo_stats_noalloc(ctx.h, n, _ptr(pos), None, _ptr(group), (1 << 18) + 1,
                                        _ptr(dummy), C.byref(cp), _ptr(dummy), _ptr(dummy), None,
                                        ctx._stream(None))
    assert rc == -1 and "HOP_NOALLOC_MAX_GROUPS" in ctx.lib.hop_last_error(ctx.h).decode()
