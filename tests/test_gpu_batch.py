"""The batched path: many independent subvolumes in one call.

Every subvolume's result must equal the oracle run on that subvolume alone
(non-periodic frame, padded rules, its own mean density), element by
element, whatever launch settings are used.
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


def concat(subs):
    pos = np.ascontiguousarray(np.concatenate([p.pos for p in subs]))
    padded = np.ascontiguousarray(np.concatenate([p.padded for p in subs]))
    off = np.concatenate([[0], np.cumsum([p.n for p in subs])]).astype(np.int64)
    md = [p.mean_density for p in subs]
    return pos, padded, off, md


def run_batch(ctx, subs, **kw):
    from paper_1001_3411_amd import HopParams
    pos, padded, off, md = concat(subs)
    prm = HopParams(periodic=False, padded_rules=True, **kw)
    out = ctx.run_batch(pos, off, prm, padded=padded, mean_density=md)
    host = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    return host


def check_against_oracle(orc, subs, g, label):
    off = g["offsets"]
    for s, p in enumerate(subs):
        r = orc.run(p.pos, periodic=False, mean_density=p.mean_density, padded=p.padded,
                    padded_rules=True)
        a, b = off[s], off[s + 1]
        what = f"{label} subvolume {s} (n={p.n})"
        assert np.array_equal(g["nbr"][a:b], r.nbr), what + ": nbr"
        assert np.array_equal(g["density"][a:b], r.density), what + ": density"
        for k in ("hop", "root", "chain_of", "group"):
            assert np.array_equal(g[k][a:b], getattr(r, k)), f"{what}: {k}"
        assert g["n_chains"][s] == r.n_chains, what + ": n_chains"
        assert g["n_groups"][s] == r.n_groups, what + ": n_groups"
        ga, gb = g["group_off"][s], g["group_off"][s + 1]
        assert np.array_equal(g["g_count"][ga:gb], r.g_count), what + ": g_count"
        assert np.array_equal(g["g_peak"][ga:gb], r.g_peak), what + ": g_peak"
        assert np.array_equal(g["g_peak_dens"][ga:gb], r.g_peak_dens), what + ": g_peak_dens"


def small_batch():
    # uneven sizes, ragged against the 64-particle buckets, down to n = n_dens
    subs = synth.subvolume_batch(n_sub=6, seed=4100, scale=0.05)
    subs += [synth.padded_subvolume(n, 4200 + n) for n in (64, 100, 1000, 4097)]
    return subs


def test_batch_matches_oracle_per_subvolume(ctx, orc):
    subs = small_batch()
    print(f"[batch] sizes {[p.n for p in subs]}", flush=True)
    g = run_batch(ctx, subs)
    assert sum(g["n_groups"]) > 0
    check_against_oracle(orc, subs, g, "small")


def test_batch_independent_of_launch_settings(ctx):
    subs = small_batch()
    ref = run_batch(ctx, subs)
    for t in (dict(front_cap=4), dict(xcd_queues=0, largest_first=0),
              dict(persistent_waves=37, front_cap=256)):
        ctx.set_tuning(**t)
        try:
            g = run_batch(ctx, subs)
        finally:
            ctx.set_tuning(front_cap=1024, persistent_waves=0, xcd_queues=1, largest_first=1)
        for k in ("nbr", "density", "hop", "root", "chain_of", "group", "g_count", "g_peak"):
            assert np.array_equal(g[k], ref[k]), f"{t}: {k}"


def test_batch_single_subvolume_equals_plain_call(ctx):
    from paper_1001_3411_amd import HopParams
    p = synth.padded_subvolume(30000, 4300)
    g = run_batch(ctx, [p])
    prm = HopParams(periodic=False, padded_rules=True, mean_density=p.mean_density)
    q = ctx.run(p.pos, prm, padded=p.padded)
    for k in ("nbr", "density", "hop", "root", "chain_of", "group"):
        assert np.array_equal(g[k], q[k].cpu().numpy()), k


@pytest.mark.slow
def test_batch_64_subvolumes_full(ctx, orc):
    subs = synth.config(4)
    print(f"[batch] 64 subvolumes, {sum(p.n for p in subs)} particles", flush=True)
    g = run_batch(ctx, subs)
    check_against_oracle(orc, subs, g, "config4")


def test_batch_many_small_subvolumes_every_setting_matches_oracle(ctx, orc):
    """Regression for wrong lists seen once in the persistent kernel: many
    small subvolumes make each wave run buckets of different subvolumes one
    after another (state left from the previous bucket would show), under
    launch settings that change which wave runs which bucket.  Every setting
    is checked against the oracle, subvolume by subvolume."""
    subs = [synth.padded_subvolume(n, 4400 + i)
            for i, n in enumerate((13233, 64, 65, 127, 700, 2049, 5000, 9001, 13233, 301))]
    settings = (dict(), dict(persistent_waves=8), dict(persistent_waves=37, front_cap=4),
                dict(persistent_waves=1024, xcd_queues=0), dict(largest_first=0, front_cap=64),
                dict(persistent_waves=64, xcd_queues=0, largest_first=0))
    for t in settings:
        ctx.set_tuning(**t)
        try:
            g = run_batch(ctx, subs)
        finally:
            ctx.set_tuning(front_cap=1024, persistent_waves=0, xcd_queues=1, largest_first=1)
        check_against_oracle(orc, subs, g, f"setting {t}")
