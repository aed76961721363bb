"""GPU parity at the full workload sizes.

The 16.8M-particle Zel'dovich box is checked element by element against the
oracle.  The 134M-particle clustered box (the benchmark's workload) is
checked against the oracle's bounded-memory pipeline: densities, links,
roots, chains, groups and the group table element by element, the first 16
list columns exactly and every whole 64-column list by its fingerprint;
sampled lists are also checked against brute force over all 134M particles.
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from listhash import row_fnv1a

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1001_3411_amd import HopContext
    c = HopContext(0)
    yield c
    c.close()


def _params(p, **kw):
    from paper_1001_3411_amd import HopParams
    return HopParams(periodic=p.periodic, mean_density=p.mean_density, **kw)


@pytest.mark.timeout(900)
def test_zeldovich_16m_full_parity(ctx, orc):
    p = synth.config(3)
    print(f"[fullsize] {p.name} n={p.n}", flush=True)
    r = orc.run(p.pos, mean_density=p.mean_density)
    out = ctx.run(p.pos, _params(p))
    g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    del out
    assert r.n_groups > 100
    assert np.array_equal(g["nbr"], r.nbr), "nbr"
    assert np.array_equal(g["density"], r.density), "density"
    for k in ("hop", "root", "chain_of", "group", "g_count", "g_peak", "g_peak_dens"):
        assert np.array_equal(g[k], getattr(r, k)), k
    assert g["n_chains"] == r.n_chains and g["n_groups"] == r.n_groups


def _host_rows(nbr_d, k_keep, chunk=1 << 23):
    """First k_keep columns and fingerprints of all rows of a device list array,
    copied to the host in pieces."""
    n = nbr_d.shape[0]
    heads = np.empty((n, k_keep), np.int32)
    hashes = np.empty(n, np.uint64)

    def piece(a):
        b = min(a + chunk, n)
        rows = nbr_d[a:b].cpu().numpy()
        heads[a:b] = rows[:, :k_keep]
        hashes[a:b] = row_fnv1a(rows)

    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(piece, range(0, n, chunk)))
    return heads, hashes


@pytest.mark.timeout(1500)
def test_134m_full_oracle_parity(ctx, orc, capsys):
    import torch

    def say(msg):
        with capsys.disabled():
            print(f"[fullsize] {msg}", flush=True)

    t0 = time.time()
    p = synth.config(5)
    n = p.n
    prm = _params(p)
    say(f"{p.name} n={n} generated in {time.time() - t0:.0f}s")
    out = ctx.run(p.pos, prm)
    torch.cuda.synchronize()
    g = {k: out[k].cpu().numpy() for k in ("density", "hop", "root", "chain_of", "group",
                                           "g_count", "g_peak", "g_peak_dens")}
    g_nbr16, g_hash = _host_rows(out["nbr"], 16)
    nc, ng = out["n_chains"], out["n_groups"]

    # sampled lists by brute force over the whole box (independent of any tree)
    rng = np.random.default_rng(12345)
    q = np.unique(np.concatenate([rng.choice(n, 96, replace=False),
                                  np.argpartition(g["density"], n - 32)[-32:]])).astype(np.int64)
    ref_nbr, ref_d2 = orc.knn(p.pos, prm.n_dens, periodic=True, queries=q, method="brute")
    assert np.array_equal(out["nbr"][torch.from_numpy(q).cuda()].cpu().numpy(), ref_nbr)
    assert np.array_equal(g["density"][q], orc.density(ref_d2, p.mean_density))
    del out
    torch.cuda.empty_cache()
    say(f"GPU run, host copies and {q.size} brute-force rows done ({time.time() - t0:.0f}s)")

    L = orc.Lite(p.pos, mean_density=p.mean_density, k_keep=16)
    say(f"oracle tree built ({time.time() - t0:.0f}s)")
    step = 1 << 24
    for c0 in range(0, n, step):
        L.query(c0, min(c0 + step, n))
        say(f"oracle lists {min(c0 + step, n)}/{n} ({time.time() - t0:.0f}s)")
    hop, root, chain_of, group, gc, gp, gd, r_nc, r_ne, r_ng = L.finish()
    say(f"oracle stages done: {r_ng} groups, {r_nc} chains ({time.time() - t0:.0f}s)")

    assert np.array_equal(g["density"], L.density), "density"
    assert np.array_equal(g_nbr16, L.nbr), "first 16 list columns"
    bad = np.flatnonzero(g_hash != L.row_hash)
    assert bad.size == 0, f"{bad.size} lists differ, first at {bad[:5]}"
    for k, ref in (("hop", hop), ("root", root), ("chain_of", chain_of), ("group", group),
                   ("g_count", gc), ("g_peak", gp), ("g_peak_dens", gd)):
        assert np.array_equal(g[k], ref), k
    assert (nc, ng) == (r_nc, r_ng)
    assert ng > 1000
    say(f"parity ok: {ng} groups, {nc} chains ({time.time() - t0:.0f}s)")
