"""The learned search radius on the GPU.

* features and targets against the FP64 reference;
* the FP32 gradient of the network against the FP64 reference (stated
  tolerance: max |g32 - g64| <= 1e-4 * max |g64|), the loss, and one Adam
  step;
* the bounded search: with any radius model (trained, analytic, or one far
  too small so that every particle falls back) the neighbour lists and
  densities equal the oracle's bit for bit, and misses are counted.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1001_3411_amd import HopContext
    c = HopContext(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def box1(ctx):
    """config-1 box with its plain neighbour lists, features and targets"""
    from paper_1001_3411_amd import HopParams
    from paper_1001_3411_amd.radius import cell_bits_for
    p = synth.config(1)
    prm = HopParams(mean_density=p.mean_density)
    dens, nbr = ctx.density(p.pos, prm)
    cb = cell_bits_for(p.n)
    feats, target = ctx.radius_dataset(p.pos, prm, cb, nbr=nbr)
    return p, prm, cb, nbr, feats, target


def test_features_and_targets_match_reference(box1, orc):
    from oracle import mlp
    p, prm, cb, nbr, feats, target = box1
    f64 = mlp.features(p.pos, cb, periodic=True)
    f32 = feats.cpu().numpy()
    assert np.max(np.abs(f32 - f64)) <= 1e-6 * np.max(np.abs(f64))
    _, d2 = orc.knn(p.pos, 64, periodic=True)
    y64 = mlp.targets(d2[:, -1], cb)
    assert np.max(np.abs(target.cpu().numpy() - y64)) <= 1e-6


def test_gradient_matches_fp64_reference(ctx, box1):
    import torch
    from oracle import mlp
    from paper_1001_3411_amd.radius import init_weights
    p, prm, cb, nbr, feats, target = box1
    w = init_weights(7)
    wd = torch.from_numpy(w).to(feats.device)
    for batch, idx in ((1000, None),
                       (777, torch.from_numpy(np.random.default_rng(3).integers(0, p.n, 777)))):
        grad, loss = ctx.mlp_grad(feats, target, wd, batch=batch, idx=idx)
        rows = np.arange(batch) if idx is None else idx.numpy()
        X = feats.cpu().numpy()[rows].astype(np.float64)
        t = target.cpu().numpy()[rows].astype(np.float64)
        l64, g64 = mlp.loss_and_grad(w.astype(np.float64), X, t)
        g32 = grad.cpu().numpy()
        err = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
        print(f"[radius] batch {batch}: grad max err / max |g| = {err:.2e}, "
              f"loss {loss:.6f} vs {l64:.6f}", flush=True)
        assert err <= GRAD_TOL
        assert abs(loss - l64) <= 1e-5 * l64


def test_adam_step_matches_fp64_reference(ctx, box1):
    import torch
    from oracle import mlp
    from paper_1001_3411_amd.radius import init_weights
    p, prm, cb, nbr, feats, target = box1
    rng = np.random.default_rng(11)
    w = init_weights(5)
    m = rng.normal(0, 1e-3, w.size).astype(np.float32)
    v = rng.uniform(1e-7, 1e-5, w.size).astype(np.float32)
    dev = feats.device
    wd, md, vd = (torch.from_numpy(a.copy()).to(dev) for a in (w, m, v))
    ctx.mlp_train(feats, target, wd, md, vd, None, 1, 512, first_step=3, lr=1e-3)
    X = feats.cpu().numpy()[:512].astype(np.float64)
    t = target.cpu().numpy()[:512].astype(np.float64)
    _, g64 = mlp.loss_and_grad(w.astype(np.float64), X, t)
    w64, m64, v64 = mlp.adam_step(w, m, v, g64, 3, lr=1e-3)
    assert np.max(np.abs(wd.cpu().numpy() - w64)) <= 1e-6
    assert np.max(np.abs(md.cpu().numpy() - m64)) <= 1e-4 * np.max(np.abs(m64))
    assert np.max(np.abs(vd.cpu().numpy() - v64)) <= 1e-4 * np.max(np.abs(v64))


def test_training_lowers_the_loss(ctx, box1):
    from paper_1001_3411_amd.radius import train
    p, prm, cb, nbr, feats, target = box1
    w, losses = train(ctx, feats, target, steps=400, batch=1024, seed=2)
    print(f"[radius] loss {losses[:20].mean():.4f} -> {losses[-20:].mean():.4f}", flush=True)
    assert losses[-20:].mean() < 0.5 * losses[:20].mean()


def _exact_with(ctx, orc, p, prm, label):
    from dataclasses import replace
    r = orc.run(p.pos, periodic=p.periodic, mean_density=p.mean_density, padded=p.padded,
                padded_rules=p.padded is not None)
    dens, nbr = ctx.density(p.pos, replace(prm, learned_radius=True))
    st = ctx.stats()
    assert np.array_equal(nbr.cpu().numpy(), r.nbr), label
    assert np.array_equal(dens.cpu().numpy(), r.density), label
    return st


def test_bounded_search_is_exact(ctx, orc, box1):
    from paper_1001_3411_amd import HOP_RADIUS_ANALYTIC, HOP_RADIUS_MLP, HopParams
    from paper_1001_3411_amd.radius import calibrate, train
    p, prm, cb, nbr, feats, target = box1
    w, _ = train(ctx, feats, target, steps=300, batch=1024, seed=4)
    cases = [p, synth.tiny_case("uniform", 4097, 8), synth.padded_subvolume(9000, 41)]
    for kind in (HOP_RADIUS_MLP, HOP_RADIUS_ANALYTIC):
        margin = calibrate(ctx, w, feats, target, miss_rate=0.02, kind=kind)
        for q in cases:
            qp = HopParams(mean_density=q.mean_density, periodic=q.periodic)
            st = _exact_with(ctx, orc, q, qp, f"kind {kind} {q.name}")
            print(f"[radius] kind {kind} margin {margin:.3f} {q.name}: misses {st['misses']} "
                  f"of {q.n}, redo buckets {st['redo_buckets']}", flush=True)
    # far too small a radius: every particle misses and is searched again
    ctx.radius_load(HOP_RADIUS_MLP, w, -8.0)
    st = _exact_with(ctx, orc, p, prm, "all-miss")
    assert st["misses"] == p.n
    ctx.radius_load(0)


@pytest.mark.parametrize("waves", [8, 37])
def test_bounded_search_with_few_persistent_waves(ctx, orc, box1, waves):
    """The one-box kNN launch is persistent: each wave takes many buckets in
    turn.  The bounded search records its misses per bucket and the fallback
    pass searches those lanes again; with few waves the results are still
    the oracle's."""
    from paper_1001_3411_amd import HOP_RADIUS_ANALYTIC
    from paper_1001_3411_amd.radius import calibrate
    p, prm, cb, nbr, feats, target = box1
    calibrate(ctx, None, feats, target, miss_rate=0.05, kind=HOP_RADIUS_ANALYTIC)
    ctx.set_tuning(persistent_waves=waves)
    try:
        st = _exact_with(ctx, orc, p, prm, f"analytic, {waves} waves")
        assert st["misses"] > 0 and st["redo_buckets"] > 0
    finally:
        ctx.set_tuning(persistent_waves=0)
        ctx.radius_load(0)


def test_search_modes_on_the_clustered_box(ctx):
    """The 16.8M-particle Zel'dovich box under the plain search, the analytic
    radius and the trained network (each calibrated for a 1% miss rate):
    neighbour lists, densities, links and groups are the same in all three,
    and the work each does (tree nodes tested, leaf batches streamed,
    misses searched again, kNN time) is recorded."""
    import time
    from dataclasses import replace

    import torch
    from paper_1001_3411_amd import HOP_RADIUS_ANALYTIC, HOP_RADIUS_MLP, HopParams
    from paper_1001_3411_amd.radius import calibrate, cell_bits_for, train
    p = synth.config(3)
    prm = HopParams(mean_density=p.mean_density)
    pos = torch.from_numpy(p.pos.view(np.int32)).cuda()
    _, nbr = ctx.density(pos, prm)
    feats, target = ctx.radius_dataset(pos, prm, cell_bits_for(p.n), nbr=nbr)
    del nbr
    w, losses = train(ctx, feats, target, steps=1500, batch=4096, seed=0)
    models = {"analytic": (HOP_RADIUS_ANALYTIC, None), "mlp": (HOP_RADIUS_MLP, w)}
    margins = {k: calibrate(ctx, m[1], feats, target, miss_rate=0.01, kind=m[0])
               for k, m in models.items()}
    del feats, target
    ref, rows = None, {}
    for name in ("plain", "analytic", "mlp"):
        q = prm
        if name != "plain":
            ctx.radius_load(models[name][0], models[name][1], margins[name])
            q = replace(prm, learned_radius=True)
        ctx.set_profiling(3)
        out = ctx.run(pos, q)
        st = ctx.stats()
        ctx.set_profiling(1)
        ms = []
        for _ in range(3):
            ctx.run(pos, q)
            ms.append(ctx.stats()["ms_knn"])
        ctx.set_profiling(0)
        got = {k: out[k] for k in ("nbr", "density", "hop", "group")}
        if ref is None:
            ref = got
        else:
            for k in ref:
                assert torch.equal(got[k], ref[k]), (name, k)
        rows[name] = (st["nodes_visited"] / p.n, st["leaves_scanned"] / p.n / 4,
                      st["misses"] / p.n, float(np.median(ms)))
        print(f"[radius] {p.name} {name}: nodes/particle {rows[name][0]:.2f}, leaf batches/"
              f"particle {rows[name][1]:.3f}, miss fraction {rows[name][2]:.4f}, "
              f"kNN {rows[name][3]:.1f} ms", flush=True)
        del out, got
    ctx.radius_load(0)
    assert rows["plain"][2] == 0.0
    assert 0.0 < rows["mlp"][2] < 0.05 and 0.0 < rows["analytic"][2] < 0.05
