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
