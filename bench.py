"""Benchmark of the whole HOP hot path on one MI355X.

One step = hop_density_link (Morton sort, tree, kNN + FP64 density, links
formed in Morton order) + hop_groups + hop_merge over the 134,217,728-particle clustered box (40,000
NFW clumps, 30% uniform background), inputs resident in HBM.  Prints one
JSON line with the roofline of the kNN kernel and the CPU oracle's rate.

    python bench.py [--steps K] [--warmup W] [--config 5] [--no-cpu] [--search S]
    python bench.py --workload batch64 [--tune-cache PATH]

--search compare (the default) also runs the same steps with the search
radius predicted per cell -- by the network trained on the Zel'dovich box's
own kNN radii, and by the analytic uniform-density estimate -- checks that
every output is identical to the plain run's, and reports both beside the
plain line; --search plain skips that.

The batch64 workload runs the 64 padded subvolumes (about 18M particles,
lognormal sizes) through one hop_run_batch call per step, after the
autotuner has picked its launch settings, and times 64 sequential
single-subvolume runs of the same data beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per particle of the kNN + density kernel (what the
# method must move): read the sorted position (12) and its tie key (4);
# write 64 neighbour indices (256) and the density (8)
KNN_BYTES_PER_PARTICLE = 12 + 4 + 4 * 64 + 8
# written besides by this library's fused density + link call (its own
# layout, not the method's work): the Morton-order copy of the first 16
# indices and the density (72) that the link kernel reads
KNN_COPY_BYTES_PER_PARTICLE = 4 * 16 + 8
# whole path (all stages), bytes per particle, same accounting
PATH_BYTES_PER_PARTICLE = 438
# VALU peak: 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz, one lane
# operation per lane and cycle (a wave64 VALU instruction occupies a SIMD
# for 4 cycles)
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# HBM traffic of the kNN kernel from hardware counters (FETCH_SIZE and
# WRITE_SIZE, each scaled by what the counter reads for a device copy of
# known size), kept with a hash of the kernel's sources: the figure is
# reported only while the sources are the ones it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "knn_traffic_nfw134m.txt")
KNN_SOURCES = [os.path.join(ROOT, "paper_1001_3411_amd", "csrc", f)
               for f in ("hop_knn.hip", "hop_internal.h")]


VALU_FILE = os.path.join(ROOT, "profiles", "knn_valu_nfw134m.txt")


def knn_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KNN_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _summary(path):
    """key: value lines of a counter summary, or None when the kernel sources
    no longer hash to the ones it was measured on."""
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        return kv if kv.get("source_hash") == knn_source_hash() else None
    except OSError:
        return None


def measured_traffic():
    """Bytes per kNN launch from the counter summary, or None."""
    kv = _summary(TRAFFIC_FILE)
    try:
        return None if kv is None else float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_valu(n, knn_ms):
    """VALU use of the kNN kernel from the counter summary, or None."""
    kv = _summary(VALU_FILE)
    if kv is None:
        return None
    try:
        insts = float(kv["SQ_INSTS_VALU_per_launch"])
        busy = float(kv["valu_busy"])
    except (KeyError, ValueError):
        return None
    buckets = (n + 63) // 64
    achieved = insts * 64 / (knn_ms / 1e3)
    return {"insts_per_bucket": round(insts / buckets, 1),
            "achieved_lane_ops": achieved, "peak_lane_ops": VALU_PEAK_LANE_OPS,
            "frac": round(achieved / VALU_PEAK_LANE_OPS, 4), "valu_busy": busy,
            "source": os.path.relpath(VALU_FILE, ROOT)}


def copy_probe():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB), twice: the
    reference the traffic counters are scaled by."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: 2 x 1 GiB device copies")
    del src, dst


def _oracle_rate(pos, mean_density, periodic, threads=None):
    import oracle
    before = oracle.num_threads()
    if threads is not None:
        oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        r = oracle.run(pos, periodic=periodic, mean_density=mean_density)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_threads(before)
    return pos.shape[0] / dt, dt, r.n_groups


def cpu_baseline(p, budget_frac=4):
    """The CPU oracle on a bounded sample of the same workload: the particles
    of one sub-cube of side 1/budget_frac of the box, as a non-periodic
    subvolume, normalised by the whole box's mean density; then one thread
    on the 32,768-particle box and on a smaller sub-cube (the per-core rate
    to set beside the paper's)."""
    import numpy as np
    import oracle
    import synth
    threads = oracle.num_threads()
    side = (1 << 21) // budget_frac
    sub = np.ascontiguousarray(p.pos[np.all(p.pos < side, axis=1)])
    rate, dt, ng = _oracle_rate(sub, p.mean_density, False)
    out = {"value": rate, "unit": "particles/s", "cores": threads, "kind": "oracle",
           "sample": f"{sub.shape[0]} particles in the [0, 1/{budget_frac})^3 sub-cube of the "
                     f"same box, whole pipeline (kd-tree kNN, density, links, chains, "
                     f"boundaries, merge, labels), {dt:.1f} s, {ng} groups"}
    one = []
    p1 = synth.config(1)
    r1, d1, _ = _oracle_rate(p1.pos, p1.mean_density, True, threads=1)
    one.append({"value": r1, "sample": f"{p1.name} whole box, {d1:.1f} s"})
    side8 = (1 << 21) // 8
    sub8 = np.ascontiguousarray(p.pos[np.all(p.pos < side8, axis=1)])
    r8, d8, _ = _oracle_rate(sub8, p.mean_density, False, threads=1)
    one.append({"value": r8, "sample": f"{sub8.shape[0]} particles in the [0, 1/8)^3 sub-cube "
                                       f"of the same box, {d8:.1f} s"})
    out["one_thread"] = one
    return out


def knn_roofline(n, knn_ms, kernel, value, fused=False):
    """HBM roofline of the kNN kernel on the method's bytes (280 per
    particle); the fused call's Morton-order copy is reported apart as
    overhead.  The kernel is bound by its VALU work, reported in "valu"."""
    knn_s = knn_ms / 1e3
    per = KNN_BYTES_PER_PARTICLE
    over = KNN_COPY_BYTES_PER_PARTICLE if fused else 0
    achieved = per * n / knn_s / 1e9
    # counter-measured figures hold for the 134M box's kernel only
    box = kernel == "k_knn_density" and n == 134217728
    traffic = measured_traffic() if box else None
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": traffic, "traffic_gbs": None if traffic is None else round(traffic / knn_s / 1e9, 2),
            "kernel_ms": round(knn_ms, 3),
            "bytes_per_particle": per,
            "overhead_bytes_per_particle": over,
            "frac_with_overhead": round((per + over) * n / knn_s / 1e9 / HBM_PEAK_GBS, 5),
            "path_frac": round(PATH_BYTES_PER_PARTICLE * value / 1e9 / HBM_PEAK_GBS, 5),
            "valu": measured_valu(n, knn_ms) if box else None}


def radius_models(ctx, log_fn):
    """Train the radius network on the 16.8M-particle Zel'dovich box's own
    kNN radii; calibrate it and the analytic estimate for a 1% miss rate."""
    import numpy as np
    import torch

    import synth
    from paper_1001_3411_amd import HOP_RADIUS_ANALYTIC, HOP_RADIUS_MLP, HopParams
    from paper_1001_3411_amd.radius import calibrate, cell_bits_for, train

    t0 = time.perf_counter()
    p3 = synth.config(3)
    prm3 = HopParams(mean_density=p3.mean_density)
    pos3 = torch.from_numpy(p3.pos.view(np.int32)).cuda()
    _, nbr = ctx.density(pos3, prm3)
    feats, target = ctx.radius_dataset(pos3, prm3, cell_bits_for(p3.n), nbr=nbr)
    del nbr, pos3
    w, losses = train(ctx, feats, target, steps=3000, batch=4096, seed=0)
    m_mlp = calibrate(ctx, w, feats, target, miss_rate=0.01, kind=HOP_RADIUS_MLP)
    m_an = calibrate(ctx, None, feats, target, miss_rate=0.01, kind=HOP_RADIUS_ANALYTIC)
    del feats, target
    torch.cuda.empty_cache()
    log_fn(f"radius models from {p3.name} in {time.perf_counter() - t0:.1f}s: "
           f"loss {losses[:50].mean():.3f} -> {losses[-50:].mean():.3f}, margins mlp {m_mlp:.3f} "
           f"analytic {m_an:.3f}")
    return {"mlp": (HOP_RADIUS_MLP, w, m_mlp), "analytic": (HOP_RADIUS_ANALYTIC, None, m_an),
            "train": {"dataset": p3.name, "samples": p3.n, "steps": 3000, "batch": 4096,
                      "loss_first": float(losses[:50].mean()),
                      "loss_last": float(losses[-50:].mean())}}


def bench_box(args):
    import numpy as np
    import torch

    import synth
    from paper_1001_3411_amd import HopContext, HopParams

    t0 = time.perf_counter()
    p = synth.config(args.config)
    log(f"generated {p.name}: n={p.n} in {time.perf_counter() - t0:.1f}s")
    n = p.n
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(p.pos.view(np.int32)).to(dev)
    prm = HopParams(mean_density=p.mean_density, periodic=p.periodic)
    ctx = HopContext(0)
    stream = torch.cuda.current_stream(dev)

    def step():
        return ctx.run(pos, prm, stream=stream)

    for w in range(args.warmup):
        out = step()
        torch.cuda.synchronize()
        log(f"warmup {w}: groups={out['n_groups']} chains={out['n_chains']}")
        del out

    # timed region: the kNN kernel is bracketed by HIP events on its stream
    ctx.set_profiling(1)
    knn_ms, sort_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        st = ctx.stats()
        knn_ms.append(st["ms_knn"])
        sort_ms.append(st["ms_sort"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_profiling(0)
    ms_step = dt * 1e3 / args.steps
    value = n / (dt / args.steps)
    groups, chains = out["n_groups"], out["n_chains"]
    log(f"{args.steps} steps: {ms_step:.2f} ms/step, knn {np.mean(knn_ms):.2f} ms, "
        f"sort+tree {np.mean(sort_ms):.2f} ms, groups={groups} chains={chains}")
    roofline = knn_roofline(n, float(np.mean(knn_ms)), "k_knn_density", value, fused=True)
    # the kNN kernel's work, from its device counters (one untimed run)
    ctx.set_profiling(3)
    out = step()
    st = ctx.stats()
    ctx.set_profiling(0)
    buckets = (n + 63) // 64
    roofline["work"] = {"nodes_per_particle": st["nodes_visited"] / n,
                        "leaf_batches_per_particle": st["leaves_scanned"] / n / 4,
                        "insert_iterations_per_bucket": st["insert_iterations"] / buckets,
                        "offered_per_query": st["offered"] / n}
    log(f"kNN work: {roofline['work']}")
    # per-halo statistics of the last step's labels (an output after the
    # path, outside the timed step): centre, maximum radius, and the bulk
    # velocity of a seeded synthetic velocity field
    gen = torch.Generator(device=dev).manual_seed(7)
    vel = torch.randn((n, 3), generator=gen, device=dev, dtype=torch.float32) * 300.0
    ctx.halo_stats(pos, out["group"], out["table"], prm, vel=vel, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        ctx.halo_stats(pos, out["group"], out["table"], prm, vel=vel, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    halo_ms = e0.elapsed_time(e1) / 3
    del vel
    log(f"halo statistics: {groups} halos, {halo_ms:.2f} ms")
    halo = {"ms": round(halo_ms, 3), "halos": groups,
            "bytes_per_particle": 56, "achieved_gbs": round(56 * n / (halo_ms / 1e3) / 1e9, 2)}
    search = None
    if args.search == "compare":
        from dataclasses import replace
        ref = {k: out[k] for k in ("nbr", "density", "hop", "group")}
        del out
        models = radius_models(ctx, log)
        search = {"training": models.pop("train")}
        for name in ("plain", "analytic", "mlp"):
            q = prm
            if name != "plain":
                kind, w, margin = models[name]
                ctx.radius_load(kind, w, margin)
                q = replace(prm, learned_radius=True)
            # counters: one untimed run
            ctx.set_profiling(3)
            o = ctx.run(pos, q, stream=stream)
            st = ctx.stats()
            same = all(torch.equal(o[k], ref[k]) for k in ref)
            del o
            ctx.set_profiling(1)
            kms, rms = [], []
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for k in range(args.steps):
                o = ctx.run(pos, q, stream=stream)
                s2 = ctx.stats()
                kms.append(s2["ms_knn"])
                rms.append(s2["ms_radius"])
                del o
            torch.cuda.synchronize()
            d1 = (time.perf_counter() - t1) / args.steps
            ctx.set_profiling(0)
            search[name] = {"ms_per_step": d1 * 1e3, "value": n / d1,
                            "ms_knn": float(np.mean(kms)), "ms_radius": float(np.mean(rms)),
                            "nodes_per_particle": st["nodes_visited"] / n,
                            "leaf_batches_per_particle": st["leaves_scanned"] / n / 4,
                            "insert_iterations_per_bucket": st["insert_iterations"] / ((n + 63) // 64),
                            "offered_per_query": st["offered"] / n,
                            "misses": st["misses"], "miss_fraction": st["misses"] / n,
                            "fallback_buckets": st["redo_buckets"], "identical_output": same}
            if name != "plain":
                search[name]["margin"] = models[name][2]
            log(f"search {name}: {d1 * 1e3:.1f} ms/step, kNN {np.mean(kms):.1f} ms, "
                f"misses {st['misses']}, identical {same}")
            if not same:
                raise SystemExit(f"{name} search changed the output")
        ctx.radius_load(0)
        del ref
    else:
        del out
    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(p)
            log(f"cpu baseline: {cpu['value']:.3g} particles/s on {cpu['cores']} threads; "
                f"one thread: {[round(o['value']) for o in cpu['one_thread']]}")
        except Exception as e:  # the baseline is reported, never required
            log(f"cpu baseline failed: {e}")
    batch = None
    if args.batch:
        # the batched form on the same GPU: the 64-subvolume workload, one
        # batched call against 64 sequential calls, identical outputs
        ctx.close()
        del pos
        torch.cuda.empty_cache()
        b = bench_batch(args, cpu=False)
        batch = {k: b[k] for k in ("value", "ms_per_step", "sequential", "speedup_vs_sequential",
                                   "config")}
        batch["kernel_ms"] = b["roofline"]["kernel_ms"]
    return {"metric": "HOP particles/sec at 134M clustered (plain vs learned-radius); % HBM roofline",
            "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": p.name, "n": n, "n_dens": prm.n_dens, "n_hop": prm.n_hop,
                       "n_merge": prm.n_merge, "k_store": prm.k_store, "periodic": p.periodic,
                       "search": "plain", "groups": groups, "chains": chains},
            "roofline": roofline, "halo_stats": halo,
            "cpu_baseline": cpu, "search_compare": search, "batch64": batch}


def bench_batch(args, cpu=True):
    import numpy as np
    import torch

    import synth
    from paper_1001_3411_amd import HopContext, HopParams
    from paper_1001_3411_amd.autotune import tune_batch

    t0 = time.perf_counter()
    subs = synth.config(4)
    off = np.concatenate([[0], np.cumsum([q.n for q in subs])]).astype(np.int64)
    n = int(off[-1])
    log(f"generated {len(subs)} subvolumes, n={n} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(np.concatenate([q.pos for q in subs]).view(np.int32)).to(dev)
    padded = torch.from_numpy(np.concatenate([q.padded for q in subs])).to(dev)
    md = [q.mean_density for q in subs]
    prm = HopParams(periodic=False, padded_rules=True)
    ctx = HopContext(0)

    t0 = time.perf_counter()
    tune = tune_batch(ctx, pos, off, prm, padded=padded, mean_density=md,
                      cache_path=args.tune_cache)
    log(f"tuning {'(cached) ' if tune['cached'] else ''}{tune['tuning']} "
        f"{tune['ms']:.1f} ms in {time.perf_counter() - t0:.1f}s")

    def batched():
        return ctx.run_batch(pos, off, prm, padded=padded, mean_density=md)

    def sequential():
        outs = []
        for s in range(len(subs)):
            a, b = int(off[s]), int(off[s + 1])
            q = HopParams(periodic=False, padded_rules=True, mean_density=md[s])
            outs.append(ctx.run(pos[a:b], q, padded=padded[a:b]))
        return outs

    for w in range(args.warmup):
        out = batched()
        seq = sequential()
        torch.cuda.synchronize()
        same = all(torch.equal(out["group"][int(off[s]):int(off[s + 1])], seq[s]["group"])
                   and torch.equal(out["nbr"][int(off[s]):int(off[s + 1])], seq[s]["nbr"])
                   for s in range(len(subs)))
        log(f"warmup {w}: groups={sum(out['n_groups'])}, batched == sequential: {same}")
        if not same:
            raise SystemExit("batched and sequential results differ")
        del out, seq

    ctx.set_profiling(1)
    knn_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = batched()
        knn_ms.append(ctx.stats()["ms_knn"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_profiling(0)
    groups = sum(out["n_groups"])
    del out
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        seq = sequential()
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t1
    del seq
    ms_step = dt * 1e3 / args.steps
    ms_seq = dt_seq * 1e3 / args.steps
    value = n / (dt / args.steps)
    log(f"{args.steps} steps: batched {ms_step:.2f} ms/step (kNN {np.mean(knn_ms):.2f} ms), "
        f"sequential {ms_seq:.2f} ms/step")
    cpu_line = None
    if cpu and not args.no_cpu:
        try:
            import oracle
            k, t_cpu, done = 0, 0.0, 0
            while k < len(subs) and t_cpu < 10.0:
                q = subs[k]
                t2 = time.perf_counter()
                oracle.run(q.pos, periodic=False, mean_density=q.mean_density, padded=q.padded,
                           padded_rules=True)
                t_cpu += time.perf_counter() - t2
                done += q.n
                k += 1
            cpu_line = {"value": done / t_cpu, "unit": "particles/s", "cores": oracle.num_threads(),
                   "kind": "oracle",
                   "sample": f"the first {k} subvolumes ({done} particles), whole pipeline "
                             f"each, {t_cpu:.1f} s"}
        except Exception as e:
            log(f"cpu baseline failed: {e}")
    return {"metric": "HOP particles/sec, 64 padded subvolumes in one batched call",
            "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "batch64_subvolumes", "n": n, "n_sub": len(subs),
                       "periodic": False, "padded_rules": True, "groups": groups,
                       "tuning": tune["tuning"]},
            "sequential": {"ms_per_step": ms_seq, "value": n / (dt_seq / args.steps),
                           "launches": "64 x (hop_density_link, hop_groups, hop_merge)"},
            "speedup_vs_sequential": ms_seq / ms_step,
            "roofline": knn_roofline(n, float(np.mean(knn_ms)), "k_knn_batch", value),
            "cpu_baseline": cpu_line}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--workload", choices=["box", "batch64"], default="box")
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--search", choices=["compare", "plain"], default="compare")
    ap.add_argument("--no-batch", dest="batch", action="store_false",
                    help="box workload: skip the batched-vs-sequential comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy first (reference for the traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              f"decomposition is described in the design notes but not built.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
    line = bench_batch(args) if args.workload == "batch64" else bench_box(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
