"""Benchmark of the level-by-level k-d tree build on one MI355X.

A step is one complete kd_build (every level of the hot path) over the
resident synthetic input of the workload.  Prints ONE JSON line on stdout;
progress goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--rule exact]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def source_hash():
    """sha256 over the library's sources, to tell whether stored hardware
    counter readings still describe the kernels being run."""
    import hashlib
    from paper_2201_08288_amd import _build
    h = hashlib.sha256()
    for f in _build.sources():
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def stored_traffic(workload, rule, kernel):
    """HBM bytes per launch of `kernel` from rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs (scaled by the copy calibration), if taken on these sources."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_hash():
        return None
    e = t.get("entries", {}).get(f"{workload}/{rule}/{kernel}")
    return None if e is None else e["bytes_per_launch"]


RULES = {"exact": 0, "fourier": 1, "subset": 2}
KEYS = {"cyclic": 0, "maxvar": 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_arrays(name, rng_seed=None):
    from paper_2201_08288_amd import synth
    w = synth.WORKLOADS[name]
    x = synth.generate(w["gen"], w["n"], w["d"])
    pool = None
    if w.get("pool_entries"):
        pool = synth.dirichlet_pool(w["pool_entries"], w["num_subsets"], w.get("pool_alpha", 0.5))
    return w, x, pool


def tree_kwargs(w, rule):
    return dict(leaf_size=w["leaf_size"], num_subsets=w["num_subsets"], key_rule=KEYS[w["key"]],
                split_rule=RULES[rule], fourier_J=15, seed=w.get("seed", 0))


def cpu_baseline(w, rule, sample_n):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    from paper_2201_08288_amd import synth
    x = synth.generate(w["gen"], sample_n, w["d"], stream=1)
    pool = None
    if w.get("pool_entries"):
        pool = synth.dirichlet_pool(w["pool_entries"], w["num_subsets"], w.get("pool_alpha", 0.5))
    kw = tree_kwargs(w, rule)
    t0 = time.perf_counter()
    t = oracle.build_tree(x, pool=pool, **kw)
    dt = time.perf_counter() - t0
    return {"value": t["point_levels"] / dt, "unit": "point-levels/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{sample_n} points of the same {w['gen']} recipe (d={w['d']}), "
                      f"same tree parameters, single-threaded C oracle, {dt:.2f} s, "
                      f"{t['point_levels']} point-levels"}


def gpu_uniform24(n, d, gen):
    import torch
    k = torch.randint(0, 1 << 24, (d, n), generator=gen, device="cuda", dtype=torch.int32)
    return k.to(torch.float32) * (2.0 ** -24)


def gpu_gmm(n, d, gen, components=10, box=5.0, sigma=0.5):
    import torch
    means = (torch.rand((components, d), generator=gen, device="cuda", dtype=torch.float64)
             * 2 * box - box)
    comp = torch.randint(0, components, (n,), generator=gen, device="cuda")
    z = torch.randn((n, d), generator=gen, device="cuda", dtype=torch.float64)
    return (means[comp] + sigma * z).to(torch.float32).t().contiguous()


def bench_batched(trees=512, reps=3):
    """512 independent trees: one kd_build_batched against 512 plain kd_build
    calls on the same inputs; trees must be identical."""
    import torch

    from paper_2201_08288_amd import kdtree, synth
    shapes = synth.batched_shapes(trees)
    gen = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + 4)
    pts = [gpu_uniform24(n, d, gen) for n, d in shapes]
    kw = dict(leaf_size=32, num_subsets=32)
    plain = [kdtree.build(x, **kw) for x in pts]  # also allocates outputs/workspaces
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for x, t in zip(pts, plain):
            kdtree.build(x, workspace=t.workspace, tree=t, **kw)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    bt = kdtree.build_batched(pts, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bt = kdtree.build_batched(pts, **kw)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    same = True
    for a, b in zip(plain, bt):
        ha, hb = a.header(), b.header()
        same &= ha == hb
        if ha != hb:
            continue
        size = {"perm": a.n, "node_child": ha["num_nodes"], "node_split": ha["num_nodes"],
                "node_dim": ha["num_nodes"], "leaf_offsets": ha["num_leaves"] + 1}
        for f, m in size.items():
            same &= bool(torch.equal(getattr(a, f)[:m], getattr(b, f)[:m]))
    total = sum(n for n, _ in shapes)
    pl = sum(t.header()["point_levels"] for t in bt)
    return {"trees": trees, "points": total, "point_levels": pl,
            "plain_trees_per_s": trees / t_plain, "batched_trees_per_s": trees / t_batched,
            "speedup": t_plain / t_batched, "plain_ms": 1e3 * t_plain,
            "batched_ms": 1e3 * t_batched, "identical": bool(same),
            "workload": "512 trees, n log-uniform [2^10, 2^20], d in {2,3,8,32}, uniform24, "
                        "S=32, leaf 32, EXACT, cyclic"}


def bench_queries(tree, xt, nbox=1 << 16, k=8, reps=3):
    """Queries on the built tree: k nearest neighbours of data points moved by
    a small Gaussian step (2^20 queries up to 8 dimensions, 2^12 above, where
    each query visits many more leaves), and boxes of half-width 0.05 around
    data points (counts only)."""
    import torch

    from paper_2201_08288_amd import kdtree, synth
    gen = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + 6)
    d, n = xt.shape
    nq = 1 << 20 if d <= 8 else 1 << 12
    q = xt[:, torch.randint(0, n, (nq,), generator=gen, device="cuda")]
    q = (q + 0.05 * torch.randn(q.shape, generator=gen, device="cuda")).contiguous()
    c = xt[:, torch.randint(0, n, (nbox,), generator=gen, device="cuda")]
    lo, hi = (c - 0.05).contiguous(), (c + 0.05).contiguous()
    kdtree.query_knn(tree, q, k)
    cnt = kdtree.query_box(tree, lo, hi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        kdtree.query_knn(tree, q, k)
    torch.cuda.synchronize()
    t_knn = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        cnt = kdtree.query_box(tree, lo, hi)
    torch.cuda.synchronize()
    t_box = (time.perf_counter() - t0) / reps
    return {"knn": {"queries": nq, "k": k, "ms": 1e3 * t_knn, "queries_per_s": nq / t_knn},
            "box": {"boxes": nbox, "half_width": 0.05, "ms": 1e3 * t_box, "boxes_per_s": nbox / t_box,
                    "mean_count": float(cnt.double().mean().item())},
            "workload": "the benchmark tree; kNN of data points plus N(0, 0.05^2) steps, "
                        "boxes of half-width 0.05 around data points"}


def bench_global(n=1 << 26, J=15, depths=(6, 10), reps=3):
    """The paper's global single-pass construction on its §5 workload shape:
    trivariate normal, common correlation 0.5, each coordinate mapped into
    (0,1) by the standard normal CDF (generated on the device)."""
    import numpy as np
    import torch

    from paper_2201_08288_amd import kdtree, synth
    gen = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + 7)
    rho = 0.5
    cov = torch.full((3, 3), rho, dtype=torch.float64, device="cuda")
    cov.fill_diagonal_(1.0)
    L = torch.linalg.cholesky(cov)
    z = torch.randn((3, n), generator=gen, device="cuda", dtype=torch.float64)
    u = torch.special.ndtr(L @ z).clamp(2.0 ** -24, 1 - 2.0 ** -24).to(torch.float32).contiguous()
    del z
    C = kdtree.global_moments(u, J)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        C = kdtree.global_moments(u, J)
    torch.cuda.synchronize()
    t_map = (time.perf_counter() - t0) / reps
    flops = 2.0 * n * (2 * J + 1) ** 3
    out = {"n": n, "p": 3, "J": J, "map_ms": 1e3 * t_map, "map_points_per_s": n / t_map,
           "map_fp64_TFLOPs": flops / t_map / 1e12, "fp64_peak_TFLOPs": 78.6,
           "workload": "trivariate normal, rho 0.5, mapped into (0,1) by the normal CDF"}
    for depth in depths:
        med = kdtree.global_solve(C, 3, J, depth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        med = kdtree.global_solve(C, 3, J, depth)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        cnt = kdtree.global_counts(u, med, depth)
        torch.cuda.synchronize()
        rel = np.log2(cnt.cpu().numpy() / (n / 2 ** depth))
        q1, q3 = np.percentile(rel, [25, 75])
        out[f"depth{depth}"] = {"solve_ms": 1e3 * t_solve, "log2_rel_min": float(rel.min()),
                                "log2_rel_max": float(rel.max()), "log2_rel_iqr": [float(q1), float(q3)]}
    del u
    torch.cuda.empty_cache()
    return out


def bench_serving(rates=(50, 200, 1000, 2000), per_rate=150, warm=20, workers=3):
    """Poisson build requests (n log-uniform [2^12, 2^22], d in {3,16},
    Gaussian mixture, S=64, leaf 64) each followed by 1,024 lookups of its
    own points; p50/p99 latency from arrival to lookups done."""
    import numpy as np
    import torch

    from paper_2201_08288_amd import serve, synth
    gen = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + 5)
    params = dict(leaf_size=64, num_subsets=64)
    eng = serve.ServeEngine(params, cap_bytes=64 << 30, workers=workers)
    out = {}
    try:
        for rate in rates:
            reqs = synth.poisson_requests(warm + per_rate, rate, stream=rate)
            data = []
            for k, (_, n, d) in enumerate(reqs):
                x = gpu_gmm(n, d, gen)
                idx = torch.randint(0, n, (1024,), generator=gen, device="cuda")
                data.append((x, x[:, idx].contiguous()))
            torch.cuda.synchronize()
            done = serve.run_poisson(eng, data, rate, seed=rate)
            ok = all(r.status == 0 for r in done)
            st = serve.latency_stats(done[warm:])
            st["all_ok"] = ok
            st["mean_batch"] = float(np.mean(eng.batch_sizes)) if eng.batch_sizes else 0.0
            eng.batch_sizes.clear()
            out[str(rate)] = st
            del data, done
            torch.cuda.empty_cache()
    finally:
        eng.close()
    return {"rates_per_s": out, "workers": workers,
            "workload": "Poisson arrivals; n log-uniform [2^12, 2^22], d in {3,16}, Gaussian "
                        "mixture, S=64, leaf 64, EXACT; 1,024 lookups per request; cap 64 GB"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale_n2^24_d8")
    ap.add_argument("--rule", default="exact", choices=sorted(RULES))
    ap.add_argument("--cpu-sample", type=int, default=1 << 22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-queries", action="store_true")
    ap.add_argument("--no-global", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch shapes instead of kd_autotune's choice")
    ap.add_argument("--tuning", default=None, metavar="HIST,SCATTER,SMALL",
                    help="use these launch shapes (workgroup counts, 0 = default) instead of "
                         "kd_autotune's choice")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (a kernel of known "
                         "traffic for calibrating hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the build does not shard across GPUs); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2201_08288_amd import kdtree
    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        m = args.copy_probe_mib << 20
        a = torch.ones(m // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {m} bytes read, {m} bytes written")
        del a, b
    # context for the roofline: what a plain device-to-device copy reaches
    a = torch.empty(1 << 26, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    copy_gbps = 10 * 2 * a.numel() * 4 / (time.perf_counter() - t0) / 1e9
    del a, b
    log(f"[bench] generating workload {args.workload}")
    w, x, pool = workload_arrays(args.workload)
    d, n = x.shape
    xt = torch.from_numpy(x).to(dev)
    pool_t = None if pool is None else torch.from_numpy(pool.view(np.int32)).to(dev)
    kw = tree_kwargs(w, args.rule)
    tuning = kdtree.get_tuning()
    if args.tuning is not None:
        h, sc, sm = (int(v) for v in args.tuning.split(","))
        kdtree.set_tuning(h, sc, sm)
        tuning = kdtree.get_tuning()
    elif not args.no_autotune:
        log("[bench] autotune")
        tuning = kdtree.autotune(xt, subset_pool=pool_t, **kw)
    tree = kdtree.build(xt, subset_pool=pool_t, **kw)
    torch.cuda.synchronize()
    hdr = tree.header()
    assert hdr["status"] == 0, hdr
    ws = tree.workspace
    log(f"[bench] tree: {hdr}")

    for _ in range(args.warmup):
        kdtree.build(xt, subset_pool=pool_t, workspace=ws, tree=tree, **kw)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        kdtree.build(xt, subset_pool=pool_t, workspace=ws, tree=tree, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    pl = hdr["point_levels"]
    value = pl * args.steps / dt

    # Same steps again with HIP events around every launch (on the build stream).
    log("[bench] profiled steps")
    agg = {}
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        prof = kdtree.Profile()
        kdtree.build(xt, subset_pool=pool_t, workspace=ws, tree=tree, profile=prof, **kw)
        for k, v in prof.to_dict().items():
            if k == "levels":
                agg["levels"] = v
                continue
            a = agg.setdefault(k, {"ms": 0.0, "launches": 0, "points": 0, "bytes": 0})
            for f in ("ms", "launches", "points", "bytes"):
                a[f] += v[f]
    torch.cuda.synchronize()
    ms_events = 1e3 * (time.perf_counter() - tp0) / args.steps
    kernels = {}
    for k, v in agg.items():
        if k == "levels" or v["launches"] == 0:
            continue
        kernels[k] = {"ms_per_step": v["ms"] / args.steps,
                      "avg_launch_us": 1e3 * v["ms"] / v["launches"],
                      "launches_per_step": v["launches"] / args.steps,
                      "alg_GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
    byte_kinds = [k for k in ("big_scatter", "small", "select", "count", "ingest") if k in agg
                  and agg[k]["bytes"] > 0]
    dom = max(byte_kinds, key=lambda k: agg[k]["ms"])
    a = agg[dom]
    achieved = a["bytes"] / (a["ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": stored_traffic(args.workload, args.rule, dom),
                "kernel": dom, "avg_launch_us": round(1e3 * a["ms"] / a["launches"], 2),
                "alg_bytes_per_launch": a["bytes"] / a["launches"]}
    b_alg = 8 * d + 12
    level_gbps = b_alg * pl / (ms * 1e-3) / 1e9

    queries = None
    if not args.no_queries:
        log("[bench] queries (kNN, boxes)")
        queries = bench_queries(tree, xt)

    glob = None
    if not args.no_global:
        log("[bench] global single-pass construction")
        glob = bench_global()

    batched = serving = None
    kdtree.set_tuning()  # batched and serving run the default launch shapes
    if not args.no_batched:
        log("[bench] batched vs plain (512 trees)")
        batched = bench_batched()
    if not args.no_serving:
        log("[bench] serving")
        serving = bench_serving()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline on {args.cpu_sample} points")
        cpu = cpu_baseline(w, args.rule, args.cpu_sample)

    out = {
        "metric": "points·levels/s", "value": value, "unit": "point-levels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "gen": w["gen"],
                   "split_rule": args.rule, "key": w["key"], "leaf_size": w["leaf_size"],
                   "num_subsets": w["num_subsets"], "parallelism": "single-gpu",
                   "launch_shapes": tuning},
        "point_levels_per_step": pl, "levels": agg.get("levels"),
        "ms_per_step_event_pass": round(ms_events, 4),
        "whole_build_alg_GBps": round(level_gbps, 1),
        "whole_build_alg_frac": round(level_gbps / HBM_PEAK_GBPS, 4),
        "roofline": roofline, "kernels": kernels, "cpu_baseline": cpu,
        "copy_GBps": round(copy_gbps, 1),
        "batched": batched, "serving": serving, "queries": queries, "global": glob,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
