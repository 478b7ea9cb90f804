"""Benchmark of the level-by-level k-d tree build on one MI355X.

A step is one complete kd_build (every level of the hot path) over the
resident synthetic input of the workload: by default n = 2^26 points, d = 16
(Student-t on a 2^-10 grid, Dirichlet(1/2) subset pool of 64 subsets,
largest-variance key, leaf 128), EXACT rule.  Prints ONE JSON line on
stdout; progress goes to stderr.

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
DEFAULT_WORKLOAD = "hard_n2^26_d16"

RULES = {"exact": 0, "fourier": 1, "subset": 2}
KEYS = {"cyclic": 0, "maxvar": 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stored_traffic(key):
    """Hardware-counter HBM bytes stored in profiles/traffic.json under `key`
    (rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a copy calibration),
    if they were taken on the current sources."""
    from paper_2201_08288_amd import _build
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != _build.source_hash():
        return None
    return t.get("entries", {}).get(key)


def workload_arrays(name):
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, pool, kw, w):
    """The oracle as it stands (C, OpenMP over a level's cells and inside
    large cells) on every host thread, on the same input as the GPU steps;
    plus its single-thread rate on the small plain workload."""
    import oracle
    from paper_2201_08288_amd import synth
    threads = oracle.set_threads(0)
    t0 = time.perf_counter()
    t = oracle.build_tree(x, pool=pool, **kw)
    dt = time.perf_counter() - t0
    pw = synth.WORKLOADS["plain_n65536_d3"]
    xp = synth.generate(pw["gen"], pw["n"], pw["d"])
    prev = oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        tp = oracle.build_tree(xp, leaf_size=pw["leaf_size"], num_subsets=pw["num_subsets"])
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(prev)
    return {"value": t["point_levels"] / dt, "unit": "point-levels/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the whole benchmark input ({w['n']} points, d={w['d']}, same tree "
                      f"parameters), one oracle build: {dt:.2f} s, {t['point_levels']} "
                      f"point-levels, {threads} OpenMP threads",
            "seconds": dt, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "single_thread_plain": {"value": tp["point_levels"] / dt1, "seconds": dt1,
                                    "workload": "plain_n65536_d3, EXACT"}}


def time_builds(kdtree, xt, pool_t, kw, ws, tree, steps, warmup, flags=0):
    """Wall time per build (ms) of `steps` builds after `warmup`, input
    resident, between two device synchronizations."""
    import torch
    for _ in range(warmup):
        kdtree.build(xt, subset_pool=pool_t, workspace=ws, tree=tree, flags=flags, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        kdtree.build(xt, subset_pool=pool_t, workspace=ws, tree=tree, flags=flags, **kw)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def event_pass(kdtree, xt, pool_t, kw, ws, tree, steps, flags=0):
    """The same builds with HIP events around every launch on the build's
    stream (kd_build_profiled): per-kernel-class time, launches and
    algorithmic bytes, summed over `steps` builds."""
    import torch
    agg = {}
    torch.cuda.synchronize()
    for _ in range(steps):
        prof = kdtree.Profile()
        kdtree.build(xt, subset_pool=pool_t, workspace=ws, tree=tree, profile=prof, flags=flags,
                     **kw)
        for k, v in prof.to_dict().items():
            if k == "levels":
                agg["levels"] = v
                continue
            a = agg.setdefault(k, {"ms": 0.0, "launches": 0, "points": 0, "bytes": 0})
            for f in ("ms", "launches", "points", "bytes"):
                a[f] += v[f]
    torch.cuda.synchronize()
    return agg


def kernel_table(agg, steps):
    out = {}
    for k, v in agg.items():
        if k == "levels" or v["launches"] == 0:
            continue
        out[k] = {"ms_per_step": v["ms"] / steps, "avg_launch_us": 1e3 * v["ms"] / v["launches"],
                  "launches_per_step": v["launches"] / steps,
                  "alg_GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
    return out


def whole_build(ms, pl, d, workload, rule, mode):
    """Algorithmic bytes B_alg = 8d + 12 per point-level (the key read once
    for the statistic; d columns and the permutation read and written) over
    the wall time of a build, beside the counter bytes of one build when
    stored for these sources."""
    b_alg = 8 * d + 12
    gbps = b_alg * pl / (ms * 1e-3) / 1e9
    out = {"ms": round(ms, 3), "alg_bytes": b_alg * pl, "alg_GBps": round(gbps, 1),
           "alg_frac": round(gbps / HBM_PEAK_GBPS, 4), "counter_bytes": None,
           "counter_GBps": None}
    e = stored_traffic(f"{workload}/{rule}/whole/{mode}")
    if e is not None:
        out["counter_bytes"] = e["bytes_per_build"]
        out["counter_GBps"] = round(e["bytes_per_build"] / (ms * 1e-3) / 1e9, 1)
        out["counter_over_alg"] = round(e["bytes_per_build"] / (b_alg * pl), 3)
    return out


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


def bench_other_workload(name, rules, steps=5, warmup=1, queries=False):
    """Build time and whole-build fraction of another workload under each rule
    (kd_build, default launch shapes); with queries, the kNN and box queries
    on its EXACT tree."""
    import numpy as np
    import torch

    from paper_2201_08288_amd import kdtree
    w, x, pool = workload_arrays(name)
    d = x.shape[0]
    xt = torch.from_numpy(x).cuda()
    pool_t = None if pool is None else torch.from_numpy(pool.view(np.int32)).cuda()
    out = {}
    for rule in rules:
        kw = tree_kwargs(w, rule)
        tree = kdtree.build(xt, subset_pool=pool_t, **kw)
        torch.cuda.synchronize()
        hdr = tree.header()
        assert hdr["status"] == 0, hdr
        ms = time_builds(kdtree, xt, pool_t, kw, tree.workspace, tree, steps, warmup)
        res = whole_build(ms, hdr["point_levels"], d, name, rule, "with_subtree")
        res.update({"depth": hdr["depth"], "point_levels": hdr["point_levels"],
                    "point_levels_per_s": hdr["point_levels"] / (ms * 1e-3)})
        out[rule] = res
        if queries and rule == "exact":
            out["queries"] = bench_queries(tree, xt)
        del tree
        torch.cuda.empty_cache()
    return out


def bench_batched(trees=512, reps=3):
    """512 independent trees: one kd_build_batched call, the same call
    captured in a graph and replayed, and 512 plain kd_build calls, on the
    same device inputs; every tree must be identical."""
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
    ws = None
    t0 = time.perf_counter()
    for _ in range(reps):
        bt = kdtree.build_batched(pts, **kw)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    # the batched call captured once, replayed: no host work per build
    prm = kdtree.make_params(**kw)
    gt = [kdtree.KDTree(x.shape[1], x.shape[0], kdtree.tree_bounds(x.shape[1], x.shape[0], prm)[0],
                        x.device) for x in pts]
    items = (kdtree.BatchItem * trees)()
    for i, (x, t) in enumerate(zip(pts, gt)):
        items[i].pts, items[i].n, items[i].d = x.data_ptr(), x.shape[1], x.shape[0]
        items[i].ld, items[i].out = (x.stride(0) if x.shape[0] > 1 else x.shape[1]), t.struct
    wsb = kdtree._u64()
    kdtree._check(kdtree.lib().kd_batch_bounds(trees, items, kdtree.ctypes.byref(prm),
                                               kdtree.ctypes.byref(wsb)), "kd_batch_bounds")
    ws = torch.empty(wsb.value, dtype=torch.uint8, device="cuda")
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=s):
        kdtree._check(kdtree.lib().kd_build_batched(
            trees, items, kdtree.ctypes.byref(prm), ws.data_ptr(), ws.numel(),
            torch.cuda.current_stream().cuda_stream), "kd_build_batched")
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    same = True
    for a, b, c in zip(plain, bt, gt):
        ha, hb, hc = a.header(), b.header(), c.header()
        same &= ha == hb == hc
        if not same:
            continue
        size = {"perm": a.n, "node_child": ha["num_nodes"], "node_split": ha["num_nodes"],
                "node_dim": ha["num_nodes"], "leaf_offsets": ha["num_leaves"] + 1}
        for f, m in size.items():
            same &= bool(torch.equal(getattr(a, f)[:m], getattr(b, f)[:m]))
            same &= bool(torch.equal(getattr(a, f)[:m], getattr(c, f)[:m]))
    total = sum(n for n, _ in shapes)
    pl = sum(t.header()["point_levels"] for t in bt)
    return {"trees": trees, "points": total, "point_levels": pl,
            "plain_trees_per_s": trees / t_plain, "batched_trees_per_s": trees / t_batched,
            "graph_trees_per_s": trees / t_graph,
            "speedup": t_plain / t_batched, "graph_speedup": t_plain / t_graph,
            "plain_ms": 1e3 * t_plain, "batched_ms": 1e3 * t_batched, "graph_ms": 1e3 * t_graph,
            "identical": bool(same),
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


def bench_serving(rates=(50, 100, 200, 500, 1000, 2000), per_rate=2000, warm=200, workers=3):
    """Poisson build requests (n log-uniform [2^12, 2^22], d in {3,16},
    Gaussian mixture, S=64, leaf 64) each followed by 1,024 lookups of its
    own points; p50/p99 latency from arrival to lookups done over `per_rate`
    requests after `warm` warm-up requests, at each rate.  The same request
    shapes and points serve every rate (arrival gaps differ)."""
    import numpy as np
    import torch

    from paper_2201_08288_amd import serve, synth
    gen = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + 5)
    params = dict(leaf_size=64, num_subsets=64)
    reqs = synth.poisson_requests(warm + per_rate, 100.0, stream=5)
    data = []
    for k, (_, n, d) in enumerate(reqs):
        x = gpu_gmm(n, d, gen)
        idx = torch.randint(0, n, (1024,), generator=gen, device="cuda")
        data.append((x, x[:, idx].contiguous()))
    torch.cuda.synchronize()
    eng = serve.ServeEngine(params, cap_bytes=64 << 30, workers=workers)
    out = {}
    try:
        for rate in rates:
            log(f"[bench] serving at {rate}/s")
            done = serve.run_poisson(eng, data, rate, seed=rate)
            ok = all(r.status == 0 for r in done)
            st = serve.latency_stats(done[warm:])
            st["all_ok"] = ok
            st["mean_batch"] = float(np.mean(eng.batch_sizes)) if eng.batch_sizes else 0.0
            eng.batch_sizes.clear()
            out[str(rate)] = st
            for r in done:
                r.tree = r.leaves = None
            del done
    finally:
        eng.close()
    del data
    torch.cuda.empty_cache()
    return {"rates_per_s": out, "workers": workers, "requests_per_rate": per_rate,
            "warmup_requests": warm,
            "workload": "Poisson arrivals; n log-uniform [2^12, 2^22], d in {3,16}, Gaussian "
                        "mixture, S=64, leaf 64, EXACT; 1,024 lookups per request; cap 64 GB"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--rule", default="exact", choices=sorted(RULES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rules", action="store_true",
                    help="skip the other split rules on the benchmark input")
    ap.add_argument("--no-scale", action="store_true", help="skip the n = 2^24 workload")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--no-queries", action="store_true")
    ap.add_argument("--no-global", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch shapes instead of kd_autotune's choice")
    ap.add_argument("--tuning", default=None, metavar="HIST,SCATTER,SMALL[,DIGIT]",
                    help="use these launch shapes (workgroup counts, 0 = default) and digit "
                         "width (11 or 8, 0 = 11) instead of kd_autotune's choice")
    ap.add_argument("--no-other-path", action="store_true",
                    help="skip timing the build's other path (per-level / on-chip small cells)")
    ap.add_argument("--level-by-level", action="store_true",
                    help="time the plain per-level build (KD_FLAG_LEVEL_BY_LEVEL) in the main "
                         "steps, e.g. for a profiler run")
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
    main_flags = kdtree.FLAG_LEVEL_BY_LEVEL if args.level_by_level else 0
    tuning = kdtree.get_tuning()
    if args.tuning is not None:
        kdtree.set_tuning(*(int(v) for v in args.tuning.split(",")))
        tuning = kdtree.get_tuning()
    elif not args.no_autotune:
        log("[bench] autotune")
        tuning = kdtree.autotune(xt, subset_pool=pool_t, flags=main_flags, **kw)
    tree = kdtree.build(xt, subset_pool=pool_t, flags=main_flags, **kw)
    torch.cuda.synchronize()
    hdr = tree.header()
    assert hdr["status"] == 0, hdr
    ws = tree.workspace
    pl = hdr["point_levels"]
    log(f"[bench] tree: {hdr}")

    log(f"[bench] timing {args.steps} steps")
    ms = time_builds(kdtree, xt, pool_t, kw, ws, tree, args.steps, args.warmup, main_flags)
    value = pl / (ms * 1e-3)

    # Same steps again with HIP events around every launch (on the build stream).
    log("[bench] profiled steps")
    tp0 = time.perf_counter()
    agg = event_pass(kdtree, xt, pool_t, kw, ws, tree, args.steps, main_flags)
    ms_events = 1e3 * (time.perf_counter() - tp0) / args.steps
    kernels = kernel_table(agg, args.steps)
    byte_kinds = [k for k in ("big_scatter", "small", "select", "count", "ingest") if k in agg
                  and agg[k]["bytes"] > 0]
    dom = max(byte_kinds, key=lambda k: agg[k]["ms"])
    a = agg[dom]
    achieved = a["bytes"] / (a["ms"] * 1e-3) / 1e9
    mode = "per_level" if args.level_by_level else "with_subtree"
    tr = stored_traffic(f"{args.workload}/{args.rule}/{mode}/{dom}")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if tr is None else tr["bytes_per_launch"],
                "kernel": dom, "avg_launch_us": round(1e3 * a["ms"] / a["launches"], 2),
                "alg_bytes_per_launch": a["bytes"] / a["launches"]}

    # The whole build both ways: small cells finished on chip (the library's
    # default) and the plain per-level build (every level through HBM).
    wb = {mode: whole_build(ms, pl, d, args.workload, args.rule, mode)}
    other = "with_subtree" if args.level_by_level else "per_level"
    other_flags = 0 if args.level_by_level else kdtree.FLAG_LEVEL_BY_LEVEL
    if not args.no_other_path:
        log(f"[bench] whole build, {other}")
        t2 = kdtree.build(xt, subset_pool=pool_t, flags=other_flags, **kw)
        torch.cuda.synchronize()
        assert t2.header() == hdr
        ms2 = time_builds(kdtree, xt, pool_t, kw, t2.workspace, t2, args.steps, args.warmup,
                          other_flags)
        wb[other] = whole_build(ms2, pl, d, args.workload, args.rule, other)
        agg2 = event_pass(kdtree, xt, pool_t, kw, t2.workspace, t2, max(2, args.steps // 3),
                          other_flags)
        wb[other]["kernels"] = kernel_table(agg2, max(2, args.steps // 3))
        del t2
        torch.cuda.empty_cache()

    rules = None
    if not args.no_rules:
        others = [r for r in RULES if r != args.rule]
        log(f"[bench] rules {others} on the same input")
        rules = {}
        for r in others:
            kr = tree_kwargs(w, r)
            t3 = kdtree.build(xt, subset_pool=pool_t, **kr)
            torch.cuda.synchronize()
            h3 = t3.header()
            ms3 = time_builds(kdtree, xt, pool_t, kr, t3.workspace, t3, max(3, args.steps // 2), 1)
            rules[r] = whole_build(ms3, h3["point_levels"], d, args.workload, r, "with_subtree")
            rules[r].update({"depth": h3["depth"], "point_levels": h3["point_levels"],
                             "point_levels_per_s": h3["point_levels"] / (ms3 * 1e-3)})
            del t3
            torch.cuda.empty_cache()

    queries = None
    if not args.no_queries and (args.no_scale or args.workload == "scale_n2^24_d8"):
        log("[bench] queries (kNN, boxes)")
        queries = bench_queries(tree, xt)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: the oracle on the same input, every host thread")
        cpu = cpu_baseline(x, pool, kw, w)

    del tree, ws
    xt = None
    torch.cuda.empty_cache()

    kdtree.set_tuning()  # everything below runs the default launch shapes
    scale = None
    if not args.no_scale and args.workload != "scale_n2^24_d8":
        log("[bench] scale workload n=2^24 d=8, every rule (and queries on its tree)")
        scale = bench_other_workload("scale_n2^24_d8", list(RULES), queries=not args.no_queries)
        queries = scale.pop("queries", None)

    glob = None
    if not args.no_global:
        log("[bench] global single-pass construction")
        glob = bench_global()

    batched = serving = None
    if not args.no_batched:
        log("[bench] batched vs plain (512 trees)")
        batched = bench_batched()
    if not args.no_serving:
        log("[bench] serving")
        serving = bench_serving(per_rate=args.serving_requests,
                                warm=max(1, args.serving_requests // 10))

    out = {
        "metric": "points·levels/s", "value": value, "unit": "point-levels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "gen": w["gen"],
                   "split_rule": args.rule, "key": w["key"], "leaf_size": w["leaf_size"],
                   "num_subsets": w["num_subsets"],
                   "subsets": "Dirichlet(1/2) pool" if pool is not None else "equal",
                   "path": mode, "parallelism": "single-gpu", "launch_shapes": tuning},
        "point_levels_per_step": pl, "depth": hdr["depth"], "levels": agg.get("levels"),
        "ms_per_step_event_pass": round(ms_events, 4),
        "whole_build": wb,
        "whole_build_alg_GBps": wb[mode]["alg_GBps"],
        "whole_build_alg_frac": wb[mode]["alg_frac"],
        "roofline": roofline, "kernels": kernels, "cpu_baseline": cpu,
        "rules": rules, "scale": scale, "copy_GBps": round(copy_gbps, 1),
        "batched": batched, "serving": serving, "queries": queries, "global": glob,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
