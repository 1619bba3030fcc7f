"""Benchmark of the Pkd-tree hot path on one MI355X.

One step = the whole path over one batch of synthetic input: build a tree of
1e8 uniform 3-D int64 points in [0, 1e9), answer 1e7 uniform 10-NN queries and
1e5 range counts (boxes with log-uniform sides in [1e5, 1e8]), free the tree.
Inputs are generated on the host (seeded) and resident in HBM before timing.

Prints one JSON line (the bench contract) with:
  value      build throughput, Mpts/s (n / mean build time)
  roofline   the sieve scatter kernel (the largest HBM mover of the build):
             algorithmic bytes per launch / mean launch duration, from HIP
             events the library records on the launch stream
  cpu_baseline  the sequential CPU oracle timed on a bounded sample
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--queries", type=int, default=10_000_000)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--boxes", type=int, default=100_000)
    ap.add_argument("--tile", type=int, default=2048)
    ap.add_argument("--cpu-sample", type=int, default=100_000_000,
                    help="points of the oracle's Build (default: the whole benchmark point set)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="build",
                    choices=["build", "batching", "serving", "updates", "large_updates", "range_report",
                             "alpha_sweep", "sliding_window", "pkd_bb", "ablation"],
                    help="build: the headline (1e8 3-D build + queries); batching: 4096 trees in one pass")
    ap.add_argument("--serve-n", type=int, default=1_000_000_000, help="points of the resident serving tree")
    ap.add_argument("--requests", type=int, default=300, help="requests in the serving stream")
    ap.add_argument("--loads", default="0.5,0.8,0.95",
                    help="offered Poisson rates as fractions of the serial handler's capacity")
    ap.add_argument("--batch", type=int, default=1_000_000, help="points per BatchInsert / BatchDelete (updates)")
    ap.add_argument("--trees", type=int, default=4096)
    ap.add_argument("--tree-hi", type=float, default=1e6, help="batching: largest tree size (log-uniform from 1e3)")
    ap.add_argument("--batches", type=int, default=1000, help="alpha_sweep: batches the stream is cut into")
    ap.add_argument("--alphas", default="1/100,5/100,1/10,2/10,3/10,4/10,1/2",
                    help="alpha_sweep: balance parameters num/den")
    ap.add_argument("--years", type=int, default=20, help="sliding_window: batches (years) in the stream")
    ap.add_argument("--window", type=int, default=5, help="sliding_window: years the tree holds")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="batching: skip the one-call-per-tree comparison")
    ap.add_argument("--params", default=None, help="batching: fixed lambda,sigma,phi,tile instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 2 GiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


# the sources a kernel's counter figures depend on
TRAFFIC_SOURCES = {"sieve_scatter": ("build.hip", "pkd_internal.h"), "knn": ("query.hip", "pkd_internal.h"),
                   "finisher": ("build.hip", "pkd_internal.h")}


def source_hash(kernel="sieve_scatter"):
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2411_09275_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it is missing or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash(kernel):
        return None
    return t.get("traffic_bytes_per_launch")


def host_info():
    """Threads this process may use and the host CPU model."""
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, model


def knn_bytes_per_query(work, dim, k):
    """Algorithmic bytes of one k-NN query from its search work: every node
    record read (32 B), the packed 32-bit coordinates of every point scanned
    (4 B per dimension), the query (8 B per dimension) and its k (id, d2)
    results (16 B each)."""
    return 32.0 * work["nodes"] + 4.0 * dim * work["points"] + 8.0 * dim + 16.0 * k


def stored_knn_work(n, dim, k):
    """Per-query k-NN work of the benchmark's tree from the committed oracle
    count (oracle/knn_work.py), when it covers this workload."""
    path = os.path.join(ROOT, "profiles", "knn_work_1e8_3d.json")
    if n != 100_000_000 or dim != 3 or not os.path.exists(path):
        return None
    with open(path) as f:
        w = json.load(f)
    return w["per_query"].get(str(k))


def cpu_baseline(coords, ids, q, dim, k, build_sample):
    """The sequential oracle on the host cores: Build of the benchmark's own
    point set (or its first build_sample points) on one thread, then its
    k-NN on that tree with one thread and with every thread this process may
    use (queries split over threads, the per-query search unchanged); also the
    search work of a query sample (nodes read, points scanned)."""
    import oracle
    threads, model = host_info()
    n = min(build_sample, ids.shape[0])
    c = np.ascontiguousarray(coords[:, :n]) if n < ids.shape[0] else coords
    t0 = time.perf_counter()
    T = oracle.Tree(oracle.Params(dim), c, ids[:n])
    t_build = time.perf_counter() - t0
    nq1 = min(100_000, q.shape[1])
    t0 = time.perf_counter()
    T.knn(np.ascontiguousarray(q[:, :nq1]), k)
    t1 = time.perf_counter() - t0
    nqt = min(1_000_000, q.shape[1])
    qt = np.ascontiguousarray(q[:, :nqt])
    t0 = time.perf_counter()
    T.knn_threads(qt, k, threads)
    tt = time.perf_counter() - t0
    rows = np.sort(np.random.default_rng(77).choice(q.shape[1], size=min(20000, q.shape[1]), replace=False))
    nodes, leaves, points = T.knn_visits(np.ascontiguousarray(q[:, rows]), k)
    work = {"nodes": float(nodes.mean()), "leaves": float(leaves.mean()), "points": float(points.mean())}
    del T
    return {
        "value": round(n / t_build / 1e6, 3),
        "unit": "Mpts/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "sequential oracle Build of %s (%d points, %.1f s, one thread); %d-NN of %d queries on one "
                  "thread and of %d queries on %d threads on that tree" % (
                      "the whole benchmark point set" if n == ids.shape[0] else "the first %d points" % n, n,
                      t_build, k, nq1, nqt, threads),
        "knn_qps_1_thread": round(nq1 / t1, 1),
        "knn_qps_all_threads": round(nqt / tt, 1),
        "knn_threads": threads,
        "host_threads": threads,
        "cpu_model": model,
    }, work


def bench_batching(a):
    """Many independent trees (sizes log-uniform in [1e3, 1e6], D from {2, 3},
    uniform int64 points) built by one batched pass per dimension, then 256
    k-NN queries per tree with k from {1, 10, 100}; compared with one build
    and one query call per tree, with identical results required."""
    import torch

    import paper_2411_09275_amd as pk
    from paper_2411_09275_amd import autotune
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    T = a.trees
    sizes = synth.log_uniform_sizes(T, 1e3, a.tree_hi, seed=10)
    rng = np.random.Generator(np.random.PCG64(12))
    dims = rng.choice([2, 3], size=T)
    ks = rng.choice([1, 10, 100], size=(T, 256))
    g = torch.Generator(device=dev)
    groups = {}
    for D in (2, 3):
        sel = np.nonzero(dims == D)[0]
        off = np.concatenate([[0], np.cumsum(sizes[sel])]).astype(np.int64)
        g.manual_seed(11 + D)
        c = torch.randint(0, 10 ** 9, (D, int(off[-1])), generator=g, device=dev, dtype=torch.int64)
        i = torch.arange(int(off[-1]), device=dev, dtype=torch.int64)
        q = torch.randint(0, 10 ** 9, (D, sel.shape[0] * 256), generator=g, device=dev, dtype=torch.int64)
        tree_of = np.repeat(np.arange(sel.shape[0]), 256).astype(np.int32)
        kq = ks[sel].reshape(-1)
        byk = {}
        for k in (1, 10, 100):
            idx = np.nonzero(kq == k)[0]
            byk[k] = (torch.from_numpy(idx).to(dev), q[:, torch.from_numpy(idx).to(dev)].contiguous(),
                      torch.from_numpy(tree_of[idx]).to(dev))
        groups[D] = dict(sel=sel, off=off, c=c, i=i, byk=byk)
    torch.cuda.synchronize()
    n_total = int(sizes.sum())
    log("batching workload: %d trees, %d points" % (T, n_total))

    params = {}
    for D, gr in groups.items():
        if a.params:
            lam, sigma, phi, tile = (int(x) for x in a.params.split(","))
            params[D] = (pk.Params(D, lam=lam, sigma=sigma, phi=phi), tile)
            continue
        if a.no_autotune:
            params[D] = (pk.Params(D), 2048)
            continue
        # tune on the first 128 trees of the group
        nt = min(128, gr["sel"].shape[0])
        o = gr["off"][: nt + 1]
        cs = gr["c"][:, : int(o[-1])].contiguous()
        is_ = gr["i"][: int(o[-1])].contiguous()
        # the sample's own query mix: every k, the queries of its trees
        mix = []
        for k, (idx, qk, tk) in gr["byk"].items():
            mine = torch.nonzero(tk < nt).flatten()
            mix.append((qk[:, mine].contiguous(), k, tk[mine].contiguous()))
        p, tile, sec = autotune.tune(D, cs, is_, offsets=o, queries=mix, log=log)
        params[D] = (p, tile)
        log("autotuned D=%d: lambda=%d sigma=%d phi=%d tile=%d" % (D, p.lam, p.sigma, p.phi, tile))

    def batched():
        res = {}
        for D, gr in groups.items():
            p, tile = params[D]
            t = pk.Tree.batch(p, gr["c"], gr["i"], gr["off"], tile=tile)
            for k, (idx, qk, tk) in gr["byk"].items():
                res[(D, k)] = t.knn(qk, k, tree_of=tk)
            t.free()
        return res

    for w in range(a.warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        res = batched()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / a.steps
    log("batched: %.1f ms per pass" % (t_batched * 1e3))
    graph = query_graph(groups, params, a, log)
    graph["build_and_queries"] = plan_graph(groups, params, a, log, res)

    if a.no_single:
        print(json.dumps({"metric": "batched build + k-NN over many trees", "batched_ms": round(t_batched * 1e3, 3),
                          "points": n_total, "query_phase": graph}))
        return
    # one build and one query call per tree (same parameters); the per-tree
    # query selections are made before the timed region, the result checks after
    per_tree = []
    for D, gr in groups.items():
        off = gr["off"]
        tk_host = {k: tk.cpu().numpy() for k, (idx, qk, tk) in gr["byk"].items()}
        order = {k: np.argsort(tk_host[k], kind="stable") for k in tk_host}
        bounds = {k: np.searchsorted(tk_host[k][order[k]], np.arange(gr["sel"].shape[0] + 1)) for k in tk_host}
        for j in range(gr["sel"].shape[0]):
            a0, a1 = int(off[j]), int(off[j + 1])
            qs = []
            for k, (idx, qk, tk) in gr["byk"].items():
                mine = order[k][bounds[k][j]:bounds[k][j + 1]]
                if mine.shape[0]:
                    mt = torch.from_numpy(mine).to(dev)
                    qs.append((k, mt, qk[:, mt].contiguous()))
            per_tree.append((D, gr["c"][:, a0:a1].contiguous(), gr["i"][a0:a1].contiguous(), qs))
    torch.cuda.synchronize()
    outs = []
    t0 = time.perf_counter()
    for D, cj, ij, qs in per_tree:
        p, tile = params[D]
        t = pk.Tree(p, cj, ij, tile=tile)
        outs.append([t.knn(qq, k) for k, _, qq in qs])
        t.free()
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    same = True
    for (D, _, _, qs), o in zip(per_tree, outs):
        for (k, mt, _), (oi, od) in zip(qs, o):
            bi, bd = res[(D, k)]
            same &= bool(torch.equal(oi, bi[mt]) and torch.equal(od, bd[mt]))
    del per_tree, outs
    log("one call per tree: %.1f ms; identical results: %s" % (t_single * 1e3, same))
    nq = T * 256
    out = {
        "metric": "batched build + k-NN over many trees: Mpts/s (vs one launch per tree)",
        "value": round(n_total / t_batched / 1e6, 2),
        "unit": "Mpts/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(t_batched * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "%d trees, sizes log-uniform [1e3,%.0e], D in {2,3}, uniform int64 in [0,1e9); "
                               "256 k-NN queries per tree, k in {1,10,100}" % (T, a.tree_hi), "points": n_total,
                   "queries": nq,
                   "params": {str(D): {"lambda": p.lam, "sigma": p.sigma, "phi": p.phi, "tile": tile}
                              for D, (p, tile) in params.items()}},
        "batched_ms": round(t_batched * 1e3, 3),
        "one_call_per_tree_ms": round(t_single * 1e3, 3),
        "speedup_vs_one_call_per_tree": round(t_single / t_batched, 2),
        "identical_results": same,
        "query_phase": graph,
    }
    print(json.dumps(out))


def query_graph(groups, params, a, log):
    """The query phase of the batching workload (k-NN over the batch handles,
    one launch per dimension and k) eagerly and as one captured hipGraph
    replayed; both timed over the same handles, results compared."""
    import torch

    import paper_2411_09275_amd as pk
    handles = {D: pk.Tree.batch(params[D][0], gr["c"], gr["i"], gr["off"], tile=params[D][1])
               for D, gr in groups.items()}
    calls = [(D, k, qk, tk) for D, gr in groups.items() for k, (idx, qk, tk) in gr["byk"].items()]
    outs = {(D, k): (torch.empty((qk.shape[1], k), dtype=torch.int64, device="cuda"),
                     torch.empty((qk.shape[1], k), dtype=torch.int64, device="cuda")) for D, k, qk, tk in calls}
    status = torch.zeros(1, dtype=torch.int32, device="cuda")

    def eager():
        return {(D, k): handles[D].knn(qk, k, tree_of=tk) for D, k, qk, tk in calls}

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for D, k, qk, tk in calls:
            handles[D].knn_async(qk, k, *outs[(D, k)], status, tree_of=tk, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        status.zero_()
        for D, k, qk, tk in calls:
            handles[D].knn_async(qk, k, *outs[(D, k)], status, tree_of=tk, stream=side)
    reps = max(3, a.steps)
    for _ in range(2):
        ref = eager()
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ref = eager()
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    same = int(status.item()) == 0 and all(torch.equal(outs[key][0], ref[key][0]) and
                                           torch.equal(outs[key][1], ref[key][1]) for key in ref)
    for h in handles.values():
        h.free()
    log("query phase: eager %.2f ms, graph replay %.2f ms, identical %s" % (t_eager * 1e3, t_graph * 1e3, same))
    return {"launches": len(calls), "eager_ms": round(t_eager * 1e3, 3), "graph_replay_ms": round(t_graph * 1e3, 3),
            "identical_results": same}


def plan_graph(groups, params, a, log, ref):
    """The whole batching step (the build of every tree and the k-NN launches)
    captured once into a hipGraph through build plans and replayed; each
    replay is checked by the plans (finish) and its results compared with the
    eager pass.  The plans keep their memory between replays (the eager pass
    allocates and frees its trees)."""
    import torch

    import paper_2411_09275_amd as pk
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    t0 = time.perf_counter()
    plans = {D: pk.BuildPlan(params[D][0], gr["off"], tile=params[D][1]) for D, gr in groups.items()}
    log("build plans created in %.1f s" % (time.perf_counter() - t0))
    calls = [(D, k, qk, tk) for D, gr in groups.items() for k, (idx, qk, tk) in gr["byk"].items()]
    outs = {(D, k): (torch.empty((qk.shape[1], k), dtype=torch.int64, device="cuda"),
                     torch.empty((qk.shape[1], k), dtype=torch.int64, device="cuda")) for D, k, qk, tk in calls}

    def step():
        for D, gr in groups.items():
            plans[D].enqueue(gr["c"], gr["i"], stream=side)
        for D, k, qk, tk in calls:
            plans[D].tree().knn_async(qk, k, *outs[(D, k)], status, tree_of=tk, stream=side)

    with torch.cuda.stream(side):
        step()
    redone = [plans[D].finish(stream=side) for D in plans]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        status.zero_()
        step()
    reps = max(3, a.steps)
    g.replay()
    for D in plans:
        plans[D].finish()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
        redone += [plans[D].finish() for D in plans]
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    same = int(status.item()) == 0 and not any(redone) and all(
        torch.equal(outs[key][0], ref[key][0]) and torch.equal(outs[key][1], ref[key][1]) for key in ref)
    for pl in plans.values():
        pl.free()
    log("build + queries replayed from one graph: %.2f ms per step, redone %d of %d, identical %s" % (
        t_graph * 1e3, sum(redone), len(redone), same))
    return {"graph_replay_ms": round(t_graph * 1e3, 3), "builds_redone": int(sum(redone)),
            "builds": len(redone), "identical_results": same}


def bench_serving(a):
    """A resident tree of 1e9 hashed-uniform 2-D points answers a Poisson stream
    of BatchInsert / BatchDelete / k-NN requests (1:1:8; update sizes
    log-uniform in [1e3, 1e7], query batches in [1e2, 1e6], k in {1, 10, 100}).
    Passes over the same stream, each on a freshly built tree: serial and
    continuous with every request waiting at time 0 (throughput), then, for
    each offered load, serial and continuous with Poisson arrivals at that
    fraction of the serial capacity (p50 / p99 latency).  Every pass must give
    identical results."""
    import torch
    import xxhash

    import paper_2411_09275_amd as pk
    from paper_2411_09275_amd.serve import Request, Server, latency_stats
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    D, n0, point_seed = 2, a.serve_n, 21
    t0 = time.perf_counter()
    raw = synth.request_stream(D, a.requests, seed=22, rate_hz=1.0, n_initial=n0, point_seed=point_seed)
    kinds = [r["kind"] for r in raw]
    log("stream: %d requests (%d insert, %d delete, %d k-NN) generated in %.1f s" % (
        len(raw), kinds.count("insert"), kinds.count("delete"), kinds.count("knn"), time.perf_counter() - t0))

    build_s = []

    def fresh():
        ids = torch.arange(n0, device=dev, dtype=torch.int64)
        c = synth.hashed_points_torch(ids, D, point_seed)
        torch.cuda.synchronize()
        s = time.perf_counter()
        t = pk.Tree(pk.Params(D), c, ids)
        build_s.append(time.perf_counter() - s)
        del c, ids
        torch.cuda.empty_cache()
        return t

    def one_pass(mode, realtime, rate):
        reqs = [Request.from_dict(dict(r, arrival=r["arrival"] / rate)) for r in raw]
        tree = fresh()
        srv = Server(tree, D)
        log("pass %s realtime=%s rate=%.2f/s" % (mode, realtime, rate))
        span = srv.run(reqs, mode=mode, realtime=realtime)
        digest = []
        for r in reqs:
            if r.kind == "knn":
                h = xxhash.xxh3_64()
                h.update(np.ascontiguousarray(r.result[0]).data)
                h.update(np.ascontiguousarray(r.result[1]).data)
                digest.append(h.intdigest())
                r.result = None
            elif r.kind == "delete":
                digest.append(int(r.result))
        size = tree.size()
        tree.free()
        digest.append(size)
        if not realtime:
            for r in reqs:
                r.arrival = 0.0
        lat = latency_stats(reqs)
        busy = {kd: sum(r.done - r.start for r in reqs if r.kind == kd) for kd in ("insert", "delete", "knn")}
        log("  makespan %.3f s, p50 %.2f ms, p99 %.2f ms, %d batches / %d launches; sum of per-request start-to-done s: %s" % (
            span, lat["p50_ms"], lat["p99_ms"], srv.batches, srv.launches,
            ", ".join("%s %.3f" % kv for kv in busy.items())))
        return span, lat, digest, srv.batches

    for _ in range(a.warmup):
        one_pass("continuous", False, 1.0)
    span_sc, _, dig_sc, _ = one_pass("serial", False, 1.0)
    span_cc, lat_cc, dig_cc, nb_cc = one_pass("continuous", False, 1.0)
    same = dig_sc == dig_cc
    opened = []
    for load in [float(x) for x in a.loads.split(",")]:
        rate = load * len(raw) / span_sc
        span_sr, lat_sr, dig_sr, _ = one_pass("serial", True, rate)
        span_cr, lat_cr, dig_cr, nb_cr = one_pass("continuous", True, rate)
        same = same and dig_sr == dig_sc and dig_cr == dig_sc
        opened.append({"load_vs_serial_capacity": load, "rate_per_s": round(rate, 3),
                       "serial": lat_sr, "continuous": lat_cr, "continuous_batches": nb_cr,
                       "serial_makespan_s": round(span_sr, 4), "continuous_makespan_s": round(span_cr, 4)})
    n_upd = sum(r["coords"].shape[1] for r in raw if r["kind"] != "knn")
    n_q = sum(r["coords"].shape[1] for r in raw if r["kind"] == "knn")
    out = {
        "metric": "serving throughput, continuous batching: requests/s (1:1:8 insert/delete/k-NN mix)",
        "value": round(len(raw) / span_cc, 2),
        "unit": "req/s",
        "n_gpus": 1, "steps": 1, "warmup": a.warmup,
        "ms_per_step": round(span_cc * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "resident tree of %.0e 2-D points (hashed uniform int64 in [0,1e9)); %d Poisson "
                               "requests insert:delete:k-NN 1:1:8, updates log-uniform [1e3,1e7], queries "
                               "log-uniform [1e2,1e6], k in {1,10,100}" % (n0, len(raw)),
                   "update_points": n_upd, "queries": n_q},
        "build_ms": round(min(build_s) * 1e3, 1),
        "closed": {"serial_s": round(span_sc, 4), "continuous_s": round(span_cc, 4),
                   "speedup": round(span_sc / span_cc, 3), "continuous_batches": nb_cc,
                   "items_per_s": round((n_upd + n_q) / span_cc, 1)},
        "open": opened,
        "identical_results": same,
    }
    print(json.dumps(out))


def bench_updates(a):
    """Clustered 3-D points (1e8, 1000 random-walk clusters with step lengths
    log-uniform in [1, 1e6]), then BatchInsert of 1e6 fresh points from the same
    walks, 10-NN of 1e6 in-distribution queries, BatchDelete of 1e6 existing
    ids drawn uniformly, 10-NN again.  alpha = 0.3.  One step = build + the four
    operations + free; the value is the update throughput (inserted plus
    deleted points per second of update time)."""
    import torch

    import paper_2411_09275_amd as pk
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    n, D, nb, nq = a.n, 3, a.batch, a.queries
    t0 = time.perf_counter()
    c, i, state = synth.clustered_points(n, D, seed=31)
    ci, ii, _ = synth.clustered_points(nb, D, seed=32, id_base=n, continue_from=state)
    q, _, _ = synth.clustered_points(nq, D, seed=33, continue_from=state)
    di = synth.sample_existing(i, nb, seed=34)
    dc = np.ascontiguousarray(c[:, di])
    log("clustered workload generated in %.1f s" % (time.perf_counter() - t0))
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    c, i, ci, ii, q, dc, di = (dev(x) for x in (c, i, ci, ii, q, dc, di))
    p = pk.Params(D)
    times = {"build": [], "insert": [], "knn_after_insert": [], "delete": [], "knn_after_delete": []}
    removed = None
    res = None

    def timed(key, fn):
        torch.cuda.synchronize()
        s = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        times[key].append(time.perf_counter() - s)
        return r

    for step in range(a.warmup + a.steps):
        t = timed("build", lambda: pk.Tree(p, c, i, tile=a.tile))
        timed("insert", lambda: t.insert(ci, ii))
        r1 = timed("knn_after_insert", lambda: t.knn(q, 10))
        removed = timed("delete", lambda: t.delete(dc, di))
        r2 = timed("knn_after_delete", lambda: t.knn(q, 10))
        h = t.height()
        size = t.size()
        t.free()
        cur = (r1[0].sum().item(), r1[1].sum().item(), r2[0].sum().item(), r2[1].sum().item(), removed, size, h)
        assert res is None or res == cur, "results differ between steps"
        res = cur
        if step < a.warmup:
            for v in times.values():
                v.clear()
        log("step %d: %s" % (step, ", ".join("%s %.1f ms" % (k, v[-1] * 1e3) for k, v in times.items() if v)))
    ms = {k: float(np.mean(v) * 1e3) for k, v in times.items()}
    upd_s = (ms["insert"] + ms["delete"]) / 1e3
    out = {
        "metric": "batch updates on clustered 1e8 3-D: Mpts/s of BatchInsert + BatchDelete",
        "value": round(2 * nb / upd_s / 1e6, 2),
        "unit": "Mpts/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(sum(ms.values()), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "%.0e clustered 3-D int64 points (1000 random-walk clusters, steps log-uniform "
                               "[1,1e6]) in [0,1e9); insert %.0e fresh clustered points, delete %.0e uniform ids, "
                               "%.0e in-distribution 10-NN after each batch; alpha 0.3" % (n, nb, nb, nq)},
        "ms": {k: round(v, 3) for k, v in ms.items()},
        "insert_mpts_s": round(nb / ms["insert"] / 1e3, 2),
        "delete_mpts_s": round(nb / ms["delete"] / 1e3, 2),
        "knn_mq_s": round(nq / ms["knn_after_delete"] / 1e3, 2),
        "points_removed": removed, "final_size": res[5], "final_height": res[6],
    }
    print(json.dumps(out))


def bench_large_updates(a):
    """Batch updates on a resident tree of --serve-n hashed-uniform 2-D points
    (1e9 by default, as in the paper's update table): for each batch size in
    1e3, 1e5, 1e6, 1e7, BatchInsert of fresh hashed points, then BatchDelete of
    the same points (the tree returns to its original set).  Reports the time of
    each; the value is the update throughput over all batches."""
    import torch

    import paper_2411_09275_amd as pk
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    D, n0 = 2, a.serve_n
    ids = torch.arange(n0, device="cuda", dtype=torch.int64)
    c = synth.hashed_points_torch(ids, D, 21)
    torch.cuda.synchronize()
    s = time.perf_counter()
    t = pk.Tree(pk.Params(D), c, ids)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - s) * 1e3
    del c, ids
    torch.cuda.empty_cache()
    sizes = (1000, 100000, 1000000, 10000000)
    rows = {}
    for rep in range(a.warmup + 1):
        for m in sizes:
            nid = torch.arange(2 * n0 + m, 2 * n0 + 2 * m, device="cuda", dtype=torch.int64)
            nc = synth.hashed_points_torch(nid, D, 99)
            torch.cuda.synchronize()
            s = time.perf_counter()
            t.insert(nc, nid)
            torch.cuda.synchronize()
            ti = time.perf_counter() - s
            s = time.perf_counter()
            k = t.delete(nc, nid)
            torch.cuda.synchronize()
            td = time.perf_counter() - s
            assert k == m and t.size() == n0, (k, t.size())
            if rep >= a.warmup:
                rows[str(m)] = {"insert_ms": round(ti * 1e3, 2), "delete_ms": round(td * 1e3, 2)}
            log("batch %d: insert %.1f ms, delete %.1f ms" % (m, ti * 1e3, td * 1e3))
    t.free()
    total_s = sum(r["insert_ms"] + r["delete_ms"] for r in rows.values()) / 1e3
    out = {
        "metric": "batch updates on a resident %.0e-point 2-D tree: Mpts/s of BatchInsert + BatchDelete" % n0,
        "value": round(2 * sum(sizes) / total_s / 1e6, 2),
        "unit": "Mpts/s",
        "n_gpus": 1, "steps": 1, "warmup": a.warmup,
        "ms_per_step": round(total_s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "resident tree of %.0e hashed uniform 2-D int64 points in [0,1e9); insert then "
                               "delete batches of 1e3, 1e5, 1e6, 1e7 fresh points" % n0},
        "build_ms": round(build_ms, 1),
        "batches": rows,
    }
    print(json.dumps(out))


def bench_range_report(a):
    """Range report on the 1e8 uniform 3-D tree (seed 3): 1e4 cubes whose
    outputs are log-uniform in [1e4, 1e6] points (seed 6), all in one call,
    into a preallocated id buffer.  The tree is built once; a step is one
    report call.  The roofline is that of the report phase (walk + copy):
    16 bytes per reported id (read from the tree's point array, written to
    the output) over its duration, from HIP events on the launch stream."""
    import torch

    import paper_2411_09275_amd as pk
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    nb = 10_000
    coords, ids = synth.uniform_points(a.n, a.dim, seed=3)
    lo, hi = synth.report_boxes(nb, a.dim, a.n, seed=6)
    t = pk.Tree(pk.Params(a.dim), torch.from_numpy(coords).to(dev), torch.from_numpy(ids).to(dev), tile=a.tile)
    glo, ghi = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    _, total = t.range_report_size(glo, ghi)
    buf = torch.empty(total, dtype=torch.int64, device=dev)
    log("range report workload: %d boxes, %d ids (%.1f GB of ids)" % (nb, total, total * 8 / 1e9))
    for _ in range(a.warmup):
        t.range_report(glo, ghi, out=buf)
    torch.cuda.synchronize()
    pk.profile_enable(True)
    times, sums = [], set()
    for k in range(a.steps):
        s0 = time.perf_counter()
        o, r = t.range_report(glo, ghi, out=buf)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - s0)
        sums.add(int(r.sum()))
        log("step %d: %.2f ms" % (k, times[-1] * 1e3))
    rn, rms, rbytes = pk.profile_get("range_report")
    pk.profile_enable(False)
    ms = float(np.mean(times) * 1e3)
    gbs = rbytes / (rms * 1e-3) / 1e9 if rms > 0 else 0.0
    out = {
        "metric": "range report: reported ids/s (1e4 boxes, outputs log-uniform [1e4,1e6], 1e8 pts 3D)",
        "value": round(total / (ms * 1e-3) / 1e6, 2),
        "unit": "M ids/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "tree of %.0e uniform %d-D int64 points in [0,1e9); %d cubes with outputs log-uniform "
                               "in [1e4,1e6] points, one call" % (a.n, a.dim, nb), "ids": total},
        "identical_results": len(sums) == 1,
        "roofline": {"kernel": "k_report_walk + k_report_copy", "bound": "hbm", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "launches": rn, "alg_bytes_per_launch": round(rbytes / max(rn, 1))},
    }
    t.free()
    if not a.no_cpu_baseline:
        import oracle
        n2 = 10_000_000
        c2, i2 = np.ascontiguousarray(coords[:, :n2]), ids[:n2]
        T2 = oracle.Tree(oracle.Params(a.dim), c2, i2)
        l2, h2 = synth.report_boxes(100, a.dim, n2, seed=7)
        s0 = time.perf_counter()
        o2, r2 = T2.range_report(l2, h2)
        sec = time.perf_counter() - s0
        out["cpu_baseline"] = {"value": round(r2.shape[0] / sec / 1e6, 3), "unit": "M ids/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "sequential oracle report of 100 boxes (same output law) on a tree of the "
                                         "first 1e7 points: %d ids in %.2f s" % (r2.shape[0], sec)}
    print(json.dumps(out))


def _stream_type(kind, n, dim):
    """TYPE I: clustered points in cluster order (1000 random-walk clusters,
    dense regions arrive one after another); TYPE II: a tenth uniform, then
    clustered points."""
    import synth
    if kind == "I":
        c, i, _ = synth.clustered_points(n, dim, seed=51)
        return c, i
    u, _ = synth.uniform_points(n // 10, dim, seed=52)
    c, _, _ = synth.clustered_points(n - n // 10, dim, seed=53)
    return np.ascontiguousarray(np.concatenate([u, c], axis=1)), np.arange(n, dtype=np.int64)


def bench_alpha_sweep(a):
    """Section 6.5 / Appendix G on one GPU: a 3-D stream of --n points (TYPE I
    and TYPE II) cut into --batches batches and inserted into an empty tree,
    for each alpha; after every batch 1-NN of 1e6 uniform queries.  Reported
    per alpha: incremental insertion time over the time of one Build of all
    points, rebuild volume (points in rebuilt subtrees, summed) over the final
    size, final height, and the 1-NN times over those on a fresh Build of the
    same points (checked every tenth of the stream: geometric mean and
    maximum).  The value is the TYPE I insertion throughput at alpha = 0.3."""
    import torch

    import paper_2411_09275_amd as pk
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    D, n, B = 3, a.n, a.batches
    alphas = [tuple(int(v) for v in x.split("/")) for x in a.alphas.split(",")]
    q = torch.from_numpy(synth.uniform_queries(1_000_000, D, seed=54)).to(dev)
    step = n // B
    checks = set(range(B // 10 - 1, B, max(1, B // 10)))
    res = {}
    value = None
    for kind in ("I", "II"):
        c, i = _stream_type(kind, n, D)
        gc, gi = torch.from_numpy(c).to(dev), torch.from_numpy(i).to(dev)
        del c, i
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        t = pk.Tree(pk.Params(D), gc, gi)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - s0
        t.free()
        res[kind] = {"build_s": round(build_s, 4)}
        for al in alphas:
            p = pk.Params(D, alpha=al)
            t = pk.Tree(p, gc[:, :0], gi[:0])
            ins, vol, ratios, capacity = 0.0, 0, [], None
            for b in range(B):
                torch.cuda.synchronize()
                s0 = time.perf_counter()
                t.insert(gc[:, b * step:(b + 1) * step], gi[b * step:(b + 1) * step])
                torch.cuda.synchronize()
                ins += time.perf_counter() - s0
                vol += t.update_stats()[1]
                try:
                    s0 = time.perf_counter()
                    t.knn(q, 1)
                    torch.cuda.synchronize()
                    tq = time.perf_counter() - s0
                except pk.PkdError as e:
                    if e.code != -6:
                        raise
                    capacity = capacity if capacity is not None else b   # deeper than the traversal stack
                    continue
                if b in checks:
                    log("TYPE %s alpha %d/%d: batch %d of %d, insertion %.2f s" % (kind, al[0], al[1], b + 1, B, ins))
                    f = pk.Tree(pk.Params(D), gc[:, :(b + 1) * step], gi[:(b + 1) * step])
                    f.knn(q, 1)   # warm
                    torch.cuda.synchronize()
                    s0 = time.perf_counter()
                    f.knn(q, 1)
                    torch.cuda.synchronize()
                    ratios.append(tq / (time.perf_counter() - s0))
                    f.free()
            row = {"insert_over_build": round(ins / build_s, 3), "insert_s": round(ins, 4),
                   "rebuild_volume_over_n": round(vol / (step * B), 3), "height": t.height(),
                   "knn1_over_fresh_geomean": round(float(np.exp(np.mean(np.log(ratios)))), 3) if ratios else None,
                   "knn1_over_fresh_max": round(float(max(ratios)), 3) if ratios else None,
                   "knn1_stack_exceeded_from_batch": capacity}
            res[kind]["%d/%d" % al] = row
            log("TYPE %s alpha %d/%d: %s" % (kind, al[0], al[1], row))
            if kind == "I" and al == (3, 10):
                value = step * B / ins / 1e6
            t.free()
        del gc, gi
        torch.cuda.empty_cache()
    out = {"metric": "incremental insertion of a %.0e-point stream in %d batches: Mpts/s at alpha 0.3 (TYPE I)"
                     % (n, B),
           "value": round(value, 2) if value is not None else None, "unit": "Mpts/s",
           "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "3-D int64 stream of %.0e points cut into %d batches, inserted into an empty tree; "
                                  "TYPE I clustered in cluster order, TYPE II a uniform tenth then clustered; 1-NN "
                                  "of 1e6 uniform queries after each batch" % (n, B),
                      "alphas": a.alphas},
           "results": res}
    print(json.dumps(out))


def bench_sliding_window(a):
    """Section 6.2 on synthetic data: --years batches of clustered 2-D points
    (the walks continue from year to year, 1e6 points per year by default
    through --n / --years); the tree holds the last --window years: each step
    inserts the newest year and deletes the oldest, then answers 1e6 10-NN of
    in-distribution queries.  The value is the update throughput."""
    import torch

    import paper_2411_09275_amd as pk
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    D, Y, W = 2, a.years, a.window
    per = a.n // Y
    state = None
    years = []
    for y in range(Y):
        c, i, state = synth.clustered_points(per, D, seed=60 + y, continue_from=state, id_base=y * per)
        years.append((torch.from_numpy(c).to(dev), torch.from_numpy(i).to(dev)))
    q, _, _ = synth.clustered_points(1_000_000, D, seed=59, continue_from=state)
    q = torch.from_numpy(q).to(dev)
    t = pk.Tree(pk.Params(D), *years[0])
    upd, qry, steps = 0.0, 0.0, 0
    for y in range(1, Y):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        t.insert(*years[y])
        if y >= W:
            assert t.delete(*years[y - W]) == per
        torch.cuda.synchronize()
        du = time.perf_counter() - s0
        s0 = time.perf_counter()
        t.knn(q, 10)
        torch.cuda.synchronize()
        dq = time.perf_counter() - s0
        if y >= W:
            upd += du
            qry += dq
            steps += 1
        log("year %d: size %d, update %.1f ms, 10-NN %.1f ms" % (y, t.size(), du * 1e3, dq * 1e3))
    out = {"metric": "sliding window over a clustered 2-D stream: Mpts/s of insert + delete",
           "value": round(2 * per * steps / upd / 1e6, 2), "unit": "Mpts/s",
           "n_gpus": 1, "steps": steps, "warmup": W - 1, "ms_per_step": round((upd + qry) / steps * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "%d years of %d clustered 2-D int64 points; window of %d years (insert the "
                                  "newest, delete the oldest); 1e6 in-distribution 10-NN per step" % (Y, per, W)},
           "update_ms_per_step": round(upd / steps * 1e3, 3), "knn_ms_per_step": round(qry / steps * 1e3, 3),
           "final_size": t.size(), "final_height": t.height()}
    t.free()
    print(json.dumps(out))


def bench_pkd_bb(a):
    """Section 6.3 on synthetic data: the Pkd-tree (cells derived from the
    splitters) against the Pkd-bb variant (stored node boxes) on the same
    trees: 1e7 points, D in {2, 3, 7}, uniform and clustered; 1e6 10-NN
    queries, 1e5 range counts and a range report of 1e3 cubes with outputs
    log-uniform in [1e3, 1e5].  Reported: milliseconds of each query kind with
    cells and with boxes (identical results required) and the time to compute
    the boxes."""
    import torch

    import paper_2411_09275_amd as pk
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n = 10_000_000
    rows = {}

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            s0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - s0)
        return best * 1e3, r

    for D in (2, 3, 7):
        for gen in ("uniform", "clustered"):
            if gen == "uniform":
                c, i = synth.uniform_points(n, D, seed=80 + D)
                q = synth.uniform_queries(1_000_000, D, seed=81)
            else:
                c, i, st = synth.clustered_points(n, D, seed=82 + D)
                q, _, _ = synth.clustered_points(1_000_000, D, seed=83, continue_from=st)
            lo, hi = synth.log_uniform_boxes(100_000, D, seed=84)
            rlo, rhi = synth.report_boxes(1000, D, n, seed=85, out_lo=1e3, out_hi=1e5)
            gq, glo, ghi, grlo, grhi = (torch.from_numpy(x).to(dev) for x in (q, lo, hi, rlo, rhi))
            t = pk.Tree(pk.Params(D), torch.from_numpy(c).to(dev), torch.from_numpy(i).to(dev))
            _, total = t.range_report_size(grlo, grhi)
            buf = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
            res = {}
            for mode in ("cells", "boxes"):
                if mode == "boxes":
                    torch.cuda.synchronize()
                    s0 = time.perf_counter()
                    t.set_bbox(True)
                    res["bbox_compute_ms"] = round((time.perf_counter() - s0) * 1e3, 3)
                kms, kr = timed(lambda: t.knn(gq, 10))
                cms, cr = timed(lambda: t.range_count(glo, ghi))
                rms, rr = timed(lambda: t.range_report(grlo, grhi, out=buf))
                res[mode] = {"knn10_ms": round(kms, 3), "range_count_ms": round(cms, 3),
                             "range_report_ms": round(rms, 3)}
                res[mode + "_digest"] = (int(kr[0].sum()), int(kr[1].sum()), int(cr.sum()),
                                         int(torch.sort(rr[1])[0].sum()))
            same = res.pop("cells_digest") == res.pop("boxes_digest")
            res["identical_results"] = same
            res["speedup"] = {k: round(res["cells"][k] / res["boxes"][k], 3) for k in res["cells"]}
            rows["D=%d %s" % (D, gen)] = res
            log("D=%d %s: %s" % (D, gen, res))
            t.free()
            del buf
            torch.cuda.empty_cache()
    out = {"metric": "Pkd-bb (stored node boxes) against Pkd (derived cells): query time ratios, 1e7 points",
           "value": rows["D=7 uniform"]["speedup"]["range_report_ms"], "unit": "x (range report, D=7 uniform)",
           "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "1e7 int64 points, D in {2,3,7}, uniform and clustered; 1e6 10-NN, 1e5 range "
                                  "counts, 1e3 range reports with outputs log-uniform [1e3,1e5]; best of 3"},
           "results": rows}
    print(json.dumps(out))


def bench_ablation(a):
    """Section 6.4 on one GPU: Build of 1e8 3-D points (uniform and clustered)
    three ways: the sieve with sampling and lambda = 6 (the method), the sieve
    with sampling one level at a time (lambda = 1, sample 2048), and one level
    at a time at exact medians without sampling.  All hand subproblems below
    2048 points to the same finisher.  Reported: build milliseconds (mean of
    --steps after --warmup) and the ratios."""
    import torch

    import paper_2411_09275_amd as pk
    import synth

    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n, D = a.n, 3
    variants = {"lambda6_sampling": dict(lam=6, sigma=32), "lambda1_sampling": dict(lam=1, sigma=1024),
                "lambda1_exact_median": dict(lam=1, sigma=0)}
    res = {}
    for gen in ("uniform", "clustered"):
        if gen == "uniform":
            c, i = synth.uniform_points(n, D, seed=3)
        else:
            c, i, _ = synth.clustered_points(n, D, seed=31)
        gc, gi = torch.from_numpy(c).to(dev), torch.from_numpy(i).to(dev)
        del c, i
        row = {}
        for name, kw in variants.items():
            p = pk.Params(D, **kw)
            times = []
            for s in range(a.warmup + a.steps):
                torch.cuda.synchronize()
                s0 = time.perf_counter()
                t = pk.Tree(p, gc, gi)
                torch.cuda.synchronize()
                if s >= a.warmup:
                    times.append(time.perf_counter() - s0)
                h = t.height()
                t.free()
            row[name] = {"build_ms": round(float(np.mean(times)) * 1e3, 3), "height": h}
            log("%s %s: %s" % (gen, name, row[name]))
        row["lambda1_over_lambda6"] = round(row["lambda1_sampling"]["build_ms"] / row["lambda6_sampling"]["build_ms"], 3)
        row["exact_over_sampling"] = round(row["lambda1_exact_median"]["build_ms"] / row["lambda1_sampling"]["build_ms"], 3)
        res[gen] = row
        del gc, gi
        torch.cuda.empty_cache()
    out = {"metric": "technique ablation of Build (1e8 3-D): time of lambda=1 over lambda=6, exact medians over sampling",
           "value": res["uniform"]["lambda1_over_lambda6"], "unit": "x (lambda=1 / lambda=6, uniform)",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "Build of %.0e 3-D int64 points (uniform seed 3; clustered seed 31) with lambda 6 "
                                  "and sampling, lambda 1 and sampling (sample 2048), lambda 1 at exact medians" % n},
           "results": res}
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.workload == "batching":
        bench_batching(a)
        return
    if a.workload == "large_updates":
        bench_large_updates(a)
        return
    if a.workload == "range_report":
        bench_range_report(a)
        return
    if a.workload == "alpha_sweep":
        bench_alpha_sweep(a)
        return
    if a.workload == "pkd_bb":
        bench_pkd_bb(a)
        return
    if a.workload == "ablation":
        bench_ablation(a)
        return
    if a.workload == "sliding_window":
        bench_sliding_window(a)
        return
    if a.workload == "serving":
        bench_serving(a)
        return
    if a.workload == "updates":
        if a.queries == 10_000_000:
            a.queries = 1_000_000
        bench_updates(a)
        return
    import torch

    import paper_2411_09275_amd as pk
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if a.copy_calibration:
        # a plain copy of known size: reads and writes exactly 2 GiB each
        src = torch.empty(1 << 28, dtype=torch.int64, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("copy calibration: %d bytes read, %d bytes written" % (src.numel() * 8, dst.numel() * 8),
              file=sys.stderr, flush=True)
        del src, dst
    copy_gbs = stream_copy_gbps(torch, dev)
    t0 = time.perf_counter()
    coords, ids = synth.uniform_points(a.n, a.dim, seed=3)
    q = synth.uniform_queries(a.queries, a.dim, seed=4)
    lo, hi = synth.log_uniform_boxes(a.boxes, a.dim, seed=5)
    gc = torch.from_numpy(coords).to(dev)
    gi = torch.from_numpy(ids).to(dev)
    gq = torch.from_numpy(q).to(dev)
    glo = torch.from_numpy(lo).to(dev)
    ghi = torch.from_numpy(hi).to(dev)
    torch.cuda.synchronize()
    print("inputs ready in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    params = pk.Params(a.dim)

    def step(rec):
        s = torch.cuda.current_stream()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(s)
        t = pk.Tree(params, gc, gi, tile=a.tile)
        e[1].record(s)
        t.knn(gq, a.k)
        e[2].record(s)
        t.range_count(glo, ghi)
        e[3].record(s)
        t.free()
        if rec is not None:
            e[3].synchronize()
            rec.append((e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])))

    for w in range(a.warmup):
        step(None)
        print("warmup %d done" % w, file=sys.stderr, flush=True)
    pk.profile_enable(True)
    rec = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(a.steps):
        step(rec)
        print("step %d: build %.2f ms, %d-NN %.2f ms, range %.2f ms" % (k, rec[-1][0], a.k, rec[-1][1], rec[-1][2]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    rec = np.array(rec)
    build_ms, knn_ms, range_ms = rec[:, 0].mean(), rec[:, 1].mean(), rec[:, 2].mean()
    sc_n, sc_ms, sc_bytes = pk.profile_get("sieve_scatter")
    ct_n, ct_ms, ct_bytes = pk.profile_get("sieve_count")
    sel_n, sel_ms, _ = pk.profile_get("select_skeleton")
    fin_n, fin_ms, _ = pk.profile_get("finisher")
    kn_n, kn_ms, _ = pk.profile_get("knn")
    pk.profile_enable(False)
    scatter_gbs = sc_bytes / (sc_ms * 1e-3) / 1e9 if sc_ms > 0 else 0.0
    sieve_gbs = (sc_bytes + ct_bytes) / ((sc_ms + ct_ms) * 1e-3) / 1e9 if sc_ms + ct_ms > 0 else 0.0
    # the committed counters cover the default workload only
    measured = a.n == 100_000_000 and a.dim == 3 and a.tile == 2048 and params.lam == 6
    traffic = load_traffic("sieve_scatter") if measured else None
    out = {
        "metric": "build Mpts/s + sieve HBM GB/s (% peak); 10-NN queries/s; 1e8 pts 3D",
        "value": round(a.n / (build_ms * 1e-3) / 1e6, 2),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall * 1e3 / a.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "build %.0e uniform %d-D int64 points in [0,1e9) + %.0e uniform %d-NN queries + "
                               "%.0e range counts (sides log-uniform [1e5,1e8])" % (a.n, a.dim, a.queries, a.k, a.boxes),
                   "n": a.n, "dim": a.dim, "queries": a.queries, "k": a.k, "boxes": a.boxes,
                   "lambda": params.lam, "phi": params.phi, "sigma": params.sigma, "tile": a.tile},
        "build_ms": round(build_ms, 3),
        "build_ms_median": round(float(np.median(rec[:, 0])), 3),
        "knn_qps": round(a.queries / (knn_ms * 1e-3), 1),
        "knn_ms": round(knn_ms, 3),
        "range_qps": round(a.boxes / (range_ms * 1e-3), 1),
        "range_ms": round(range_ms, 3),
        "sieve_gbps": round(sieve_gbs, 1),
        "sieve_frac_peak": round(sieve_gbs / HBM_PEAK_GBS, 4),
        "stream_copy_gbps": round(copy_gbs, 1),
        "sieve_frac_of_copy": round(sieve_gbs / copy_gbs, 4) if copy_gbs > 0 else None,
        "kernel_ms_per_step": {"sieve_count": round(ct_ms / a.steps, 3), "sieve_scatter": round(sc_ms / a.steps, 3),
                               "select_skeleton": round(sel_ms / a.steps, 3), "finisher": round(fin_ms / a.steps, 3)},
        "roofline": {"kernel": "k_scatter (sieve scatter)", "bound": "hbm", "achieved": round(scatter_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(scatter_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "launches": sc_n, "alg_bytes_per_launch": round(sc_bytes / max(sc_n, 1))},
    }
    # k-NN: algorithmic bytes from the search work of the oracle on the same
    # tree (live with the CPU baseline, else the committed count)
    work = None
    if not a.no_cpu_baseline:
        print("timing the CPU oracle ...", file=sys.stderr, flush=True)
        out["cpu_baseline"], work = cpu_baseline(coords, ids, q, a.dim, a.k, a.cpu_sample)
    else:
        out["cpu_baseline"] = None
        work = stored_knn_work(a.n, a.dim, a.k)
    if work is not None and kn_ms > 0:
        per_q = knn_bytes_per_query(work, a.dim, a.k)
        kn_gbs = per_q * a.queries / (kn_ms / kn_n * 1e-3) / 1e9
        out["roofline_knn"] = {"kernel": "k_knn (%d-NN, one lane per query)" % a.k, "bound": "hbm",
                               "achieved": round(kn_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(kn_gbs / HBM_PEAK_GBS, 4),
                               "traffic": load_traffic("knn") if measured and a.k == 10 and a.queries == 10 ** 7 else None,
                               "launches": kn_n, "alg_bytes_per_launch": round(per_q * a.queries),
                               "work_per_query": work}
    print(json.dumps(out))


def stream_copy_gbps(torch, dev, nbytes=2 << 30, reps=5):
    """Device-to-device copy of nbytes (read nbytes, write nbytes), timed
    with events on the current stream: the practical HBM rate of a plain
    streaming kernel on this GPU, beside the nominal peak."""
    src = torch.empty(nbytes // 8, dtype=torch.int64, device=dev).fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(reps):
        e0.record(s)
        dst.copy_(src)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (best * 1e-3) / 1e9


if __name__ == "__main__":
    main()
