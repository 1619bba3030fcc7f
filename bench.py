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
    ap.add_argument("--cpu-sample", type=int, default=4_000_000, help="points of the oracle's build sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 2 GiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


def source_hash():
    h = hashlib.sha256()
    for f in ("build.hip", "pkd_internal.h"):
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
    if t.get("source_hash") != source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


def cpu_baseline(coords, ids, q, lo, hi, sample_n, dim):
    import oracle
    n = min(sample_n, ids.shape[0])
    c = np.ascontiguousarray(coords[:, :n])
    i = ids[:n]
    t0 = time.perf_counter()
    T = oracle.Tree(oracle.Params(dim), c, i)
    t_build = time.perf_counter() - t0
    nq = min(100_000, q.shape[1])
    t0 = time.perf_counter()
    T.knn(np.ascontiguousarray(q[:, :nq]), 10)
    t_knn = time.perf_counter() - t0
    return {
        "value": round(n / t_build / 1e6, 3),
        "unit": "Mpts/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "sequential oracle build of the first %d of the %d points (%.1f s); "
                  "oracle tree 10-NN of %d of the queries: %.0f q/s" % (n, ids.shape[0], t_build, nq, nq / t_knn),
        "knn_qps": round(nq / t_knn, 1),
    }


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
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
        print("step %d: build %.2f ms, 10-NN %.2f ms, range %.2f ms" % ((k,) + rec[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    rec = np.array(rec)
    build_ms, knn_ms, range_ms = rec[:, 0].mean(), rec[:, 1].mean(), rec[:, 2].mean()
    sc_n, sc_ms, sc_bytes = pk.profile_get("sieve_scatter")
    ct_n, ct_ms, ct_bytes = pk.profile_get("sieve_count")
    sel_n, sel_ms, _ = pk.profile_get("select_skeleton")
    fin_n, fin_ms, _ = pk.profile_get("finisher")
    pk.profile_enable(False)
    scatter_gbs = sc_bytes / (sc_ms * 1e-3) / 1e9 if sc_ms > 0 else 0.0
    sieve_gbs = (sc_bytes + ct_bytes) / ((sc_ms + ct_ms) * 1e-3) / 1e9 if sc_ms + ct_ms > 0 else 0.0
    traffic = load_traffic("sieve_scatter")
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
        "config": {"workload": "build %.0e uniform %d-D int64 points in [0,1e9) + %.0e uniform 10-NN queries + "
                               "%.0e range counts (sides log-uniform [1e5,1e8])" % (a.n, a.dim, a.queries, a.boxes),
                   "n": a.n, "dim": a.dim, "queries": a.queries, "k": a.k, "boxes": a.boxes,
                   "lambda": params.lam, "phi": params.phi, "sigma": params.sigma, "tile": a.tile},
        "build_ms": round(build_ms, 3),
        "knn_qps": round(a.queries / (knn_ms * 1e-3), 1),
        "knn_ms": round(knn_ms, 3),
        "range_qps": round(a.boxes / (range_ms * 1e-3), 1),
        "range_ms": round(range_ms, 3),
        "sieve_gbps": round(sieve_gbs, 1),
        "sieve_frac_peak": round(sieve_gbs / HBM_PEAK_GBS, 4),
        "kernel_ms_per_step": {"sieve_count": round(ct_ms / a.steps, 3), "sieve_scatter": round(sc_ms / a.steps, 3),
                               "select_skeleton": round(sel_ms / a.steps, 3), "finisher": round(fin_ms / a.steps, 3)},
        "roofline": {"kernel": "k_scatter (sieve scatter)", "bound": "hbm", "achieved": round(scatter_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(scatter_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "launches": sc_n, "alg_bytes_per_launch": round(sc_bytes / max(sc_n, 1))},
    }
    if not a.no_cpu_baseline:
        print("timing the CPU oracle on a sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(coords, ids, q, lo, hi, a.cpu_sample, a.dim)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
