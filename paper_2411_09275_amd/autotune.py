"""Autotuner for the skeleton height lambda, the oversampling rate sigma, the
leaf size phi and the sieve tile size.

lambda, sigma and phi change the tree (Section 5 discusses their trade-off:
larger lambda means fewer sieve rounds, larger phi fewer nodes but longer leaf
scans); the tile size never changes any result.  The tuner times candidate
settings on a sample of the caller's workload (build plus its queries) on the
GPU and returns the fastest; every caller that checks results against the CPU
oracle must pass the chosen parameters to the oracle as well.

The choice is cached in a JSON file keyed by device name, dimension, the
decade of the sample size, whether the sample is one tree or a batch handle
(and how many trees), the query mix (k of each query set) and a hash of the
searched grid, so a stored choice is reused only for the same kind of workload.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

from . import Params, Tree

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

GRID = {
    "lam": [5, 6, 7],
    "sigma": [16, 32],
    "phi": [16, 32, 64],
    "tile": [1024, 2048, 4096],
}


def _key(dim, n_points, n_trees, ks, grid):
    import torch
    dev = torch.cuda.get_device_name(0)
    decade = len(str(max(1, int(n_points))))
    shape = "single" if n_trees is None else "batch%d" % n_trees
    g = hashlib.sha256(json.dumps({k: list(v) for k, v in sorted(grid.items())}).encode()).hexdigest()[:12]
    return "%s|D=%d|n~1e%d|%s|k=%s|grid=%s" % (dev, dim, decade - 1, shape, ",".join(str(k) for k in ks) or "-", g)


def _time(fn, reps=2):
    import torch
    fn()   # warm-up
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune(dim, coords, ids, offsets=None, queries=None, k=10, grid=None, cache=DEFAULT_CACHE, force=False,
         log=None):
    """Pick (Params, tile) for a workload sample.

    coords/ids: device or host int64 points of the sample (one tree, or many
    trees back to back with host `offsets`); queries: optional [dim, nq]
    (with offsets, query j goes to tree j % n_trees), or a list of
    (queries, k, tree_of) triples that together make the sample's query mix
    (tree_of may be None).  Returns (Params, tile, seconds of the best
    setting)."""
    import numpy as np
    import torch

    grid = grid or GRID
    n_points = int(ids.shape[0])
    if queries is None:
        ks = []
    elif isinstance(queries, (list, tuple)):
        ks = [kk for _, kk, _ in queries]
    else:
        ks = [k]
    key = _key(dim, n_points, None if offsets is None else len(offsets) - 1, ks, grid)
    if not force and cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)
        if key in stored:
            c = stored[key]
            return Params(dim, lam=c["lam"], phi=c["phi"], sigma=c["sigma"]), c["tile"], c["seconds"]
    if queries is None:
        mix = []
    elif isinstance(queries, (list, tuple)):
        mix = list(queries)
    else:
        tree_of = None
        if offsets is not None:
            nt = len(offsets) - 1
            tree_of = torch.from_numpy((np.arange(queries.shape[1]) % nt).astype(np.int32)).cuda()
        mix = [(queries, k, tree_of)]
    best = None
    for lam, sigma, phi, tile in itertools.product(grid["lam"], grid["sigma"], grid["phi"], grid["tile"]):
        if (sigma << lam) > 2048:   # the library caps the sample at 2048
            continue
        p = Params(dim, lam=lam, phi=phi, sigma=sigma)

        def run():
            t = Tree(p, coords, ids, tile=tile) if offsets is None else Tree.batch(p, coords, ids, offsets, tile=tile)
            for qq, kk, to in mix:
                t.knn(qq, kk, tree_of=to)
            t.free()

        sec = _time(run)
        if log:
            log("autotune lam=%d sigma=%d phi=%d tile=%d: %.2f ms" % (lam, sigma, phi, tile, sec * 1e3))
        if best is None or sec < best[0]:
            best = (sec, lam, sigma, phi, tile)
    sec, lam, sigma, phi, tile = best
    if cache:
        stored = {}
        if os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
        stored[key] = {"lam": lam, "sigma": sigma, "phi": phi, "tile": tile, "seconds": sec}
        with open(cache, "w") as f:
            json.dump(stored, f, indent=1)
    return Params(dim, lam=lam, phi=phi, sigma=sigma), tile, sec
