"""Per-query work of k-NN on the benchmark's tree, from the oracle (the counts
Appendix H reports): the oracle builds the tree of the default benchmark
workload (1e8 uniform 3-D points, seed 3; default parameters), which equals
the GPU library's tree node for node, and runs the search of Section 5 for a
uniform sample of its 10-NN queries (seed 4), counting the nodes read, the
leaves scanned and the points scanned.  The result goes to
profiles/knn_work_1e8_3d.json; the benchmark turns it into the algorithmic
bytes of its k-NN launch.  Test infrastructure: it calls only oracle/ and the
input generators.

    python oracle/knn_work.py [--n 100000000] [--sample 20000]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--queries", type=int, default=10_000_000)
    ap.add_argument("--k", type=int, nargs="+", default=[1, 10, 100])
    ap.add_argument("--sample", type=int, default=20000)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "knn_work_1e8_3d.json"))
    a = ap.parse_args()
    t0 = time.perf_counter()
    c, i = synth.uniform_points(a.n, a.dim, seed=3)
    q = synth.uniform_queries(a.queries, a.dim, seed=4)
    rows = np.sort(np.random.default_rng(77).choice(a.queries, size=a.sample, replace=False))
    qs = np.ascontiguousarray(q[:, rows])
    del q
    T = oracle.Tree(oracle.Params(a.dim), c, i)
    del c, i
    print("oracle tree built in %.1f s" % (time.perf_counter() - t0), flush=True)
    out = {"workload": "%d uniform %d-D points (seed 3), default parameters; %d of the %d uniform queries "
                       "(seed 4, rows drawn with seed 77)" % (a.n, a.dim, a.sample, a.queries),
           "tree_nodes": T.num_nodes(), "tree_height": T.height(), "per_query": {}}
    for k in a.k:
        nodes, leaves, points = T.knn_visits(qs, k)
        out["per_query"][str(k)] = {"nodes": float(nodes.mean()), "leaves": float(leaves.mean()),
                                    "points": float(points.mean()), "points_max": int(points.max())}
        print(k, out["per_query"][str(k)], flush=True)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
