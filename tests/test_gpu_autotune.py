"""Trees built with autotuned parameters equal the oracle's with the same
parameters.  lambda, sigma and phi change the tree, so a caller that checks
results passes the tuner's choice to the oracle; these tests do exactly that
for a tuner run on a small batch workload (trees with sizes log-uniform in
[1e3, 1e5], D in {2, 3}, uniform points; k in {1, 10, 100}) and for the
setting the batching benchmark recorded (lambda 6, sigma 16, phi 64, tiles of
2048)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _workload(D, T, seed):
    sizes = synth.log_uniform_sizes(T, 1e3, 1e5, seed=seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    c, i = synth.uniform_points(int(off[-1]), D, seed=seed + 1)
    q = synth.uniform_queries(T * 24, D, seed=seed + 2)
    tree_of = (np.arange(T * 24) % T).astype(np.int32)
    return off, c, i, q, tree_of


def _check_trees(orc, pk, p, tile, off, c, i, q, tree_of, picks):
    import torch
    t = pk.Tree.batch(p, torch.from_numpy(c).cuda(), torch.from_numpy(i).cuda(), off, tile=tile)
    op = orc.Params(p.dim, lam=p.lam, phi=p.phi, sigma=p.sigma)
    res = {k: t.knn(torch.from_numpy(q).cuda(), k, tree_of=torch.from_numpy(tree_of).cuda()) for k in (1, 10, 100)}
    for tr in picks:
        a, b = int(off[tr]), int(off[tr + 1])
        ot = orc.Tree(op, np.ascontiguousarray(c[:, a:b]), i[a:b])
        for x, y in zip(t.export(tr), ot.export()):
            assert np.array_equal(x, y), (p.lam, p.sigma, p.phi, tile, tr)
        mine = np.nonzero(tree_of == tr)[0]
        for k, (gi, gd) in res.items():
            oi, od = ot.knn(np.ascontiguousarray(q[:, mine]), k)
            sel = torch.from_numpy(mine).cuda()
            assert np.array_equal(gi[sel].cpu().numpy(), oi), (k, tr)
            assert np.array_equal(gd[sel].cpu().numpy(), od), (k, tr)
    t.free()


@pytest.mark.parametrize("D", [2, 3])
def test_autotuned_parameters_match_oracle(orc, pk, D):
    import torch
    from paper_2411_09275_amd import autotune
    off, c, i, q, tree_of = _workload(D, 96, seed=500 + D)
    gc, gi = torch.from_numpy(c).cuda(), torch.from_numpy(i).cuda()
    mix = []
    for k in (1, 10, 100):
        sel = np.nonzero(np.arange(q.shape[1]) % 3 == (1, 10, 100).index(k))[0]
        mix.append((torch.from_numpy(np.ascontiguousarray(q[:, sel])).cuda(), k,
                    torch.from_numpy(tree_of[sel]).cuda()))
    grid = {"lam": [5, 6], "sigma": [16, 32], "phi": [32, 64], "tile": [2048, 4096]}
    p, tile, _ = autotune.tune(D, gc, gi, offsets=off, queries=mix, grid=grid, cache=None)
    _check_trees(orc, pk, p, tile, off, c, i, q, tree_of, picks=[0, 1, 17, 50, 95])


@pytest.mark.parametrize("D", [2, 3])
def test_benchmark_batching_setting_matches_oracle(orc, pk, D):
    off, c, i, q, tree_of = _workload(D, 64, seed=520 + D)
    p = pk.Params(D, lam=6, sigma=16, phi=64)
    _check_trees(orc, pk, p, 2048, off, c, i, q, tree_of, picks=list(range(0, 64, 7)))
