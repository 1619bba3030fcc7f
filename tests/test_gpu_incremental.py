"""Incremental and sliding-window workloads (Section 6.5 and Appendix G: a
stream cut into batches and inserted into an empty tree, for balance
parameters from almost-always-rebuild to never-rebuild; Section 6.2: a window
of the most recent batches, insert the newest and delete the oldest).  After
every batch the GPU tree equals the oracle's node for node, the rebuild volume
the library reports equals what the oracle rebuilt, and 1-NN answers equal the
plain definition."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _same(gt, ot, label):
    for a, b in zip(gt.export(), ot.export()):
        assert np.array_equal(a, b), label


def _rebuilt(ot):
    log = ot.update_log()
    return log["interior_points"] + log["leaf_points"]


def _stream(kind, n, D, seed):
    """TYPE I: clustered points in cluster order (dense regions arrive one
    after another); TYPE II: a uniform tenth first, then clustered points."""
    if kind == "I":
        c, i, _ = synth.clustered_points(n, D, seed=seed, n_clusters=30)
        return c, i
    u, _ = synth.uniform_points(n // 10, D, seed=seed)
    c, _, _ = synth.clustered_points(n - n // 10, D, seed=seed + 1, n_clusters=27)
    allc = np.ascontiguousarray(np.concatenate([u, c], axis=1))
    return allc, np.arange(n, dtype=np.int64)


@pytest.mark.parametrize("kind", ["I", "II"])
@pytest.mark.parametrize("alpha", [(1, 100), (1, 10), (3, 10), (1, 2)])
def test_incremental_inserts_follow_the_oracle(pk, orc, kind, alpha):
    D, n, nbatch = 3, 60000, 30
    c, i = _stream(kind, n, D, seed=400)
    empty_c, empty_i = np.zeros((D, 0), np.int64), np.zeros(0, np.int64)
    gt = pk.Tree(pk.Params(D, alpha=alpha), empty_c, empty_i)
    ot = orc.Tree(orc.Params(D, alpha=alpha), empty_c, empty_i)
    q = synth.uniform_queries(300, D, seed=401)
    step = n // nbatch
    total = 0
    for b in range(nbatch):
        bc, bi = np.ascontiguousarray(c[:, b * step:(b + 1) * step]), i[b * step:(b + 1) * step]
        gt.insert(bc, bi)
        ot.insert(bc, bi)
        label = "%s alpha=%s batch %d" % (kind, alpha, b)
        _same(gt, ot, label)
        regions, points = gt.update_stats()
        assert points == _rebuilt(ot), label
        total += points
        if b % 10 == 9:
            gi, gd = gt.knn(q, 1)
            bi_, bd_ = orc.brute_knn(c[:, :(b + 1) * step], i[:(b + 1) * step], q, 1)
            assert np.array_equal(gi.cpu().numpy(), bi_) and np.array_equal(gd.cpu().numpy(), bd_), label
    if alpha == (1, 2):
        # alpha = 1/2 never rebuilds for balance: only leaves that receive points
        assert gt.update_stats()[1] > 0
    gt.free()


def test_alpha_orders_the_rebuild_volume(pk):
    # a smaller alpha rebuilds more (Section 6.5): on the adversarial stream the
    # cumulative rebuild volume falls as alpha grows
    D, n, nbatch = 3, 200000, 40
    c, i = _stream("I", n, D, seed=410)
    vols = []
    for alpha in [(1, 100), (1, 10), (3, 10), (1, 2)]:
        t = pk.Tree(pk.Params(D, alpha=alpha), np.zeros((D, 0), np.int64), np.zeros(0, np.int64))
        vol = 0
        step = n // nbatch
        for b in range(nbatch):
            t.insert(np.ascontiguousarray(c[:, b * step:(b + 1) * step]), i[b * step:(b + 1) * step])
            vol += t.update_stats()[1]
        vols.append(vol)
        t.free()
    assert all(a > b for a, b in zip(vols, vols[1:])), vols


def test_sliding_window_follows_the_oracle(pk, orc):
    # "years" of clustered points (the walks continue from year to year); the
    # tree holds the last four: insert the newest year, delete the oldest
    D, per_year, years, window = 2, 6000, 12, 4
    state = None
    yc, yi = [], []
    for y in range(years):
        c, i, state = synth.clustered_points(per_year, D, seed=420 + y, n_clusters=12, continue_from=state,
                                             id_base=y * per_year)
        yc.append(c)
        yi.append(i)
    gt = pk.Tree(pk.Params(D), yc[0], yi[0])
    ot = orc.Tree(orc.Params(D), yc[0], yi[0])
    q = synth.uniform_queries(200, D, seed=430)
    for y in range(1, years):
        gt.insert(yc[y], yi[y])
        ot.insert(yc[y], yi[y])
        assert gt.update_stats()[1] == _rebuilt(ot)
        if y >= window:
            old = y - window
            assert gt.delete(yc[old], yi[old]) == ot.delete(yc[old], yi[old]) == per_year
            assert gt.update_stats()[1] == ot.update_log()["interior_points"]
        _same(gt, ot, "year %d" % y)
        lo = max(0, y - window + 1)
        cur_c = np.concatenate(yc[lo:y + 1], axis=1)
        cur_i = np.concatenate(yi[lo:y + 1])
        gi, gd = gt.knn(q, 1)
        bi, bd = orc.brute_knn(cur_c, cur_i, q, 1)
        assert np.array_equal(gi.cpu().numpy(), bi) and np.array_equal(gd.cpu().numpy(), bd), y
    gt.free()
