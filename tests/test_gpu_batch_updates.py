"""Updates on the trees of a batch handle: after every insert or delete on
one tree, every tree of the handle equals the oracle's tree of its own points
(the updated one as BatchInsert / BatchDelete make it, the others unchanged),
and queries routed by tree index equal the plain definitions."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _check_all(bt, trees, pts, label, orc, D):
    for t, ot in enumerate(trees):
        for a, b in zip(bt.export(t), ot.export()):
            assert np.array_equal(a, b), (label, t)
    q = synth.uniform_queries(600, D, seed=801)
    tree_of = (np.arange(600) % len(trees)).astype(np.int32)
    gi, gd = bt.knn(q, 5, tree_of=tree_of)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    for t, (c, i) in enumerate(pts):
        mine = np.nonzero(tree_of == t)[0]
        bi, bd = orc.brute_knn(c, i, np.ascontiguousarray(q[:, mine]), 5)
        assert np.array_equal(gi[mine], bi) and np.array_equal(gd[mine], bd), (label, t)


# events: how an update places the old points (0: by the batch's density,
# 1: sorted event lists, 2: per-point arrays); the trees are the same
@pytest.mark.parametrize("bbox,events", [(False, 0), (True, 0), (False, 1), (False, 2)])
def test_updates_tree_by_tree(pk, orc, bbox, events):
    D = 3
    sizes = [0, 5000, 30000, 200, 80000]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    c, i = synth.uniform_points(int(off[-1]), D, seed=800)
    bt = pk.Tree.batch(pk.Params(D), c, i, off, update_events=events)
    if bbox:
        bt.set_bbox(True)
    op = orc.Params(D)
    pts = [(np.ascontiguousarray(c[:, off[t]:off[t + 1]]), i[off[t]:off[t + 1]]) for t in range(len(sizes))]
    trees = [orc.Tree(op, pc, pi) for pc, pi in pts]
    _check_all(bt, trees, pts, "built", orc, D)
    nid = 10 ** 8
    steps = [("ins", 0, 4000), ("ins", 2, 9000), ("del", 4, 20000), ("ins", 3, 300), ("del", 1, None),
             ("ins", 1, 2500), ("del", 2, 15000), ("ins", 4, 50000), ("del", 0, 1000)]
    for k, (kind, t, m) in enumerate(steps):
        pc, pi = pts[t]
        if kind == "ins":
            nc, ni = synth.uniform_points(m, D, seed=810 + k, id_base=nid)
            nid += m
            bt.insert(nc, ni, tree=t)
            trees[t].insert(nc, ni)
            pts[t] = (np.ascontiguousarray(np.concatenate([pc, nc], axis=1)), np.concatenate([pi, ni]))
        else:
            sel = np.arange(pi.shape[0]) if m is None else np.sort(
                np.random.default_rng(820 + k).choice(pi.shape[0], m, replace=False))
            assert bt.delete(pc[:, sel], pi[sel], tree=t) == trees[t].delete(pc[:, sel], pi[sel]) == sel.shape[0]
            keep = np.ones(pi.shape[0], dtype=bool)
            keep[sel] = False
            pts[t] = (np.ascontiguousarray(pc[:, keep]), pi[keep])
        _check_all(bt, trees, pts, "step %d" % k, orc, D)
    assert bt.size() == sum(p[1].shape[0] for p in pts)
    bt.free()
