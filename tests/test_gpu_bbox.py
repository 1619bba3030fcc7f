"""The bounding-box variant (Pkd-bb, Section 6.3): every node's stored box is
the tight box of its points (checked against the exported tree), and queries
pruned with the boxes give exactly the results of the splitter cells, the
oracle and the plain definitions, also after updates and on batch handles."""
import numpy as np
import pytest

import synth
from tests import treecheck

pytestmark = pytest.mark.gpu


def _check_boxes(t, D):
    rows, ids, coords = t.export()
    boxes = t.export_bbox()
    start, parent, lc, rc = treecheck.parse(rows)
    for v in range(rows.shape[0]):
        a, n = start[v], rows[v, 3]
        if n == 0:
            assert np.all(boxes[v, :D] == 2 ** 31 - 1) and np.all(boxes[v, D:] == -1), v
            continue
        seg = coords[:, a:a + n]
        assert np.array_equal(boxes[v, :D], seg.min(axis=1)) and np.array_equal(boxes[v, D:], seg.max(axis=1)), v


def _queries_equal(t, orc, c, i, D, seed):
    q = synth.uniform_queries(3000, D, seed=seed)
    for k in (1, 10, 32, 100):
        gi, gd = t.knn(q, k)
        bi, bd = orc.brute_knn(c, i, q, k)
        assert np.array_equal(gi.cpu().numpy(), bi) and np.array_equal(gd.cpu().numpy(), bd), k
    lo, hi = synth.log_uniform_boxes(400, D, seed=seed + 1, side_lo=1e6, side_hi=6e8)
    assert np.array_equal(t.range_count(lo, hi).cpu().numpy(), orc.brute_range_count(c, lo, hi))
    off, rid = t.range_report(lo, hi)
    off, rid = off.cpu().numpy(), rid.cpu().numpy()
    for j in range(0, 400, 13):
        inside = np.all((c >= lo[:, j:j + 1]) & (c <= hi[:, j:j + 1]), axis=0)
        assert np.array_equal(np.sort(rid[off[j]:off[j + 1]]), np.sort(i[inside])), j


@pytest.mark.parametrize("D,gen", [(2, "uniform"), (3, "clustered"), (7, "uniform"), (2, "dups")])
def test_boxes_are_tight_and_queries_unchanged(pk, orc, D, gen):
    n = 150000
    if gen == "uniform":
        c, i = synth.uniform_points(n, D, seed=700 + D)
    elif gen == "clustered":
        c, i, _ = synth.clustered_points(n, D, seed=701, n_clusters=50)
    else:
        c, i = synth.duplicate_heavy_points(n, D, seed=702, n_distinct=800, hot_fraction=0.2)
    t = pk.Tree(pk.Params(D), c, i)
    t.set_bbox(True)
    _check_boxes(t, D)
    _queries_equal(t, orc, c, i, D, seed=710 + D)
    t.set_bbox(False)
    _queries_equal(t, orc, c, i, D, seed=710 + D)
    t.free()


def test_boxes_follow_updates(pk, orc):
    D = 3
    c, i = synth.uniform_points(100000, D, seed=720)
    t = pk.Tree(pk.Params(D), c, i)
    t.set_bbox(True)
    cur_c, cur_i = c, i
    for step in range(6):
        nc, ni = synth.uniform_points(20000, D, seed=721 + step, id_base=10 ** 7 * (step + 1))
        t.insert(nc, ni)
        cur_c = np.concatenate([cur_c, nc], axis=1)
        cur_i = np.concatenate([cur_i, ni])
        sel = np.arange(step, cur_i.shape[0], 9)
        assert t.delete(cur_c[:, sel], cur_i[sel]) == sel.shape[0]
        keep = np.ones(cur_i.shape[0], dtype=bool)
        keep[sel] = False
        cur_c, cur_i = np.ascontiguousarray(cur_c[:, keep]), cur_i[keep]
        _check_boxes(t, D)
    _queries_equal(t, orc, cur_c, cur_i, D, seed=730)
    # everything deleted, then inserted again
    assert t.delete(cur_c, cur_i) == cur_i.shape[0]
    _check_boxes(t, D)
    t.insert(c, i)
    _check_boxes(t, D)
    t.free()


def test_boxes_on_batch_handles(pk, orc):
    D = 2
    sizes = [3000, 0, 50000, 120000]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    c, i = synth.uniform_points(int(off[-1]), D, seed=740)
    t = pk.Tree.batch(pk.Params(D), c, i, off)
    t.set_bbox(True)
    q = synth.uniform_queries(4000, D, seed=741)
    tree_of = (np.arange(4000) % 4).astype(np.int32)
    gi, gd = t.knn(q, 10, tree_of=tree_of)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    lo, hi = synth.log_uniform_boxes(4000, D, seed=742, side_lo=1e7, side_hi=6e8)
    rc = t.range_count(lo, hi, tree_of=tree_of).cpu().numpy()
    for tr in range(4):
        a, b = int(off[tr]), int(off[tr + 1])
        mine = np.nonzero(tree_of == tr)[0]
        bi, bd = orc.brute_knn(c[:, a:b], i[a:b], np.ascontiguousarray(q[:, mine]), 10)
        assert np.array_equal(gi[mine], bi) and np.array_equal(gd[mine], bd), tr
        assert np.array_equal(rc[mine], orc.brute_range_count(c[:, a:b], np.ascontiguousarray(lo[:, mine]),
                                                               np.ascontiguousarray(hi[:, mine]))), tr
    t.free()
