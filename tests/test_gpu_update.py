"""GPU parity of BatchInsert / BatchDelete: after every batch the exported GPU
tree equals the oracle's node for node, and queries equal brute force on the
current point set.  All through the C-ABI."""
import numpy as np
import pytest

import synth
from tests import treecheck

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_09275_amd as pk
    pk.lib()
    return pk


def _same(gt, ot, label):
    g = gt.export()
    o = ot.export()
    assert g[0].shape == o[0].shape, (label, g[0].shape, o[0].shape)
    rows_eq = np.all(g[0] == o[0], axis=1)
    if not rows_eq.all():
        bad = np.nonzero(~rows_eq)[0][:5]
        raise AssertionError("%s: rows differ at %s gpu %s oracle %s" % (label, bad, g[0][bad], o[0][bad]))
    assert np.array_equal(g[1], o[1]), label
    assert np.array_equal(g[2], o[2]), label
    return g


class Pair:
    """The same tree on the GPU and in the oracle, plus the current point set."""

    def __init__(self, orc, pk, c, i, events=0, **kw):
        D = c.shape[0]
        self.orc, self.pk = orc, pk
        self.op = orc.Params(D, **kw)
        self.g = pk.Tree(pk.Params(D, **kw), c, i, update_events=events)
        self.o = orc.Tree(self.op, c, i)
        self.c, self.i = c, i

    def insert(self, c, i):
        self.g.insert(c, i)
        self.o.insert(c, i)
        self.c = np.concatenate([self.c, c], axis=1)
        self.i = np.concatenate([self.i, i])

    def delete(self, c, i):
        a = self.g.delete(c, i)
        b = self.o.delete(c, i)
        assert a == b, (a, b)
        # an entry only removes a point when its coordinates match too
        self.c, self.i = self._remaining(c, i)
        return a

    def _remaining(self, c, i):
        pos = {int(x): k for k, x in enumerate(self.i)}
        keep = np.ones(self.i.shape[0], dtype=bool)
        for j in range(i.shape[0]):
            k = pos.get(int(i[j]))
            if k is not None and keep[k] and np.array_equal(self.c[:, k], c[:, j]):
                keep[k] = False
        return np.ascontiguousarray(self.c[:, keep]), self.i[keep]

    def check(self, label, q=None, boxes=None):
        rows, ids, coords = _same(self.g, self.o, label)
        treecheck.check_tree(rows, ids, coords, self.op.phi, self.c, self.i)
        assert self.g.size() == self.i.shape[0]
        # the queries read the tree's packed coordinate copy, which every
        # update must leave equal to the point array
        D = self.c.shape[0]
        if q is None:
            q = synth.uniform_queries(200, D, seed=990)
        if boxes is None:
            boxes = synth.log_uniform_boxes(200, D, seed=991)
        if q is not None:
            gi, gd = self.g.knn(q, 10)
            bi, bd = self.orc.brute_knn(self.c, self.i, q, 10)
            assert np.array_equal(gi.cpu().numpy(), bi) and np.array_equal(gd.cpu().numpy(), bd), label
        if boxes is not None:
            got = self.g.range_count(*boxes).cpu().numpy()
            assert np.array_equal(got, self.orc.brute_range_count(self.c, *boxes)), label


# events: how an update places the old points (0: by the batch's density,
# 1: sorted event lists, 2: per-point arrays); the trees are the same
@pytest.mark.parametrize("D,kw,events", [(3, {}, 0), (2, dict(lam=3, phi=4, sigma=4), 0), (2, dict(alpha=(1, 10)), 0),
                                         (3, {}, 1), (2, dict(lam=3, phi=4, sigma=4), 2)])
def test_insert_delete_sequence(orc, pk, D, kw, events):
    c, i, state = synth.clustered_points(120000, D, seed=60, n_clusters=60)
    P = Pair(orc, pk, c, i, events=events, **kw)
    q = synth.uniform_queries(300, D, seed=61)
    boxes = synth.log_uniform_boxes(300, D, seed=62)
    P.check("build", q, boxes)
    nid = 10 ** 7
    for step in range(3):
        nc, ni, state = synth.clustered_points(15000, D, seed=63 + step, continue_from=state, id_base=nid)
        nid += 15000
        P.insert(nc, ni)
        P.check("insert %d" % step, q, boxes)
        pick = synth.sample_existing(P.i, 12000, seed=70 + step)
        assert P.delete(P.c[:, pick], P.i[pick]) == 12000
        P.check("delete %d" % step, q, boxes)


@pytest.mark.parametrize("events", [0, 2])
def test_uniform_small_batches(orc, pk, events):
    c, i = synth.uniform_points(200000, 3, seed=80)
    P = Pair(orc, pk, c, i, events=events)
    nid = 10 ** 7
    for step, m in enumerate([1, 7, 100, 1000]):
        nc, ni = synth.uniform_points(m, 3, seed=81 + step, id_base=nid)
        nid += m
        P.insert(nc, ni)
        P.check("insert m=%d" % m)
        pick = synth.sample_existing(P.i, m, seed=90 + step)
        P.delete(P.c[:, pick], P.i[pick])
        P.check("delete m=%d" % m)


@pytest.mark.parametrize("events", [0, 1])
def test_large_batches(orc, pk, events):
    c, i = synth.uniform_points(100000, 2, seed=100)
    P = Pair(orc, pk, c, i, events=events)
    nc, ni = synth.uniform_points(150000, 2, seed=101, id_base=10 ** 7)
    P.insert(nc, ni)
    P.check("insert 150%")
    pick = synth.sample_existing(P.i, 200000, seed=102)
    P.delete(P.c[:, pick], P.i[pick])
    P.check("delete 80%")


def test_root_rebuild_at_balance_bound(orc, pk):
    c, i = synth.uniform_points(3000, 2, seed=81)
    P = Pair(orc, pk, c, i)
    rows, _, _ = P.g.export()
    d, x, n, l = rows[0, 1], rows[0, 2], rows[0, 3], rows[1, 3]
    k = 4 * n - 5 * l
    rng = np.random.default_rng(82)
    newc = rng.integers(0, 10 ** 9, size=(2, k + 1)).astype(np.int64)
    newc[d] = rng.integers(0, x, size=k + 1)
    newi = np.arange(10 ** 6, 10 ** 6 + k + 1, dtype=np.int64)
    P.insert(np.ascontiguousarray(newc[:, :k]), newi[:k])
    P.check("at bound")
    P.insert(np.ascontiguousarray(newc[:, k:]), newi[k:])
    P.check("past bound")


def test_empty_tree_and_delete_everything(orc, pk):
    E = Pair(orc, pk, np.zeros((3, 0), dtype=np.int64), np.zeros(0, dtype=np.int64))
    c, i = synth.uniform_points(20000, 3, seed=110)
    E.insert(c, i)
    E.check("insert into empty")
    assert E.delete(c, i) == 20000
    E.check("delete all")
    E.insert(c[:, :50].copy(), i[:50])
    E.check("reinsert small")
    assert E.delete(c[:, :50].copy(), i[:50]) == 50
    E.check("delete all small")


@pytest.mark.parametrize("events", [0, 2])
def test_delete_absent_mismatched_and_repeated(orc, pk, events):
    c, i = synth.uniform_points(30000, 2, seed=120)
    P = Pair(orc, pk, c, i, events=events)
    ac, ai = synth.uniform_points(500, 2, seed=121, id_base=10 ** 8)
    assert P.delete(ac, ai) == 0
    wrong = c[:, :300].copy()
    wrong[1] += 1
    assert P.delete(wrong, i[:300]) == 0
    P.check("no-op deletes")
    rc = np.concatenate([c[:, :400], c[:, :400]], axis=1)
    ri = np.concatenate([i[:400], i[:400]])
    assert P.delete(rc, ri) == 400
    P.check("repeated entries")


def test_duplicates_with_updates(orc, pk):
    c, i = synth.duplicate_heavy_points(50000, 2, seed=130, n_distinct=20)
    P = Pair(orc, pk, c, i)
    nc, ni = synth.duplicate_heavy_points(20000, 2, seed=130, n_distinct=20, id_base=10 ** 7)
    P.insert(nc, ni)
    P.check("dup insert")
    pick = synth.sample_existing(P.i, 30000, seed=131)
    P.delete(P.c[:, pick], P.i[pick])
    P.check("dup delete")


def test_update_rejects_out_of_range(pk):
    c, i = synth.uniform_points(5000, 2, seed=140)
    t = pk.Tree(pk.Params(2), c, i)
    before = t.export()
    bad = synth.uniform_points(10, 2, seed=141, id_base=10 ** 7)[0]
    bad[0, 3] = 1 << 30
    with pytest.raises(pk.PkdError) as e:
        t.insert(bad, np.arange(10 ** 7, 10 ** 7 + 10, dtype=np.int64))
    assert e.value.code == -2
    for a, b in zip(before, t.export()):
        assert np.array_equal(a, b)


def test_scattered_batches_route_by_sort(orc, pk):
    # uniform batches spread over thousands of subtrees: the deeper routing
    # rounds hold many small subproblems and take the sort path
    c, i = synth.uniform_points(400000, 3, seed=110)
    P = Pair(orc, pk, c, i)
    q = synth.uniform_queries(200, 3, seed=111)
    nc, ni = synth.uniform_points(60000, 3, seed=112, id_base=10 ** 7)
    P.insert(nc, ni)
    P.check("scattered insert", q)
    pick = synth.sample_existing(P.i, 60000, seed=113)
    assert P.delete(P.c[:, pick], P.i[pick]) == 60000
    P.check("scattered delete", q)
    # entries that match nothing and repeated entries
    extra_c = np.concatenate([P.c[:, :50], nc[:, :50] + 1], axis=1)
    extra_i = np.concatenate([P.i[:50], ni[:50]])
    P.delete(np.ascontiguousarray(extra_c), extra_i)
    P.check("partial matches", q)


def test_updates_on_a_tree_above_2_27_points(pk):
    # small batches on a 1.5e8-point tree (new places from the sorted update
    # events and their chunk tables), then a batch of 1.4e8 points, whose
    # per-entry prefix sums take the recursive form of the scan (inputs above
    # 2^27); answers are checked against brute force over the current set on
    # the device (exact int64 arithmetic)
    import torch
    D, n0, m, m2 = 2, 150_000_000, 100_000, 140_000_000
    assert m2 > (1 << 27)
    ids = torch.arange(n0, device="cuda", dtype=torch.int64)
    c = synth.hashed_points_torch(ids, D, 21)
    print("large tree build", flush=True)
    t = pk.Tree(pk.Params(D), c, ids)
    nid = torch.arange(n0, n0 + m, device="cuda", dtype=torch.int64)
    nc = synth.hashed_points_torch(nid, D, 99)
    t.insert(nc, nid)
    assert t.size() == n0 + m
    # delete every third original point of the first 3m
    did = torch.arange(0, 3 * m, 3, device="cuda", dtype=torch.int64)
    assert t.delete(c[:, did].contiguous(), did) == m
    assert t.size() == n0
    print("large batch insert", flush=True)
    bid = torch.arange(n0 + m, n0 + m + m2, device="cuda", dtype=torch.int64)
    bc = synth.hashed_points_torch(bid, D, 123)
    t.insert(bc, bid)
    assert t.size() == n0 + m2
    keep = torch.ones(n0, dtype=torch.bool, device="cuda")
    keep[did] = False
    allc = torch.cat([c[:, keep], nc, bc], dim=1)
    alli = torch.cat([ids[keep], nid, bid])
    del c, bc, keep
    # no point lost or duplicated by the relayout: every id is reported once
    # in the box of the whole domain (range report, a different kernel)
    full_lo = torch.zeros((D, 1), dtype=torch.int64, device="cuda")
    full_hi = torch.full((D, 1), (1 << 30) - 1, dtype=torch.int64, device="cuda")
    off, rid = t.range_report(full_lo, full_hi)
    assert int(off[-1]) == n0 + m2
    assert torch.equal(torch.sort(rid).values, torch.sort(alli).values)
    del rid
    q = torch.from_numpy(synth.uniform_queries(32, D, seed=5)).cuda()
    gi, gd = t.knn(q, 10)
    for j in range(q.shape[1]):
        d2 = ((allc - q[:, j:j + 1]) ** 2).sum(0)
        top = torch.topk(-d2, 64).indices
        cand = sorted(zip(d2[top].tolist(), alli[top].tolist()))[:10]
        assert gd[j].tolist() == [x for x, _ in cand] and gi[j].tolist() == [y for _, y in cand], j
    lo, hi = (torch.from_numpy(x).cuda() for x in synth.log_uniform_boxes(32, D, seed=6))
    rc = t.range_count(lo, hi)
    for j in range(lo.shape[1]):
        inside = ((allc >= lo[:, j:j + 1]) & (allc <= hi[:, j:j + 1])).all(0).sum().item()
        assert rc[j].item() == inside, j
    t.free()
