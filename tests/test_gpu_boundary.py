"""The boundary's memory contract, through the C-ABI: device memory from a
caller-installed allocator (PyTorch's caching allocator), a failing allocation
at any point of an update leaving the tree exactly as it was, records of
replaced nodes reclaimed, and stream-ordered release."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """Allocations from PyTorch's caching allocator; call number `fail_at`
    (1-based) returns NULL instead."""

    def __init__(self, torch, fail_at=None):
        self.torch, self.fail_at, self.calls, self.live = torch, fail_at, 0, {}
        self.dev = torch.cuda.current_device()

    def alloc(self, n, stream):
        self.calls += 1
        if self.fail_at is not None and self.calls == self.fail_at:
            return 0
        p = self.torch.cuda.caching_allocator_alloc(n, self.dev, stream)
        self.live[p] = n
        return p

    def free(self, p, n, stream):
        assert self.live.pop(p) == n
        self.torch.cuda.caching_allocator_delete(p)


def _export(t):
    return tuple(np.copy(a) for a in t.export())


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def _insert_rc(pk, t, c, i):
    try:
        t.insert(c, i)
        return 0
    except pk.PkdError as e:
        return e.code


def _delete_rc(pk, t, c, i):
    try:
        t.delete(c, i)
        return 0
    except pk.PkdError as e:
        return e.code


@pytest.mark.parametrize("kind", ["insert", "delete", "insert_into_empty"])
def test_failed_allocation_leaves_the_tree_unchanged(pk, orc, kind):
    import torch
    D = 3
    c, i, state = synth.clustered_points(60000, D, seed=160, n_clusters=20)
    nc, ni, _ = synth.clustered_points(9000, D, seed=161, continue_from=state, id_base=10 ** 6)
    pick = synth.sample_existing(i, 9000, seed=162)
    dc, di = np.ascontiguousarray(c[:, pick]), i[pick]
    op = orc.Params(D)
    if kind == "insert_into_empty":
        ref = orc.Tree(op, nc, ni)
    else:
        ref = orc.Tree(op, c, i)
        if kind == "insert":
            ref.insert(nc, ni)
        else:
            ref.delete(dc, di)
    expected = ref.export()

    def fresh():
        t = pk.Tree(pk.Params(D), c, i)
        if kind == "insert_into_empty":
            assert t.delete(c, i) == c.shape[1]
        return t

    def run(t):
        if kind == "delete":
            return _delete_rc(pk, t, dc, di)
        return _insert_rc(pk, t, nc, ni)

    # how many allocations a successful update makes
    t = fresh()
    count = CountingAllocator(torch)
    pk.set_allocator(count.alloc, count.free)
    try:
        assert run(t) == 0
    finally:
        pk.set_allocator()
    assert _same(_export(t), expected)
    t.free()
    assert count.calls > 3, count.calls
    fails = 0
    for n in range(1, count.calls + 1):
        t = fresh()
        before = _export(t)
        a = CountingAllocator(torch, fail_at=n)
        pk.set_allocator(a.alloc, a.free)
        try:
            rc = run(t)
        finally:
            pk.set_allocator()
        if rc == 0:
            # only an optional step (node compaction) may shrug off a failure
            assert _same(_export(t), expected), n
        else:
            assert rc == -4, (n, rc)          # PKD_ERR_OOM
            fails += 1
            assert _same(_export(t), before), "allocation %d of %d changed the tree" % (n, count.calls)
            # the tree still works: the same update now succeeds
            assert run(t) == 0
            assert _same(_export(t), expected), n
        t.free()
    assert fails >= count.calls - 2, (fails, count.calls)


def test_torch_allocator_end_to_end(pk, orc):
    import torch
    D = 2
    c, i = synth.uniform_points(150000, D, seed=170)
    pk.use_torch_allocator()
    try:
        t = pk.Tree(pk.Params(D), c, i)
        o = orc.Tree(orc.Params(D), c, i)
        nc, ni = synth.uniform_points(20000, D, seed=171, id_base=10 ** 7)
        t.insert(nc, ni)
        o.insert(nc, ni)
        assert t.delete(c[:, :5000], i[:5000]) == o.delete(c[:, :5000], i[:5000]) == 5000
        assert _same(_export(t), o.export())
        q = synth.uniform_queries(30000, D, seed=172)
        gi, gd = t.knn(q, 10)
        oi, od = o.knn(q, 10)
        assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gd.cpu().numpy(), od)
        t.free()
    finally:
        pk.set_allocator()


def test_replaced_node_records_are_reclaimed(pk, orc):
    # many small update batches: every one replaces leaves (their records
    # die); the node array is compacted once dead records outnumber live ones,
    # so the records held stay within a constant of the live nodes
    D = 2
    c, i = synth.uniform_points(40000, D, seed=180)
    t = pk.Tree(pk.Params(D), c, i)
    o = orc.Tree(orc.Params(D), c, i)
    rng = np.random.default_rng(181)
    live_c, live_i = c, i
    nid = 10 ** 6
    most = 0
    for step in range(60):
        if step % 2 == 0:
            bc, bi = synth.uniform_points(1500, D, seed=200 + step, id_base=nid)
            nid += 1500
            t.insert(bc, bi)
            o.insert(bc, bi)
            live_c = np.concatenate([live_c, bc], axis=1)
            live_i = np.concatenate([live_i, bi])
        else:
            sel = rng.choice(live_i.shape[0], 1500, replace=False)
            assert t.delete(live_c[:, sel], live_i[sel]) == o.delete(live_c[:, sel], live_i[sel]) == 1500
            keep = np.ones(live_i.shape[0], dtype=bool)
            keep[sel] = False
            live_c, live_i = np.ascontiguousarray(live_c[:, keep]), live_i[keep]
        g = _export(t)
        assert _same(g, o.export()), step
        live = g[0].shape[0]
        slots = t.node_slots()
        most = max(most, slots / live)
        assert slots <= 4 * live + 4096, (step, slots, live)
    assert most > 1.2, most     # records did pile up between compactions
    t.free()


def test_stream_ordered_free(pk, orc):
    import torch
    D = 3
    side = torch.cuda.Stream()
    c, i = synth.uniform_points(300000, D, seed=190)
    q = torch.from_numpy(synth.uniform_queries(200000, D, seed=191)).cuda()
    ref = None
    for rep in range(3):
        with torch.cuda.stream(side):
            t = pk.Tree(pk.Params(D), c, i, stream=side)
            gi, gd = t.knn(q, 10, stream=side)
            t.free(stream=side)            # no wait: the next build reuses the memory in order
        side.synchronize()
        got = (gi.cpu().numpy(), gd.cpu().numpy())
        if ref is None:
            ref = got
            o = orc.Tree(orc.Params(D), c, i)
            rows = np.arange(0, 200000, 997)
            oi, od = o.knn(np.ascontiguousarray(q.cpu().numpy()[:, rows]), 10)
            assert np.array_equal(got[0][rows], oi) and np.array_equal(got[1][rows], od)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), rep
