"""GPU range report against the plain definition (brute force) and the
oracle's report over its own tree: per box the same set of ids; offsets are
the exclusive prefix sums of the range counts.  All through the C-ABI."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _check(t, ot, c, i, lo, hi, label):
    import torch
    off, ids = t.range_report(lo, hi)
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    cnt = t.range_count(lo, hi).cpu().numpy()
    assert off[0] == 0 and np.array_equal(np.diff(off), cnt), label
    oo, oi = ot.range_report(lo, hi)
    assert np.array_equal(oo, off), label
    for j in range(lo.shape[1]):
        g = np.sort(ids[off[j]:off[j + 1]])
        assert np.array_equal(g, np.sort(oi[oo[j]:oo[j + 1]])), (label, j)
    # the plain definition on a subset of the boxes
    for j in range(0, lo.shape[1], max(1, lo.shape[1] // 40)):
        inside = np.all((c >= lo[:, j:j + 1]) & (c <= hi[:, j:j + 1]), axis=0)
        assert np.array_equal(np.sort(ids[off[j]:off[j + 1]]), np.sort(i[inside])), (label, j)
    return off, ids


@pytest.mark.parametrize("D,n", [(2, 100000), (3, 200000), (5, 50000), (1, 30000)])
def test_report_matches_definition_and_oracle(pk, orc, D, n):
    c, i = synth.uniform_points(n, D, seed=300 + D)
    t = pk.Tree(pk.Params(D), c, i)
    ot = orc.Tree(orc.Params(D), c, i)
    lo, hi = synth.log_uniform_boxes(300, D, seed=301, side_lo=1e7, side_hi=8e8)
    # the whole domain, an inverted box, a one-point box
    lo[:, 0], hi[:, 0] = 0, 2 ** 30 - 1
    lo[:, 1], hi[:, 1] = 5, 4
    lo[:, 2], hi[:, 2] = c[:, 7], c[:, 7]
    off, ids = _check(t, ot, c, i, lo, hi, "uniform D=%d" % D)
    assert off[1] - off[0] == n and off[2] == off[1] and off[3] - off[2] >= 1
    t.free()


def test_report_large_outputs_use_copy_records(pk, orc):
    # outputs of 1e4..3e5 points: contained subtrees beyond the wave-copied
    # size go through copy records of several chunks
    D, n = 3, 1_000_000
    c, i = synth.uniform_points(n, D, seed=310)
    t = pk.Tree(pk.Params(D), c, i)
    ot = orc.Tree(orc.Params(D), c, i)
    lo, hi = synth.report_boxes(60, D, n, seed=311, out_lo=1e4, out_hi=3e5)
    off, _ = _check(t, ot, c, i, lo, hi, "large")
    assert np.diff(off).max() > 1e5
    t.free()


def test_report_heavy_leaves_and_duplicates(pk, orc):
    D = 2
    c, i = synth.duplicate_heavy_points(60000, D, seed=320, n_distinct=300)
    t = pk.Tree(pk.Params(D), c, i)
    ot = orc.Tree(orc.Params(D), c, i)
    lo, hi = synth.log_uniform_boxes(200, D, seed=321, side_lo=1e6, side_hi=5e8)
    lo[:, :10] = c[:, :10]
    hi[:, :10] = c[:, :10]                 # boxes that are exactly one duplicated point
    _check(t, ot, c, i, lo, hi, "duplicates")
    t.free()


def test_report_after_updates_and_on_batch_handles(pk, orc):
    import torch
    D = 3
    c, i = synth.uniform_points(120000, D, seed=330)
    t = pk.Tree(pk.Params(D), c, i)
    ot = orc.Tree(orc.Params(D), c, i)
    nc, ni = synth.uniform_points(30000, D, seed=331, id_base=10 ** 7)
    t.insert(nc, ni)
    ot.insert(nc, ni)
    assert t.delete(c[:, :20000], i[:20000]) == ot.delete(c[:, :20000], i[:20000])
    cur_c = np.concatenate([c[:, 20000:], nc], axis=1)
    cur_i = np.concatenate([i[20000:], ni])
    lo, hi = synth.log_uniform_boxes(150, D, seed=332, side_lo=1e7, side_hi=6e8)
    _check(t, ot, cur_c, cur_i, lo, hi, "after updates")
    t.free()
    # a batch handle: box j runs on tree tree_of[j]
    sizes = [5000, 0, 17000, 40000]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    bc, bi = synth.uniform_points(int(off[-1]), D, seed=333)
    bt = pk.Tree.batch(pk.Params(D), bc, bi, off)
    lo, hi = synth.log_uniform_boxes(80, D, seed=334, side_lo=1e8, side_hi=8e8)
    tree_of = (np.arange(80) % 4).astype(np.int32)
    goff, gids = bt.range_report(lo, hi, tree_of=tree_of)
    goff, gids = goff.cpu().numpy(), gids.cpu().numpy()
    for j in range(80):
        tr = tree_of[j]
        a, b = int(off[tr]), int(off[tr + 1])
        inside = np.all((bc[:, a:b] >= lo[:, j:j + 1]) & (bc[:, a:b] <= hi[:, j:j + 1]), axis=0)
        assert np.array_equal(np.sort(gids[goff[j]:goff[j + 1]]), np.sort(bi[a:b][inside])), j
    bt.free()


def test_report_sizing_and_capacity(pk):
    import torch
    D = 2
    c, i = synth.uniform_points(50000, D, seed=340)
    t = pk.Tree(pk.Params(D), c, i)
    lo, hi = (torch.from_numpy(x).cuda() for x in synth.log_uniform_boxes(50, D, seed=341, side_lo=1e8, side_hi=5e8))
    L = pk.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    off = torch.empty(51, dtype=torch.int64, device="cuda")
    total = C.c_int64()
    # sizing call: offsets and total only
    assert L.pkd_range_report(t.h, s, C.c_void_p(lo.data_ptr()), C.c_void_p(hi.data_ptr()), 50,
                              C.c_void_p(off.data_ptr()), None, 0, C.byref(total)) == 0
    cnt = t.range_count(lo, hi)
    assert total.value == int(cnt.sum()) and total.value > 100
    # too small a buffer: PKD_ERR_CAPACITY, nothing written
    buf = torch.full((total.value - 1,), -9, dtype=torch.int64, device="cuda")
    assert L.pkd_range_report(t.h, s, C.c_void_p(lo.data_ptr()), C.c_void_p(hi.data_ptr()), 50,
                              C.c_void_p(off.data_ptr()), C.c_void_p(buf.data_ptr()), total.value - 1,
                              C.byref(total)) == -6
    assert bool((buf == -9).all())
    # an out-of-range corner: PKD_ERR_RANGE
    bad = lo.clone()
    bad[0, 3] = 2 ** 30
    assert L.pkd_range_report(t.h, s, C.c_void_p(bad.data_ptr()), C.c_void_p(hi.data_ptr()), 50,
                              C.c_void_p(off.data_ptr()), None, 0, C.byref(total)) == -2
    # no boxes
    assert L.pkd_range_report(t.h, s, C.c_void_p(lo.data_ptr()), C.c_void_p(hi.data_ptr()), 0,
                              C.c_void_p(off.data_ptr()), None, 0, C.byref(total)) == 0
    assert total.value == 0 and int(off[0]) == 0
    t.free()
