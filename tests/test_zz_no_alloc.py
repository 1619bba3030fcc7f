"""pkd_knn_noalloc (k-NN with its scratch in a static device array) gives
exactly pkd_knn's results, over several calls in a row whose sizes shrink, so
the shared array is reused with the previous call's contents still in it."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _call(L, fn, t, s, q, k):
    import torch
    nq = q.shape[1]
    oi = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    od = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    rc = getattr(L, fn)(t.h, s, C.c_void_p(q.data_ptr()), nq, k, C.c_void_p(oi.data_ptr()),
                        C.c_void_p(od.data_ptr()))
    return rc, oi, od


def test_noalloc_knn_equals_pkd_knn(pk, orc):
    import torch
    L = pk.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    D = 3
    c, i = synth.uniform_points(500000, D, seed=140)
    t = pk.Tree(pk.Params(D), c, i)
    # sizes shrink from call to call: Morton-ordered batches (>= 16384
    # queries) first, then batches kept in their order
    for nq, k in ((600000, 10), (300000, 100), (40000, 1), (5000, 32), (700, 10)):
        q = torch.from_numpy(synth.uniform_queries(nq, D, seed=141 + nq % 97)).cuda()
        rc, oi, od = _call(L, "pkd_knn_noalloc", t, s, q, k)
        assert rc == 0, (nq, k, rc)
        rc2, ri, rd = _call(L, "pkd_knn", t, s, q, k)
        assert rc2 == 0
        assert torch.equal(oi, ri) and torch.equal(od, rd), (nq, k)
        rows = np.arange(0, nq, max(1, nq // 200))
        bi, bd = orc.brute_knn(c, i, np.ascontiguousarray(q.cpu().numpy()[:, rows]), k)
        assert np.array_equal(oi.cpu().numpy()[rows], bi) and np.array_equal(od.cpu().numpy()[rows], bd)
    t.free()


def test_noalloc_knn_limits_and_errors(pk):
    import torch
    L = pk.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    D = 2
    c, i = synth.uniform_points(50000, D, seed=150)
    t = pk.Tree(pk.Params(D), c, i)
    # more queries than the static array serves: refused before any work
    big = 1048577
    q = torch.zeros((D, big), dtype=torch.int64, device="cuda")
    rc, _, _ = _call(L, "pkd_knn_noalloc", t, s, q, 1)
    assert rc == -3
    # an out-of-range query is reported like pkd_knn reports it; the next
    # call (flags cleared again) succeeds
    q = torch.from_numpy(synth.uniform_queries(20000, D, seed=151)).cuda()
    q[0, 5] = 2 ** 30
    assert _call(L, "pkd_knn_noalloc", t, s, q, 10)[0] == -2
    q[0, 5] = 17
    rc, oi, od = _call(L, "pkd_knn_noalloc", t, s, q, 10)
    assert rc == 0
    _, ri, rd = _call(L, "pkd_knn", t, s, q, 10)
    assert torch.equal(oi, ri) and torch.equal(od, rd)
    t.free()
