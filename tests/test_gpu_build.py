"""GPU parity: the HIP build equals the oracle's tree node for node (splitters,
sizes, leaf membership as sorted id sets, coordinates), and queries equal the
plain definitions (brute force) and the oracle.  All through the C-ABI."""
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


def _params(orc, pk, D, **kw):
    return orc.Params(D, **kw), pk.Params(D, **kw)


def _same_tree(gt, ot, label=""):
    g = gt.export()
    o = ot.export()
    assert g[0].shape == o[0].shape, (label, g[0].shape, o[0].shape)
    rows_eq = np.all(g[0] == o[0], axis=1)
    if not rows_eq.all():
        bad = np.nonzero(~rows_eq)[0][:5]
        raise AssertionError("%s: node rows differ at %s: gpu %s oracle %s" % (label, bad, g[0][bad], o[0][bad]))
    assert np.array_equal(g[1], o[1]), label
    assert np.array_equal(g[2], o[2]), label
    return g


def _build_both(orc, pk, c, i, tile=2048, **kw):
    D = c.shape[0]
    op, gp = _params(orc, pk, D, **kw)
    ot = orc.Tree(op, c, i)
    gt = pk.Tree(gp, c, i, tile=tile)
    return gt, ot, op


CASES = [
    ("2d-uniform-100k", lambda: synth.uniform_points(100000, 2, seed=1), {}),
    ("3d-uniform-300k", lambda: synth.uniform_points(300000, 3, seed=2), {}),
    ("1d-dups", lambda: synth.uniform_points(50000, 1, seed=3, hi=5000), {}),
    ("5d-uniform", lambda: synth.uniform_points(60000, 5, seed=4), {}),
    ("7d-uniform", lambda: synth.uniform_points(30000, 7, seed=5), {}),
    ("3d-clustered", lambda: synth.clustered_points(200000, 3, seed=6, n_clusters=50)[:2], {}),
    ("2d-small-params", lambda: synth.uniform_points(40000, 2, seed=7), dict(lam=3, phi=4, sigma=4)),
    ("3d-lambda8", lambda: synth.uniform_points(200000, 3, seed=8), dict(lam=8, sigma=8)),
    ("2d-dup-heavy", lambda: synth.duplicate_heavy_points(60000, 2, seed=9, n_distinct=40), {}),
    ("2d-lambda1", lambda: synth.uniform_points(30000, 2, seed=10), dict(lam=1, sigma=64)),
]


@pytest.mark.parametrize("name,gen,kw", CASES, ids=[c[0] for c in CASES])
def test_build_matches_oracle(orc, pk, name, gen, kw):
    print("case", name, flush=True)
    c, i = gen()
    gt, ot, op = _build_both(orc, pk, c, i, **kw)
    rows, ids, coords = _same_tree(gt, ot, name)
    treecheck.check_tree(rows, ids, coords, op.phi, c, i)
    assert gt.size() == i.shape[0]
    assert gt.height() == ot.height()


@pytest.mark.parametrize("n", [0, 1, 2, 31, 32, 33, 100, 2047, 2048, 2049, 6144, 6145, 13000])
def test_build_boundary_sizes(orc, pk, n):
    c, i = synth.uniform_points(n, 3, seed=100 + n)
    gt, ot, op = _build_both(orc, pk, c, i)
    _same_tree(gt, ot, "n=%d" % n)


@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_tile_size_does_not_change_the_tree(orc, pk, tile):
    c, i = synth.uniform_points(400000, 2, seed=11)
    gt, ot, op = _build_both(orc, pk, c, i, tile=tile)
    _same_tree(gt, ot, "tile=%d" % tile)


def test_input_order_does_not_change_the_tree(orc, pk):
    c, i = synth.uniform_points(150000, 3, seed=12)
    perm = np.random.default_rng(0).permutation(i.shape[0])
    a = pk.Tree(pk.Params(3), c, i).export()
    b = pk.Tree(pk.Params(3), np.ascontiguousarray(c[:, perm]), i[perm]).export()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_identical_points_and_degenerate_sample(orc, pk):
    c = np.full((2, 9000), 1234, dtype=np.int64)
    i = np.arange(9000, dtype=np.int64)
    gt, ot, op = _build_both(orc, pk, c, i)
    _same_tree(gt, ot, "identical")
    # all points on one location except a few the root sample misses: the
    # sample is entirely identical while the set is not (exact split path)
    n = 200000
    i = np.arange(n, dtype=np.int64)
    c = np.full((2, n), 500, dtype=np.int64)
    samp = orc.sample(42, 0, i, 2048)
    others = np.setdiff1d(np.arange(0, n, 997), samp)[:40]
    c[:, others] = synth.uniform_points(40, 2, seed=26)[0]
    gt, ot, op = _build_both(orc, pk, c, i)
    _same_tree(gt, ot, "degenerate-sample")


def test_repeat_build_is_deterministic(pk):
    c, i = synth.uniform_points(500000, 3, seed=13)
    a = pk.Tree(pk.Params(3), c, i).export()
    for _ in range(2):
        b = pk.Tree(pk.Params(3), c, i).export()
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_out_of_range_coordinates_rejected(pk):
    c, i = synth.uniform_points(10000, 2, seed=14)
    for bad in (-1, 1 << 30):
        cc = c.copy()
        cc[1, 777] = bad
        with pytest.raises(pk.PkdError) as e:
            pk.Tree(pk.Params(2), cc, i)
        assert e.value.code == -2
    small = c[:, :100].copy()
    small[0, 5] = -3
    with pytest.raises(pk.PkdError):
        pk.Tree(pk.Params(2), small, i[:100])


# --------------------------------------------------------------------- queries
@pytest.mark.parametrize("D,n,k,hi", [(2, 100000, 10, 10 ** 9), (3, 200000, 1, 10 ** 9), (3, 100000, 16, 10 ** 9),
                                      (2, 50000, 7, 300), (1, 20000, 5, 1000), (5, 40000, 10, 10 ** 6),
                                      (3, 30000, 100, 10 ** 9), (2, 20, 10, 10 ** 9), (3, 50000, 33, 10 ** 9),
                                      (2, 20, 100, 10 ** 9), (3, 50000, 128, 10 ** 9), (2, 50000, 17, 300),
                                      (4, 30000, 64, 10 ** 9), (3, 60000, 9, 10 ** 9), (2, 40000, 10, 200),
                                      (3, 40000, 32, 10 ** 9)])
def test_knn_matches_definition(orc, pk, D, n, k, hi):
    c, i = synth.uniform_points(n, D, seed=20 + D, hi=hi)
    q = synth.uniform_queries(500, D, seed=21, hi=hi)
    t = pk.Tree(pk.Params(D), c, i)
    gi, gd = t.knn(q, k)
    bi, bd = orc.brute_knn(c, i, q, k)
    assert np.array_equal(gd.cpu().numpy(), bd)
    assert np.array_equal(gi.cpu().numpy(), bi)


def test_knn_empty_tree_and_duplicates(orc, pk):
    q = synth.uniform_queries(50, 2, seed=22)
    t = pk.Tree(pk.Params(2), np.zeros((2, 0), dtype=np.int64), np.zeros(0, dtype=np.int64))
    for k in (5, 40):
        gi, gd = t.knn(q, k)
        assert (gi.cpu().numpy() == -1).all() and (gd.cpu().numpy() == -1).all()
    # heavy leaves of identical points, scanned in several passes of 64 by the wave kernel
    c, i = synth.duplicate_heavy_points(30000, 2, seed=23, n_distinct=30)
    t = pk.Tree(pk.Params(2), c, i)
    for k in (1, 3, 10, 24, 100):
        gi, gd = t.knn(q, k)
        bi, bd = orc.brute_knn(c, i, q, k)
        assert np.array_equal(gi.cpu().numpy(), bi) and np.array_equal(gd.cpu().numpy(), bd), k


@pytest.mark.parametrize("D,hi,dups", [(2, 10 ** 9, 0), (3, 10 ** 9, 0), (2, 60, 0), (2, 10 ** 9, 25)])
def test_range_count_matches_definition(orc, pk, D, hi, dups):
    if dups:
        c, i = synth.duplicate_heavy_points(60000, D, seed=30, n_distinct=dups)
    else:
        c, i = synth.uniform_points(100000, D, seed=30 + D, hi=hi)
    lo, up = synth.log_uniform_boxes(1000, D, seed=31, side_lo=1, side_hi=hi, hi=hi)
    t = pk.Tree(pk.Params(D), c, i)
    got = t.range_count(lo, up).cpu().numpy()
    assert np.array_equal(got, orc.brute_range_count(c, lo, up))
    lo2 = lo.copy()
    lo2[0] = up[0] + 1
    assert (t.range_count(lo2, up).cpu().numpy() == 0).all()


def test_queries_reject_out_of_range(pk):
    c, i = synth.uniform_points(1000, 2, seed=32)
    t = pk.Tree(pk.Params(2), c, i)
    q = synth.uniform_queries(10, 2, seed=33)
    q[0, 3] = 1 << 30
    with pytest.raises(pk.PkdError):
        t.knn(q, 3)
    lo, hi = synth.log_uniform_boxes(10, 2, seed=34)
    lo[1, 2] = -5
    with pytest.raises(pk.PkdError):
        t.range_count(lo, hi)


# --------------------------------------------------------------------- batching
def test_batch_build_equals_single_builds(orc, pk):
    rng = np.random.default_rng(200)
    sizes = synth.log_uniform_sizes(60, 1, 3e5, seed=201)
    sizes[3] = 0                                   # an empty tree
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    c, i = synth.uniform_points(int(offsets[-1]), 3, seed=202)
    B = pk.Tree.batch(pk.Params(3), c, i, offsets)
    assert B.num_trees() == 60
    for t in range(60):
        a, b = offsets[t], offsets[t + 1]
        ot = orc.Tree(orc.Params(3), np.ascontiguousarray(c[:, a:b]), i[a:b])
        g = B.export(t)
        o = ot.export()
        for x, y in zip(g, o):
            assert np.array_equal(x, y), t
    # queries routed to their trees
    nq = 2000
    q = synth.uniform_queries(nq, 3, seed=203)
    tree_of = rng.integers(0, 60, size=nq).astype(np.int32)
    for k in (1, 10, 100):
        gi, gd = B.knn(q, k, tree_of=tree_of)
        gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
        for t in range(0, 60, 7):
            sel = np.nonzero(tree_of == t)[0]
            a, b = offsets[t], offsets[t + 1]
            bi, bd = orc.brute_knn(np.ascontiguousarray(c[:, a:b]), i[a:b], np.ascontiguousarray(q[:, sel]), k)
            assert np.array_equal(gi[sel], bi) and np.array_equal(gd[sel], bd), (t, k)
    lo, hi = synth.log_uniform_boxes(nq, 3, seed=204)
    got = B.range_count(lo, hi, tree_of=tree_of).cpu().numpy()
    for t in range(0, 60, 5):
        sel = np.nonzero(tree_of == t)[0]
        a, b = offsets[t], offsets[t + 1]
        ref = orc.brute_range_count(np.ascontiguousarray(c[:, a:b]), np.ascontiguousarray(lo[:, sel]),
                                    np.ascontiguousarray(hi[:, sel]))
        assert np.array_equal(got[sel], ref), t
    # updates go to one tree of the handle (tree 0 here); the others stay
    extra_c, extra_i = c[:, :5].copy(), i[:5] + 10 ** 9
    B.insert(extra_c, extra_i, tree=0)
    a, b = offsets[0], offsets[1]
    ot = orc.Tree(orc.Params(3), np.ascontiguousarray(c[:, a:b]), i[a:b])
    ot.insert(extra_c, extra_i)
    for x, y in zip(B.export(0), ot.export()):
        assert np.array_equal(x, y)
    with pytest.raises(pk.PkdError):
        B.insert(extra_c, extra_i + 1, tree=60)     # no such tree


# ------------------------------------------------ large batches (spatial order)
# Batches of at least 16384 queries are processed in Morton order; every
# result must still land in its own row and equal the oracle's.
@pytest.mark.parametrize("D,nq,k", [(3, 40000, 10), (2, 16384, 1), (5, 20000, 7), (1, 30000, 3), (3, 40000, 100),
                                    (2, 30000, 24)])
def test_knn_large_batch_matches_oracle(orc, pk, D, nq, k):
    c, i = synth.uniform_points(120000, D, seed=40 + D)
    q = synth.uniform_queries(nq, D, seed=41)
    print("knn large batch D=%d nq=%d k=%d" % (D, nq, k), flush=True)
    t = pk.Tree(pk.Params(D), c, i)
    gi, gd = t.knn(q, k)
    oi, od = orc.Tree(orc.Params(D), c, i).knn(q, k)
    assert np.array_equal(gd.cpu().numpy(), od)
    assert np.array_equal(gi.cpu().numpy(), oi)
    # the same queries in small unordered pieces give the same rows
    si, sd = t.knn(q[:, :5000].copy(), k)
    assert np.array_equal(si.cpu().numpy(), oi[:5000]) and np.array_equal(sd.cpu().numpy(), od[:5000])


def test_range_count_large_batch_matches_oracle(orc, pk):
    c, i = synth.uniform_points(150000, 3, seed=50)
    lo, hi = synth.log_uniform_boxes(30000, 3, seed=51, side_lo=1e5, side_hi=1e8)
    print("range large batch", flush=True)
    t = pk.Tree(pk.Params(3), c, i)
    got = t.range_count(lo, hi).cpu().numpy()
    assert np.array_equal(got, orc.Tree(orc.Params(3), c, i).range_count(lo, hi))


def test_range_count_lane_and_wave_kernels_agree(orc, pk):
    # 2^20 boxes take the one-lane-per-box kernel, a smaller batch the
    # one-wave-per-box kernel: the same boxes give the same counts
    c, i = synth.uniform_points(150000, 3, seed=52)
    nb = 1 << 20
    lo, hi = synth.log_uniform_boxes(nb, 3, seed=53, side_lo=1e5, side_hi=1e8)
    print("range lane vs wave", flush=True)
    t = pk.Tree(pk.Params(3), c, i)
    big = t.range_count(lo, hi).cpu().numpy()
    part = t.range_count(np.ascontiguousarray(lo[:, :200000]), np.ascontiguousarray(hi[:, :200000])).cpu().numpy()
    assert np.array_equal(big[:200000], part)
    rows = np.sort(np.random.default_rng(54).choice(nb, size=3000, replace=False))
    ref = orc.Tree(orc.Params(3), c, i).range_count(np.ascontiguousarray(lo[:, rows]), np.ascontiguousarray(hi[:, rows]))
    assert np.array_equal(big[rows], ref)


def test_batch_handle_large_query_batch(orc, pk):
    sizes = synth.log_uniform_sizes(40, 1, 5e4, seed=60)
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    c, i = synth.uniform_points(int(offsets[-1]), 2, seed=61)
    B = pk.Tree.batch(pk.Params(2), c, i, offsets)
    nq = 50000
    q = synth.uniform_queries(nq, 2, seed=62)
    tree_of = np.random.default_rng(63).integers(0, 40, size=nq).astype(np.int32)
    print("batch handle large query batch", flush=True)
    gi, gd = B.knn(q, 10, tree_of=tree_of)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    lo, hi = synth.log_uniform_boxes(nq, 2, seed=64)
    rc = B.range_count(lo, hi, tree_of=tree_of).cpu().numpy()
    for t in range(40):
        sel = np.nonzero(tree_of == t)[0]
        a, b = offsets[t], offsets[t + 1]
        ot = orc.Tree(orc.Params(2), np.ascontiguousarray(c[:, a:b]), i[a:b])
        oi, od = ot.knn(np.ascontiguousarray(q[:, sel]), 10)
        assert np.array_equal(gi[sel], oi) and np.array_equal(gd[sel], od), t
        ref = ot.range_count(np.ascontiguousarray(lo[:, sel]), np.ascontiguousarray(hi[:, sel]))
        assert np.array_equal(rc[sel], ref), t


# ------------------------------------------------ forced sampler retries
# A biased candidate threshold makes the sampler overflow (negative bias: too
# many candidates) or underflow (positive: fewer than s) on every sieving
# subproblem; the retry must converge to the same sample, so the tree is the
# same as without the bias.
@pytest.mark.parametrize("bias", [-4, -1, 2, 4])
def test_sampler_retry_keeps_the_tree(orc, pk, bias):
    c, i = synth.uniform_points(600000, 3, seed=70)
    ref = pk.Tree(pk.Params(3), c, i).export()
    print("cand bias", bias, flush=True)
    got = pk.Tree(pk.Params(3), c, i, cand_bias=bias).export()
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)
    sizes = np.array([300000, 0, 5000, 120000], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)])
    cb, ib = synth.clustered_points(int(off[-1]), 2, seed=71, n_clusters=20)[:2]
    B0 = pk.Tree.batch(pk.Params(2), cb, ib, off)
    B1 = pk.Tree.batch(pk.Params(2), cb, ib, off, cand_bias=bias)
    for t in range(4):
        for x, y in zip(B0.export(t), B1.export(t)):
            assert np.array_equal(x, y)


# ------------------------------------------------ asynchronous entry points
def test_async_queries_match_and_report_errors_in_status(pk):
    import torch
    c, i = synth.uniform_points(80000, 3, seed=80)
    t = pk.Tree(pk.Params(3), c, i)
    q = synth.uniform_queries(20000, 3, seed=81)
    lo, hi = synth.log_uniform_boxes(20000, 3, seed=82)
    ri, rd = t.knn(q, 10)
    rc = t.range_count(lo, hi)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        oi = torch.empty((20000, 10), dtype=torch.int64, device="cuda")
        od = torch.empty((20000, 10), dtype=torch.int64, device="cuda")
        oc = torch.empty(20000, dtype=torch.int64, device="cuda")
        dq, dlo, dhi = (torch.from_numpy(x).cuda() for x in (q, lo, hi))
    t.knn_async(dq, 10, oi, od, st, stream=s)
    t.range_count_async(dlo, dhi, oc, st, stream=s)
    s.synchronize()
    assert int(st.item()) == 0
    assert torch.equal(oi, ri) and torch.equal(od, rd) and torch.equal(oc, rc)
    # a coordinate out of range is reported in the status word, not raised
    bad = q.copy()
    bad[1, 7] = 1 << 30
    with torch.cuda.stream(s):
        st2 = torch.zeros(1, dtype=torch.int32, device="cuda")
        dbad = torch.from_numpy(bad).cuda()
    t.knn_async(dbad, 10, oi, od, st2, stream=s)
    s.synchronize()
    assert int(st2.item()) & 1


def test_direct_knn_and_range_count_entry_points(orc, pk):
    # pkd_knn / pkd_range_count themselves (the binding's Tree methods go
    # through the batch forms); results against the plain definitions
    import ctypes as C
    import torch
    D = 3
    c, i = synth.uniform_points(200000, D, seed=130)
    op, gp = _params(orc, pk, D)
    t = pk.Tree(gp, c, i)
    L = pk.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for nq, k in ((1000, 10), (20000, 1), (3000, 100)):
        q = torch.from_numpy(synth.uniform_queries(nq, D, seed=131 + k)).cuda()
        oi = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
        od = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
        assert L.pkd_knn(t.h, s, C.c_void_p(q.data_ptr()), nq, k, C.c_void_p(oi.data_ptr()),
                         C.c_void_p(od.data_ptr())) == 0
        rows = np.arange(0, nq, max(1, nq // 300))
        bi, bd = orc.brute_knn(c, i, np.ascontiguousarray(q.cpu().numpy()[:, rows]), k)
        assert np.array_equal(oi.cpu().numpy()[rows], bi) and np.array_equal(od.cpu().numpy()[rows], bd), (nq, k)
    lo, hi = (torch.from_numpy(x).cuda() for x in synth.log_uniform_boxes(500, D, seed=135))
    out = torch.full((500,), -7, dtype=torch.int64, device="cuda")
    assert L.pkd_range_count(t.h, s, C.c_void_p(lo.data_ptr()), C.c_void_p(hi.data_ptr()), 500,
                             C.c_void_p(out.data_ptr())) == 0
    assert np.array_equal(out.cpu().numpy(), orc.brute_range_count(c, lo.cpu().numpy(), hi.cpu().numpy()))
    # a query outside [0, 2^30) is refused with PKD_ERR_RANGE
    bad = torch.zeros((D, 4), dtype=torch.int64, device="cuda")
    bad[1, 2] = 2 ** 30
    assert L.pkd_knn(t.h, s, C.c_void_p(bad.data_ptr()), 4, 10, C.c_void_p(oi.data_ptr()),
                     C.c_void_p(od.data_ptr())) == -2
    t.free()


@pytest.mark.parametrize("D,n,gen", [(1, 50000, "uniform"), (2, 300000, "uniform"), (3, 200000, "clustered"),
                                     (5, 60000, "uniform"), (2, 120000, "dups")])
def test_exact_median_mode_matches_oracle(orc, pk, D, n, gen):
    # oversample 0: every node split at the exact median of all its points,
    # one level per round, by the segmented device split (Section 6.4's
    # comparison of sampling against exact medians)
    if gen == "uniform":
        c, i = synth.uniform_points(n, D, seed=600 + D)
    elif gen == "clustered":
        c, i, _ = synth.clustered_points(n, D, seed=601, n_clusters=40)
    else:
        c, i = synth.duplicate_heavy_points(n, D, seed=602, n_distinct=500, hot_fraction=0.3)
    gt = pk.Tree(pk.Params(D, lam=1, sigma=0), c, i)
    ot = orc.Tree(orc.Params(D, lam=1, sigma=0), c, i)
    _same_tree(gt, ot, "exact %s D=%d" % (gen, D))
    # updates rebuild with exact medians too
    nc, ni = synth.uniform_points(n // 10, D, seed=603, id_base=10 ** 8)
    gt.insert(nc, ni)
    ot.insert(nc, ni)
    assert gt.delete(c[:, : n // 7], i[: n // 7]) == ot.delete(c[:, : n // 7], i[: n // 7])
    _same_tree(gt, ot, "exact after updates")
    gt.free()


def test_exact_median_mode_rejects_lambda_above_one(pk):
    with pytest.raises(pk.PkdError) as e:
        pk.Tree(pk.Params(2, lam=6, sigma=0), *synth.uniform_points(100, 2, seed=1))
    assert e.value.code == -1
