"""Eight and nine dimensions (the D = 9 rows of the paper's summary table):
builds, k-NN, range counts, range reports and updates equal the oracle and the
plain definitions, also with coordinates at the nine-dimensional bound, where
a squared distance comes within 0.01 % of 2^63.  All through the C-ABI."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

BOUND9 = 1012333500          # exclusive coordinate bound for D = 9


def _corner_points(n, D, seed, hi):
    """Uniform points with every 8th point pushed to a corner coordinate (0 or hi-1)."""
    c, i = synth.uniform_points(n, D, seed=seed, hi=hi)
    rng = np.random.default_rng(seed + 1)
    sel = np.arange(0, n, 8)
    c[:, sel] = np.where(rng.random((D, sel.shape[0])) < 0.5, 0, hi - 1)
    return np.ascontiguousarray(c), i


def _same(g, o):
    return all(np.array_equal(x, y) for x, y in zip(g, o))


CASES = [
    ("8d-uniform", lambda: synth.uniform_points(40000, 8, seed=900), {}),
    ("9d-uniform", lambda: synth.uniform_points(50000, 9, seed=901), {}),
    ("9d-clustered", lambda: synth.clustered_points(50000, 9, seed=902, n_clusters=40)[:2], {}),
    ("9d-at-bound", lambda: _corner_points(30000, 9, 903, BOUND9), {}),
    ("9d-small-params", lambda: synth.uniform_points(20000, 9, seed=904), dict(lam=3, phi=8, sigma=8)),
    ("9d-exact-medians", lambda: synth.uniform_points(20000, 9, seed=905), dict(lam=1, sigma=0)),
]


@pytest.mark.parametrize("name,gen,kw", CASES, ids=[c[0] for c in CASES])
def test_high_dim_build_and_queries_match_oracle(orc, pk, name, gen, kw):
    print("case", name, flush=True)
    c, i = gen()
    D = c.shape[0]
    hi = BOUND9 if name.endswith("at-bound") else synth.DEFAULT_RANGE
    ot = orc.Tree(orc.Params(D, **kw), c, i)
    gt = pk.Tree(pk.Params(D, **kw), c, i)
    assert _same(gt.export(), ot.export()), name
    q = synth.uniform_queries(3000, D, seed=910, hi=hi)
    q[:, 0] = 0
    q[:, 1] = hi - 1
    for k in (1, 10, 40):
        gi, gd = gt.knn(q, k)
        oi, od = ot.knn(q, k)
        assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gd.cpu().numpy(), od), (name, k)
        bi, bd = orc.brute_knn(c, i, q[:, :300].copy(), k)
        assert np.array_equal(oi[:300], bi) and np.array_equal(od[:300], bd), (name, k)
    lo, up = synth.log_uniform_boxes(2000, D, seed=911, side_lo=3e8, side_hi=9e8, hi=hi)
    got = gt.range_count(lo, up).cpu().numpy()
    assert np.array_equal(got, ot.range_count(lo, up)), name
    assert np.array_equal(got, orc.brute_range_count(c, lo, up)), name
    assert got.sum() > 0
    off, ids = gt.range_report(lo[:, :200].copy(), up[:, :200].copy())
    ooff, oids = ot.range_report(lo[:, :200].copy(), up[:, :200].copy())
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    assert np.array_equal(off, ooff)
    for b in range(200):
        assert np.array_equal(np.sort(ids[off[b]:off[b + 1]]), np.sort(oids[ooff[b]:ooff[b + 1]])), (name, b)
    gt.free()


def test_nine_dim_distances_near_two_to_the_63(orc, pk):
    # opposite corners of the nine-dimensional cube: 9 * (bound - 1)^2
    D = 9
    c = np.zeros((D, 4), dtype=np.int64)
    c[:, 1] = BOUND9 - 1
    c[:4, 2] = BOUND9 - 1
    c[:, 3] = 7
    i = np.array([10, 11, 12, 13], dtype=np.int64)
    t = pk.Tree(pk.Params(D), c, i)
    q = np.zeros((D, 2), dtype=np.int64)
    q[:, 1] = BOUND9 - 1
    gi, gd = t.knn(q, 4)
    far = D * (BOUND9 - 1) ** 2
    assert far < 2 ** 63 and far > 2 ** 63 - 2 ** 63 // 10000
    assert gd.cpu().numpy()[0, -1] == far and gi.cpu().numpy()[0, -1] == 11
    assert gd.cpu().numpy()[1, -1] == far and gi.cpu().numpy()[1, -1] == 10
    oi, od = orc.Tree(orc.Params(D), c, i).knn(q, 4)
    assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gd.cpu().numpy(), od)
    t.free()


def test_coordinate_bounds_by_dimension(pk):
    for D, bound in ((8, 1 << 30), (9, BOUND9)):
        c, i = synth.uniform_points(2000, D, seed=920 + D)
        c[3, 5] = bound - 1
        t = pk.Tree(pk.Params(D), c, i)          # the largest allowed coordinate
        bad = c.copy()
        bad[2, 9] = bound
        with pytest.raises(pk.PkdError) as e:
            pk.Tree(pk.Params(D), bad, i)
        assert e.value.code == -2
        q = synth.uniform_queries(10, D, seed=930)
        q[0, 4] = bound
        with pytest.raises(pk.PkdError):
            t.knn(q, 3)
        with pytest.raises(pk.PkdError):
            t.insert(bad[:, :20].copy(), i[:20] + 10 ** 6)
        assert t.size() == 2000
        t.free()
    with pytest.raises(pk.PkdError) as e:
        pk.Tree(pk.Params(10), np.zeros((10, 4), dtype=np.int64), np.arange(4, dtype=np.int64))
    assert e.value.code == -3


@pytest.mark.parametrize("bbox", [False, True])
def test_nine_dim_updates_match_oracle(orc, pk, bbox):
    D = 9
    c, i, state = synth.clustered_points(60000, D, seed=940, n_clusters=30)
    t = pk.Tree(pk.Params(D), c, i)
    if bbox:
        t.set_bbox(True)
    o = orc.Tree(orc.Params(D), c, i)
    nc, ni, _ = synth.clustered_points(20000, D, seed=941, continue_from=state, id_base=10 ** 7)
    t.insert(nc, ni)
    o.insert(nc, ni)
    assert _same(t.export(), o.export())
    pick = synth.sample_existing(i, 15000, seed=942)
    dc, di = np.ascontiguousarray(c[:, pick]), i[pick]
    assert t.delete(dc, di) == o.delete(dc, di) == 15000
    assert _same(t.export(), o.export())
    q = synth.uniform_queries(2000, D, seed=943)
    for k in (1, 10):
        gi, gd = t.knn(q, k)
        oi, od = o.knn(q, k)
        assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gd.cpu().numpy(), od), k
    t.free()
