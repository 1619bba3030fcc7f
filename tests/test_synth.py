"""The seeded input generators: the hashed-coordinate points agree between
their numpy and torch forms, and the serving request stream keeps its
contract (fresh insert ids, deletes of live distinct ids with the right
coordinates, the requested mix and size laws)."""
import numpy as np
import pytest

import synth


def test_hashed_points_numpy_equals_torch():
    torch = pytest.importorskip("torch")
    ids = np.concatenate([np.arange(0, 5000), np.array([2 ** 31 - 1, 10 ** 9, 2 ** 40 + 3])]).astype(np.int64)
    for dim, seed, hi in ((1, 0, 10 ** 9), (2, 21, 10 ** 9), (3, 5, 1000), (7, 2 ** 40, 2 ** 30)):
        a = synth.hashed_points(ids, dim, seed, hi)
        b = synth.hashed_points_torch(torch.from_numpy(ids), dim, seed, hi).numpy()
        assert np.array_equal(a, b)
        assert a.min() >= 0 and a.max() < hi


def test_hashed_points_look_uniform():
    a = synth.hashed_points(np.arange(200000, dtype=np.int64), 2, 3)
    hist = np.histogram(a[0], bins=20, range=(0, 10 ** 9))[0]
    assert hist.min() > 0.9 * 10000 and hist.max() < 1.1 * 10000
    assert abs(np.corrcoef(a[0], a[1])[0, 1]) < 0.01


def test_request_stream_contract():
    n0, seed = 50000, 9
    raw = synth.request_stream(2, 400, 4, 50.0, n0, seed, insert_range=(10, 3000), query_range=(10, 500))
    kinds = [r["kind"] for r in raw]
    frac = kinds.count("knn") / len(kinds)
    assert 0.7 < frac < 0.9
    alive = set(range(n0))
    nxt = n0
    last = 0.0
    for r in raw:
        assert r["arrival"] > last
        last = r["arrival"]
        m = r["coords"].shape[1]
        if r["kind"] == "knn":
            assert 10 <= m < 500 and r["k"] in (1, 10, 100)
            continue
        ids = r["ids"]
        assert ids.shape[0] == m and np.array_equal(r["coords"], synth.hashed_points(ids, 2, seed))
        if r["kind"] == "insert":
            assert np.array_equal(ids, np.arange(nxt, nxt + m))
            nxt += m
            alive.update(ids.tolist())
        else:
            s = ids.tolist()
            assert len(set(s)) == m and all(x in alive for x in s)
            alive.difference_update(s)
    assert abs(last / 400 - 1 / 50.0) < 0.3 / 50.0   # mean inter-arrival 1/rate


def test_report_boxes_hit_their_output_sizes():
    # cubes sized for log-uniform expected counts in [1e4, 1e6] of n uniform points
    n, D = 2_000_000, 3
    c, _ = synth.uniform_points(n, D, seed=1)
    lo, hi = synth.report_boxes(200, D, n, seed=2, out_lo=1e3, out_hi=1e5)
    inside = np.array([np.all((c >= lo[:, j:j + 1]) & (c <= hi[:, j:j + 1]), axis=0).sum() for j in range(200)])
    side = hi[0] - lo[0] + 1
    expect = n * (side / 1e9) ** D
    assert np.all(np.abs(inside - expect) <= 6 * np.sqrt(expect) + 2)
    assert inside.min() >= 500 and inside.max() <= 2e5
    assert np.all(hi - lo + 1 == side)      # cubes
