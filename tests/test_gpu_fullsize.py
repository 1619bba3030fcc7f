"""Parity at the benchmark's full size and launch configuration: 1e8 uniform
3-D points (seed 3), default parameters, tiles of 2048; 1e7 uniform 10-NN
queries (seed 4) and 1e5 range boxes (seed 5) each in one call, as the
benchmark issues them.  The whole GPU tree equals the oracle's node for node;
query results are compared with the oracle on a sample of rows (the oracle
answers them one by one from its own tree)."""
import time

import numpy as np
import pytest

import synth
from tests import progress

pytestmark = pytest.mark.gpu

N, DIM, NQ, NB = 100_000_000, 3, 10_000_000, 100_000


def _log(msg, t0):
    progress.log("fullsize", msg)


@pytest.fixture(scope="module")
def full(orc):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_09275_amd as pk
    t0 = time.perf_counter()
    coords, ids = synth.uniform_points(N, DIM, seed=3)
    _log("inputs generated", t0)
    gt = pk.Tree(pk.Params(DIM), torch.from_numpy(coords).cuda(), torch.from_numpy(ids).cuda(), tile=2048)
    torch.cuda.synchronize()
    _log("GPU build done", t0)
    ot = orc.Tree(orc.Params(DIM), coords, ids)
    _log("oracle build done", t0)
    yield pk, gt, ot, coords, ids, t0
    gt.free()


@pytest.mark.timeout(900)
def test_full_size_tree_equals_oracle(full):
    pk, gt, ot, coords, ids, t0 = full
    g = gt.export()
    _log("GPU export done", t0)
    o = ot.export()
    _log("oracle export done", t0)
    assert g[0].shape == o[0].shape
    rows_eq = np.all(g[0] == o[0], axis=1)
    if not rows_eq.all():
        bad = np.nonzero(~rows_eq)[0][:5]
        raise AssertionError("node rows differ at %s: gpu %s oracle %s" % (bad, g[0][bad], o[0][bad]))
    assert np.array_equal(g[1], o[1])
    assert np.array_equal(g[2], o[2])
    # every input id once
    seen = np.zeros(N, dtype=bool)
    seen[g[1]] = True
    assert seen.all() and g[1].shape[0] == N
    assert gt.height() == ot.height()
    _log("tree compared: %d nodes" % g[0].shape[0], t0)


@pytest.mark.timeout(900)
def test_full_size_queries_sampled(full, orc):
    import torch
    pk, gt, ot, coords, ids, t0 = full
    q = synth.uniform_queries(NQ, DIM, seed=4)
    lo, hi = synth.log_uniform_boxes(NB, DIM, seed=5)
    gi, gd = gt.knn(torch.from_numpy(q).cuda(), 10)
    rc = gt.range_count(torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda())
    torch.cuda.synchronize()
    _log("GPU queries done", t0)
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(NQ, size=20000, replace=False))
    rows = np.concatenate([rows, [0, NQ - 1]])
    oi, od = ot.knn(np.ascontiguousarray(q[:, rows]), 10)
    assert np.array_equal(gd[torch.from_numpy(rows).cuda()].cpu().numpy(), od)
    assert np.array_equal(gi[torch.from_numpy(rows).cuda()].cpu().numpy(), oi)
    boxes = np.sort(rng.choice(NB, size=2000, replace=False))
    ref = ot.range_count(np.ascontiguousarray(lo[:, boxes]), np.ascontiguousarray(hi[:, boxes]))
    assert np.array_equal(rc.cpu().numpy()[boxes], ref)
    # a few rows against the plain definition over all 1e8 points
    few = rows[:4]
    bi, bd = orc.brute_knn(coords, ids, np.ascontiguousarray(q[:, few]), 10)
    assert np.array_equal(gi[torch.from_numpy(few).cuda()].cpu().numpy(), bi)
    assert np.array_equal(gd[torch.from_numpy(few).cuda()].cpu().numpy(), bd)
    _log("queries compared", t0)



@pytest.mark.timeout(900)
def test_full_size_range_report_sampled(full, orc):
    # the range-report workload on the full tree: 1e4 cubes whose outputs are
    # log-uniform in [1e4, 1e6] points (about 2e9 ids in one call)
    import torch
    pk, gt, ot, coords, ids, t0 = full
    lo, hi = synth.report_boxes(10_000, DIM, N, seed=6)
    glo, ghi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    off, rid = gt.range_report(glo, ghi)
    torch.cuda.synchronize()
    _log("GPU range report done: %d ids" % rid.numel(), t0)
    cnt = gt.range_count(glo, ghi)
    assert torch.equal(off[1:] - off[:-1], cnt) and int(off[0]) == 0
    rng = np.random.default_rng(8)
    boxes = np.concatenate([rng.choice(10_000, size=24, replace=False), [0, 9_999]])
    o_off, o_ids = ot.range_report(np.ascontiguousarray(lo[:, boxes]), np.ascontiguousarray(hi[:, boxes]))
    offh = off.cpu().numpy()
    for k, j in enumerate(boxes):
        g = np.sort(rid[int(offh[j]):int(offh[j + 1])].cpu().numpy())
        assert np.array_equal(g, np.sort(o_ids[o_off[k]:o_off[k + 1]])), j
    del rid
    torch.cuda.empty_cache()
    _log("range report compared", t0)
