"""Parity of batch updates at full size: the clustered workload of the update
benchmark (1e8 clustered 3-D points from 1000 random-walk clusters with step
lengths log-uniform in [1, 1e6], seed 31), BatchInsert of 1e6 fresh points from
the same walks (seed 32), BatchDelete of 1e6 existing ids drawn uniformly
(seed 34), alpha = 0.3, with the benchmark's default parameters and tiles.
After the build and after each batch the whole GPU tree equals the oracle's
node for node, and 10-NN answers for a sample of the 1e6 in-distribution
queries (seed 33) equal the oracle's.  The three tests share one tree pair and
run in file order."""
import time

import numpy as np
import pytest

import synth
from tests import progress

pytestmark = pytest.mark.gpu

N, DIM, NB, NQ = 100_000_000, 3, 1_000_000, 1_000_000


def _log(msg):
    progress.log("fullsize-updates", msg)


@pytest.fixture(scope="module")
def c3(orc):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_09275_amd as pk
    c, i, state = synth.clustered_points(N, DIM, seed=31)
    ci, ii, _ = synth.clustered_points(NB, DIM, seed=32, id_base=N, continue_from=state)
    q, _, _ = synth.clustered_points(NQ, DIM, seed=33, continue_from=state)
    di = synth.sample_existing(i, NB, seed=34)
    dc = np.ascontiguousarray(c[:, di])
    _log("inputs generated")
    gt = pk.Tree(pk.Params(DIM), torch.from_numpy(c).cuda(), torch.from_numpy(i).cuda(), tile=2048)
    torch.cuda.synchronize()
    _log("GPU build done")
    ot = orc.Tree(orc.Params(DIM), c, i)
    _log("oracle build done")
    st = dict(pk=pk, gt=gt, ot=ot, c=c, i=i, ci=ci, ii=ii, q=q, di=di, dc=dc)
    yield st
    gt.free()


def _compare(st, what):
    g = st["gt"].export()
    o = st["ot"].export()
    _log("%s: exports taken (%d nodes)" % (what, o[0].shape[0]))
    assert g[0].shape == o[0].shape, (what, g[0].shape, o[0].shape)
    rows_eq = np.all(g[0] == o[0], axis=1)
    if not rows_eq.all():
        bad = np.nonzero(~rows_eq)[0][:5]
        raise AssertionError("%s: node rows differ at %s: gpu %s oracle %s" % (what, bad, g[0][bad], o[0][bad]))
    assert np.array_equal(g[1], o[1]), what
    assert np.array_equal(g[2], o[2]), what
    assert st["gt"].size() == st["ot"].size()


def _knn_sample(st, what, seed):
    import torch
    gi, gd = st["gt"].knn(torch.from_numpy(st["q"]).cuda(), 10)
    rng = np.random.default_rng(seed)
    rows = np.concatenate([np.sort(rng.choice(NQ, size=5000, replace=False)), [0, NQ - 1]])
    oi, od = st["ot"].knn(np.ascontiguousarray(st["q"][:, rows]), 10)
    sel = torch.from_numpy(rows).cuda()
    assert np.array_equal(gd[sel].cpu().numpy(), od), what
    assert np.array_equal(gi[sel].cpu().numpy(), oi), what
    _log("%s: 10-NN sample equal" % what)


@pytest.mark.timeout(900)
def test_clustered_1e8_build_equals_oracle(c3):
    _compare(c3, "build")


@pytest.mark.timeout(900)
def test_clustered_1e8_insert_1e6_equals_oracle(c3):
    import torch
    c3["gt"].insert(torch.from_numpy(c3["ci"]).cuda(), torch.from_numpy(c3["ii"]).cuda())
    torch.cuda.synchronize()
    _log("GPU insert done")
    c3["ot"].insert(c3["ci"], c3["ii"])
    _log("oracle insert done: %s" % c3["ot"].update_log())
    _compare(c3, "insert")
    _knn_sample(c3, "insert", 41)


@pytest.mark.timeout(900)
def test_clustered_1e8_delete_1e6_equals_oracle(c3):
    import torch
    k = c3["gt"].delete(torch.from_numpy(c3["dc"]).cuda(), torch.from_numpy(c3["i"][c3["di"]]).cuda())
    _log("GPU delete done")
    ko = c3["ot"].delete(c3["dc"], c3["i"][c3["di"]])
    _log("oracle delete done: %s" % c3["ot"].update_log())
    assert k == ko == NB
    _compare(c3, "delete")
    _knn_sample(c3, "delete", 42)
