"""Query batches over a batch handle captured once into a hipGraph and
replayed with new queries in the same buffers: k-NN with k = 1, 10, 100 and
range counts in one graph, every replay equal to the eager calls and, for a
few trees, to the oracle.  Eager work and synchronizations run between the
replays."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

D, T, NQ, NB = 3, 64, 40000, 20000


def _handle(pk):
    sizes = synth.log_uniform_sizes(T, 1e3, 1e5, seed=700)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    c, i = synth.uniform_points(int(off[-1]), D, seed=701)
    return pk.Tree.batch(pk.Params(D), c, i, off), off, c, i


def test_query_batches_replayed_from_a_graph(orc, pk):
    import torch
    B, off, c, i = _handle(pk)
    dev = torch.device("cuda")
    tree_of = torch.from_numpy((np.arange(NQ) % T).astype(np.int32)).to(dev)
    box_tree = torch.from_numpy((np.arange(NB) % T).astype(np.int32)).to(dev)
    q = torch.empty((D, NQ), dtype=torch.int64, device=dev)
    lo = torch.empty((D, NB), dtype=torch.int64, device=dev)
    hi = torch.empty((D, NB), dtype=torch.int64, device=dev)
    ks = (1, 10, 100)
    outs = {k: (torch.empty((NQ, k), dtype=torch.int64, device=dev),
                torch.empty((NQ, k), dtype=torch.int64, device=dev)) for k in ks}
    cnt = torch.empty(NB, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)

    def fill(rep):
        q.copy_(torch.from_numpy(synth.uniform_queries(NQ, D, seed=710 + rep)))
        a, b = synth.log_uniform_boxes(NB, D, seed=720 + rep, side_lo=1e7, side_hi=5e8)
        lo.copy_(torch.from_numpy(a))
        hi.copy_(torch.from_numpy(b))

    fill(0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):            # one eager pass on the capture stream first
        for k in ks:
            B.knn_async(q, k, *outs[k], status, tree_of=tree_of, stream=side)
        B.range_count_async(lo, hi, cnt, status, tree_of=box_tree, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print("capture", flush=True)
    with torch.cuda.graph(g, stream=side):
        status.zero_()
        for k in ks:
            B.knn_async(q, k, *outs[k], status, tree_of=tree_of, stream=side)
        B.range_count_async(lo, hi, cnt, status, tree_of=box_tree, stream=side)
    for rep in range(3):
        fill(rep + 1)
        torch.cuda.synchronize()
        print("replay", rep, flush=True)
        g.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0, rep
        qn = q.cpu().numpy()
        for k in ks:
            ei, ed = B.knn(q, k, tree_of=tree_of)            # eager, spatially ordered
            assert torch.equal(outs[k][0], ei) and torch.equal(outs[k][1], ed), (rep, k)
        assert torch.equal(cnt, B.range_count(lo, hi, tree_of=box_tree)), rep
        for t in (0, 17, 63):
            a, b = int(off[t]), int(off[t + 1])
            ot = orc.Tree(orc.Params(D), np.ascontiguousarray(c[:, a:b]), i[a:b])
            sel = np.nonzero(np.arange(NQ) % T == t)[0]
            oi, od = ot.knn(np.ascontiguousarray(qn[:, sel]), 10)
            assert np.array_equal(outs[10][0].cpu().numpy()[sel], oi), (rep, t)
            assert np.array_equal(outs[10][1].cpu().numpy()[sel], od), (rep, t)
        # eager work of the program between replays
        B.knn(q[:, :1000].contiguous(), 5, tree_of=tree_of[:1000].contiguous())
    B.free()
