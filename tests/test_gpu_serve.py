"""Serving loop: every request's result in the continuously batched mix equals
its result when the requests are handled one at a time, and equals the
oracle's tree replaying the same updates in arrival order.  Forcing the
admission budget down (every batch alone, one in flight) changes no result."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

D = 2
N0 = 150_000
POINT_SEED = 77


@pytest.fixture(scope="module")
def pk():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_09275_amd as pk
    pk.lib()
    return pk


def _initial():
    ids = np.arange(N0, dtype=np.int64)
    return synth.hashed_points(ids, D, POINT_SEED), ids


def _stream(seed, n=40, rate=2000.0):
    from paper_2411_09275_amd.serve import Request
    raw = synth.request_stream(D, n, seed, rate, N0, POINT_SEED, insert_range=(1e2, 2e4), query_range=(1e2, 5e3))
    return [Request.from_dict(r) for r in raw]


def _oracle_replay(orc, reqs):
    c, i = _initial()
    ot = orc.Tree(orc.Params(D), c, i)
    out = {}
    for r in sorted(reqs, key=lambda r: (r.arrival, r.seq)):
        if r.kind == "insert":
            ot.insert(r.coords, r.ids)
        elif r.kind == "delete":
            out[r.seq] = ot.delete(r.coords, r.ids)
        else:
            out[r.seq] = ot.knn(r.coords, r.k)
    return out


def _check_against(reqs, ref):
    n_knn = 0
    for r in reqs:
        assert r.done is not None and r.done >= r.start >= 0, r.seq
        if r.kind == "knn":
            n_knn += 1
            assert r.result[0].shape == (r.size, r.k)
            assert np.array_equal(r.result[0], ref[r.seq][0]), ("ids", r.seq)
            assert np.array_equal(r.result[1], ref[r.seq][1]), ("d2", r.seq)
        elif r.kind == "delete":
            assert r.result == ref[r.seq], (r.seq, r.result, ref[r.seq])
    return n_knn


def _serve(pk, reqs, mode, realtime, **kw):
    from paper_2411_09275_amd.serve import Server
    c, i = _initial()
    t = pk.Tree(pk.Params(D), c, i)
    with Server(t, D, **kw) as s:
        s.run(reqs, mode=mode, realtime=realtime)
    size = t.size()
    t.free()
    return s, size


def test_mix_equals_serial_and_oracle(orc, pk):
    reqs = _stream(seed=5)
    print("continuous, all at once", flush=True)
    s, size_c = _serve(pk, reqs, "continuous", realtime=False)
    ref = _oracle_replay(orc, reqs)
    n_knn = _check_against(reqs, ref)
    assert s.batches < n_knn            # requests were merged
    serial = _stream(seed=5)
    print("serial", flush=True)
    _, size_s = _serve(pk, serial, "serial", realtime=False)
    _check_against(serial, ref)
    assert size_c == size_s


def test_realtime_arrivals(orc, pk):
    reqs = _stream(seed=6, n=30, rate=400.0)
    print("continuous, Poisson arrivals", flush=True)
    _serve(pk, reqs, "continuous", realtime=True)
    _check_against(reqs, _oracle_replay(orc, reqs))
    for r in reqs:
        assert r.start >= r.arrival - 1e-9


def test_forced_queueing_keeps_results(orc, pk):
    reqs = _stream(seed=7, n=30)
    print("budget 1 byte, one in flight", flush=True)
    s, _ = _serve(pk, reqs, "continuous", realtime=False, budget_bytes=1, max_inflight=1)
    n_knn = _check_against(reqs, _oracle_replay(orc, reqs))
    assert s.batches == n_knn            # every request ran alone
    reqs = _stream(seed=7, n=30)
    print("batch cap 300 queries", flush=True)
    _serve(pk, reqs, "continuous", realtime=False, max_batch_queries=300, max_inflight=2)
    _check_against(reqs, _oracle_replay(orc, reqs))


def test_device_error_reaches_the_caller(pk):
    # a query coordinate out of range makes the batch's device status nonzero;
    # the retire thread raises and run() re-raises it
    from paper_2411_09275_amd.serve import Request, Server
    reqs = _stream(seed=8, n=12)
    bad = next(r for r in reqs if r.kind == "knn")
    bad.coords = bad.coords.copy()
    bad.coords[0, 0] = 1 << 30
    c, i = _initial()
    t = pk.Tree(pk.Params(D), c, i)
    print("device status error", flush=True)
    with pytest.raises(RuntimeError):
        Server(t, D).run(reqs, mode="continuous", realtime=False)
    t.free()


def test_update_out_of_memory_with_batches_in_flight(orc, pk):
    # an update no longer drains the batches in flight; when it runs out of
    # device memory (forced here: the allocation after arming returns NULL) the
    # tree is unchanged, the server retires the batches and runs it again
    import torch
    from paper_2411_09275_amd.serve import Server
    dev = torch.cuda.current_device()
    state = {"armed": False, "failed": 0}

    def alloc(n, stream):
        if state["armed"]:
            state["armed"] = False
            state["failed"] += 1
            return 0
        return torch.cuda.caching_allocator_alloc(n, dev, stream)

    def free(p, n, stream):
        torch.cuda.caching_allocator_delete(p)

    class ArmedServer(Server):
        def _run_update(self, r, now, inflight=None):
            state["armed"] = bool(inflight)
            try:
                super()._run_update(r, now, inflight)
            finally:
                state["armed"] = False

    reqs = _stream(seed=9, n=40)
    c, i = _initial()
    pk.set_allocator(alloc, free)
    try:
        t = pk.Tree(pk.Params(D), c, i)
        print("updates fail once with batches in flight", flush=True)
        with ArmedServer(t, D, max_batch_queries=400) as s:
            s.run(reqs, mode="continuous", realtime=False)
        t.free()
    finally:
        pk.set_allocator()
    assert state["failed"] >= 1
    _check_against(reqs, _oracle_replay(orc, reqs))
