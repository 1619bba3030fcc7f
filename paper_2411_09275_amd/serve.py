"""Serving loop: one resident tree answers a stream of BatchInsert, BatchDelete
and k-NN requests with continuous batching.

Semantics: serializable by arrival order.  A k-NN request sees exactly the
updates that arrived before it, and updates apply in arrival order, so every
result equals the one obtained when the requests are handled one at a time.

Continuous batching: whenever the device can take more work, the server takes
the longest run of waiting k-NN requests in front of the next update that fits
the admission limits, merges it into one launch per distinct k and enqueues it
without waiting (pkd_knn_async, errors land in a per-batch device status word).
Admission: at most `max_inflight` batches in flight, at most
`max_batch_queries` queries per batch, and the query, id and distance buffers
of the batches in flight within the byte budget (free HBM less a reserve, or
the caller's `budget_bytes` if smaller).  A request larger than the budget on
its own runs alone once nothing else is in flight.

Streams: queries go up on an upload stream, the kernels run on the compute
stream, results come down on a download stream; events order the three.  So
batch i+1's upload runs while batch i computes, and batch i's download while
batch i+1 computes.  Each in-flight slot owns pinned staging buffers for
queries and results that grow when a batch needs more and are otherwise
reused (batch i uses slot i mod max_inflight, which batch i - max_inflight
has released), so no pinned memory is allocated per batch.  A retire thread
waits for each batch's download and copies every request's rows out of the
slot's buffers into the request's own host arrays, in row chunks spread over
a few copy threads (the copy is bound by the first touch of those fresh
pages); it overlaps the next batches' transfers and kernels instead of
holding up the issuing loop.  A batch stays in flight,
holding its slot, until its copy is done.  Requests that arrive while batches
are in flight join the next batch.  An update runs on the compute stream with
the blocking calls as soon as it reaches the front of the queue, without
draining the batches in flight: their k-NN kernels precede it on the compute
stream, so they have read the tree before the update's first kernel rewrites
it, while their downloads and copy-outs go on beside the update.  Should the
update run out of device memory (it then leaves the tree as it was), the
batches in flight are retired, releasing their buffers, and it runs again.

The serial reference (mode "serial") handles each request alone, in arrival
order, with the blocking calls.
"""
from __future__ import annotations

import collections
import concurrent.futures
import time
from dataclasses import dataclass

import numpy as np


@dataclass
class Request:
    seq: int
    kind: str                 # "insert", "delete" or "knn"
    arrival: float            # seconds after the start of the stream
    coords: np.ndarray        # host int64 [D, m]: points of an update, or queries
    ids: np.ndarray = None    # host int64 [m] for updates
    k: int = 10
    start: float = None       # set by the server
    done: float = None
    result: object = None     # knn: (ids, d2) host int64 [m, k]; delete: points removed

    @classmethod
    def from_dict(cls, d):
        return cls(seq=d["seq"], kind=d["kind"], arrival=d["arrival"], coords=d["coords"], ids=d.get("ids"),
                   k=d.get("k", 10))

    @property
    def size(self):
        return int(self.coords.shape[1])


class _Batch:
    __slots__ = ("groups", "event", "status", "nbytes", "retired")

    def __init__(self, groups, event, status, nbytes):
        self.groups = groups      # [(requests, host ids, host d2)]
        self.event = event        # recorded on the download stream after the last copy
        self.status = status
        self.nbytes = nbytes
        self.retired = None       # future of the retire thread's copy-out


class Server:
    COPY_THREADS = 8
    COPY_CHUNK_BYTES = 16 << 20

    def __init__(self, tree, dim, max_inflight=3, max_batch_queries=4_000_000, hbm_reserve_bytes=4 << 30,
                 budget_bytes=None):
        import torch
        self.torch = torch
        self.tree = tree
        self.dim = dim
        self.max_inflight = max_inflight
        self.max_batch_queries = max_batch_queries
        self.reserve = hbm_reserve_bytes
        self.budget = budget_bytes
        self.upload = torch.cuda.Stream()
        self.compute = torch.cuda.Stream()
        self.download = torch.cuda.Stream()
        self.inflight_bytes = 0
        self.batches = 0          # k-NN batches issued by the last run
        self.launches = 0         # k-NN launches issued by the last run
        self._stage = [dict() for _ in range(max_inflight)]
        self._issued = 0
        self._retirer = concurrent.futures.ThreadPoolExecutor(max_workers=1)
        # copying results out of the pinned buffers into fresh host arrays is
        # bound by first-touch page faults: several threads copy row chunks
        self._copiers = concurrent.futures.ThreadPoolExecutor(max_workers=self.COPY_THREADS)

    def close(self):
        """Stop the retire and copy threads (the server is not used afterwards)."""
        self._retirer.shutdown(wait=True)
        self._copiers.shutdown(wait=True)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _pinned(self, slot, name, n):
        """A pinned int64 buffer of at least n elements owned by `slot`."""
        buf = self._stage[slot].get(name)
        if buf is None or buf.numel() < n:
            cap = max(n, int(1.5 * (buf.numel() if buf is not None else 0)), 1 << 16)
            buf = self.torch.empty(cap, dtype=self.torch.int64, pin_memory=True)
            self._stage[slot][name] = buf
        return buf

    # ---------------------------------------------------------------- admission
    def _knn_bytes(self, r):
        return r.size * (8 * self.dim + 16 * r.k)

    def _admit(self, need):
        """May a batch of `need` more bytes be enqueued now?"""
        free, _ = self.torch.cuda.mem_get_info()
        limit = free - self.reserve + self.inflight_bytes   # bytes in flight are already out of `free`
        if self.budget is not None:
            limit = min(limit, self.budget)
        return self.inflight_bytes + need <= limit

    # ---------------------------------------------------------------- work
    def _apply(self, r):
        torch = self.torch
        with torch.cuda.stream(self.compute):
            c = torch.from_numpy(np.ascontiguousarray(r.coords)).cuda()
            i = torch.from_numpy(np.ascontiguousarray(r.ids)).cuda()
            if r.kind == "insert":
                self.tree.insert(c, i, stream=self.compute)
            else:
                r.result = self.tree.delete(c, i, stream=self.compute)

    def _run_update(self, r, now, inflight=None):
        from . import PkdError
        r.start = now()
        try:
            self._apply(r)
        except PkdError as e:
            if e.code != -4 or not inflight:          # -4: PKD_ERR_OOM
                raise
            while inflight:                           # the tree is unchanged: free what the batches hold
                self._retire(inflight.popleft())
            self._apply(r)
        self.compute.synchronize()
        r.done = now()

    def _issue(self, reqs, nbytes, now):
        """Enqueue one batch of k-NN requests: one launch per distinct k."""
        torch = self.torch
        t = now()
        for r in reqs:
            r.start = t
        slot = self._issued % self.max_inflight
        self._issued += 1
        by_k = collections.defaultdict(list)
        for r in reqs:
            by_k[r.k].append(r)
        nq_all = sum(r.size for r in reqs)
        nres = sum(r.size * r.k for r in reqs)
        up = self._pinned(slot, "up", self.dim * nq_all)
        hi_all = self._pinned(slot, "ids", nres)
        hd_all = self._pinned(slot, "d2", nres)
        with torch.cuda.stream(self.compute):
            status = torch.zeros(1, dtype=torch.int32, device="cuda")
        groups = []
        q_at = r_at = 0
        for k, rs in by_k.items():
            nq = sum(r.size for r in rs)
            hq = up[q_at:q_at + self.dim * nq].view(self.dim, nq)
            col = 0
            for r in rs:
                hq[:, col:col + r.size].numpy()[...] = r.coords
                col += r.size
            q_at += self.dim * nq
            with torch.cuda.stream(self.upload):
                dq = hq.to("cuda", non_blocking=True)
            ev_up = torch.cuda.Event()
            ev_up.record(self.upload)
            self.compute.wait_event(ev_up)
            dq.record_stream(self.compute)
            with torch.cuda.stream(self.compute):
                oi = torch.empty((nq, k), dtype=torch.int64, device="cuda")
                od = torch.empty((nq, k), dtype=torch.int64, device="cuda")
            self.tree.knn_async(dq, k, oi, od, status, stream=self.compute)
            self.launches += 1
            fin = torch.cuda.Event()
            fin.record(self.compute)
            self.download.wait_event(fin)
            hi = hi_all[r_at:r_at + nq * k].view(nq, k)
            hd = hd_all[r_at:r_at + nq * k].view(nq, k)
            r_at += nq * k
            with torch.cuda.stream(self.download):
                hi.copy_(oi, non_blocking=True)
                hd.copy_(od, non_blocking=True)
            oi.record_stream(self.download)
            od.record_stream(self.download)
            groups.append((rs, hi, hd))
        ev = torch.cuda.Event()
        ev.record(self.download)
        self.inflight_bytes += nbytes
        self.batches += 1
        b = _Batch(groups, ev, status, nbytes)
        b.retired = self._retirer.submit(self._copy_out, b, now)
        return b

    def _copy_out(self, b, now):
        """Retire thread: wait for the batch's download, check its status and
        copy each request's rows into arrays of its own."""
        b.event.synchronize()
        st = int(b.status.item())
        if st != 0:
            raise RuntimeError("k-NN batch reported device status %d" % st)
        jobs = []
        for rs, hi, hd in b.groups:
            hi, hd = hi.numpy(), hd.numpy()
            k = hi.shape[1]
            rows = max(1, self.COPY_CHUNK_BYTES // (8 * k))
            at = 0
            for r in rs:
                m = r.size
                oi = np.empty((m, k), dtype=np.int64)
                od = np.empty((m, k), dtype=np.int64)
                r.result = (oi, od)
                for a in range(0, m, rows):
                    e = min(m, a + rows)
                    jobs.append(self._copiers.submit(np.copyto, oi[a:e], hi[at + a:at + e]))
                    jobs.append(self._copiers.submit(np.copyto, od[a:e], hd[at + a:at + e]))
                at += m
        for j in jobs:
            j.result()
        t = now()
        for rs, _, _ in b.groups:
            for r in rs:
                r.done = t

    def _retire(self, b):
        """Wait until the batch's results are copied out; frees its slot."""
        b.retired.result()        # re-raises what the retire thread raised
        self.inflight_bytes -= b.nbytes

    # ---------------------------------------------------------------- run
    def run(self, requests, mode="continuous", realtime=True):
        """Handle `requests`; returns the makespan in seconds.  mode
        "continuous" batches as described above, "serial" handles one request
        at a time.  realtime=False lets every request arrive at time 0."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.seq))
        self.batches = self.launches = 0
        self._issued = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0   # noqa: E731
        arr = (lambda r: r.arrival) if realtime else (lambda r: 0.0)
        if mode == "serial":
            for r in reqs:
                while arr(r) > now():
                    time.sleep(min(arr(r) - now(), 1e-3) if arr(r) - now() > 2e-4 else 0)
                if r.kind == "knn":
                    r.start = now()
                    oi, od = self.tree.knn(r.coords, r.k)
                    r.result = (oi.cpu().numpy(), od.cpu().numpy())
                    r.done = now()
                    self.batches += 1
                    self.launches += 1
                else:
                    self._run_update(r, now)
            return now()
        if mode != "continuous":
            raise ValueError("mode must be 'continuous' or 'serial'")
        ready = collections.deque()
        inflight = collections.deque()
        try:
            self._continuous(reqs, ready, inflight, arr, now)
        except BaseException:
            # leave nothing running on the device or in the retire thread
            torch.cuda.synchronize()
            for b in inflight:
                concurrent.futures.wait([b.retired])
            raise
        torch.cuda.synchronize()
        return now()

    def _continuous(self, reqs, ready, inflight, arr, now):
        i = 0
        while i < len(reqs) or ready or inflight:
            t = now()
            while i < len(reqs) and arr(reqs[i]) <= t:
                ready.append(reqs[i])
                i += 1
            while inflight and inflight[0].retired.done():
                self._retire(inflight.popleft())
            if not ready:
                if inflight:
                    time.sleep(2e-5)
                elif i < len(reqs):
                    wait = arr(reqs[i]) - now()
                    if wait > 2e-4:
                        time.sleep(min(wait, 1e-3))
                continue
            if ready[0].kind != "knn":
                self._run_update(ready.popleft(), now, inflight)
                continue
            if len(inflight) >= self.max_inflight:
                self._retire(inflight.popleft())
                continue
            batch, nq, nbytes = [], 0, 0
            while ready and ready[0].kind == "knn":
                r = ready[0]
                need = self._knn_bytes(r)
                if batch and nq + r.size > self.max_batch_queries:
                    break
                if not self._admit(nbytes + need) and (batch or inflight):
                    break
                batch.append(ready.popleft())
                nq += r.size
                nbytes += need
            if not batch:
                self._retire(inflight.popleft())   # wait for memory held by batches in flight
                continue
            inflight.append(self._issue(batch, nbytes, now))


def latency_stats(requests):
    """p50 / p99 / mean of arrival-to-result latency in milliseconds."""
    lat = np.array([r.done - r.arrival for r in requests])
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}
