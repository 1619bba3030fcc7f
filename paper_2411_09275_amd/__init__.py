"""Python binding of libpkd, the MI355X Pkd-tree library.

Argument marshalling only: every step of build, update and query runs in the
HIP kernels of ``libpkd.so``; PyTorch supplies device memory and the stream.
The library must be built (``python -m paper_2411_09275_amd.build`` or
``__graft_entry__.build()``); importing this module on a machine without it
raises immediately rather than falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpkd.so")

PKD_OK = 0
ERRORS = {
    -1: "PKD_ERR_INVALID_ARG", -2: "PKD_ERR_RANGE", -3: "PKD_ERR_UNSUPPORTED", -4: "PKD_ERR_OOM",
    -5: "PKD_ERR_HIP", -6: "PKD_ERR_CAPACITY", -7: "PKD_ERR_INTERNAL",
}

# Every symbol the C header declares (checked by the ABI test).
EXPORTS = ["pkd_default_params", "pkd_default_tuning", "pkd_build", "pkd_batch_insert", "pkd_batch_delete",
           "pkd_knn", "pkd_range_count", "pkd_size", "pkd_export_sizes", "pkd_export", "pkd_height",
           "pkd_free", "pkd_strerror", "pkd_profile_enable", "pkd_profile_get", "pkd_build_batch",
           "pkd_num_trees", "pkd_knn_batch", "pkd_range_count_batch", "pkd_export_tree_sizes", "pkd_export_tree",
           "pkd_knn_async", "pkd_range_count_async", "pkd_knn_noalloc", "pkd_set_allocator", "pkd_free_async",
           "pkd_node_slots", "pkd_range_report", "pkd_range_report_batch",
           "pkd_update_stats", "pkd_set_bbox", "pkd_export_bbox", "pkd_batch_insert_tree",
           "pkd_batch_delete_tree", "pkd_build_plan_create", "pkd_build_plan_enqueue", "pkd_build_plan_finish",
           "pkd_build_plan_tree", "pkd_build_plan_free"]


class PkdError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, ERRORS.get(code, "unknown"), code))


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("lambda_", C.c_int32), ("leaf_size", C.c_int32), ("oversample", C.c_int32),
                ("alpha_num", C.c_int32), ("alpha_den", C.c_int32), ("seed", C.c_uint64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class _Tuning(C.Structure):
    _fields_ = [("tile_points", C.c_int32), ("cand_shift_bias", C.c_int32), ("update_events", C.c_int32),
                ("reserved", C.c_int32 * 5)]


_lib = None


def lib():
    """Load libpkd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpkd.so is not built (%s); run paper_2411_09275_amd/build.py" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.pkd_default_params.argtypes = [C.POINTER(_Params), i32]
        L.pkd_default_tuning.argtypes = [C.POINTER(_Tuning)]
        L.pkd_build.argtypes = [C.POINTER(_Params), C.POINTER(_Tuning), vp, vp, vp, i64, C.POINTER(vp)]
        L.pkd_batch_insert.argtypes = [vp, vp, vp, vp, i64]
        L.pkd_batch_delete.argtypes = [vp, vp, vp, vp, i64, C.POINTER(i64)]
        L.pkd_knn.argtypes = [vp, vp, vp, i64, i32, vp, vp]
        L.pkd_range_count.argtypes = [vp, vp, vp, vp, i64, vp]
        L.pkd_size.argtypes = [vp, C.POINTER(i64)]
        L.pkd_height.argtypes = [vp, C.POINTER(i32)]
        L.pkd_export_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.pkd_export.argtypes = [vp, vp, vp, vp, vp]
        L.pkd_free.argtypes = [vp]
        L.pkd_free.restype = None
        L.pkd_profile_enable.argtypes = [i32]
        L.pkd_profile_get.argtypes = [i32, C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pkd_build_batch.argtypes = [C.POINTER(_Params), C.POINTER(_Tuning), vp, i32, vp, vp, vp, C.POINTER(vp)]
        L.pkd_num_trees.argtypes = [vp, C.POINTER(i32)]
        L.pkd_knn_batch.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp]
        L.pkd_range_count_batch.argtypes = [vp, vp, vp, vp, vp, i64, vp]
        L.pkd_export_tree_sizes.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i64)]
        L.pkd_export_tree.argtypes = [vp, i32, vp, vp, vp, vp]
        L.pkd_knn_async.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp]
        L.pkd_knn_noalloc.argtypes = [vp, vp, vp, i64, i32, vp, vp]
        L.pkd_set_allocator.argtypes = [C.POINTER(_Allocator)]
        L.pkd_free_async.argtypes = [vp, vp]
        L.pkd_node_slots.argtypes = [vp, C.POINTER(i64)]
        L.pkd_update_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.pkd_set_bbox.argtypes = [vp, vp, i32]
        L.pkd_batch_insert_tree.argtypes = [vp, i32, vp, vp, vp, i64]
        L.pkd_batch_delete_tree.argtypes = [vp, i32, vp, vp, vp, i64, C.POINTER(i64)]
        L.pkd_export_bbox.argtypes = [vp, i32, vp]
        L.pkd_range_report.argtypes = [vp, vp, vp, vp, i64, vp, vp, i64, C.POINTER(i64)]
        L.pkd_range_report_batch.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, i64, C.POINTER(i64)]
        L.pkd_range_count_async.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.pkd_build_plan_create.argtypes = [C.POINTER(_Params), C.POINTER(_Tuning), i32, vp, C.POINTER(vp)]
        L.pkd_build_plan_enqueue.argtypes = [vp, vp, vp, vp]
        L.pkd_build_plan_finish.argtypes = [vp, vp, C.POINTER(i32)]
        L.pkd_build_plan_tree.argtypes = [vp, C.POINTER(vp)]
        L.pkd_build_plan_free.argtypes = [vp]
        L.pkd_build_plan_free.restype = None
        L.pkd_strerror.argtypes = [C.c_int]
        L.pkd_strerror.restype = C.c_char_p
        for f in ("pkd_build_plan_create", "pkd_build_plan_enqueue", "pkd_build_plan_finish", "pkd_build_plan_tree",
                  "pkd_batch_insert_tree", "pkd_batch_delete_tree", "pkd_set_bbox", "pkd_export_bbox", "pkd_update_stats", "pkd_range_report", "pkd_range_report_batch", "pkd_set_allocator", "pkd_free_async", "pkd_node_slots", "pkd_knn_noalloc", "pkd_knn_async", "pkd_range_count_async", "pkd_build_batch", "pkd_num_trees", "pkd_knn_batch", "pkd_range_count_batch",
                  "pkd_export_tree_sizes", "pkd_export_tree", "pkd_profile_enable", "pkd_profile_get", "pkd_build", "pkd_batch_insert", "pkd_batch_delete", "pkd_knn", "pkd_range_count", "pkd_size",
                  "pkd_height", "pkd_export_sizes", "pkd_export"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != PKD_OK:
        raise PkdError(rc, what)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, shape=None):
    """A contiguous int64 CUDA tensor (the caller's buffer when it already is one)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.from_numpy(np.ascontiguousarray(t, dtype=np.int64))
    t = t.to(device="cuda", dtype=torch.int64).contiguous()
    if shape is not None:
        assert tuple(t.shape) == tuple(shape), (tuple(t.shape), shape)
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr() if t.numel() > 0 else 0)


def _to_i32(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.from_numpy(np.ascontiguousarray(t, dtype=np.int32))
    return t.to(device="cuda", dtype=torch.int32).contiguous()


PROFILE_KERNELS = {"sieve_count": 0, "sieve_scatter": 1, "select_skeleton": 2, "finisher": 3, "knn": 4,
                   "range_count": 5, "range_report": 6}


def profile_enable(on: bool = True):
    """Clear and (re)start per-kernel timing with HIP events on the launch stream."""
    _check(lib().pkd_profile_enable(1 if on else 0), "pkd_profile_enable")


def profile_get(name: str):
    """(launches, total milliseconds, algorithmic bytes) of one profiled kernel."""
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    _check(lib().pkd_profile_get(PROFILE_KERNELS[name], C.byref(n), C.byref(ms), C.byref(b)), "pkd_profile_get")
    return n.value, ms.value, b.value


# every allocator ever installed: blocks go back to the allocator that made
# them, also after another one was installed, so its ctypes callbacks must
# outlive it
_installed = []


def set_allocator(alloc=None, free=None):
    """Route the library's device allocations through Python callables:
    alloc(bytes, stream_handle) -> device pointer (int) or 0, and
    free(ptr, bytes, stream_handle).  With no arguments the library's own
    block cache is used again."""
    if alloc is None:
        _check(lib().pkd_set_allocator(None), "pkd_set_allocator")
        return

    def _a(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), stream or 0)) or None
        except Exception:   # an exception cannot cross the C boundary
            return None

    def _f(ptr, nbytes, stream, ctx):
        try:
            free(int(ptr), int(nbytes), stream or 0)
        except Exception:
            pass

    a = _Allocator(ALLOC_FN(_a), FREE_FN(_f), None)
    _installed.append(a)
    _check(lib().pkd_set_allocator(C.byref(a)), "pkd_set_allocator")


def use_torch_allocator():
    """Take the library's device memory from PyTorch's caching allocator."""
    torch = _torch()
    dev = torch.cuda.current_device()
    set_allocator(lambda n, s: torch.cuda.caching_allocator_alloc(n, dev, s),
                  lambda p, n, s: torch.cuda.caching_allocator_delete(p))


class Params:
    """Result-affecting parameters; defaults follow Section 5 of the paper
    (lambda=6, phi=32, sigma=32, alpha=0.3)."""

    def __init__(self, dim, lam=6, phi=32, sigma=32, alpha=(3, 10), seed=42):
        self.dim, self.lam, self.phi, self.sigma = int(dim), int(lam), int(phi), int(sigma)
        self.alpha = (int(alpha[0]), int(alpha[1]))
        self.seed = int(seed)

    def _c(self):
        p = _Params()
        p.dim, p.lambda_, p.leaf_size, p.oversample = self.dim, self.lam, self.phi, self.sigma
        p.alpha_num, p.alpha_den = self.alpha
        p.seed = self.seed & (2 ** 64 - 1)
        return p


def _tuning(tile, cand_bias=0, update_events=0):
    t = _Tuning()
    lib().pkd_default_tuning(C.byref(t))
    t.tile_points = tile
    t.cand_shift_bias = cand_bias
    t.update_events = update_events
    return t


class Tree:
    """A device-resident Pkd-tree (``pkd_tree*``).  Tree(params, coords, ids)
    builds one tree; Tree.batch(params, coords, ids, offsets) builds many trees
    in one pass (tree t owns points offsets[t]:offsets[t+1])."""

    def __init__(self, params: Params, coords, ids, tile: int = 2048, stream=None, _handle=None, cand_bias: int = 0,
                 update_events: int = 0):
        self.p = params
        if _handle is not None:
            self.h = _handle
            return
        c = _dev(coords)
        i = _dev(ids)
        n = i.shape[0]
        assert tuple(c.shape) == (params.dim, n)
        h = C.c_void_p()
        _check(lib().pkd_build(C.byref(params._c()), C.byref(_tuning(tile, cand_bias, update_events)), _stream(stream),
                               _ptr(c), _ptr(i), n, C.byref(h)), "pkd_build")
        self.h = h

    @classmethod
    def batch(cls, params: Params, coords, ids, offsets, tile: int = 2048, stream=None, cand_bias: int = 0,
              update_events: int = 0):
        c = _dev(coords)
        i = _dev(ids)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        assert tuple(c.shape) == (params.dim, i.shape[0]) and off[-1] == i.shape[0]
        h = C.c_void_p()
        _check(lib().pkd_build_batch(C.byref(params._c()), C.byref(_tuning(tile, cand_bias, update_events)),
                                     _stream(stream),
                                     off.shape[0] - 1, _ptr(c), _ptr(i), off.ctypes.data_as(C.c_void_p),
                                     C.byref(h)), "pkd_build_batch")
        return cls(params, None, None, _handle=h)

    def num_trees(self) -> int:
        n = C.c_int32()
        _check(lib().pkd_num_trees(self.h, C.byref(n)), "pkd_num_trees")
        return n.value

    def __del__(self):
        self.free()

    def free(self, stream=None):
        """Release the tree; with a stream, in stream order without waiting
        (pkd_free_async), else after all device work (pkd_free).  The tree of
        a build plan belongs to the plan and is left alone."""
        if getattr(self, "_borrowed", False):
            self.h = None
            return
        if getattr(self, "h", None) is not None and self.h.value:
            if stream is None:
                lib().pkd_free(self.h)
            else:
                _check(lib().pkd_free_async(self.h, _stream(stream)), "pkd_free_async")
        self.h = None

    def set_bbox(self, on: bool = True, stream=None):
        """Keep node bounding boxes and prune queries with them (Pkd-bb)."""
        _check(lib().pkd_set_bbox(self.h, _stream(stream), 1 if on else 0), "pkd_set_bbox")

    def export_bbox(self, t: int = 0):
        """Node boxes in export pre-order: int32 [N, 2*dim] (lo..., hi...)."""
        N, n = C.c_int64(), C.c_int64()
        _check(lib().pkd_export_tree_sizes(self.h, t, C.byref(N), C.byref(n)), "pkd_export_sizes")
        out = np.empty((N.value, 2 * self.p.dim), dtype=np.int32)
        _check(lib().pkd_export_bbox(self.h, t, out.ctypes.data_as(C.c_void_p)), "pkd_export_bbox")
        return out

    def update_stats(self):
        """(subtrees rebuilt, points in them) by the last insert or delete."""
        r, p = C.c_int64(), C.c_int64()
        _check(lib().pkd_update_stats(self.h, C.byref(r), C.byref(p)), "pkd_update_stats")
        return r.value, p.value

    def node_slots(self) -> int:
        n = C.c_int64()
        _check(lib().pkd_node_slots(self.h, C.byref(n)), "pkd_node_slots")
        return n.value

    def size(self) -> int:
        n = C.c_int64()
        _check(lib().pkd_size(self.h, C.byref(n)), "pkd_size")
        return n.value

    def height(self) -> int:
        h = C.c_int32()
        _check(lib().pkd_height(self.h, C.byref(h)), "pkd_height")
        return h.value

    def knn(self, queries, k: int, tree_of=None, stream=None, out=None):
        """(ids, d2) as int64 CUDA tensors [nq, k]; tree_of (int32, per query)
        picks the tree of a batch handle."""
        torch = _torch()
        q = _dev(queries)
        nq = q.shape[1] if q.dim() == 2 else 0
        if out is None:
            oi = torch.empty((nq, k), dtype=torch.int64, device="cuda")
            od = torch.empty((nq, k), dtype=torch.int64, device="cuda")
        else:
            oi, od = out
        to = None if tree_of is None else _to_i32(tree_of)
        _check(lib().pkd_knn_batch(self.h, _stream(stream), _ptr(q), None if to is None else _ptr(to), nq, k,
                                   _ptr(oi), _ptr(od)), "pkd_knn")
        return oi, od

    def knn_async(self, queries, k: int, out_ids, out_d2, status, tree_of=None, stream=None):
        """Enqueue k-NN on `stream` without waiting; errors are ORed into the
        device int32 tensor `status` (zero it first)."""
        q = _dev(queries)
        nq = q.shape[1] if q.dim() == 2 else 0
        to = None if tree_of is None else _to_i32(tree_of)
        _check(lib().pkd_knn_async(self.h, _stream(stream), _ptr(q), None if to is None else _ptr(to), nq, k,
                                   _ptr(out_ids), _ptr(out_d2), _ptr(status)), "pkd_knn_async")

    def range_count_async(self, lo, hi, out, status, tree_of=None, stream=None):
        """Enqueue range counts on `stream` without waiting; errors are ORed
        into the device int32 tensor `status` (zero it first)."""
        lo, hi = _dev(lo), _dev(hi)
        nb = lo.shape[1] if lo.dim() == 2 else 0
        to = None if tree_of is None else _to_i32(tree_of)
        _check(lib().pkd_range_count_async(self.h, _stream(stream), _ptr(lo), _ptr(hi),
                                           None if to is None else _ptr(to), nb, _ptr(out), _ptr(status)),
               "pkd_range_count_async")

    def range_count(self, lo, hi, tree_of=None, stream=None):
        torch = _torch()
        lo, hi = _dev(lo), _dev(hi)
        nb = lo.shape[1]
        out = torch.empty(nb, dtype=torch.int64, device="cuda")
        to = None if tree_of is None else _to_i32(tree_of)
        _check(lib().pkd_range_count_batch(self.h, _stream(stream), _ptr(lo), _ptr(hi),
                                           None if to is None else _ptr(to), nb, _ptr(out)), "pkd_range_count")
        return out

    def range_report(self, lo, hi, tree_of=None, stream=None, out=None):
        """(offsets [nb+1], ids [total]) as int64 CUDA tensors: box j's point
        ids are ids[offsets[j]:offsets[j+1]] (in no particular order).  `out`
        may supply an id buffer; it is used when large enough."""
        torch = _torch()
        lo, hi = _dev(lo), _dev(hi)
        nb = lo.shape[1]
        off = torch.empty(nb + 1, dtype=torch.int64, device="cuda")
        to = None if tree_of is None else _to_i32(tree_of)
        total = C.c_int64()
        L = lib()

        def call(buf, cap):
            return L.pkd_range_report_batch(self.h, _stream(stream), _ptr(lo), _ptr(hi),
                                            None if to is None else _ptr(to), nb, _ptr(off),
                                            None if buf is None else _ptr(buf), cap, C.byref(total))

        if out is not None:
            rc = call(out, out.numel())
            if rc == PKD_OK:
                return off, out[: total.value]
            if rc != -6:
                _check(rc, "pkd_range_report")
        else:
            _check(call(None, 0), "pkd_range_report")
        ids = torch.empty(max(total.value, 1), dtype=torch.int64, device="cuda")
        _check(call(ids, ids.numel()), "pkd_range_report")
        return off, ids[: total.value]

    def range_report_size(self, lo, hi, tree_of=None, stream=None):
        """(offsets [nb+1] CUDA tensor, total ids) without reporting."""
        torch = _torch()
        lo, hi = _dev(lo), _dev(hi)
        nb = lo.shape[1]
        off = torch.empty(nb + 1, dtype=torch.int64, device="cuda")
        to = None if tree_of is None else _to_i32(tree_of)
        total = C.c_int64()
        _check(lib().pkd_range_report_batch(self.h, _stream(stream), _ptr(lo), _ptr(hi),
                                            None if to is None else _ptr(to), nb, _ptr(off), None, 0,
                                            C.byref(total)), "pkd_range_report")
        return off, total.value

    def insert(self, coords, ids, stream=None, tree: int = 0):
        """BatchInsert into tree `tree` of the handle (0 for a single tree)."""
        c, i = _dev(coords), _dev(ids)
        _check(lib().pkd_batch_insert_tree(self.h, tree, _stream(stream), _ptr(c), _ptr(i), i.shape[0]),
               "pkd_batch_insert")

    def delete(self, coords, ids, stream=None, tree: int = 0) -> int:
        """BatchDelete from tree `tree` of the handle; returns the points removed."""
        c, i = _dev(coords), _dev(ids)
        n = C.c_int64()
        _check(lib().pkd_batch_delete_tree(self.h, tree, _stream(stream), _ptr(c), _ptr(i), i.shape[0],
                                           C.byref(n)), "pkd_batch_delete")
        return n.value

    def export(self, t: int = 0):
        """Canonical pre-order form of tree t: rows [N,4] (kind, dim, x, size),
        leaf ids (ascending inside each leaf) and their coordinates [D, n]; numpy."""
        N, n = C.c_int64(), C.c_int64()
        _check(lib().pkd_export_tree_sizes(self.h, t, C.byref(N), C.byref(n)), "pkd_export_sizes")
        rows = np.empty((N.value, 4), dtype=np.int64)
        ids = np.empty(n.value, dtype=np.int64)
        coords = np.empty((self.p.dim, n.value), dtype=np.int64)
        depths = np.empty(N.value, dtype=np.int32)
        _check(lib().pkd_export_tree(self.h, t, rows.ctypes.data_as(C.c_void_p), ids.ctypes.data_as(C.c_void_p),
                                     coords.ctypes.data_as(C.c_void_p), depths.ctypes.data_as(C.c_void_p)),
               "pkd_export")
        self.last_depths = depths
        return rows, ids, coords


class BuildPlan:
    """A batch build enqueued without host reads (pkd_build_plan_*): create it
    for fixed tree sizes, enqueue builds (also inside a captured graph), call
    finish() after each, then query tree().  finish() returns True when the
    build had to be redone the usual way (the tree is the same)."""

    def __init__(self, params: Params, offsets, tile: int = 2048, cand_bias: int = 0):
        self.p = params
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        h = C.c_void_p()
        _check(lib().pkd_build_plan_create(C.byref(params._c()), C.byref(_tuning(tile, cand_bias)),
                                           self.offsets.shape[0] - 1, self.offsets.ctypes.data_as(C.c_void_p),
                                           C.byref(h)), "pkd_build_plan_create")
        self.h = h
        t = C.c_void_p()
        _check(lib().pkd_build_plan_tree(self.h, C.byref(t)), "pkd_build_plan_tree")
        self._tree = Tree(params, None, None, _handle=t)
        self._tree._borrowed = True

    def enqueue(self, coords, ids, stream=None):
        """Enqueue one build over device buffers (kept alive by the caller)."""
        assert tuple(coords.shape) == (self.p.dim, int(self.offsets[-1])) and coords.is_contiguous()
        _check(lib().pkd_build_plan_enqueue(self.h, _stream(stream), _ptr(coords), _ptr(ids)),
               "pkd_build_plan_enqueue")

    def finish(self, stream=None) -> bool:
        redone = C.c_int32(0)
        _check(lib().pkd_build_plan_finish(self.h, _stream(stream), C.byref(redone)), "pkd_build_plan_finish")
        return bool(redone.value)

    def tree(self) -> Tree:
        return self._tree

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._tree.h = None
            lib().pkd_build_plan_free(self.h)
        self.h = None

    def __del__(self):
        self.free()
