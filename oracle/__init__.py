"""ctypes wrapper of the sequential CPU oracle (``pkd_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` are the only callers.  The GPU library never loads
or calls anything here, and nothing here loads the GPU library.

Every function takes and returns numpy arrays; coordinates are int64 ``[D, n]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pkd_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_balanced.restype = C.c_int
        L.orc_balanced.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64]
        L.orc_sample_key.restype = C.c_uint64
        L.orc_sample_key.argtypes = [C.c_uint64, C.c_int64, C.c_int64]
        L.orc_build.restype = C.c_void_p
        L.orc_build.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_uint64,
                                _i64p, _i64p, C.c_int64]
        L.orc_build_at.restype = C.c_void_p
        L.orc_build_at.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_uint64,
                                   _i64p, _i64p, C.c_int64, C.c_int]
        L.orc_update_log.argtypes = [C.c_void_p, _i64p]
        L.orc_knn_threads.argtypes = [C.c_void_p, _i64p, C.c_int64, C.c_int, _i64p, _i64p, C.c_int]
        L.orc_knn_visits.argtypes = [C.c_void_p, _i64p, C.c_int64, C.c_int, _i64p, _i64p, _i64p]
        L.orc_range_report.argtypes = [C.c_void_p, _i64p, _i64p, C.c_int64, _i64p, _i64p]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_size.restype = C.c_int64
        L.orc_size.argtypes = [C.c_void_p]
        L.orc_num_nodes.restype = C.c_int64
        L.orc_num_nodes.argtypes = [C.c_void_p]
        L.orc_height.restype = C.c_int
        L.orc_height.argtypes = [C.c_void_p]
        L.orc_insert.argtypes = [C.c_void_p, _i64p, _i64p, C.c_int64]
        L.orc_delete.restype = C.c_int64
        L.orc_delete.argtypes = [C.c_void_p, _i64p, _i64p, C.c_int64]
        L.orc_knn.argtypes = [C.c_void_p, _i64p, C.c_int64, C.c_int, _i64p, _i64p]
        L.orc_range_count.argtypes = [C.c_void_p, _i64p, _i64p, C.c_int64, _i64p]
        L.orc_export.argtypes = [C.c_void_p, _i64p, _i64p, _i64p]
        L.orc_export_depths.argtypes = [C.c_void_p, _i32p, _i8p]
        L.orc_sample.argtypes = [C.c_uint64, C.c_int64, _i64p, C.c_int64, C.c_int64, _i64p]
        L.orc_split_rule.restype = C.c_int
        L.orc_split_rule.argtypes = [C.c_int, _i64p, C.c_int64, C.POINTER(C.c_int), C.POINTER(C.c_int64)]
        L.orc_skeleton.argtypes = [C.c_int, C.c_int, _i64p, C.c_int64, _i32p, _i64p, _i8p]
        L.orc_sieve.argtypes = [C.c_int, C.c_int, _i32p, _i64p, _i8p, _i64p, C.c_int64, _i32p, _i64p]
        L.orc_root_skeleton.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_int64, _i64p, _i64p,
                                        C.c_int64, _i32p, _i64p, _i8p]
        L.orc_brute_knn.argtypes = [C.c_int, _i64p, _i64p, C.c_int64, _i64p, C.c_int64, C.c_int, _i64p, _i64p]
        L.orc_brute_range_count.argtypes = [C.c_int, _i64p, C.c_int64, _i64p, _i64p, C.c_int64, _i64p]
        _lib = L
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.int64)


class Params:
    """Result-affecting parameters (Section 5 defaults: lambda=6, phi=32,
    sigma=32, alpha=0.3)."""

    def __init__(self, dim, lam=6, phi=32, sigma=32, alpha=(3, 10), seed=42):
        self.dim, self.lam, self.phi, self.sigma = int(dim), int(lam), int(phi), int(sigma)
        self.alpha = (int(alpha[0]), int(alpha[1]))
        self.seed = int(seed)


class Tree:
    """A sequential Pkd-tree held by the oracle library."""

    def __init__(self, params: Params, coords, ids, depth: int = 0):
        """Build(P); `depth` places the root at that depth of an enclosing
        tree (the depth salts the samples, as for a rebuilt node)."""
        coords, ids = _c(coords), _c(ids)
        assert coords.shape == (params.dim, ids.shape[0])
        self.p = params
        self.h = lib().orc_build_at(params.dim, params.lam, params.phi, params.sigma, params.alpha[0],
                                    params.alpha[1], C.c_uint64(params.seed & (2 ** 64 - 1)), coords, ids,
                                    ids.shape[0], int(depth))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def size(self) -> int:
        return lib().orc_size(self.h)

    def num_nodes(self) -> int:
        return lib().orc_num_nodes(self.h)

    def height(self) -> int:
        return lib().orc_height(self.h)

    def insert(self, coords, ids):
        coords, ids = _c(coords), _c(ids)
        lib().orc_insert(self.h, coords, ids, ids.shape[0])

    def delete(self, coords, ids) -> int:
        coords, ids = _c(coords), _c(ids)
        return lib().orc_delete(self.h, coords, ids, ids.shape[0])

    def knn(self, q, k):
        q = _c(q)
        nq = q.shape[1]
        ids = np.empty((nq, k), dtype=np.int64)
        d2 = np.empty((nq, k), dtype=np.int64)
        lib().orc_knn(self.h, q, nq, k, ids, d2)
        return ids, d2

    def knn_threads(self, q, k, threads):
        """knn() with the queries split over `threads` host threads."""
        q = _c(q)
        nq = q.shape[1]
        ids = np.empty((nq, k), dtype=np.int64)
        d2 = np.empty((nq, k), dtype=np.int64)
        lib().orc_knn_threads(self.h, q, nq, k, ids, d2, int(threads))
        return ids, d2

    def knn_visits(self, q, k):
        """Per-query work of the search: (nodes read, leaves scanned, points
        scanned), each int64 [nq]."""
        q = _c(q)
        nq = q.shape[1]
        out = [np.empty(nq, dtype=np.int64) for _ in range(3)]
        lib().orc_knn_visits(self.h, q, nq, k, *out)
        return tuple(out)

    def range_count(self, lo, hi):
        lo, hi = _c(lo), _c(hi)
        out = np.empty(lo.shape[1], dtype=np.int64)
        lib().orc_range_count(self.h, lo, hi, lo.shape[1], out)
        return out

    def range_report(self, lo, hi):
        """(offsets [nb+1], ids): box j's point ids are ids[offsets[j]:offsets[j+1]],
        in the tree's in-order."""
        lo, hi = _c(lo), _c(hi)
        cnt = self.range_count(lo, hi)
        off = np.zeros(cnt.shape[0] + 1, dtype=np.int64)
        np.cumsum(cnt, out=off[1:])
        ids = np.empty(int(off[-1]), dtype=np.int64)
        lib().orc_range_report(self.h, lo, hi, lo.shape[1], off, ids)
        return off, ids

    def update_log(self):
        """What the last insert/delete rebuilt: dict with interior_rebuilds,
        interior_points, leaf_rebuilds, leaf_points, kept."""
        out = np.zeros(5, dtype=np.int64)
        lib().orc_update_log(self.h, out)
        keys = ("interior_rebuilds", "interior_points", "leaf_rebuilds", "leaf_points", "kept")
        return dict(zip(keys, (int(v) for v in out)))

    def export(self):
        """Pre-order canonical form: rows [N,4] = (kind, dim, x, size) with kind
        0 interior / 1 leaf; leaf ids (ascending inside each leaf) and their
        coordinates [D, n]."""
        N = self.num_nodes()
        n = self.size()
        rows = np.empty((N, 4), dtype=np.int64)
        ids = np.empty(n, dtype=np.int64)
        coords = np.empty((self.p.dim, n), dtype=np.int64)
        lib().orc_export(self.h, rows, ids, coords)
        return rows, ids, coords

    def depths(self):
        """Pre-order node depths and plain-split flags (1 = interior node made
        by one exact split, 0 = skeleton node or leaf)."""
        out = np.empty(self.num_nodes(), dtype=np.int32)
        plain = np.empty(self.num_nodes(), dtype=np.int8)
        lib().orc_export_depths(self.h, out, plain)
        return out, plain


def mix64(z: int) -> int:
    return lib().orc_mix64(C.c_uint64(z & (2 ** 64 - 1)))


def balanced(l: int, n: int, alpha=(3, 10)) -> bool:
    return bool(lib().orc_balanced(l, n, alpha[0], alpha[1]))


def sample_key(seed: int, h: int, pid: int) -> int:
    return lib().orc_sample_key(C.c_uint64(seed & (2 ** 64 - 1)), h, pid)


def sample(seed: int, h: int, ids, s: int):
    ids = _c(ids)
    out = np.empty(s, dtype=np.int64)
    lib().orc_sample(C.c_uint64(seed & (2 ** 64 - 1)), h, ids, ids.shape[0], s, out)
    return out


def split_rule(coords):
    coords = _c(coords)
    d = C.c_int(0)
    x = C.c_int64(0)
    rc = lib().orc_split_rule(coords.shape[0], coords, coords.shape[1], C.byref(d), C.byref(x))
    return None if rc != 0 else (d.value, x.value)


def skeleton(coords, lam: int):
    coords = _c(coords)
    dim = np.empty(1 << lam, dtype=np.int32)
    x = np.empty(1 << lam, dtype=np.int64)
    ext = np.empty(2 << lam, dtype=np.int8)
    lib().orc_skeleton(coords.shape[0], lam, coords, coords.shape[1], dim, x, ext)
    return dim, x, ext


def sieve(coords, lam: int, sk):
    coords = _c(coords)
    dim, x, ext = sk
    n = coords.shape[1]
    labels = np.empty(n, dtype=np.int32)
    order = np.empty(n, dtype=np.int64)
    lib().orc_sieve(coords.shape[0], lam, np.ascontiguousarray(dim, dtype=np.int32), _c(x),
                    np.ascontiguousarray(ext, dtype=np.int8), coords, n, labels, order)
    return labels, order


def root_skeleton(params: Params, coords, ids, h: int = 0):
    coords, ids = _c(coords), _c(ids)
    lam = params.lam
    dim = np.empty(1 << lam, dtype=np.int32)
    x = np.empty(1 << lam, dtype=np.int64)
    ext = np.empty(2 << lam, dtype=np.int8)
    lib().orc_root_skeleton(params.dim, lam, params.sigma, C.c_uint64(params.seed & (2 ** 64 - 1)), h,
                            coords, ids, ids.shape[0], dim, x, ext)
    return dim, x, ext


def brute_knn(coords, ids, q, k):
    coords, ids, q = _c(coords), _c(ids), _c(q)
    nq = q.shape[1]
    oi = np.empty((nq, k), dtype=np.int64)
    od = np.empty((nq, k), dtype=np.int64)
    lib().orc_brute_knn(coords.shape[0], coords, ids, ids.shape[0], q, nq, k, oi, od)
    return oi, od


def brute_range_count(coords, lo, hi):
    coords, lo, hi = _c(coords), _c(lo), _c(hi)
    out = np.empty(lo.shape[1], dtype=np.int64)
    lib().orc_brute_range_count(coords.shape[0], coords, coords.shape[1], lo, hi, lo.shape[1], out)
    return out
