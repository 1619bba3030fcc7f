"""What a batch update must do to a tree, restated from the paper node by node.

BatchInsert (Algorithm 2, Section 4.1) and BatchDelete (Section 4.2) walk the
tree top-down.  At an interior node t that the batch reaches, with l' and n'
the sizes of t's left subtree and of t after the update, t keeps its splitter
and takes size n' if Balanced(l', n') (0.5 - alpha <= l'/n' <= 0.5 + alpha,
Section 2); otherwise t is replaced by Build of its points after the update, at
t's depth.  A leaf that receives points becomes Build(leaf + points); a leaf
that loses points keeps the rest.  A subtree the batch does not reach stays as
it is.  A delete entry removes the stored point with the same id and the same
coordinates in the leaf its coordinates route to.

This module works on the canonical pre-order export (rows (kind, dim, x, size),
leaf ids ascending per leaf, their coordinates) and is written independently of
the oracle's update code: given the tree before a batch it returns the export
the tree must have after it, calling the oracle only for fresh Builds, which
other tests pin.  It also returns the points of every rebuilt subtree, so the
amortized rebuild volume can be checked against the update theorem.
"""
from __future__ import annotations

import numpy as np

from tests import treecheck


def balanced(l: int, n: int, alpha) -> bool:
    num, den = alpha
    return n > 0 and (den - 2 * num) * n <= 2 * den * l <= (den + 2 * num) * n


class _Old:
    def __init__(self, export):
        self.rows, self.ids, self.coords = export
        self.start, self.parent, self.lc, self.rc = treecheck.parse(self.rows)
        N = self.rows.shape[0]
        self.depth = np.zeros(N, dtype=np.int64)
        for i in range(1, N):
            self.depth[i] = self.depth[self.parent[i]] + 1
        # subtree node counts (pre-order: the subtree of i is rows[i : i + cnt[i]])
        self.cnt = np.ones(N, dtype=np.int64)
        for i in range(N - 1, -1, -1):
            if self.rows[i, 0] == 0:
                self.cnt[i] = 1 + self.cnt[self.lc[i]] + self.cnt[self.rc[i]]

    def pts(self, i):
        a = self.start[i]
        b = a + self.rows[i, 3]
        return a, b


class _Out:
    def __init__(self, D):
        self.rows, self.ids, self.coords = [], [], []
        self.D = D
        self.rebuilt = []        # (kind 'interior' | 'leaf', points, depth)

    def verbatim(self, old, i):
        self.rows.append(old.rows[i:i + old.cnt[i]])
        a, b = old.pts(i)
        self.ids.append(old.ids[a:b])
        self.coords.append(old.coords[:, a:b])

    def fresh(self, oracle, params, c, ids, depth, kind):
        T = oracle.Tree(params, c, ids, depth=int(depth))
        r, fi, fc = T.export()
        self.rows.append(r)
        self.ids.append(fi)
        self.coords.append(fc)
        self.rebuilt.append((kind, ids.shape[0], int(depth)))

    def row(self, r):
        self.rows.append(np.array([r], dtype=np.int64))

    def leaf(self, ids, coords):
        self.rows.append(np.array([[1, -1, 0, ids.shape[0]]], dtype=np.int64))
        order = np.argsort(ids, kind="stable")
        self.ids.append(ids[order])
        self.coords.append(coords[:, order])

    def result(self):
        return (np.concatenate(self.rows), np.concatenate(self.ids) if self.ids else np.zeros(0, np.int64),
                np.concatenate(self.coords, axis=1) if self.coords else np.zeros((self.D, 0), np.int64))


def expected_insert(oracle, params, export, bc, bi):
    """Export after BatchInsert of points (bc [D, m], bi [m]) into the tree
    whose export is `export`; also the list of rebuilt subtrees."""
    old = _Old(export)
    D = params.dim
    out = _Out(D)

    def rec(i, P):
        if P.shape[0] == 0:
            out.verbatim(old, i)
            return
        a, b = old.pts(i)
        if old.rows[i, 0] == 1:
            c = np.concatenate([old.coords[:, a:b], bc[:, P]], axis=1)
            ids = np.concatenate([old.ids[a:b], bi[P]])
            out.fresh(oracle, params, c, ids, old.depth[i], "leaf")
            return
        d, x = old.rows[i, 1], old.rows[i, 2]
        go_left = bc[d, P] < x
        PL, PR = P[go_left], P[~go_left]
        n2 = old.rows[i, 3] + P.shape[0]
        l2 = old.rows[old.lc[i], 3] + PL.shape[0]
        if balanced(l2, n2, params.alpha):
            out.row((0, d, x, n2))
            rec(old.lc[i], PL)
            rec(old.rc[i], PR)
        else:
            c = np.concatenate([old.coords[:, a:b], bc[:, P]], axis=1)
            ids = np.concatenate([old.ids[a:b], bi[P]])
            out.fresh(oracle, params, c, ids, old.depth[i], "interior")

    rec(0, np.arange(bi.shape[0]))
    return out.result(), out.rebuilt


def matched_points(export, bc, bi):
    """Boolean mask over the exported points: the points a delete batch
    removes (same id and coordinates, in the leaf the coordinates route to;
    a repeated entry removes once)."""
    old = _Old(export)
    marked = np.zeros(old.ids.shape[0], dtype=bool)
    for j in range(bi.shape[0]):
        i = 0
        while old.rows[i, 0] == 0:
            i = old.lc[i] if bc[old.rows[i, 1], j] < old.rows[i, 2] else old.rc[i]
        a, b = old.pts(i)
        for p in range(a, b):
            if old.ids[p] == bi[j] and not marked[p] and np.array_equal(old.coords[:, p], bc[:, j]):
                marked[p] = True
                break
    return marked


def expected_delete(oracle, params, export, bc, bi):
    """Export after BatchDelete of entries (bc, bi); also the number of points
    removed and the list of rebuilt subtrees."""
    old = _Old(export)
    D = params.dim
    marked = matched_points(export, bc, bi)
    csum = np.concatenate([[0], np.cumsum(marked)])
    out = _Out(D)

    def dels(i):
        a, b = old.pts(i)
        return int(csum[b] - csum[a])

    def rec(i):
        if dels(i) == 0:
            out.verbatim(old, i)
            return
        a, b = old.pts(i)
        keep = ~marked[a:b]
        if old.rows[i, 0] == 1:
            out.leaf(old.ids[a:b][keep], old.coords[:, a:b][:, keep])
            return
        n2 = old.rows[i, 3] - dels(i)
        l2 = old.rows[old.lc[i], 3] - dels(old.lc[i])
        if balanced(l2, n2, params.alpha):
            out.row((0, old.rows[i, 1], old.rows[i, 2], n2))
            rec(old.lc[i])
            rec(old.rc[i])
        else:
            out.fresh(oracle, params, np.ascontiguousarray(old.coords[:, a:b][:, keep]),
                      np.ascontiguousarray(old.ids[a:b][keep]), old.depth[i], "interior")

    rec(0)
    return out.result(), int(marked.sum()), out.rebuilt
