"""Structural checks on an exported kd-tree (the canonical pre-order form).

Export format (shared by the oracle and the GPU library's export):
  rows   int64 [N, 4]: (kind, dim, x, size) in pre-order; kind 0 = interior,
         1 = leaf; a leaf holds `size` points.
  ids    int64 [n]: leaf point ids, leaves in pre-order, ascending per leaf.
  coords int64 [D, n]: the coordinates of those points.

The checks restate the paper's definitions (Section 2): every point lies on the
correct side of every ancestor's splitter (coordinate < x on the left), stored
subtree sizes equal the true counts, leaves hold at most phi points unless all
their points are identical (a heavy leaf, Appendix C), and no point is lost or
duplicated.
"""
from __future__ import annotations

import numpy as np

COORD_MAX = (1 << 30) - 1


def parse(rows):
    """Return per-node (start, parent, is_left) arrays and the leaf list."""
    N = rows.shape[0]
    start = np.zeros(N, dtype=np.int64)
    parent = np.full(N, -1, dtype=np.int64)
    left_child = np.full(N, -1, dtype=np.int64)
    right_child = np.full(N, -1, dtype=np.int64)
    kind = rows[:, 0]
    size = rows[:, 3]
    # iterative pre-order parse: a stack of (interior node, children seen)
    stack = []
    pos = 0
    for i in range(N):
        if stack:
            p = stack[-1]
            parent[i] = p
            if left_child[p] < 0:
                left_child[p] = i
                start[i] = start[p]
            else:
                right_child[p] = i
                start[i] = start[p] + size[left_child[p]]
                stack.pop()
        else:
            assert i == 0, "more than one root in the export"
        if kind[i] == 0:
            stack.append(i)
        else:
            assert start[i] == pos, "leaf ranges are not consecutive"
            pos += size[i]
    assert not stack, "truncated pre-order export"
    return start, parent, left_child, right_child


def check_tree(rows, ids, coords, phi, in_coords=None, in_ids=None, lam=None):
    rows = np.asarray(rows)
    N = rows.shape[0]
    D = coords.shape[0]
    n = ids.shape[0]
    kind, dim, x, size = rows[:, 0], rows[:, 1], rows[:, 2], rows[:, 3]
    assert N >= 1
    assert size[0] == n, "root size %d != number of exported points %d" % (size[0], n)
    start, parent, lc, rc = parse(rows)
    interior = np.nonzero(kind == 0)[0]
    leaves = np.nonzero(kind == 1)[0]
    # sizes add up and children are non-empty
    assert np.all(size[interior] == size[lc[interior]] + size[rc[interior]]), "size mismatch"
    if N > 1:
        assert np.all(size[interior] >= 2)
        assert np.all(size[leaves] >= 1), "empty leaf below the root"
    assert np.all((dim[interior] >= 0) & (dim[interior] < D))
    # cells top-down (pre-order guarantees parents come first)
    lo = np.zeros((N, D), dtype=np.int64)
    hi = np.full((N, D), COORD_MAX, dtype=np.int64)
    for i in range(1, N):
        p = parent[i]
        lo[i] = lo[p]
        hi[i] = hi[p]
        if lc[p] == i:
            hi[i, dim[p]] = x[p] - 1
        else:
            lo[i, dim[p]] = x[p]
    # every leaf's points inside its cell; leaf size <= phi unless identical
    ls = start[leaves]
    lsz = size[leaves]
    nonempty = lsz > 0
    if np.any(nonempty):
        st = ls[nonempty]
        for d in range(D):
            mn = np.minimum.reduceat(coords[d], st)
            mx = np.maximum.reduceat(coords[d], st)
            L = leaves[nonempty]
            assert np.all(mn >= lo[L, d]) and np.all(mx <= hi[L, d]), "point outside its cell (dim %d)" % d
            big = lsz[nonempty] > phi
            assert np.all(mn[big] == mx[big]), "leaf larger than phi with distinct points"
    # ids ascending inside each leaf (canonical form)
    if n > 1:
        seg = np.repeat(np.arange(leaves.shape[0]), lsz)
        same_leaf = seg[1:] == seg[:-1]
        assert np.all(ids[1:][same_leaf] > ids[:-1][same_leaf]), "ids not ascending inside a leaf"
    # nothing lost or duplicated
    if in_ids is not None:
        order = np.argsort(ids, kind="stable")
        assert np.array_equal(ids[order], np.sort(in_ids)), "id multiset differs from the input"
        ref = np.argsort(in_ids, kind="stable")
        assert np.array_equal(coords[:, order], in_coords[:, ref]), "coordinates do not match their ids"
    return dict(start=start, parent=parent, lc=lc, rc=rc, lo=lo, hi=hi)


def height(rows):
    start, parent, lc, rc = parse(rows)
    depth = np.zeros(rows.shape[0], dtype=np.int64)
    for i in range(1, rows.shape[0]):
        depth[i] = depth[parent[i]] + 1
    return int(depth.max()), depth
