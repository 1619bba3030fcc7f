"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws numbers: it holds none of the kd-tree method's arithmetic
(no sampling key, no split rule, no sieve).  Every array is produced by numpy's
PCG64 generator from an explicit seed, so both sides of a parity test receive the
very same bytes.

Layouts
-------
* points: ``coords`` is int64 ``[D, n]`` (structure of arrays, C-contiguous),
  ``ids`` is int64 ``[n]`` = ``id_base + arange(n)`` (generation order).
* queries: int64 ``[D, nq]``.
* boxes: ``lo`` and ``hi`` int64 ``[D, nb]``, closed boxes ``lo <= p <= hi``.

Workload shapes follow the paper's synthetic sets (Section 6, "Datasets"):
``Uniform`` draws points uniformly in a box; ``Varden`` is a clustered random
walk whose generator is not available here, so :func:`clustered_points` stands
in for it (random walks around uniform centres, step lengths log-uniform so that
densities differ by orders of magnitude).
"""
from __future__ import annotations

import numpy as np

COORD_LIMIT = 1 << 30          # coordinates live in [0, 2^30)
DEFAULT_RANGE = 10 ** 9        # the paper-shaped workloads draw from [0, 1e9)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(n: int, dim: int, seed: int, hi: int = DEFAULT_RANGE,
                   id_base: int = 0):
    """n points uniform in [0, hi)^dim; ids id_base .. id_base+n-1."""
    rng = _rng(seed)
    coords = np.empty((dim, n), dtype=np.int64)
    for d in range(dim):            # one row at a time keeps peak memory at 1x
        coords[d] = rng.integers(0, hi, size=n, dtype=np.int64)
    ids = np.arange(id_base, id_base + n, dtype=np.int64)
    return coords, ids


def _fold(y: np.ndarray, hi: int) -> np.ndarray:
    """Map an unreflected walk onto [0, hi) as if it bounced off 0 and hi-1.

    Reflecting after every step equals folding the free walk once, provided no
    single step is longer than hi-1.
    """
    period = 2 * (hi - 1)
    t = np.mod(y, period)
    return np.where(t <= hi - 1, t, period - t)


def clustered_points(n: int, dim: int, seed: int, n_clusters: int = 1000,
                     hi: int = DEFAULT_RANGE, step_lo: float = 1.0,
                     step_hi: float = 1e6, id_base: int = 0,
                     continue_from=None):
    """Clustered random walks (stand-in for the paper's Varden set).

    ``n_clusters`` centres are uniform in the box; cluster c draws a step length
    L_c log-uniform in [step_lo, step_hi] (integer >= 1) and walks ``n //
    n_clusters`` steps (the first clusters take one extra point when n does not
    divide), each coordinate moving by U{-L_c..L_c} and reflecting at the box
    faces.  Points are emitted cluster by cluster in walk order.

    ``continue_from`` = (state, steps) returned by a previous call lets a batch
    continue the same walks (fresh points near the old ones); returns
    ``coords, ids, state`` where state = (last positions [dim, C], L [C]).
    """
    rng = _rng(seed)
    if continue_from is None:
        start = rng.integers(0, hi, size=(dim, n_clusters), dtype=np.int64)
        u = rng.random(n_clusters)
        L = np.maximum(1, np.floor(np.exp(np.log(step_lo) + u * (np.log(step_hi) - np.log(step_lo))))).astype(np.int64)
    else:
        start, L = continue_from
        start = np.asarray(start, dtype=np.int64)
        L = np.asarray(L, dtype=np.int64)
        n_clusters = L.shape[0]
    per = np.full(n_clusters, n // n_clusters, dtype=np.int64)
    per[: n % n_clusters] += 1
    coords = np.empty((dim, n), dtype=np.int64)
    last = np.empty((dim, n_clusters), dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(per)])
    for d in range(dim):
        steps = rng.integers(-1 << 40, 1 << 40, size=n, dtype=np.int64)
        # U{-L..L} per cluster: reduce a wide uniform draw modulo 2L+1.
        Lrep = np.repeat(L, per)
        steps = np.mod(steps, 2 * Lrep + 1) - Lrep
        for c in range(n_clusters):
            a, b = offs[c], offs[c + 1]
            if a == b:
                last[d, c] = start[d, c]
                continue
            walk = start[d, c] + np.cumsum(steps[a:b])
            coords[d, a:b] = _fold(walk, hi)
            last[d, c] = walk[-1]
        del steps, Lrep
    ids = np.arange(id_base, id_base + n, dtype=np.int64)
    # the state keeps the unfolded positions so a continuation folds identically
    return coords, ids, (last, L)


def duplicate_heavy_points(n: int, dim: int, seed: int, n_distinct: int,
                           hi: int = DEFAULT_RANGE, id_base: int = 0,
                           hot_fraction: float = 0.0):
    """Points drawn from only ``n_distinct`` locations (many exact duplicates).

    With ``hot_fraction`` > 0 that share of the points sits on one single
    location, which makes samples that are entirely identical while the whole
    set is not.
    """
    rng = _rng(seed)
    base = rng.integers(0, hi, size=(dim, n_distinct), dtype=np.int64)
    pick = rng.integers(0, n_distinct, size=n, dtype=np.int64)
    if hot_fraction > 0:
        hot = rng.random(n) < hot_fraction
        pick[hot] = 0
    coords = np.ascontiguousarray(base[:, pick])
    ids = np.arange(id_base, id_base + n, dtype=np.int64)
    return coords, ids


def uniform_queries(nq: int, dim: int, seed: int, hi: int = DEFAULT_RANGE):
    """nq query points uniform in [0, hi)^dim, int64 [dim, nq]."""
    rng = _rng(seed)
    q = np.empty((dim, nq), dtype=np.int64)
    for d in range(dim):
        q[d] = rng.integers(0, hi, size=nq, dtype=np.int64)
    return q


def log_uniform_boxes(nb: int, dim: int, seed: int, side_lo: float = 1e5,
                      side_hi: float = 1e8, hi: int = DEFAULT_RANGE):
    """Axis-aligned closed boxes whose side lengths are log-uniform.

    Per box and dimension: side L = floor(exp(U * ln(side_hi/side_lo)) * side_lo)
    (independent per dimension), lo uniform in [0, hi - L], hi = lo + L - 1.
    """
    rng = _rng(seed)
    lo = np.empty((dim, nb), dtype=np.int64)
    up = np.empty((dim, nb), dtype=np.int64)
    for d in range(dim):
        u = rng.random(nb)
        side = np.floor(np.exp(u * np.log(side_hi / side_lo)) * side_lo).astype(np.int64)
        side = np.clip(side, 1, hi)
        lo[d] = rng.integers(0, hi - side + 1, dtype=np.int64)
        up[d] = lo[d] + side - 1
    return lo, up


def report_boxes(nb: int, dim: int, n: int, seed: int, out_lo: float = 1e4, out_hi: float = 1e6,
                 hi: int = DEFAULT_RANGE):
    """Cubes whose expected number of points of n uniform points in [0, hi)^dim
    is log-uniform in [out_lo, out_hi] (the range-report workload: outputs of
    1e4..1e6 points).  Per box: target t = exp(U * ln(out_hi/out_lo)) * out_lo,
    side L = floor(hi * (t/n)^(1/dim)) clipped to [1, hi], then per dimension
    lo uniform in [0, hi - L], hi = lo + L - 1."""
    rng = _rng(seed)
    t = np.exp(rng.random(nb) * np.log(out_hi / out_lo)) * out_lo
    side = np.clip(np.floor(hi * (t / float(n)) ** (1.0 / dim)).astype(np.int64), 1, hi)
    lo = np.empty((dim, nb), dtype=np.int64)
    up = np.empty((dim, nb), dtype=np.int64)
    for d in range(dim):
        lo[d] = rng.integers(0, hi - side + 1, dtype=np.int64)
        up[d] = lo[d] + side - 1
    return lo, up


def sample_existing(ids: np.ndarray, m: int, seed: int) -> np.ndarray:
    """m distinct positions chosen uniformly without replacement from ids."""
    rng = _rng(seed)
    return np.sort(rng.choice(ids.shape[0], size=m, replace=False))


def log_uniform_sizes(count: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """``count`` integers log-uniform in [lo, hi]."""
    rng = _rng(seed)
    u = rng.random(count)
    return np.floor(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.int64)


# --------------------------------------------------------------- hashed points
# For very large resident sets (the serving workload holds 1e9 points) the
# coordinates of a point are a function of its id, so a stream generator can
# name the points it deletes without holding a host copy of the set, and the
# GPU can generate the initial set in place.  The function is MurmurHash3's
# 64-bit finaliser (fmix64) over (id, dimension, seed); the top 63 bits of the
# hash, reduced modulo hi, give the coordinate (the bias of the reduction is
# below hi / 2^63).
_FM1 = 0xFF51AFD7ED558CCD
_FM2 = 0xC4CEB9FE1A85EC53
_SEED_MUL = 0xD6E8FEB86659FD93
_M64 = (1 << 64) - 1


def _fmix64_np(h: np.ndarray) -> np.ndarray:
    h = h ^ (h >> np.uint64(33))
    h = h * np.uint64(_FM1)
    h = h ^ (h >> np.uint64(33))
    h = h * np.uint64(_FM2)
    return h ^ (h >> np.uint64(33))


def hashed_points(ids: np.ndarray, dim: int, seed: int, hi: int = DEFAULT_RANGE) -> np.ndarray:
    """Coordinates [dim, m] of the points with the given ids (see above)."""
    ids = np.asarray(ids, dtype=np.int64).astype(np.uint64)
    salt = np.uint64((seed * _SEED_MUL) & _M64)
    out = np.empty((dim, ids.shape[0]), dtype=np.int64)
    with np.errstate(over="ignore"):
        for d in range(dim):
            h = _fmix64_np((ids << np.uint64(3)) + np.uint64(d) + salt)
            out[d] = ((h >> np.uint64(1)) % np.uint64(hi)).astype(np.int64)
    return out


def hashed_points_torch(ids, dim: int, seed: int, hi: int = DEFAULT_RANGE):
    """The same coordinates as :func:`hashed_points`, computed with torch int64
    ops on the device of `ids` (two's-complement wrap-around; logical right
    shifts by masking)."""
    import torch

    def s64(v):                      # an unsigned 64-bit constant as int64
        return v - (1 << 64) if v >= (1 << 63) else v

    def shr(h, s):
        return (h >> s) & ((1 << (64 - s)) - 1)

    ids = ids.to(torch.int64)
    salt = s64((seed * _SEED_MUL) & _M64)
    out = torch.empty((dim, ids.shape[0]), dtype=torch.int64, device=ids.device)
    for d in range(dim):
        h = (ids << 3) + (d + salt)
        h = h ^ shr(h, 33)
        h = h * s64(_FM1)
        h = h ^ shr(h, 33)
        h = h * s64(_FM2)
        h = h ^ shr(h, 33)
        out[d] = torch.remainder(shr(h, 1), hi)
    return out


def request_stream(dim: int, n_requests: int, seed: int, rate_hz: float, n_initial: int,
                   point_seed: int, insert_range=(1e3, 1e7), query_range=(1e2, 1e6),
                   mix=(1, 1, 8), k_choices=(1, 10, 100), hi: int = DEFAULT_RANGE):
    """A Poisson stream of requests against a resident set whose points are
    ``hashed_points(arange(n_initial), dim, point_seed)``.

    Kinds insert / delete / k-NN in the ratio `mix`; update sizes log-uniform
    in `insert_range`, query batch sizes log-uniform in `query_range`, k
    uniform in `k_choices`.  Inserts take fresh ids (from n_initial upward,
    coordinates by the same hash); deletes pick ids uniformly among those
    present at their position in the stream.  Inter-arrival times are
    exponential with mean 1/rate_hz.  Returns a list of dicts with keys seq,
    kind, arrival, coords ([dim, m] int64), ids (updates) and k (k-NN)."""
    rng = _rng(seed)
    p = np.asarray(mix, dtype=float) / float(sum(mix))
    alive = np.ones(n_initial, dtype=bool)
    alive_count = n_initial
    next_id = n_initial
    t = 0.0
    out = []

    def log_size(lo, hi_):
        return int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi_)))))

    for s in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        kind = ("insert", "delete", "knn")[int(rng.choice(3, p=p))]
        if kind == "knn":
            m = log_size(*query_range)
            q = np.empty((dim, m), dtype=np.int64)
            for d in range(dim):
                q[d] = rng.integers(0, hi, size=m, dtype=np.int64)
            out.append(dict(seq=s, kind=kind, arrival=t, coords=q, ids=None,
                            k=int(k_choices[int(rng.integers(0, len(k_choices)))])))
            continue
        m = log_size(*insert_range)
        if kind == "insert":
            ids = np.arange(next_id, next_id + m, dtype=np.int64)
            next_id += m
            grow = next_id - alive.shape[0]
            if grow > 0:
                alive = np.concatenate([alive, np.zeros(max(grow, alive.shape[0] // 8), dtype=bool)])
            alive[ids] = True
            alive_count += m
        else:
            m = min(m, alive_count)
            picked = np.zeros(0, dtype=np.int64)
            while picked.shape[0] < m:          # rejection: uniform over the live ids
                want = m - picked.shape[0]
                cand = rng.integers(0, next_id, size=2 * want + 16, dtype=np.int64)
                cand = cand[alive[cand]]
                cand = np.unique(cand)
                cand = rng.permutation(cand)[:want]
                alive[cand] = False
                picked = np.concatenate([picked, cand])
            ids = picked
            alive_count -= m
        out.append(dict(seq=s, kind=kind, arrival=t, coords=hashed_points(ids, dim, point_seed, hi), ids=ids, k=0))
    return out
