"""CPU oracle for the kNN and friends-of-friends results (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It is a plain, slow, obviously correct
implementation of what the GPU library computes, written from the paper's
problem statements and sharing no code with the GPU library:

* ``knn_bf`` / ``fof_bf``: the definitions written out (all pairs).
* ``knn_kd`` / ``fof_kd``: exact kd-tree accelerations for large inputs, pinned
  bit-for-bit to the brute-force versions by the tests.
* ``knn_cross_bf`` / ``knn_cross_kd``: kNN of separate query points among
  source points (the paper's multiple point types).
* ``knn_bf_periodic`` / ``fof_bf_periodic`` (and ``*_kd_periodic``): the same
  in a periodic cube with the minimum-image distance (each coordinate
  difference moved by one period when beyond half of it).
* ``KdTree``: the kd-tree of ``knn_kd`` kept between calls, answering row
  ranges, so that a result too large for host memory is compared in chunks.
* ``components_uf`` / ``components_bfs``: two independent component labelings
  of an explicit edge list.
* ``knn_f64_report`` / ``fof_f64_report``: binary64 cross-checks (reports, not
  gates) that list the kNN rows and count the FoF pairs whose decision flips
  between the fixed float32 expression and the same expression in binary64.
* :mod:`oracle.planes`: the tree-plane construction of the paper's section on
  the plane-based hierarchy (gap levels, node sizes, split selection), pinned to
  the paper's worked example (Fig. 3).

Fixed arithmetic (the paper fixes only float32 precision; this reading is shared
with the GPU side): ``dist2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz))`` with
``dx = fl(x_i - x_j)`` etc., IEEE binary32, no FMA, subnormals kept. kNN rows
are ordered by (dist2, index); FoF links pairs with ``dist2 <= fl(b*b)``;
labels are the smallest member index.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)


def default_threads() -> int:
    """Threads for the oracle: the process's CPU share, capped by OMP_NUM_THREADS."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB) or (
            os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    lib.jzo_knn_bf.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, _i64p, ctypes.c_int64,
                               _i32p, _f32p, ctypes.c_int]
    lib.jzo_knn_kd.argtypes = lib.jzo_knn_bf.argtypes
    lib.jzo_fof_bf.argtypes = [_f32p, ctypes.c_int64, ctypes.c_float, _i32p, ctypes.c_int]
    lib.jzo_fof_kd.argtypes = lib.jzo_fof_bf.argtypes
    lib.jzo_components_uf.argtypes = [ctypes.c_int64, _i32p, ctypes.c_int64, _i32p]
    lib.jzo_components_bfs.argtypes = lib.jzo_components_uf.argtypes
    lib.jzo_range_rows_bf.argtypes = [_f32p, ctypes.c_int64, ctypes.c_float, _i64p,
                                      ctypes.c_int64, ctypes.c_int64, _i64p, _i32p,
                                      ctypes.c_int]
    lib.jzo_kd_new.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int]
    lib.jzo_kd_new.restype = ctypes.c_void_p
    lib.jzo_kd_knn.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, ctypes.c_int64,
                               ctypes.c_int64, _i32p, _f32p, ctypes.c_int]
    lib.jzo_kd_free.argtypes = [ctypes.c_void_p]
    lib.jzo_kd_free.restype = None
    lib.jzo_fof_f64_report.argtypes = [_f32p, ctypes.c_int64, ctypes.c_float, _i64p, _i64p,
                                       _i32p, ctypes.c_int]
    lib.jzo_knn_cross_bf.argtypes = [_f32p, ctypes.c_int64, _f32p, ctypes.c_int64, ctypes.c_int,
                                     _i32p, _f32p, ctypes.c_int]
    lib.jzo_knn_cross_kd.argtypes = lib.jzo_knn_cross_bf.argtypes
    lib.jzo_knn_bf_per.argtypes = [_f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_int, _i64p,
                                   ctypes.c_int64, _i32p, _f32p, ctypes.c_int]
    lib.jzo_knn_kd_per.argtypes = lib.jzo_knn_bf_per.argtypes
    lib.jzo_fof_bf_per.argtypes = [_f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_float, _i32p,
                                   ctypes.c_int]
    lib.jzo_fof_kd_per.argtypes = lib.jzo_fof_bf_per.argtypes
    for f in ("jzo_knn_bf", "jzo_knn_kd", "jzo_fof_bf", "jzo_fof_kd", "jzo_components_uf",
              "jzo_components_bfs", "jzo_range_rows_bf", "jzo_kd_knn", "jzo_fof_f64_report",
              "jzo_knn_cross_bf", "jzo_knn_cross_kd", "jzo_knn_bf_per", "jzo_knn_kd_per",
              "jzo_fof_bf_per", "jzo_fof_kd_per"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _pts(points) -> np.ndarray:
    p = np.ascontiguousarray(points, dtype=np.float32)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("points must have shape (n, 3)")
    return p


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _knn(fn, points, k, rows, threads):
    p = _pts(points)
    n = p.shape[0]
    if rows is None:
        r = None
        nr = n
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        nr = r.shape[0]
    idx = np.empty((nr, k), dtype=np.int32)
    d2 = np.empty((nr, k), dtype=np.float32)
    rc = fn(_ptr(p, _f32p), n, int(k), None if r is None else _ptr(r, _i64p), nr,
            _ptr(idx, _i32p), _ptr(d2, _f32p), threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle kNN failed (%d)" % rc)
    return idx, d2


def knn_bf(points, k: int, rows=None, threads: int = 0):
    """Brute-force kNN: (idx [r, k] int32, dist2 [r, k] float32) for all or given rows."""
    return _knn(_load().jzo_knn_bf, points, k, rows, threads)


def knn_kd(points, k: int, rows=None, threads: int = 0):
    """Exact kd-tree kNN; same output as :func:`knn_bf`."""
    return _knn(_load().jzo_knn_kd, points, k, rows, threads)


def _cross(fn, sources, queries, k, threads):
    s = _pts(sources)
    q = _pts(queries)
    idx = np.empty((q.shape[0], k), dtype=np.int32)
    d2 = np.empty((q.shape[0], k), dtype=np.float32)
    rc = fn(_ptr(s, _f32p), s.shape[0], _ptr(q, _f32p), q.shape[0], int(k), _ptr(idx, _i32p),
            _ptr(d2, _f32p), threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle cross kNN failed (%d)" % rc)
    return idx, d2


def knn_cross_bf(sources, queries, k: int, threads: int = 0):
    """Brute-force kNN of separate query points among source points:
    (idx [nq, k] source indices, dist2 [nq, k]), ascending (dist2, index)."""
    return _cross(_load().jzo_knn_cross_bf, sources, queries, k, threads)


def knn_cross_kd(sources, queries, k: int, threads: int = 0):
    """Exact kd-tree version of :func:`knn_cross_bf` (same output)."""
    return _cross(_load().jzo_knn_cross_kd, sources, queries, k, threads)


def _knn_per(fn, points, period, k, rows, threads):
    p = _pts(points)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = p.shape[0] if r is None else r.shape[0]
    idx = np.empty((nr, k), dtype=np.int32)
    d2 = np.empty((nr, k), dtype=np.float32)
    rc = fn(_ptr(p, _f32p), p.shape[0], float(np.float32(period)), int(k),
            None if r is None else _ptr(r, _i64p), nr, _ptr(idx, _i32p), _ptr(d2, _f32p),
            threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle periodic kNN failed (%d)" % rc)
    return idx, d2


def knn_bf_periodic(points, period: float, k: int, rows=None, threads: int = 0):
    """:func:`knn_bf` in the periodic cube [0, period)^3 (minimum image)."""
    return _knn_per(_load().jzo_knn_bf_per, points, period, k, rows, threads)


def knn_kd_periodic(points, period: float, k: int, rows=None, threads: int = 0):
    """Exact kd-tree version of :func:`knn_bf_periodic` (same output)."""
    return _knn_per(_load().jzo_knn_kd_per, points, period, k, rows, threads)


def _fof_per(fn, points, period, b, threads):
    p = _pts(points)
    lab = np.empty(p.shape[0], dtype=np.int32)
    rc = fn(_ptr(p, _f32p), p.shape[0], float(np.float32(period)), float(np.float32(b)),
            _ptr(lab, _i32p), threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle periodic FoF failed (%d)" % rc)
    return lab


def fof_bf_periodic(points, period: float, b: float, threads: int = 0) -> np.ndarray:
    """:func:`fof_bf` in the periodic cube [0, period)^3 (minimum image)."""
    return _fof_per(_load().jzo_fof_bf_per, points, period, b, threads)


def fof_kd_periodic(points, period: float, b: float, threads: int = 0) -> np.ndarray:
    """Exact kd-tree version of :func:`fof_bf_periodic` (same output)."""
    return _fof_per(_load().jzo_fof_kd_per, points, period, b, threads)


def dist2_f32_periodic(p, q, period: float) -> np.ndarray:
    """The periodic distance of the library, elementwise over broadcast rows."""
    p = np.asarray(p, dtype=np.float32)
    q = np.asarray(q, dtype=np.float32)
    L = np.float32(period)
    h = np.float32(0.5) * L
    d = p - q
    d = np.where(d > h, d - L, np.where(d < -h, d + L, d)).astype(np.float32)
    xx = d[..., 0] * d[..., 0]
    yy = d[..., 1] * d[..., 1]
    zz = d[..., 2] * d[..., 2]
    return (xx + yy) + zz


def _fof(fn, points, b, threads):
    p = _pts(points)
    lab = np.empty(p.shape[0], dtype=np.int32)
    rc = fn(_ptr(p, _f32p), p.shape[0], float(np.float32(b)), _ptr(lab, _i32p),
            threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle FoF failed (%d)" % rc)
    return lab


def fof_bf(points, b: float, threads: int = 0) -> np.ndarray:
    """Brute-force FoF labels (min member index), int32 [n]."""
    return _fof(_load().jzo_fof_bf, points, b, threads)


def fof_kd(points, b: float, threads: int = 0) -> np.ndarray:
    """Exact kd-tree FoF labels; same output as :func:`fof_bf`."""
    return _fof(_load().jzo_fof_kd, points, b, threads)


def _components(fn, n, edges):
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    lab = np.empty(n, dtype=np.int32)
    rc = fn(n, _ptr(e, _i32p), e.shape[0], _ptr(lab, _i32p))
    if rc != 0:
        raise RuntimeError("oracle components failed (%d)" % rc)
    return lab


def components_uf(n: int, edges) -> np.ndarray:
    return _components(_load().jzo_components_uf, n, edges)


def components_bfs(n: int, edges) -> np.ndarray:
    return _components(_load().jzo_components_bfs, n, edges)


def range_rows_bf(points, b: float, rows, cap: int = 4096, threads: int = 0):
    """Neighbours within b (inclusive) of the given rows, brute force.

    Returns (counts [r] int64, neighbours [r, cap] int32); a row's first
    ``min(count, cap)`` entries are its neighbour indices in ascending order.
    """
    p = _pts(points)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    cnt = np.empty(r.shape[0], dtype=np.int64)
    nbr = np.full((r.shape[0], cap), -1, dtype=np.int32)
    rc = _load().jzo_range_rows_bf(_ptr(p, _f32p), p.shape[0], float(np.float32(b)),
                                   _ptr(r, _i64p), r.shape[0], cap, _ptr(cnt, _i64p),
                                   _ptr(nbr, _i32p), threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle range search failed (%d)" % rc)
    return cnt, nbr


def dist2_f32(p, q) -> np.ndarray:
    """The fixed float32 distance expression, elementwise over broadcast rows."""
    p = np.asarray(p, dtype=np.float32)
    q = np.asarray(q, dtype=np.float32)
    d = p - q
    xx = d[..., 0] * d[..., 0]
    yy = d[..., 1] * d[..., 1]
    zz = d[..., 2] * d[..., 2]
    return (xx + yy) + zz


class KdTree:
    """An exact kd-tree over a fixed point set, answering kNN rows in ranges.

    ``rows(first, count, k)`` gives the same output as :func:`knn_bf` for rows
    ``first .. first + count - 1``; a large result can so be compared chunk by
    chunk without holding all of it in host memory.
    """

    def __init__(self, points, threads: int = 0):
        self._p = _pts(points)
        self.n = self._p.shape[0]
        self._threads = threads or default_threads()
        self._h = _load().jzo_kd_new(_ptr(self._p, _f32p), self.n, self._threads)
        if not self._h:
            raise RuntimeError("oracle kd-tree build failed")

    def rows(self, first: int, count: int, k: int):
        idx = np.empty((count, k), dtype=np.int32)
        d2 = np.empty((count, k), dtype=np.float32)
        rc = _load().jzo_kd_knn(self._h, int(k), None, int(first), int(count),
                                _ptr(idx, _i32p), _ptr(d2, _f32p), self._threads)
        if rc != 0:
            raise RuntimeError("oracle kd-tree query failed (%d)" % rc)
        return idx, d2

    def select(self, rows, k: int):
        r = np.ascontiguousarray(rows, dtype=np.int64)
        idx = np.empty((r.shape[0], k), dtype=np.int32)
        d2 = np.empty((r.shape[0], k), dtype=np.float32)
        rc = _load().jzo_kd_knn(self._h, int(k), _ptr(r, _i64p), 0, r.shape[0],
                                _ptr(idx, _i32p), _ptr(d2, _f32p), self._threads)
        if rc != 0:
            raise RuntimeError("oracle kd-tree query failed (%d)" % rc)
        return idx, d2

    def close(self):
        if self._h:
            _load().jzo_kd_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()


def knn_f64_report(points, idx, rows=None, margin: int = 4, threads: int = 0):
    """FP64 cross-check of a kNN result (a report, not a gate).

    ``idx`` holds the result rows for ``rows`` (all rows if None). For each
    row the float32 top k plus the next ``margin`` candidates (an exact float32
    kNN row of length k + margin) are re-ranked by (binary64 squared distance,
    index), with the distance evaluated from the float32 coordinates in
    binary64. Returns the positions (into ``rows``) of the rows whose binary64
    top k differs from ``idx`` in membership or order: decisions that flip at
    near-ties of the float32 expression.
    """
    p = _pts(points)
    idx = np.asarray(idx)
    k = idx.shape[1]
    r = np.arange(p.shape[0]) if rows is None else np.asarray(rows, dtype=np.int64)
    if r.shape[0] != idx.shape[0]:
        raise ValueError("idx must have one row per requested row")
    with KdTree(p, threads) as kd:
        ext, _ = kd.select(r, k + margin)
    p64 = p.astype(np.float64)
    flipped = []
    for t in range(r.shape[0]):
        cand = ext[t][ext[t] >= 0]
        dd = p64[cand] - p64[r[t]]
        d = (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]
        order = np.lexsort((cand, d))
        want = cand[order][:k]
        got = idx[t][idx[t] >= 0]
        if want.shape != got.shape or not np.array_equal(want, got):
            flipped.append(t)
    return np.asarray(flipped, dtype=np.int64)


def fof_f64_report(points, b: float, labels=None, threads: int = 0) -> dict:
    """FP64 cross-check of FoF linking (a report, not a gate).

    Counts the pairs i < j where the float32 test ``dist2 <= fl(b*b)`` and the
    binary64 test ``d64 <= b*b`` (both from the same float32 coordinates)
    disagree, and computes the binary64 partition. With ``labels`` (a float32
    result, smallest-member labels) it also reports whether the partition
    changes and how many points change group label.
    """
    p = _pts(points)
    n = p.shape[0]
    o32 = ctypes.c_int64()
    o64 = ctypes.c_int64()
    lab64 = np.empty(n, dtype=np.int32)
    rc = _load().jzo_fof_f64_report(_ptr(p, _f32p), n, float(np.float32(b)), ctypes.byref(o32),
                                    ctypes.byref(o64), _ptr(lab64, _i32p),
                                    threads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle FoF f64 report failed (%d)" % rc)
    out = {"pairs_f32_only": int(o32.value), "pairs_f64_only": int(o64.value),
           "labels_f64": lab64}
    if labels is not None:
        lab = np.asarray(labels)
        moved = int(np.count_nonzero(lab != lab64))
        out["partition_differs"] = moved > 0
        out["points_relabelled"] = moved
    return out


def fof_catalogue(points, labels, min_members: int = 20, velocities=None) -> dict:
    """FoF catalogue reduction (the paper's FoF section, catalogue reduction),
    written out in binary64 with numpy.

    Group order: a stable sort of the input indices by group label, so groups
    follow their labels (the smallest member index) in ascending order and
    each group is one contiguous block of ascending input indices. For every
    group with at least ``min_members`` points, in label order: its label,
    the offset of its block in ``order``, its member count (the mass, at unit
    point mass), the centre of mass (mean position), the inertia radius
    (root-mean-square distance of the members from the centre of mass) and,
    with ``velocities``, the centre-of-mass velocity (mean velocity).
    """
    p = _pts(points).astype(np.float64)
    lab = np.asarray(labels, dtype=np.int64)
    order = np.argsort(lab, kind="stable").astype(np.int32)
    gl, first, count = np.unique(lab[order], return_index=True, return_counts=True)
    keep = count >= min_members
    out = {"order": order, "label": gl[keep].astype(np.int32),
           "first": first[keep].astype(np.int64), "count": count[keep].astype(np.int64)}
    cm = np.zeros((int(keep.sum()), 3))
    r = np.zeros(int(keep.sum()))
    vcm = np.zeros((int(keep.sum()), 3)) if velocities is not None else None
    v = None if velocities is None else np.asarray(velocities, dtype=np.float32).astype(np.float64)
    for g, (f, c) in enumerate(zip(out["first"], out["count"])):
        members = order[f:f + c]
        x = p[members]
        cm[g] = x.sum(axis=0) / c
        d = x - cm[g]
        r[g] = np.sqrt((d * d).sum() / c)
        if v is not None:
            vcm[g] = v[members].sum(axis=0) / c
    out["cm"] = cm
    out["r_inertia"] = r
    if vcm is not None:
        out["vcm"] = vcm
    return out
