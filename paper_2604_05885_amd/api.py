"""Python binding of the C ABI in ``include/jz.h`` (argument marshalling only).

Every step of the method runs in the HIP library ``libjz.so``; this module
passes torch tensor pointers and HIP streams to it. There is no fallback: if
the library is missing or fails to load, the import raises.

Functions keep the C names (``jz_build``, ``jz_knn``, ``jz_fof``, ...);
:class:`Tree` wraps a tree handle with ``knn`` / ``fof`` methods.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

# torch before libjz.so: both need libamdhip64.so.7, and the dynamic loader
# binds a later library to the copy already loaded. Loaded first, libjz.so
# would bind torch to the system HIP runtime instead of the one torch ships
# with, and the library's hipGetDevice then finds no device in a process
# where torch's own calls work.
import torch  # noqa: F401  (load order only)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjz.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "jz.h")

JZ_OK, JZ_E_INVALID, JZ_E_NONFINITE, JZ_E_UNSUPPORTED, JZ_E_CAPACITY, JZ_E_OOM, JZ_E_DEVICE = range(7)
MAX_PLANES = 16


class JzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("jz status %d: %s" % (status, msg))
        self.status = status


class BuildOpts(ctypes.Structure):
    _fields_ = [("leaf_max", ctypes.c_int), ("coarsen", ctypes.c_int), ("n_target", ctypes.c_int),
                ("ngr", ctypes.c_int), ("key_bits", ctypes.c_int),
                ("list_per_node", ctypes.c_float), ("auto_regrow", ctypes.c_int),
                ("keep_keys", ctypes.c_int), ("sort_max", ctypes.c_int),
                ("period", ctypes.c_float), ("reg_fmax", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("planes", ctypes.c_int),
                ("nodes", ctypes.c_int64 * MAX_PLANES), ("super_nodes", ctypes.c_int64),
                ("list_entries", ctypes.c_int64 * (MAX_PLANES + 1)),
                ("leaf_pairs", ctypes.c_int64), ("leaf_pairs_visited", ctypes.c_int64),
                ("evaluations", ctypes.c_double), ("leaf_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("reruns", ctypes.c_int),
                ("insert_rounds", ctypes.c_int64), ("tile_steps", ctypes.c_int64),
                ("lists_sorted_long", ctypes.c_int64), ("lists_unordered", ctypes.c_int64),
                ("lists_presorted", (ctypes.c_int64 * 2) * (MAX_PLANES + 1))]

    def as_dict(self) -> dict:
        P = self.planes
        return {"n": self.n, "planes": P, "nodes": list(self.nodes[:P]),
                "super_nodes": self.super_nodes,
                "list_entries": list(self.list_entries[:P]),
                "leaf_pairs": self.leaf_pairs, "leaf_pairs_visited": self.leaf_pairs_visited,
                "evaluations": self.evaluations, "leaf_ms": self.leaf_ms,
                "total_ms": self.total_ms, "reruns": self.reruns,
                "insert_rounds": self.insert_rounds, "tile_steps": self.tile_steps,
                "lists_sorted_long": self.lists_sorted_long,
                "lists_unordered": self.lists_unordered,
                "lists_presorted_walk": [list(self.lists_presorted[q]) for q in range(max(P - 1, 0))],
                "lists_presorted_leaf": list(self.lists_presorted[MAX_PLANES])}


class Allocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p),
                ("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p))]


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("k", ctypes.c_int), ("b", ctypes.c_float),
                ("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("idx", ctypes.c_void_p),
                ("dist2", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("stream", ctypes.c_void_p)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("streams", ctypes.c_int),
                ("max_batch_points", ctypes.c_int64), ("max_batch_sets", ctypes.c_int),
                ("build", BuildOpts)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("points_done", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("in_flight_bytes", ctypes.c_int64), ("max_batch_sets_seen", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Group(ctypes.Structure):
    _fields_ = [("label", ctypes.c_int32), ("count", ctypes.c_int32), ("first", ctypes.c_int64),
                ("cm", ctypes.c_double * 3), ("vcm", ctypes.c_double * 3),
                ("r_inertia", ctypes.c_double)]


GROUP_DTYPE = np.dtype([("label", np.int32), ("count", np.int32), ("first", np.int64),
                        ("cm", np.float64, 3), ("vcm", np.float64, 3), ("r_inertia", np.float64)])
assert GROUP_DTYPE.itemsize == ctypes.sizeof(Group)

JZ_OP_KNN, JZ_OP_FOF = 0, 1

_vp = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_intp = ctypes.POINTER(ctypes.c_int)
_SIGS = {
    "jz_default_opts": (None, [ctypes.POINTER(BuildOpts)]),
    "jz_build": (ctypes.c_int, [_vp, ctypes.c_int64, _vp, ctypes.POINTER(BuildOpts),
                                ctypes.POINTER(Allocator), ctypes.POINTER(_vp)]),
    "jz_knn": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "jz_fof": (ctypes.c_int, [_vp, ctypes.c_float, _vp, _vp]),
    "jz_knn_fof": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_float, _vp, _vp,
                                  ctypes.POINTER(Stats), ctypes.POINTER(Stats)]),
    "jz_tree_free": (None, [_vp]),
    "jz_build_joint": (ctypes.c_int, [_vp, ctypes.c_int64, _vp, ctypes.c_int64, _vp,
                                      ctypes.POINTER(BuildOpts), ctypes.POINTER(Allocator),
                                      ctypes.POINTER(_vp)]),
    "jz_knn_query": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "jz_tree_size": (ctypes.c_int64, [_vp]),
    "jz_knn_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "jz_forest_build": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, _vp,
                                       ctypes.POINTER(BuildOpts), ctypes.POINTER(Allocator),
                                       ctypes.POINTER(_vp)]),
    "jz_forest_fof": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), _vp, _vp]),
    "jz_tree_stats": (ctypes.c_int, [_vp, ctypes.POINTER(Stats)]),
    "jz_set_profiling": (None, [ctypes.c_int]),
    "jz_tree_export": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
    "jz_release_cached": (None, []),
    "jz_last_error": (ctypes.c_char_p, []),
    "jz_abi_version": (ctypes.c_int, []),
    "jz_server_default_opts": (None, [ctypes.POINTER(ServerOpts)]),
    "jz_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]),
    "jz_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(Request), _u64p]),
    "jz_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _intp, _intp, _i64p]),
    "jz_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, _intp, _i64p]),
    "jz_server_release": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "jz_server_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ServeStats)]),
    "jz_server_destroy": (None, [_vp]),
    "jz_now_ns": (ctypes.c_int64, []),
    "jz_fof_catalogue": (ctypes.c_int, [_vp, ctypes.c_float, ctypes.c_int, _vp, _vp, _vp, _vp,
                                        ctypes.c_int64, _i64p, _vp]),
    "jz_autotune": (ctypes.c_int, [_vp, _i64p, ctypes.c_int64, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_float), _vp, ctypes.POINTER(BuildOpts),
                                   ctypes.POINTER(BuildOpts), ctypes.POINTER(ctypes.c_double)]),
}


def header_functions(path: str = HEADER_PATH) -> list:
    """Names of the functions ``include/jz.h`` declares (JZ_API lines)."""
    with open(path) as f:
        text = f.read()
    return re.findall(r"^JZ_API[^(]*?\b(jz_\w+)\s*\(", text, flags=re.M)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libjz.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2604_05885_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int):
    if status != JZ_OK:
        raise JzError(status, lib.jz_last_error().decode(errors="replace"))


def default_opts(**kw) -> BuildOpts:
    o = BuildOpts()
    lib.jz_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    return o


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _points(points):
    import torch
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
        raise TypeError("points must be float32 with shape (n, 3)")
    return points.contiguous()


class TorchAllocator:
    """A ``jz_allocator`` that takes the library's device memory from torch's
    caching allocator (so it shows in ``torch.cuda.memory_allocated`` and is
    reused by torch after the library frees it).

    The library frees every block with the stream it was last used on; its
    calls are synchronous, so that work has finished when a block returns to
    torch. ``live`` counts the blocks currently handed out, ``live_bytes``
    their sizes.
    """

    def __init__(self, device=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.live = 0
        self.live_bytes = 0
        self.allocs = 0
        self._sizes = {}
        self._alloc_cb = Allocator._fields_[1][1](self._alloc)
        self._free_cb = Allocator._fields_[2][1](self._free)
        self.struct = Allocator(None, self._alloc_cb, self._free_cb)

    def _alloc(self, ctx, nbytes, stream):
        import torch
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
        except Exception:  # out of memory: the library reports JZ_E_OOM
            return None
        self.live += 1
        self.live_bytes += int(nbytes)
        self._sizes[p] = int(nbytes)
        self.allocs += 1
        return p

    def _free(self, ctx, ptr, nbytes, stream):
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
        self.live -= 1
        self.live_bytes -= self._sizes.pop(int(ptr), int(nbytes))


_torch_allocators = {}


def torch_allocator(device=None) -> TorchAllocator:
    """The process's TorchAllocator for a device (created on first use)."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _torch_allocators:
        _torch_allocators[dev] = TorchAllocator(dev)
    return _torch_allocators[dev]


def _alloc_arg(allocator):
    """ctypes argument for an allocator: None = the library's own pool,
    "torch" = torch's caching allocator, or an object with a ``struct``
    (jz_allocator) attribute."""
    if allocator is None:
        return None, None
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError("allocator must be None, 'torch' or an allocator object")
        allocator = torch_allocator()
    return ctypes.byref(allocator.struct), allocator


def jz_set_profiling(on: bool):
    lib.jz_set_profiling(1 if on else 0)


def jz_release_cached():
    lib.jz_release_cached()


class Tree:
    """A built tree (owns device memory until :meth:`free`)."""

    def __init__(self, handle: ctypes.c_void_p, n: int, nsets: int = 1, offsets=None,
                 allocator=None):
        self._h = handle
        self.n = n
        self.nsets = nsets
        self.offsets = offsets
        self._allocator = allocator  # kept alive while the tree may call it
        self.n_src = -1              # joint trees: number of source points

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("tree already freed")
        return self._h

    def knn(self, k: int, idx=None, dist2=None, stream=None):
        """(idx [n, k] int32, dist2 [n, k] float32) on the tree's device."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if idx is None:
            idx = torch.empty((self.n, k), dtype=torch.int32, device=dev)
        if dist2 is None:
            dist2 = torch.empty((self.n, k), dtype=torch.float32, device=dev)
        if tuple(idx.shape) != (self.n, k) or tuple(dist2.shape) != (self.n, k) or \
                not idx.is_contiguous() or not dist2.is_contiguous() or \
                idx.dtype != torch.int32 or dist2.dtype != torch.float32:
            raise TypeError("idx / dist2 must be contiguous int32 / float32 of shape (n, k)")
        _check(lib.jz_knn(self.handle, int(k), ctypes.c_void_p(idx.data_ptr()),
                          ctypes.c_void_p(dist2.data_ptr()), _stream(stream)))
        return idx, dist2

    def knn_query(self, k: int, idx=None, dist2=None, stream=None):
        """On a joint tree (jz_build_joint): (idx [n_qry, k] source indices,
        dist2 [n_qry, k])."""
        import torch
        nq = self.n - self.n_src
        dev = torch.device("cuda", torch.cuda.current_device())
        if idx is None:
            idx = torch.empty((nq, k), dtype=torch.int32, device=dev)
        if dist2 is None:
            dist2 = torch.empty((nq, k), dtype=torch.float32, device=dev)
        if tuple(idx.shape) != (nq, k) or tuple(dist2.shape) != (nq, k) or \
                not idx.is_contiguous() or not dist2.is_contiguous() or \
                idx.dtype != torch.int32 or dist2.dtype != torch.float32:
            raise TypeError("idx / dist2 must be contiguous int32 / float32 of shape (n_qry, k)")
        _check(lib.jz_knn_query(self.handle, int(k), ctypes.c_void_p(idx.data_ptr()),
                                ctypes.c_void_p(dist2.data_ptr()), _stream(stream)))
        return idx, dist2

    def fof(self, b, label=None, stream=None):
        """Group labels [n] int32 (smallest member index). ``b`` is a float, or
        for a forest also a sequence of one linking length per set."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if label is None:
            label = torch.empty(self.n, dtype=torch.int32, device=dev)
        if tuple(label.shape) != (self.n,) or label.dtype != torch.int32 or \
                not label.is_contiguous():
            raise TypeError("label must be a contiguous int32 tensor of shape (n,)")
        if np.ndim(b) == 0:
            _check(lib.jz_fof(self.handle, float(np.float32(b)),
                              ctypes.c_void_p(label.data_ptr()), _stream(stream)))
        else:
            bb = np.ascontiguousarray(b, dtype=np.float32)
            if bb.shape != (self.nsets,):
                raise ValueError("need one linking length per set")
            _check(lib.jz_forest_fof(self.handle, bb.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     ctypes.c_void_p(label.data_ptr()), _stream(stream)))
        return label

    def knn_fof(self, k: int, b: float, idx=None, dist2=None, label=None, stream=None):
        """kNN and FoF in one call, run concurrently (jz_knn_fof): (idx, dist2,
        label) as :meth:`knn` and :meth:`fof` give them. The two halves'
        statistics are kept in ``self.last_stats`` as (knn, fof) dicts."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if idx is None:
            idx = torch.empty((self.n, k), dtype=torch.int32, device=dev)
        if dist2 is None:
            dist2 = torch.empty((self.n, k), dtype=torch.float32, device=dev)
        if label is None:
            label = torch.empty(self.n, dtype=torch.int32, device=dev)
        if tuple(idx.shape) != (self.n, k) or tuple(dist2.shape) != (self.n, k) or \
                not idx.is_contiguous() or not dist2.is_contiguous() or \
                idx.dtype != torch.int32 or dist2.dtype != torch.float32:
            raise TypeError("idx / dist2 must be contiguous int32 / float32 of shape (n, k)")
        if tuple(label.shape) != (self.n,) or label.dtype != torch.int32 or \
                not label.is_contiguous():
            raise TypeError("label must be a contiguous int32 tensor of shape (n,)")
        ks, fs = Stats(), Stats()
        _check(lib.jz_knn_fof(self.handle, int(k), ctypes.c_void_p(idx.data_ptr()),
                              ctypes.c_void_p(dist2.data_ptr()), float(np.float32(b)),
                              ctypes.c_void_p(label.data_ptr()), _stream(stream),
                              ctypes.byref(ks), ctypes.byref(fs)))
        self.last_stats = (ks.as_dict(), fs.as_dict())
        return idx, dist2, label

    def size(self) -> int:
        """Device bytes the tree holds between calls (jz_tree_size)."""
        return int(lib.jz_tree_size(self.handle))

    def catalogue(self, b: float, min_members: int = 20, vel=None, max_groups=None,
                  stream=None):
        """FoF catalogue (jz_fof_catalogue): dict with ``label`` and ``order``
        (device int32 [n]) and ``groups`` (host structured array, GROUP_DTYPE)."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        label = torch.empty(self.n, dtype=torch.int32, device=dev)
        order = torch.empty(self.n, dtype=torch.int32, device=dev)
        if max_groups is None:
            max_groups = self.n // max(1, int(min_members)) + 1
        gbuf = torch.empty(max(1, int(max_groups)) * GROUP_DTYPE.itemsize, dtype=torch.uint8,
                           device=dev)
        vp = None
        if vel is not None:
            if not isinstance(vel, torch.Tensor) or not vel.is_cuda or vel.dtype != torch.float32 \
                    or tuple(vel.shape) != (self.n, 3):
                raise TypeError("vel must be a CUDA float32 tensor of shape (n, 3)")
            vel = vel.contiguous()
            vp = ctypes.c_void_p(vel.data_ptr())
        ng = ctypes.c_int64()
        _check(lib.jz_fof_catalogue(self.handle, float(np.float32(b)), int(min_members), vp,
                                    ctypes.c_void_p(label.data_ptr()),
                                    ctypes.c_void_p(order.data_ptr()),
                                    ctypes.c_void_p(gbuf.data_ptr()), int(max_groups),
                                    ctypes.byref(ng), _stream(stream)))
        g = gbuf[:ng.value * GROUP_DTYPE.itemsize].cpu().numpy().view(GROUP_DTYPE)
        return {"label": label, "order": order, "groups": g}

    def stats(self) -> dict:
        s = Stats()
        _check(lib.jz_tree_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def export(self, plane=None, order=False, keys=False):
        """Host copies of tree internals (for tests)."""
        out = {}
        o = np.empty(self.n, dtype=np.int32) if order else None
        k = np.empty(self.n, dtype=np.uint64) if keys else None
        spl = None
        if plane is not None:
            st = self.stats()
            spl = np.empty(st["nodes"][plane] + 1, dtype=np.int32)
        _check(lib.jz_tree_export(self.handle,
                                  o.ctypes.data_as(ctypes.c_void_p) if o is not None else None,
                                  k.ctypes.data_as(ctypes.c_void_p) if k is not None else None,
                                  int(plane if plane is not None else 0),
                                  spl.ctypes.data_as(ctypes.c_void_p) if spl is not None else None))
        if order:
            out["order"] = o
        if keys:
            out["keys"] = k
        if spl is not None:
            out["spl"] = spl
        return out

    def free(self):
        if self._h:
            lib.jz_tree_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def jz_build(points, opts: BuildOpts | None = None, stream=None, allocator=None) -> Tree:
    """Sort and build the tree for a CUDA float32 (n, 3) tensor. ``allocator``:
    None (the library's caching pool), "torch" (torch's caching allocator) or
    an allocator object (see :class:`TorchAllocator`)."""
    p = _points(points)
    h = ctypes.c_void_p()
    aref, keep = _alloc_arg(allocator)
    _check(lib.jz_build(ctypes.c_void_p(p.data_ptr()), p.shape[0], _stream(stream),
                        ctypes.byref(opts) if opts is not None else None, aref, ctypes.byref(h)))
    return Tree(h, p.shape[0], allocator=keep)


def jz_build_joint(sources, queries, opts: BuildOpts | None = None, stream=None,
                   allocator=None) -> Tree:
    """One tree over source and query points (CUDA float32 (n, 3) tensors),
    for :meth:`Tree.knn_query`."""
    s = _points(sources)
    q = _points(queries)
    h = ctypes.c_void_p()
    aref, keep = _alloc_arg(allocator)
    _check(lib.jz_build_joint(ctypes.c_void_p(s.data_ptr()), s.shape[0],
                              ctypes.c_void_p(q.data_ptr()), q.shape[0], _stream(stream),
                              ctypes.byref(opts) if opts is not None else None, aref,
                              ctypes.byref(h)))
    t = Tree(h, s.shape[0] + q.shape[0], allocator=keep)
    t.n_src = s.shape[0]
    return t


def jz_forest_build(points, offsets, opts: BuildOpts | None = None, stream=None,
                    allocator=None) -> Tree:
    """One tree over many independent sets; ``offsets`` is a host int array [B+1]."""
    p = _points(points)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    h = ctypes.c_void_p()
    aref, keep = _alloc_arg(allocator)
    _check(lib.jz_forest_build(ctypes.c_void_p(p.data_ptr()),
                               off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(off) - 1,
                               _stream(stream), ctypes.byref(opts) if opts is not None else None,
                               aref, ctypes.byref(h)))
    return Tree(h, p.shape[0], len(off) - 1, off, allocator=keep)


def jz_knn(tree: Tree, k: int, stream=None):
    return tree.knn(k, stream=stream)


def jz_fof(tree: Tree, b, stream=None):
    return tree.fof(b, stream=stream)


def jz_tree_free(tree: Tree):
    tree.free()


def knn(points, k: int, opts: BuildOpts | None = None):
    """Build + kNN in one call; returns (idx, dist2)."""
    with jz_build(points, opts) as t:
        return t.knn(k)


def fof(points, b: float, opts: BuildOpts | None = None):
    """Build + FoF in one call; returns labels."""
    with jz_build(points, opts) as t:
        return t.fof(b)


def jz_autotune(points, offsets=None, k: int = 16, b=None, base: BuildOpts | None = None,
                stream=None):
    """Fastest build options for this workload: (BuildOpts, ms)."""
    p = _points(points)
    best = BuildOpts()
    ms = ctypes.c_double()
    if offsets is not None:
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        offp, nsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(off) - 1
    else:
        off, offp, nsets = None, None, p.shape[0]
    bb = None
    if b is not None:
        bb = np.ascontiguousarray(np.atleast_1d(b), dtype=np.float32)
    _check(lib.jz_autotune(ctypes.c_void_p(p.data_ptr()), offp, nsets, int(k),
                           bb.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if bb is not None
                           else None, _stream(stream),
                           ctypes.byref(base) if base is not None else None,
                           ctypes.byref(best), ctypes.byref(ms)))
    return best, ms.value


def now_ns() -> int:
    """The library's monotonic clock (ns), the clock of server completion times."""
    return int(lib.jz_now_ns())


class Server:
    """Continuous-batching request loop (``jz_server_*``).

    ``submit_knn`` / ``submit_fof`` queue a request on CUDA tensors and return
    a ticket; the tensors are kept alive until the ticket is released.
    """

    def __init__(self, hbm_budget: int | None = None, streams: int | None = None,
                 max_batch_points: int | None = None, max_batch_sets: int | None = None,
                 build: BuildOpts | None = None):
        o = ServerOpts()
        lib.jz_server_default_opts(ctypes.byref(o))
        if hbm_budget is not None:
            o.hbm_budget = int(hbm_budget)
        if streams is not None:
            o.streams = int(streams)
        if max_batch_points is not None:
            o.max_batch_points = int(max_batch_points)
        if max_batch_sets is not None:
            o.max_batch_sets = int(max_batch_sets)
        if build is not None:
            o.build = build
        h = ctypes.c_void_p()
        _check(lib.jz_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def _submit(self, req: Request, keep) -> int:
        t = ctypes.c_uint64()
        _check(lib.jz_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def submit_knn(self, points, k: int, idx=None, dist2=None, stream=None) -> int:
        """Queue kNN on ``points``; the request waits for the work queued on
        ``stream`` (default: the current stream) before it reads them."""
        import torch
        p = _points(points)
        n = p.shape[0]
        if idx is None:
            idx = torch.empty((n, k), dtype=torch.int32, device=p.device)
        if dist2 is None:
            dist2 = torch.empty((n, k), dtype=torch.float32, device=p.device)
        r = Request(JZ_OP_KNN, int(k), 0.0, p.data_ptr(), n, idx.data_ptr(), dist2.data_ptr(), None,
                    _stream(stream))
        return self._submit(r, (p, idx, dist2))

    def submit_fof(self, points, b: float, label=None, stream=None) -> int:
        """Queue FoF on ``points`` (ordered after ``stream`` as submit_knn)."""
        import torch
        p = _points(points)
        n = p.shape[0]
        if label is None:
            label = torch.empty(n, dtype=torch.int32, device=p.device)
        r = Request(JZ_OP_FOF, 0, float(np.float32(b)), p.data_ptr(), n, None, None,
                    label.data_ptr(), _stream(stream))
        return self._submit(r, (p, label))

    def poll(self, ticket: int):
        """(done, status, completion time ns)."""
        d, st, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        _check(lib.jz_server_poll(self._h, ticket, ctypes.byref(d), ctypes.byref(st),
                                  ctypes.byref(t)))
        return bool(d.value), st.value, t.value

    def wait(self, ticket: int):
        """Block until done; returns (outputs tuple, completion time ns)."""
        st, t = ctypes.c_int(), ctypes.c_int64()
        _check(lib.jz_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(t)))
        _check(st.value)
        return self._keep[ticket][1:], t.value

    def release(self, ticket: int):
        _check(lib.jz_server_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        s = ServeStats()
        _check(lib.jz_server_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self._h:
            lib.jz_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
