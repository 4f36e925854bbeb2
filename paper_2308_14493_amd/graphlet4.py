"""Python binding of libgraphlet4.so (argument marshalling only).

Every step of the counting runs in the library's HIP kernels; this module
converts arrays, calls the C ABI declared in include/graphlet4.h and turns
error codes into exceptions.  torch is used only by the ``*_dev`` entry
points, for device memory and the current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraphlet4.so")

CLASSES = ["P4", "star", "C4", "paw", "diamond", "K4",
           "tri+K1", "P3+K1", "2K2", "K2+2K1", "empty"]

_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_P = ctypes.c_void_p


class Options(ctypes.Structure):
    _fields_ = [("radius", _I32), ("slack", ctypes.c_float), ("device", _I32), ("stream", _P), ("autotune", _I32),
                ("graphs", _I32), ("delta", _I32), ("vertex_capacity", _I64),
                ("tri_small_max", _I32), ("c4_small_max", _I32), ("c4_mid_max", _I32)]


class BatchStats(ctypes.Structure):
    _fields_ = [(n, _I64) for n in (
        "offered_ins", "offered_del", "eff_ins", "eff_del", "loops", "dups", "cancelled",
        "ins_existing", "del_missing", "touched_vertices", "region_vertices", "region_entries",
        "wedges", "c4_entries_small", "c4_entries_mid", "c4_entries_large", "c4_tail_wedges",
        "max_out_degree", "tier_tri_small", "tier_tri_large", "tier_c4_small",
        "tier_c4_mid", "tier_c4_large", "c4_dense_min")] + [
        ("whole_graph", _I32), ("overflow_mask", ctypes.c_uint32), ("pass_batches", _I32)] + [
        (n, ctypes.c_float) for n in ("ms_total", "ms_prepare", "ms_tri", "ms_edge", "ms_c4_small",
                                      "ms_c4_mid", "ms_c4_large", "ms_finish")] + [
        ("c4_windows", _I64), ("c4_searches", _I64), ("tri_global_vertices", _I64), ("tri_exc_rebuilds", _I64),
        ("retries", _I32), ("delta", _I32), ("tri_entries", _I64),
        ("tri_small_max", _I32), ("c4_small_max", _I32), ("c4_mid_max", _I32), ("k4_split_edges", _I64)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class BatchDesc(ctypes.Structure):
    _fields_ = [("ins_src", _P), ("ins_dst", _P), ("n_ins", _I64),
                ("del_src", _P), ("del_dst", _P), ("n_del", _I64)]


class GraphletError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("graphlet4 error %d: %s" % (code, msg))
        self.code = code


_lib = None

EXPORTS = ["gc_options_default", "gc_graph_init", "gc_pool_init", "gc_apply_batch", "gc_apply_batch_dev",
           "gc_apply_batch_dev_noalloc",
           "gc_apply_batches", "gc_apply_batch_seq", "gc_add_vertices", "gc_remove_vertices", "gc_get_counts", "gc_get_counts_exact", "gc_get_counts3", "gc_recount_exact", "gc_graph_info",
           "gc_export_edges", "gc_graph_footprint", "gc_graph_replays", "gc_copy_tuning", "gc_graph_free", "gc_strerror", "gc_last_error",
           "gc_server_opts_default", "gc_server_create", "gc_server_add_graph", "gc_server_submit",
           "gc_server_wait", "gc_server_counts", "gc_server_destroy"]


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", _I32), ("max_graphs", _I32), ("hbm_reserve_bytes", _I64),
                ("hbm_budget_bytes", _I64), ("batch_budget_bytes", _I64)]


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libgraphlet4.so is not built (python -m paper_2308_14493_amd.build)")
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # soname); importing it first lets the library bind to that copy
    # instead of loading a second runtime that cannot open the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    lib.gc_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.gc_graph_init.argtypes = [_I64, _P, _P, _I64, ctypes.POINTER(Options), ctypes.POINTER(_P), _P]
    lib.gc_pool_init.argtypes = [_I32, _P, _P, _P, _P, ctypes.POINTER(Options), ctypes.POINTER(_P), _P]
    lib.gc_apply_batch.argtypes = [_P, _P, _P, _I64, _P, _P, _I64, _P, ctypes.POINTER(BatchStats)]
    lib.gc_apply_batch_dev.argtypes = [_P, _P, _P, _I64, _P, _P, _I64, _P, ctypes.POINTER(BatchStats)]
    lib.gc_apply_batch_dev_noalloc.argtypes = [_P, _P, _P, _I64, _P, _P, _I64, _P, ctypes.POINTER(BatchStats)]
    lib.gc_apply_batches.argtypes = [_P, _P, _P, ctypes.POINTER(BatchStats)]
    lib.gc_apply_batch_seq.argtypes = [_P, _P, _I32, _P, _P]
    lib.gc_add_vertices.argtypes = [_P, _I64, ctypes.POINTER(_I64), _P]
    lib.gc_remove_vertices.argtypes = [_P, _P, _I64, _P, ctypes.POINTER(BatchStats)]
    lib.gc_get_counts.argtypes = [_P, _I32, _P, ctypes.POINTER(ctypes.c_uint32)]
    lib.gc_get_counts_exact.argtypes = [_P, _I32, _P, _P]
    lib.gc_recount_exact.argtypes = [_P, _I32, _P, _P]
    lib.gc_get_counts3.argtypes = [_P, _I32, _P, _P]
    lib.gc_graph_info.argtypes = [_P, ctypes.POINTER(_I32), _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]
    lib.gc_export_edges.argtypes = [_P, _I32, _P, _P, _I64, ctypes.POINTER(_I64)]
    lib.gc_graph_replays.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]
    lib.gc_copy_tuning.argtypes = [_P, _P]
    lib.gc_graph_footprint.argtypes = [_I64, _P, _P, _I64, ctypes.POINTER(Options), ctypes.POINTER(_I64)]
    lib.gc_graph_free.argtypes = [_P]
    lib.gc_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
    lib.gc_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]
    lib.gc_server_add_graph.argtypes = [_P, _I64, _P, _P, _I64, ctypes.POINTER(Options), ctypes.POINTER(_I32)]
    lib.gc_server_submit.argtypes = [_P, _I32, ctypes.POINTER(BatchDesc), ctypes.POINTER(ctypes.c_uint64)]
    lib.gc_server_wait.argtypes = [_P, ctypes.c_uint64, _P, ctypes.POINTER(BatchStats), _P]
    lib.gc_server_counts.argtypes = [_P, _I32, _P, _P]
    lib.gc_server_destroy.argtypes = [_P]
    lib.gc_strerror.argtypes = [ctypes.c_int]
    lib.gc_strerror.restype = ctypes.c_char_p
    lib.gc_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("gc_strerror", "gc_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise GraphletError(rc, _lib.gc_last_error().decode())


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _join(hi, lo):
    return [(int(h) << 64) | int(l) for h, l in zip(hi.tolist(), lo.tolist())]


def _opts(radius, slack, device, stream, autotune=None, graphs=None, delta=None, vertex_capacity=None, tiers=None):
    lib = load()
    o = Options()
    lib.gc_options_default(ctypes.byref(o))
    if tiers is not None:
        o.tri_small_max, o.c4_small_max, o.c4_mid_max = (int(x) for x in tiers)
    if vertex_capacity is not None:
        o.vertex_capacity = int(vertex_capacity)
    if delta is not None:
        o.delta = int(delta)
    if autotune is not None:
        o.autotune = int(autotune)
    if graphs is not None:
        o.graphs = int(graphs)
    if radius is not None:
        o.radius = radius
    if slack is not None:
        o.slack = slack
    o.device = device
    o.stream = stream
    return o


def footprint(n, src, dst, slack=None):
    """Estimated device bytes of a handle built from this edge list."""
    lib = load()
    s, d = _i32(src), _i32(dst)
    opt = _opts(None, slack, 0, None)
    b = _I64()
    _check(lib.gc_graph_footprint(int(n), s.ctypes.data, d.ctypes.data, s.size, ctypes.byref(opt), ctypes.byref(b)))
    return b.value


class Graph:
    """A resident graph (or a pool of graphs) on one GPU."""

    def __init__(self, n, src=(), dst=(), radius=None, slack=None, device=0, stream=None, autotune=None,
                 graphs=None, delta=None, vertex_capacity=None, tiers=None, _pool=None):
        lib = load()
        self._h = _P()
        opt = _opts(radius, slack, device, stream, autotune, graphs, delta, vertex_capacity, tiers)
        if _pool is None:
            s, d = _i32(src), _i32(dst)
            assert s.shape == d.shape
            self.k = 1
            _check(lib.gc_graph_init(int(n), s.ctypes.data, d.ctypes.data, s.size, ctypes.byref(opt),
                                     ctypes.byref(self._h), None))
        else:
            ns, srcs, dsts = _pool
            self.k = len(ns)
            keep = [(_i32(a), _i32(b)) for a, b in zip(srcs, dsts)]
            n_arr = np.asarray(ns, dtype=np.int64)
            m_arr = np.asarray([a.size for a, _ in keep], dtype=np.int64)
            sp = (_P * self.k)(*[a.ctypes.data for a, _ in keep])
            dp = (_P * self.k)(*[b.ctypes.data for _, b in keep])
            _check(lib.gc_pool_init(self.k, n_arr.ctypes.data, ctypes.cast(sp, _P), ctypes.cast(dp, _P),
                                    m_arr.ctypes.data, ctypes.byref(opt), ctypes.byref(self._h), None))

    @classmethod
    def pool(cls, ns, srcs, dsts, **kw):
        return cls(None, _pool=(ns, srcs, dsts), **kw)

    # ------------------------------------------------------------------
    def close(self):
        if self._h:
            load().gc_graph_free(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------
    def apply_batch(self, ins_src=(), ins_dst=(), del_src=(), del_dst=(), stats=False):
        """Applies one batch; returns the 11 exact counts (Python ints).  The
        library's int64 output of the call (low 64 bits of each class, as
        unsigned values) is kept in ``last_int64``."""
        lib = load()
        iu, iv, du, dv = _i32(ins_src), _i32(ins_dst), _i32(del_src), _i32(del_dst)
        assert iu.shape == iv.shape and du.shape == dv.shape
        st = BatchStats()
        out = np.zeros(11, np.int64)
        _check(lib.gc_apply_batch(self._h, iu.ctypes.data, iv.ctypes.data, iu.size, du.ctypes.data,
                                  dv.ctypes.data, du.size, out.ctypes.data,
                                  ctypes.byref(st) if stats else None))
        self.last_int64 = [int(x) for x in out.view(np.uint64)]
        c = self.counts()
        return (c, st.as_dict()) if stats else c

    def apply_batch_dev(self, ins_src, ins_dst, del_src, del_dst, stats=False):
        """Device-array variant: int32 torch tensors on this graph's device."""
        lib = load()
        st = BatchStats()
        out = np.zeros(11, np.int64)
        import torch
        for t in (ins_src, ins_dst, del_src, del_dst):
            assert t.dtype == torch.int32 and t.is_cuda and t.is_contiguous()
        # the library runs on its own stream: the producer's work must be done
        torch.cuda.current_stream().synchronize()
        _check(lib.gc_apply_batch_dev(self._h, ins_src.data_ptr(), ins_dst.data_ptr(), ins_src.numel(),
                                      del_src.data_ptr(), del_dst.data_ptr(), del_src.numel(),
                                      out.ctypes.data, ctypes.byref(st) if stats else None))
        self.last_int64 = [int(x) for x in out.view(np.uint64)]
        c = self.counts()
        return (c, st.as_dict()) if stats else c

    def apply_batch_dev_noalloc(self, ins_src, ins_dst, del_src, del_dst, stats=False):
        """gc_apply_batch_dev_noalloc: device arrays, no allocation in the
        library call (staging in a static device array)."""
        lib = load()
        st = BatchStats()
        out = np.zeros(11, np.int64)
        import torch
        for t in (ins_src, ins_dst, del_src, del_dst):
            assert t.dtype == torch.int32 and t.is_cuda and t.is_contiguous()
        torch.cuda.current_stream().synchronize()
        _check(lib.gc_apply_batch_dev_noalloc(self._h, ins_src.data_ptr(), ins_dst.data_ptr(), ins_src.numel(),
                                              del_src.data_ptr(), del_dst.data_ptr(), del_src.numel(),
                                              out.ctypes.data, ctypes.byref(st) if stats else None))
        self.last_int64 = [int(x) for x in out.view(np.uint64)]
        c = self.counts()
        return (c, st.as_dict()) if stats else c

    def apply_batches(self, batches, stats=False):
        """Pool: one batch (ins_src, ins_dst, del_src, del_dst) per graph."""
        lib = load()
        assert len(batches) == self.k
        keep = []
        descs = (BatchDesc * self.k)()
        for g, b in enumerate(batches):
            iu, iv, du, dv = (_i32(x) for x in b)
            keep.append((iu, iv, du, dv))
            descs[g] = BatchDesc(iu.ctypes.data, iv.ctypes.data, iu.size, du.ctypes.data, dv.ctypes.data, du.size)
        st = BatchStats()
        _check(lib.gc_apply_batches(self._h, ctypes.cast(descs, _P), None, ctypes.byref(st) if stats else None))
        out = [self.counts(g) for g in range(self.k)]
        return (out, st.as_dict()) if stats else out

    def apply_batch_seq(self, batches, stats=False):
        """Applies batches (ins_src, ins_dst, del_src, del_dst) in order, up to
        three per counting pass; returns the counts after each batch as int64
        values (the low 64 bits where a class leaves int64; counts() gives the
        exact values after the last batch)."""
        lib = load()
        nb = len(batches)
        keep = []
        descs = (BatchDesc * max(nb, 1))()
        for j, b in enumerate(batches):
            iu, iv, du, dv = (_i32(x) for x in b)
            assert iu.shape == iv.shape and du.shape == dv.shape
            keep.append((iu, iv, du, dv))
            descs[j] = BatchDesc(iu.ctypes.data, iv.ctypes.data, iu.size, du.ctypes.data, dv.ctypes.data, du.size)
        out = np.zeros((max(nb, 1), 11), np.int64)
        sts = (BatchStats * max(nb, 1))()
        _check(lib.gc_apply_batch_seq(self._h, ctypes.cast(descs, _P), nb, out.ctypes.data,
                                      ctypes.cast(sts, _P) if stats else None))
        rows = [[int(x) for x in out[j]] for j in range(nb)]
        return (rows, [sts[j].as_dict() for j in range(nb)]) if stats else rows

    def copy_tuning(self, src):
        """gc_copy_tuning: start from what the autotuner of handle `src` has
        learned (speed knobs only; counts do not change)."""
        _check(load().gc_copy_tuning(self._h, src._h))

    def graph_replays(self):
        """(passes captured as HIP graphs, passes launched from captured graphs)."""
        lib = load()
        c, n = _I64(), _I64()
        _check(lib.gc_graph_replays(self._h, ctypes.byref(c), ctypes.byref(n)))
        return c.value, n.value

    def add_vertices(self, count):
        """gc_add_vertices: `count` new isolated vertices; returns (first id,
        counts)."""
        lib = load()
        first = _I64()
        _check(lib.gc_add_vertices(self._h, int(count), ctypes.byref(first), None))
        return first.value, self.counts()

    def remove_vertices(self, ids, stats=False):
        """gc_remove_vertices: deletes the edges at `ids`, then the vertices;
        returns the counts (and the batch statistics)."""
        lib = load()
        v = _i32(ids)
        st = BatchStats()
        _check(lib.gc_remove_vertices(self._h, v.ctypes.data, v.size, None, ctypes.byref(st) if stats else None))
        c = self.counts()
        return (c, st.as_dict()) if stats else c

    def counts(self, graph=0):
        """Exact counts (Python ints) of graph `graph`."""
        lib = load()
        hi = np.zeros(11, np.int64)
        lo = np.zeros(11, np.uint64)
        _check(lib.gc_get_counts_exact(self._h, graph, hi.ctypes.data, lo.ctypes.data))
        return _join(hi, lo)

    def counts3(self, graph=0):
        """Exact induced 3-vertex counts [triangle, 2-path, edge + isolated,
        empty] of graph `graph`."""
        lib = load()
        hi = np.zeros(4, np.int64)
        lo = np.zeros(4, np.uint64)
        _check(lib.gc_get_counts3(self._h, graph, hi.ctypes.data, lo.ctypes.data))
        return _join(hi, lo)

    def counts_int64(self, graph=0):
        lib = load()
        out = np.zeros(11, np.int64)
        mask = ctypes.c_uint32()
        _check(lib.gc_get_counts(self._h, graph, out.ctypes.data, ctypes.byref(mask)))
        return out, int(mask.value)

    def recount(self, graph=0):
        """Static recount on the GPU (does not change the maintained counts)."""
        lib = load()
        hi = np.zeros(11, np.int64)
        lo = np.zeros(11, np.uint64)
        _check(lib.gc_recount_exact(self._h, graph, hi.ctypes.data, lo.ctypes.data))
        return _join(hi, lo)

    def info(self, graph=0):
        lib = load()
        k, n, m = _I32(), _I64(), _I64()
        _check(lib.gc_graph_info(self._h, ctypes.byref(k), graph, ctypes.byref(n), ctypes.byref(m)))
        return dict(num_graphs=k.value, n=n.value, m=m.value)

    def edges(self, graph=0):
        lib = load()
        m = self.info(graph)["m"]
        s = np.zeros(max(m, 1), np.int32)
        d = np.zeros(max(m, 1), np.int32)
        mo = _I64()
        _check(lib.gc_export_edges(self._h, graph, s.ctypes.data, d.ctypes.data, s.size, ctypes.byref(mo)))
        return s[: mo.value], d[: mo.value]


class Server:
    """Serving loop: resident graphs answering asynchronously submitted
    batches through tickets (see gc_server_* in include/graphlet4.h)."""

    def __init__(self, device=0, max_graphs=64, hbm_reserve_bytes=None, hbm_budget_bytes=0,
                 batch_budget_bytes=None):
        lib = load()
        o = ServerOpts()
        lib.gc_server_opts_default(ctypes.byref(o))
        o.device = device
        o.max_graphs = max_graphs
        if hbm_reserve_bytes is not None:
            o.hbm_reserve_bytes = hbm_reserve_bytes
        o.hbm_budget_bytes = hbm_budget_bytes
        if batch_budget_bytes is not None:
            o.batch_budget_bytes = batch_budget_bytes
        self._h = _P()
        _check(lib.gc_server_create(ctypes.byref(o), ctypes.byref(self._h)))

    def add_graph(self, n, src, dst, radius=None, slack=None, delta=None):
        lib = load()
        s, d = _i32(src), _i32(dst)
        opt = _opts(radius, slack, 0, None, delta=delta)
        gid = _I32()
        _check(lib.gc_server_add_graph(self._h, int(n), s.ctypes.data, d.ctypes.data, s.size, ctypes.byref(opt),
                                       ctypes.byref(gid)))
        return gid.value

    def submit(self, graph, ins_src=(), ins_dst=(), del_src=(), del_dst=()):
        lib = load()
        iu, iv, du, dv = _i32(ins_src), _i32(ins_dst), _i32(del_src), _i32(del_dst)
        desc = BatchDesc(iu.ctypes.data, iv.ctypes.data, iu.size, du.ctypes.data, dv.ctypes.data, du.size)
        t = ctypes.c_uint64()
        _check(lib.gc_server_submit(self._h, graph, ctypes.byref(desc), ctypes.byref(t)))
        return t.value

    def wait(self, ticket):
        """Returns (int64 counts, stats dict, latency ms, queueing ms)."""
        lib = load()
        out = np.zeros(11, np.int64)
        st = BatchStats()
        lat = np.zeros(2, np.float64)
        _check(lib.gc_server_wait(self._h, ticket, out.ctypes.data, ctypes.byref(st), lat.ctypes.data))
        return out, st.as_dict(), float(lat[0]), float(lat[1])

    def counts(self, graph):
        lib = load()
        hi = np.zeros(11, np.int64)
        lo = np.zeros(11, np.uint64)
        _check(lib.gc_server_counts(self._h, graph, hi.ctypes.data, lo.ctypes.data))
        return _join(hi, lo)

    def close(self):
        if self._h:
            load().gc_server_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
