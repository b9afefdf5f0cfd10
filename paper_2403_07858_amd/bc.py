"""Python binding of the C ABI in include/bc.h (argument marshalling only).

Every function keeps the C name and runs the device library ``libbc.so``;
there is no Python or CPU fallback.  Importing this module on a machine
where the library cannot be loaded raises ImportError.

CSR inputs are host numpy arrays (indptr uint64, indices uint32).  A torch
stream may be passed as ``stream=torch.cuda.current_stream()`` (or a raw
``hipStream_t`` integer); the default is the library's own stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: its HIP runtime (torch/lib/libamdhip64.so, soname
# libamdhip64.so.7) is then the one libbc.so binds to.  Loaded the other way
# round, the process would hold two HIP runtimes, and torch's could not
# open the GPU that the first one holds.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is part of this environment
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbc.so")

BC_OK = 0
BC_E_INVALID_ARG = -1
BC_E_BAD_CSR = -2
BC_E_INCONSISTENT = -3
BC_E_OOM = -4
BC_E_DEVICE = -5
BC_E_OVERFLOW = -6
BC_E_REJECTED = -7
BC_E_TIMEOUT = -8
BC_E_CANCELLED = -9
BC_E_PENDING = -10
BC_E_NOT_FOUND = -11

BC_ANCHOR_AUTO, BC_ANCHOR_U, BC_ANCHOR_V = -1, 0, 1
BC_ORDER_DEGREE, BC_ORDER_TWO_HOP, BC_ORDER_BORDER = 0, 1, 2
BC_ROOT_BUILD_AUTO, BC_ROOT_BUILD_TWO_PASS = 0, 1
BC_SETS_LOCAL_BITMAP, BC_SETS_HTB, BC_SETS_SORTED = 0, 1, 2


class bc_u128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]

    @property
    def value(self) -> int:
        return (int(self.hi) << 64) | int(self.lo)


class bc_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_uint64), ("n_cols", ctypes.c_uint64), ("nnz", ctypes.c_uint64),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class bc_allocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


class bc_opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("stream", ctypes.c_void_p), ("anchor", ctypes.c_int32),
                ("lds_words", ctypes.c_uint32), ("waves_per_cu", ctypes.c_uint32),
                ("instrument", ctypes.c_uint32), ("timeout_ms", ctypes.c_uint32),
                ("alloc", ctypes.POINTER(bc_allocator)), ("order_key", ctypes.c_int32),
                ("order_k", ctypes.c_uint32), ("roots_per_wave", ctypes.c_uint32),
                ("switch_depth", ctypes.c_uint32), ("split_rows", ctypes.c_uint32),
                ("root_build", ctypes.c_uint32), ("sets", ctypes.c_uint32), ("bitmap_bits", ctypes.c_uint32),
                ("border_iters", ctypes.c_uint32), ("scratch_cap_bytes", ctypes.c_uint64),
                ("pure_dfs", ctypes.c_uint32)]


class Allocator:
    """A ``bc_allocator`` made of two Python callables: ``alloc(nbytes, stream)``
    returns a device pointer (int; 0 or None when it cannot) and
    ``free(ptr, stream)`` gives it back.  Keep the object alive while any call
    or graph uses it."""

    def __init__(self, alloc, free):
        self.errors = []   # exceptions the callables raised (a raising alloc is a failed allocation)

        def _a(_ctx, n, st):
            try:
                return alloc(int(n), int(st or 0)) or None
            except Exception as e:
                self.errors.append(repr(e))
                return None

        def _f(_ctx, ptr, st):
            try:
                free(int(ptr), int(st or 0))
            except Exception as e:
                self.errors.append(repr(e))

        self._a, self._f = _ALLOC_FN(_a), _FREE_FN(_f)
        self.struct = bc_allocator(None, self._a, self._f)


def torch_allocator(device=None) -> Allocator:
    """Device memory from torch's caching allocator (stream-ordered on the
    stream the library passes)."""
    import torch

    torch.cuda.init()   # the caching allocator must exist before the library calls into it
    dev = torch.cuda.current_device() if device is None else device
    return Allocator(lambda n, st: torch.cuda.caching_allocator_alloc(n, dev, st),
                     lambda ptr, st: torch.cuda.caching_allocator_delete(ptr))


class bc_stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_candidates", ctypes.c_double), ("ms_plan", ctypes.c_double),
                ("ms_rows", ctypes.c_double), ("ms_enumerate", ctypes.c_double), ("anchor", ctypes.c_int32),
                ("roots", ctypes.c_uint64), ("roots_active", ctypes.c_uint64), ("tasks", ctypes.c_uint64),
                ("candidate_edges", ctypes.c_uint64), ("row_words", ctypes.c_uint64),
                ("pair_ops", ctypes.c_uint64), ("filter_ops", ctypes.c_uint64),
                ("cyc_setup", ctypes.c_uint64), ("cyc_compact", ctypes.c_uint64), ("cyc_pair", ctypes.c_uint64),
                ("cyc_filter", ctypes.c_uint64), ("pairs", ctypes.c_uint64), ("pair_slots", ctypes.c_uint64),
                ("cyc_pack", ctypes.c_uint64), ("scratch_bytes", ctypes.c_uint64),
                ("ms_wave_makespan", ctypes.c_double), ("ms_wave_spread", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2403_07858_amd/build.py (hipcc, gfx950)")
    try:
        lib = ctypes.CDLL(LIB_PATH)
    except OSError as e:  # pragma: no cover - depends on the machine
        raise ImportError(f"cannot load {LIB_PATH}: {e}") from e
    P, I32, U32, U64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "bc_build": ([P, P, P, P], I32),
        "bc_free": ([P], None),
        "bc_graph_info": ([P, P, P, P], I32),
        "bc_ranks": ([P, I32, P], I32),
        "bc_htb_stats": ([P, I32, P, P], I32),
        "bc_count": ([P, U32, U32, P, P, P], I32),
        "bc_count_roots": ([P, U32, U32, I32, U64, U64, P, P, P], I32),
        "bc_count_batch": ([P, P, P, SZ, P, P, P, P], I32),
        "bc_tune_batch": ([P, P, P, SZ, P, P], I32),
        "bc_scratch_estimate": ([P, U32, U32, P, P], I32),
        "bc_partition": ([P, U32, U32, I32, U64, P, P], I32),
        "bc_count_partition": ([P, U32, U32, I32, P, U32, P, P, P], I32),
        "bc_count_noalloc": ([P, U32, U32, P, P], I32),
        "bc_count_per_vertex": ([P, U32, U32, I32, P, P], I32),
        "bc_status_string": ([I32], ctypes.c_char_p),
        "bc_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()

EXPORTED = ("bc_build", "bc_free", "bc_graph_info", "bc_ranks", "bc_htb_stats", "bc_count", "bc_count_roots", "bc_count_batch",
            "bc_tune_batch", "bc_scratch_estimate", "bc_partition", "bc_count_partition", "bc_count_noalloc", "bc_count_per_vertex", "bc_status_string",
            "bc_last_error")


class BCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = bc_last_error()
        super().__init__(f"{where}: {bc_status_string(status)}" + (f" ({detail})" if detail else ""))


def bc_status_string(s: int) -> str:
    return _lib.bc_status_string(s).decode()


def bc_last_error() -> str:
    return _lib.bc_last_error().decode()


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    h = getattr(stream, "cuda_stream", None)   # torch.cuda.Stream
    if h is None:
        raise TypeError("stream must be a torch.cuda.Stream or a raw stream handle")
    return int(h)


def make_opts(stream=None, anchor=BC_ANCHOR_AUTO, lds_words=0, waves_per_cu=0, instrument=False,
              timeout_ms=0, allocator=None, order_key=BC_ORDER_DEGREE, order_k=0, roots_per_wave=0,
              switch_depth=0, split_rows=0, root_build=BC_ROOT_BUILD_AUTO, sets=0, bitmap_bits=0,
              border_iters=0, scratch_cap_bytes=0, pure_dfs=False) -> bc_opts:
    o = bc_opts()
    o.struct_size = ctypes.sizeof(bc_opts)
    o.stream = _stream_handle(stream)
    o.anchor = anchor
    o.lds_words = lds_words
    o.waves_per_cu = waves_per_cu
    o.instrument = 1 if instrument else 0
    o.timeout_ms = timeout_ms
    if allocator is not None:
        o.alloc = ctypes.pointer(allocator.struct)
    o.order_key = order_key
    o.order_k = order_k
    o.roots_per_wave = roots_per_wave
    o.switch_depth = switch_depth
    o.split_rows = split_rows
    o.root_build = root_build
    o.sets = sets
    o.bitmap_bits = bitmap_bits
    o.border_iters = border_iters
    o.scratch_cap_bytes = scratch_cap_bytes
    o.pure_dfs = 1 if pure_dfs else 0
    return o


def _csr(n_rows, n_cols, indptr, indices, keep):
    ip = np.ascontiguousarray(indptr, dtype=np.uint64)
    ix = np.ascontiguousarray(indices, dtype=np.uint32)
    keep += [ip, ix]
    c = bc_csr()
    c.n_rows, c.n_cols, c.nnz = n_rows, n_cols, int(ix.shape[0])
    c.indptr = ip.ctypes.data
    c.indices = ix.ctypes.data if ix.size else None
    return c


class Graph:
    """A graph resident on the device (owns a ``bc_graph *``)."""

    def __init__(self, handle: int, n_u: int, n_v: int, n_edges: int, allocator=None):
        self.handle = handle
        self.n_u, self.n_v, self.n_edges = n_u, n_v, n_edges
        self._allocator = allocator   # a hook the graph's arrays came from must outlive them

    def close(self):
        if self.handle:
            _lib.bc_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bc_build(n_u, n_v, indptr_u, indices_u, indptr_v, indices_v, **opt) -> Graph:
    """Validate and upload a bipartite graph given as its two CSR sides."""
    keep = []
    cu = _csr(n_u, n_v, indptr_u, indices_u, keep)
    cv = _csr(n_v, n_u, indptr_v, indices_v, keep)
    o = make_opts(**opt)
    h = ctypes.c_void_p()
    s = _lib.bc_build(ctypes.byref(cu), ctypes.byref(cv), ctypes.byref(o), ctypes.byref(h))
    if s != BC_OK:
        raise BCError(s, "bc_build")
    return Graph(h.value, n_u, n_v, cu.nnz, opt.get("allocator"))


def build_graph(g, **opt) -> Graph:
    """bc_build from any object with n_u, n_v, indptr_u, indices_u, indptr_v, indices_v."""
    return bc_build(g.n_u, g.n_v, g.indptr_u, g.indices_u, g.indptr_v, g.indices_v, **opt)


def bc_free(g: Graph) -> None:
    g.close()


def bc_graph_info(g: Graph):
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    s = _lib.bc_graph_info(g.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    if s != BC_OK:
        raise BCError(s, "bc_graph_info")
    return a.value, b.value, c.value


def bc_ranks(g: Graph, side: int) -> np.ndarray:
    n = g.n_u if side == 0 else g.n_v
    out = np.zeros(max(1, n), dtype=np.uint32)
    s = _lib.bc_ranks(g.handle, side, out.ctypes.data)
    if s != BC_OK:
        raise BCError(s, "bc_ranks")
    return out[:n]


def bc_count(g: Graph, p: int, q: int, with_stats=False, **opt):
    """Exact number of (p,q)-bicliques (python int); optionally with stats."""
    o = make_opts(**opt)
    out, st = bc_u128(), bc_stats()
    s = _lib.bc_count(g.handle, p, q, ctypes.byref(o), ctypes.byref(out), ctypes.byref(st))
    if s != BC_OK:
        raise BCError(s, "bc_count")
    return (out.value, st.as_dict()) if with_stats else out.value


def bc_htb_stats(g: Graph, side: int):
    """(words, one_blocks) of the HTB of one side's rows."""
    w, o = ctypes.c_uint64(), ctypes.c_uint64()
    s = _lib.bc_htb_stats(g.handle, side, ctypes.byref(w), ctypes.byref(o))
    if s != BC_OK:
        raise BCError(s, "bc_htb_stats")
    return w.value, o.value


def bc_count_noalloc(g: Graph, p: int, q: int, **opt):
    """Exact count with all device scratch in the library's fixed buffer."""
    o = make_opts(**opt)
    out = bc_u128()
    s = _lib.bc_count_noalloc(g.handle, p, q, ctypes.byref(o), ctypes.byref(out))
    if s != BC_OK:
        raise BCError(s, "bc_count_noalloc")
    return out.value


def bc_count_per_vertex(g: Graph, p: int, q: int, side: int, **opt):
    """Per-vertex counts (python ints) for the vertices of `side`, by vertex id:
    the (p,q)-bicliques holding each vertex."""
    n = g.n_u if side == BC_ANCHOR_U else g.n_v
    o = make_opts(**opt)
    out = (bc_u128 * max(1, n))()
    s = _lib.bc_count_per_vertex(g.handle, p, q, side, ctypes.byref(o), out)
    if s != BC_OK:
        raise BCError(s, "bc_count_per_vertex")
    return [out[i].value for i in range(n)]


def bc_count_roots(g: Graph, p: int, q: int, anchor: int, rank_lo: int, rank_hi: int, with_stats=False, **opt):
    """Partial count over roots with rank in [rank_lo, rank_hi) on the anchor side."""
    o = make_opts(**opt)
    out, st = bc_u128(), bc_stats()
    s = _lib.bc_count_roots(g.handle, p, q, anchor, rank_lo, rank_hi, ctypes.byref(o), ctypes.byref(out),
                            ctypes.byref(st))
    if s != BC_OK:
        raise BCError(s, "bc_count_roots")
    return (out.value, st.as_dict()) if with_stats else out.value


def bc_count_batch(graphs, ps, qs, with_stats=False, **opt):
    """Counts for many (graph, p, q) in one set of launches: (values, statuses),
    plus the aggregate stats when with_stats."""
    n = len(graphs)
    hs = (ctypes.c_void_p * max(1, n))(*[g.handle for g in graphs])
    pa = np.ascontiguousarray(ps, dtype=np.uint32)
    qa = np.ascontiguousarray(qs, dtype=np.uint32)
    out = (bc_u128 * max(1, n))()
    st = np.zeros(max(1, n), dtype=np.int32)
    o = make_opts(**opt)
    agg = bc_stats()
    s = _lib.bc_count_batch(hs, pa.ctypes.data, qa.ctypes.data, n, ctypes.byref(o), out, st.ctypes.data,
                            ctypes.byref(agg))
    if s != BC_OK:
        raise BCError(s, "bc_count_batch")
    res = ([out[i].value for i in range(n)], [int(x) for x in st[:n]])
    return res + (agg.as_dict(),) if with_stats else res


def bc_scratch_estimate(g: Graph, p: int, q: int, **opt) -> int:
    """Upper bound on the device scratch (bytes) of bc_count(g, p, q) capped at it."""
    o = make_opts(**opt)
    b = ctypes.c_uint64()
    s = _lib.bc_scratch_estimate(g.handle, p, q, ctypes.byref(o), ctypes.byref(b))
    if s != BC_OK:
        raise BCError(s, "bc_scratch_estimate")
    return b.value


def bc_partition(g: Graph, p: int, q: int, anchor: int, budget_bytes: int):
    """(part_of_rank array, number of groups) of BCPar over the anchor side's roots."""
    n = g.n_u if anchor == BC_ANCHOR_U else g.n_v
    part = np.zeros(max(1, n), dtype=np.uint32)
    npart = ctypes.c_uint32()
    s = _lib.bc_partition(g.handle, p, q, anchor, budget_bytes, part.ctypes.data, ctypes.byref(npart))
    if s != BC_OK:
        raise BCError(s, "bc_partition")
    return part[:n], npart.value


def bc_count_partition(g: Graph, p: int, q: int, anchor: int, part_of_rank, part: int, **opt):
    """(count of group `part`, edges of its closure subgraph)."""
    pr = np.ascontiguousarray(part_of_rank, dtype=np.uint32)
    o = make_opts(**opt)
    out, edges = bc_u128(), ctypes.c_uint64()
    s = _lib.bc_count_partition(g.handle, p, q, anchor, pr.ctypes.data, part, ctypes.byref(o), ctypes.byref(out),
                                ctypes.byref(edges))
    if s != BC_OK:
        raise BCError(s, "bc_count_partition")
    return out.value, edges.value


def bc_tune_batch(graphs, ps, qs, **opt) -> dict:
    """Schedule options chosen for bc_count_batch over these items, as a dict
    of the TUNED_KNOBS (pass them on with **)."""
    n = len(graphs)
    hs = (ctypes.c_void_p * max(1, n))(*[g.handle for g in graphs])
    pa = np.ascontiguousarray(ps, dtype=np.uint32)
    qa = np.ascontiguousarray(qs, dtype=np.uint32)
    base = make_opts(**opt)
    tuned = bc_opts()
    s = _lib.bc_tune_batch(hs, pa.ctypes.data, qa.ctypes.data, n, ctypes.byref(base), ctypes.byref(tuned))
    if s != BC_OK:
        raise BCError(s, "bc_tune_batch")
    return {k: getattr(tuned, k) for k in TUNED_KNOBS}


TUNED_KNOBS = ("waves_per_cu", "lds_words", "roots_per_wave", "switch_depth", "split_rows")


# ---------------------------------------------------------------------------
# Counting service (include/bc_server.h).

class bc_server_opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("max_pending", ctypes.c_uint32),
                ("memory_budget_bytes", ctypes.c_uint64), ("batch_timeout_ms", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class bc_query_stats(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("batch_id", ctypes.c_uint64), ("batch_size", ctypes.c_uint32), ("pad", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}


class bc_server_summary(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("timed_out", ctypes.c_uint64), ("failed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("qps", ctypes.c_double), ("mean_batch", ctypes.c_double), ("max_overlap", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}


def _bind_server():
    P, I32, U32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "bc_server_create": ([P, P], I32),
        "bc_server_add_graph": ([P, P, P], I32),
        "bc_server_submit": ([P, U32, U32, U32, U64, P], I32),
        "bc_server_poll": ([P, U64, ctypes.c_int, P, P], I32),
        "bc_server_stats": ([P, P], I32),
        "bc_server_now_ns": ([], U64),
        "bc_server_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(_lib, name)
        f.argtypes = args
        f.restype = res


_bind_server()
EXPORTED = EXPORTED + ("bc_server_create", "bc_server_add_graph", "bc_server_submit", "bc_server_poll",
                       "bc_server_stats", "bc_server_now_ns", "bc_server_destroy")


class Server:
    """Thin wrapper of a ``bc_server *``; graphs must outlive it."""

    def __init__(self, max_inflight=2, max_batch=256, max_pending=0, memory_budget_bytes=0, batch_timeout_ms=0):
        o = bc_server_opts()
        o.struct_size = ctypes.sizeof(bc_server_opts)
        o.max_inflight, o.max_batch, o.max_pending = max_inflight, max_batch, max_pending
        o.memory_budget_bytes, o.batch_timeout_ms = memory_budget_bytes, batch_timeout_ms
        h = ctypes.c_void_p()
        s = _lib.bc_server_create(ctypes.byref(o), ctypes.byref(h))
        if s != BC_OK:
            raise BCError(s, "bc_server_create")
        self.handle = h.value
        self._graphs = []

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_uint32()
        s = _lib.bc_server_add_graph(self.handle, g.handle, ctypes.byref(gid))
        if s != BC_OK:
            raise BCError(s, "bc_server_add_graph")
        self._graphs.append(g)
        return gid.value

    def submit(self, graph_id: int, p: int, q: int, deadline_ns: int = 0) -> int:
        """Ticket id, or raises BCError (e.g. BC_E_REJECTED)."""
        t = ctypes.c_uint64()
        s = _lib.bc_server_submit(self.handle, graph_id, p, q, deadline_ns, ctypes.byref(t))
        if s != BC_OK:
            raise BCError(s, "bc_server_submit")
        return t.value

    def poll(self, ticket: int, block: bool = True):
        """(status, count or None, stats dict)."""
        out, st = bc_u128(), bc_query_stats()
        s = _lib.bc_server_poll(self.handle, ticket, 1 if block else 0, ctypes.byref(out), ctypes.byref(st))
        return s, (out.value if s == BC_OK else None), st.as_dict()

    def stats(self) -> dict:
        st = bc_server_summary()
        s = _lib.bc_server_stats(self.handle, ctypes.byref(st))
        if s != BC_OK:
            raise BCError(s, "bc_server_stats")
        return st.as_dict()

    @staticmethod
    def now_ns() -> int:
        return _lib.bc_server_now_ns()

    def close(self):
        if self.handle:
            _lib.bc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
