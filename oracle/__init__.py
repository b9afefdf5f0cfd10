"""CPU oracle for exact (p,q)-biclique counting -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``oracle.c`` (plain C, compiled with gcc) via
ctypes and holds a pure-Python brute force for tiny graphs in ``brute.py``.
It shares no code with the device library and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_CSR, E_OVERFLOW, E_OOM, E_BUDGET = 0, -1, -2, -3, -4, -5
ORDER_ID, ORDER_DEGREE, ORDER_TWO_HOP = 0, 1, 2


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, no -march: the
    library may run on a different host CPU than the one that built it)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                        "-pthread", _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        lib.oracle_count.argtypes = [U64, U64, P, P, U32, U32, I, I, U64, U64, I, P, P, P]
        lib.oracle_count_ranks.argtypes = [U64, U64, P, P, U32, U32, I, P, U64, I, U64, P, P, P]
        lib.oracle_order.argtypes = [U64, U64, P, P, I, U32, P]
        lib.oracle_basic_sets.argtypes = [U64, U64, P, P, U32, P, U32, P, P, P, P]
        lib.oracle_htb_encode.argtypes = [P, U32, U32, P, P, P]
        lib.oracle_htb_intersect.argtypes = [P, P, U32, P, P, U32, P, P, P]
        lib.oracle_binom.argtypes = [U32, U32, P, P]
        lib.oracle_count_per_vertex.argtypes = [U64, U64, P, P, U32, U32, P, P, P, P]
        for f in (lib.oracle_count, lib.oracle_count_ranks, lib.oracle_order,
                  lib.oracle_basic_sets, lib.oracle_htb_encode, lib.oracle_htb_intersect,
                  lib.oracle_binom, lib.oracle_count_per_vertex):
            f.restype = I
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(indptr, indices):
    ip = np.ascontiguousarray(indptr, dtype=np.uint64)
    ix = np.ascontiguousarray(indices, dtype=np.uint32)
    if ix.size == 0:
        ix = np.zeros(1, dtype=np.uint32)
    return ip, ix


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def count_csr(n_u, n_v, indptr_u, indices_u, p, q, *, order_key=ORDER_ID, prune=True,
              rank_lo=0, rank_hi=None, threads=None, with_nodes=False):
    """Exact count of (p,q)-bicliques with L on the side whose CSR is given."""
    lib = _load()
    ip, ix = _csr(indptr_u, indices_u)
    lo, hi, nodes = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib.oracle_count(n_u, n_v, _ptr(ip), _ptr(ix), p, q, order_key, 1 if prune else 0,
                          rank_lo, n_u if rank_hi is None else rank_hi,
                          threads or default_threads(), ctypes.byref(lo), ctypes.byref(hi),
                          ctypes.byref(nodes))
    if rc != OK:
        raise OracleError(rc, "count")
    val = (hi.value << 64) | lo.value
    return (val, nodes.value) if with_nodes else val


def count(g, p, q, *, anchor="U", **kw):
    """Exact count for a ``graphgen.BipartiteGraph``-like object.  anchor="V"
    counts on the transposed graph with (q, p), which is the same number."""
    if anchor == "U":
        return count_csr(g.n_u, g.n_v, g.indptr_u, g.indices_u, p, q, **kw)
    return count_csr(g.n_v, g.n_u, g.indptr_v, g.indices_v, q, p, **kw)


def count_per_vertex(g, p, q):
    """Per-vertex counts (python ints): ([bicliques holding x in L for x in U],
    [bicliques holding v in R for v in V]).  Single-threaded; small graphs."""
    lib = _load()
    ip, ix = _csr(g.indptr_u, g.indices_u)
    ul = np.zeros(max(1, g.n_u), dtype=np.uint64)
    uh = np.zeros(max(1, g.n_u), dtype=np.uint64)
    vl = np.zeros(max(1, g.n_v), dtype=np.uint64)
    vh = np.zeros(max(1, g.n_v), dtype=np.uint64)
    rc = lib.oracle_count_per_vertex(g.n_u, g.n_v, _ptr(ip), _ptr(ix), p, q, _ptr(ul), _ptr(uh), _ptr(vl),
                                     _ptr(vh))
    if rc != OK:
        raise OracleError(rc, "count_per_vertex")
    return ([(int(h) << 64) | int(l) for l, h in zip(ul[:g.n_u], uh[:g.n_u])],
            [(int(h) << 64) | int(l) for l, h in zip(vl[:g.n_v], vh[:g.n_v])])


def count_ranks(g, p, q, ranks, *, anchor="U", order_key=ORDER_DEGREE, threads=None, max_nodes=0):
    """Per-root counts for the roots of the given ranks (list of python ints).

    With max_nodes > 0, a root needing more intersections than that is not
    computed and its entry is None."""
    lib = _load()
    if anchor == "U":
        n_u, n_v, ip, ix, pp, qq = g.n_u, g.n_v, g.indptr_u, g.indices_u, p, q
    else:
        n_u, n_v, ip, ix, pp, qq = g.n_v, g.n_u, g.indptr_v, g.indices_v, q, p
    ip, ix = _csr(ip, ix)
    r = np.ascontiguousarray(ranks, dtype=np.uint64)
    lo = np.zeros(max(1, r.size), dtype=np.uint64)
    hi = np.zeros(max(1, r.size), dtype=np.uint64)
    st = np.zeros(max(1, r.size), dtype=np.int32)
    rc = lib.oracle_count_ranks(n_u, n_v, _ptr(ip), _ptr(ix), pp, qq, order_key,
                                _ptr(r) if r.size else None, r.size,
                                threads or default_threads(), max_nodes, _ptr(lo), _ptr(hi), _ptr(st))
    if rc != OK:
        raise OracleError(rc, "count_ranks")
    return [((int(h) << 64) | int(l)) if s == OK else None
            for l, h, s in zip(lo[:r.size], hi[:r.size], st[:r.size])]


def order(n_u, n_v, indptr_u, indices_u, order_key, q=1):
    """by_rank array of the oracle's vertex order."""
    lib = _load()
    ip, ix = _csr(indptr_u, indices_u)
    out = np.zeros(max(1, n_u), dtype=np.uint32)
    rc = lib.oracle_order(n_u, n_v, _ptr(ip), _ptr(ix), order_key, q, _ptr(out))
    if rc != OK:
        raise OracleError(rc, "order")
    return out[:n_u]


def basic_sets(n_u, n_v, indptr_u, indices_u, q, L):
    """(C_R, C_L) of the Basic model after adding the vertices of L."""
    lib = _load()
    ip, ix = _csr(indptr_u, indices_u)
    Ls = np.ascontiguousarray(L, dtype=np.uint32)
    cr = np.zeros(max(1, n_v), dtype=np.uint32)
    cl = np.zeros(max(1, n_u), dtype=np.uint32)
    ncr, ncl = ctypes.c_uint32(), ctypes.c_uint32()
    rc = lib.oracle_basic_sets(n_u, n_v, _ptr(ip), _ptr(ix), q, _ptr(Ls), Ls.size, _ptr(cr),
                               ctypes.byref(ncr), _ptr(cl), ctypes.byref(ncl))
    if rc != OK:
        raise OracleError(rc, "basic_sets")
    return cr[:ncr.value].tolist(), cl[:ncl.value].tolist()


def htb_encode(ids, word_bits=32):
    """(Idx, Val) lists of the truncated-bitmap encoding of a sorted id list."""
    lib = _load()
    a = np.ascontiguousarray(ids, dtype=np.uint32)
    idx = np.zeros(max(1, a.size), dtype=np.uint64)
    val = np.zeros(max(1, a.size), dtype=np.uint64)
    n = ctypes.c_uint32()
    rc = lib.oracle_htb_encode(_ptr(a), a.size, word_bits, _ptr(idx), _ptr(val), ctypes.byref(n))
    if rc != OK:
        raise OracleError(rc, "htb_encode")
    return idx[:n.value].tolist(), val[:n.value].tolist()


def htb_intersect(a, b):
    """Intersection of two (Idx, Val) encodings, as an (Idx, Val) pair."""
    lib = _load()
    ia, va = (np.ascontiguousarray(x, dtype=np.uint64) for x in a)
    ib, vb = (np.ascontiguousarray(x, dtype=np.uint64) for x in b)
    n_max = max(1, min(ia.size, ib.size))
    oi = np.zeros(n_max, dtype=np.uint64)
    ov = np.zeros(n_max, dtype=np.uint64)
    n = ctypes.c_uint32()
    rc = lib.oracle_htb_intersect(_ptr(ia), _ptr(va), ia.size, _ptr(ib), _ptr(vb), ib.size,
                                  _ptr(oi), _ptr(ov), ctypes.byref(n))
    if rc != OK:
        raise OracleError(rc, "htb_intersect")
    return oi[:n.value].tolist(), ov[:n.value].tolist()


def binom(n, k):
    """C(n, k) from the oracle's Pascal table (raises on 128-bit overflow)."""
    lib = _load()
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib.oracle_binom(n, k, ctypes.byref(lo), ctypes.byref(hi))
    if rc != OK:
        raise OracleError(rc, "binom")
    return (hi.value << 64) | lo.value
