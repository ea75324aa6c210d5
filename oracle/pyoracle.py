"""ctypes front-end of the C oracle -- TEST INFRASTRUCTURE ONLY.

Every function takes a canonical CSR (row_ptr int64[n+1], col int32[nnz])
and returns exact Python ints.  Pattern edge lists are 0-based vertex pairs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

P_I64 = ctypes.POINTER(ctypes.c_int64)
P_I32 = ctypes.POINTER(ctypes.c_int32)
P_U64 = ctypes.POINTER(ctypes.c_uint64)

# The named patterns of the paper's problems (Sec. 2.1; motif shapes are the
# connected 3- and 4-vertex graphs), as 0-based edge lists.
PATTERNS = {
    "edge": (2, [(0, 1)]),
    "wedge": (3, [(0, 1), (0, 2)]),
    "triangle": (3, [(0, 1), (1, 2), (0, 2)]),
    "path4": (4, [(0, 1), (1, 2), (2, 3)]),
    "star3": (4, [(0, 1), (0, 2), (0, 3)]),
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "tailed_triangle": (4, [(0, 1), (1, 2), (0, 2), (2, 3)]),
    "diamond": (4, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3)]),
    "clique4": (4, [(i, j) for i in range(4) for j in range(i + 1, 4)]),
    "clique5": (5, [(i, j) for i in range(5) for j in range(i + 1, 5)]),
}
MOTIF3 = ["wedge", "triangle"]
MOTIF4 = ["path4", "star3", "cycle4", "tailed_triangle", "diamond", "clique4"]


def clique(k):
    return (k, [(i, j) for i in range(k) for j in range(i + 1, k)])


def load(path):
    """Load an oracle library from `path` with its argument types declared."""
    L = ctypes.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = load(path)
    return _lib


def _declare(L):
    L.orc_pattern_aut.argtypes = [ctypes.c_int, P_I32, ctypes.c_int, P_U64]
    for name in ("orc_count_subsets", "orc_count_embed"):
        f = getattr(L, name)
        f.argtypes = [ctypes.c_int64, P_I64, P_I32, ctypes.c_int, P_I32,
                      ctypes.c_int, ctypes.c_int, P_U64]
    L.orc_list_embed.argtypes = [ctypes.c_int64, P_I64, P_I32, ctypes.c_int, P_I32,
                                 ctypes.c_int, ctypes.c_int, P_I32, ctypes.c_int64, P_U64]
    L.orc_triangles.argtypes = [ctypes.c_int64, P_I64, P_I32, ctypes.c_int,
                                P_U64, P_U64, P_U64]
    L.orc_cliques.argtypes = [ctypes.c_int64, P_I64, P_I32, ctypes.c_int,
                              ctypes.c_int, P_U64]
    L.orc_cycle4.argtypes = [ctypes.c_int64, P_I64, P_I32, P_U64]
    L.orc_cycle4_trace.argtypes = [ctypes.c_int64, P_I64, P_I32, P_U64]
    for name in ("orc_nonind4", "orc_motifs3", "orc_motifs4", "orc_nonind4_local"):
        getattr(L, name).argtypes = [ctypes.c_int64, P_I64, P_I32,
                                     ctypes.c_int, P_U64]
    L.orc_num_threads.restype = ctypes.c_int


class OracleError(RuntimeError):
    pass


def _check(st):
    if st != 0:
        raise OracleError({-1: "invalid argument", -2: "count overflows 64 bits",
                           -3: "out of memory"}.get(st, str(st)))


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return g.n, rp, col, rp.ctypes.data_as(P_I64), col.ctypes.data_as(P_I32)


def _pat(pattern):
    if isinstance(pattern, str):
        pattern = PATTERNS[pattern]
    k, edges = pattern
    pe = np.ascontiguousarray(np.array(edges, dtype=np.int32).reshape(-1))
    if pe.size == 0:
        pe = np.zeros(2, dtype=np.int32)
    return k, len(edges), pe


def num_threads() -> int:
    return lib().orc_num_threads()


def aut(pattern) -> int:
    k, npe, pe = _pat(pattern)
    out = ctypes.c_uint64()
    _check(lib().orc_pattern_aut(k, pe.ctypes.data_as(P_I32), npe, ctypes.byref(out)))
    return out.value


def count_subsets(g, pattern, induced: bool) -> int:
    """The definition itself (tiny graphs, n <= 64)."""
    n, rp, col, prp, pcol = _csr(g)
    k, npe, pe = _pat(pattern)
    out = ctypes.c_uint64()
    _check(lib().orc_count_subsets(n, prp, pcol, k, pe.ctypes.data_as(P_I32),
                                   npe, int(induced), ctypes.byref(out)))
    return out.value


def count_embed(g, pattern, induced: bool) -> int:
    """Embeddings / |Aut(P)| (moderate graphs)."""
    n, rp, col, prp, pcol = _csr(g)
    k, npe, pe = _pat(pattern)
    out = ctypes.c_uint64()
    _check(lib().orc_count_embed(n, prp, pcol, k, pe.ctypes.data_as(P_I32),
                                 npe, int(induced), ctypes.byref(out)))
    return out.value


def list_embed(g, pattern, induced: bool, cap: int | None = None):
    """Listing: one row per distinct match, row[i] = graph vertex of pattern
    vertex i, each the smallest of its automorphic images (serial; moderate
    graphs).  Returns (rows[min(count, cap), k] int32, count)."""
    n, rp, col, prp, pcol = _csr(g)
    k, npe, pe = _pat(pattern)
    if cap is None:
        cap = count_embed(g, pattern, induced)
    out = np.zeros((max(cap, 1), k), dtype=np.int32)
    cnt = ctypes.c_uint64()
    _check(lib().orc_list_embed(n, prp, pcol, k, pe.ctypes.data_as(P_I32), npe, int(induced),
                                out.ctypes.data_as(P_I32), cap, ctypes.byref(cnt)))
    return out[:min(cap, cnt.value)], cnt.value


def triangles(g, order: int = 1, local: bool = False):
    n, rp, col, prp, pcol = _csr(g)
    out = ctypes.c_uint64()
    if local:
        tv = np.zeros(max(n, 1), dtype=np.uint64)
        te = np.zeros(max(g.nnz, 1), dtype=np.uint64)
        _check(lib().orc_triangles(n, prp, pcol, order, ctypes.byref(out),
                                   tv.ctypes.data_as(P_U64), te.ctypes.data_as(P_U64)))
        return out.value, tv[:n], te[:g.nnz]
    _check(lib().orc_triangles(n, prp, pcol, order, ctypes.byref(out), None, None))
    return out.value


def cliques(g, k: int, order: int = 1) -> int:
    n, rp, col, prp, pcol = _csr(g)
    out = ctypes.c_uint64()
    _check(lib().orc_cliques(n, prp, pcol, k, order, ctypes.byref(out)))
    return out.value


def cycle4(g) -> int:
    n, rp, col, prp, pcol = _csr(g)
    out = ctypes.c_uint64()
    _check(lib().orc_cycle4(n, prp, pcol, ctypes.byref(out)))
    return out.value


def cycle4_trace(g) -> int:
    """4-cycles from tr(A^4) (closed 4-walks), a route with no ranking."""
    n, rp, col, prp, pcol = _csr(g)
    out = ctypes.c_uint64()
    _check(lib().orc_cycle4_trace(n, prp, pcol, ctypes.byref(out)))
    return out.value


def _vec(name, g, order, size):
    n, rp, col, prp, pcol = _csr(g)
    out = np.zeros(size, dtype=np.uint64)
    _check(getattr(lib(), name)(n, prp, pcol, order, out.ctypes.data_as(P_U64)))
    return [int(x) for x in out]


def nonind4(g, order: int = 1):
    """[path4, star3, cycle4, tailed_triangle, diamond, clique4], non-induced."""
    return _vec("orc_nonind4", g, order, 6)


def nonind4_local(g, order: int = 1):
    """[path4, star3, tailed_triangle, diamond], non-induced (the counts that
    need only triangle and degree terms)."""
    return _vec("orc_nonind4_local", g, order, 4)


def motifs3(g, order: int = 1):
    """Induced [wedge, triangle]."""
    return _vec("orc_motifs3", g, order, 2)


def motifs4(g, order: int = 1):
    """Induced [path4, star3, cycle4, tailed_triangle, diamond, clique4]."""
    return _vec("orc_motifs4", g, order, 6)


def count(g, name: str, induced: bool, order: int = 1) -> int:
    """Count a named pattern by the fastest oracle route for it."""
    k, _ = PATTERNS[name]
    if name == "edge":
        return g.m
    if name == "triangle":
        return triangles(g, order)
    if name.startswith("clique"):
        return cliques(g, k, order)
    if k == 3:
        m3 = motifs3(g, order)
        if induced:
            return m3[MOTIF3.index(name)]
        # non-induced wedge = sum C(d,2)
        return m3[0] + 3 * m3[1]
    if k == 4:
        if induced:
            return motifs4(g, order)[MOTIF4.index(name)]
        if name == "cycle4":
            return cycle4(g)
        return nonind4(g, order)[MOTIF4.index(name)]
    return count_embed(g, PATTERNS[name], induced)
