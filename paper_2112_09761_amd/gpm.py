"""Python binding of libgpm (include/gpm.h): argument marshalling only.

Every count is computed by the HIP library; this module only converts
arguments.  If libgpm.so is missing it raises instead of falling back to
anything else.  Names follow the C entry points (``gpm_count`` ->
``Context.count`` etc.).  Device arrays may be passed as torch tensors on the
context's device (their data pointers go to the library with
GPM_PTRS_DEVICE); host arrays as numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpm.so")

GPM_OK = 0
STATUS = {0: "GPM_OK", -1: "GPM_E_INVAL", -2: "GPM_E_CSR", -3: "GPM_E_PATTERN",
          -4: "GPM_E_NOMEM", -5: "GPM_E_DEVICE", -6: "GPM_E_UNSUPPORTED",
          -7: "GPM_E_BUSY", -8: "GPM_E_TIMEOUT"}
GPM_VERTEX_INDUCED = 0
GPM_EDGE_INDUCED = 1
GPM_CSR_SYMMETRIC = 1
GPM_CSR_DAG = 2
GPM_PTRS_DEVICE = 4
GPM_VALIDATE = 8
GPM_QUERY_COUNT = 0
GPM_QUERY_MOTIFS = 1
MAX_K = 8
MAX_PATTERN_EDGES = 28

MOTIF3 = ["wedge", "triangle"]
MOTIF4 = ["path4", "star3", "cycle4", "tailed_triangle", "diamond", "clique4"]

EXPORTS = [
    "gpm_create", "gpm_destroy", "gpm_last_error", "gpm_set_option", "gpm_get_stats",
    "gpm_load_csr", "gpm_unload", "gpm_graph_info", "gpm_pattern_clique",
    "gpm_pattern_named", "gpm_pattern_from_edges", "gpm_plan", "gpm_frontier_waves",
    "gpm_count", "gpm_motifs", "gpm_count_batch", "gpm_submit", "gpm_poll", "gpm_wait",
    "gpm_inflight", "gpm_validate_csr", "gpm_prepare", "gpm_list", "gpm_serve_state",
    "gpm_count_noalloc",
]


class Pattern(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("edges", ctypes.c_int32 * (2 * MAX_PATTERN_EDGES))]

    def edge_list(self):
        return [(self.edges[2 * i], self.edges[2 * i + 1]) for i in range(self.n_edges)]


class Query(ctypes.Structure):
    _fields_ = [("graph_id", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("mode_or_k", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pattern", Pattern)]


class GraphMeta(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("max_out_degree", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


MAX_LAUNCH_STATS = 8   # GPM_MAX_LAUNCH_STATS
# launch_kinds bits
KIND_LGS_WAVE = 1 << 5
KIND_LGS_BLOCK = 1 << 7


class Stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("tasks", ctypes.c_int64), ("waves", ctypes.c_int64),
                ("chunk", ctypes.c_int64), ("elements", ctypes.c_int64),
                ("list_fetches", ctypes.c_int64), ("frontier_written", ctypes.c_int64),
                ("bitmap_words", ctypes.c_int64),
                ("frontier_bytes", ctypes.c_int64),
                ("launches", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("n_launch_stats", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("launch_kinds", ctypes.c_uint32 * MAX_LAUNCH_STATS),
                ("launch_ms", ctypes.c_double * MAX_LAUNCH_STATS),
                ("launch_elements", ctypes.c_int64 * MAX_LAUNCH_STATS),
                ("launch_fetches", ctypes.c_int64 * MAX_LAUNCH_STATS),
                ("launch_written", ctypes.c_int64 * MAX_LAUNCH_STATS),
                ("launch_words", ctypes.c_int64 * MAX_LAUNCH_STATS)]

    def as_dict(self):
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = list(v)[:self.n_launch_stats] if f.startswith("launch_") else v
        return d


class ServeInfo(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int64), ("running", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("busy_slots", ctypes.c_int64),
                ("frontier_in_use", ctypes.c_int64), ("budget", ctypes.c_int64),
                ("memory_waits", ctypes.c_int64), ("admitted", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("clique", ctypes.c_int32), ("aut", ctypes.c_int32),
                ("root_bound", ctypes.c_int32), ("n_buffers", ctypes.c_int32),
                ("n_restrictions", ctypes.c_int32), ("order", ctypes.c_int32 * MAX_K),
                ("restrictions", ctypes.c_int32 * (2 * MAX_PATTERN_EDGES)),
                ("count_only_r", ctypes.c_int32)]


class GpmError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {message}")


_lib = None
P = ctypes.POINTER
c_i32, c_i64, c_u64, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
c_vp = ctypes.c_void_p


def lib():
    """Load libgpm.so (built by build_lib.build()); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.gpm_create.argtypes = [P(c_vp), ctypes.c_int, c_vp, c_sz]
        L.gpm_destroy.argtypes = [c_vp]
        L.gpm_last_error.argtypes = [c_vp]
        L.gpm_last_error.restype = ctypes.c_char_p
        L.gpm_set_option.argtypes = [c_vp, ctypes.c_char_p, c_i64]
        L.gpm_get_stats.argtypes = [c_vp, P(Stats)]
        L.gpm_load_csr.argtypes = [c_vp, c_i64, c_i64, c_vp, c_vp, ctypes.c_uint32, P(c_i32)]
        L.gpm_unload.argtypes = [c_vp, c_i32]
        L.gpm_graph_info.argtypes = [c_vp, c_i32, P(GraphMeta)]
        L.gpm_pattern_clique.argtypes = [ctypes.c_int, P(Pattern)]
        L.gpm_pattern_named.argtypes = [ctypes.c_char_p, P(Pattern)]
        L.gpm_pattern_from_edges.argtypes = [ctypes.c_int, ctypes.c_int, P(c_i32), P(Pattern)]
        L.gpm_plan.argtypes = [P(Pattern), ctypes.c_int, P(PlanInfo)]
        L.gpm_frontier_waves.argtypes = [c_i64, c_i32, c_i64, c_i64, c_i64, P(c_i64)]
        L.gpm_count.argtypes = [c_vp, c_i32, P(Pattern), ctypes.c_int, P(c_u64)]
        L.gpm_count_noalloc.argtypes = [c_vp, c_i32, P(Pattern), ctypes.c_int, P(c_u64)]
        L.gpm_motifs.argtypes = [c_vp, c_i32, ctypes.c_int, P(c_u64), c_sz]
        L.gpm_list.argtypes = [c_vp, c_i32, P(Pattern), ctypes.c_int, c_vp, c_i64, P(c_u64)]
        L.gpm_count_batch.argtypes = [c_vp, c_i32, P(Query), P(c_u64)]
        L.gpm_submit.argtypes = [c_vp, P(Query), P(c_i64)]
        L.gpm_poll.argtypes = [c_vp, c_i64, P(ctypes.c_int), P(c_u64)]
        L.gpm_wait.argtypes = [c_vp, c_i64, c_i64, P(c_u64)]
        L.gpm_inflight.argtypes = [c_vp, P(c_i64)]
        L.gpm_serve_state.argtypes = [c_vp, P(ServeInfo)]
        L.gpm_validate_csr.argtypes = [c_i64, c_i64, c_vp, c_vp, ctypes.c_uint32]
        L.gpm_prepare.argtypes = [c_vp, c_i32]
        for name in EXPORTS:
            if name != "gpm_last_error":
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(st, ctx=None):
    if st != GPM_OK:
        msg = ""
        if ctx:
            msg = (lib().gpm_last_error(ctx) or b"").decode(errors="replace")
        raise GpmError(st, msg)


# --- patterns ----------------------------------------------------------------

def pattern_clique(k: int) -> Pattern:
    p = Pattern()
    _check(lib().gpm_pattern_clique(k, ctypes.byref(p)))
    return p


def pattern_named(name: str) -> Pattern:
    p = Pattern()
    _check(lib().gpm_pattern_named(name.encode(), ctypes.byref(p)))
    return p


def pattern_from_edges(k: int, edges) -> Pattern:
    arr = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))
    if arr.size == 0:
        arr = np.zeros(2, dtype=np.int32)
    p = Pattern()
    _check(lib().gpm_pattern_from_edges(k, len(edges), arr.ctypes.data_as(P(c_i32)),
                                        ctypes.byref(p)))
    return p


def as_pattern(p) -> Pattern:
    if isinstance(p, Pattern):
        return p
    if isinstance(p, str):
        return pattern_named(p)
    k, edges = p
    return pattern_from_edges(k, edges)


def plan(pattern, mode: int) -> dict:
    info = PlanInfo()
    _check(lib().gpm_plan(ctypes.byref(as_pattern(pattern)), mode, ctypes.byref(info)))
    return {
        "k": info.k, "clique": bool(info.clique), "aut": info.aut,
        "root_bound": bool(info.root_bound), "n_buffers": info.n_buffers,
        "order": list(info.order[:info.k]),
        "restrictions": [(info.restrictions[2 * i], info.restrictions[2 * i + 1])
                         for i in range(info.n_restrictions)],
        "count_only_r": info.count_only_r,
    }


def frontier_waves(free_bytes, x_levels, cap_elems, n_tasks, max_resident) -> int:
    out = c_i64()
    _check(lib().gpm_frontier_waves(free_bytes, x_levels, cap_elems, n_tasks, max_resident,
                                    ctypes.byref(out)))
    return out.value


def validate_csr(row_ptr, col, flags: int = GPM_CSR_SYMMETRIC) -> int:
    """gpm_validate_csr on host arrays; returns the status code."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    nnz = cl.size
    if nnz == 0:
        cl = np.zeros(1, dtype=np.int32)
    return lib().gpm_validate_csr(rp.size - 1, nnz, rp.ctypes.data_as(c_vp),
                                  cl.ctypes.data_as(c_vp), flags)


def count_query(graph_id, pattern, mode) -> Query:
    q = Query()
    q.graph_id = graph_id
    q.kind = GPM_QUERY_COUNT
    q.mode_or_k = mode
    q.pattern = as_pattern(pattern)
    return q


def motif_query(graph_id, k) -> Query:
    q = Query()
    q.graph_id = graph_id
    q.kind = GPM_QUERY_MOTIFS
    q.mode_or_k = k
    return q


# --- context -----------------------------------------------------------------

def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


class Context:
    """gpm_create / gpm_destroy around a device and a HIP stream."""

    def __init__(self, device: int = 0, stream=None, budget: int = 0):
        self._h = c_vp()
        _check(lib().gpm_create(ctypes.byref(self._h), device, _stream_handle(stream), budget))
        self.device = device
        self._keep = []

    def close(self):
        if self._h:
            lib().gpm_destroy(self._h)
            self._h = c_vp()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _ck(self, st):
        _check(st, self._h)

    def set_option(self, key: str, value: int):
        self._ck(lib().gpm_set_option(self._h, key.encode(), int(value)))

    def stats(self) -> dict:
        s = Stats()
        self._ck(lib().gpm_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def load_csr(self, row_ptr, col, flags: int = GPM_CSR_SYMMETRIC) -> int:
        """gpm_load_csr from numpy arrays or torch tensors (device tensors are
        passed by pointer with GPM_PTRS_DEVICE)."""
        gid = c_i32()
        if hasattr(row_ptr, "data_ptr"):
            n = int(row_ptr.numel()) - 1
            nnz = int(col.numel())
            if row_ptr.is_cuda:
                flags |= GPM_PTRS_DEVICE
            self._ck(lib().gpm_load_csr(self._h, n, nnz, c_vp(row_ptr.data_ptr()),
                                        c_vp(col.data_ptr()), flags, ctypes.byref(gid)))
            return gid.value
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        if cl.size == 0:
            cl = np.zeros(1, dtype=np.int32)
        self._ck(lib().gpm_load_csr(self._h, rp.size - 1, int(np.asarray(col).size),
                                    rp.ctypes.data_as(c_vp), cl.ctypes.data_as(c_vp),
                                    flags, ctypes.byref(gid)))
        return gid.value

    def load(self, g, flags: int = GPM_CSR_SYMMETRIC) -> int:
        """Load a synth.CSR graph."""
        return self.load_csr(g.row_ptr, g.col, flags)

    def prepare(self, graph_id: int):
        self._ck(lib().gpm_prepare(self._h, graph_id))

    def unload(self, graph_id: int):
        self._ck(lib().gpm_unload(self._h, graph_id))

    def graph_info(self, graph_id: int) -> dict:
        m = GraphMeta()
        self._ck(lib().gpm_graph_info(self._h, graph_id, ctypes.byref(m)))
        return {f: getattr(m, f) for f, _ in m._fields_}

    def count(self, graph_id: int, pattern, mode: int = GPM_VERTEX_INDUCED) -> int:
        out = c_u64()
        p = as_pattern(pattern)
        self._ck(lib().gpm_count(self._h, graph_id, ctypes.byref(p), mode, ctypes.byref(out)))
        return out.value

    def count_noalloc(self, graph_id: int, pattern, mode: int = GPM_VERTEX_INDUCED) -> int:
        """gpm_count_noalloc: the count with no allocation (the graph must be
        prepared for the query by an earlier count)."""
        out = c_u64()
        p = as_pattern(pattern)
        self._ck(lib().gpm_count_noalloc(self._h, graph_id, ctypes.byref(p), mode,
                                         ctypes.byref(out)))
        return out.value

    def list(self, graph_id: int, pattern, out, mode: int = GPM_VERTEX_INDUCED) -> int:
        """gpm_list into `out`, an int32 device tensor of shape [cap, k] on the
        context's device; returns the total number of matches (rows beyond
        out.shape[0] were counted, not written)."""
        import torch
        p = as_pattern(pattern)
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 device tensor")
        if out.dim() != 2 or out.shape[1] != p.k:
            raise ValueError(f"out must have shape [cap, {p.k}]")
        total = c_u64()
        ptr = c_vp(out.data_ptr()) if out.shape[0] > 0 else None
        self._ck(lib().gpm_list(self._h, graph_id, ctypes.byref(p), mode, ptr,
                                int(out.shape[0]), ctypes.byref(total)))
        return total.value

    def motifs(self, graph_id: int, k: int):
        n = 2 if k == 3 else 6
        out = (c_u64 * 6)()
        self._ck(lib().gpm_motifs(self._h, graph_id, k, out, n))
        return [int(x) for x in out[:n]]

    def count_batch(self, queries):
        qs = (Query * max(len(queries), 1))(*queries)
        out = (c_u64 * (6 * max(len(queries), 1)))()
        self._ck(lib().gpm_count_batch(self._h, len(queries), qs, out))
        res = []
        for i, q in enumerate(queries):
            row = [int(x) for x in out[6 * i:6 * i + 6]]
            if q.kind == GPM_QUERY_COUNT:
                res.append(row[0])
            else:
                res.append(row[:2] if q.mode_or_k == 3 else row)
        return res

    def submit(self, query: Query) -> int:
        t = c_i64()
        self._ck(lib().gpm_submit(self._h, ctypes.byref(query), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        done = ctypes.c_int()
        out = (c_u64 * 6)()
        self._ck(lib().gpm_poll(self._h, ticket, ctypes.byref(done), out))
        return bool(done.value), [int(x) for x in out]

    def wait(self, ticket: int, timeout_ns: int = -1):
        out = (c_u64 * 6)()
        self._ck(lib().gpm_wait(self._h, ticket, timeout_ns, out))
        return [int(x) for x in out]

    def serve_state(self) -> dict:
        r = ServeInfo()
        self._ck(lib().gpm_serve_state(self._h, ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in r._fields_}

    def inflight(self) -> int:
        n = c_i64()
        self._ck(lib().gpm_inflight(self._h, ctypes.byref(n)))
        return n.value
