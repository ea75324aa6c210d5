"""Seeded synthetic input graphs.

This module only *generates inputs*: it holds none of the counting method's
arithmetic.  Both the CPU oracle (test side) and the HIP path consume what it
produces, so it is deliberately kept free of any set operation, orientation,
plan or count.

Every generator returns a canonical undirected simple graph in CSR form
(the input format of the graph loader, paper Sec. 4.2 "Graph Loader and
Preprocessor" and Table 3's note that data graphs are symmetric with no loops
or duplicate edges):

* ``row_ptr``: int64[n + 1], ``col``: int32[2m]
* every undirected edge {u, v} appears as u->v and v->u
* each neighbour list sorted ascending, no self loops, no duplicates.

The random families stand in for the paper's real-world datasets (Table 3),
which are not available: Erdos-Renyi G(n, p), R-MAT / Kronecker, and
Chung-Lu power-law graphs.  Small structured families (complete, complete
multipartite, bipartite, paths, cycles, stars, grids, hypercubes) give closed
form counts for tests.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def max_degree(self) -> int:
        return int(self.degrees().max()) if self.n else 0

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()


# ---------------------------------------------------------------------------
# canonicalisation of an undirected edge multiset into CSR
# ---------------------------------------------------------------------------

def from_edges(n: int, u, v, name: str = "") -> CSR:
    """Symmetrise, drop self loops and duplicates, sort, and build CSR."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.shape != v.shape:
        raise ValueError("edge endpoint arrays differ in length")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n
    hi = key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    key2 = np.sort(src * np.int64(n) + dst)
    src = key2 // n
    dst = key2 % n
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr, dst.astype(np.int32), name)


def relabel(g: CSR, perm: np.ndarray, name: str | None = None) -> CSR:
    """Rename vertex i to perm[i]; the result is canonical again."""
    perm = np.asarray(perm, dtype=np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    return from_edges(g.n, perm[src], perm[g.col.astype(np.int64)],
                      g.name if name is None else name)


def disjoint_union(*gs: CSR) -> CSR:
    us, vs, off = [], [], 0
    for g in gs:
        src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
        us.append(src + off)
        vs.append(g.col.astype(np.int64) + off)
        off += g.n
    return from_edges(off, np.concatenate(us) if us else [],
                      np.concatenate(vs) if vs else [], "union")


def to_edge_list(g: CSR):
    """Upper-triangle (u < v) edge list of a canonical CSR."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    k = src < dst
    return src[k], dst[k]


# ---------------------------------------------------------------------------
# structured families (closed-form counts)
# ---------------------------------------------------------------------------

def complete(n: int) -> CSR:
    iu = np.triu_indices(n, 1)
    return from_edges(n, iu[0], iu[1], f"K{n}")


def complete_multipartite(parts) -> CSR:
    parts = [int(p) for p in parts]
    lab = np.repeat(np.arange(len(parts)), parts)
    n = int(sum(parts))
    iu = np.triu_indices(n, 1)
    k = lab[iu[0]] != lab[iu[1]]
    return from_edges(n, iu[0][k], iu[1][k], "K" + ",".join(map(str, parts)))


def complete_bipartite(a: int, b: int) -> CSR:
    return complete_multipartite([a, b])


def path(n: int) -> CSR:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, f"P{n}")


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, f"C{n}")


def star(leaves: int) -> CSR:
    return from_edges(leaves + 1, np.zeros(leaves, dtype=np.int64),
                      np.arange(1, leaves + 1), f"S{leaves}")


def grid(r: int, c: int) -> CSR:
    idx = np.arange(r * c).reshape(r, c)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(r * c, u, v, f"grid{r}x{c}")


def hypercube(d: int) -> CSR:
    n = 1 << d
    us, vs = [], []
    for b in range(d):
        x = np.arange(n)
        y = x ^ (1 << b)
        k = x < y
        us.append(x[k])
        vs.append(y[k])
    return from_edges(n, np.concatenate(us), np.concatenate(vs), f"Q{d}")


def empty(n: int) -> CSR:
    return from_edges(n, [], [], f"E{n}")


# ---------------------------------------------------------------------------
# random families
# ---------------------------------------------------------------------------

def erdos_renyi(n: int, p: float, seed: int) -> CSR:
    """G(n, p): each unordered pair is an edge independently with prob. p.

    For up to ~8M pairs one Bernoulli draw is made per pair i < j in
    row-major order.  Larger graphs walk the n*n grid of ordered cells with
    geometric skips (the same distribution) and keep the cells with i < j.
    """
    rng = np.random.default_rng(seed)
    pairs = n * (n - 1) // 2
    if pairs <= 8_000_000:
        iu = np.triu_indices(n, 1)
        hit = rng.random(pairs) < p
        return from_edges(n, iu[0][hit], iu[1][hit], f"ER({n},{p})")
    if p <= 0:
        return empty(n)
    total = n * n
    cells = []
    pos = -1
    batch = int(total * p * 1.1) + 1024
    while True:
        gaps = rng.geometric(p, size=batch).astype(np.int64)
        c = pos + np.cumsum(gaps)
        c = c[c < total]
        if c.size:
            cells.append(c)
            pos = int(c[-1])
        if c.size < batch:
            break
    c = np.concatenate(cells) if cells else np.zeros(0, np.int64)
    i = c // n
    j = c % n
    k = i < j
    return from_edges(n, i[k], j[k], f"ER({n},{p})")


def rmat(scale: int, edge_factor: float, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0, n_keep: int | None = None,
         samples: int | None = None) -> CSR:
    """R-MAT / Kronecker generator (no per-level noise).

    ``samples`` edge draws (default edge_factor * 2^scale); each draw descends
    ``scale`` levels choosing quadrant a/b/c/d.  Vertex ids are then permuted
    by a seeded permutation of 2^scale ids.  With ``n_keep`` the draws touching
    ids >= n_keep are dropped.  Loops and duplicates are removed and the graph
    symmetrised.
    """
    rng = np.random.default_rng(seed)
    nv = 1 << scale
    m = int(samples if samples is not None else round(edge_factor * nv))
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for lvl in range(scale):
        r = rng.random(m, dtype=np.float32)
        bit = np.int64(1) << (scale - 1 - lvl)
        down = r >= ab                       # quadrant c or d: source bit set
        right = ((r >= a) & (r < ab)) | (r >= abc)   # quadrant b or d: dest bit set
        src |= np.where(down, bit, 0)
        dst |= np.where(right, bit, 0)
    perm = rng.permutation(nv).astype(np.int64)
    src = perm[src]
    dst = perm[dst]
    n = nv
    if n_keep is not None:
        k = (src < n_keep) & (dst < n_keep)
        src, dst = src[k], dst[k]
        n = int(n_keep)
    return from_edges(n, src, dst, f"RMAT(s{scale},ef{edge_factor})")


def chung_lu(n: int, avg_degree: float, gamma: float, w_max: float,
             m_target: int, seed: int) -> CSR:
    """Chung-Lu power-law graph with exactly ``m_target`` distinct edges.

    Expected weights w_i = w_max * (i0 / (i + i0))^(1/(gamma-1)), with i0
    solved by bisection so the mean weight equals ``avg_degree``.  Endpoint
    pairs are drawn proportionally to w; loops and duplicates are dropped and
    the first ``m_target`` distinct edges (in draw order) are kept.  Ids are
    then permuted by a seeded permutation.
    """
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.float64)
    ex = 1.0 / (gamma - 1.0)

    def mean_w(i0):
        return float(np.mean(w_max * (i0 / (i + i0)) ** ex))

    lo, hi = 1e-6, float(n)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_w(mid) < avg_degree:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    w = w_max * (i0 / (i + i0)) ** ex
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    keys = []
    have = 0
    while True:
        need = m_target - have
        batch = int(need * 1.25) + 4096
        x = np.searchsorted(cdf, rng.random(batch), side="right")
        y = np.searchsorted(cdf, rng.random(batch), side="right")
        x = np.minimum(x, n - 1).astype(np.int64)
        y = np.minimum(y, n - 1).astype(np.int64)
        k = x != y
        kk = np.minimum(x[k], y[k]) * np.int64(n) + np.maximum(x[k], y[k])
        keys.append(kk)
        allk = np.concatenate(keys)
        uniq, first = np.unique(allk, return_index=True)
        have = uniq.size
        if have >= m_target:
            order = np.argsort(first, kind="stable")[:m_target]
            sel = uniq[order]
            break
        keys = [allk]
    u = sel // n
    v = sel % n
    perm = rng.permutation(n).astype(np.int64)
    return from_edges(n, perm[u], perm[v],
                      f"ChungLu({n},{avg_degree},{gamma},{w_max})")


# ---------------------------------------------------------------------------
# the benchmark workloads (sizes of the paper's graphs, synthetic stand-ins)
# ---------------------------------------------------------------------------

def workload_er_triangle(seed: int = 1) -> CSR:
    """Erdos-Renyi G(n=2000, p=0.01): the small triangle-counting case."""
    return erdos_renyi(2000, 0.01, seed)


def workload_rmat_s20(seed: int = 2) -> CSR:
    """R-MAT scale 20, edge factor 16, (a,b,c) = (0.57, 0.19, 0.19)."""
    return rmat(20, 16, 0.57, 0.19, 0.19, seed)


def workload_rmat_s16(seed: int = 1) -> CSR:
    """R-MAT scale 16, edge factor 16, (a,b,c) = (0.57, 0.19, 0.19): the
    listing workload (its 4-cliques fit a device buffer)."""
    return rmat(16, 16, 0.57, 0.19, 0.19, seed)


def workload_chung_lu_4m(seed: int = 3) -> CSR:
    """Chung-Lu, n = 4M, 60M edges (average degree 30), exponent 2.1."""
    return chung_lu(4_000_000, 30.0, 2.1, 1e5, 60_000_000, seed)


def batch_graph(i: int) -> CSR:
    """Graph i (0 <= i < 256) of the many-small-graphs batch.

    n = round(exp(U(ln 1e3, ln 2e5))); even i: G(n, p = d/(n-1)) with
    d ~ U(8, 40); odd i: R-MAT at scale ceil(log2 n) with edge factor
    ~ U{8..32}, ef*n samples, ids >= n dropped.
    """
    rng = np.random.default_rng(10_000 + i)
    n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
    sub = int(rng.integers(0, 2**31 - 1))
    if i % 2 == 0:
        d = float(rng.uniform(8, 40))
        g = erdos_renyi(n, d / (n - 1), sub)
    else:
        s = int(math.ceil(math.log2(n)))
        ef = int(rng.integers(8, 33))
        g = rmat(s, ef, seed=sub, n_keep=n, samples=ef * n)
    g.name = f"batch{i}"
    return g


def serve_pool_graph(i: int) -> CSR:
    """Graph i (0 <= i < 32) of the resident serving pool: R-MAT ef 16,
    four graphs per scale for scales 16..23."""
    s = 16 + i // 4
    g = rmat(s, 16, seed=20_000 + i)
    g.name = f"pool{i}"
    return g
