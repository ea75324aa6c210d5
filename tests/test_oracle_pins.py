"""Pins of the CPU oracle to things other than itself.

Closed forms, dense trace formulas, networkx, and agreement between routes
that share no code (the subset definition, embeddings / |Aut|, marker-array
triangles and cliques under two orientations, codegree 4-cycles, and the
decomposition terms).  Each named family below has a textbook count.
"""
import itertools
import math

import networkx as nx
import numpy as np
import pytest

from paper_2112_09761_amd import synth

C = math.comb
NAMES = ["edge", "wedge", "triangle", "path4", "star3", "cycle4",
         "tailed_triangle", "diamond", "clique4", "clique5"]
M4 = ["path4", "star3", "cycle4", "tailed_triangle", "diamond", "clique4"]


def to_nx(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(zip(*[a.tolist() for a in synth.to_edge_list(g)]))
    return G


def dense(g):
    A = np.zeros((g.n, g.n), dtype=np.float64)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[src, g.col] = 1.0
    return A


# --- |Aut(P)| --------------------------------------------------------------

AUT = {"edge": 2, "wedge": 2, "triangle": 6, "path4": 2, "star3": 6,
       "cycle4": 8, "tailed_triangle": 2, "diamond": 4, "clique4": 24,
       "clique5": 120}


@pytest.mark.parametrize("name", NAMES)
def test_aut_textbook_and_networkx(oracle, name):
    k, edges = oracle.PATTERNS[name]
    assert oracle.aut(name) == AUT[name]
    P = nx.Graph(edges)
    gm = nx.algorithms.isomorphism.GraphMatcher(P, P)
    assert sum(1 for _ in gm.isomorphisms_iter()) == AUT[name]


# --- closed forms on complete graphs ---------------------------------------

def kn_counts(n):
    """Edge-induced (non-induced) counts in K_n: copies of P = C(n,k) * k!/|Aut|."""
    return {
        "edge": C(n, 2), "wedge": 3 * C(n, 3), "triangle": C(n, 3),
        "path4": 12 * C(n, 4), "star3": 4 * C(n, 4), "cycle4": 3 * C(n, 4),
        "tailed_triangle": 12 * C(n, 4), "diamond": 6 * C(n, 4),
        "clique4": C(n, 4), "clique5": C(n, 5),
    }


@pytest.mark.parametrize("n", [1, 3, 5, 7])
def test_complete_graph_subset_definition(oracle, n):
    g = synth.complete(n)
    exp = kn_counts(n)
    for name in NAMES:
        assert oracle.count_subsets(g, name, False) == exp[name], name
        ind = exp[name] if name in ("edge", "triangle", "clique4", "clique5") else 0
        assert oracle.count_subsets(g, name, True) == ind, name


@pytest.mark.parametrize("n", [6, 11, 16])
def test_complete_graph_fast_routes(oracle, n):
    g = synth.complete(n)
    exp = kn_counts(n)
    for name in NAMES:
        assert oracle.count_embed(g, name, False) == exp[name], name
        assert oracle.count(g, name, False) == exp[name], name
    assert oracle.motifs4(g) == [0, 0, 0, 0, 0, C(n, 4)]
    assert oracle.motifs3(g) == [0, C(n, 3)]
    for k in range(1, 9):
        assert oracle.cliques(g, k, 0) == C(n, k)
        assert oracle.cliques(g, k, 1) == C(n, k)


# --- bipartite and multipartite -------------------------------------------

@pytest.mark.parametrize("a,b", [(2, 2), (3, 5), (7, 4), (20, 30)])
def test_complete_bipartite(oracle, a, b):
    g = synth.complete_bipartite(a, b)
    assert oracle.triangles(g) == 0
    assert oracle.cycle4(g) == C(a, 2) * C(b, 2)
    assert oracle.count(g, "diamond", False) == 0
    assert oracle.count(g, "tailed_triangle", False) == 0
    assert oracle.motifs4(g) == [0, a * C(b, 3) + b * C(a, 3), C(a, 2) * C(b, 2), 0, 0, 0]
    assert oracle.motifs3(g) == [a * C(b, 2) + b * C(a, 2), 0]
    if a + b <= 12:
        assert oracle.count_subsets(g, "cycle4", True) == C(a, 2) * C(b, 2)


def elem_sym(parts, k):
    return sum(math.prod(c) for c in itertools.combinations(parts, k))


@pytest.mark.parametrize("parts", [[3, 4, 5], [2, 2, 2, 2, 2], [40, 40, 40, 40, 40, 40],
                                   [17, 23, 5, 31, 12, 8, 19]])
def test_multipartite_cliques(oracle, parts):
    g = synth.complete_multipartite(parts)
    for k in range(3, 7):
        exp = elem_sym(parts, k)
        assert oracle.cliques(g, k, 0) == exp
        assert oracle.cliques(g, k, 1) == exp
    assert oracle.triangles(g) == elem_sym(parts, 3)


# --- sparse families --------------------------------------------------------

@pytest.mark.parametrize("n", [4, 5, 9, 30])
def test_paths_and_cycles(oracle, n):
    p = synth.path(n)
    assert oracle.motifs4(p) == [n - 3, 0, 0, 0, 0, 0]
    assert oracle.motifs3(p) == [n - 2, 0]
    c = synth.cycle(n)
    assert oracle.cycle4(c) == (1 if n == 4 else 0)
    assert oracle.cycle4_trace(c) == (1 if n == 4 else 0)
    assert oracle.cycle4_trace(p) == 0
    if n >= 5:
        assert oracle.motifs4(c) == [n, 0, 0, 0, 0, 0]
    assert oracle.motifs3(c) == ([n, 0] if n > 3 else [0, 1])


@pytest.mark.parametrize("leaves", [3, 4, 10, 100])
def test_star(oracle, leaves):
    s = synth.star(leaves)
    assert oracle.motifs4(s) == [0, C(leaves, 3), 0, 0, 0, 0]
    assert oracle.motifs3(s) == [C(leaves, 2), 0]


@pytest.mark.parametrize("r,c", [(2, 2), (3, 7), (25, 40)])
def test_grid_cycles(oracle, r, c):
    g = synth.grid(r, c)
    assert oracle.cycle4(g) == (r - 1) * (c - 1)
    assert oracle.cycle4_trace(g) == (r - 1) * (c - 1)
    assert oracle.triangles(g) == 0
    if r * c <= 30:
        assert oracle.count_embed(g, "cycle4", False) == (r - 1) * (c - 1)


@pytest.mark.parametrize("d", [2, 3, 4, 8])
def test_hypercube_cycles(oracle, d):
    g = synth.hypercube(d)
    assert oracle.cycle4(g) == C(d, 2) * 2 ** (d - 2)
    assert oracle.cycle4_trace(g) == C(d, 2) * 2 ** (d - 2)
    assert oracle.count_embed(g, "cycle4", False) == C(d, 2) * 2 ** (d - 2)


def test_disjoint_union_adds(oracle):
    a, b = synth.complete(9), synth.complete_multipartite([3, 3, 4])
    u = synth.disjoint_union(a, b)
    for name in ["triangle", "clique4", "cycle4", "diamond"]:
        assert oracle.count(u, name, False) == oracle.count(a, name, False) + oracle.count(b, name, False)
    assert oracle.motifs4(u) == [x + y for x, y in zip(oracle.motifs4(a), oracle.motifs4(b))]


# --- dense trace formulas ----------------------------------------------------

def test_triangle_trace_full_er_size(oracle):
    """trace(A^3)/6 on the 2000-vertex Erdos-Renyi workload (exact in fp64)."""
    for seed in (1, 2, 3):
        g = synth.workload_er_triangle(seed)
        A = dense(g)
        A2 = A @ A
        t = int(round(np.einsum("ij,ji->", A2, A))) // 6
        assert oracle.triangles(g, 0) == t
        assert oracle.triangles(g, 1) == t


def test_cycle4_trace(oracle):
    """4-cycles = [tr(A^4) - 2 sum d^2 + sum d] / 8."""
    for g in [synth.erdos_renyi(600, 0.05, 4), synth.rmat(10, 8, seed=5),
              synth.erdos_renyi(1500, 0.02, 6)]:
        A = dense(g)
        A2 = A @ A
        tr4 = float(np.einsum("ij,ji->", A2, A2))
        d = g.degrees().astype(np.float64)
        c4 = (tr4 - 2 * float((d * d).sum()) + float(d.sum())) / 8
        assert oracle.cycle4(g) == int(round(c4))
        assert oracle.count(g, "cycle4", False) == int(round(c4))
        assert oracle.cycle4_trace(g) == int(round(c4))


@pytest.mark.parametrize("n", [4, 5, 12, 40])
def test_cycle4_trace_route_closed_forms(oracle, n):
    """The closed-walk route (no ranking) on K_n, K_{m,n} and stars."""
    assert oracle.cycle4_trace(synth.complete(n)) == 3 * C(n, 4)
    assert oracle.cycle4_trace(synth.complete_bipartite(n, n + 3)) == C(n, 2) * C(n + 3, 2)
    assert oracle.cycle4_trace(synth.star(n)) == 0


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_cycle4_routes_agree_power_law(oracle, seed):
    """Codegree counting at the maximum-rank vertex and the closed-walk count
    share neither code nor any ranking; hub-skewed graphs stress both."""
    for g in [synth.rmat(13, 16, seed=seed),
              synth.chung_lu(20000, 12.0, 2.1, 2000.0, 120000, seed)]:
        assert oracle.cycle4(g) == oracle.cycle4_trace(g)


# --- networkx ----------------------------------------------------------------

@pytest.mark.parametrize("seed", [11, 12])
def test_networkx_cliques(oracle, seed):
    g = synth.erdos_renyi(400, 0.08, seed)
    G = to_nx(g)
    by_k = {}
    for cl in nx.enumerate_all_cliques(G):
        by_k[len(cl)] = by_k.get(len(cl), 0) + 1
    for k in range(3, 7):
        assert oracle.cliques(g, k, 0) == by_k.get(k, 0)
        assert oracle.cliques(g, k, 1) == by_k.get(k, 0)
    assert oracle.triangles(g) == sum(nx.triangles(G).values()) // 3


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_networkx_subgraph_matching(oracle, seed):
    """Induced: induced subgraph isomorphisms / |Aut|; edge-induced:
    monomorphisms / |Aut| (networkx GraphMatcher)."""
    g = synth.erdos_renyi(11, 0.45, seed)
    G = to_nx(g)
    for name in NAMES[1:]:
        k, edges = oracle.PATTERNS[name]
        P = nx.Graph(edges)
        gm = nx.algorithms.isomorphism.GraphMatcher(G, P)
        ind = sum(1 for _ in gm.subgraph_isomorphisms_iter()) // AUT[name]
        gm = nx.algorithms.isomorphism.GraphMatcher(G, P)
        mono = sum(1 for _ in gm.subgraph_monomorphisms_iter()) // AUT[name]
        assert oracle.count_subsets(g, name, True) == ind, name
        assert oracle.count_subsets(g, name, False) == mono, name
        assert oracle.count_embed(g, name, True) == ind, name
        assert oracle.count_embed(g, name, False) == mono, name


# --- route agreement on random graphs -----------------------------------------

@pytest.mark.parametrize("seed,n,p", [(31, 9, 0.3), (32, 9, 0.5), (33, 9, 0.7),
                                      (34, 13, 0.4), (35, 16, 0.3), (36, 14, 0.6)])
def test_subsets_vs_fast_routes(oracle, seed, n, p):
    g = synth.erdos_renyi(n, p, seed)
    sub_i = [oracle.count_subsets(g, x, True) for x in M4]
    sub_e = [oracle.count_subsets(g, x, False) for x in M4]
    for order in (0, 1):
        assert oracle.motifs4(g, order) == sub_i
        assert oracle.nonind4(g, order) == sub_e
        assert oracle.motifs3(g, order) == [oracle.count_subsets(g, x, True) for x in ("wedge", "triangle")]
    for name in NAMES:
        for ind in (False, True):
            assert oracle.count_embed(g, name, ind) == oracle.count_subsets(g, name, ind)


@pytest.mark.parametrize("mk", [lambda: synth.erdos_renyi(300, 0.06, 41),
                                lambda: synth.rmat(9, 8, seed=42),
                                lambda: synth.chung_lu(800, 8.0, 2.1, 120.0, 3200, 43)])
def test_embed_vs_fast_routes_moderate(oracle, mk):
    g = mk()
    for name in ["triangle", "clique4", "clique5", "cycle4", "diamond", "tailed_triangle",
                 "wedge", "path4", "star3"]:
        for ind in (False, True):
            assert oracle.count(g, name, ind) == oracle.count_embed(g, name, ind), (name, ind)


def test_relabel_invariance(oracle):
    g = synth.rmat(10, 8, seed=51)
    perm = np.random.default_rng(52).permutation(g.n)
    h = synth.relabel(g, perm)
    assert h.sha256() != g.sha256()
    assert oracle.motifs4(g) == oracle.motifs4(h)
    assert oracle.nonind4(g) == oracle.nonind4(h)
    for k in (3, 4, 5):
        assert oracle.cliques(g, k, 0) == oracle.cliques(h, k, 1)


def test_local_triangle_counts(oracle):
    g = synth.erdos_renyi(200, 0.1, 61)
    T, tv, te = oracle.triangles(g, 1, local=True)
    G = to_nx(g)
    tri = nx.triangles(G)
    assert [int(x) for x in tv] == [tri[v] for v in range(g.n)]
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for e in range(0, g.nnz, 7):
        u, v = int(src[e]), int(g.col[e])
        assert int(te[e]) == len(set(G[u]) & set(G[v]))
    assert int(tv.sum()) == 3 * T and int(te.sum()) == 6 * T


# --- edge cases ---------------------------------------------------------------

def test_degenerate_inputs(oracle):
    e = synth.empty(5)
    for name in NAMES:
        assert oracle.count(e, name, False) == 0
    assert oracle.count_subsets(e, (1, []), True) == 5
    assert oracle.count_embed(e, (1, []), False) == 5
    g = synth.complete(3)
    assert oracle.count(g, "clique4", False) == 0
    assert oracle.cliques(g, 4) == 0


def test_invalid_patterns(oracle):
    g = synth.complete(4)
    with pytest.raises(oracle.OracleError):
        oracle.count_embed(g, (4, [(0, 1), (2, 3)]), False)       # disconnected
    with pytest.raises(oracle.OracleError):
        oracle.count_embed(g, (3, [(0, 0), (1, 2)]), False)       # loop
    with pytest.raises(oracle.OracleError):
        oracle.count_embed(g, (9, [(i, i + 1) for i in range(8)]), False)  # k > 8


def test_overflow_detected(oracle):
    """C(5e6, 3) 3-stars exceed 2^64: the oracle must refuse, not wrap."""
    s = synth.star(5_000_000)
    with pytest.raises(oracle.OracleError):
        oracle.nonind4(s)


@pytest.mark.parametrize("seed", [31, 32])
def test_nonind4_local_terms(oracle, seed):
    """The local-term entry point returns the same path, star, tailed-triangle
    and diamond counts as the full non-induced vector, and networkx's
    monomorphism counts for the two triangle-based shapes."""
    g = synth.erdos_renyi(40, 0.3, seed)
    full = oracle.nonind4(g, 0)
    assert oracle.nonind4_local(g, 0) == [full[0], full[1], full[3], full[4]]
    assert oracle.nonind4_local(g, 1) == oracle.nonind4_local(g, 0)
    G = to_nx(g)
    for name, idx in (("tailed_triangle", 2), ("diamond", 3)):
        P = nx.Graph(oracle.PATTERNS[name][1])
        mono = sum(1 for _ in nx.algorithms.isomorphism.GraphMatcher(G, P)
                   .subgraph_monomorphisms_iter()) // AUT[name]
        assert oracle.nonind4_local(g, 0)[idx] == mono

