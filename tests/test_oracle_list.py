"""Pins of the oracle's listing routine (Sec. 2.1: listing enumerates every
distinct match).  A listing is right when its rows are valid embeddings, no
two rows are the same subgraph, and the rows cover every subgraph; each is
checked here against something other than the oracle's own enumeration:
networkx's subgraph matcher, closed forms, and the definition of a
representative (the smallest automorphic image).  CPU only."""
import itertools
import math

import networkx as nx
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2112_09761_amd import synth


def automorphisms(k, edges):
    es = {frozenset(e) for e in edges}
    return [p for p in itertools.permutations(range(k))
            if {frozenset((p[a], p[b])) for a, b in edges} == es]


def edge_set(row, edges):
    return frozenset(frozenset((int(row[a]), int(row[b]))) for a, b in edges)


def nx_subgraphs(g, k, edges, induced):
    """Distinct matches as edge sets, from networkx's matcher."""
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(zip(*[x.tolist() for x in synth.to_edge_list(g)]))
    P = nx.Graph()
    P.add_nodes_from(range(k))
    P.add_edges_from(edges)
    gm = nx.algorithms.isomorphism.GraphMatcher(G, P)
    it = gm.subgraph_isomorphisms_iter() if induced else gm.subgraph_monomorphisms_iter()
    out = set()
    for m in it:
        inv = {pv: gv for gv, pv in m.items()}
        out.add(frozenset(frozenset((inv[a], inv[b])) for a, b in edges))
    return out


def valid_row(g, row, k, edges, induced):
    adj = set(zip(*[x.tolist() for x in synth.to_edge_list(g)]))
    has = lambda u, v: (u, v) in adj or (v, u) in adj
    if len(set(int(x) for x in row)) != k:
        return False
    es = {frozenset(e) for e in edges}
    for a in range(k):
        for b in range(a + 1, k):
            e = has(int(row[a]), int(row[b]))
            if frozenset((a, b)) in es and not e:
                return False
            if induced and frozenset((a, b)) not in es and e:
                return False
    return True


PATTERNS = dict(O.PATTERNS)
PATTERNS["house"] = (5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4)])
PATTERNS["bull"] = (5, [(0, 1), (1, 2), (0, 2), (0, 3), (1, 4)])


@pytest.mark.parametrize("name", sorted(PATTERNS))
@pytest.mark.parametrize("induced", [True, False])
def test_list_equals_networkx_subgraphs(name, induced):
    k, edges = PATTERNS[name]
    for seed in (3, 4):
        g = synth.erdos_renyi(12, 0.45, 700 + seed)
        rows, cnt = O.list_embed(g, PATTERNS[name], induced)
        assert cnt == len(rows)
        got = [edge_set(r, edges) for r in rows]
        assert len(set(got)) == len(got), "two rows are the same subgraph"
        assert set(got) == nx_subgraphs(g, k, edges, induced)
        assert all(valid_row(g, r, k, edges, induced) for r in rows)


@pytest.mark.parametrize("name", ["triangle", "cycle4", "diamond", "tailed_triangle", "house"])
def test_list_rows_are_smallest_images(name):
    k, edges = PATTERNS[name]
    auts = automorphisms(k, edges)
    g = synth.erdos_renyi(14, 0.5, 77)
    rows, _ = O.list_embed(g, PATTERNS[name], False)
    for r in rows:
        t = tuple(int(x) for x in r)
        assert t == min(tuple(t[s[i]] for i in range(k)) for s in auts)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_list_cliques_of_kn(k):
    n = 8
    rows, cnt = O.list_embed(synth.complete(n), O.clique(k), True)
    assert cnt == math.comb(n, k)
    assert sorted(tuple(sorted(r.tolist())) for r in rows) == \
        list(itertools.combinations(range(n), k))


def test_list_of_bipartite_cycles():
    a, b = 4, 5
    rows, cnt = O.list_embed(synth.complete_bipartite(a, b), "cycle4", False)
    assert cnt == math.comb(a, 2) * math.comb(b, 2)
    # every 4-cycle of K_{a,b} alternates sides
    side = lambda v: v < a
    for r in rows:
        assert [side(int(x)) for x in r] in ([True, False, True, False],
                                             [False, True, False, True])


def test_list_overflow_counts_all_and_writes_cap_rows():
    g = synth.erdos_renyi(40, 0.3, 9)
    full, cnt = O.list_embed(g, "triangle", True)
    assert cnt == O.triangles(g, 0) and cnt > 10
    part, cnt2 = O.list_embed(g, "triangle", True, cap=10)
    assert cnt2 == cnt and part.shape == (10, 3)
    assert np.array_equal(part, full[:10])  # serial: a fixed enumeration order
    _, cnt0 = O.list_embed(g, "triangle", True, cap=0)
    assert cnt0 == cnt


def test_list_small_cases():
    g = synth.erdos_renyi(20, 0.2, 5)
    rows, cnt = O.list_embed(g, (1, []), True)
    assert cnt == g.n and sorted(rows[:, 0].tolist()) == list(range(g.n))
    rows, cnt = O.list_embed(g, "edge", True)
    assert cnt == g.m
    assert {frozenset(r.tolist()) for r in rows} == \
        {frozenset(e) for e in zip(*[x.tolist() for x in synth.to_edge_list(g)])}
