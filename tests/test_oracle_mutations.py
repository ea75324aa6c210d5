"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle/oracle.c, plants one plausible mistake (a dropped
term, a wrong constant or sign, a wrong bound, a lost check), compiles the
copy and runs a battery of the pins against it (closed forms, networkx,
dense traces, route agreement).  The unmodified oracle must pass the
battery; every mutant must fail it.  Everything runs on the CPU.
"""
import itertools
import math
import os
import subprocess

import networkx as nx
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2112_09761_amd import synth

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "oracle.c")
C = math.comb

MUTATIONS = {
    "cycle4_pairs_off": ("local += (u128)c * (c - 1) / 2;", "local += (u128)c * c / 2;"),
    "cycle4_middle_unranked": ("if (!precedes(rp, 1, u, v)) continue;\n                for",
                               "if (0) continue;\n                for"),
    "orient_ties_both_ways": ("return du < dv || (du == dv && u < v);",
                              "return du <= dv;"),
    "path4_triangle_term": ("np4 -= (u128)3 * T;", "np4 -= (u128)2 * T;"),
    "tailed_degree_term": ("if (d >= 2) *ntt += (u128)tv[u] * (d - 2);",
                           "if (d >= 2) *ntt += (u128)tv[u] * (d - 1);"),
    "diamond_pairs": ("if (t >= 2) *nd += t * (t - 1) / 2;", "if (t >= 2) *nd += t * t / 2;"),
    "star_binomial": ("if (d >= 3) *ns3 += d * (d - 1) * (d - 2) / 6;",
                      "if (d >= 3) *ns3 += d * (d - 1) * (d - 2) / 2;"),
    "motif_k4_in_diamond": ("__int128 d = (__int128)N[4] - 6 * k4;",
                            "__int128 d = (__int128)N[4] - 5 * k4;"),
    "motif_cycle_in_diamond": ("__int128 c4 = (__int128)N[2] - d - 3 * k4;",
                               "__int128 c4 = (__int128)N[2] - 3 * k4;"),
    "motif_path_in_tailed": ("__int128 p4 = (__int128)N[0] - 4 * c4 - 2 * tt - 6 * d - 12 * k4;",
                             "__int128 p4 = (__int128)N[0] - 4 * c4 - 1 * tt - 6 * d - 12 * k4;"),
    "wedge_triangle_term": ("w -= (u128)3 * T;", "w -= (u128)2 * T;"),
    "clique_mark_reset": ("for (int64_t j = 0; j < nl; j++) c->mark[nxt[j]] = chosen;",
                          "for (int64_t j = 0; j < nl; j++) c->mark[nxt[j]] = 0;"),
    "clique_leaf_off_by_one": ("if (chosen == c->k - 1) return (u128)len;",
                               "if (chosen == c->k - 1) return (u128)len + (len > 0);"),
    "embed_not_injective": ("if (img[d] == x) { ok = 0; break; }", "if (0) { ok = 0; break; }"),
    "embed_induced_ignored": ("else if (pl->induced) { if (has_edge(pl->rp, pl->col, x, img[d])) ok = 0; }",
                              "else if (0) { if (has_edge(pl->rp, pl->col, x, img[d])) ok = 0; }"),
    "subsets_enumeration": ("while (i >= 0 && w[i] == n - k + i) i--;",
                            "while (i >= 0 && w[i] >= n - k + i - 1) i--;"),
    "aut_transposed": ("if (adj[i][j] != adj[p[i]][p[j]]) { ok = 0; break; }",
                       "if (adj[i][j] != adj[p[i]][j]) { ok = 0; break; }"),
    "triangle_marker_first": ("for (int64_t p = orp[a]; p < orp[a + 1]; p++) marker[ocol[p]] = p + 1;",
                              "for (int64_t p = orp[a] + 1; p < orp[a + 1]; p++) marker[ocol[p]] = p + 1;"),
    "list_not_injective": ("if (x == img[d]) good = 0;", "if (0) good = 0;"),
    "list_induced_ignored": ("else if (pl->induced) good = !has_edge(pl->rp, pl->col, x, img[d]);",
                             "else if (0) good = !has_edge(pl->rp, pl->col, x, img[d]);"),
    "list_every_embedding": ("if (!smallest_image(c, t)) return;", "if (0) return;"),
    "list_image_compare": ("if (t[s[i]] > t[i]) break;", "if (t[s[i]] > t[i]) continue;"),
    "list_row_columns": ("for (int d = 0; d < k; d++) t[pl->order[d]] = img[d];",
                         "for (int d = 0; d < k; d++) t[d] = img[d];"),
    "trace_retrace_walks": ("u128 c4 = (tr4 + sd - 2 * sd2) / 8;", "u128 c4 = (tr4 + sd - sd2) / 8;"),
    "trace_square": ("local += c * c;", "local += c * (c - 1);"),
    "trace_diagonal_dropped": ("int64_t w = col[f];\n                    if (cnt[w]++ == 0)",
                               "int64_t w = col[f];\n                    if (w == v) continue;\n                    if (cnt[w]++ == 0)"),
    "has_edge_search": ("if (col[mid] < v) lo = mid + 1; else hi = mid;\n    }\n    return lo < rp[u + 1]",
                        "if (col[mid] <= v) lo = mid + 1; else hi = mid;\n    }\n    return lo < rp[u + 1]"),
}

NAMES = ["wedge", "triangle", "path4", "star3", "cycle4", "tailed_triangle", "diamond",
         "clique4", "clique5"]
AUT = {"wedge": 2, "triangle": 6, "path4": 2, "star3": 6, "cycle4": 8, "tailed_triangle": 2,
       "diamond": 4, "clique4": 24, "clique5": 120}


def battery():
    """A quick subset of the oracle pins.  Returns the list of failures."""
    fails = []

    def check(name, a, b):
        if a != b:
            fails.append(name)

    try:
        for name in NAMES:
            check("aut " + name, O.aut(name), AUT[name])
        n = 7
        kn = {"wedge": 3 * C(n, 3), "triangle": C(n, 3), "path4": 12 * C(n, 4),
              "star3": 4 * C(n, 4), "cycle4": 3 * C(n, 4), "tailed_triangle": 12 * C(n, 4),
              "diamond": 6 * C(n, 4), "clique4": C(n, 4), "clique5": C(n, 5)}
        g = synth.complete(n)
        for name in NAMES:
            check("Kn subsets " + name, O.count_subsets(g, name, False), kn[name])
            check("Kn embed " + name, O.count_embed(g, name, False), kn[name])
            check("Kn fast " + name, O.count(g, name, False), kn[name])
        check("Kn motifs4", O.motifs4(g), [0, 0, 0, 0, 0, C(n, 4)])
        for a, b in [(3, 5), (6, 4)]:
            g = synth.complete_bipartite(a, b)
            check("Kmn motifs4", O.motifs4(g),
                  [0, a * C(b, 3) + b * C(a, 3), C(a, 2) * C(b, 2), 0, 0, 0])
            check("Kmn c4", O.cycle4(g), C(a, 2) * C(b, 2))
            check("Kmn c4 trace", O.cycle4_trace(g), C(a, 2) * C(b, 2))
        parts = [3, 4, 5, 2, 6]
        g = synth.complete_multipartite(parts)
        for k in (3, 4, 5):
            exp = sum(math.prod(c) for c in itertools.combinations(parts, k))
            check("multipartite id", O.cliques(g, k, 0), exp)
            check("multipartite deg", O.cliques(g, k, 1), exp)
        check("grid", O.cycle4(synth.grid(5, 7)), 24)
        check("grid trace", O.cycle4_trace(synth.grid(5, 7)), 24)
        check("Kn c4 trace", O.cycle4_trace(synth.complete(8)), 3 * C(8, 4))
        check("path motifs", O.motifs4(synth.path(9)), [6, 0, 0, 0, 0, 0])
        check("star motifs", O.motifs4(synth.star(10)), [0, C(10, 3), 0, 0, 0, 0])
        check("cycle motifs", O.motifs4(synth.cycle(9)), [9, 0, 0, 0, 0, 0])
        for seed in (1, 2):
            g = synth.erdos_renyi(11, 0.45, 900 + seed)
            G = nx.Graph()
            G.add_nodes_from(range(g.n))
            G.add_edges_from(zip(*[x.tolist() for x in synth.to_edge_list(g)]))
            for name in NAMES:
                P = nx.Graph(O.PATTERNS[name][1])
                ind = sum(1 for _ in nx.algorithms.isomorphism.GraphMatcher(G, P)
                          .subgraph_isomorphisms_iter()) // AUT[name]
                mono = sum(1 for _ in nx.algorithms.isomorphism.GraphMatcher(G, P)
                           .subgraph_monomorphisms_iter()) // AUT[name]
                check("nx subsets ind " + name, O.count_subsets(g, name, True), ind)
                check("nx subsets mono " + name, O.count_subsets(g, name, False), mono)
                check("nx embed ind " + name, O.count_embed(g, name, True), ind)
                check("nx embed mono " + name, O.count_embed(g, name, False), mono)
                check("nx fast ind " + name, O.count(g, name, True), ind)
                check("nx fast mono " + name, O.count(g, name, False), mono)
                for induced, exp in ((True, ind), (False, mono)):
                    rows, cnt = O.list_embed(g, name, induced, cap=exp + 8)
                    check("list count " + name, cnt, exp)
                    edges = O.PATTERNS[name][1]
                    ok = all(len(set(r.tolist())) == len(r) and
                             all(G.has_edge(int(r[a]), int(r[b])) for a, b in edges) and
                             (not induced or
                              G.subgraph([int(x) for x in r]).number_of_edges() == len(edges))
                             for r in rows)
                    check("list rows valid " + name, ok, True)
                    sets = {frozenset(frozenset((int(r[a]), int(r[b]))) for a, b in edges)
                            for r in rows}
                    check("list rows distinct " + name, len(sets), len(rows))
        g = synth.erdos_renyi(300, 0.05, 950)
        A = np.zeros((g.n, g.n))
        A[np.repeat(np.arange(g.n), np.diff(g.row_ptr)), g.col] = 1
        A2 = A @ A
        check("trace3", O.triangles(g, 0), int(round(np.einsum("ij,ji->", A2, A))) // 6)
        d = g.degrees().astype(float)
        c4 = (float(np.einsum("ij,ji->", A2, A2)) - 2 * (d * d).sum() + d.sum()) / 8
        check("trace4", O.cycle4(g), int(round(c4)))
        check("trace4 sparse", O.cycle4_trace(g), int(round(c4)))
    except Exception as e:  # a mutant may also crash an assertion path
        fails.append(f"exception {e!r}")
    return fails


def build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation {name} does not apply exactly once"
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", str(c), "-o",
                    str(so)], check=True, capture_output=True)
    return str(so)


def with_library(path, fn):
    saved = O._lib
    O._lib = O.load(path)
    try:
        return fn()
    finally:
        O._lib = saved


def test_unmodified_oracle_passes_battery():
    assert battery() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    so = build_variant(tmp_path, name, old, new)
    fails = with_library(so, battery)
    assert fails, f"planted mistake {name} passed every pin"
