"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host-only logic (patterns, search plans, frontier sizing)
behaves as the paper states.  No device call is made here."""
import ctypes
import os
import re

import pytest

from paper_2112_09761_amd import gpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gpm.h")).read()
    return sorted(set(re.findall(r"\b(gpm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gpm.lib()
    names = declared_symbols()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(gpm.EXPORTS)


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(gpm.Pattern) == 4 * (2 + 56)
    assert ctypes.sizeof(gpm.Query) == 16 + ctypes.sizeof(gpm.Pattern)


def test_struct_layouts_match_c_compiler(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's struct."""
    import subprocess
    structs = {"gpm_stats": gpm.Stats, "gpm_graph_meta": gpm.GraphMeta,
               "gpm_plan_info": gpm.PlanInfo, "gpm_pattern": gpm.Pattern,
               "gpm_query": gpm.Query, "gpm_serve_info": gpm.ServeInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gpm.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('return 0; }')
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, v = line.split()
        got[(name, field)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_named_patterns():
    for name, (k, ne) in {"edge": (2, 1), "wedge": (3, 2), "triangle": (3, 3),
                          "path4": (4, 3), "star3": (4, 3), "cycle4": (4, 4),
                          "tailed_triangle": (4, 4), "diamond": (4, 5),
                          "clique4": (4, 6), "clique5": (5, 10)}.items():
        p = gpm.pattern_named(name)
        assert (p.k, p.n_edges) == (k, ne)
    with pytest.raises(gpm.GpmError):
        gpm.pattern_named("nonsense")


def test_invalid_patterns_rejected():
    for k, edges in [(4, [(0, 1), (2, 3)]), (3, [(0, 0)]), (3, [(0, 3)]),
                     (9, [(i, i + 1) for i in range(8)]), (3, [(0, 1), (1, 0), (1, 2)])]:
        with pytest.raises(gpm.GpmError) as e:
            gpm.pattern_from_edges(k, edges)
        assert e.value.status == -3


def test_diamond_symmetry_order_worked_example():
    """Sec. 2.2 / Fig. 4: the diamond's symmetry order is {v1 > v2, v3 > v4}
    (1-based) under matching order u1, u2, u3, u4 (both degree-3 vertices
    first)."""
    import json
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "diamond_symmetry_order.json")))
    p = gpm.pattern_from_edges(4, fx["pattern_edges"])
    for mode in (0, 1):
        pl = gpm.plan(p, mode)
        assert pl["order"] == fx["matching_order"]
        assert sorted(map(tuple, pl["restrictions"])) == sorted(map(tuple, fx["restrictions"]))
        assert pl["root_bound"]  # v0 > v1 halves the root edge list (Sec. 7.2 (2))


@pytest.mark.parametrize("name", ["wedge", "path4", "star3", "cycle4", "tailed_triangle",
                                  "diamond", "clique4", "clique5"])
def test_plan_properties(name, oracle):
    """Buffers X <= k - 3; every restriction orders an earlier depth above a
    later one; |Aut| matches the oracle's brute force."""
    for mode in (0, 1):
        pl = gpm.plan(name, mode)
        k = pl["k"]
        assert pl["n_buffers"] <= max(k - 3, 0)
        depth = {v: d for d, v in enumerate(pl["order"])}
        for a, b in pl["restrictions"]:
            assert depth[a] < depth[b]
        assert pl["aut"] == oracle.aut(name)
        # matching order is connected
        p = gpm.pattern_named(name)
        adj = set(p.edge_list()) | {(b, a) for a, b in p.edge_list()}
        for d in range(1, k):
            assert any((pl["order"][d], pl["order"][e]) in adj for e in range(d))


def test_counting_only_suffix():
    """Counting-only pruning (Sec. 5.4 (1)) in the count plan: the last r >= 2
    vertices of the matching order are pairwise non-adjacent twins beside a
    connected rest of >= 2 vertices, edge-induced mode only; the 4-cycle, the
    paper's example of a pattern without the opportunity, has none."""
    book3 = (5, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (0, 4), (1, 4)])
    k23 = (5, [(0, 2), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4)])
    k24 = (6, [(0, 2), (0, 3), (0, 4), (0, 5), (1, 2), (1, 3), (1, 4), (1, 5)])
    star4 = (5, [(0, 1), (0, 2), (0, 3), (0, 4)])
    pendants = (5, [(0, 1), (1, 2), (0, 2), (0, 3), (0, 4)])
    expect = {"diamond": 2, "star3": 2, "cycle4": 0, "path4": 0, "tailed_triangle": 0,
              "wedge": 0, "triangle": 0, "clique4": 0}
    for name, r in expect.items():
        assert gpm.plan(name, 1)["count_only_r"] == r, name
        assert gpm.plan(name, 0)["count_only_r"] == 0, name
    for pat, r in ((book3, 3), (k23, 2), (k24, 3), (star4, 3), (pendants, 2)):
        pl = gpm.plan(pat, 1)
        assert pl["count_only_r"] == r, pat
        assert gpm.plan(pat, 0)["count_only_r"] == 0
        # the twins close the order, each adjacent to an earlier vertex
        k, edges = pat
        adj = {(a, b) for a, b in edges} | {(b, a) for a, b in edges}
        tail = pl["order"][k - r:]
        for x in tail:
            for y in tail:
                assert (x, y) not in adj
            assert {z for z in range(k) if (x, z) in adj} == \
                {z for z in range(k) if (tail[0], z) in adj}


def test_stabiliser_chain_count_identity(oracle):
    """The restrictions admit exactly one of the |Aut| automorphic images of
    every embedding: counting the embeddings of P into P itself that satisfy
    them gives 1 (T9-style check on the pattern as its own data graph)."""
    import itertools
    for name in ["wedge", "path4", "star3", "cycle4", "tailed_triangle", "diamond"]:
        p = gpm.pattern_named(name)
        pl = gpm.plan(p, 1)
        k = p.k
        E = set(p.edge_list()) | {(b, a) for a, b in p.edge_list()}
        ok = 0
        for perm in itertools.permutations(range(k)):
            if all((perm[a], perm[b]) in E for a, b in p.edge_list()):
                if all(perm[a] > perm[b] for a, b in pl["restrictions"]):
                    ok += 1
        assert ok == 1, name


def test_frontier_sizing():
    """Adaptive buffering, Sec. 7.2 (3): waves = min(Y / (X * Delta), |Omega|)."""
    assert gpm.frontier_waves(10**9, 2, 1000, 10**9, 10**6) == 10**9 // (2 * 1000 * 4)
    assert gpm.frontier_waves(10**9, 2, 1000, 50, 10**6) == 50
    assert gpm.frontier_waves(10**9, 1, 10, 10**9, 4096) == 4096
    assert gpm.frontier_waves(10**9, 0, 1000, 10**9, 4096) == 4096
    with pytest.raises(gpm.GpmError):
        gpm.frontier_waves(100, 1, 1000, 10, 10)


def test_validate_csr_error_paths():
    """gpm_load_csr's input checks (host only): canonical CSR accepted, every
    kind of malformed input rejected with GPM_E_CSR or GPM_E_INVAL."""
    import numpy as np
    from paper_2112_09761_amd import synth
    OK, INVAL, CSR = 0, -1, -2
    g = synth.erdos_renyi(50, 0.2, 3)
    assert gpm.validate_csr(g.row_ptr, g.col) == OK
    assert gpm.validate_csr(g.row_ptr, g.col, gpm.GPM_CSR_SYMMETRIC | gpm.GPM_VALIDATE) == OK
    e = synth.empty(7)
    assert gpm.validate_csr(e.row_ptr, e.col) == OK

    def bad(rp, col, flags=gpm.GPM_CSR_SYMMETRIC, exp=CSR):
        assert gpm.validate_csr(np.array(rp), np.array(col), flags) == exp

    bad([0, 2, 3, 4], [2, 1, 0, 0])                 # unsorted list
    bad([0, 2, 3, 4], [1, 1, 0, 0])                 # duplicate neighbour
    bad([0, 1, 2], [0, 1])                          # self loops
    bad([0, 1, 2], [1, 5])                          # id out of range
    bad([0, 1, 1], [1, 0])                          # row_ptr[n] != nnz
    bad([1, 1, 2], [1, 0])                          # row_ptr[0] != 0
    bad([0, 2, 1, 2], [1, 2])                       # not monotone
    bad([0, 1, 1], [1])                             # odd entries, symmetric
    bad([0, 1, 1, 1], [1], gpm.GPM_CSR_SYMMETRIC | gpm.GPM_VALIDATE)        # asymmetric
    dag = gpm.GPM_CSR_DAG
    assert gpm.validate_csr(np.array([0, 1, 2, 2]), np.array([1, 2]), dag | gpm.GPM_VALIDATE) == OK
    bad([0, 1, 2], [1, 0], dag | gpm.GPM_VALIDATE)                          # both directions
    bad([0, 1, 2, 3], [1, 2, 0], dag | gpm.GPM_VALIDATE)                    # 3-cycle
    bad([0, 1, 2], [1, 0], dag | gpm.GPM_CSR_SYMMETRIC, INVAL)              # conflicting flags
    bad([0, 1, 2], [1, 0], gpm.GPM_CSR_SYMMETRIC | gpm.GPM_PTRS_DEVICE, INVAL)
