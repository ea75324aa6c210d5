"""Full-size workloads on the GPU against stored oracle counts.

The stored counts in tests/golden/*_oracle.json were written by
tests/golden/gen_golden.py, which calls only the CPU oracle on the same
seeded generator; the sha256 of the regenerated CSR must match the record.
"""
import json
import os

import pytest

from paper_2112_09761_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    p = os.path.join(HERE, "golden", f"{name}_oracle.json")
    if not os.path.exists(p):
        pytest.skip(f"stored oracle counts for {name} not generated")
    with open(p) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2112_09761_amd import gpm
    c = gpm.Context(0, torch.cuda.current_stream())
    yield c
    c.close()


def clique(k):
    return (k, [(i, j) for i in range(k) for j in range(i + 1, k)])


def test_rmat_s20_cliques(ctx):
    gold = golden("rmat_s20")
    g = synth.workload_rmat_s20()
    assert g.sha256() == gold["sha256"]
    gid = ctx.load(g)
    try:
        info = ctx.graph_info(gid)
        assert info["m"] == gold["m"] and info["max_degree"] == gold["max_degree"]
        for k, key in ((3, "triangle"), (4, "clique4"), (5, "clique5")):
            print("rmat_s20 clique", k, flush=True)
            assert ctx.count(gid, clique(k)) == gold["counts"][key], k
        # the sorted-list edge kernel must agree on the 4-clique count
        ctx.set_option("clique_algo", 1)
        assert ctx.count(gid, clique(4)) == gold["counts"]["clique4"]
    finally:
        ctx.set_option("clique_algo", 0)
        ctx.unload(gid)


def test_chung_lu_4m(ctx):
    gold = golden("chung_lu_4m")
    g = synth.workload_chung_lu_4m()
    assert g.sha256() == gold["sha256"]
    gid = ctx.load(g)
    try:
        m3 = gold["counts"]["motifs3"]
        n4 = gold["counts"]["nonind4"]  # path4, star3, cycle4, tailed_triangle, diamond, clique4
        print("chung_lu motifs3", flush=True)
        assert ctx.motifs(gid, 3) == m3
        for name, idx in (("diamond", 4), ("tailed_triangle", 3), ("cycle4", 2)):
            print("chung_lu", name, flush=True)
            assert ctx.count(gid, name, 1) == n4[idx], name
    finally:
        ctx.unload(gid)
