"""The allocation-free count (gpm_count_noalloc) against gpm_count, through
the C ABI: the same counts on two calls in a row (the second on a smaller
graph, so the scratch holds what the larger call left), for every kind of
launch whose buffers now come from the device scratch -- local-graph cliques
in LDS and with rows in HBM frontiers, the plan-driven DFS with stored
levels, 4-cycle wedge counters, per-edge triangle counters -- plus its two
refusals (a graph not prepared for the query; buffers beyond the scratch)."""
import pytest

from paper_2112_09761_amd import synth

pytestmark = pytest.mark.gpu

V, E = 0, 1
BOOK = (5, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (0, 4), (1, 4)])
K6 = (6, [(i, j) for i in range(6) for j in range(i + 1, 6)])
CASES = [("clique4", V, {}), ("clique5", V, {}), ("triangle", E, {}),
         ("clique5", V, {"lgs_block": 0, "lgs_tile": 64}),   # rows in HBM frontiers
         (K6, V, {}),                                          # edge kernel
         ("diamond", E, {"decompose": 0}),                     # DFS, one stored level
         ("diamond", V, {}),                                   # decomposed: triangle scatter
         ("tailed_triangle", V, {}),
         ("cycle4", E, {}),                                    # wedge counters
         ("path4", V, {"decompose": 0}),
         (BOOK, V, {})]


def _ctx():
    import torch
    from paper_2112_09761_amd import gpm
    assert torch.cuda.is_available()
    return gpm.Context(0, torch.cuda.current_stream())


def _with_options(ctx, opts, fn):
    defaults = {"decompose": 1, "lgs_block": 1, "lgs_tile": 128}
    try:
        for k, v in opts.items():
            ctx.set_option(k, v)
        return fn()
    finally:
        for k in opts:
            ctx.set_option(k, defaults[k])


def test_noalloc_equals_count_on_two_calls(oracle):
    big = synth.rmat(13, 16, seed=1701)
    small = synth.rmat(9, 8, seed=1702)
    with _ctx() as ctx:
        ids = [ctx.load(big), ctx.load(small)]
        for pat, mode, opts in CASES:
            def run():
                exp = [ctx.count(gid, pat, mode) for gid in ids]      # prepares the graphs
                got = [ctx.count_noalloc(gid, pat, mode) for gid in ids]  # two calls in a row
                return exp, got
            exp, got = _with_options(ctx, opts, run)
            assert got == exp, (pat, mode, opts, got, exp)
        # the counts themselves, against the oracle
        for pat, mode in (("clique4", V), ("cycle4", E), ("diamond", E)):
            assert ctx.count_noalloc(ids[1], pat, mode) == oracle.count(small, pat, mode == V)


def test_noalloc_refusals():
    from paper_2112_09761_amd import gpm
    with _ctx() as ctx:
        g = synth.rmat(10, 8, seed=1703)
        gid = ctx.load(g)
        # nothing prepared yet: the call refuses instead of building
        with pytest.raises(gpm.GpmError) as e:
            ctx.count_noalloc(gid, "clique4")
        assert e.value.status == -6
        exp = ctx.count(gid, "clique4")
        assert ctx.count_noalloc(gid, "clique4") == exp
        # a frontier of one stored level of 5M vertex ids per wave (20 MB)
        # cannot give one workgroup's four waves room in the 64 MiB scratch
        s = synth.star(5_000_000)
        sid = ctx.load(s)
        ctx.set_option("decompose", 0)
        try:
            assert ctx.count(sid, "diamond", E) == 0
            with pytest.raises(gpm.GpmError) as e:
                ctx.count_noalloc(sid, "diamond", E)
            assert e.value.status == -4
        finally:
            ctx.set_option("decompose", 1)
        # the context still counts afterwards, both ways
        assert ctx.count_noalloc(gid, "clique4") == exp
        assert ctx.count(gid, "clique4") == exp
