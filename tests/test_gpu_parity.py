"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every count is an exact integer, so the bar is bit-exact equality.  Inputs
are seeded synthetic graphs: structured families with closed forms, and
random Erdos-Renyi / R-MAT / Chung-Lu graphs at sizes that span many chunks
and ragged tails.
"""
import numpy as np
import pytest

from paper_2112_09761_amd import synth

pytestmark = pytest.mark.gpu

NAMES = ["triangle", "wedge", "path4", "star3", "cycle4", "tailed_triangle",
         "diamond", "clique4", "clique5"]
V, E = 0, 1


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2112_09761_amd import gpm
    assert torch.cuda.is_available()
    c = gpm.Context(0, torch.cuda.current_stream())
    yield c
    c.close()


def graphs_small():
    return [
        synth.complete(9),
        synth.complete_bipartite(5, 7),
        synth.complete_multipartite([3, 4, 5, 2]),
        synth.grid(6, 9),
        synth.hypercube(5),
        synth.star(40),
        synth.path(30),
        synth.cycle(17),
        synth.erdos_renyi(60, 0.2, 101),
        synth.rmat(8, 6, seed=102),
        synth.chung_lu(500, 6.0, 2.1, 80.0, 1500, 103),
        synth.disjoint_union(synth.complete(6), synth.empty(5), synth.cycle(4)),
    ]


@pytest.mark.parametrize("gi", range(12))
def test_named_patterns_small(ctx, oracle, gi):
    g = graphs_small()[gi]
    gid = ctx.load(g)
    try:
        for name in NAMES:
            for mode in (V, E):
                got = ctx.count(gid, name, mode)
                exp = oracle.count(g, name, mode == V)
                assert got == exp, (g.name, name, mode, got, exp)
    finally:
        ctx.unload(gid)


@pytest.mark.parametrize("gi", range(12))
def test_motifs_small(ctx, oracle, gi):
    g = graphs_small()[gi]
    gid = ctx.load(g)
    try:
        assert ctx.motifs(gid, 3) == oracle.motifs3(g), g.name
        assert ctx.motifs(gid, 4) == oracle.motifs4(g), g.name
    finally:
        ctx.unload(gid)


@pytest.mark.parametrize("seed", range(1, 9))
def test_er_triangle_workload(ctx, oracle, seed):
    """Triangle counting on G(2000, 0.01), id-oriented oracle route."""
    g = synth.workload_er_triangle(seed)
    gid = ctx.load(g)
    try:
        assert ctx.count(gid, "triangle") == oracle.triangles(g, 0)
    finally:
        ctx.unload(gid)


@pytest.mark.parametrize("mk", [
    lambda: synth.rmat(12, 16, seed=201),
    lambda: synth.erdos_renyi(3000, 0.01, 202),
    lambda: synth.chung_lu(5000, 12.0, 2.1, 600.0, 30000, 203),
])
def test_medium_graphs_all_patterns(ctx, oracle, mk):
    g = mk()
    gid = ctx.load(g)
    try:
        for name in NAMES:
            for mode in (V, E):
                got = ctx.count(gid, name, mode)
                exp = oracle.count(g, name, mode == V)
                assert got == exp, (g.name, name, mode, got, exp)
        assert ctx.motifs(gid, 4) == oracle.motifs4(g)
    finally:
        ctx.unload(gid)


def random_pattern(rng, k):
    while True:
        edges = [(i, j) for i in range(k) for j in range(i + 1, k) if rng.random() < 0.5]
        # connected?
        adj = {i: set() for i in range(k)}
        for a, b in edges:
            adj[a].add(b)
            adj[b].add(a)
        seen, st = {0}, [0]
        while st:
            x = st.pop()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y)
                    st.append(y)
        if len(seen) == k:
            return (k, edges)


@pytest.mark.parametrize("seed", range(6))
def test_random_patterns(ctx, oracle, seed):
    rng = np.random.default_rng(300 + seed)
    g = synth.erdos_renyi(40, 0.3, 400 + seed)
    gid = ctx.load(g)
    try:
        for k in (3, 4, 5, 6):
            pat = random_pattern(rng, k)
            for mode in (V, E):
                exp = oracle.count_embed(g, pat, mode == V)
                for setop in (1, 2, 3):          # every set-op variant (Sec. 6.1)
                    ctx.set_option("setop", setop)
                    got = ctx.count(gid, pat, mode)
                    assert got == exp, (pat, mode, setop, got, exp)
    finally:
        ctx.set_option("setop", 0)
        ctx.unload(gid)


@pytest.mark.parametrize("seed", range(4))
def test_random_patterns_seven_eight(ctx, oracle, seed):
    """Random connected 7- and 8-vertex patterns (the largest plans: seven
    levels, up to six stored depths)."""
    rng = np.random.default_rng(500 + seed)
    g = synth.erdos_renyi(30, 0.3, 600 + seed)
    gid = ctx.load(g)
    try:
        for k in (7, 8):
            pat = random_pattern(rng, k)
            for mode in (V, E):
                exp = oracle.count_embed(g, pat, mode == V)
                for setop in (1, 2, 3):
                    ctx.set_option("setop", setop)
                    got = ctx.count(gid, pat, mode)
                    assert got == exp, (pat, mode, setop, got, exp)
    finally:
        ctx.set_option("setop", 0)
        ctx.unload(gid)


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7, 8])
def test_cliques_multipartite(ctx, k):
    import itertools
    import math
    parts = [9, 7, 8, 6, 9, 5, 7, 8, 6]
    g = synth.complete_multipartite(parts)
    exp = sum(math.prod(c) for c in itertools.combinations(parts, k))
    gid = ctx.load(g)
    try:
        assert ctx.count(gid, synth_clique(k)) == exp
    finally:
        ctx.unload(gid)


def synth_clique(k):
    return (k, [(i, j) for i in range(k) for j in range(i + 1, k)])


def test_tuning_options_do_not_change_counts(ctx, oracle):
    g = synth.rmat(11, 12, seed=501)
    gid = ctx.load(g)
    exp = {n: oracle.count(g, n, True) for n in ["clique4", "clique5", "cycle4", "diamond",
                                                 "tailed_triangle", "path4"]}
    exp_c4e = oracle.cycle4(g)
    try:
        for opt, vals in [("chunk", [1, 3, 64]), ("waves_per_cu", [1, 4, 32]),
                          ("lds_tile", [32, 64, 4096]), ("clique_lds", [0]),
                          ("granularity", [1]), ("clique_algo", [1, 2]),
                          ("lgs_tile", [64, 256]), ("lgs_max", [64, 100]),
                          ("lgs_split", [0]), ("leaf_cap", [0, 1, 4096]),
                          ("rename", [0]), ("cycle4_algo", [1, 2]), ("decompose", [0]),
                          ("edge_terms", [1]), ("cycle4_mode", [1, 2]), ("setop", [1, 2, 3]),
                          ("cycle4_batch", [16, 1 << 20]), ("lgs_lanes", [32, 8, 4])]:
            for v in vals:
                ctx.set_option(opt, v)
                for n, e in exp.items():
                    assert ctx.count(gid, n, V) == e, (opt, v, n)
                assert ctx.count(gid, "cycle4", E) == exp_c4e, (opt, v)
            ctx.set_option(opt, {"chunk": 0, "waves_per_cu": 0, "lds_tile": 0,
                                 "clique_lds": 1, "granularity": 0, "clique_algo": 0,
                                 "lgs_tile": 128, "lgs_max": 2048, "lgs_split": 1,
                                 "leaf_cap": 128, "rename": 1, "cycle4_algo": 0,
                                 "decompose": 1, "edge_terms": 0, "cycle4_mode": 0, "setop": 0,
                                 "cycle4_batch": 8192, "lgs_lanes": 64}[opt])
    finally:
        ctx.unload(gid)


def test_autotuner_keeps_counts(ctx, oracle):
    g = synth.rmat(12, 12, seed=901)
    gid = ctx.load(g)
    try:
        ctx.set_option("autotune", 1)
        ctx.set_option("tune_min_ms", 0)
        for name, mode in [("clique4", V), ("clique5", V), ("diamond", E), ("path4", V)]:
            exp = oracle.count(g, name, mode == V)
            assert ctx.count(gid, name, mode) == exp, name    # tunes
            assert ctx.count(gid, name, mode) == exp, name    # cached configuration
            assert ctx.stats()["variant"] == 1
    finally:
        ctx.set_option("autotune", 0)
        ctx.set_option("tune_min_ms", 20)
        ctx.unload(gid)


def test_large_roots_take_edge_kernel(ctx, oracle):
    """Roots above the local-graph limit go to the edge-parallel kernel; the
    split must not change any count (K_n has out-degrees up to n - 1)."""
    g = synth.disjoint_union(synth.complete(150), synth.rmat(10, 8, seed=801))
    gid = ctx.load(g)
    try:
        for lim in (64, 100, 1024):
            ctx.set_option("lgs_max", lim)
            for k in (3, 4, 5):
                assert ctx.count(gid, synth_clique(k)) == oracle.cliques(g, k), (lim, k)
        assert ctx.motifs(gid, 4) == oracle.motifs4(g)
    finally:
        ctx.set_option("lgs_max", 2048)
        ctx.unload(gid)


def esym(parts, k):
    """k-cliques of the complete multipartite graph with these part sizes: the
    elementary symmetric polynomial e_k of the sizes."""
    e = [1] + [0] * k
    for p in parts:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * p
    return e[k]


def test_esym_closed_form():
    import itertools
    import math
    parts = [3, 1, 4, 1, 5, 2]
    for k in range(1, 7):
        assert esym(parts, k) == sum(math.prod(c) for c in itertools.combinations(parts, k))
    assert esym([1] * 30, 5) == math.comb(30, 5)


@pytest.mark.parametrize("parts,k5_both", [
    ([1] * 65, True),                 # K_65: out-degrees 0..64
    ([3] * 97 + [1] * 10, True),      # n = 301, ragged rows
    ([1] * 897, False),               # K_897: the largest workgroup root, d = 896
    ([1] * 1025, False),              # K_1025: roots just above the workgroup limit
    ([2] * 550, False),               # n = 1100: roots above the workgroup limit too
])
def test_workgroup_local_graphs(ctx, parts, k5_both):
    """Roots with more out-neighbours than the per-wave tile are searched by a
    whole workgroup (up to 896 out-neighbours with 160 KB of LDS per
    workgroup); larger ones by one wave with rows in HBM.  Dense multipartite
    graphs put roots in all three ranges; every count must equal the closed
    form, with the workgroup path on and off."""
    g = synth.complete_multipartite(parts)
    gid = ctx.load(g)
    try:
        ctx.set_option("lgs_tile", 64)
        for lanes in (64, 16, 4):
            ctx.set_option("lgs_lanes", lanes)
            for k in (3, 4, 5):
                for blk in ((1, 0) if (k < 5 or k5_both) else (1,)):
                    ctx.set_option("lgs_block", blk)
                    assert ctx.count(gid, synth_clique(k)) == esym(parts, k), (k, blk, lanes)
    finally:
        ctx.set_option("lgs_block", 1)
        ctx.set_option("lgs_tile", 128)
        ctx.set_option("lgs_lanes", 64)
        ctx.unload(gid)


def test_workgroup_rmat_options(ctx, oracle):
    """R-MAT graph with 245 roots above a 64-vertex tile: workgroup path with
    and without splitting, instrumented kernels, and a batch that mixes the
    workgroup kernel with the per-wave kernel, all equal to the oracle."""
    from paper_2112_09761_amd import gpm
    g = synth.rmat(13, 16, seed=1301)
    gid = ctx.load(g)
    exp = {k: oracle.cliques(g, k) for k in (3, 4, 5)}
    try:
        ctx.set_option("lgs_tile", 64)
        for opt, v in [("lgs_split", 0), ("lgs_split", 1), ("count_elements", 1),
                       ("lgs_lanes", 16), ("count_elements", 0), ("lgs_lanes", 4),
                       ("lgs_block", 0), ("lgs_block", 1), ("lgs_lanes", 8)]:
            ctx.set_option(opt, v)
            for k in (3, 4, 5):
                assert ctx.count(gid, synth_clique(k)) == exp[k], (opt, v, k)
        qs = [gpm.count_query(gid, synth_clique(5), V), gpm.motif_query(gid, 4),
              gpm.count_query(gid, "clique4", V), gpm.count_query(gid, "diamond", E)]
        res = ctx.count_batch(qs)
        assert res[0] == exp[5] and res[2] == exp[4]
        assert res[1] == oracle.motifs4(g)
        assert res[3] == oracle.count(g, "diamond", False)
    finally:
        ctx.set_option("lgs_tile", 128)
        ctx.set_option("lgs_split", 1)
        ctx.set_option("count_elements", 0)
        ctx.set_option("lgs_block", 1)
        ctx.set_option("lgs_lanes", 64)
        ctx.unload(gid)


def test_per_launch_statistics(ctx):
    """Per-launch statistics: one entry per launch in launch order, the
    workgroup launch first, instrumented totals equal to the per-launch sums,
    and launch durations that add up to the call's kernel time."""
    from paper_2112_09761_amd import gpm
    g = synth.rmat(13, 16, seed=1301)
    gid = ctx.load(g)
    try:
        ctx.set_option("lgs_tile", 64)
        ctx.set_option("count_elements", 1)
        ctx.count(gid, synth_clique(5))
        st = ctx.stats()
        assert st["n_launch_stats"] == st["launches"] == 2
        assert st["launch_kinds"] == [gpm.KIND_LGS_BLOCK, gpm.KIND_LGS_WAVE]
        for f, tot in [("launch_elements", "elements"), ("launch_fetches", "list_fetches"),
                       ("launch_written", "frontier_written"), ("launch_words", "bitmap_words")]:
            assert sum(st[f]) == st[tot], f
        assert all(x > 0 for x in st["launch_words"])
        assert 0 < sum(st["launch_ms"]) <= st["kernel_ms"] * 1.001 + 0.01
        ctx.set_option("count_elements", 0)
        ctx.count(gid, synth_clique(4))
        st = ctx.stats()
        assert st["launch_elements"] == [-1, -1] and st["elements"] == -1
    finally:
        ctx.set_option("count_elements", 0)
        ctx.set_option("lgs_tile", 128)
        ctx.unload(gid)


def test_workgroup_unordered_dag(ctx):
    """A DAG given by the caller whose orientation does not follow vertex ids
    (u -> v iff pi(u) < pi(v) for a random permutation pi): the workgroup
    path takes its unordered branches."""
    from paper_2112_09761_amd import gpm
    parts = [3] * 97 + [1] * 10
    g = synth.complete_multipartite(parts)
    rng = np.random.default_rng(1302)
    pi = rng.permutation(g.n)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = pi[src] < pi[g.col]
    rp = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src[keep], minlength=g.n), out=rp[1:])
    did = ctx.load_csr(rp, g.col[keep], gpm.GPM_CSR_DAG | gpm.GPM_VALIDATE)
    try:
        ctx.set_option("lgs_tile", 64)
        for k in (3, 4, 5):
            assert ctx.count(did, synth_clique(k)) == esym(parts, k), k
    finally:
        ctx.set_option("lgs_tile", 128)
        ctx.unload(did)


def test_cycle4_task_kinds(ctx, oracle):
    """Edge-induced 4-cycles by the workgroup kernel's three kinds of task --
    direct id windows (16- and 32-bit counters), hash tasks over id ranges of
    one root, packed light roots -- and its split of a hash task whose
    distinct endpoints overflow the table: every mode and task size gives the
    closed forms and the oracle, interleaved with other graphs and with motif
    queries that share the launch."""
    import math
    gs = [synth.rmat(12, 8, seed=1401), synth.grid(5, 7), synth.complete(9),
          synth.rmat(14, 16, seed=1402), synth.chung_lu(30000, 8.0, 2.1, 3000.0, 120000, 1403),
          synth.complete_bipartite(2, 70000),    # a root with 70000 lower neighbours
          synth.complete_bipartite(3, 40000),    # 16-bit window counters up to 39999
          synth.hypercube(10)]
    exp_c4 = [oracle.cycle4(g) for g in gs]
    assert exp_c4[5] == math.comb(70000, 2)
    assert exp_c4[6] == 3 * math.comb(40000, 2)
    assert exp_c4[7] == math.comb(10, 2) * 2 ** 8
    exp_m4 = {i: oracle.motifs4(gs[i]) for i in (0, 1, 2, 3, 4)}
    ids = [ctx.load(g) for g in gs]
    try:
        for mode, batch in ((0, 8192), (1, 8192), (2, 8192), (1, 16), (2, 64), (0, 1 << 20),
                            (1, 1 << 20)):
            ctx.set_option("cycle4_mode", mode)
            ctx.set_option("cycle4_batch", batch)
            for rep in range(2):
                order = range(len(gs)) if rep == 0 else reversed(range(len(gs)))
                for i in order:
                    assert ctx.count(ids[i], "cycle4", E) == exp_c4[i], (mode, batch, i)
                    if i in exp_m4 and rep == 0:
                        assert ctx.motifs(ids[i], 4) == exp_m4[i], (mode, batch, i)
    finally:
        ctx.set_option("cycle4_mode", 0)
        ctx.set_option("cycle4_batch", 8192)
        for gid in ids:
            ctx.unload(gid)


def test_edge_cases(ctx):
    from paper_2112_09761_amd import gpm
    e = synth.empty(10)
    gid = ctx.load(e)
    assert ctx.count(gid, "triangle") == 0
    assert ctx.count(gid, (1, [])) == 10
    assert ctx.motifs(gid, 4) == [0] * 6
    ctx.unload(gid)
    k3 = synth.complete(3)
    gid = ctx.load(k3)
    ctx.prepare(gid)
    assert ctx.count(gid, "clique4") == 0
    assert ctx.count(gid, "edge") == 3
    assert ctx.count(gid, "triangle") == 1
    ctx.unload(gid)
    z = synth.empty(0)
    gid = ctx.load(z)
    assert ctx.count(gid, "triangle") == 0
    ctx.unload(gid)
    with pytest.raises(gpm.GpmError):
        ctx.count(12345, "triangle")


def test_batch_equals_single(ctx, oracle):
    from paper_2112_09761_amd import gpm
    gs = [synth.rmat(9, 8, seed=600 + i) if i % 2 else synth.erdos_renyi(700, 0.02, 600 + i)
          for i in range(10)]
    ids = [ctx.load(g) for g in gs]
    try:
        qs = []
        for gid in ids:
            qs.append(gpm.motif_query(gid, 4))
            qs.append(gpm.count_query(gid, "clique5", V))
            qs.append(gpm.count_query(gid, "diamond", E))
        res = ctx.count_batch(qs)
        for i, g in enumerate(gs):
            assert res[3 * i] == oracle.motifs4(g)
            assert res[3 * i + 1] == oracle.cliques(g, 5)
            assert res[3 * i + 2] == oracle.count(g, "diamond", False)
    finally:
        for gid in ids:
            ctx.unload(gid)


def test_serving_alone_vs_mix(ctx, oracle):
    from paper_2112_09761_amd import gpm
    gs = [synth.rmat(9 + i % 3, 8, seed=700 + i) for i in range(6)]
    ids = [ctx.load(g) for g in gs]
    pats = ["triangle", "clique4", "clique5", "cycle4", "diamond", "tailed_triangle"]
    try:
        rng = np.random.default_rng(7)
        qs = [(int(rng.integers(0, len(ids))), pats[int(rng.integers(0, len(pats)))])
              for _ in range(40)]
        alone = [ctx.count(ids[a], p, E) for a, p in qs]
        tickets = [ctx.submit(gpm.count_query(ids[a], p, E)) for a, p in qs]
        mixed = [ctx.wait(t)[0] for t in tickets]
        assert alone == mixed
        for (a, p), x in zip(qs, alone):
            assert x == oracle.count(gs[a], p, False)
        assert ctx.inflight() == 0
    finally:
        for gid in ids:
            ctx.unload(gid)


def test_serving_counter_buffers_grow(ctx, oracle):
    """One serving slot whose zero-initialised counter buffers (4-cycle
    wedges, per-edge triangles) must grow from group to group: a grown buffer
    may come back at the same address with uncleared memory beyond its old
    size, which must be cleared before use."""
    from paper_2112_09761_amd import gpm
    gs = [synth.rmat(8, 8, seed=1501), synth.rmat(11, 12, seed=1502),
          synth.rmat(13, 12, seed=1503)]
    ids = [ctx.load(g) for g in gs]
    kinds = [("cycle4", E), ("diamond", E), ("tailed_triangle", V), ("path4", V)]
    exp = {(i, p, m): oracle.count(g, p, m == V) for i, g in enumerate(gs) for p, m in kinds}
    exp_m4 = [oracle.motifs4(g) for g in gs]
    try:
        ctx.set_option("serve_slots", 1)
        for upto in (1, 2, 3, 2, 3):
            tickets = []
            for i in range(upto):
                for p, m in kinds:
                    tickets.append(((i, p, m), ctx.submit(gpm.count_query(ids[i], p, m))))
                tickets.append((("m4", i), ctx.submit(gpm.motif_query(ids[i], 4))))
            for key, t in tickets:
                got = ctx.wait(t)
                if key[0] == "m4":
                    assert got == exp_m4[key[1]], (upto, key)
                else:
                    assert got[0] == exp[key], (upto, key)
    finally:
        ctx.set_option("serve_slots", 4)
        for gid in ids:
            ctx.unload(gid)


def test_serving_admission_waits_for_memory(oracle):
    """Admission by frontier memory (adaptive buffering, Sec. 7.2 (3)): with a
    budget that one running query fills, a second query that does not fit
    beside it waits, first in line, and completes after it with the oracle's
    count; a query whose buffers exceed the whole budget completes with
    GPM_E_NOMEM through gpm_wait; an unknown ticket is refused at once."""
    import time
    import torch
    from paper_2112_09761_amd import gpm
    g = synth.rmat(16, 16, seed=1601)
    small = synth.rmat(10, 8, seed=1602)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    with gpm.Context(0, torch.cuda.current_stream()) as c0:
        gid = c0.load(g)
        dmax = c0.graph_info(gid)["max_degree"]
    x = gpm.plan("diamond", V)["n_buffers"]   # the DFS plan stores one level
    assert x >= 1
    stride = -(-x * dmax // 64) * 64            # frontier words per wave
    min_bytes = stride * 4 * cus                # one wave per CU
    exp_big = oracle.count(g, "diamond", True)
    exp_small = oracle.count(small, "diamond", True)
    with gpm.Context(0, torch.cuda.current_stream(), budget=min_bytes * 3 // 2) as c:
        c.set_option("decompose", 0)            # the DFS plan: it needs frontier memory
        ids = [c.load(g), c.load(small)]
        t_alone = time.perf_counter()
        assert c.count(ids[0], "diamond", V) == exp_big
        t_alone = time.perf_counter() - t_alone
        st0 = c.serve_state()
        t1 = c.submit(gpm.count_query(ids[0], "diamond", V))
        t2 = c.submit(gpm.count_query(ids[1], "diamond", V))
        st = c.serve_state()
        # the first launch holds more than half the budget, so the second
        # query cannot start beside it
        assert st["running"] == 1 and st["pending"] == 1, (st, t_alone)
        assert st["frontier_in_use"] > st["budget"] - min_bytes, st
        assert st["memory_waits"] == st0["memory_waits"] + 1, st
        done2, _ = c.poll(t2)
        assert not done2 or c.serve_state()["running"] == 0
        assert c.wait(t1)[0] == exp_big
        assert c.wait(t2)[0] == exp_small
        st = c.serve_state()
        assert st["pending"] == 0 and st["running"] == 0 and st["frontier_in_use"] == 0, st
        assert st["admitted"] == st0["admitted"] + 2, st
        with pytest.raises(gpm.GpmError) as e:
            c.wait(987654321)
        assert e.value.status == -1
        with pytest.raises(gpm.GpmError) as e:
            c.wait(t1)                          # already collected
        assert e.value.status == -1
        # a budget below one wave per CU: the query completes with NOMEM
        c.set_option("budget", min_bytes // 4)
        t3 = c.submit(gpm.count_query(ids[0], "diamond", V))
        with pytest.raises(gpm.GpmError) as e:
            c.wait(t3)
        assert e.value.status == -4
        assert c.inflight() == 0
        # submit-time checks: no ticket for a query that cannot run
        with pytest.raises(gpm.GpmError) as e:
            c.submit(gpm.count_query(ids[0], (4, [(0, 1), (2, 3)]), E))
        assert e.value.status == -3
        with pytest.raises(gpm.GpmError) as e:
            c.submit(gpm.count_query(12345, "triangle", E))
        assert e.value.status == -1


def test_counting_only_pruning(ctx, oracle):
    """Counting-only pruning of twin suffixes (Sec. 5.4 (1)): edge-induced
    counts of patterns whose last r twins are chosen as C(n, r) from one
    candidate set equal the plain DFS plan (decompose = 0), the oracle's
    embeddings / |Aut|, and the closed forms on K_n."""
    import math
    book3 = (5, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (0, 4), (1, 4)])
    k23 = (5, [(0, 2), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4)])
    k24 = (6, [(0, 2), (0, 3), (0, 4), (0, 5), (1, 2), (1, 3), (1, 4), (1, 5)])
    star4 = (5, [(0, 1), (0, 2), (0, 3), (0, 4)])
    pendants = (5, [(0, 1), (1, 2), (0, 2), (0, 3), (0, 4)])
    house_twins = (6, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4), (0, 5), (1, 5)])
    pats = [book3, k23, k24, star4, pendants, house_twins]
    for p in pats:
        assert gpm_plan_r(p) >= 2, p
    gs = [synth.erdos_renyi(60, 0.2, 1801), synth.rmat(8, 8, seed=1802),
          synth.chung_lu(400, 6.0, 2.1, 60.0, 1200, 1803), synth.complete_multipartite([3, 4, 5])]
    for g in gs:
        gid = ctx.load(g)
        try:
            for p in pats:
                exp = oracle.count_embed(g, p, False)
                ctx.set_option("decompose", 0)
                plain = ctx.count(gid, p, E)
                ctx.set_option("decompose", 1)
                got = ctx.count(gid, p, E)
                assert got == plain == exp, (g.name, p, got, plain, exp)
        finally:
            ctx.set_option("decompose", 1)
            ctx.unload(gid)
    # closed forms: a spine edge and 3 of the other n - 2 vertices (book, K_{2,3})
    kn = synth.complete(12)
    gid = ctx.load(kn)
    try:
        assert ctx.count(gid, book3, E) == math.comb(12, 2) * math.comb(10, 3)
        assert ctx.count(gid, k23, E) == math.comb(12, 2) * math.comb(10, 3)
        assert ctx.count(gid, star4, E) == 12 * math.comb(11, 4)
    finally:
        ctx.unload(gid)
    # larger leaf sets (C(n, r) far beyond 32 bits) on an R-MAT graph with
    # hubs, against the closed forms: books = sum over edges of C(t_e, 3)
    # (t_e from A^2 on the edges), 4-stars = sum over vertices of C(d, 4)
    g = synth.rmat(12, 16, seed=1804)
    A = np.zeros((g.n, g.n), dtype=np.float32)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[src, g.col] = 1.0
    t = (A @ A)[src, g.col].astype(np.int64)          # exact: entries < 2^24
    up = src < g.col
    books = sum(math.comb(int(x), 3) for x in t[up])
    stars = sum(math.comb(int(d), 4) for d in np.diff(g.row_ptr))
    assert stars > 1 << 32
    gid = ctx.load(g)
    try:
        assert ctx.count(gid, book3, E) == books
        assert ctx.count(gid, star4, E) == stars
    finally:
        ctx.unload(gid)


def gpm_plan_r(p):
    from paper_2112_09761_amd import gpm
    return gpm.plan(p, E)["count_only_r"]


def test_edge_terms_fallback_with_large_roots(ctx, oracle):
    """Per-edge motif terms: with roots beyond the local-graph limit the
    triangle scatter cannot see every triangle, so the per-edge intersections
    run instead; both routes must give the closed forms and the oracle."""
    import math
    kn = synth.complete(100)
    g = synth.rmat(13, 16, seed=1301)   # 245 roots with more than 64 out-neighbours
    ids = [ctx.load(kn), ctx.load(g)]
    c4 = math.comb(100, 4)
    try:
        for lim in (64, 2048):
            ctx.set_option("lgs_max", lim)
            assert ctx.motifs(ids[0], 4) == [0, 0, 0, 0, 0, c4], lim
            assert ctx.count(ids[0], "diamond", E) == 6 * c4, lim
            assert ctx.count(ids[0], "tailed_triangle", E) == 12 * c4, lim
            assert ctx.motifs(ids[1], 4) == oracle.motifs4(g), lim
            assert ctx.count(ids[1], "path4", V) == oracle.count(g, "path4", True), lim
    finally:
        ctx.set_option("lgs_max", 2048)
        for gid in ids:
            ctx.unload(gid)


def test_error_paths_on_device(oracle):
    """Load-time validation, unknown ids, bad modes, unsupported patterns on a
    DAG-only graph, a memory budget too small for any frontier, and a full
    serving queue all return their status codes (no abort, no count).  The
    test changes the budget, so it runs on a context of its own."""
    import numpy as np
    import torch
    from paper_2112_09761_amd import gpm
    with gpm.Context(0, torch.cuda.current_stream()) as ctx:
        _error_paths(ctx, oracle)


def _error_paths(ctx, oracle):
    import numpy as np
    from paper_2112_09761_amd import gpm
    with pytest.raises(gpm.GpmError) as e:
        ctx.load_csr(np.array([0, 1, 2]), np.array([0, 1]))          # self loops
    assert e.value.status == -2
    g = synth.rmat(9, 8, seed=951)
    gid = ctx.load(g)
    with pytest.raises(gpm.GpmError) as e:
        ctx.count(gid, "triangle", 7)
    assert e.value.status == -1
    with pytest.raises(gpm.GpmError) as e:
        ctx.count(gid, (4, [(0, 1), (2, 3)]))                        # disconnected
    assert e.value.status == -3
    # a DAG-only graph supports cliques only
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = g.col > src
    rp = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src[keep], minlength=g.n), out=rp[1:])
    did = ctx.load_csr(rp, g.col[keep], gpm.GPM_CSR_DAG | gpm.GPM_VALIDATE)
    assert ctx.count(did, "clique4") == ctx.count(gid, "clique4")
    with pytest.raises(gpm.GpmError) as e:
        ctx.count(did, "diamond", 1)
    assert e.value.status == -6
    ctx.unload(did)
    # budget too small for even one wave's frontier (the DFS plan stores a
    # level; the decomposed count would need no frontier at all)
    ctx.set_option("budget", 1024)
    ctx.set_option("decompose", 0)
    try:
        with pytest.raises(gpm.GpmError) as e:
            ctx.count(gid, "diamond", 1)
        assert e.value.status == -4
        ctx.set_option("decompose", 1)
        assert ctx.count(gid, "diamond", 1) == oracle.count(g, "diamond", False)
    finally:
        ctx.set_option("budget", 1 << 36)
        ctx.set_option("decompose", 1)
    # serving: a full pending list says busy, the queued query still completes
    ctx.set_option("max_pending", 1)
    try:
        t1 = ctx.submit(gpm.count_query(gid, "clique5", 0))
        extra = []
        for _ in range(64):
            try:
                extra.append(ctx.submit(gpm.count_query(gid, "clique4", 0)))
            except gpm.GpmError as err:
                assert err.status == -7
        assert ctx.wait(t1)[0] == ctx.count(gid, "clique5")
        for t in extra:
            ctx.wait(t)
    finally:
        ctx.set_option("max_pending", 1 << 20)
    ctx.unload(gid)
