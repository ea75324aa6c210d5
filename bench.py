#!/usr/bin/env python
"""Benchmark: exact 4-clique + 5-clique counting on the R-MAT scale-20 graph.

One step = gpm_count(4-clique) + gpm_count(5-clique) on the resident,
prepared graph (2^20 vertices, edge factor 16, (a,b,c) = (0.57, 0.19, 0.19),
degree-oriented).  Preparation (generation, upload, orientation) happens
before the timed region, as in the paper's evaluation.

Prints ONE JSON line: intersected elements/s over the timed steps, the
roofline of the dominant kernel (the longest launch of a step) and the CPU oracle's
rate on a bounded sample.  Other workloads (--workload batch | serve |
triangle | chunglu | list) print their own line.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 64-bit AND + popcount(-accumulate) word operations: 2 v_and_b32 + 2
# v_bcnt_u32_b32 per word; 256 CUs x 64 int32 lanes/clock x 2.4 GHz / 4
WORD_OP_PEAK_TOPS = 256 * 64 * 2.4e9 / 4 / 1e12

# HBM traffic of the dominant launch: two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE; KiB per dispatch) each scaled by what the same counter reads for
# a plain device copy of 1 GiB (--copy-calibration): FETCH_SIZE reads 0.5 GiB
# for it (factor 2.0), WRITE_SIZE 1 GiB (factor 1.0).  The figures hold for
# the kernel sources they were taken on (and that launch) only; else null.
TRAFFIC = {"sources_sha256": "a2a57d884de457215b6a386dcdf1294a3f9e53688a4565386683db919aff8356",
           "k": 5, "kinds": 1 << 7, "fetch_kib": 1914028.1, "write_kib": 3938.2,
           "fetch_factor": 2.0, "write_factor": 1.0}
TRAFFIC_SOURCES = ["kernels.hip", "gpm_internal.h", "runtime.cpp"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="clique",
                    choices=["clique", "triangle", "chunglu", "batch", "serve", "list"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--queries", default="cycle4,diamond,tailed_triangle,motifs3",
                    help="chunglu workload: the queries to time (comma separated)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default kernel knobs (fixed dispatch sequence)")
    ap.add_argument("--option", action="append", default=[],
                    help="library option key=value (tuning sweeps)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (x steps), the "
                         "reference for scaling hardware byte counters")
    return ap.parse_args()


def golden(name):
    p = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json")
    if os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return None


def algorithmic_bytes(st):
    # 4 B per intersected element, 16 B per neighbour-list fetch (row offsets),
    # 4 B per frontier element written
    return 4 * st["elements"] + 16 * st["list_fetches"] + 4 * st["frontier_written"]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2112_09761_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(k, kinds):
    """HBM bytes per launch from the counters, or None if stale."""
    if (not TRAFFIC["sources_sha256"] or TRAFFIC["sources_sha256"] != sources_sha256()
            or TRAFFIC["k"] != k or TRAFFIC["kinds"] != kinds):
        return None
    return 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_factor"] +
                     TRAFFIC["write_kib"] * TRAFFIC["write_factor"])


# gpm_list on the listing workload: the same two counter passes (KiB per
# dispatch), valid for the sources they were taken on
LIST_TRAFFIC = {"sources_sha256": "a2a57d884de457215b6a386dcdf1294a3f9e53688a4565386683db919aff8356",
                "fetch_kib": 160709.2, "write_kib": 5046334.9,
                "fetch_factor": 2.0, "write_factor": 1.0}


# gpm_cycle_block (4-cycles) on the Chung-Lu workload: the same two counter
# passes (KiB per dispatch), valid for the sources they were taken on
CYC_TRAFFIC = {"sources_sha256": "a2a57d884de457215b6a386dcdf1294a3f9e53688a4565386683db919aff8356",
               "fetch_kib": 128985724.3, "write_kib": 19542572.4,
               "fetch_factor": 2.0, "write_factor": 1.0}


def measured_cycle_traffic():
    if not CYC_TRAFFIC["sources_sha256"] or CYC_TRAFFIC["sources_sha256"] != sources_sha256():
        return None
    return 1024.0 * (CYC_TRAFFIC["fetch_kib"] * CYC_TRAFFIC["fetch_factor"] +
                     CYC_TRAFFIC["write_kib"] * CYC_TRAFFIC["write_factor"])


def cpu_baseline_chunglu(g, names):
    """The oracle's routes for the same queries on the same graph, timed on
    the host's cores: codegree 4-cycles, the local 4-vertex terms (diamond,
    tailed triangle), the induced 3-motifs."""
    from oracle import pyoracle
    progress("CPU oracle baseline (Chung-Lu queries)")
    routes = {"cycle4": lambda: pyoracle.cycle4(g),
              "diamond": lambda: pyoracle.nonind4_local(g, 1)[3],
              "tailed_triangle": lambda: pyoracle.nonind4_local(g, 1)[2],
              "motifs3": lambda: pyoracle.motifs3(g, 1)}
    per, total = {}, 0.0
    counts = {}
    for name in names:
        t = time.perf_counter()
        counts[name] = routes[name]()
        dt = (time.perf_counter() - t) * 1e3
        per[name] = dt
        total += dt
    out = {"value": total, "unit": "ms", "cores": pyoracle.num_threads(), "kind": "oracle",
           "sample": "the full graph, the same queries, each by the oracle's own route "
                     "(sum of one run each)", "ms_by_query": per}
    out.update(host_cpu())
    return out, counts


def measured_list_traffic():
    if not LIST_TRAFFIC["sources_sha256"] or LIST_TRAFFIC["sources_sha256"] != sources_sha256():
        return None
    return 1024.0 * (LIST_TRAFFIC["fetch_kib"] * LIST_TRAFFIC["fetch_factor"] +
                     LIST_TRAFFIC["write_kib"] * LIST_TRAFFIC["write_factor"])


def host_cpu():
    """The host CPU the oracle ran on: model name and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline_clique4(g, elements4):
    from oracle import pyoracle
    progress("CPU oracle baseline (4-clique)")
    t = time.perf_counter()
    c = pyoracle.cliques(g, 4, 1)
    dt = time.perf_counter() - t
    out = {"value": elements4 / dt, "unit": "elem/s", "cores": pyoracle.num_threads(),
           "kind": "oracle",
           "sample": f"4-clique count of the full graph (one of the step's two counts): "
                     f"{dt:.1f} s, count {c}; elements = those the timed GPU kernels "
                     f"intersect for that count"}
    out.update(host_cpu())
    return out, c


KERNEL_NAMES = {1 << 7: "gpm_lgs_block (local-graph cliques, one workgroup per root)",
                1 << 5: "gpm_persistent<local-graph cliques> (one wave per root)"}


def kernel_name(kinds):
    return KERNEL_NAMES.get(kinds, f"gpm_persistent<kinds 0x{kinds:x}>")


def run_clique(args, ctx, torch):
    from paper_2112_09761_amd import synth
    g = synth.workload_rmat_s20()
    progress("graph generated")
    tp = time.perf_counter()
    gid = ctx.load(g)           # host arrays -> HBM (PCIe) and validation
    info = ctx.graph_info(gid)  # forces the degree orientation (untimed)
    torch.cuda.synchronize()
    prepare_s = time.perf_counter() - tp
    progress("graph loaded and prepared")
    pats = {k: (k, [(i, j) for i in range(k) for j in range(i + 1, k)]) for k in (4, 5)}
    if not args.no_autotune:
        ctx.set_option("autotune", 1)   # the first (warm-up) call of each count tunes
    for _ in range(max(args.warmup, 1)):
        for k in (4, 5):
            ctx.count(gid, pats[k])
    progress("warm-up done")
    # instrumented passes (never timed), with the knobs the timed calls use:
    # the elements the timed kernels (local-graph bitmaps) intersect, their
    # word operations and list fetches per launch (roofline of the dominant
    # launch); and, for context only, the elements the paper's sorted-list
    # plan (edge kernel, clique_algo=1) would intersect for the same counts.
    ctx.set_option("count_elements", 1)
    inst, inst_lgs = {}, {}
    for k in (4, 5):
        ctx.set_option("clique_algo", 1)
        ctx.count(gid, pats[k])
        inst[k] = ctx.stats()
        ctx.set_option("clique_algo", 0)
        ctx.count(gid, pats[k])
        inst_lgs[k] = ctx.stats()
    ctx.set_option("count_elements", 0)
    progress("instrumented passes done")
    torch.cuda.synchronize()
    kms = {4: [], 5: []}
    lms = {4: [], 5: []}
    kinds = {}
    counts = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for k in (4, 5):
            counts[k] = ctx.count(gid, pats[k])
            st = ctx.stats()
            kms[k].append(st["kernel_ms"])
            lms[k].append(st["launch_ms"])
            kinds[k] = st["launch_kinds"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    E = inst_lgs[4]["elements"] + inst_lgs[5]["elements"]
    value = E * args.steps / dt
    E_plan = inst[4]["elements"] + inst[5]["elements"]
    gold = golden("rmat_s20")
    parity = None
    if gold and gold["sha256"] == g.sha256():
        parity = (counts[4] == gold["counts"]["clique4"] and counts[5] == gold["counts"]["clique5"])
    # per-launch means over the timed region (HIP events on the library's stream)
    launches = {}
    for k in (4, 5):
        assert inst_lgs[k]["launch_kinds"] == kinds[k], "instrumented and timed launches differ"
        launches[k] = []
        for i, kd in enumerate(kinds[k]):
            ms = statistics.mean(x[i] for x in lms[k])
            words = inst_lgs[k]["launch_words"][i]
            byts = (4 * inst_lgs[k]["launch_elements"][i] + 16 * inst_lgs[k]["launch_fetches"][i]
                    + 4 * inst_lgs[k]["launch_written"][i])
            launches[k].append({"kernel": kernel_name(kd), "kinds": kd, "ms": ms,
                                "word_ops": words, "algorithmic_bytes": byts})
    # dominant launch: the longest one of the step
    dom_k, dom = max(((k, L) for k in (4, 5) for L in launches[k]), key=lambda x: x[1]["ms"])
    achieved = dom["word_ops"] / (dom["ms"] * 1e-3) / 1e12
    hbm_gbs = dom["algorithmic_bytes"] / (dom["ms"] * 1e-3) / 1e9
    out = {
        "metric": "intersected elements/s of the timed kernels, exact 4-clique + 5-clique counts",
        "value": value, "unit": "elem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "rmat_s20_ef16_clique4_clique5", "n": g.n, "m": g.m,
                   "max_degree": info["max_degree"],
                   "max_out_degree": info["max_out_degree"],
                   "orientation": "degree", "counts_per_step": 2},
        "prepare_s": prepare_s,
        "counts": {"clique4": counts[4], "clique5": counts[5]},
        "parity_vs_stored_oracle": parity,
        "ms_per_count": {"clique4": statistics.mean(kms[4]), "clique5": statistics.mean(kms[5])},
        "launches": {"clique4": launches[4], "clique5": launches[5]},
        "elements_per_count": {"clique4": inst_lgs[4]["elements"],
                               "clique5": inst_lgs[5]["elements"]},
        "sorted_list_plan": {
            "note": "elements the paper's sorted-list plan would intersect for the same "
                    "counts (instrumented edge kernel), over the timed step: an "
                    "effective rate, not work the timed kernels do",
            "elements_per_count": {"clique4": inst[4]["elements"], "clique5": inst[5]["elements"]},
            "effective_elem_per_s": E_plan * args.steps / dt},
        "roofline": {"bound": "alu", "kernel": f"{dom['kernel']}, {dom_k}-clique launch",
                     "achieved": achieved, "peak": WORD_OP_PEAK_TOPS,
                     "unit": "TOP/s (64-bit AND+popcount word ops)",
                     "frac": achieved / WORD_OP_PEAK_TOPS,
                     "traffic": measured_traffic(dom_k, dom["kinds"]),
                     "word_ops_per_launch": dom["word_ops"], "launch_ms": dom["ms"],
                     "hbm_view": {"algorithmic_bytes_per_launch": dom["algorithmic_bytes"],
                                  "achieved_GBs": hbm_gbs, "peak_GBs": HBM_PEAK_GBS,
                                  "frac": hbm_gbs / HBM_PEAK_GBS}},
    }
    return out, g, inst_lgs


def run_triangle(args, ctx, torch):
    from paper_2112_09761_amd import synth
    g = synth.workload_er_triangle(1)
    gid = ctx.load(g)
    ctx.graph_info(gid)
    ctx.set_option("count_elements", 1)
    ctx.count(gid, "triangle")
    inst = ctx.stats()
    ctx.set_option("count_elements", 0)
    for _ in range(args.warmup):
        ctx.count(gid, "triangle")
    torch.cuda.synchronize()
    ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c = ctx.count(gid, "triangle")
        ms.append(ctx.stats()["kernel_ms"])
    dt = time.perf_counter() - t0
    return {"metric": "triangle count time (ER G(2000, 0.01))", "value": dt * 1e3 / args.steps,
            "unit": "ms/count", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": "er_2000_p0.01_triangle"}, "count": c,
            "kernel_ms": statistics.mean(ms), "elements": inst["elements"]}


def rows_are_cliques(g, rows):
    """Every row k distinct vertices, every pair adjacent (sorted CSR lookup)."""
    import numpy as np
    rows = rows.astype(np.int64)
    k = rows.shape[1]
    if (np.sort(rows, axis=1)[:, 1:] == np.sort(rows, axis=1)[:, :-1]).any():
        return False
    for a in range(k):
        for b in range(a + 1, k):
            u, v = rows[:, a], rows[:, b]
            lo, hi = g.row_ptr[u], g.row_ptr[u + 1]
            for i in range(len(u)):
                j = lo[i] + np.searchsorted(g.col[lo[i]:hi[i]], v[i])
                if j >= hi[i] or g.col[j] != v[i]:
                    return False
    return True


def cpu_baseline_list():
    from oracle import pyoracle
    from paper_2112_09761_amd import synth
    progress("CPU oracle baseline (4-clique listing, R-MAT scale 11)")
    g = synth.rmat(11, 16, 0.57, 0.19, 0.19, 1)
    cap = pyoracle.cliques(g, 4, 1)
    t = time.perf_counter()
    _, c = pyoracle.list_embed(g, pyoracle.clique(4), True, cap=cap)
    dt = time.perf_counter() - t
    return {"value": c / dt, "unit": "matches/s", "cores": 1, "kind": "oracle",
            "sample": f"4-clique listing of R-MAT scale 11, edge factor 16 (same generator, "
                      f"1/32 of the vertices): {c} rows in {dt:.1f} s (serial routine)"}


def run_list(args, ctx, torch):
    """4-clique listing (gpm_list) on R-MAT scale 16, edge factor 16: every
    4-clique written once as a row of 4 vertex ids into a device buffer sized
    for all of them (4.7 GB); one step = one gpm_list call."""
    import numpy as np
    from paper_2112_09761_amd import synth
    g = synth.workload_rmat_s16()
    gid = ctx.load(g)
    ctx.graph_info(gid)
    pat = (4, [(i, j) for i in range(4) for j in range(i + 1, 4)])
    total = ctx.count(gid, pat)   # sizes the buffer (untimed)
    buf = torch.empty((total, 4), dtype=torch.int32, device="cuda")
    for _ in range(max(args.warmup, 1)):
        ctx.list(gid, pat, buf)
    torch.cuda.synchronize()
    progress("warm-up done")
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        n = ctx.list(gid, pat, buf)
        kms.append(ctx.stats()["kernel_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gold = golden("rmat_s16")
    parity = None
    if gold and gold["sha256"] == g.sha256():
        rng = np.random.default_rng(11)
        pick = torch.from_numpy(rng.choice(n, size=min(n, 20000), replace=False)).cuda()
        sample = buf[pick].cpu().numpy()
        parity = bool(n == gold["counts"]["clique4"] and rows_are_cliques(g, sample))
    launch_ms = statistics.mean(kms)
    cms = []
    for _ in range(3):  # the same 4-cliques counted (context for the listing cost)
        ctx.count(gid, pat)
        cms.append(ctx.stats()["kernel_ms"])
    # algorithmic bytes of the launch: the rows written plus one read of the
    # degree-oriented DAG (offsets and out-lists)
    dag_bytes = 8 * (g.n + 1) + 4 * g.m
    byts = 16 * n + dag_bytes
    gbs = byts / (launch_ms * 1e-3) / 1e9
    return {"metric": "4-cliques listed/s (rows written to HBM)", "value": n * args.steps / dt,
            "unit": "matches/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": "rmat_s16_ef16_list_clique4", "n": g.n, "m": g.m,
                       "rows": n, "row_bytes": 16},
            "parity_vs_stored_oracle": parity, "kernel_ms": launch_ms,
            "count_kernel_ms": statistics.mean(cms),
            "roofline": {"bound": "hbm", "limiter": "latency of the leaf's dependent loads "
                                                    "(the HBM fraction is low by that, not by bytes)",
                         "kernel": "gpm_list (plan-driven walk, rows staged in LDS)",
                         "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": measured_list_traffic(),
                         "algorithmic_bytes_per_launch": byts, "launch_ms": launch_ms}}


def run_chunglu(args, ctx, torch):
    """Chung-Lu graph, n = 4M, m = 60M (power-law weights, gamma 2.1): edge-induced
    4-cycle, diamond and tailed-triangle counts and the induced 3-motifs, each
    timed as the median of warm calls on the resident, prepared graph."""
    from paper_2112_09761_amd import synth
    g = synth.workload_chung_lu_4m()
    progress("graph generated")
    tp = time.perf_counter()
    gid = ctx.load(g)
    ctx.prepare(gid)
    info = ctx.graph_info(gid)
    torch.cuda.synchronize()
    prepare_s = time.perf_counter() - tp
    progress("graph loaded and prepared")
    gold = golden("chung_lu_4m")
    ok = bool(gold and gold["sha256"] == g.sha256())
    nonind = gold["counts"]["nonind4"] if ok else None
    expect = {"cycle4": nonind[2] if ok else None, "tailed_triangle": nonind[3] if ok else None,
              "diamond": nonind[4] if ok else None,
              "motifs3": gold["counts"]["motifs3"] if ok else None}
    if not args.no_autotune:
        ctx.set_option("autotune", 1)
    res = {}
    total = 0.0
    names = [q for q in args.queries.split(",") if q]
    for name in names:
        def call():
            return ctx.motifs(gid, 3) if name == "motifs3" else ctx.count(gid, name, 1)
        for _ in range(max(args.warmup, 1)):
            call()
        torch.cuda.synchronize()
        wall, kms = [], []
        for _ in range(args.steps):
            t = time.perf_counter()
            c = call()
            wall.append((time.perf_counter() - t) * 1e3)
            kms.append(ctx.stats()["kernel_ms"])
        med = statistics.median(wall)
        total += med
        res[name] = {"median_ms": med, "kernel_ms_median": statistics.median(kms), "count": c,
                     "parity_vs_stored_oracle": (c == expect[name]) if ok else None}
        progress(f"{name}: {med:.1f} ms")
    out = {"metric": f"count time, Chung-Lu n=4M m=60M (sum of the medians of {len(names)} "
                     f"queries)",
           "value": total, "unit": "ms", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": total, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "chung_lu_4m_gamma2.1", "n": g.n, "m": g.m,
                      "max_degree": info["max_degree"], "queries": names},
           "prepare_s": prepare_s, "queries": res}
    if "cycle4" in names:
        # roofline of the 4-cycle launch (the step's longest): algorithmic
        # bytes = 4 B per wedge endpoint read + 16 B per neighbour-list visit
        # (offsets), from an instrumented pass (never timed)
        ctx.set_option("count_elements", 1)
        ctx.count(gid, "cycle4", 1)
        si = ctx.stats()
        ctx.set_option("count_elements", 0)
        ms = res["cycle4"]["kernel_ms_median"]
        byts = 4 * si["elements"] + 16 * si["list_fetches"]
        gbs = byts / (ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": "gpm_cycle_block (4-cycle wedge aggregation "
                                                     "in LDS, one workgroup per task)",
                           "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS, "traffic": measured_cycle_traffic(),
                           "algorithmic_bytes_per_launch": byts, "launch_ms": ms,
                           "wedges_per_launch": si["elements"],
                           "list_visits_per_launch": si["list_fetches"],
                           "wedges_per_s": si["elements"] / (ms * 1e-3)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"], oc = cpu_baseline_chunglu(g, names)
        out["cpu_baseline_counts_match"] = all(oc[q] == res[q]["count"] for q in names)
    return out


def _gen_batch(i):
    from paper_2112_09761_amd import synth
    g = synth.batch_graph(i)
    return g.n, g.row_ptr, g.col


def _gen_pool(i):
    from paper_2112_09761_amd import synth
    g = synth.serve_pool_graph(i)
    return g.n, g.row_ptr, g.col


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gen_parallel(fn, count, procs=16):
    import multiprocessing as mp
    out = [None] * count
    with mp.get_context("spawn").Pool(procs) as pool:
        for i, r in enumerate(pool.imap(fn, range(count), chunksize=1)):
            out[i] = r
            progress(f"generated graph {i + 1}/{count} (n={r[0]})")
    return out


def run_batch(args, ctx, torch):
    """256 graphs x induced 4-motifs: 256 plain per-graph calls vs ONE batched
    persistent launch over all of them."""
    from paper_2112_09761_amd import gpm
    t = time.perf_counter()
    graphs = gen_parallel(_gen_batch, 256)
    gen_s = time.perf_counter() - t
    ids = [ctx.load_csr(rp, col) for n, rp, col in graphs]
    for gid in ids:
        ctx.graph_info(gid)
    progress("batch graphs loaded and prepared")
    qs = [gpm.motif_query(gid, 4) for gid in ids]
    ctx.count_batch(qs)  # preparation of every graph (untimed) and warm-up
    for gid in ids[:8]:
        ctx.motifs(gid, 4)
    plain_t, batch_t = [], []
    for _ in range(max(args.steps, 1)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plain = [ctx.motifs(gid, 4) for gid in ids]
        torch.cuda.synchronize()
        plain_t.append(time.perf_counter() - t)
        t = time.perf_counter()
        batched = ctx.count_batch(qs)
        torch.cuda.synchronize()
        batch_t.append(time.perf_counter() - t)
    gold = golden("batch256")
    parity = None
    if gold:
        parity = all(r["motifs4"] == plain[i] == batched[i] for i, r in enumerate(gold["graphs"]))
    tp, tb = statistics.median(plain_t), statistics.median(batch_t)
    return {"metric": "batched vs plain speedup (256 graphs x induced 4-motifs)",
            "value": tp / tb, "unit": "x", "n_gpus": 1, "steps": len(plain_t),
            "warmup": 1, "ms_per_step": tb * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": "batch256_motifs4", "graphs": 256,
                       "adjacency_entries": int(sum(c.size for _, _, c in graphs))},
            "plain_ms": tp * 1e3, "batched_ms": tb * 1e3, "generation_s": gen_s,
            "results_identical_plain_vs_batched": plain == batched,
            "parity_vs_stored_oracle": parity}


SERVE_PATTERNS = [("triangle", 0), ("clique4", 0), ("clique5", 0),
                  ("cycle4", 1), ("diamond", 1), ("tailed_triangle", 1)]


def run_serve(args, ctx, torch):
    """Poisson stream of (graph, pattern) queries over a resident pool of 32
    R-MAT graphs (scales 16..23), continuous batching; per offered load 100
    warm-up queries, then 1000 measured ones; p50/p99 latency overall and per
    pattern; the served form against a plain one-query-at-a-time run of the
    same stream."""
    import numpy as np
    from paper_2112_09761_amd import gpm
    n_pool = int(os.environ.get("GPM_SERVE_POOL", "32"))
    n_q = int(os.environ.get("GPM_SERVE_QUERIES", "1000"))
    n_warm = int(os.environ.get("GPM_SERVE_WARMUP", "100"))
    t = time.perf_counter()
    graphs = gen_parallel(_gen_pool, n_pool)
    gen_s = time.perf_counter() - t
    ids, shas = [], []
    for i, (n, rp, col) in enumerate(graphs):
        ids.append(ctx.load_csr(rp, col))
        ctx.prepare(ids[-1])   # resident and prepared before any query
        progress(f"pool graph {i + 1}/{n_pool} loaded and prepared")
    del graphs
    ctx.set_option("max_batch", int(os.environ.get("GPM_SERVE_MAX_BATCH", "8")))
    # every (graph, pattern) pair alone (the graphs are prepared): reference
    # results and costs
    alone, cost = {}, {}
    for gi, gid in enumerate(ids):
        for pi, (name, mode) in enumerate(SERVE_PATTERNS):
            t = time.perf_counter()
            alone[(gi, pi)] = ctx.count(gid, name, mode)
            cost[(gi, pi)] = time.perf_counter() - t
        progress(f"alone: graph {gi + 1}/{n_pool} done")
    gold = golden("serve_pool")
    oracle_checked = oracle_ok = 0
    if gold:
        by_i = {r["i"]: r for r in gold["graphs"]}
        for (gi, pi), c in alone.items():
            rec = by_i.get(gi, {}).get("counts", {})
            name = SERVE_PATTERNS[pi][0]
            if name in rec:
                oracle_checked += 1
                oracle_ok += int(rec[name] == c)
    rng = np.random.default_rng(20_000)

    def draw(n):
        return [(int(rng.integers(0, n_pool)), int(rng.integers(0, len(SERVE_PATTERNS))))
                for _ in range(n)]

    def query(gi, pi):
        name, mode = SERVE_PATTERNS[pi]
        return gpm.count_query(ids[gi], name, mode)

    mix_ok = True
    mismatches = []

    def check(phase, pair, got):
        nonlocal mix_ok
        if got != alone[pair]:
            mix_ok = False
            if len(mismatches) < 20:
                mismatches.append({"phase": phase, "graph": pair[0],
                                   "pattern": SERVE_PATTERNS[pair[1]][0], "got": got,
                                   "alone": alone[pair]})
                progress(f"MISMATCH {mismatches[-1]}")

    def closed_loop(qs, label):
        """All queries submitted at once (as the slots and the pending list
        take them); returns queries/s."""
        t0 = time.perf_counter()
        pending = {}
        nxt = 0
        done_n = 0
        while nxt < len(qs) or pending:
            while nxt < len(qs):
                try:
                    pending[ctx.submit(query(*qs[nxt]))] = nxt
                    nxt += 1
                except gpm.GpmError as e:
                    if e.status != -7:
                        raise
                    break
            for tk in list(pending):
                done, out = ctx.poll(tk)
                if done:
                    i = pending.pop(tk)
                    check(label, qs[i], out[0])
                    done_n += 1
                    if done_n % 200 == 0:
                        progress(f"{label}: {done_n}/{len(qs)} done")
        return len(qs) / (time.perf_counter() - t0)

    # saturated throughput mu (closed loop), then the plain form: the same
    # stream one query at a time, each waiting for the previous one
    sat = draw(n_q)
    mu = closed_loop(sat, "saturated")
    progress(f"saturated throughput {mu:.1f} queries/s")
    t0 = time.perf_counter()
    for j, (gi, pi) in enumerate(sat):
        name, mode = SERVE_PATTERNS[pi]
        check("plain", (gi, pi), ctx.count(ids[gi], name, mode))
        if (j + 1) % 200 == 0:
            progress(f"plain: {j + 1}/{n_q} done")
    plain_qps = n_q / (time.perf_counter() - t0)
    progress(f"plain throughput {plain_qps:.1f} queries/s")
    loads = []
    for frac in (0.3, 0.6, 0.9):
        lam = frac * mu
        total = n_warm + n_q
        qs = draw(total)
        arrive = np.cumsum(rng.exponential(1.0 / lam, size=total))
        lat = [None] * total
        pending = {}
        t0 = time.perf_counter()
        nxt = 0
        finished = 0
        t_first = t_last = None
        while nxt < total or pending:
            now = time.perf_counter() - t0
            while nxt < total and arrive[nxt] <= now:
                gi, pi = qs[nxt]
                pending[ctx.submit(query(gi, pi))] = nxt
                nxt += 1
            for tk in list(pending):
                done, out = ctx.poll(tk)
                if done:
                    i = pending.pop(tk)
                    lat[i] = (time.perf_counter() - t0) - arrive[i]
                    check(f"load {frac}", qs[i], out[0])
                    finished += 1
                    if finished % 200 == 0:
                        progress(f"load {frac}: {finished}/{total} done")
            if not pending and nxt < total:
                time.sleep(max(0.0, min(arrive[nxt] - (time.perf_counter() - t0), 0.001)))
        # measured window: the queries after the warm-up ones
        meas = list(range(n_warm, total))
        span = max(arrive[i] + lat[i] for i in meas) - arrive[n_warm]
        la = np.array([lat[i] for i in meas]) * 1e3
        per = {}
        for pi, (name, _) in enumerate(SERVE_PATTERNS):
            x = np.array([lat[i] for i in meas if qs[i][1] == pi]) * 1e3
            if x.size:
                per[name] = {"p50_ms": float(np.percentile(x, 50)),
                             "p99_ms": float(np.percentile(x, 99)), "queries": int(x.size)}
        achieved = n_q / span
        progress(f"load {frac}: {achieved:.1f} queries/s, p50 {np.percentile(la, 50):.0f} ms, "
                 f"p99 {np.percentile(la, 99):.0f} ms")
        loads.append({"offered_qps": lam, "achieved_qps": achieved,
                      "p50_ms": float(np.percentile(la, 50)),
                      "p99_ms": float(np.percentile(la, 99)), "queries": n_q,
                      "warmup_queries": n_warm, "per_pattern": per})
    per_pattern = {SERVE_PATTERNS[pi][0]: float(np.median([cost[(g, pi)] for g in range(n_pool)]) * 1e3)
                   for pi in range(len(SERVE_PATTERNS))}
    return {"metric": "served queries/s and p99 latency (Poisson stream, continuous batching)",
            "value": loads[-1]["achieved_qps"], "unit": "queries/s", "n_gpus": 1,
            "steps": n_q, "warmup": n_warm, "ms_per_step": 1e3 / loads[-1]["achieved_qps"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "int32", "data": "synthetic",
            "config": {"workload": "serve_rmat_pool", "pool_graphs": n_pool,
                       "scales": sorted({16 + i // 4 for i in range(n_pool)}),
                       "patterns": [p for p, _ in SERVE_PATTERNS]},
            "saturated_qps": mu, "plain_qps": plain_qps, "served_vs_plain": mu / plain_qps,
            "loads": loads, "alone_vs_mix_identical": bool(mix_ok), "mismatches": mismatches,
            "pairs_checked_against_stored_oracle": oracle_checked,
            "pairs_equal_to_stored_oracle": oracle_ok,
            "median_alone_ms_by_pattern": per_pattern, "generation_s": gen_s}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the counting "
              f"path needs no collective and is measured on one MI355X.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2112_09761_amd import gpm
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": args.steps}), flush=True)
        return
    ctx = gpm.Context(0, torch.cuda.current_stream())
    for kv in args.option:
        k, v = kv.split("=")
        ctx.set_option(k, int(v))
    if args.workload == "clique":
        out, g, inst = run_clique(args, ctx, torch)
        if not args.no_cpu_baseline:
            out["cpu_baseline"], c4 = cpu_baseline_clique4(g, inst[4]["elements"])
            out["cpu_baseline_count_matches"] = c4 == out["counts"]["clique4"]
        else:
            out["cpu_baseline"] = None
    elif args.workload == "chunglu":
        out = run_chunglu(args, ctx, torch)
    elif args.workload == "triangle":
        out = run_triangle(args, ctx, torch)
    elif args.workload == "batch":
        out = run_batch(args, ctx, torch)
    elif args.workload == "list":
        out = run_list(args, ctx, torch)
        out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline_list()
    else:
        out = run_serve(args, ctx, torch)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
