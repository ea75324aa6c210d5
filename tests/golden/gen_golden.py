"""Write stored oracle counts for the large synthetic workloads.

Calls only the CPU oracle (oracle/) on graphs from the seeded generators;
each record carries the sha256 of the generated CSR so a test can confirm
it regenerated the same graph.  Run:  python tests/golden/gen_golden.py NAME
(NAME: rmat_s20, rmat_s16, chung_lu_4m, batch256, or serve_pool with optional
pattern list, largest scale and first degree-oriented scale).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import pyoracle as O  # noqa: E402
from paper_2112_09761_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

WORKLOADS = {
    # R-MAT scale 20, edge factor 16: 4- and 5-clique counting (and triangles)
    "rmat_s20": (synth.workload_rmat_s20,
                 [("triangle", lambda g: O.cliques(g, 3, 1)),
                  ("clique4", lambda g: O.cliques(g, 4, 1)),
                  ("clique5", lambda g: O.cliques(g, 5, 1))]),
    # R-MAT scale 16, edge factor 16: the 4-clique listing workload
    "rmat_s16": (synth.workload_rmat_s16,
                 [("triangle", lambda g: O.cliques(g, 3, 1)),
                  ("clique4", lambda g: O.cliques(g, 4, 1))]),
    # Chung-Lu n = 4M, 60M edges: edge-induced 4-cycle, diamond, tailed
    # triangle, induced 3-motifs
    "chung_lu_4m": (synth.workload_chung_lu_4m,
                    [("motifs3", lambda g: O.motifs3(g, 1)),
                     ("nonind4", lambda g: O.nonind4(g, 1))]),
}


def batch_golden():
    """Induced 4-motif counts of the 256 graphs of the batched workload."""
    recs = []
    t0 = time.time()
    for i in range(256):
        g = synth.batch_graph(i)
        t = time.time()
        recs.append({"i": i, "n": g.n, "m": g.m, "sha256": g.sha256(),
                     "motifs4": O.motifs4(g, 1), "seconds": round(time.time() - t, 2)})
        print(i, g.n, g.m, recs[-1]["motifs4"], recs[-1]["seconds"], flush=True)
    with open(os.path.join(HERE, "batch256_oracle.json"), "w") as f:
        json.dump({"workload": "batch256", "oracle_threads": O.num_threads(),
                   "seconds": round(time.time() - t0, 1), "graphs": recs}, f, indent=0)


# The patterns of the serving workload: (name, induced mode as served, route).
# Cliques use the id-oriented DAG (the library orients by degree), edge-induced
# 4-cycles the codegree count, diamond and tailed triangle the local triangle
# terms.
POOL_ROUTES = {
    "triangle": lambda g, o: O.triangles(g, o),
    "clique4": lambda g, o: O.cliques(g, 4, o),
    "clique5": lambda g, o: O.cliques(g, 5, o),
    "cycle4": lambda g, o: O.cycle4(g),
    "diamond": lambda g, o: O.nonind4_local(g, o)[3],
    "tailed_triangle": lambda g, o: O.nonind4_local(g, o)[2],
}


def pool_golden(patterns, max_scale, degree_from_scale):
    """Oracle counts of the 32-graph serving pool (R-MAT ef 16, four graphs per
    scale 16..23), one record per graph, written after every count so a long
    run can be resumed; pairs already stored for the same CSR are skipped.
    Cliques are counted on the id-oriented DAG below `degree_from_scale` and
    on the (degree, id)-oriented one from that scale on (recorded per count).
    """
    path = os.path.join(HERE, "serve_pool_oracle.json")
    db = {"workload": "serve_pool", "graphs": []}
    if os.path.exists(path):
        with open(path) as f:
            db = json.load(f)
    by_i = {r["i"]: r for r in db["graphs"]}
    for i in range(32):
        scale = 16 + i // 4
        if scale > max_scale:
            continue
        todo = [p for p in patterns if p not in by_i.get(i, {}).get("counts", {})]
        if not todo:
            continue
        g = synth.serve_pool_graph(i)
        rec = by_i.get(i)
        if rec is None or rec["sha256"] != g.sha256():
            rec = {"i": i, "scale": scale, "n": g.n, "m": g.m, "max_degree": g.max_degree(),
                   "sha256": g.sha256(), "counts": {}, "orientation": {}, "seconds": {},
                   "oracle_threads": O.num_threads()}
            by_i[i] = rec
        for p in todo:
            order = 1 if scale >= degree_from_scale else 0
            t = time.time()
            rec["counts"][p] = POOL_ROUTES[p](g, order)
            rec["seconds"][p] = round(time.time() - t, 2)
            if p in ("triangle", "clique4", "clique5", "diamond", "tailed_triangle"):
                rec["orientation"][p] = "degree" if order else "id"
            print(i, scale, p, rec["counts"][p], rec["seconds"][p], flush=True)
            db["graphs"] = [by_i[j] for j in sorted(by_i)]
            with open(path + ".tmp", "w") as f:
                json.dump(db, f, indent=1)
            os.replace(path + ".tmp", path)


def main(name, *rest):
    if name == "batch256":
        return batch_golden()
    if name == "serve_pool":
        # serve_pool [patterns,comma,separated] [max_scale] [degree_from_scale]
        pats = rest[0].split(",") if rest else list(POOL_ROUTES)
        max_scale = int(rest[1]) if len(rest) > 1 else 23
        deg_from = int(rest[2]) if len(rest) > 2 else 24
        return pool_golden(pats, max_scale, deg_from)
    mk, items = WORKLOADS[name]
    g = mk()
    rec = {"workload": name, "generator": mk.__name__, "n": g.n, "m": g.m,
           "max_degree": g.max_degree(), "sha256": g.sha256(),
           "oracle_threads": O.num_threads(), "counts": {}, "seconds": {}}
    for key, fn in items:
        t = time.time()
        rec["counts"][key] = fn(g)
        rec["seconds"][key] = round(time.time() - t, 2)
        print(key, rec["counts"][key], rec["seconds"][key], flush=True)
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main(*sys.argv[1:])
