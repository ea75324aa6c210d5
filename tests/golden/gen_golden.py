"""Write stored oracle counts for the large synthetic workloads.

Calls only the CPU oracle (oracle/) on graphs from the seeded generators;
each record carries the sha256 of the generated CSR so a test can confirm
it regenerated the same graph.  Run:  python tests/golden/gen_golden.py NAME
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


def main(name):
    if name == "batch256":
        return batch_golden()
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
    main(sys.argv[1])
