/*
 * gpm.h -- exact subgraph counting on one AMD Instinct MI355X (gfx950).
 *
 * Method: pattern-aware depth-first subgraph extension (Chen & Arvind,
 * "Efficient and Scalable Graph Pattern Mining on GPUs", OSDI'22 /
 * arXiv 2112.09761).  A partial match is extended one pattern vertex at a
 * time by intersecting / subtracting sorted neighbour lists under the
 * pattern's matching order and symmetry order (Sec. 2.2, "Pattern-Aware GPM
 * Algorithms"; Alg. 1), and the exact match count is reduced at the leaves.
 *
 * Conventions shared by every entry point
 *   - Functions never abort and never print.  They return GPM_OK (0) or a
 *     negative gpm_status; outputs are written only on GPM_OK.
 *     gpm_last_error() describes the last failure on a context.
 *   - A context is bound to one device and is not thread-safe: use it from
 *     one host thread at a time.
 *   - Counts are exact unsigned 64-bit integers.  The device adds partial
 *     counts modulo 2^64, so any summation order gives the same bits; no
 *     shipped workload comes near 2^64.
 *   - Graph vertices are 0..n-1 (int32 ids, so n < 2^31); adjacency offsets
 *     are int64.
 *   - Pattern vertices are 0..k-1 with 1 <= k <= 8; a pattern must be
 *     connected (vertex extension only grows connected subgraphs, Sec. 2.2).
 */
#ifndef GPM_H
#define GPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gpm_ctx gpm_ctx;
typedef int32_t gpm_status;

enum {
    GPM_OK = 0,
    GPM_E_INVAL = -1,        /* bad argument (null pointer, bad id, bad size) */
    GPM_E_CSR = -2,          /* CSR not canonical: unsorted / duplicate
                                neighbours, self loop, id out of range, or
                                asymmetric when GPM_VALIDATE asks to check */
    GPM_E_PATTERN = -3,      /* k < 1, k > 8, bad edge, disconnected pattern */
    GPM_E_NOMEM = -4,        /* device memory budget too small */
    GPM_E_DEVICE = -5,       /* a HIP runtime call failed */
    GPM_E_UNSUPPORTED = -6,  /* e.g. a non-clique pattern on a DAG-only graph */
    GPM_E_BUSY = -7,         /* no serving slot free; retry after gpm_poll */
    GPM_E_TIMEOUT = -8       /* gpm_wait timed out; the query is still live */
};

/* Induced-ness of a match (Sec. 2.1 "GPM Problems"): vertex-induced is the
 * default of the paper's API; edge-induced is subgraph listing's. */
enum { GPM_VERTEX_INDUCED = 0, GPM_EDGE_INDUCED = 1 };

/* gpm_load_csr flags */
enum {
    GPM_CSR_SYMMETRIC = 1,   /* every edge stored in both directions        */
    GPM_CSR_DAG = 2,         /* already oriented (each edge once): cliques
                                only (orientation, Sec. 4.2, graph loader)   */
    GPM_PTRS_DEVICE = 4,     /* row_ptr / col are device pointers on the
                                context's device (e.g. torch data_ptr())     */
    GPM_VALIDATE = 8         /* also check symmetry, O(m log d) on the host  */
};

#define GPM_MAX_K 8
#define GPM_MAX_PATTERN_EDGES 28

/* A pattern: k vertices, n_edges undirected edges (a_i, b_i) stored as
 * edges[2i], edges[2i+1], 0-based. */
typedef struct {
    int32_t k;
    int32_t n_edges;
    int32_t edges[2 * GPM_MAX_PATTERN_EDGES];
} gpm_pattern;

typedef struct {
    int64_t n;               /* vertices                                    */
    int64_t m;               /* undirected edges                            */
    int64_t max_degree;      /* Delta of the symmetric graph (0 if DAG-only) */
    int64_t max_out_degree;  /* Delta of the degree-oriented DAG             */
    int64_t device_bytes;    /* device memory held by this graph now         */
} gpm_graph_meta;

/* Statistics of the last gpm_count / gpm_motifs / gpm_count_batch call. */
#define GPM_MAX_LAUNCH_STATS 8

typedef struct {
    double kernel_ms;        /* sum of the call's kernel times (HIP events)  */
    double total_ms;         /* host wall time of the call                   */
    int64_t tasks;           /* root tasks (vertices / edges) issued          */
    int64_t waves;           /* persistent waves launched                    */
    int64_t chunk;           /* tasks per queue pop                          */
    int64_t elements;        /* intersected elements (only when the option
                                "count_elements" is 1; else -1)               */
    int64_t list_fetches;    /* neighbour-list reads (same option)            */
    int64_t frontier_written;/* frontier elements stored (same option)        */
    int64_t bitmap_words;    /* 64-bit AND+popcount word operations of the
                                local-graph bitmap kernel (same option)      */
    int64_t frontier_bytes;  /* device frontier buffer size                  */
    int32_t launches;        /* kernel launches of the call                   */
    int32_t variant;         /* kernel variant the autotuner chose            */
    /* per launch, in launch order (the first GPM_MAX_LAUNCH_STATS launches) */
    int32_t n_launch_stats;  /* entries filled in the arrays below           */
    int32_t reserved;
    uint32_t launch_kinds[GPM_MAX_LAUNCH_STATS];  /* job kinds of the launch as
                                a bit mask: 1<<1 clique edge kernel, 1<<2 DFS
                                plan, 1<<3 per-edge motif terms, 1<<4
                                per-vertex motif terms, 1<<5 local-graph
                                cliques (one wave per root), 1<<6 4-cycle
                                wedge aggregation (one workgroup per task;
                                its own kernel), 1<<7 local-graph cliques
                                (one workgroup per root; its own kernel),
                                1<<8 per-edge terms from triangle counters,
                                1<<9 triangle scatter                        */
    double launch_ms[GPM_MAX_LAUNCH_STATS];        /* duration (HIP events)   */
    int64_t launch_elements[GPM_MAX_LAUNCH_STATS]; /* as the totals above, per */
    int64_t launch_fetches[GPM_MAX_LAUNCH_STATS];  /* launch (-1 unless       */
    int64_t launch_written[GPM_MAX_LAUNCH_STATS];  /* "count_elements" is 1)  */
    int64_t launch_words[GPM_MAX_LAUNCH_STATS];
} gpm_stats;

/* ---------------------------------------------------------------------- */
/* context                                                                 */
/* ---------------------------------------------------------------------- */

/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t,
 * may be NULL for the null stream) is where every kernel of the context is
 * queued; the caller keeps ownership of the stream.  `hbm_budget_bytes`
 * bounds the device memory the context allocates for frontiers and task
 * lists (0 = 90% of the free memory at creation).  *out is owned by the
 * caller and released with gpm_destroy. */
gpm_status gpm_create(gpm_ctx **out, int device, void *hip_stream,
                      size_t hbm_budget_bytes);

/* Release every graph, buffer and stream of the context. Waits for pending
 * device work first.  NULL is accepted. */
gpm_status gpm_destroy(gpm_ctx *ctx);

/* Message of the last failure on ctx (static storage owned by ctx; valid
 * until the next call on ctx).  Never NULL. */
const char *gpm_last_error(const gpm_ctx *ctx);

/* Set a tuning option (for tests and the autotuner's search space):
 *   "granularity"     0 auto, 1 vertex tasks, 2 edge tasks
 *   "chunk"           tasks per queue pop (0 = auto)
 *   "waves_per_cu"    persistent waves per compute unit (0 = auto: 24 for
 *                     local-graph clique launches, 16 otherwise)
 *   "setop"           how the plan-driven DFS tests membership (Sec. 6.1):
 *                     1 binary search in global memory, 2 merge path (each
 *                     chunk of 64 candidates searches only the probed list's
 *                     range between its first and last candidate, staged in
 *                     LDS when it holds at most 256 elements; a lane's own
 *                     leaf walks each list once by galloping), 3 binary
 *                     search with the top 5 levels (31 pivots) of each probed
 *                     list's search tree in LDS; 0 = the default, 3
 *                     (identical counts in every mode)
 *   "clique_lds"      1 = clique kernel keeps frontiers in LDS (default),
 *                     0 = force the generic kernel with HBM frontiers
 *   "rename"          non-clique patterns run on a copy relabelled by
 *                     ascending (degree, id) (1, default) or on the ids as
 *                     given (0); counts are identical either way
 *   "clique_algo"     0 auto (local-graph bitmaps for cliques up to 5
 *                     vertices), 1 sorted-list edge kernel, 2 bitmaps
 *   "lgs_tile"        local graphs up to this many vertices stay in one
 *                     wave's LDS (64..256, default 128)
 *   "lgs_block"       1 (default) = larger local graphs that fit a
 *                     workgroup's LDS (up to 896 vertices with 160 KB, fewer when the
 *                     device's per-workgroup LDS is smaller) are searched by
 *                     a whole workgroup each; 0 = by one wave, rows in HBM
 *   "lgs_lanes"       local-graph row build: lanes that scan one row's
 *                     out-list together (4, 8, 16, 32 or 64 = a whole wave);
 *                     fewer lanes put more rows in flight per wave
 *   "lgs_max"         roots with more out-neighbours (64..2048) use the
 *                     edge kernel
 *   "lgs_split"       1 = split the heaviest roots (5-cliques per wave,
 *                     4- and 5-cliques per workgroup) into sub-tasks
 *   "leaf_cap"        generic DFS: last-level candidates whose leaf set is
 *                     at most this long are counted one per lane (0 = off)
 *   "cycle4_algo"     edge-induced 4-cycles: 0/2 wedge aggregation in LDS
 *                     (one workgroup per task), 1 the DFS plan (identical
 *                     counts)
 *   "cycle4_mode"     wedge aggregation tasks: 0 (default) a cost model picks
 *                     per root between direct id windows and hash tasks, 1
 *                     hash tasks only, 2 direct windows for every root with
 *                     more than "cycle4_batch" wedges (identical counts)
 *   "cycle4_batch"    wedges per 4-cycle hash task (2..2^30, default 8192);
 *                     a task whose distinct endpoints overflow the LDS table
 *                     splits on the device (identical counts)
 *   "decompose"       counting-only pruning (Sec. 5.4 (1)), 1 (default):
 *                     wedge, 3-star, 4-path, tailed-triangle and diamond
 *                     counts (both modes) come from per-vertex and per-edge
 *                     terms (plus the 4-clique, triangle or 4-cycle count
 *                     their induced forms need); any other edge-induced
 *                     count whose pattern has r >= 2 pairwise non-adjacent
 *                     twin vertices (same neighbours) beside a connected
 *                     rest of >= 2 vertices walks only the rest and adds
 *                     ext * C(n, r) per match of it (n: the twins' common
 *                     candidate set, ext: the twins' orderings its symmetry
 *                     restrictions allow); 0 = the plain DFS plan (identical
 *                     counts)
 *   "edge_terms"      per-edge motif terms (4-motifs, decomposed counts):
 *                     0 (default) = the k = 3 local-graph search adds each
 *                     triangle to its three edges' counters, then one pass
 *                     over the edges; 1 = one list intersection per edge
 *                     (identical counts)
 *   "budget"          device memory budget in bytes (as in gpm_create)
 *   "max_batch", "serve_slots", "max_pending", "serve_light_ms"   serving
 *                     limits (see gpm_submit)
 *   "tune_min_ms"     autotuner threshold (see "autotune")
 *   "count_elements"  1 = instrumented kernels count intersected elements
 *                     (slower; never used for timing)
 *   "autotune"        1 = on the first gpm_count of a (graph, pattern, mode)
 *                     that takes at least "tune_min_ms" (default 20), try the
 *                     knob values of its search space (LDS tile, waves per
 *                     CU, chunk, leaf mode, set-op mode, granularity,
 *                     renaming, row-build lanes) by
 *                     coordinate descent -- every trial must return the same
 *                     count, else GPM_E_DEVICE -- and reuse the fastest
 *                     values on later calls of that triple
 * Unknown keys give GPM_E_INVAL. */
gpm_status gpm_set_option(gpm_ctx *ctx, const char *key, int64_t value);

gpm_status gpm_get_stats(const gpm_ctx *ctx, gpm_stats *out);

/* ---------------------------------------------------------------------- */
/* graphs (graph loader and preprocessor, Sec. 4.2)                        */
/* ---------------------------------------------------------------------- */

/* Load a data graph in CSR form: row_ptr[n+1] (int64, row_ptr[0] = 0,
 * row_ptr[n] = nnz), col[nnz] (int32).  Lists must be sorted ascending with
 * no self loops and no duplicates (Table 3's data graphs are symmetric with
 * no loops or duplicate edges).  With GPM_CSR_SYMMETRIC the graph is the
 * undirected graph (nnz = 2m); with GPM_CSR_DAG it is an orientation (each
 * edge once) usable for cliques only.  The arrays are copied (host or, with
 * GPM_PTRS_DEVICE, device pointers); the caller keeps ownership.  The graph
 * stays resident until gpm_unload / gpm_destroy.  Preparation (validation,
 * degree orientation, task lists) runs here or lazily on first use and is
 * never part of a count's timing, as in the paper's evaluation.
 * Errors: GPM_E_INVAL (n < 0, nnz < 0, null), GPM_E_CSR, GPM_E_NOMEM. */
gpm_status gpm_load_csr(gpm_ctx *ctx, int64_t n, int64_t nnz,
                        const int64_t *row_ptr, const int32_t *col,
                        uint32_t flags, int32_t *graph_id_out);

/* The checks of gpm_load_csr on host arrays, without a context or device:
 * GPM_OK, GPM_E_INVAL (bad sizes / null / conflicting or device flags) or
 * GPM_E_CSR (not canonical; with GPM_VALIDATE also asymmetric, or a DAG with
 * both directions of an edge or a cycle). */
gpm_status gpm_validate_csr(int64_t n, int64_t nnz, const int64_t *row_ptr,
                            const int32_t *col, uint32_t flags);

/* Run every preparation step now (relabelling by degree, orientation, root
 * task lists) instead of lazily at the first count that needs it, e.g. for
 * a serving pool whose queries must not pay for preparation. */
gpm_status gpm_prepare(gpm_ctx *ctx, int32_t graph_id);

gpm_status gpm_unload(gpm_ctx *ctx, int32_t graph_id);

gpm_status gpm_graph_info(gpm_ctx *ctx, int32_t graph_id, gpm_graph_meta *out);

/* ---------------------------------------------------------------------- */
/* patterns (the paper's generateClique / Pattern(file) API, Sec. 4)       */
/* ---------------------------------------------------------------------- */

gpm_status gpm_pattern_clique(int k, gpm_pattern *out);

/* Built-in shapes: "edge", "wedge", "triangle", "path4", "star3", "cycle4",
 * "tailed_triangle", "diamond", "clique4", "clique5" (the 3- and 4-vertex
 * motifs of Sec. 2.1 plus cliques).  GPM_E_INVAL for an unknown name. */
gpm_status gpm_pattern_named(const char *name, gpm_pattern *out);

/* Build a pattern from an edge list of n_edges pairs; validates it. */
gpm_status gpm_pattern_from_edges(int k, int n_edges, const int32_t *edges,
                                  gpm_pattern *out);

/* The search plan the library uses for a pattern (the paper's pattern
 * analyzer, Sec. 4): matching order, symmetry order and buffer count.  Host
 * only; needs no device.  For a clique the plan is the one used on the
 * degree-oriented DAG (no restrictions: orientation breaks every symmetry). */
typedef struct {
    int32_t k;
    int32_t clique;              /* 1: runs on the oriented DAG              */
    int32_t aut;                 /* |Aut(P)|                                 */
    int32_t root_bound;          /* 1: root edges keep one direction (v1<v0),
                                    the edge-list halving of Sec. 7.2 (2)    */
    int32_t n_buffers;           /* stored frontier levels X (X <= k-3)      */
    int32_t n_restrictions;
    int32_t order[GPM_MAX_K];    /* pattern vertex matched at depth d        */
    int32_t restrictions[2 * GPM_MAX_PATTERN_EDGES];  /* pairs (a, b):
                                    v_a > v_b, pattern vertex ids            */
    int32_t count_only_r;        /* counting-only pruning of the count plan
                                    (option "decompose", Sec. 5.4 (1)): the
                                    last r pattern vertices of the order are
                                    twins counted as C(n, r) at one leaf (0:
                                    none; edge-induced non-cliques only)     */
} gpm_plan_info;

gpm_status gpm_plan(const gpm_pattern *pattern, int mode, gpm_plan_info *out);

/* Adaptive buffering (Sec. 7.2 (3)): waves = min(Y / (X * B * 4 bytes),
 * tasks, max_resident), at least 1 when X * B * 4 <= Y.  Y = free bytes,
 * X = stored levels, B = capacity (elements) per level.  Host only.
 * GPM_E_NOMEM when not even one wave fits. */
gpm_status gpm_frontier_waves(int64_t free_bytes, int32_t x_levels,
                              int64_t cap_elems, int64_t n_tasks,
                              int64_t max_resident, int64_t *waves_out);

/* ---------------------------------------------------------------------- */
/* counting                                                                */
/* ---------------------------------------------------------------------- */

/* Exact number of distinct matches of `pattern` in graph `graph_id`
 * (each subgraph once: completeness and uniqueness, Sec. 2.1), vertex- or
 * edge-induced (`mode`).  Cliques run on the degree-oriented DAG (Sec. 4.2,
 * orientation); other patterns on the symmetric graph with the symmetry
 * order of Sec. 2.2.  k = 1 returns n, k = 2 returns m, n < k returns 0.
 * Blocks until the count is on the host (the context's stream is
 * synchronised).  Errors: GPM_E_PATTERN, GPM_E_UNSUPPORTED, GPM_E_NOMEM,
 * GPM_E_DEVICE. */
gpm_status gpm_count(gpm_ctx *ctx, int32_t graph_id, const gpm_pattern *pattern,
                     int mode, uint64_t *count_out);

/* gpm_count without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, semantics and errors as gpm_count; the
 * call allocates no device or pinned host memory (no hipMalloc, hipFree or
 * hipHostMalloc): the job table, queue counters, result slots and frontier /
 * counter buffers of the call live in a device scratch array of 64 MiB that
 * the library holds per GPU until the process ends (its address is looked up
 * once per device at gpm_create), and the host staging was reserved at
 * gpm_create.  Requirements and limits:
 *   - the graph must already hold what the query needs (orientation,
 *     relabelling, root lists): run gpm_count with the same pattern and mode
 *     once first (or gpm_prepare where it covers it); else GPM_E_UNSUPPORTED
 *     and nothing is built;
 *   - frontier sizing works within the scratch (fewer waves when buffers are
 *     large); a query whose buffers for one workgroup's waves, or whose job
 *     tables, exceed it fails with GPM_E_NOMEM;
 *   - every call on a GPU uses that GPU's one scratch array: calls that
 *     overlap on one GPU (two contexts of the device, or several host
 *     threads) race and give wrong counts.  Sequential calls are safe: the
 *     call returns after its results are on the host, and it clears every
 *     buffer that must start at zero. */
gpm_status gpm_count_noalloc(gpm_ctx *ctx, int32_t graph_id,
                             const gpm_pattern *pattern, int mode,
                             uint64_t *count_out);

/* Vertex-induced counts of every connected k-vertex pattern (k-motif
 * counting, Sec. 2.1), k = 3 or 4, written to counts_out[len]:
 *   k = 3 (len >= 2): [wedge, triangle]
 *   k = 4 (len >= 6): [path4, star3, cycle4, tailed_triangle, diamond, clique4]
 * Triangle-sharing patterns are computed in one fused kernel and the
 * 4-cycle separately (multi-pattern kernel fission, Sec. 5.3); the star and
 * path terms come from degree sums (counting-only pruning, Sec. 5.4 (1)). */
gpm_status gpm_motifs(gpm_ctx *ctx, int32_t graph_id, int k,
                      uint64_t *counts_out, size_t len);

/* ---------------------------------------------------------------------- */
/* listing                                                                 */
/* ---------------------------------------------------------------------- */

/* Subgraph listing (Sec. 2.1: listing enumerates every match, where
 * counting only reports how many there are; the list() call of the paper's
 * interface, Sec. 4).  Each distinct match of `pattern` in graph `graph_id`
 * is written once, as a row of k int32 vertex ids in the caller's
 * numbering: out[r*k + j] is the graph vertex matched to pattern vertex j.
 * `out` is device memory on the context's device with room for `cap` rows
 * (cap * k int32, caller-owned); it may be NULL when cap == 0.
 * *count_out (host) receives the total number of matches, which equals
 * gpm_count's.  Overflow: when *count_out > cap only cap rows were written
 * (which ones is unspecified), and the caller can retry with a larger
 * buffer.  Row order is unspecified.  Each row is one representative
 * embedding of its subgraph: no two rows share a vertex set (cliques,
 * vertex-induced mode) or an edge set (edge-induced mode).  Every pattern
 * runs the plan-driven walk, never a counting-only shortcut: cliques on the
 * degree-oriented DAG, other patterns on the symmetric graph.  Blocks until
 * the rows and the count are complete.  Errors: GPM_E_INVAL (unknown graph,
 * cap < 0, out NULL with cap > 0, bad mode), GPM_E_PATTERN,
 * GPM_E_UNSUPPORTED (non-clique pattern on a DAG-only graph), GPM_E_NOMEM
 * (frontier buffers), GPM_E_DEVICE; on error nothing is reported in
 * *count_out and the contents of out are unspecified. */
gpm_status gpm_list(gpm_ctx *ctx, int32_t graph_id, const gpm_pattern *pattern,
                    int mode, int32_t *out, int64_t cap, uint64_t *count_out);

/* ---------------------------------------------------------------------- */
/* batched and served execution                                            */
/* ---------------------------------------------------------------------- */

enum { GPM_QUERY_COUNT = 0, GPM_QUERY_MOTIFS = 1 };

typedef struct {
    int32_t graph_id;
    int32_t kind;            /* GPM_QUERY_COUNT or GPM_QUERY_MOTIFS          */
    int32_t mode_or_k;       /* COUNT: GPM_*_INDUCED; MOTIFS: 3 or 4          */
    int32_t reserved;
    gpm_pattern pattern;     /* COUNT only                                   */
} gpm_query;

/* Run nq queries in ONE persistent launch whose waves steal chunks of root
 * tasks from every query through a device-wide queue; outs[6*i ..] receives
 * query i's result (1 value for COUNT, 2 or 6 for MOTIFS; the rest zero).
 * outs is a host array of 6*nq uint64 owned by the caller. */
gpm_status gpm_count_batch(gpm_ctx *ctx, int32_t nq, const gpm_query *queries,
                           uint64_t *outs);

/* Serving: submit one query without blocking.  The query is checked here
 * (graph id, kind, mode, pattern, and a pattern the graph can run) and gets
 * no ticket when a check fails: GPM_E_INVAL, GPM_E_PATTERN or
 * GPM_E_UNSUPPORTED, as gpm_count would return; GPM_E_BUSY when the pending
 * list is full ("max_pending").  An accepted query is admitted when a launch
 * slot is free and its frontier memory fits what the running launches leave
 * of the budget (adaptive buffering, Sec. 7.2 (3)); queries are admitted in
 * arrival order, and one that does not fit beside the running launches
 * waits, first in line, until they finish.  Launches on different slots
 * overlap on the device.  Queries whose last run alone took at most
 * "serve_light_ms" (default 50) are light: light queries admitted together
 * share one persistent launch (at most "max_batch").  Other queries (heavy,
 * or not yet measured) run alone and hold at most half of the slots, so
 * light queries keep slots of their own.  *ticket_out identifies the query
 * for gpm_poll / gpm_wait until its result is collected. */
gpm_status gpm_submit(gpm_ctx *ctx, const gpm_query *query, int64_t *ticket_out);

/* Progress the serving loop and look at one ticket.  *done_out = 0: the query
 * is still pending or running (return GPM_OK), or the call itself failed
 * (GPM_E_INVAL for a ticket that was never issued or was already collected;
 * GPM_E_DEVICE).  *done_out = 1: the query completed and the ticket is
 * released; the return value is the query's own status -- GPM_OK with
 * counts_out[6] (host, caller-owned; 1 value for COUNT, 2 or 6 for MOTIFS,
 * the rest zero) written, or the error that stopped it (GPM_E_NOMEM when its
 * buffers do not fit the whole memory budget, GPM_E_DEVICE, ...; counts_out
 * untouched, gpm_last_error() describes it). */
gpm_status gpm_poll(gpm_ctx *ctx, int64_t ticket, int *done_out,
                    uint64_t *counts_out);

/* Block until the ticket completes, then return as gpm_poll does for a
 * completed ticket; GPM_E_TIMEOUT (query still live) once timeout_ns passes
 * (timeout_ns < 0: no limit); GPM_E_INVAL at once for an unknown ticket. */
gpm_status gpm_wait(gpm_ctx *ctx, int64_t ticket, int64_t timeout_ns,
                    uint64_t *counts_out);

/* Number of queries submitted but not yet collected. */
gpm_status gpm_inflight(gpm_ctx *ctx, int64_t *count_out);

/* State of the serving loop (admission by frontier memory, Sec. 7.2 (3)),
 * for monitoring and tests.  The call only reads: it does not progress the
 * loop, so a launch that has finished on the device is counted as running
 * until the next gpm_submit / gpm_poll / gpm_wait. */
typedef struct {
    int64_t pending;          /* accepted queries not yet admitted            */
    int64_t running;          /* queries in launches on the device            */
    int64_t completed;        /* completed queries whose result is not yet
                                 collected                                    */
    int64_t busy_slots;       /* launch slots with a launch in flight         */
    int64_t frontier_in_use;  /* bytes of frontier and counter buffers the
                                 running launches hold                        */
    int64_t budget;           /* the context's memory budget (bytes)          */
    int64_t memory_waits;     /* queries that had to wait, first in line, for
                                 running launches to free memory (since
                                 gpm_create)                                  */
    int64_t admitted;         /* queries admitted into launches (since
                                 gpm_create)                                  */
} gpm_serve_info;

gpm_status gpm_serve_state(gpm_ctx *ctx, gpm_serve_info *out);

#ifdef __cplusplus
}
#endif

#endif /* GPM_H */
