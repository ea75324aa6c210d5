/*
 * oracle.c -- CPU oracle for exact subgraph counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library: it is an independent, plain, slow
 * and obviously correct statement of what the counting method computes.
 *
 * What is counted (paper, Sec. 2.1 "GPM Problems"):
 *   G = (V, E) simple undirected; P a connected pattern on k vertices.
 *   - a vertex-induced match is a k-subset W of V with G[W] isomorphic to P;
 *   - an edge-induced match is a subgraph (W, F), F subset of E, W the
 *     endpoints of F, isomorphic to P.
 *   Completeness and uniqueness (same section) mean every distinct match is
 *   counted exactly once, so a count is a number of distinct subgraphs, i.e.
 *   (number of embeddings) / |Aut(P)|.
 *
 * Routes (each a different road to the same number):
 *   orc_count_subsets   the definition itself: every k-subset, every edge
 *                       subset, isomorphism by all k! bijections (tiny n);
 *   orc_count_embed     injective homomorphisms (plus non-edge preservation
 *                       in induced mode) divided by |Aut(P)|;
 *   orc_list_embed      listing: the same embeddings, one emitted per
 *                       distinct subgraph (the smallest of its automorphic
 *                       images);
 *   orc_triangles       triangles with marker arrays on an oriented graph,
 *                       also per-vertex and per-edge triangle counts;
 *   orc_cliques         k-cliques by recursive marker-array enumeration on
 *                       an oriented graph (orientation: paper Sec. 4.2,
 *                       "Graph Loader and Preprocessor");
 *   orc_cycle4          4-cycles by codegree (wedge-pair) counting;
 *   orc_cycle4_trace    4-cycles from tr(A^4), the closed 4-walks, with the
 *                       edge-retracing walks removed (no ranking at all);
 *   orc_nonind4         the six non-induced 4-vertex counts from local
 *                       triangle and degree terms (the counting-only
 *                       decomposition of Sec. 5.4 (1), Alg. 3, for diamond);
 *   orc_motifs3/4       induced (vertex-induced) motif counts (Sec. 2.1, k-MC)
 *                       from the non-induced ones by the unitriangular
 *                       inclusion relation between 4-vertex graphs.
 *
 * All accumulation is in unsigned __int128 and every result is checked to fit
 * in 64 bits (ORC_EOVERFLOW otherwise).
 *
 * Parity pins: every function here is pinned by the CPU tests against
 * closed forms (K_n, K_{m,n}, multipartite, paths, cycles, stars, grids,
 * hypercubes), dense trace formulas, networkx, and against one another.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EOVERFLOW -2
#define ORC_ENOMEM -3

typedef unsigned __int128 u128;

#define MAXK 8
#define MAXT 512

static int fits64(u128 x) { return (x >> 64) == 0; }

/* ------------------------------------------------------------------ */
/* adjacency test on a sorted neighbour list (binary search)           */
/* ------------------------------------------------------------------ */
static int has_edge(const int64_t *rp, const int32_t *col, int64_t u, int64_t v)
{
    int64_t lo = rp[u], hi = rp[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < rp[u + 1] && col[lo] == v;
}

/* ------------------------------------------------------------------ */
/* pattern helpers                                                      */
/* ------------------------------------------------------------------ */
static int pattern_matrix(int k, const int32_t *pe, int npe, int adj[MAXK][MAXK])
{
    if (k < 1 || k > MAXK || npe < 0) return ORC_EINVAL;
    memset(adj, 0, sizeof(int) * MAXK * MAXK);
    for (int i = 0; i < npe; i++) {
        int a = pe[2 * i], b = pe[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b) return ORC_EINVAL;
        adj[a][b] = adj[b][a] = 1;
    }
    /* connectivity (vertex extension grows connected subgraphs, Sec. 2.2) */
    int seen[MAXK] = {0}, stack[MAXK], top = 0;
    seen[0] = 1; stack[top++] = 0;
    while (top) {
        int x = stack[--top];
        for (int y = 0; y < k; y++)
            if (adj[x][y] && !seen[y]) { seen[y] = 1; stack[top++] = y; }
    }
    for (int i = 0; i < k; i++) if (!seen[i]) return ORC_EINVAL;
    return ORC_OK;
}

/* next permutation in lexicographic order; returns 0 after the last one */
static int next_perm(int *p, int k)
{
    int i = k - 2;
    while (i >= 0 && p[i] > p[i + 1]) i--;
    if (i < 0) return 0;
    int j = k - 1;
    while (p[j] < p[i]) j--;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int a = i + 1, b = k - 1; a < b; a++, b--) { t = p[a]; p[a] = p[b]; p[b] = t; }
    return 1;
}

/* does the permutation p of the pattern vertices preserve adjacency? */
static int is_automorphism(int k, int adj[MAXK][MAXK], const int *p)
{
    int ok = 1;
    for (int i = 0; i < k && ok; i++)
        for (int j = 0; j < k; j++)
            if (adj[i][j] != adj[p[i]][p[j]]) { ok = 0; break; }
    return ok;
}

/* |Aut(P)|: permutations of the pattern vertices preserving adjacency. */
int orc_pattern_aut(int k, const int32_t *pe, int npe, uint64_t *aut_out)
{
    int adj[MAXK][MAXK];
    int st = pattern_matrix(k, pe, npe, adj);
    if (st) return st;
    int p[MAXK];
    for (int i = 0; i < k; i++) p[i] = i;
    uint64_t cnt = 0;
    do {
        cnt += is_automorphism(k, adj, p);
    } while (next_perm(p, k));
    *aut_out = cnt;
    return ORC_OK;
}

/* is the k-vertex graph with matrix h isomorphic to the pattern matrix? */
static int iso_to_pattern(int k, int h[MAXK][MAXK], int adj[MAXK][MAXK])
{
    int p[MAXK];
    for (int i = 0; i < k; i++) p[i] = i;
    do {
        int ok = 1;
        for (int i = 0; i < k && ok; i++)
            for (int j = i + 1; j < k; j++)
                if (adj[i][j] != h[p[i]][p[j]]) { ok = 0; break; }
        if (ok) return 1;
    } while (next_perm(p, k));
    return 0;
}

/* ------------------------------------------------------------------ */
/* O1: the definition, literally, for tiny graphs                       */
/* ------------------------------------------------------------------ */
/*
 * Vertex-induced: every k-subset W, test G[W] ~ P.
 * Edge-induced: every k-subset W, every subset F of the edges of G[W] with
 * |F| = |E(P)| whose endpoints are all of W, test (W, F) ~ P.
 * (A single-vertex pattern counts the vertices in both modes.)
 */
int orc_count_subsets(int64_t n, const int64_t *rp, const int32_t *col,
                      int k, const int32_t *pe, int npe, int induced,
                      uint64_t *out)
{
    int adj[MAXK][MAXK];
    int st = pattern_matrix(k, pe, npe, adj);
    if (st) return st;
    if (n < 0 || n > 64) return ORC_EINVAL;
    if (k == 1) { *out = (uint64_t)n; return ORC_OK; }
    if (n < k) { *out = 0; return ORC_OK; }
    u128 total = 0;
    int w[MAXK];
    for (int i = 0; i < k; i++) w[i] = i;
    for (;;) {
        int h[MAXK][MAXK];
        int eu[MAXK * MAXK], ev[MAXK * MAXK], ne = 0;
        memset(h, 0, sizeof h);
        for (int i = 0; i < k; i++)
            for (int j = i + 1; j < k; j++)
                if (has_edge(rp, col, w[i], w[j])) {
                    h[i][j] = h[j][i] = 1;
                    eu[ne] = i; ev[ne] = j; ne++;
                }
        if (induced) {
            total += (u128)iso_to_pattern(k, h, adj);
        } else if (ne >= npe && ne <= 30) {
            for (uint32_t mask = 0; mask < (1u << ne); mask++) {
                if (__builtin_popcount(mask) != npe) continue;
                int f[MAXK][MAXK], covered[MAXK] = {0};
                memset(f, 0, sizeof f);
                for (int e = 0; e < ne; e++)
                    if (mask >> e & 1) {
                        f[eu[e]][ev[e]] = f[ev[e]][eu[e]] = 1;
                        covered[eu[e]] = covered[ev[e]] = 1;
                    }
                int all = 1;
                for (int i = 0; i < k; i++) all &= covered[i];
                if (all) total += (u128)iso_to_pattern(k, f, adj);
            }
        }
        /* next k-subset of [0, n) in lexicographic order */
        int i = k - 1;
        while (i >= 0 && w[i] == n - k + i) i--;
        if (i < 0) break;
        w[i]++;
        for (int j = i + 1; j < k; j++) w[j] = w[j - 1] + 1;
    }
    if (!fits64(total)) return ORC_EOVERFLOW;
    *out = (uint64_t)total;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O1b: embeddings / |Aut(P)|, any connected pattern, moderate graphs   */
/* ------------------------------------------------------------------ */
typedef struct {
    int k, induced;
    int order[MAXK];          /* pattern vertex matched at each depth      */
    int parent[MAXK];         /* an earlier depth adjacent in the pattern  */
    int padj[MAXK][MAXK];     /* pattern adjacency, indexed by depth       */
    const int64_t *rp;
    const int32_t *col;
} embed_plan;

static u128 embed_rec(const embed_plan *pl, int depth, int64_t *img)
{
    if (depth == pl->k) return 1;
    u128 s = 0;
    int64_t p = img[pl->parent[depth]];
    for (int64_t e = pl->rp[p]; e < pl->rp[p + 1]; e++) {
        int64_t x = pl->col[e];
        int ok = 1;
        for (int d = 0; d < depth && ok; d++) {
            if (img[d] == x) { ok = 0; break; }
            int adjp = pl->padj[depth][d];
            if (adjp) { if (!has_edge(pl->rp, pl->col, x, img[d])) ok = 0; }
            else if (pl->induced) { if (has_edge(pl->rp, pl->col, x, img[d])) ok = 0; }
        }
        if (!ok) continue;
        img[depth] = x;
        s += embed_rec(pl, depth + 1, img);
    }
    return s;
}

int orc_count_embed(int64_t n, const int64_t *rp, const int32_t *col,
                    int k, const int32_t *pe, int npe, int induced,
                    uint64_t *out)
{
    int adj[MAXK][MAXK];
    int st = pattern_matrix(k, pe, npe, adj);
    if (st) return st;
    if (k == 1) { *out = (uint64_t)n; return ORC_OK; }
    uint64_t aut;
    orc_pattern_aut(k, pe, npe, &aut);

    embed_plan pl;
    pl.k = k; pl.induced = induced; pl.rp = rp; pl.col = col;
    /* breadth-first order from pattern vertex 0: every depth > 0 has an
     * earlier neighbour to draw candidates from */
    int seen[MAXK] = {0}, depth_of[MAXK], head = 0, tail = 0;
    pl.order[tail++] = 0; seen[0] = 1;
    while (head < tail) {
        int x = pl.order[head++];
        for (int y = 0; y < k; y++)
            if (adj[x][y] && !seen[y]) { seen[y] = 1; pl.order[tail++] = y; }
    }
    for (int d = 0; d < k; d++) depth_of[pl.order[d]] = d;
    for (int d = 0; d < k; d++)
        for (int e = 0; e < k; e++)
            pl.padj[d][e] = adj[pl.order[d]][pl.order[e]];
    pl.parent[0] = -1;
    for (int d = 1; d < k; d++) {
        pl.parent[d] = -1;
        for (int e = 0; e < d; e++)
            if (pl.padj[d][e]) { pl.parent[d] = e; break; }
    }
    (void)depth_of;

    static u128 acc[MAXT];
    int nt = omp_get_max_threads();
    if (nt > MAXT) nt = MAXT;
    memset(acc, 0, sizeof acc);
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        int64_t img[MAXK];
        u128 local = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; v++) {
            img[0] = v;
            local += embed_rec(&pl, 1, img);
        }
        acc[t] = local;
    }
    u128 total = 0;
    for (int t = 0; t < nt; t++) total += acc[t];
    if (total % aut) return ORC_EINVAL;   /* cannot happen for a valid count */
    total /= aut;
    if (!fits64(total)) return ORC_EOVERFLOW;
    *out = (uint64_t)total;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O1c: listing (Sec. 2.1: listing enumerates every match), serial.     */
/* Every embedding is enumerated as in O1b; of the |Aut(P)| embeddings  */
/* of one subgraph exactly one is emitted: the one whose tuple of       */
/* images (indexed by pattern vertex) is lexicographically smallest     */
/* among its compositions with the automorphisms.                       */
/* ------------------------------------------------------------------ */
typedef struct {
    embed_plan pl;
    int n_aut;
    int aut[40320][MAXK];     /* all automorphisms (k! <= 40320)           */
    int32_t *out;
    int64_t cap;
    u128 found;
} list_ctx;

/* is the match t (t[i] = image of pattern vertex i) the smallest of its
 * automorphic images t o s? */
static int smallest_image(const list_ctx *c, const int64_t *t)
{
    int k = c->pl.k;
    for (int a = 0; a < c->n_aut; a++) {
        const int *s = c->aut[a];
        for (int i = 0; i < k; i++) {
            if (t[s[i]] < t[i]) return 0;   /* t o s precedes t */
            if (t[s[i]] > t[i]) break;
        }
    }
    return 1;
}

static void list_rec(list_ctx *c, int depth, int64_t *img)
{
    const embed_plan *pl = &c->pl;
    int k = pl->k;
    if (depth == k) {
        int64_t t[MAXK];
        for (int d = 0; d < k; d++) t[pl->order[d]] = img[d];
        if (!smallest_image(c, t)) return;
        if ((u128)c->cap > c->found)
            for (int i = 0; i < k; i++) c->out[(int64_t)c->found * k + i] = (int32_t)t[i];
        c->found++;
        return;
    }
    int64_t p = img[pl->parent[depth]];
    for (int64_t e = pl->rp[p]; e < pl->rp[p + 1]; e++) {
        int64_t x = pl->col[e];
        int good = 1;
        for (int d = 0; d < depth && good; d++) {
            if (x == img[d]) good = 0;                       /* injective */
            else if (pl->padj[depth][d]) good = has_edge(pl->rp, pl->col, x, img[d]);
            else if (pl->induced) good = !has_edge(pl->rp, pl->col, x, img[d]);
        }
        if (!good) continue;
        img[depth] = x;
        list_rec(c, depth + 1, img);
    }
}

/* Rows out[cap][k] (row r: the graph vertex of each pattern vertex) and the
 * total number of matches in *count_out; rows past cap are counted only. */
int orc_list_embed(int64_t n, const int64_t *rp, const int32_t *col,
                   int k, const int32_t *pe, int npe, int induced,
                   int32_t *out, int64_t cap, uint64_t *count_out)
{
    int adj[MAXK][MAXK];
    int st = pattern_matrix(k, pe, npe, adj);
    if (st) return st;
    if (cap < 0 || (cap > 0 && !out)) return ORC_EINVAL;
    list_ctx *c = (list_ctx *)calloc(1, sizeof(list_ctx));
    if (!c) return ORC_ENOMEM;
    c->out = out;
    c->cap = cap;
    int p[MAXK];
    for (int i = 0; i < k; i++) p[i] = i;
    do {
        if (is_automorphism(k, adj, p)) memcpy(c->aut[c->n_aut++], p, sizeof p);
    } while (next_perm(p, k));

    embed_plan *pl = &c->pl;
    pl->k = k; pl->induced = induced; pl->rp = rp; pl->col = col;
    /* breadth-first order from pattern vertex 0, as in O1b */
    int seen[MAXK] = {0}, head = 0, tail = 0;
    pl->order[tail++] = 0; seen[0] = 1;
    while (head < tail) {
        int x = pl->order[head++];
        for (int y = 0; y < k; y++)
            if (adj[x][y] && !seen[y]) { seen[y] = 1; pl->order[tail++] = y; }
    }
    for (int d = 0; d < k; d++)
        for (int e = 0; e < k; e++)
            pl->padj[d][e] = adj[pl->order[d]][pl->order[e]];
    pl->parent[0] = -1;
    for (int d = 1; d < k; d++) {
        pl->parent[d] = -1;
        for (int e = 0; e < d; e++)
            if (pl->padj[d][e]) { pl->parent[d] = e; break; }
    }
    int64_t img[MAXK];
    for (int64_t v = 0; v < n; v++) {
        img[0] = v;
        list_rec(c, 1, img);
    }
    u128 found = c->found;
    free(c);
    if (!fits64(found)) return ORC_EOVERFLOW;
    *count_out = (uint64_t)found;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* orientation (paper Sec. 4.2, "Graph Loader and Preprocessor"):       */
/* keep u->v when u precedes v; by id (order 0) or by (degree, id)     */
/* (order 1).  The oriented lists keep the ascending id order.          */
/* ------------------------------------------------------------------ */
static int precedes(const int64_t *rp, int order, int64_t u, int64_t v)
{
    if (order == 0) return u < v;
    int64_t du = rp[u + 1] - rp[u], dv = rp[v + 1] - rp[v];
    return du < dv || (du == dv && u < v);
}

static int orient(int64_t n, const int64_t *rp, const int32_t *col, int order,
                  int64_t **orp_out, int32_t **ocol_out)
{
    int64_t *orp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!orp) return ORC_ENOMEM;
    orp[0] = 0;
    for (int64_t u = 0; u < n; u++) {
        int64_t c = 0;
        for (int64_t e = rp[u]; e < rp[u + 1]; e++)
            c += precedes(rp, order, u, col[e]);
        orp[u + 1] = orp[u] + c;
    }
    int32_t *ocol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(orp[n] + 1));
    if (!ocol) { free(orp); return ORC_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t u = 0; u < n; u++) {
        int64_t o = orp[u];
        for (int64_t e = rp[u]; e < rp[u + 1]; e++)
            if (precedes(rp, order, u, col[e])) ocol[o++] = col[e];
    }
    *orp_out = orp; *ocol_out = ocol;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O2: triangles with marker arrays                                     */
/* ------------------------------------------------------------------ */
/*
 * Each triangle {a, b, c} is found once, at its first vertex a in the
 * orientation order: a->b and a->c and b->c.  The per-vertex counts t_v
 * (triangles containing v) and per-edge counts t_e (triangles containing
 * the undirected edge; written for both directed copies of the edge, at
 * its CSR positions) are filled when the arrays are given.
 */
int orc_triangles(int64_t n, const int64_t *rp, const int32_t *col, int order,
                  uint64_t *total_out, uint64_t *t_v, uint64_t *t_e)
{
    int64_t *orp; int32_t *ocol;
    int st = orient(n, rp, col, order, &orp, &ocol);
    if (st) return st;
    int64_t om = orp[n];
    uint32_t *tdag = NULL;
    if (t_e) {
        tdag = (uint32_t *)calloc((size_t)om + 1, sizeof(uint32_t));
        if (!tdag) { free(orp); free(ocol); return ORC_ENOMEM; }
    }
    if (t_v) memset(t_v, 0, sizeof(uint64_t) * (size_t)n);
    static u128 acc[MAXT];
    int nt = omp_get_max_threads();
    if (nt > MAXT) nt = MAXT;
    memset(acc, 0, sizeof acc);
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        /* marker[x] = 1 + DAG position of a->x while a is the current root */
        int64_t *marker = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        u128 local = 0;
        if (!marker) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < n; a++) {
            if (!marker) continue;
            for (int64_t p = orp[a]; p < orp[a + 1]; p++) marker[ocol[p]] = p + 1;
            for (int64_t p = orp[a]; p < orp[a + 1]; p++) {
                int64_t b = ocol[p];
                for (int64_t q = orp[b]; q < orp[b + 1]; q++) {
                    int64_t c = ocol[q];
                    int64_t r = marker[c];
                    if (!r) continue;
                    local++;
                    if (t_v) {
#pragma omp atomic
                        t_v[a]++;
#pragma omp atomic
                        t_v[b]++;
#pragma omp atomic
                        t_v[c]++;
                    }
                    if (tdag) {
#pragma omp atomic
                        tdag[p]++;
#pragma omp atomic
                        tdag[q]++;
#pragma omp atomic
                        tdag[r - 1]++;
                    }
                }
            }
            for (int64_t p = orp[a]; p < orp[a + 1]; p++) marker[ocol[p]] = 0;
        }
        acc[t] = local;
        free(marker);
    }
    if (fail) { free(orp); free(ocol); free(tdag); return ORC_ENOMEM; }
    if (t_e) {
        /* copy each oriented edge's count to both directed CSR positions */
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t u = 0; u < n; u++) {
            int64_t p = orp[u];
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
                int64_t v = col[e];
                if (precedes(rp, order, u, v)) {
                    /* the oriented list of u keeps ascending id order */
                    t_e[e] = tdag[p++];
                }
            }
        }
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t u = 0; u < n; u++) {
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
                int64_t v = col[e];
                if (!precedes(rp, order, u, v)) {
                    /* mirror: find u in v's list */
                    int64_t lo = rp[v], hi = rp[v + 1];
                    while (lo < hi) {
                        int64_t mid = lo + (hi - lo) / 2;
                        if (col[mid] < u) lo = mid + 1; else hi = mid;
                    }
                    t_e[e] = t_e[lo];
                }
            }
        }
    }
    u128 total = 0;
    for (int t = 0; t < nt; t++) total += acc[t];
    free(orp); free(ocol); free(tdag);
    if (!fits64(total)) return ORC_EOVERFLOW;
    *total_out = (uint64_t)total;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O3: k-cliques by recursive marker-array enumeration                  */
/* ------------------------------------------------------------------ */
/*
 * After orientation every k-clique is a chain v1->v2->...->vk and is found
 * once, from its first vertex.  cand[c] holds the common out-neighbours of
 * the c vertices chosen so far; membership is tracked in mark[] by level.
 */
typedef struct {
    const int64_t *orp;
    const int32_t *ocol;
    int k;
    int32_t *mark;        /* per thread, size n                           */
    int32_t *buf[MAXK];   /* per thread, candidate list per level          */
} clique_ctx;

static u128 clique_rec(clique_ctx *c, int chosen, int64_t len)
{
    if (chosen == c->k - 1) return (u128)len;
    u128 s = 0;
    int32_t *cur = c->buf[chosen];
    int32_t *nxt = c->buf[chosen + 1];
    for (int64_t i = 0; i < len; i++) {
        int64_t w = cur[i];
        int64_t nl = 0;
        for (int64_t e = c->orp[w]; e < c->orp[w + 1]; e++) {
            int32_t x = c->ocol[e];
            if (c->mark[x] == chosen) { c->mark[x] = chosen + 1; nxt[nl++] = x; }
        }
        s += clique_rec(c, chosen + 1, nl);
        for (int64_t j = 0; j < nl; j++) c->mark[nxt[j]] = chosen;
    }
    return s;
}

int orc_cliques(int64_t n, const int64_t *rp, const int32_t *col, int k,
                int order, uint64_t *out)
{
    if (k < 1 || k > MAXK) return ORC_EINVAL;
    if (k == 1) { *out = (uint64_t)n; return ORC_OK; }
    if (k == 2) { *out = (uint64_t)(rp[n] / 2); return ORC_OK; }
    int64_t *orp; int32_t *ocol;
    int st = orient(n, rp, col, order, &orp, &ocol);
    if (st) return st;
    int64_t dmax = 0;
    for (int64_t u = 0; u < n; u++)
        if (orp[u + 1] - orp[u] > dmax) dmax = orp[u + 1] - orp[u];
    static u128 acc[MAXT];
    int nt = omp_get_max_threads();
    if (nt > MAXT) nt = MAXT;
    memset(acc, 0, sizeof acc);
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        clique_ctx c;
        c.orp = orp; c.ocol = ocol; c.k = k;
        c.mark = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
        int ok = c.mark != NULL;
        for (int l = 0; l < MAXK; l++) {
            c.buf[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(dmax + 1));
            ok &= c.buf[l] != NULL;
        }
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
        u128 local = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t u = 0; u < n; u++) {
            if (!ok) continue;
            int64_t len = 0;
            for (int64_t e = orp[u]; e < orp[u + 1]; e++) {
                c.mark[ocol[e]] = 1;
                c.buf[1][len++] = ocol[e];
            }
            local += clique_rec(&c, 1, len);
            for (int64_t e = orp[u]; e < orp[u + 1]; e++) c.mark[ocol[e]] = 0;
        }
        acc[t] = local;
        free(c.mark);
        for (int l = 0; l < MAXK; l++) free(c.buf[l]);
    }
    free(orp); free(ocol);
    if (fail) return ORC_ENOMEM;
    u128 total = 0;
    for (int t = 0; t < nt; t++) total += acc[t];
    if (!fits64(total)) return ORC_EOVERFLOW;
    *out = (uint64_t)total;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* 4-cycles by codegree counting                                        */
/* ------------------------------------------------------------------ */
/*
 * Rank r(v) = (degree, id).  A 4-cycle is counted once, at its maximum-rank
 * vertex v and the vertex w opposite v: paths v-u-w with r(u) < r(v) and
 * r(w) < r(v) are tallied in cnt[w], and every pair of such paths closes
 * one 4-cycle.
 */
int orc_cycle4(int64_t n, const int64_t *rp, const int32_t *col, uint64_t *out)
{
    static u128 acc[MAXT];
    int nt = omp_get_max_threads();
    if (nt > MAXT) nt = MAXT;
    memset(acc, 0, sizeof acc);
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        uint32_t *cnt = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
        if (!cnt || !touched) {
#pragma omp atomic write
            fail = 1;
        }
        u128 local = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; v++) {
            if (!cnt || !touched) continue;
            int64_t nt_ = 0;
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                int64_t u = col[e];
                if (!precedes(rp, 1, u, v)) continue;
                for (int64_t f = rp[u]; f < rp[u + 1]; f++) {
                    int64_t w = col[f];
                    if (w == v || !precedes(rp, 1, w, v)) continue;
                    if (cnt[w]++ == 0) touched[nt_++] = (int32_t)w;
                }
            }
            for (int64_t i = 0; i < nt_; i++) {
                uint64_t c = cnt[touched[i]];
                local += (u128)c * (c - 1) / 2;
                cnt[touched[i]] = 0;
            }
        }
        acc[t] = local;
        free(cnt); free(touched);
    }
    if (fail) return ORC_ENOMEM;
    u128 total = 0;
    for (int t = 0; t < nt; t++) total += acc[t];
    if (!fits64(total)) return ORC_EOVERFLOW;
    *out = (uint64_t)total;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* 4-cycles from the trace of A^4 (no ranking, no orientation)          */
/* ------------------------------------------------------------------ */
/*
 * tr(A^4) counts closed walks of length 4.  A 4-cycle gives 8 of them (4
 * starting vertices x 2 directions); every other closed 4-walk retraces an
 * edge, and there are 2 sum d^2 - sum d of those (v-u-v-u'-v: d_v^2 per
 * start v; v-u-w-u-v with w != v: sum over u in N(v) of d_u - 1).  So
 *   C4 = (tr(A^4) - 2 sum d^2 + sum d) / 8,
 * and tr(A^4) = sum over (v, w) of ((A^2)_vw)^2, where (A^2)_vw is the
 * number of 2-walks v-u-w (d_v when w = v).  Row v of A^2 is tallied in
 * cnt[] by walking v-u-w over every u and w, then squared and summed.
 */
int orc_cycle4_trace(int64_t n, const int64_t *rp, const int32_t *col, uint64_t *out)
{
    static u128 acc[MAXT];
    int nt = omp_get_max_threads();
    if (nt > MAXT) nt = MAXT;
    memset(acc, 0, sizeof acc);
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        uint32_t *cnt = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
        if (!cnt || !touched) {
#pragma omp atomic write
            fail = 1;
        }
        u128 local = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; v++) {
            if (!cnt || !touched) continue;
            int64_t nt_ = 0;
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                int64_t u = col[e];
                for (int64_t f = rp[u]; f < rp[u + 1]; f++) {
                    int64_t w = col[f];
                    if (cnt[w]++ == 0) touched[nt_++] = (int32_t)w;
                }
            }
            for (int64_t i = 0; i < nt_; i++) {
                u128 c = cnt[touched[i]];
                local += c * c;
                cnt[touched[i]] = 0;
            }
        }
        acc[t] = local;
        free(cnt); free(touched);
    }
    if (fail) return ORC_ENOMEM;
    u128 tr4 = 0, sd2 = 0, sd = 0;
    for (int t = 0; t < nt; t++) tr4 += acc[t];
    for (int64_t v = 0; v < n; v++) {
        u128 d = (u128)(rp[v + 1] - rp[v]);
        sd2 += d * d;
        sd += d;
    }
    u128 c4 = (tr4 + sd - 2 * sd2) / 8;
    if (!fits64(c4)) return ORC_EOVERFLOW;
    *out = (uint64_t)c4;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O4: non-induced (= edge-induced) 4-vertex counts                     */
/* ------------------------------------------------------------------ */
/*
 * out = [N_path4, N_star3, N_cycle4, N_tailed_triangle, N_diamond, N_clique4]
 *   N_D  = sum over edges of C(t_e, 2)        (two triangles on one edge;
 *                                              the counting-only identity of
 *                                              Sec. 5.4 (1), Alg. 3)
 *   N_TT = sum over v of t_v (d_v - 2)         (a triangle at v plus a tail
 *                                              to one of v's other neighbours)
 *   N_S3 = sum over v of C(d_v, 3)
 *   N_P4 = sum over edges (d_u - 1)(d_v - 1) - 3T   (middle edge u-v with one
 *                                              extra neighbour at each end;
 *                                              the triangle cases close a
 *                                              3-cycle and are removed)
 *   N_C4 = codegree count;  N_K4 = k-clique enumeration.
 */
static int nonind4_local_terms(int64_t n, const int64_t *rp, const int32_t *col, int order,
                               u128 *nd, u128 *ntt, u128 *ns3, u128 *np4)
{
    int64_t nnz = rp[n];
    uint64_t *tv = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    uint64_t *te = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)nnz + 1));
    if (!tv || !te) { free(tv); free(te); return ORC_ENOMEM; }
    uint64_t T;
    int st = orc_triangles(n, rp, col, order, &T, tv, te);
    if (st) { free(tv); free(te); return st; }
    *nd = 0; *ntt = 0; *ns3 = 0; *np4 = 0;
    for (int64_t u = 0; u < n; u++) {
        u128 d = (u128)(rp[u + 1] - rp[u]);
        if (d >= 3) *ns3 += d * (d - 1) * (d - 2) / 6;
        if (d >= 2) *ntt += (u128)tv[u] * (d - 2);
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            int64_t v = col[e];
            if (v <= u) continue;           /* each undirected edge once */
            u128 dv = (u128)(rp[v + 1] - rp[v]);
            u128 t = te[e];
            if (t >= 2) *nd += t * (t - 1) / 2;
            *np4 += (d - 1) * (dv - 1);
        }
    }
    *np4 -= (u128)3 * T;
    free(tv); free(te);
    return ORC_OK;
}

int orc_nonind4(int64_t n, const int64_t *rp, const int32_t *col, int order,
                uint64_t out[6])
{
    u128 nd, ntt, ns3, np4;
    int st = nonind4_local_terms(n, rp, col, order, &nd, &ntt, &ns3, &np4);
    if (st) return st;
    uint64_t c4, k4;
    st = orc_cycle4(n, rp, col, &c4);
    if (st) return st;
    st = orc_cliques(n, rp, col, 4, order, &k4);
    if (st) return st;
    if (!fits64(nd) || !fits64(ntt) || !fits64(ns3) || !fits64(np4))
        return ORC_EOVERFLOW;
    out[0] = (uint64_t)np4;
    out[1] = (uint64_t)ns3;
    out[2] = c4;
    out[3] = (uint64_t)ntt;
    out[4] = (uint64_t)nd;
    out[5] = k4;
    return ORC_OK;
}

/* The non-induced counts that need only local triangle and degree terms:
 * out = [path4, star3, tailed_triangle, diamond] (no 4-cycle or 4-clique
 * enumeration; the same terms as orc_nonind4). */
int orc_nonind4_local(int64_t n, const int64_t *rp, const int32_t *col, int order,
                      uint64_t out[4])
{
    u128 nd, ntt, ns3, np4;
    int st = nonind4_local_terms(n, rp, col, order, &nd, &ntt, &ns3, &np4);
    if (st) return st;
    if (!fits64(nd) || !fits64(ntt) || !fits64(ns3) || !fits64(np4))
        return ORC_EOVERFLOW;
    out[0] = (uint64_t)np4;
    out[1] = (uint64_t)ns3;
    out[2] = (uint64_t)ntt;
    out[3] = (uint64_t)nd;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O5 / O6: induced motif counts (k-MC, Sec. 2.1)                       */
/* ------------------------------------------------------------------ */
/*
 * 3 vertices: out = [wedge, triangle]; every induced triangle holds three
 * non-induced wedges, so induced wedges = sum C(d,2) - 3T.
 */
int orc_motifs3(int64_t n, const int64_t *rp, const int32_t *col, int order,
                uint64_t out[2])
{
    uint64_t T;
    int st = orc_triangles(n, rp, col, order, &T, NULL, NULL);
    if (st) return st;
    u128 w = 0;
    for (int64_t u = 0; u < n; u++) {
        u128 d = (u128)(rp[u + 1] - rp[u]);
        if (d >= 2) w += d * (d - 1) / 2;
    }
    w -= (u128)3 * T;
    if (!fits64(w)) return ORC_EOVERFLOW;
    out[0] = (uint64_t)w;
    out[1] = T;
    return ORC_OK;
}

/*
 * 4 vertices: out = [path4, star3, cycle4, tailed_triangle, diamond, clique4]
 * (ascending edge count).  A non-induced count is the sum over induced
 * 4-vertex graphs H of (copies of P inside H) * I_H; the copy numbers form a
 * unitriangular matrix, solved here from the densest graph down:
 *   clique4 holds 6 diamonds, 3 cycle4, 12 tailed triangles, 4 stars, 12 paths
 *   diamond holds 1 cycle4, 4 tailed triangles, 2 stars, 6 paths
 *   tailed triangle holds 1 star, 2 paths;  cycle4 holds 4 paths.
 */
int orc_motifs4(int64_t n, const int64_t *rp, const int32_t *col, int order,
                uint64_t out[6])
{
    uint64_t N[6];
    int st = orc_nonind4(n, rp, col, order, N);
    if (st) return st;
    __int128 k4 = N[5];
    __int128 d = (__int128)N[4] - 6 * k4;
    __int128 c4 = (__int128)N[2] - d - 3 * k4;
    __int128 tt = (__int128)N[3] - 4 * d - 12 * k4;
    __int128 s3 = (__int128)N[1] - tt - 2 * d - 4 * k4;
    __int128 p4 = (__int128)N[0] - 4 * c4 - 2 * tt - 6 * d - 12 * k4;
    __int128 r[6] = {p4, s3, c4, tt, d, k4};
    for (int i = 0; i < 6; i++) {
        if (r[i] < 0 || !fits64((u128)r[i])) return ORC_EOVERFLOW;
        out[i] = (uint64_t)r[i];
    }
    return ORC_OK;
}

int orc_num_threads(void) { return omp_get_max_threads(); }
