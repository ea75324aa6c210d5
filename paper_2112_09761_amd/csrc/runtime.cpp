// Host runtime of libgpm: the C ABI of include/gpm.h.
//
// Graph loader and preprocessor (Sec. 4.2, System Interface): validation, degree orientation for
// cliques, root task lists (edge list halved when the plan orders v1 < v0,
// Sec. 7.2 (2)).  Runtime (Sec. 7): frontier buffers sized to the device
// memory budget (adaptive buffering, Sec. 7.2 (3)), persistent launches fed
// by per-XCD chunk queues (the chunked scheduling idea of Sec. 7.1 on one
// GPU), batched launches over many queries, and a serving loop that admits
// queries by frontier memory and overlaps launches on several streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/gpm.h"
#include "gpm_internal.h"
#include "plan.h"

using namespace gpm;

namespace {

constexpr int kMaxSlots = 4;

struct HostCSR {
  int64_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
};

struct GraphView {
  int64_t n = 0, nnz = 0;
  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  int32_t* src = nullptr;  // row of every CSR position (root edge tasks)
  int64_t max_deg = 0;
};

struct Graph {
  bool dag_only = false;
  HostCSR host;             // symmetric graph, or the given DAG when dag_only
  GraphView sym;            // symmetric graph on device (unless dag_only)
  GraphView dag;            // degree-oriented DAG (lazy) or the given DAG
  HostCSR dag_host;
  bool dag_ready = false;
  bool dag_ordered = false;   // out-lists ordered as the orientation (ids = ranks)
  // local-graph clique tasks: vertices by out-degree, descending (lazy)
  int32_t* lgs_vtx = nullptr;
  std::vector<int64_t> lgs_deg;     // out-degree of lgs order position i
  bool lgs_ready = false;
  // DAG edges whose source has more than kLgsMaxVertices out-neighbours
  int32_t* big_src = nullptr;
  int32_t* big_dst = nullptr;
  int64_t n_big = 0;
  int64_t lgs_max_used = -1;        // root size limit the lists were built for
  // split local-graph tasks per clique size: (root, part | parts << 16)
  struct SplitTasks { int32_t* src = nullptr; int32_t* dst = nullptr; int64_t n = 0; int64_t key = -1; };
  // [0]: per-wave roots in LDS, [1]: workgroup roots, [2]: per-wave roots in HBM
  SplitTasks lgs_split[3][kMaxK + 1];
  // relabelled copy for non-clique plans: ids by ascending (degree, id), so
  // a symmetry bound v_j < v_i also bounds degree (lazy)
  HostCSR ren_host;
  GraphView ren;
  int32_t* ren_ids = nullptr;   // relabelled id -> caller's id (listing output)
  int32_t* ren_lo_src = nullptr;
  int32_t* ren_lo_dst = nullptr;
  int64_t ren_n_lo = 0;
  bool ren_ready = false;
  // 4-cycle tasks of the workgroup kernel on the relabelled graph (CycTask
  // records) and the root list of its hash tasks
  CycTask* cyc_tasks = nullptr;
  int32_t* cyc_roots = nullptr;
  int32_t* cyc_bounds = nullptr;  // id boundaries of the hash ranges
  int64_t n_cyc = 0;
  int32_t cyc_max_e = 0;          // cursor words per workgroup
  int64_t cyc_key = -1;
  int32_t* lo_src = nullptr;  // root edges (v0, v1) with v1 < v0 (lazy)
  int32_t* lo_dst = nullptr;
  int64_t n_lo = 0;
  bool lo_ready = false;
  int64_t m = 0;
  size_t bytes = 0;
};

struct QueryWork {
  // jobs of one query and how to combine their slots into results
  int kind = GPM_QUERY_COUNT;
  int k = 0;
  int first_job = 0, n_jobs = 0;
  int clique_first = 0, clique_n = 0;   // motifs(4): jobs of the 4-clique count
  int cycle_first = 0, cycle_n = 0;     // motifs(4): jobs of the 4-cycle count
  // counting-only decomposition of a single count (kDec*; 0 = none): the
  // motif terms it reads (job slots relative to first_job, -1 if absent)
  int dec = 0, dec_mode = 0;
  int deg_slot = -1, edge_slot = -1;
  uint64_t constant = 0;   // result known on the host (k <= 2, n < k, ...)
  bool has_constant = false;
  int64_t ticket = -1;
};

struct Slot {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evl[GPM_MAX_LAUNCH_STATS] = {};  // after each of the first launches
  uint32_t lkinds[GPM_MAX_LAUNCH_STATS] = {};
  int lplan[GPM_MAX_LAUNCH_STATS] = {};       // launch plan index (counter block)
  int n_lstats = 0;
  int n_launch_plans = 0;                     // counter blocks in h_res
  void* d_meta = nullptr;  size_t d_meta_bytes = 0;    // jobs, plans, offsets
  unsigned long long* d_res = nullptr; size_t d_res_words = 0;  // results + queues + counters
  int32_t* d_fbuf = nullptr; size_t d_fbuf_bytes = 0;
  int32_t* d_cursor = nullptr; size_t d_cursor_bytes = 0;  // 4-cycle cursor regions
  unsigned int* d_tri = nullptr; size_t d_tri_bytes = 0;    // per-edge triangle counters
  bool tri_dirty = true;
  void* h_stage = nullptr; size_t h_stage_bytes = 0;    // pinned
  unsigned long long* h_res = nullptr; size_t h_res_words = 0;  // pinned
  const unsigned long long* h_out = nullptr;  // where the last group's results land
  bool busy = false;
  bool heavy = false;      // serving: the running group is a heavy or unknown query
  size_t frontier_bytes_in_use = 0;
  std::vector<QueryWork> queries;
  std::vector<std::string> qkeys;  // serving: cost keys of the launch's queries
  int n_jobs = 0;
  int n_launch = 0;
  size_t counters_off = 0;   // word offset of the instrumentation counters in h_res
  std::chrono::steady_clock::time_point t_start;
};

struct Pending {
  gpm_query q;
  int64_t ticket;
  bool waited = false;   // has waited for memory at the head of the line
};

// A completed served query: its status and, on GPM_OK, its results.
struct Done {
  gpm_status st = GPM_OK;
  std::string err;
  std::array<uint64_t, 6> r{};
};

}  // namespace

// Host staging of the allocation-free count, reserved at gpm_create: the job
// table of one query and its result words.
constexpr size_t kNoallocStageBytes = 256 * 1024;
constexpr size_t kNoallocResultWords = 8192;

struct gpm_ctx {
  int device = 0;
  hipStream_t user_stream = nullptr;
  size_t budget = 0;
  int cus = 256;
  std::string err;
  std::map<int32_t, std::unique_ptr<Graph>> graphs;
  int32_t next_graph = 1;
  // options
  int64_t opt_granularity = 0, opt_chunk = 0, opt_waves_per_cu = 0, opt_setop = 0;
  int64_t opt_clique_lds = 1, opt_rename = 1, opt_count_elements = 0, opt_autotune = 0;
  int64_t opt_lds_tile = 0, opt_max_batch = 4096, opt_serve_slots = kMaxSlots;
  int64_t opt_max_pending = 1 << 20;
  int64_t opt_clique_algo = 0, opt_lgs_tile = 128, opt_lgs_max = kLgsMaxVertices;
  int64_t opt_lgs_split = 1, opt_leaf_cap = 128, opt_cycle4_algo = 0;
  int64_t opt_lgs_block = 1;                    // large roots: one workgroup each
  int64_t opt_lgs_lanes = 64;                   // local-graph row build: lanes that scan one row
  int64_t opt_decompose = 1;                    // counting-only decomposition of named motifs
  int64_t opt_cycle4_mode = 0;                  // 0 cost model, 1 hash tasks only, 2 direct windows
  int64_t opt_cycle4_batch = kCycHashCap * 2 / 3;  // wedges per 4-cycle hash task
  int64_t opt_cycle4_split = 4;                 // direct parts per workgroup (load balance)
  int64_t opt_edge_terms = 0;                   // 0 auto (triangle scatter), 1 per-edge intersection
  int lds_block_max = 65536;                    // dynamic LDS per workgroup (bytes)
  int64_t opt_tune_min_ms = 20;
  // autotuner cache: (graph, pattern, mode) -> tuned knob values
  std::map<std::string, std::vector<std::pair<std::string, int64_t>>> tuned;
  bool tuning = false;
  gpm_stats stats{};
  Slot slots[kMaxSlots + 1];  // [0]: synchronous calls on the user stream
  // serving
  std::deque<Pending> pending;
  std::unordered_map<int64_t, Done> done;
  std::unordered_set<int64_t> issued;   // tickets not yet collected
  std::unordered_map<std::string, double> qcost;  // kernel ms of queries run alone
  int64_t opt_serve_light_ms = 50;
  int64_t next_ticket = 1;
  size_t serve_frontier_in_use = 0;
  int64_t serve_memory_waits = 0;   // queries that waited for memory at the head of the line
  int64_t serve_admitted = 0;
  // allocation-free count: this device's scratch (device address), host
  // staging reserved at creation, and the flag that makes every path that
  // would allocate (graph preparation, buffer growth) fail instead
  void* scratch = nullptr;
  bool noalloc = false;
  std::vector<char> na_stage;
  std::vector<unsigned long long> na_res;
  // listing: queue and match counters (device), their copy (pinned host)
  unsigned long long* d_list = nullptr;
  unsigned long long* h_list = nullptr;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

static gpm_status fail(gpm_ctx* c, gpm_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define HIP_TRY(c, expr)                                                            \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail((c), GPM_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// The allocation-free count found a structure of the graph missing (it
// would have to build it, which allocates).
static gpm_status not_prepared(gpm_ctx* c) {
  return fail(c, GPM_E_UNSUPPORTED,
              "the allocation-free count needs the graph prepared for this query "
              "(run gpm_count with the same pattern and mode once first)");
}

template <typename T>
static gpm_status dev_upload(gpm_ctx* c, T** dst, const T* src, size_t count) {
  if (c->noalloc) return not_prepared(c);
  *dst = nullptr;
  if (count == 0) count = 1;
  HIP_TRY(c, hipMalloc((void**)dst, count * sizeof(T)));
  if (src) HIP_TRY(c, hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return GPM_OK;
}

static void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

static void free_view(GraphView& v) {
  dev_free(v.rp);
  dev_free(v.col);
  dev_free(v.src);
  v = GraphView{};
}

static void free_graph(Graph& g) {
  free_view(g.sym);
  free_view(g.ren);
  dev_free(g.ren_ids);
  g.ren_ids = nullptr;
  dev_free(g.cyc_tasks);
  dev_free(g.cyc_roots);
  dev_free(g.cyc_bounds);
  g.cyc_tasks = nullptr;
  g.cyc_roots = nullptr;
  g.cyc_bounds = nullptr;
  dev_free(g.ren_lo_src);
  dev_free(g.ren_lo_dst);
  g.ren_lo_src = g.ren_lo_dst = nullptr;
  free_view(g.dag);
  dev_free(g.lgs_vtx);
  dev_free(g.big_src);
  dev_free(g.big_dst);
  g.lgs_vtx = g.big_src = g.big_dst = nullptr;
  for (auto& row : g.lgs_split)
    for (auto& t : row) {
      dev_free(t.src);
      dev_free(t.dst);
      t = Graph::SplitTasks{};
    }
  dev_free(g.lo_src);
  dev_free(g.lo_dst);
  g.lo_src = g.lo_dst = nullptr;
}

static int64_t max_degree(const HostCSR& h) {
  int64_t m = 0;
  for (int64_t u = 0; u < h.n; ++u) m = std::max(m, h.rp[u + 1] - h.rp[u]);
  return m;
}

static gpm_status upload_view(gpm_ctx* c, const HostCSR& h, bool with_src, GraphView* v,
                              size_t* bytes) {
  v->n = h.n;
  v->nnz = h.rp[h.n];
  v->max_deg = max_degree(h);
  gpm_status st = dev_upload(c, &v->rp, h.rp.data(), h.rp.size());
  if (st) return st;
  st = dev_upload(c, &v->col, h.col.data(), h.col.size());
  if (st) return st;
  *bytes += h.rp.size() * 8 + h.col.size() * 4;
  if (with_src) {
    std::vector<int32_t> src(h.col.size());
    for (int64_t u = 0; u < h.n; ++u)
      for (int64_t p = h.rp[u]; p < h.rp[u + 1]; ++p) src[p] = (int32_t)u;
    st = dev_upload(c, &v->src, src.data(), src.size());
    if (st) return st;
    *bytes += src.size() * 4;
  }
  return GPM_OK;
}

static gpm_status ensure_ren(gpm_ctx* c, Graph& g);

// Orientation by (degree, id) (Sec. 4.2, "Graph Loader and Preprocessor":
// orientation halves the edges and shrinks the maximum degree).
static gpm_status ensure_dag(gpm_ctx* c, Graph& g) {
  if (g.dag_ready) return GPM_OK;
  if (c->noalloc) return not_prepared(c);
  if (g.dag_only) {
    g.dag_host = g.host;
  } else {
    // orient the graph relabelled by ascending (degree, id): u -> v iff u < v,
    // so every out-list is in the DAG's topological order
    gpm_status st = ensure_ren(c, g);
    if (st) return st;
    const HostCSR& R = g.ren_host;
    HostCSR& D = g.dag_host;
    D.n = R.n;
    D.rp.assign(R.n + 1, 0);
    for (int64_t u = 0; u < R.n; ++u) {
      int64_t lo = std::upper_bound(R.col.begin() + R.rp[u], R.col.begin() + R.rp[u + 1], (int32_t)u) -
                   R.col.begin();
      D.rp[u + 1] = D.rp[u] + (R.rp[u + 1] - lo);
    }
    D.col.resize(D.rp[R.n]);
    for (int64_t u = 0; u < R.n; ++u) {
      int64_t lo = std::upper_bound(R.col.begin() + R.rp[u], R.col.begin() + R.rp[u + 1], (int32_t)u) -
                   R.col.begin();
      std::copy(R.col.begin() + lo, R.col.begin() + R.rp[u + 1], D.col.begin() + D.rp[u]);
    }
    g.dag_ordered = true;
  }
  gpm_status st = upload_view(c, g.dag_host, true, &g.dag, &g.bytes);
  if (st) return st;
  g.dag_ready = true;
  return GPM_OK;
}

// Root vertices of the local-graph clique kernel, heaviest first so that the
// long tasks start early; plus the DAG edges of vertices too large for it.
static gpm_status ensure_lgs(gpm_ctx* c, Graph& g, int64_t lgs_max) {
  if (g.lgs_ready && g.lgs_max_used == lgs_max) return GPM_OK;
  if (c->noalloc) return not_prepared(c);
  if (g.lgs_ready) {
    dev_free(g.lgs_vtx);
    dev_free(g.big_src);
    dev_free(g.big_dst);
    g.lgs_vtx = g.big_src = g.big_dst = nullptr;
    g.n_big = 0;
    g.lgs_ready = false;
  }
  gpm_status st = ensure_dag(c, g);
  if (st) return st;
  const HostCSR& d = g.dag_host;
  std::vector<int32_t> order;
  std::vector<char> too_long(d.n, 0);
  for (int64_t u = 0; u < d.n; ++u) {
    if (d.rp[u + 1] - d.rp[u] < 2) continue;
    // the kernels index a root's row-build work (the summed out-degrees of its
    // out-neighbours) with int32; larger roots take the edge kernel
    int64_t work = 0;
    for (int64_t p = d.rp[u]; p < d.rp[u + 1]; ++p) work += d.rp[d.col[p] + 1] - d.rp[d.col[p]];
    if (work > (int64_t)INT32_MAX) {
      too_long[u] = 1;
      continue;
    }
    order.push_back((int32_t)u);
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return d.rp[a + 1] - d.rp[a] > d.rp[b + 1] - d.rp[b];
  });
  g.lgs_deg.resize(order.size());
  std::vector<int32_t> bs, bd;
  auto add_big = [&](int64_t u) {
    for (int64_t p = d.rp[u]; p < d.rp[u + 1]; ++p) {
      bs.push_back((int32_t)u);
      bd.push_back(d.col[p]);
    }
  };
  for (size_t i = 0; i < order.size(); ++i) {
    int64_t u = order[i];
    g.lgs_deg[i] = d.rp[u + 1] - d.rp[u];
    if (g.lgs_deg[i] > lgs_max) add_big(u);
  }
  for (int64_t u = 0; u < d.n; ++u)
    if (too_long[u]) add_big(u);
  st = dev_upload(c, &g.lgs_vtx, order.data(), order.size());
  if (st) return st;
  g.n_big = (int64_t)bs.size();
  if (g.n_big) {
    st = dev_upload(c, &g.big_src, bs.data(), bs.size());
    if (st) return st;
    st = dev_upload(c, &g.big_dst, bd.data(), bd.size());
    if (st) return st;
  }
  g.bytes += order.size() * 4 + bs.size() * 8;
  g.lgs_ready = true;
  g.lgs_max_used = lgs_max;
  return GPM_OK;
}

// Root edges (v0, v1) with v1 < v0: one direction per undirected edge.
static gpm_status ensure_lower(gpm_ctx* c, Graph& g) {
  if (g.lo_ready) return GPM_OK;
  if (c->noalloc) return not_prepared(c);
  std::vector<int32_t> s, d;
  s.reserve(g.m);
  d.reserve(g.m);
  for (int64_t u = 0; u < g.host.n; ++u)
    for (int64_t p = g.host.rp[u]; p < g.host.rp[u + 1] && g.host.col[p] < u; ++p) {
      s.push_back((int32_t)u);
      d.push_back(g.host.col[p]);
    }
  g.n_lo = (int64_t)s.size();
  gpm_status st = dev_upload(c, &g.lo_src, s.data(), s.size());
  if (st) return st;
  st = dev_upload(c, &g.lo_dst, d.data(), d.size());
  if (st) return st;
  g.bytes += s.size() * 8;
  g.lo_ready = true;
  return GPM_OK;
}

// Split the local-graph roots [lo, hi) of the heaviest-first order into
// sub-tasks: a root's cost grows like d^(k-2) (local edges for k = 4, local
// triangles for k = 5); a root gets ceil(cost / share) parts, share being a
// quarter of an even split over `waves` execution units (waves or workgroups).
static gpm_status ensure_lgs_split(gpm_ctx* c, Graph& g, int which, int k, int64_t lo,
                                   int64_t hi, int64_t waves, Graph::SplitTasks** out) {
  Graph::SplitTasks& T = g.lgs_split[which][k];
  const int64_t key = (lo << 40) ^ (hi << 8) ^ waves ^ (g.lgs_max_used << 50);
  if (T.key == key) { *out = &T; return GPM_OK; }
  if (c->noalloc) return not_prepared(c);
  dev_free(T.src);
  dev_free(T.dst);
  T = Graph::SplitTasks{};
  std::vector<double> cost(hi - lo);
  double total = 0;
  for (int64_t i = lo; i < hi; ++i) {
    double d = (double)g.lgs_deg[i];
    cost[i - lo] = std::pow(d, (double)(k - 2));
    total += cost[i - lo];
  }
  const double share = std::max(total / (double)(waves * 4), 1.0);
  std::vector<int32_t> hs, src, dst;
  hs.resize(hi - lo);
  gpm_status st = GPM_OK;
  std::vector<int32_t> order(hi - lo);
  HIP_TRY(c, hipMemcpy(order.data(), g.lgs_vtx + lo, (hi - lo) * 4, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < hi - lo; ++i) {
    int64_t parts = std::min<int64_t>(64, std::max<int64_t>(1, (int64_t)std::ceil(cost[i] / share)));
    for (int64_t p = 0; p < parts; ++p) {
      src.push_back(order[i]);
      dst.push_back((int32_t)(p | (parts << 16)));
    }
  }
  T.n = (int64_t)src.size();
  st = dev_upload(c, &T.src, src.data(), src.size());
  if (st) return st;
  st = dev_upload(c, &T.dst, dst.data(), dst.size());
  if (st) return st;
  g.bytes += src.size() * 8;
  T.key = key;
  *out = &T;
  return GPM_OK;
}

static gpm_status lower_edges(gpm_ctx* c, const HostCSR& h, int32_t** src, int32_t** dst,
                              int64_t* n, size_t* bytes) {
  std::vector<int32_t> s, d;
  s.reserve(h.rp[h.n] / 2);
  d.reserve(h.rp[h.n] / 2);
  for (int64_t u = 0; u < h.n; ++u)
    for (int64_t p = h.rp[u]; p < h.rp[u + 1] && h.col[p] < u; ++p) {
      s.push_back((int32_t)u);
      d.push_back(h.col[p]);
    }
  *n = (int64_t)s.size();
  gpm_status st = dev_upload(c, src, s.data(), s.size());
  if (st) return st;
  st = dev_upload(c, dst, d.data(), d.size());
  if (st) return st;
  *bytes += s.size() * 8;
  return GPM_OK;
}

// Relabel by ascending (degree, id) rank (Sec. 4.2: the preprocessor may sort
// and rename vertices by degree).  Counts are invariant under relabelling.
static gpm_status ensure_ren(gpm_ctx* c, Graph& g) {
  if (g.ren_ready) return GPM_OK;
  if (c->noalloc) return not_prepared(c);
  const HostCSR& h = g.host;
  std::vector<int32_t> order(h.n), rank(h.n);
  for (int64_t u = 0; u < h.n; ++u) order[u] = (int32_t)u;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return h.rp[a + 1] - h.rp[a] < h.rp[b + 1] - h.rp[b];
  });
  for (int64_t r = 0; r < h.n; ++r) rank[order[r]] = (int32_t)r;
  HostCSR& R = g.ren_host;
  R.n = h.n;
  R.rp.assign(h.n + 1, 0);
  for (int64_t r = 0; r < h.n; ++r) {
    int32_t u = order[r];
    R.rp[r + 1] = R.rp[r] + (h.rp[u + 1] - h.rp[u]);
  }
  R.col.resize(h.col.size());
  for (int64_t r = 0; r < h.n; ++r) {
    int32_t u = order[r];
    int64_t o = R.rp[r];
    for (int64_t p = h.rp[u]; p < h.rp[u + 1]; ++p) R.col[o++] = rank[h.col[p]];
    std::sort(R.col.begin() + R.rp[r], R.col.begin() + R.rp[r + 1]);
  }
  gpm_status st = upload_view(c, R, true, &g.ren, &g.bytes);
  if (st) return st;
  st = lower_edges(c, R, &g.ren_lo_src, &g.ren_lo_dst, &g.ren_n_lo, &g.bytes);
  if (st) return st;
  st = dev_upload(c, &g.ren_ids, order.data(), order.size());
  if (st) return st;
  g.bytes += order.size() * 4;
  g.ren_ready = true;
  return GPM_OK;
}

// Tasks of the 4-cycle workgroup kernel on the relabelled graph.  Root v
// (the cycle's largest vertex) has e_v lower neighbours u and
// E_v = sum_u |N(u) ∩ [0, v)| wedges; roots with fewer than two wedges hold no
// 4-cycle.  Roots with at most `batch` wedges are packed into hash batches of
// up to `batch` wedges.  A heavier root goes to direct id windows or to hash
// ranges, whichever costs less in table operations: direct = one increment
// per wedge + a table pass per window + two per u and window (cursor and
// search); hash = about four per wedge + a table pass per range + two per u
// and range.  Its id ranges of about `batch` wedges each follow the degree
// mass rp[x] (a wedge ends at w about d_w times as often as at a degree-1
// vertex).  Windows and ranges are cut into parts of about equal share.
static gpm_status ensure_cycle(gpm_ctx* c, Graph& g) {
  gpm_status st = ensure_ren(c, g);
  if (st) return st;
  const int64_t key = (c->opt_cycle4_mode << 40) ^ (c->opt_cycle4_split << 32) ^ c->opt_cycle4_batch;
  if (g.cyc_key == key) return GPM_OK;
  if (c->noalloc) return not_prepared(c);
  dev_free(g.cyc_tasks);
  dev_free(g.cyc_roots);
  dev_free(g.cyc_bounds);
  g.cyc_tasks = nullptr;
  g.cyc_roots = nullptr;
  g.cyc_bounds = nullptr;
  const HostCSR& R = g.ren_host;
  const int64_t n = R.n;
  std::vector<int32_t> ev(n, 0);
  std::vector<int64_t> Ev(n, 0);
  {
    const int nt = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&, t]() {
        for (int64_t v = t; v < n; v += nt) {
          const int32_t* b = R.col.data() + R.rp[v];
          const int32_t* e = R.col.data() + R.rp[v + 1];
          const int64_t lo = std::lower_bound(b, e, (int32_t)v) - b;
          int64_t w = 0;
          for (int64_t p = 0; p < lo; ++p) {
            const int32_t u = b[p];
            const int32_t* ub = R.col.data() + R.rp[u];
            const int32_t* ue = R.col.data() + R.rp[u + 1];
            w += std::lower_bound(ub, ue, (int32_t)v) - ub;
          }
          ev[v] = (int32_t)lo;
          Ev[v] = w;
        }
      });
    for (auto& x : th) x.join();
  }
  const int64_t batch = c->opt_cycle4_batch;
  struct Direct { int32_t v; int64_t E; };
  std::vector<Direct> direct;
  std::vector<std::pair<int64_t, int32_t>> ranged;  // (E, v)
  std::vector<int32_t> light;
  int64_t direct_total = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t E = Ev[v];
    if (E < 2) continue;
    const bool c32 = ev[v] >= 65535;
    const int64_t W = c32 ? kCycWindow / 2 : kCycWindow;
    const int64_t K = (v + W - 1) / W;
    const int64_t P = (E + batch - 1) / batch;
    const double cost_direct = (double)E + (double)K * kCycTableWords + 2.0 * ev[v] * K;
    const double cost_hash = 4.0 * (double)E + (double)P * kCycTableWords + 2.0 * ev[v] * P;
    const bool dir = c->opt_cycle4_mode == 2 ? E > batch
                   : c->opt_cycle4_mode == 1 ? false
                   : E > batch && cost_direct < cost_hash;
    if (dir) {
      direct.push_back({(int32_t)v, E});
      direct_total += E;
    } else if (E > batch) {
      ranged.push_back({E, (int32_t)v});
    } else {
      light.push_back((int32_t)v);
    }
  }
  std::sort(direct.begin(), direct.end(), [](const Direct& a, const Direct& b) { return a.E > b.E; });
  std::sort(ranged.begin(), ranged.end(), [](const std::pair<int64_t, int32_t>& a,
                                             const std::pair<int64_t, int32_t>& b) {
    return a.first > b.first;
  });
  std::vector<CycTask> tasks;
  std::vector<int32_t> roots;
  int32_t max_e = 0;
  // parts of consecutive windows or ranges, each about 1/split of an even
  // share of the heavy roots' wedges over the workgroups
  int64_t heavy_total = direct_total;
  for (const auto& hr : ranged) heavy_total += hr.first;
  const int64_t share =
      std::max<int64_t>(heavy_total / ((int64_t)c->cus * c->opt_cycle4_split), int64_t(1) << 18);
  for (const Direct& d : direct) {
    const bool c32 = ev[d.v] >= 65535;
    const int64_t W = c32 ? kCycWindow / 2 : kCycWindow;
    const int64_t K = ((int64_t)d.v + W - 1) / W;
    const int64_t parts = std::max<int64_t>(1, std::min<int64_t>(K, (d.E + share - 1) / share));
    const int64_t kn = (K + parts - 1) / parts;
    for (int64_t k0 = 0; k0 < K; k0 += kn)
      tasks.push_back(CycTask{d.v, (int32_t)k0, (int32_t)std::min(kn, K - k0), c32 ? kCycWide : 0});
    max_e = std::max(max_e, ev[d.v]);
  }
  // heavy hash roots: id ranges of about `batch` wedges by degree mass, in
  // parts of consecutive ranges
  std::vector<int32_t> bounds;
  int32_t max_e_ranged = 0;
  for (const auto& hr : ranged) {
    const int32_t v = hr.second;
    const int64_t P = (hr.first + batch - 1) / batch;
    const int32_t b0 = (int32_t)bounds.size();
    bounds.push_back(0);
    for (int64_t i = 1; i < P; ++i) {
      const int64_t target = (int64_t)((double)R.rp[v] * (double)i / (double)P);
      int32_t y = (int32_t)(std::lower_bound(R.rp.begin(), R.rp.begin() + v, target) - R.rp.begin());
      bounds.push_back(std::max(y, bounds.back()));
    }
    bounds.push_back(v);
    const int64_t parts = std::max<int64_t>(1, std::min<int64_t>(P, (hr.first + share - 1) / share));
    const int64_t pn = (P + parts - 1) / parts;
    for (int64_t r0 = 0; r0 < P; r0 += pn)
      tasks.push_back(CycTask{v, (int32_t)(b0 + r0), (int32_t)std::min(pn, P - r0), kCycRanges});
    max_e_ranged = std::max(max_e_ranged, ev[v]);
  }
  // light roots packed into tasks; keys slot * n + w + 1 stay below 2^32
  const int64_t max_slots = std::max<int64_t>(
      1, std::min<int64_t>(1024, (int64_t)(UINT32_MAX / (uint64_t)std::max<int64_t>(n, 1))));
  for (size_t i = 0; i < light.size();) {
    const int32_t r0 = (int32_t)roots.size();
    int64_t sum = 0;
    while (i < light.size() && (int64_t)roots.size() - r0 < max_slots &&
           (roots.size() == (size_t)r0 || sum + Ev[light[i]] <= batch)) {
      sum += Ev[light[i]];
      roots.push_back(light[i]);
      ++i;
    }
    tasks.push_back(CycTask{-(r0 + 1), (int32_t)roots.size(), 0, INT32_MAX});
  }
  g.n_cyc = (int64_t)tasks.size();
  // cursor words per workgroup: two int64 per lower neighbour of a direct
  // root, three per lower neighbour of a ranged root
  g.cyc_max_e = std::max(4 * max_e, 6 * max_e_ranged);
  if (!tasks.empty()) {
    st = dev_upload(c, &g.cyc_tasks, tasks.data(), tasks.size());
    if (st) return st;
  }
  if (!roots.empty()) {
    st = dev_upload(c, &g.cyc_roots, roots.data(), roots.size());
    if (st) return st;
  }
  if (!bounds.empty()) {
    st = dev_upload(c, &g.cyc_bounds, bounds.data(), bounds.size());
    if (st) return st;
  }
  g.bytes += tasks.size() * sizeof(CycTask) + roots.size() * 4 + bounds.size() * 4;
  g.cyc_key = key;
  return GPM_OK;
}

static bool is_cycle4(const gpm_pattern& p) {
  if (p.k != 4 || p.n_edges != 4) return false;
  int deg[4] = {0, 0, 0, 0};
  for (int i = 0; i < 8; ++i) deg[p.edges[i]]++;
  return deg[0] == 2 && deg[1] == 2 && deg[2] == 2 && deg[3] == 2;
}

static Graph* find_graph(gpm_ctx* c, int32_t id) {
  auto it = c->graphs.find(id);
  return it == c->graphs.end() ? nullptr : it->second.get();
}

// ---------------------------------------------------------------------------
// job construction
// ---------------------------------------------------------------------------

struct JobPlanSet {
  std::vector<Job> jobs;
  std::vector<Plan> plans;
  std::vector<int64_t> need_words;  // per job: HBM frontier words per wave
  int32_t next_tri_group = 1;       // triangle-scatter groups (Job::tri_group)
};

static int default_chunk(const gpm_ctx* c, int kind) {
  if (c->opt_chunk > 0 && kind != kJobVertexDeg) return (int)c->opt_chunk;
  switch (kind) {
    case kJobVertexDeg: return 4096;
    case kJobEdgeTri: return 32;
    default: return 8;
  }
}


// Largest local graph of the workgroup kernel: one vertex per thread in its
// scans, and its tile (plus the kernel's static LDS) within the workgroup's LDS.
static int64_t lgs_block_max_vertices(const gpm_ctx* c) {
  int64_t d = kLgsBlockMaxVertices;
  while (d > 0 && (((lgs_block_tile_words(d) + 3) & ~int64_t(3)) + kBlockSortWords) * 4 + 256 >
                      (int64_t)c->lds_block_max)
    --d;
  return d;
}

// How the DFS set operations probe (option "setop"; 0 = the default: binary
// search with the search tree's top levels in LDS, measured fastest of the
// three on R-MAT and Chung-Lu graphs).
static int32_t setop_mode(const gpm_ctx* c) {
  return c->opt_setop > 0 ? (int32_t)c->opt_setop : kSetopBst;
}

static int lds_tile(const gpm_ctx* c) {
  return c->opt_lds_tile > 0 ? (int)c->opt_lds_tile : 512;
}

// Named 3- and 4-vertex motifs whose count follows from per-vertex and
// per-edge terms (counting-only pruning, Sec. 5.4 (1)).  For a connected
// pattern the vertex count, edge count and largest degree identify the shape.
enum { kDecNone = 0, kDecWedge, kDecStar3, kDecPath4, kDecTailed, kDecDiamond };

static int decomposable(const gpm_pattern& p) {
  int deg[kMaxK] = {0};
  for (int i = 0; i < 2 * p.n_edges; ++i) deg[p.edges[i]]++;
  int dmax = 0;
  for (int i = 0; i < p.k; ++i) dmax = std::max(dmax, deg[i]);
  if (p.k == 3 && p.n_edges == 2) return kDecWedge;
  if (p.k == 4 && p.n_edges == 3) return dmax == 3 ? kDecStar3 : kDecPath4;
  if (p.k == 4 && p.n_edges == 4 && dmax == 3) return kDecTailed;
  if (p.k == 4 && p.n_edges == 5) return kDecDiamond;
  return kDecNone;
}

static gpm_status add_count_jobs(gpm_ctx* c, Graph& g, const gpm_pattern& p, int mode,
                                 JobPlanSet& js, QueryWork& qw);
static void named(const char* name, gpm_pattern* p);

// The per-edge motif terms (Σt_e, ΣC(t_e,2), Σt_e(d_u+d_v−4), Σ(d_u−1)(d_v−1))
// as one job whose four result fields hold them (the query's next slot);
// returns through *added the number of jobs appended.  Default: the k = 3
// local-graph search scatters every triangle onto its three edges' counters
// and a kJobEdgeTerms job folds them; when a root is too large for the
// local-graph kernels, the counters would take more than a quarter of the
// memory budget, or with edge_terms = 1: one intersection per edge.
static gpm_status add_edge_term_jobs(gpm_ctx* c, Graph& g, JobPlanSet& js, int* added) {
  gpm_status st = ensure_lower(c, g);
  if (st) return st;
  bool scatter = c->opt_edge_terms == 0 && !g.dag_only && c->opt_clique_lds &&
                 c->opt_clique_algo != 1;
  if (scatter) {
    st = ensure_dag(c, g);
    if (st) return st;
    st = ensure_lgs(c, g, c->opt_lgs_max);
    if (st) return st;
    st = ensure_ren(c, g);
    if (st) return st;
    // the counters (4 B per edge) may take a quarter of the memory budget;
    // beyond that the intersections, which need no memory of their own
    scatter = g.n_big == 0 && g.dag_ordered && (size_t)g.dag.nnz * 4 <= c->budget / 4;
  }
  if (!scatter) {
    Job J{};
    J.kind = kJobEdgeTri;
    J.rp = g.sym.rp;
    J.col = g.sym.col;
    J.task_src = g.lo_src;
    J.task_dst = g.lo_dst;
    J.n_tasks = g.n_lo;
    J.chunk = default_chunk(c, kJobEdgeTri);
    js.jobs.push_back(J);
    js.need_words.push_back(0);
    *added = 1;
    return GPM_OK;
  }
  const int32_t grp = js.next_tri_group++;
  Job E{};
  E.kind = kJobEdgeTerms;
  E.rp = g.dag.rp;
  E.col = g.dag.col;
  E.task_src = g.dag.src;
  E.n_tasks = g.dag.nnz;
  E.chunk = 4096;
  E.tri_group = grp;
  E.deg_rp = g.ren.rp;
  js.jobs.push_back(E);
  js.need_words.push_back(0);
  const size_t before = js.jobs.size();
  gpm_pattern p;
  QueryWork tmp;
  gpm_pattern_clique(3, &p);
  st = add_count_jobs(c, g, p, GPM_EDGE_INDUCED, js, tmp);
  if (st) return st;
  for (size_t i = before; i < js.jobs.size(); ++i) {
    js.jobs[i].tri_group = grp;
    // one-wave roots get their own kind, so that the clique kernels do not
    // carry the scatter code (the workgroup kernel branches on the group)
    if (js.jobs[i].kind == kJobCliqueLgs) js.jobs[i].kind = kJobTriScatter;
  }
  *added = 1 + (int)(js.jobs.size() - before);
  return GPM_OK;
}

// Jobs of a decomposed count: the degree terms (ΣC(d,2), ΣC(d,3)), the edge
// terms (Σt_e, ΣC(t_e,2), Σt_e(d_u+d_v−4), Σ(d_u−1)(d_v−1)) and, for the
// vertex-induced counts, the 4-clique (triangle for the wedge) and 4-cycle
// counts that the inclusion relation between the 4-vertex motifs needs.
static gpm_status add_decomposed_jobs(gpm_ctx* c, Graph& g, int dec, int mode, JobPlanSet& js,
                                      QueryWork& qw) {
  const bool vi = mode == GPM_VERTEX_INDUCED;
  const bool need_deg = dec == kDecWedge || dec == kDecStar3;
  const bool need_edge = !(dec == kDecWedge || (dec == kDecStar3 && !vi));
  qw.dec = dec;
  qw.dec_mode = mode;
  if (need_edge) {
    gpm_status st = ensure_lower(c, g);
    if (st) return st;
  }
  if (need_deg) {
    Job J{};
    J.kind = kJobVertexDeg;
    J.rp = g.sym.rp;
    J.col = g.sym.col;
    J.vertex_tasks = 1;
    J.n_tasks = g.host.n;
    J.chunk = default_chunk(c, kJobVertexDeg);
    qw.deg_slot = qw.n_jobs++;
    js.jobs.push_back(J);
    js.need_words.push_back(0);
  }
  if (need_edge) {
    int added = 0;
    qw.edge_slot = qw.n_jobs;
    gpm_status st = add_edge_term_jobs(c, g, js, &added);
    if (st) return st;
    qw.n_jobs += added;
  }
  if (vi) {
    gpm_pattern p;
    QueryWork tmp;
    gpm_pattern_clique(dec == kDecWedge ? 3 : 4, &p);
    qw.clique_first = qw.n_jobs;
    gpm_status st = add_count_jobs(c, g, p, GPM_EDGE_INDUCED, js, tmp);
    if (st) return st;
    qw.clique_n = tmp.n_jobs;  // 0 when the count is known to be 0
    qw.n_jobs += tmp.n_jobs;
    if (dec == kDecPath4) {
      named("cycle4", &p);
      tmp = QueryWork{};
      qw.cycle_first = qw.n_jobs;
      st = add_count_jobs(c, g, p, GPM_EDGE_INDUCED, js, tmp);
      if (st) return st;
      qw.cycle_n = tmp.n_jobs;
      qw.n_jobs += tmp.n_jobs;
    }
  }
  return GPM_OK;
}

// Append the jobs counting `p` in `mode` on graph g; *constant set when the
// answer needs no kernel.
static gpm_status add_count_jobs(gpm_ctx* c, Graph& g, const gpm_pattern& p, int mode,
                                 JobPlanSet& js, QueryWork& qw) {
  std::string err;
  gpm_status st = validate_pattern(p, &err);
  if (st) return fail(c, st, err);
  bool clique = is_clique(p);
  if (g.dag_only && !clique)
    return fail(c, GPM_E_UNSUPPORTED, "non-clique pattern on a DAG-only graph");
  const int64_t n = g.host.n;
  qw.k = p.k;
  if (p.k == 1) { qw.has_constant = true; qw.constant = (uint64_t)n; return GPM_OK; }
  if (p.k == 2) { qw.has_constant = true; qw.constant = (uint64_t)g.m; return GPM_OK; }
  if (n < p.k || g.m == 0) { qw.has_constant = true; qw.constant = 0; return GPM_OK; }

  if (clique) {
    st = ensure_dag(c, g);
    if (st) return st;
    const int64_t cap = std::max<int64_t>(g.dag.max_deg, 1);
    if (p.k - 2 > cap) { qw.has_constant = true; qw.constant = 0; return GPM_OK; }
    Job J{};
    J.rp = g.dag.rp;
    J.col = g.dag.col;
    J.task_src = g.dag.src;
    J.task_dst = g.dag.col;
    J.n_tasks = g.dag.nnz;
    J.k = p.k;
    J.cap = (int32_t)cap;
    J.ordered = g.dag_ordered ? 1 : 0;
    const bool lgs = c->opt_clique_lds && c->opt_clique_algo != 1 && p.k <= 5;
    if (lgs) {
      // local graph search with bitmaps for roots with at most
      // kLgsMaxVertices out-neighbours; larger roots take the edge kernel
      st = ensure_lgs(c, g, c->opt_lgs_max);
      if (st) return st;
      const auto& dg = g.lgs_deg;  // descending
      // first root with out-degree <= lgs_max, first root with out-degree < k-1
      int64_t lo = std::lower_bound(dg.begin(), dg.end(), c->opt_lgs_max,
                                    [](int64_t x, int64_t y) { return x > y; }) - dg.begin();
      int64_t hi = std::upper_bound(dg.begin(), dg.end(), (int64_t)(p.k - 1),
                                    [](int64_t x, int64_t y) { return x > y; }) - dg.begin();
      // [lo, hi) splits by out-degree d into [lo, b0): d above the workgroup
      // LDS tile (one workgroup per root, bitmap rows in its HBM region);
      // [b0, mid): above the per-wave LDS tile, one workgroup per root with
      // the tile in its LDS; [mid, hi): per wave, rows in LDS
      int64_t b0 = lo, mid = lo;
      if (c->opt_lgs_block && hi > lo) {
        auto first_at_most = [&](int64_t v) {
          return std::lower_bound(dg.begin() + lo, dg.begin() + hi, v,
                                  [](int64_t x, int64_t y) { return x > y; }) - dg.begin();
        };
        mid = first_at_most(c->opt_lgs_tile);
        b0 = std::min(first_at_most(lgs_block_max_vertices(c)), mid);
      }
      auto add_lgs = [&](int kind, int64_t a, int64_t b, int which, int64_t units,
                         bool split, bool always, int lds_rows) -> gpm_status {
        if (b <= a && !always) return GPM_OK;
        Job L = J;
        L.kind = kind;
        L.lds_ok = lds_rows;
        L.vertex_tasks = 1;
        L.task_src = g.lgs_vtx + a;
        L.task_dst = nullptr;
        L.n_tasks = std::max<int64_t>(b - a, 0);
        L.chunk = c->opt_chunk > 0 ? (int)c->opt_chunk : 1;
        if (split && c->opt_lgs_split && b > a) {
          Graph::SplitTasks* T = nullptr;
          gpm_status s2 = ensure_lgs_split(c, g, which, p.k, a, b, units, &T);
          if (s2) return s2;
          L.task_src = T->src;
          L.task_dst = T->dst;
          L.n_tasks = T->n;
        }
        // largest root of the range (heaviest first)
        L.cap = (int32_t)(b > a ? dg[a] : std::min<int64_t>(cap, c->opt_lgs_max));
        js.jobs.push_back(L);
        // workgroup roots with rows in HBM: one region of the rows per workgroup
        js.need_words.push_back(kind == kJobCliqueLgsBlock && !lds_rows
                                    ? 2 * (int64_t)L.cap * (((int64_t)L.cap + 63) / 64)
                                    : 0);
        qw.n_jobs += 1;
        return GPM_OK;
      };
      const int64_t waves = (int64_t)c->cus * 16;
      st = add_lgs(kJobCliqueLgs, mid, hi, 0, waves, p.k >= 5, true, 1);
      if (st) return st;
      st = add_lgs(kJobCliqueLgsBlock, b0, mid, 1, (int64_t)c->cus, p.k >= 4, false, 1);
      if (st) return st;
      if (c->opt_lgs_block)
        st = add_lgs(kJobCliqueLgsBlock, lo, b0, 2, (int64_t)c->cus, p.k >= 4, false, 0);
      else
        st = add_lgs(kJobCliqueLgs, lo, b0, 2, waves, p.k >= 5, false, 1);
      if (st) return st;
      if (g.n_big) {
        Job B = J;
        B.kind = kJobClique;
        B.task_src = g.big_src;
        B.task_dst = g.big_dst;
        B.n_tasks = g.n_big;
        B.chunk = default_chunk(c, kJobClique);
        B.lds_ok = 1;
        js.jobs.push_back(B);
        js.need_words.push_back(0);
        qw.n_jobs += 1;
      }
      return GPM_OK;
    }
    if (c->opt_clique_lds) {
      J.kind = kJobClique;
      J.chunk = default_chunk(c, kJobClique);
      J.lds_ok = 1;
      js.jobs.push_back(J);
      js.need_words.push_back(0);  // HBM fallback sized at launch, once the LDS tile is known
    } else {
      HostPlan hp;
      st = build_plan(p, mode, true, &hp, &err);
      if (st) return fail(c, st, err);
      J.kind = kJobDfs;
      J.setop = setop_mode(c);
      J.chunk = default_chunk(c, kJobDfs);
      J.plan = (int32_t)js.plans.size();
      js.plans.push_back(hp.plan);
      js.jobs.push_back(J);
      js.need_words.push_back((int64_t)hp.n_buffers * cap);
    }
    qw.n_jobs += 1;
    return GPM_OK;
  }

  if (c->opt_decompose && !g.dag_only) {
    const int dec = decomposable(p);
    if (dec != kDecNone) return add_decomposed_jobs(c, g, dec, mode, js, qw);
  }

  if (mode == GPM_EDGE_INDUCED && is_cycle4(p) && c->opt_cycle4_algo != 1) {
    st = ensure_cycle(c, g);
    if (st) return st;
    if (g.n_cyc == 0) { qw.has_constant = true; qw.constant = 0; return GPM_OK; }
    Job J{};
    J.kind = kJobCycleBlock;
    J.k = 4;
    J.rp = g.ren.rp;
    J.col = g.ren.col;
    J.task_src = (const int32_t*)g.cyc_tasks;
    J.task_dst = g.cyc_roots;
    J.n_tasks = g.n_cyc;
    J.chunk = 1;
    J.cap = g.cyc_max_e;  // cursor words per workgroup
    J.bounds = g.cyc_bounds;
    J.n_vertices = (int32_t)n;
    js.jobs.push_back(J);
    js.need_words.push_back(0);
    qw.n_jobs += 1;
    return GPM_OK;
  }
  // counting-only pruning of a twin suffix (edge-induced) unless decompose = 0
  HostPlan hp;
  st = build_plan(p, mode, false, &hp, &err, c->opt_decompose != 0);
  if (st) return fail(c, st, err);
  const bool ren = c->opt_rename != 0;
  if (ren) {
    st = ensure_ren(c, g);
    if (st) return st;
  }
  GraphView& V = ren ? g.ren : g.sym;
  const int64_t cap = std::max<int64_t>(V.max_deg, 1);
  Job J{};
  J.kind = kJobDfs;
  J.setop = setop_mode(c);
  J.leaf_cap = (int32_t)c->opt_leaf_cap;
  J.k = p.k;
  J.rp = V.rp;
  J.col = V.col;
  J.cap = (int32_t)cap;
  J.chunk = default_chunk(c, kJobDfs);
  J.plan = (int32_t)js.plans.size();
  bool vertex = c->opt_granularity == 1;
  if (vertex) {
    J.vertex_tasks = 1;
    J.n_tasks = n;
  } else if (hp.plan.root_bound) {
    if (ren) {
      J.task_src = g.ren_lo_src;
      J.task_dst = g.ren_lo_dst;
      J.n_tasks = g.ren_n_lo;
    } else {
      st = ensure_lower(c, g);
      if (st) return st;
      J.task_src = g.lo_src;
      J.task_dst = g.lo_dst;
      J.n_tasks = g.n_lo;
    }
  } else {
    if (!V.src) {
      const HostCSR& H = ren ? g.ren_host : g.host;
      std::vector<int32_t> src(H.col.size());
      for (int64_t u = 0; u < n; ++u)
        for (int64_t q = H.rp[u]; q < H.rp[u + 1]; ++q) src[q] = (int32_t)u;
      st = dev_upload(c, &V.src, src.data(), src.size());
      if (st) return st;
      g.bytes += src.size() * 4;
    }
    J.task_src = V.src;
    J.task_dst = V.col;
    J.n_tasks = V.nnz;
  }
  js.plans.push_back(hp.plan);
  js.jobs.push_back(J);
  js.need_words.push_back((int64_t)hp.n_buffers * cap);
  qw.n_jobs += 1;
  return GPM_OK;
}


// ---------------------------------------------------------------------------
// autotuner: task granularity, chunk size, LDS tile, waves per CU, leaf mode,
// set-op mode, row-build lanes
// ---------------------------------------------------------------------------

static int64_t* knob(gpm_ctx* c, const std::string& k) {
  if (k == "granularity") return &c->opt_granularity;
  if (k == "chunk") return &c->opt_chunk;
  if (k == "waves_per_cu") return &c->opt_waves_per_cu;
  if (k == "lgs_tile") return &c->opt_lgs_tile;
  if (k == "leaf_cap") return &c->opt_leaf_cap;
  if (k == "rename") return &c->opt_rename;
  if (k == "lds_tile") return &c->opt_lds_tile;
  if (k == "setop") return &c->opt_setop;
  if (k == "lgs_lanes") return &c->opt_lgs_lanes;
  return nullptr;
}

// Search space per kind of query: coordinate descent over these knobs, in
// this order, each value tried once with the others held at their best.
static std::vector<std::pair<std::string, std::vector<int64_t>>> tune_space(const gpm_pattern& p,
                                                                             int mode) {
  const bool clique = p.n_edges == p.k * (p.k - 1) / 2;
  if (clique && p.k <= 5)
    return {{"lgs_tile", {128, 64, 192}}, {"waves_per_cu", {0, 16, 32}}, {"chunk", {0, 2}},
            {"lgs_lanes", {64, 32}}};
  if (clique) return {{"lds_tile", {0, 256, 128}}, {"chunk", {0, 4, 16}}, {"waves_per_cu", {16, 12}}};
  (void)mode;
  return {{"leaf_cap", {128, 0, 32, 512}}, {"setop", {0, 1, 2}}, {"chunk", {0, 2, 32}},
          {"granularity", {0, 1}}, {"rename", {1, 0}}, {"waves_per_cu", {16, 12}}};
}

static std::string tune_key(int32_t gid, const gpm_pattern& p, int mode) {
  std::string k = std::to_string(gid) + ":" + std::to_string(mode) + ":" + std::to_string(p.k);
  for (int i = 0; i < 2 * p.n_edges; ++i) k += "," + std::to_string(p.edges[i]);
  return k;
}

// k-motif counting (Sec. 2.1): fused triangle-rooted edge job, degree job,
// 4-clique on the DAG and the 4-cycle plan (kernel fission, Sec. 5.3).
static gpm_status add_motif_jobs(gpm_ctx* c, Graph& g, int k, JobPlanSet& js, QueryWork& qw) {
  if (k != 3 && k != 4) return fail(c, GPM_E_INVAL, "motif size must be 3 or 4");
  if (g.dag_only) return fail(c, GPM_E_UNSUPPORTED, "motifs need the symmetric graph");
  qw.kind = GPM_QUERY_MOTIFS;
  qw.k = k;
  if (g.m == 0) { qw.has_constant = true; qw.constant = 0; return GPM_OK; }
  gpm_status st = GPM_OK;
  // slot order: [degree terms] [edge terms (k = 4)] [clique] [cycle4]
  {
    Job J{};
    J.kind = kJobVertexDeg;
    J.rp = g.sym.rp;
    J.col = g.sym.col;
    J.vertex_tasks = 1;
    J.n_tasks = g.host.n;
    J.chunk = default_chunk(c, kJobVertexDeg);
    js.jobs.push_back(J);
    js.need_words.push_back(0);
  }
  qw.n_jobs += 1;
  if (k == 3) {
    // the triangle count alone: the local-graph clique kernel
    gpm_pattern p;
    QueryWork tmp;
    gpm_pattern_clique(3, &p);
    qw.clique_first = (int)js.jobs.size() - qw.first_job;
    st = add_count_jobs(c, g, p, GPM_EDGE_INDUCED, js, tmp);
    if (st) return st;
    qw.clique_n = tmp.n_jobs;
    qw.n_jobs += tmp.n_jobs;
    return GPM_OK;
  }
  {
    int added = 0;  // slot 1: the edge terms (first job appended)
    st = add_edge_term_jobs(c, g, js, &added);
    if (st) return st;
    qw.n_jobs += added;
  }
  if (k == 4) {
    gpm_pattern p;
    QueryWork tmp;
    gpm_pattern_clique(4, &p);
    qw.clique_first = (int)js.jobs.size() - qw.first_job;
    st = add_count_jobs(c, g, p, GPM_EDGE_INDUCED, js, tmp);
    if (st) return st;
    qw.clique_n = tmp.n_jobs;  // 0 when the count is known to be 0
    named("cycle4", &p);
    tmp = QueryWork{};
    qw.cycle_first = (int)js.jobs.size() - qw.first_job;
    st = add_count_jobs(c, g, p, GPM_EDGE_INDUCED, js, tmp);
    if (st) return st;
    qw.cycle_n = tmp.n_jobs;
    qw.n_jobs += qw.clique_n + qw.cycle_n;
  }
  return GPM_OK;
}

// Combine a query's job slots into its results.
static void finish_query(const QueryWork& qw, const unsigned long long* res, uint64_t out[6]) {
  for (int i = 0; i < 6; ++i) out[i] = 0;
  if (qw.has_constant) {
    if (qw.kind == GPM_QUERY_COUNT) out[0] = qw.constant;
    return;
  }
  auto slot = [&](int j, int f) { return (uint64_t)res[(size_t)(qw.first_job + j) * kResultFields + f]; };
  auto sum0 = [&](int first, int n) {
    uint64_t x = 0;
    for (int j = 0; j < n; ++j) x += slot(first + j, 0);
    return x;
  };
  if (qw.kind == GPM_QUERY_COUNT && qw.dec == kDecNone) {
    out[0] = sum0(0, qw.n_jobs);
    return;
  }
  if (qw.kind == GPM_QUERY_COUNT) {
    // decomposed count: non-induced counts from the terms, induced ones by
    // the unitriangular inclusion relation of the 4-vertex motifs
    auto f = [&](int s, int fld) { return s >= 0 ? slot(s, fld) : 0ull; };
    const uint64_t sum_c2 = f(qw.deg_slot, 0), n_s3 = f(qw.deg_slot, 1);
    const uint64_t three_t = f(qw.edge_slot, 0), n_d = f(qw.edge_slot, 1);
    const uint64_t n_tt = f(qw.edge_slot, 2) / 2, pmid = f(qw.edge_slot, 3);
    const uint64_t T = three_t / 3;
    const bool vi = qw.dec_mode == GPM_VERTEX_INDUCED;
    const uint64_t kc = sum0(qw.clique_first, qw.clique_n);  // triangles (wedge) or 4-cliques
    const uint64_t i_d = n_d - 6 * kc, i_tt = n_tt - 4 * i_d - 12 * kc;
    uint64_t r = 0;
    switch (qw.dec) {
      case kDecWedge: r = vi ? sum_c2 - 3 * kc : sum_c2; break;
      case kDecDiamond: r = vi ? i_d : n_d; break;
      case kDecTailed: r = vi ? i_tt : n_tt; break;
      case kDecStar3: r = vi ? n_s3 - i_tt - 2 * i_d - 4 * kc : n_s3; break;
      case kDecPath4: {
        const uint64_t n_p4 = pmid - 3 * T;
        if (!vi) { r = n_p4; break; }
        const uint64_t i_c4 = sum0(qw.cycle_first, qw.cycle_n) - i_d - 3 * kc;
        r = n_p4 - 4 * i_c4 - 2 * i_tt - 6 * i_d - 12 * kc;
        break;
      }
      default: break;
    }
    out[0] = r;
    return;
  }
  const uint64_t sum_c2 = slot(0, 0), n_s3 = slot(0, 1);
  if (qw.k == 3) {
    const uint64_t T = sum0(qw.clique_first, qw.clique_n);
    out[0] = sum_c2 - 3 * T;  // induced wedges
    out[1] = T;
    return;
  }
  const uint64_t three_t = slot(1, 0), n_d = slot(1, 1), two_tt = slot(1, 2), pmid = slot(1, 3);
  const uint64_t T = three_t / 3;
  // non-induced 4-vertex counts -> induced (unitriangular inclusion relation)
  const uint64_t n_k4 = sum0(qw.clique_first, qw.clique_n);
  const uint64_t n_c4 = sum0(qw.cycle_first, qw.cycle_n);
  const uint64_t n_tt = two_tt / 2, n_p4 = pmid - 3 * T;
  const uint64_t i_k4 = n_k4;
  const uint64_t i_d = n_d - 6 * i_k4;
  const uint64_t i_c4 = n_c4 - i_d - 3 * i_k4;
  const uint64_t i_tt = n_tt - 4 * i_d - 12 * i_k4;
  const uint64_t i_s3 = n_s3 - i_tt - 2 * i_d - 4 * i_k4;
  const uint64_t i_p4 = n_p4 - 4 * i_c4 - 2 * i_tt - 6 * i_d - 12 * i_k4;
  out[0] = i_p4; out[1] = i_s3; out[2] = i_c4; out[3] = i_tt; out[4] = i_d; out[5] = i_k4;
}

// ---------------------------------------------------------------------------
// launching
// ---------------------------------------------------------------------------

static gpm_status slot_init(gpm_ctx* c, Slot& s, hipStream_t user) {
  if (s.ev0) return GPM_OK;
  if (user || &s == &c->slots[0]) {
    s.stream = user;
    s.own_stream = false;
  } else {
    HIP_TRY(c, hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
    s.own_stream = true;
  }
  HIP_TRY(c, hipEventCreate(&s.ev0));
  HIP_TRY(c, hipEventCreate(&s.ev1));
  for (auto& e : s.evl) HIP_TRY(c, hipEventCreate(&e));
  return GPM_OK;
}

static void slot_free(Slot& s) {
  if (s.stream && s.own_stream) (void)hipStreamSynchronize(s.stream);
  dev_free(s.d_meta);
  dev_free(s.d_res);
  dev_free(s.d_fbuf);
  dev_free(s.d_cursor);
  dev_free(s.d_tri);
  if (s.h_stage) (void)hipHostFree(s.h_stage);
  if (s.h_res) (void)hipHostFree(s.h_res);
  if (s.ev0) (void)hipEventDestroy(s.ev0);
  if (s.ev1) (void)hipEventDestroy(s.ev1);
  for (auto& e : s.evl)
    if (e) (void)hipEventDestroy(e);
  if (s.stream && s.own_stream) (void)hipStreamDestroy(s.stream);
  s = Slot{};
}

static gpm_status grow_dev(gpm_ctx* c, void** p, size_t* have, size_t need) {
  if (*have >= need) return GPM_OK;
  if (c->noalloc) return fail(c, GPM_E_DEVICE, "buffer growth in the allocation-free count");
  dev_free(*p);
  *p = nullptr;
  *have = 0;
  size_t n = std::max(need, (size_t)4096);
  HIP_TRY(c, hipMalloc(p, n));
  *have = n;
  return GPM_OK;
}

static gpm_status grow_host(gpm_ctx* c, void** p, size_t* have, size_t need) {
  if (*have >= need) return GPM_OK;
  if (c->noalloc) return fail(c, GPM_E_DEVICE, "buffer growth in the allocation-free count");
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *have = 0;
  size_t n = std::max(need, (size_t)4096);
  HIP_TRY(c, hipHostMalloc(p, n, hipHostMallocDefault));
  *have = n;
  return GPM_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct LaunchPlan {
  uint32_t kinds = 0;
  int first = 0, count = 0;   // jobs [first, first+count)
  int64_t chunks = 0;
  int blocks = 0;
  std::vector<int64_t> jbeg;  // count + 1
  int64_t qbeg[kQueues + 1];
};

// Split the jobs of js into launches: one launch per job kind (kernel
// fission) when `fission`, else one launch for everything.  Jobs are
// reordered so that every launch's jobs are contiguous.
static std::vector<LaunchPlan> plan_launches(JobPlanSet& js, std::vector<int>& perm,
                                             bool fission) {
  const int nj = (int)js.jobs.size();
  perm.resize(nj);
  for (int i = 0; i < nj; ++i) perm[i] = i;
  // launches run in phases: the workgroup kernels first (local-graph cliques,
  // then 4-cycles, each a kernel of its own), then the per-wave kinds, then
  // the edge-term jobs, which read what the triangle scatter of the earlier
  // phases left (kernel boundaries order them)
  auto phase = [&](int i) {
    const int k = js.jobs[i].kind;
    return k == kJobCliqueLgsBlock ? 0 : k == kJobCycleBlock ? 1 : k == kJobEdgeTerms ? 3 : 2;
  };
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
    if (phase(a) != phase(b)) return phase(a) < phase(b);
    return fission && js.jobs[a].kind < js.jobs[b].kind;
  });
  std::vector<LaunchPlan> out;
  int last_phase = -1;
  for (int i = 0; i < nj; ++i) {
    const Job& J = js.jobs[perm[i]];
    uint32_t kb = 1u << J.kind;
    const int ph = phase(perm[i]);
    if (out.empty() || ph != last_phase || (fission && out.back().kinds != kb)) {
      last_phase = ph;
      LaunchPlan L;
      L.first = i;
      L.kinds = kb;
      out.push_back(L);
    }
    LaunchPlan& L = out.back();
    L.kinds |= kb;
    L.count++;
  }
  return out;
}

// Device memory of one synchronous group that the library must not allocate:
// every buffer of the group is carved from it.
struct Arena {
  char* base;
  size_t bytes;
};

// Size, stage and enqueue the launches of one group on slot s.  Results land
// in s.h_out when s.ev1 completes: the slot's pinned buffer, or with an arena
// the context's reserved host buffer (device buffers then come from the arena,
// nothing is allocated, and the zero-initialised counters are cleared on
// every call, since the arena keeps what the last call left).
static gpm_status launch_group(gpm_ctx* c, Slot& s, JobPlanSet& js, bool fission,
                               size_t frontier_budget, size_t* frontier_used,
                               const Arena* ar = nullptr) {
  gpm_status st = slot_init(c, s, s.stream);
  if (st) return st;
  std::vector<int> perm;
  std::vector<LaunchPlan> launches = plan_launches(js, perm, fission);
  const int nj = (int)js.jobs.size();
  std::vector<Job> jobs(nj);
  std::vector<int64_t> need(nj);
  for (int i = 0; i < nj; ++i) {
    jobs[i] = js.jobs[perm[i]];
    need[i] = js.need_words[perm[i]];
    jobs[i].slot = perm[i];  // result slot = the job's original index
  }

  // staging layout: jobs | plans | per launch (jbeg, qbeg); device result
  // words: results [nj * 8] | queues [launches * 8 * 16] | counters [launches * 4]
  size_t off_jobs = 0;
  size_t off_plans = align_up(off_jobs + sizeof(Job) * nj, 256);
  size_t off_l = align_up(off_plans + sizeof(Plan) * std::max<size_t>(js.plans.size(), 1), 256);
  std::vector<size_t> off_jbeg(launches.size()), off_qbeg(launches.size());
  {
    size_t cur = off_l;
    for (size_t i = 0; i < launches.size(); ++i) {
      off_jbeg[i] = cur;
      cur = align_up(cur + 8 * ((size_t)launches[i].count + 1), 64);
      off_qbeg[i] = cur;
      cur = align_up(cur + 8 * (kQueues + 1), 64);
    }
    off_l = cur;
  }
  const size_t meta_bytes = off_l;
  const size_t res_words = (size_t)nj * kResultFields;
  const size_t q_words = launches.size() * kQueues * kQueueStride;
  const size_t all_words = res_words + q_words + 4 * std::max<size_t>(launches.size(), 1);
  // with an arena: meta | results, then the frontier and counter buffers
  size_t arena_fixed = 0;
  if (ar) {
    arena_fixed = align_up(meta_bytes, 256) + align_up(all_words * 8, 256);
    if (meta_bytes > c->na_stage.size() || all_words > c->na_res.size() ||
        arena_fixed > ar->bytes)
      return fail(c, GPM_E_NOMEM, "the query's job tables exceed the allocation-free scratch");
    frontier_budget = ar->bytes - arena_fixed;
  }

  // LDS tile of the clique kernel: U | F_2 .. F_{k-2} | pad | P (int64) per wave
  bool any_clique = false;
  int kmax = 3;
  for (int i = 0; i < nj; ++i)
    if (jobs[i].kind == kJobClique) {
      any_clique = true;
      kmax = std::max(kmax, (int)jobs[i].k);
    }
  int32_t lcap = 0, lds_words = 0;
  if (any_clique) {
    auto words = [&](int32_t cap) {
      return (int32_t)align_up((size_t)cap * (1 + std::max(kmax - 3, 0)) + 1 + 2 * ((size_t)cap + 1), 4);
    };
    lcap = lds_tile(c);
    lds_words = words(lcap);
    while ((size_t)lds_words * 4 * kWavesPerBlock > 60 * 1024 && lcap > 32) {
      lcap /= 2;
      lds_words = words(lcap);
    }
    // tasks whose N+(u) exceeds the tile keep their sets in HBM
    for (int i = 0; i < nj; ++i)
      if (jobs[i].kind == kJobClique && jobs[i].cap > lcap)
        need[i] = (int64_t)std::max((int)jobs[i].k - 3, 0) * jobs[i].cap + 1 + 2 * ((int64_t)jobs[i].cap + 1);
  }

  // local-graph tile: roots with more out-neighbours than the tile keep
  // their local graph in the wave's HBM region
  int32_t lgs_T = 0;
  for (int i = 0; i < nj; ++i)
    if (jobs[i].kind == kJobCliqueLgs || jobs[i].kind == kJobTriScatter) {
      lgs_T = (int32_t)c->opt_lgs_tile;
      if (jobs[i].cap > lgs_T) need[i] = std::max<int64_t>(need[i], lgs_tile_words(jobs[i].cap));
    }
  if (lgs_T) lds_words = std::max<int32_t>(lds_words, (int32_t)align_up((size_t)lgs_tile_words(lgs_T), 4));
  // workgroup kernel: room for the largest root of its jobs
  // (jobs with rows in HBM keep only L, P and the hash in LDS)
  int64_t blk_tile = 0, blk_vmax = 0;
  bool blk_hbm_rows = false;
  for (int i = 0; i < nj; ++i)
    if (jobs[i].kind == kJobCliqueLgsBlock) {
      const int64_t t = jobs[i].lds_ok ? lgs_block_tile_words(jobs[i].cap) : lgs_rows_offset(jobs[i].cap);
      blk_tile = std::max(blk_tile, t);
      blk_vmax = std::max<int64_t>(blk_vmax, jobs[i].cap);
      if (!jobs[i].lds_ok) blk_hbm_rows = true;
    }
  const size_t blk_lds =
      blk_tile ? ((size_t)align_up((size_t)blk_tile, 4) + kBlockSortWords) * 4 : 0;
  if (blk_tile && (blk_vmax > kLgsMaxVertices || blk_lds + 256 > (size_t)c->lds_block_max))
    return fail(c, GPM_E_DEVICE, "local graph exceeds the workgroup LDS");

  // frontier sizing (adaptive buffering): one region of `stride` words per wave
  int64_t stride = 0;
  for (int i = 0; i < nj; ++i) stride = std::max(stride, need[i]);
  stride = (int64_t)align_up((size_t)stride, 64);
  // auto: 24 waves per CU for the local-graph clique kernels (their register
  // count allows six waves per SIMD), 16 otherwise
  bool lgs_only = nj > 0;
  for (int i = 0; i < nj; ++i)
    if (jobs[i].kind != kJobCliqueLgs && jobs[i].kind != kJobCliqueLgsBlock &&
        jobs[i].kind != kJobTriScatter &&
        jobs[i].kind != kJobClique)
      lgs_only = false;
  const int64_t wpc = c->opt_waves_per_cu > 0 ? c->opt_waves_per_cu : (lgs_only ? 24 : 16);
  int64_t max_resident = (int64_t)c->cus * wpc;
  int64_t waves = max_resident;
  if (stride > 0) {
    gpm_status s2 = gpm_frontier_waves((int64_t)frontier_budget, 1, stride, max_resident,
                                       max_resident, &waves);
    if (s2 || waves < kWavesPerBlock)
      return fail(c, GPM_E_NOMEM, "frontier buffers do not fit the memory budget");
  }
  // 4-cycle workgroup kernel: one cursor region per workgroup (the lower
  // neighbours of the launch's largest direct root)
  int64_t zstride = 0;
  bool any_cyc = false;
  for (int i = 0; i < nj; ++i)
    if (jobs[i].kind == kJobCycleBlock) {
      any_cyc = true;
      zstride = std::max<int64_t>(zstride, jobs[i].cap);
    }
  zstride = any_cyc ? (int64_t)align_up((size_t)std::max<int64_t>(zstride, 1), 64) : 0;
  int cyc_blocks = 0;
  if (any_cyc && cycle_block_grid(c->cus, INT64_MAX, &cyc_blocks))
    return fail(c, GPM_E_DEVICE, "4-cycle kernel occupancy query failed");
  waves = std::max<int64_t>(kWavesPerBlock, waves / kWavesPerBlock * kWavesPerBlock);
  const int blocks = (int)(waves / kWavesPerBlock);
  const size_t fbytes = (size_t)waves * (size_t)stride * 4;
  int32_t* fbuf = nullptr;
  if (fbytes) {
    if (ar) {
      fbuf = (int32_t*)(ar->base + arena_fixed);
    } else {
      st = grow_dev(c, (void**)&s.d_fbuf, &s.d_fbuf_bytes, fbytes);
      if (st) return st;
      fbuf = s.d_fbuf;
    }
  }
  // cursor regions: fewer workgroups when they do not all fit the budget
  if (any_cyc) {
    const int64_t left = (int64_t)frontier_budget - (int64_t)fbytes;
    const int64_t fit = left > 0 ? left / (zstride * 4) : 0;
    if (fit < 1) return fail(c, GPM_E_NOMEM, "4-cycle cursor regions do not fit the memory budget");
    cyc_blocks = (int)std::min<int64_t>(cyc_blocks, fit);
  }
  const size_t zbytes = (size_t)cyc_blocks * (size_t)zstride * 4;
  int32_t* zbuf = nullptr;
  if (zbytes) {
    if (ar) {
      zbuf = (int32_t*)(ar->base + arena_fixed + fbytes);
    } else {
      st = grow_dev(c, (void**)&s.d_cursor, &s.d_cursor_bytes, zbytes);
      if (st) return st;
      zbuf = s.d_cursor;
    }
  }
  // per-edge triangle counters: one region per scatter group (its DAG edge
  // count, from the group's edge-term job), zero between launches
  std::map<int32_t, int64_t> tri_off;
  int64_t tri_words = 0;
  for (int i = 0; i < nj; ++i)
    if (jobs[i].kind == kJobEdgeTerms) {
      tri_off[jobs[i].tri_group] = tri_words;
      tri_words += (int64_t)align_up((size_t)std::max<int64_t>(jobs[i].n_tasks, 1), 64);
    }
  const size_t tbytes = (size_t)tri_words * 4;
  if (tbytes) {
    if (fbytes + zbytes + tbytes > frontier_budget)
      return fail(c, GPM_E_NOMEM, "per-edge triangle counters do not fit the memory budget");
    unsigned int* tri = nullptr;
    if (ar) {
      tri = (unsigned int*)(ar->base + arena_fixed + fbytes + zbytes);
      if (launch_fill_u64((unsigned long long*)tri, (int64_t)(tbytes / 8), 0ull, s.stream))
        return fail(c, GPM_E_DEVICE, "fill kernel launch failed");
    } else {
      const size_t cap_before = s.d_tri_bytes;  // (as for the wedge counters above)
      st = grow_dev(c, (void**)&s.d_tri, &s.d_tri_bytes, tbytes);
      if (st) return st;
      if (s.d_tri_bytes != cap_before) s.tri_dirty = true;
      if (s.tri_dirty) {
        if (launch_fill_u64((unsigned long long*)s.d_tri, (int64_t)(s.d_tri_bytes / 8), 0ull,
                            s.stream))
          return fail(c, GPM_E_DEVICE, "fill kernel launch failed");
      }
      s.tri_dirty = true;  // until this group completes (the edge-term jobs restore zeros)
      tri = s.d_tri;
    }
    for (int i = 0; i < nj; ++i)
      if (jobs[i].tri_group > 0) {
        auto it = tri_off.find(jobs[i].tri_group);
        if (it == tri_off.end()) return fail(c, GPM_E_DEVICE, "triangle scatter without edge terms");
        jobs[i].tri = tri + it->second;
      }
  }
  *frontier_used = fbytes + zbytes + tbytes;

  const size_t lds_bytes = (size_t)lds_words * 4 * kWavesPerBlock;

  // chunk ranges and queues
  for (auto& L : launches) {
    L.jbeg.assign(L.count + 1, 0);
    for (int i = 0; i < L.count; ++i) {
      const Job& J = jobs[L.first + i];
      int64_t ch = J.n_tasks > 0 ? (J.n_tasks + J.chunk - 1) / J.chunk : 0;
      L.jbeg[i + 1] = L.jbeg[i] + ch;
    }
    L.chunks = L.jbeg[L.count];
    for (int q = 0; q <= kQueues; ++q) L.qbeg[q] = L.chunks * q / kQueues;
    L.blocks = blocks;
  }

  // staging
  char* h = nullptr;
  char* dm = nullptr;
  unsigned long long* dres = nullptr;
  unsigned long long* hres = nullptr;
  if (ar) {
    h = c->na_stage.data();
    dm = ar->base;
    dres = (unsigned long long*)(ar->base + align_up(meta_bytes, 256));
    hres = c->na_res.data();
  } else {
    st = grow_host(c, &s.h_stage, &s.h_stage_bytes, meta_bytes);
    if (st) return st;
    st = grow_dev(c, &s.d_meta, &s.d_meta_bytes, meta_bytes);
    if (st) return st;
    size_t have = s.d_res_words * 8;
    st = grow_dev(c, (void**)&s.d_res, &have, all_words * 8);
    if (st) return st;
    s.d_res_words = have / 8;
    size_t hh = s.h_res_words * 8;
    st = grow_host(c, (void**)&s.h_res, &hh, all_words * 8);
    if (st) return st;
    s.h_res_words = hh / 8;
    h = (char*)s.h_stage;
    dm = (char*)s.d_meta;
    dres = s.d_res;
    hres = s.h_res;
  }
  std::memcpy(h + off_jobs, jobs.data(), sizeof(Job) * nj);
  if (!js.plans.empty()) std::memcpy(h + off_plans, js.plans.data(), sizeof(Plan) * js.plans.size());
  for (size_t i = 0; i < launches.size(); ++i) {
    std::memcpy(h + off_jbeg[i], launches[i].jbeg.data(), 8 * launches[i].jbeg.size());
    std::memcpy(h + off_qbeg[i], launches[i].qbeg, 8 * (kQueues + 1));
  }
  HIP_TRY(c, hipMemcpyAsync(dm, h, meta_bytes, hipMemcpyHostToDevice, s.stream));
  if (launch_fill_u64(dres, (int64_t)all_words, 0ull, s.stream))
    return fail(c, GPM_E_DEVICE, "fill kernel launch failed");
  HIP_TRY(c, hipEventRecord(s.ev0, s.stream));
  int n_launch = 0;
  for (size_t i = 0; i < launches.size(); ++i) {
    const LaunchPlan& L = launches[i];
    if (L.chunks == 0) continue;
    KernelArgs a{};
    a.jobs = (const Job*)(dm + off_jobs) + L.first;
    a.job_chunk_begin = (const int64_t*)(dm + off_jbeg[i]);
    a.n_jobs = L.count;
    a.lds_cap = lcap;
    a.plans = (const Plan*)(dm + off_plans);
    a.queue_begin = (const int64_t*)(dm + off_qbeg[i]);
    a.queue_cnt = dres + res_words + i * kQueues * kQueueStride;
    a.results = dres;
    a.counters = dres + res_words + q_words + 4 * i;
    a.fbuf = fbuf;
    a.wave_stride = stride;
    const bool uses_lds = (L.kinds & (kKindClique | kKindCliqueLgs | kKindTriScatter)) != 0;
    a.lds_words = uses_lds ? lds_words : 0;
    a.lgs_tile = lgs_T;
    a.lgs_lg = 31 - __builtin_clz((unsigned)c->opt_lgs_lanes);
    a.zbuf = (L.kinds & kKindCycleBlock) ? zbuf : nullptr;
    a.zstride = zstride;
    size_t lb = uses_lds ? lds_bytes : 0;
    int e;
    if (L.kinds == kKindCliqueLgsBlock) {
      a.lds_words = (int32_t)(blk_lds / 4);
      // with rows in HBM each workgroup owns one frontier region
      const int64_t max_blocks = blk_hbm_rows ? std::min<int64_t>(L.chunks, waves) : L.chunks;
      e = launch_lgs_block(c->opt_count_elements != 0, a, c->cus, max_blocks, blk_lds, s.stream);
    } else if (L.kinds == kKindCycleBlock) {
      e = launch_cycle_block(c->opt_count_elements != 0, a,
                             (int)std::min<int64_t>(cyc_blocks, L.chunks), s.stream);
    } else {
      e = launch_persistent(L.kinds, c->opt_count_elements != 0, a, L.blocks, lb, s.stream);
    }
    if (!e && n_launch < GPM_MAX_LAUNCH_STATS) {
      HIP_TRY(c, hipEventRecord(s.evl[n_launch], s.stream));
      s.lkinds[n_launch] = L.kinds;
      s.lplan[n_launch] = (int)i;
    }
    if (e) return fail(c, GPM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString((hipError_t)e));
    ++n_launch;
  }
  HIP_TRY(c, hipEventRecord(s.ev1, s.stream));
  HIP_TRY(c, hipMemcpyAsync(hres, dres, all_words * 8, hipMemcpyDeviceToHost, s.stream));
  s.h_out = hres;
  s.n_jobs = nj;
  s.n_launch = n_launch;
  s.n_lstats = std::min(n_launch, GPM_MAX_LAUNCH_STATS);
  s.n_launch_plans = (int)launches.size();
  s.counters_off = res_words + q_words;
  c->stats.waves = waves;
  c->stats.frontier_bytes = (int64_t)fbytes;
  c->stats.launches = n_launch;
  int64_t tasks = 0;
  for (auto& J : jobs) tasks += J.n_tasks;
  c->stats.tasks = tasks;
  c->stats.chunk = nj ? jobs[0].chunk : 0;
  return GPM_OK;
}

static gpm_status finish_sync(gpm_ctx* c, Slot& s) {
  HIP_TRY(c, hipStreamSynchronize(s.stream));
  s.tri_dirty = false;
  float ms = 0.f;
  if (s.n_launch > 0) HIP_TRY(c, hipEventElapsedTime(&ms, s.ev0, s.ev1));
  c->stats.kernel_ms = ms;
  c->stats.n_launch_stats = s.n_lstats;
  for (int i = 0; i < s.n_lstats; ++i) {
    float lm = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&lm, i ? s.evl[i - 1] : s.ev0, s.evl[i]));
    c->stats.launch_ms[i] = lm;
    c->stats.launch_kinds[i] = s.lkinds[i];
    const unsigned long long* ct = s.h_out + s.counters_off + 4 * (size_t)s.lplan[i];
    const bool on = c->opt_count_elements != 0;
    c->stats.launch_elements[i] = on ? (int64_t)ct[0] : -1;
    c->stats.launch_fetches[i] = on ? (int64_t)ct[1] : -1;
    c->stats.launch_written[i] = on ? (int64_t)ct[2] : -1;
    c->stats.launch_words[i] = on ? (int64_t)ct[3] : -1;
  }
  if (c->opt_count_elements) {
    int64_t t[4] = {0, 0, 0, 0};
    for (int i = 0; i < s.n_launch_plans; ++i)
      for (int f = 0; f < 4; ++f) t[f] += (int64_t)s.h_out[s.counters_off + 4 * (size_t)i + f];
    c->stats.elements = t[0];
    c->stats.list_fetches = t[1];
    c->stats.frontier_written = t[2];
    c->stats.bitmap_words = t[3];
  }
  return GPM_OK;
}

// Run a synchronous group of queries on slot 0 (the user's stream).
static gpm_status run_sync(gpm_ctx* c, JobPlanSet& js, std::vector<QueryWork>& qs,
                           bool fission, uint64_t* outs, const Arena* ar = nullptr) {
  auto t0 = std::chrono::steady_clock::now();
  Slot& s = c->slots[0];
  s.stream = c->user_stream;
  c->stats = gpm_stats{};
  c->stats.elements = -1;
  c->stats.list_fetches = -1;
  c->stats.frontier_written = -1;
  c->stats.bitmap_words = -1;
  if (js.jobs.empty()) {
    for (size_t i = 0; i < qs.size(); ++i) finish_query(qs[i], nullptr, outs + 6 * i);
    c->stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return GPM_OK;
  }
  size_t used = 0;
  size_t budget = c->budget > c->serve_frontier_in_use ? c->budget - c->serve_frontier_in_use : 0;
  gpm_status st = launch_group(c, s, js, fission, budget, &used, ar);
  if (st) return st;
  st = finish_sync(c, s);
  if (st) return st;
  for (size_t i = 0; i < qs.size(); ++i) finish_query(qs[i], s.h_out, outs + 6 * i);
  c->stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return GPM_OK;
}

// ---------------------------------------------------------------------------
// built-in patterns
// ---------------------------------------------------------------------------

static void set_edges(gpm_pattern* p, int k, std::initializer_list<std::pair<int, int>> e) {
  std::memset(p, 0, sizeof(*p));
  p->k = k;
  for (auto& x : e) {
    p->edges[2 * p->n_edges] = x.first;
    p->edges[2 * p->n_edges + 1] = x.second;
    p->n_edges++;
  }
}

static void named(const char* name, gpm_pattern* p) {
  std::string s(name);
  if (s == "edge") set_edges(p, 2, {{0, 1}});
  else if (s == "wedge") set_edges(p, 3, {{0, 1}, {0, 2}});
  else if (s == "triangle") gpm_pattern_clique(3, p);
  else if (s == "path4") set_edges(p, 4, {{0, 1}, {1, 2}, {2, 3}});
  else if (s == "star3") set_edges(p, 4, {{0, 1}, {0, 2}, {0, 3}});
  else if (s == "cycle4") set_edges(p, 4, {{0, 1}, {1, 2}, {2, 3}, {3, 0}});
  else if (s == "tailed_triangle") set_edges(p, 4, {{0, 1}, {1, 2}, {0, 2}, {2, 3}});
  else if (s == "diamond") set_edges(p, 4, {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}});
  else if (s == "clique4") gpm_pattern_clique(4, p);
  else if (s == "clique5") gpm_pattern_clique(5, p);
  else p->k = 0;
}

// ---------------------------------------------------------------------------
// serving
// ---------------------------------------------------------------------------

static gpm_status build_query(gpm_ctx* c, const gpm_query& q, JobPlanSet& js, QueryWork& qw) {
  Graph* g = find_graph(c, q.graph_id);
  if (!g) return fail(c, GPM_E_INVAL, "unknown graph id");
  qw = QueryWork{};
  qw.kind = q.kind;
  qw.first_job = (int)js.jobs.size();
  if (q.kind == GPM_QUERY_COUNT) {
    if (q.mode_or_k != GPM_VERTEX_INDUCED && q.mode_or_k != GPM_EDGE_INDUCED)
      return fail(c, GPM_E_INVAL, "bad induced mode");
    return add_count_jobs(c, *g, q.pattern, q.mode_or_k, js, qw);
  }
  if (q.kind == GPM_QUERY_MOTIFS) return add_motif_jobs(c, *g, q.mode_or_k, js, qw);
  return fail(c, GPM_E_INVAL, "bad query kind");
}

static int n_serve_slots(const gpm_ctx* c) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxSlots, c->opt_serve_slots));
}

static std::string query_key(const gpm_query& q) {
  std::string k = std::to_string(q.graph_id) + ":" + std::to_string(q.kind) + ":" +
                  std::to_string(q.mode_or_k);
  if (q.kind == GPM_QUERY_COUNT)
    for (int i = 0; i < 2 * q.pattern.n_edges; ++i) k += "," + std::to_string(q.pattern.edges[i]);
  return k;
}

// The checks a served query must pass before it gets a ticket: a known
// graph, a valid kind and mode, a valid pattern, and a pattern the graph can
// run (a DAG-only graph takes cliques only; motifs need the symmetric graph).
static gpm_status check_query(gpm_ctx* c, const gpm_query& q) {
  Graph* g = find_graph(c, q.graph_id);
  if (!g) return fail(c, GPM_E_INVAL, "unknown graph id");
  if (q.kind == GPM_QUERY_COUNT) {
    if (q.mode_or_k != GPM_VERTEX_INDUCED && q.mode_or_k != GPM_EDGE_INDUCED)
      return fail(c, GPM_E_INVAL, "bad induced mode");
    std::string err;
    gpm_status st = validate_pattern(q.pattern, &err);
    if (st) return fail(c, st, err);
    if (g->dag_only && !is_clique(q.pattern))
      return fail(c, GPM_E_UNSUPPORTED, "non-clique pattern on a DAG-only graph");
    return GPM_OK;
  }
  if (q.kind == GPM_QUERY_MOTIFS) {
    if (q.mode_or_k != 3 && q.mode_or_k != 4) return fail(c, GPM_E_INVAL, "motif size must be 3 or 4");
    if (g->dag_only) return fail(c, GPM_E_UNSUPPORTED, "motifs need the symmetric graph");
    return GPM_OK;
  }
  return fail(c, GPM_E_INVAL, "bad query kind");
}

static void complete(gpm_ctx* c, int64_t ticket, gpm_status st, const std::string& err,
                     const uint64_t* r) {
  Done d;
  d.st = st;
  d.err = err;
  if (r)
    for (int i = 0; i < 6; ++i) d.r[i] = r[i];
  c->done[ticket] = d;
}

// Collect finished launches, then admit pending queries into free slots.
// Continuous batching with cost awareness: a query whose cost is unknown or
// above serve_light_ms (measured when it last ran alone) gets a launch of
// its own, so light queries never wait behind it; light queries are batched
// together, up to max_batch per launch, in arrival order.  Admission by
// frontier memory (adaptive buffering, Sec. 7.2 (3)): a query whose buffers
// do not fit what the running launches leave free waits, first in line,
// until they finish; one that does not fit the whole budget completes with
// GPM_E_NOMEM.  A query that cannot run completes with its error status.
static gpm_status progress(gpm_ctx* c) {
  const int ns = n_serve_slots(c);
  for (int i = 1; i <= ns; ++i) {
    Slot& s = c->slots[i];
    if (!s.busy) continue;
    hipError_t e = hipEventQuery(s.ev1);
    if (e == hipErrorNotReady) continue;
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);  // result copy queued after ev1
    if (e != hipSuccess) {
      const std::string msg = std::string("serving launch: ") + hipGetErrorString(e);
      for (auto& qw : s.queries) complete(c, qw.ticket, GPM_E_DEVICE, msg, nullptr);
    } else {
      if (s.queries.size() == 1 && s.n_launch > 0) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s.ev0, s.ev1) == hipSuccess) c->qcost[s.qkeys[0]] = ms;
      }
      for (auto& qw : s.queries) {
        uint64_t r[6];
        finish_query(qw, s.h_out, r);
        complete(c, qw.ticket, GPM_OK, "", r);
      }
          s.tri_dirty = false;
    }
    s.queries.clear();
    s.qkeys.clear();
    s.busy = false;
    s.heavy = false;
    c->serve_frontier_in_use -= s.frontier_bytes_in_use;
    s.frontier_bytes_in_use = 0;
  }
  auto light = [&](const gpm_query& q) {
    auto it = c->qcost.find(query_key(q));
    return it != c->qcost.end() && it->second <= (double)c->opt_serve_light_ms;
  };
  auto busy_slots = [&]() {
    int b = 0;
    for (int i = 1; i <= ns; ++i) b += c->slots[i].busy ? 1 : 0;
    return b;
  };
  // heavy (or not yet measured) queries run alone and may hold at most half
  // of the slots, so light queries keep slots of their own
  int heavy_busy = 0;
  for (int i = 1; i <= ns; ++i)
    if (c->slots[i].busy && c->slots[i].heavy) ++heavy_busy;
  const int heavy_max = std::max(1, ns / 2);
  bool blocked = false;   // the head of the line waits for memory
  for (int i = 1; i <= ns && !c->pending.empty() && !blocked; ++i) {
    Slot& s = c->slots[i];
    if (s.busy) continue;
    gpm_status st = slot_init(c, s, nullptr);
    if (st) return st;
    size_t avail = c->budget > c->serve_frontier_in_use ? c->budget - c->serve_frontier_in_use : 0;
    JobPlanSet js;
    std::vector<QueryWork> qs;
    std::vector<Pending> taken;
    std::vector<std::string> keys;
    // the group starts at the first pending query this slot may take
    auto first = c->pending.begin();
    if (heavy_busy >= heavy_max)
      while (first != c->pending.end() && !light(first->q)) ++first;
    if (first == c->pending.end()) continue;  // only heavy work waits: keep the slot for light
    const bool batchable = light(first->q);
    for (auto it = first; it != c->pending.end() && (int64_t)qs.size() < c->opt_max_batch;) {
      if (!qs.empty() && (!batchable || !light(it->q))) {
        ++it;
        continue;
      }
      Pending pq = *it;
      QueryWork qw;
      size_t before = js.jobs.size();
      size_t pbefore = js.plans.size();
      st = build_query(c, pq.q, js, qw);
      if (st) {
        // a query that cannot run completes with its status
        js.jobs.resize(before);
        js.need_words.resize(before);
        js.plans.resize(pbefore);
        complete(c, pq.ticket, st, c->err, nullptr);
        it = c->pending.erase(it);
        continue;
      }
      // admission by frontier memory: the group's per-wave region must leave
      // room for a useful number of waves
      int64_t stride = 0;
      for (auto w : js.need_words) stride = std::max(stride, w);
      size_t min_bytes = (size_t)align_up((size_t)stride, 64) * 4 * (size_t)(c->cus);
      if (min_bytes > avail) {
        js.jobs.resize(before);
        js.need_words.resize(before);
        js.plans.resize(pbefore);
        if (!qs.empty()) break;   // the group is full; this query starts the next one
        if (busy_slots() > 0) {
          blocked = true;           // memory frees when a running launch finishes
          if (!it->waited) {
            it->waited = true;
            ++c->serve_memory_waits;
          }
          break;
        }
        // nothing else holds memory: the query does not fit the whole budget
        complete(c, pq.ticket, GPM_E_NOMEM,
                 "the query's frontier buffers exceed the memory budget", nullptr);
        it = c->pending.erase(it);
        continue;
      }
      qw.ticket = pq.ticket;
      qs.push_back(qw);
      taken.push_back(pq);
      keys.push_back(query_key(pq.q));
      it = c->pending.erase(it);
      if (!batchable) break;
    }
    if (qs.empty()) continue;
    if (js.jobs.empty()) {
      for (auto& qw : qs) {
        uint64_t r[6];
        finish_query(qw, nullptr, r);
        complete(c, qw.ticket, GPM_OK, "", r);
      }
      continue;
    }
    size_t used = 0;
    st = launch_group(c, s, js, false, avail, &used);
    if (st) {
      if (st == GPM_E_NOMEM && busy_slots() > 0) {
        // not enough memory beside the running launches: back to the head of
        // the line, in arrival order, until one of them finishes
        if (!taken[0].waited) {
          taken[0].waited = true;
          ++c->serve_memory_waits;
        }
        for (auto it = taken.rbegin(); it != taken.rend(); ++it) c->pending.push_front(*it);
        blocked = true;
      } else {
        const std::string msg = c->err;
        for (auto& qw : qs) complete(c, qw.ticket, st, msg, nullptr);
      }
      continue;
    }
    s.queries = qs;
    s.qkeys = keys;
    s.busy = true;
    c->serve_admitted += (int64_t)qs.size();
    s.heavy = !batchable;
    if (s.heavy) ++heavy_busy;
    s.frontier_bytes_in_use = used;
    c->serve_frontier_in_use += used;
  }
  return GPM_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// Canonical-form checks of a CSR (Table 3's note: symmetric, no loops, no
// duplicates; sorted lists, Sec. 4.2), plus symmetry / acyclicity with
// GPM_VALIDATE.
static gpm_status validate_csr(const HostCSR& h, uint32_t flags, std::string* why) {
  const int64_t n = h.n;
  const int64_t nnz = (int64_t)h.col.size();
  const bool dag = (flags & GPM_CSR_DAG) != 0;
  const bool sym = !dag;
  auto bad = [&](const char* m) {
    *why = m;
    return GPM_E_CSR;
  };
  if (h.rp[0] != 0 || h.rp[n] != nnz) return bad("row_ptr[0] != 0 or row_ptr[n] != nnz");
  for (int64_t u = 0; u < n; ++u) {
    if (h.rp[u + 1] < h.rp[u]) return bad("row_ptr not monotone");
    for (int64_t p = h.rp[u]; p < h.rp[u + 1]; ++p) {
      int32_t v = h.col[p];
      if (v < 0 || v >= n) return bad("neighbour id out of range");
      if (v == u) return bad("self loop");
      if (p > h.rp[u] && h.col[p - 1] >= v) return bad("neighbour list unsorted or duplicated");
    }
  }
  auto has = [&](int64_t u, int32_t v) {
    return std::binary_search(h.col.begin() + h.rp[u], h.col.begin() + h.rp[u + 1], v);
  };
  if (flags & GPM_VALIDATE) {
    for (int64_t u = 0; u < n; ++u)
      for (int64_t p = h.rp[u]; p < h.rp[u + 1]; ++p) {
        bool back = has(h.col[p], (int32_t)u);
        if (sym && !back) return bad("graph not symmetric");
        if (dag && back) return bad("DAG holds both directions of an edge");
      }
    if (dag) {  // acyclic (Kahn)
      std::vector<int64_t> indeg(n, 0);
      for (int64_t p = 0; p < nnz; ++p) indeg[h.col[p]]++;
      std::vector<int64_t> q;
      for (int64_t u = 0; u < n; ++u)
        if (!indeg[u]) q.push_back(u);
      int64_t seen = 0;
      while (!q.empty()) {
        int64_t u = q.back();
        q.pop_back();
        ++seen;
        for (int64_t p = h.rp[u]; p < h.rp[u + 1]; ++p)
          if (--indeg[h.col[p]] == 0) q.push_back(h.col[p]);
      }
      if (seen != n) return bad("oriented graph has a cycle");
    }
  } else if (sym && (nnz & 1)) {
    return bad("symmetric graph with an odd number of entries");
  }
  return GPM_OK;
}

extern "C" {

gpm_status gpm_validate_csr(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                            uint32_t flags) {
  if (n < 0 || nnz < 0 || n >= (int64_t)INT32_MAX || !row_ptr || (nnz > 0 && !col))
    return GPM_E_INVAL;
  if ((flags & GPM_CSR_DAG) && (flags & GPM_CSR_SYMMETRIC)) return GPM_E_INVAL;
  if (flags & GPM_PTRS_DEVICE) return GPM_E_INVAL;
  HostCSR h;
  h.n = n;
  h.rp.assign(row_ptr, row_ptr + n + 1);
  if (nnz) h.col.assign(col, col + nnz);
  std::string why;
  return validate_csr(h, flags, &why);
}

gpm_status gpm_create(gpm_ctx** out, int device, void* hip_stream, size_t hbm_budget_bytes) {
  if (!out) return GPM_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GPM_E_DEVICE;
  if (device < 0 || device >= ndev) return GPM_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return GPM_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return GPM_E_DEVICE;
  auto* c = new (std::nothrow) gpm_ctx();
  if (!c) return GPM_E_NOMEM;
  c->device = device;
  c->user_stream = (hipStream_t)hip_stream;
  c->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess && lds > 0)
      c->lds_block_max = lds;
  }
  size_t freeb = 0, total = 0;
  if (hipMemGetInfo(&freeb, &total) != hipSuccess) {
    delete c;
    return GPM_E_DEVICE;
  }
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : freeb / 10 * 9;
  c->slots[0].stream = c->user_stream;
  // the allocation-free count: this device's scratch address (looked up once
  // per device, the device current), the synchronous slot's events, and host
  // staging reserved now so that the call itself allocates nothing
  if (scratch_address(device, &c->scratch) != 0 ||
      slot_init(c, c->slots[0], c->user_stream) != GPM_OK) {
    slot_free(c->slots[0]);
    delete c;
    return GPM_E_DEVICE;
  }
  c->na_stage.resize(kNoallocStageBytes);
  c->na_res.resize(kNoallocResultWords);
  *out = c;
  return GPM_OK;
}

gpm_status gpm_destroy(gpm_ctx* c) {
  if (!c) return GPM_OK;
  (void)hipSetDevice(c->device);
  for (auto& s : c->slots) slot_free(s);
  for (auto& kv : c->graphs) free_graph(*kv.second);
  dev_free(c->d_list);
  if (c->h_list) (void)hipHostFree(c->h_list);
  delete c;
  return GPM_OK;
}

const char* gpm_last_error(const gpm_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

gpm_status gpm_set_option(gpm_ctx* c, const char* key, int64_t v) {
  if (!c || !key) return GPM_E_INVAL;
  std::string k(key);
  if (k == "granularity") { if (v < 0 || v > 2) return fail(c, GPM_E_INVAL, "granularity 0..2"); c->opt_granularity = v; }
  else if (k == "chunk") { if (v < 0 || v > (1 << 20)) return fail(c, GPM_E_INVAL, "chunk"); c->opt_chunk = v; }
  else if (k == "waves_per_cu") { if (v < 0 || v > 32) return fail(c, GPM_E_INVAL, "waves_per_cu 0..32"); c->opt_waves_per_cu = v; }
  else if (k == "setop") { if (v < 0 || v > 3) return fail(c, GPM_E_INVAL, "setop 0..3"); c->opt_setop = v; }
  else if (k == "clique_lds") c->opt_clique_lds = v != 0;
  else if (k == "lds_tile") { if (v < 0 || v > 4096) return fail(c, GPM_E_INVAL, "lds_tile 0..4096"); c->opt_lds_tile = v; }
  else if (k == "rename") { if (v < 0 || v > 1) return fail(c, GPM_E_INVAL, "rename 0..1"); c->opt_rename = v; }
  else if (k == "count_elements") c->opt_count_elements = v != 0;
  else if (k == "clique_algo") { if (v < 0 || v > 2) return fail(c, GPM_E_INVAL, "clique_algo 0..2"); c->opt_clique_algo = v; }
  else if (k == "lgs_split") c->opt_lgs_split = v != 0;
  else if (k == "lgs_block") c->opt_lgs_block = v != 0;
  else if (k == "lgs_lanes") {
    if (v < 4 || v > 64 || (v & (v - 1))) return fail(c, GPM_E_INVAL, "lgs_lanes 4, 8, 16, 32 or 64");
    c->opt_lgs_lanes = v;
  }
  else if (k == "decompose") c->opt_decompose = v != 0;
  else if (k == "edge_terms") { if (v < 0 || v > 1) return fail(c, GPM_E_INVAL, "edge_terms 0..1"); c->opt_edge_terms = v; }
  else if (k == "cycle4_mode") { if (v < 0 || v > 2) return fail(c, GPM_E_INVAL, "cycle4_mode 0..2"); c->opt_cycle4_mode = v; }
  else if (k == "cycle4_split") { if (v < 1 || v > 1024) return fail(c, GPM_E_INVAL, "cycle4_split 1..1024"); c->opt_cycle4_split = v; }
  else if (k == "cycle4_batch") { if (v < 2 || v > (1 << 30)) return fail(c, GPM_E_INVAL, "cycle4_batch 2..2^30"); c->opt_cycle4_batch = v; }
  else if (k == "cycle4_algo") { if (v < 0 || v > 2) return fail(c, GPM_E_INVAL, "cycle4_algo 0..2"); c->opt_cycle4_algo = v; }
  else if (k == "leaf_cap") { if (v < 0 || v > (1 << 20)) return fail(c, GPM_E_INVAL, "leaf_cap 0..2^20"); c->opt_leaf_cap = v; }
  else if (k == "lgs_max") { if (v < 64 || v > kLgsMaxVertices) return fail(c, GPM_E_INVAL, "lgs_max 64..2048"); c->opt_lgs_max = v; }
  else if (k == "lgs_tile") { if (v < 64 || v > 256) return fail(c, GPM_E_INVAL, "lgs_tile 64..256"); c->opt_lgs_tile = v; }
  else if (k == "autotune") c->opt_autotune = v != 0;
  else if (k == "tune_min_ms") { if (v < 0) return fail(c, GPM_E_INVAL, "tune_min_ms >= 0"); c->opt_tune_min_ms = v; }
  else if (k == "max_batch") { if (v < 1) return fail(c, GPM_E_INVAL, "max_batch >= 1"); c->opt_max_batch = v; }
  else if (k == "serve_slots") { if (v < 1 || v > kMaxSlots) return fail(c, GPM_E_INVAL, "serve_slots 1..4"); c->opt_serve_slots = v; }
  else if (k == "serve_light_ms") { if (v < 0) return fail(c, GPM_E_INVAL, "serve_light_ms >= 0"); c->opt_serve_light_ms = v; }
  else if (k == "max_pending") { if (v < 1) return fail(c, GPM_E_INVAL, "max_pending >= 1"); c->opt_max_pending = v; }
  else if (k == "budget") { if (v < 0) return fail(c, GPM_E_INVAL, "budget >= 0"); c->budget = (size_t)v; }
  else return fail(c, GPM_E_INVAL, "unknown option " + k);
  return GPM_OK;
}

gpm_status gpm_get_stats(const gpm_ctx* c, gpm_stats* out) {
  if (!c || !out) return GPM_E_INVAL;
  *out = c->stats;
  return GPM_OK;
}

gpm_status gpm_load_csr(gpm_ctx* c, int64_t n, int64_t nnz, const int64_t* row_ptr,
                        const int32_t* col, uint32_t flags, int32_t* graph_id_out) {
  if (!c || !graph_id_out) return GPM_E_INVAL;
  if (n < 0 || nnz < 0 || n >= (int64_t)INT32_MAX) return fail(c, GPM_E_INVAL, "bad n or nnz");
  if (!row_ptr || (nnz > 0 && !col)) return fail(c, GPM_E_INVAL, "null CSR array");
  const bool dag = (flags & GPM_CSR_DAG) != 0;
  if (dag && (flags & GPM_CSR_SYMMETRIC)) return fail(c, GPM_E_INVAL, "SYMMETRIC and DAG both set");
  HIP_TRY(c, hipSetDevice(c->device));
  auto g = std::make_unique<Graph>();
  g->dag_only = dag;
  HostCSR& h = g->host;
  h.n = n;
  h.rp.resize(n + 1);
  h.col.resize(nnz);
  if (flags & GPM_PTRS_DEVICE) {
    HIP_TRY(c, hipMemcpy(h.rp.data(), row_ptr, (n + 1) * 8, hipMemcpyDeviceToHost));
    if (nnz) HIP_TRY(c, hipMemcpy(h.col.data(), col, nnz * 4, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(h.rp.data(), row_ptr, (n + 1) * 8);
    if (nnz) std::memcpy(h.col.data(), col, nnz * 4);
  }
  {
    std::string why;
    gpm_status vs = validate_csr(h, flags, &why);
    if (vs) return fail(c, vs, why);
  }
  g->m = dag ? nnz : nnz / 2;
  if (!dag) {
    gpm_status st = upload_view(c, h, false, &g->sym, &g->bytes);
    if (st) { free_graph(*g); return st; }
  }
  int32_t id = c->next_graph++;
  c->graphs[id] = std::move(g);
  *graph_id_out = id;
  return GPM_OK;
}

gpm_status gpm_unload(gpm_ctx* c, int32_t id) {
  if (!c) return GPM_E_INVAL;
  auto it = c->graphs.find(id);
  if (it == c->graphs.end()) return fail(c, GPM_E_INVAL, "unknown graph id");
  for (auto& s : c->slots)
    if (s.busy) return fail(c, GPM_E_BUSY, "serving launches in flight");
  (void)hipDeviceSynchronize();
  free_graph(*it->second);
  c->graphs.erase(it);
  return GPM_OK;
}

gpm_status gpm_prepare(gpm_ctx* c, int32_t id) {
  if (!c) return GPM_E_INVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  Graph* g = find_graph(c, id);
  if (!g) return fail(c, GPM_E_INVAL, "unknown graph id");
  gpm_status st = ensure_dag(c, *g);
  if (st) return st;
  st = ensure_lgs(c, *g, c->opt_lgs_max);
  if (st) return st;
  if (g->dag_only) return GPM_OK;
  st = ensure_ren(c, *g);
  if (st) return st;
  st = ensure_lower(c, *g);
  if (st) return st;
  return ensure_cycle(c, *g);
}

gpm_status gpm_graph_info(gpm_ctx* c, int32_t id, gpm_graph_meta* out) {
  if (!c || !out) return GPM_E_INVAL;
  Graph* g = find_graph(c, id);
  if (!g) return fail(c, GPM_E_INVAL, "unknown graph id");
  gpm_status st = ensure_dag(c, *g);
  if (st) return st;
  out->n = g->host.n;
  out->m = g->m;
  out->max_degree = g->dag_only ? 0 : g->sym.max_deg;
  out->max_out_degree = g->dag.max_deg;
  out->device_bytes = (int64_t)g->bytes;
  return GPM_OK;
}

gpm_status gpm_pattern_clique(int k, gpm_pattern* out) {
  if (!out || k < 1 || k > GPM_MAX_K) return GPM_E_PATTERN;
  std::memset(out, 0, sizeof(*out));
  out->k = k;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j) {
      out->edges[2 * out->n_edges] = i;
      out->edges[2 * out->n_edges + 1] = j;
      out->n_edges++;
    }
  return GPM_OK;
}

gpm_status gpm_pattern_named(const char* name, gpm_pattern* out) {
  if (!name || !out) return GPM_E_INVAL;
  named(name, out);
  return out->k ? GPM_OK : GPM_E_INVAL;
}

gpm_status gpm_pattern_from_edges(int k, int n_edges, const int32_t* edges, gpm_pattern* out) {
  if (!out || (n_edges > 0 && !edges)) return GPM_E_INVAL;
  if (n_edges < 0 || n_edges > GPM_MAX_PATTERN_EDGES) return GPM_E_PATTERN;
  gpm_pattern p;
  std::memset(&p, 0, sizeof(p));
  p.k = k;
  p.n_edges = n_edges;
  for (int i = 0; i < 2 * n_edges; ++i) p.edges[i] = edges[i];
  gpm_status st = validate_pattern(p, nullptr);
  if (st) return st;
  *out = p;
  return GPM_OK;
}

gpm_status gpm_plan(const gpm_pattern* p, int mode, gpm_plan_info* out) {
  if (!p || !out) return GPM_E_INVAL;
  if (mode != GPM_VERTEX_INDUCED && mode != GPM_EDGE_INDUCED) return GPM_E_INVAL;
  HostPlan hp;
  gpm_status st = validate_pattern(*p, nullptr);
  if (st) return st;
  st = build_plan(*p, mode, is_clique(*p) && p->k >= 3, &hp, nullptr, true);
  if (st) return st;
  std::memset(out, 0, sizeof(*out));
  out->count_only_r = hp.choose_r;
  out->k = hp.k;
  out->clique = hp.clique;
  out->aut = hp.aut;
  out->root_bound = hp.plan.root_bound;
  out->n_buffers = hp.n_buffers;
  for (int d = 0; d < hp.k; ++d) out->order[d] = hp.order[d];
  out->n_restrictions = (int)hp.restrictions.size();
  for (size_t i = 0; i < hp.restrictions.size(); ++i) {
    out->restrictions[2 * i] = hp.restrictions[i].first;
    out->restrictions[2 * i + 1] = hp.restrictions[i].second;
  }
  return GPM_OK;
}

gpm_status gpm_frontier_waves(int64_t free_bytes, int32_t x_levels, int64_t cap_elems,
                              int64_t n_tasks, int64_t max_resident, int64_t* waves_out) {
  if (!waves_out || free_bytes < 0 || x_levels < 0 || cap_elems < 0 || n_tasks < 0 ||
      max_resident < 1)
    return GPM_E_INVAL;
  const int64_t per = (int64_t)x_levels * cap_elems * 4;
  int64_t w = per > 0 ? free_bytes / per : max_resident;
  if (per > 0 && w < 1) return GPM_E_NOMEM;
  w = std::min(w, std::max<int64_t>(n_tasks, 1));
  w = std::min(w, max_resident);
  *waves_out = w;
  return GPM_OK;
}

static gpm_status count_once(gpm_ctx* c, const gpm_query& q, uint64_t* out0) {
  JobPlanSet js;
  std::vector<QueryWork> qs(1);
  gpm_status st = build_query(c, q, js, qs[0]);
  if (st) return st;
  uint64_t out[6];
  st = run_sync(c, js, qs, true, out);
  if (st) return st;
  *out0 = out[0];
  return GPM_OK;
}

gpm_status gpm_count(gpm_ctx* c, int32_t graph_id, const gpm_pattern* pattern, int mode,
                     uint64_t* count_out) {
  if (!c || !pattern || !count_out) return GPM_E_INVAL;
  gpm_query q{};
  q.graph_id = graph_id;
  q.kind = GPM_QUERY_COUNT;
  q.mode_or_k = mode;
  q.pattern = *pattern;
  HIP_TRY(c, hipSetDevice(c->device));
  if (!c->opt_autotune || c->tuning) return count_once(c, q, count_out);

  const std::string key = tune_key(graph_id, *pattern, mode);
  auto space = tune_space(*pattern, mode);
  // remember the caller's knob values; tuned values apply to this call only
  std::vector<std::pair<int64_t*, int64_t>> saved;
  for (auto& kv : space) saved.push_back({knob(c, kv.first), *knob(c, kv.first)});
  auto restore = [&]() {
    for (auto& sv : saved) *sv.first = sv.second;
  };
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    for (auto& kv : it->second) *knob(c, kv.first) = kv.second;
    gpm_status st = count_once(c, q, count_out);
    restore();
    c->stats.variant = 1;
    return st;
  }
  uint64_t ref = 0;
  gpm_status st = count_once(c, q, &ref);
  if (st) { restore(); return st; }
  double best = c->stats.kernel_ms;
  std::vector<std::pair<std::string, int64_t>> cfg;
  for (auto& kv : space) cfg.push_back({kv.first, *knob(c, kv.first)});
  if (best >= (double)c->opt_tune_min_ms) {
    c->tuning = true;
    for (size_t d = 0; d < space.size(); ++d) {
      for (int64_t v : space[d].second) {
        if (v == cfg[d].second) continue;
        for (auto& kv : cfg) *knob(c, kv.first) = kv.second;
        *knob(c, space[d].first) = v;
        uint64_t got = 0;
        st = count_once(c, q, &got);
        if (st) break;
        if (got != ref) {
          c->tuning = false;
          restore();
          return fail(c, GPM_E_DEVICE, "autotuner: configurations disagree on the count");
        }
        if (c->stats.kernel_ms < best) {
          best = c->stats.kernel_ms;
          cfg[d].second = v;
        }
      }
      if (st) break;
    }
    c->tuning = false;
    if (st) { restore(); return st; }
  }
  c->tuned[key] = cfg;
  restore();
  *count_out = ref;
  return GPM_OK;
}

gpm_status gpm_count_noalloc(gpm_ctx* c, int32_t graph_id, const gpm_pattern* pattern,
                             int mode, uint64_t* count_out) {
  if (!c || !pattern || !count_out) return GPM_E_INVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  if (!c->scratch) return fail(c, GPM_E_DEVICE, "no device scratch");
  gpm_query q{};
  q.graph_id = graph_id;
  q.kind = GPM_QUERY_COUNT;
  q.mode_or_k = mode;
  q.pattern = *pattern;
  // the knob values the autotuner chose for this triple, as gpm_count uses them
  std::vector<std::pair<int64_t*, int64_t>> saved;
  if (c->opt_autotune) {
    auto it = c->tuned.find(tune_key(graph_id, *pattern, mode));
    if (it != c->tuned.end())
      for (auto& kv : it->second) {
        int64_t* k = knob(c, kv.first);
        saved.push_back({k, *k});
        *k = kv.second;
      }
  }
  c->noalloc = true;
  JobPlanSet js;
  std::vector<QueryWork> qs(1);
  gpm_status st = build_query(c, q, js, qs[0]);
  uint64_t out[6];
  if (!st) {
    const Arena ar{(char*)c->scratch, kScratchBytes};
    st = run_sync(c, js, qs, true, out, &ar);
  }
  c->noalloc = false;
  for (auto& sv : saved) *sv.first = sv.second;
  if (st) return st;
  *count_out = out[0];
  return GPM_OK;
}

gpm_status gpm_motifs(gpm_ctx* c, int32_t graph_id, int k, uint64_t* counts_out, size_t len) {
  if (!c || !counts_out) return GPM_E_INVAL;
  if ((k == 3 && len < 2) || (k == 4 && len < 6)) return fail(c, GPM_E_INVAL, "counts_out too short");
  gpm_query q{};
  q.graph_id = graph_id;
  q.kind = GPM_QUERY_MOTIFS;
  q.mode_or_k = k;
  HIP_TRY(c, hipSetDevice(c->device));
  JobPlanSet js;
  std::vector<QueryWork> qs(1);
  gpm_status st = build_query(c, q, js, qs[0]);
  if (st) return st;
  uint64_t out[6];
  st = run_sync(c, js, qs, true, out);
  if (st) return st;
  for (int i = 0; i < (k == 3 ? 2 : 6); ++i) counts_out[i] = out[i];
  return GPM_OK;
}

gpm_status gpm_list(gpm_ctx* c, int32_t graph_id, const gpm_pattern* pattern, int mode,
                    int32_t* out, int64_t cap, uint64_t* count_out) {
  if (!c || !pattern || !count_out) return GPM_E_INVAL;
  if (cap < 0 || (cap > 0 && !out)) return fail(c, GPM_E_INVAL, "bad output buffer");
  if (mode != GPM_VERTEX_INDUCED && mode != GPM_EDGE_INDUCED)
    return fail(c, GPM_E_INVAL, "bad induced mode");
  HIP_TRY(c, hipSetDevice(c->device));
  Graph* gp = find_graph(c, graph_id);
  if (!gp) return fail(c, GPM_E_INVAL, "unknown graph id");
  Graph& g = *gp;
  const gpm_pattern& p = *pattern;
  std::string err;
  gpm_status st = validate_pattern(p, &err);
  if (st) return fail(c, st, err);
  const bool clique = is_clique(p);
  if (g.dag_only && !clique)
    return fail(c, GPM_E_UNSUPPORTED, "non-clique pattern on a DAG-only graph");
  c->stats = gpm_stats{};
  c->stats.elements = c->stats.list_fetches = c->stats.frontier_written = -1;
  c->stats.bitmap_words = -1;
  const int64_t n = g.host.n;
  if (n < p.k || (p.k >= 2 && g.m == 0)) {
    *count_out = 0;
    return GPM_OK;
  }

  ListArgs a{};
  a.k = p.k;
  a.out = out;
  a.out_cap = cap;
  HostPlan hp;
  // cliques (k >= 2) on the DAG: each clique once, with no symmetry bounds;
  // other patterns on the symmetric graph (relabelled unless "rename" is 0)
  const bool on_dag = clique && p.k >= 2;
  st = build_plan(p, mode, on_dag, &hp, &err);
  if (st) return fail(c, st, err);
  a.plan = hp.plan;
  for (int d = 0; d < p.k; ++d) a.out_col[d] = (int8_t)hp.order[d];
  GraphView* V = nullptr;
  if (on_dag) {
    st = ensure_dag(c, g);
    if (st) return st;
    V = &g.dag;
    a.ids = g.dag_only ? nullptr : g.ren_ids;
    a.ordered = g.dag_ordered ? 1 : 0;
    a.task_src = g.dag.src;
    a.task_dst = g.dag.col;
    a.n_tasks = g.dag.nnz;
  } else {
    const bool ren = c->opt_rename != 0 && !g.dag_only;
    if (ren) {
      st = ensure_ren(c, g);
      if (st) return st;
    }
    V = g.dag_only ? &g.dag : (ren ? &g.ren : &g.sym);
    if (g.dag_only) {
      st = ensure_dag(c, g);
      if (st) return st;
    }
    a.ids = ren ? g.ren_ids : nullptr;
    if (p.k == 1) {
      a.n_tasks = n;  // vertex tasks
    } else if (ren) {
      // root edges (v0, v1) with v1 < v0: every plan of k >= 2 bounds v1 by
      // v0 or is a clique (on the DAG above)
      a.task_src = g.ren_lo_src;
      a.task_dst = g.ren_lo_dst;
      a.n_tasks = g.ren_n_lo;
    } else {
      st = ensure_lower(c, g);
      if (st) return st;
      a.task_src = g.lo_src;
      a.task_dst = g.lo_dst;
      a.n_tasks = g.n_lo;
    }
    if (p.k >= 2 && !hp.plan.root_bound) {
      // a root edge with no bound would need both directions
      if (!V->src) {
        const HostCSR& H = ren ? g.ren_host : g.host;
        std::vector<int32_t> src(H.col.size());
        for (int64_t u = 0; u < n; ++u)
          for (int64_t q = H.rp[u]; q < H.rp[u + 1]; ++q) src[q] = (int32_t)u;
        st = dev_upload(c, &V->src, src.data(), src.size());
        if (st) return st;
        g.bytes += src.size() * 4;
      }
      a.task_src = V->src;
      a.task_dst = V->col;
      a.n_tasks = V->nnz;
    }
  }
  a.rp = V->rp;
  a.col = V->col;
  const int64_t fcap = std::max<int64_t>(V->max_deg, 1);
  a.cap = (int32_t)fcap;
  a.chunk = p.k <= 2 ? 4096 : 8;

  Slot& s = c->slots[0];
  s.stream = c->user_stream;
  st = slot_init(c, s, s.stream);
  if (st) return st;
  const int64_t stride = (int64_t)align_up((size_t)(hp.n_buffers * fcap), 64);
  const int64_t max_resident = (int64_t)c->cus * 16;
  int64_t waves = max_resident;
  if (stride > 0) {
    const size_t budget = c->budget > c->serve_frontier_in_use ? c->budget - c->serve_frontier_in_use : 0;
    gpm_status s2 = gpm_frontier_waves((int64_t)budget, 1, stride, max_resident, max_resident, &waves);
    if (s2 || waves < kWavesPerBlock)
      return fail(c, GPM_E_NOMEM, "frontier buffers do not fit the memory budget");
  }
  waves = std::max<int64_t>(kWavesPerBlock, waves / kWavesPerBlock * kWavesPerBlock);
  const int blocks = (int)(waves / kWavesPerBlock);
  if (stride > 0) {
    st = grow_dev(c, (void**)&s.d_fbuf, &s.d_fbuf_bytes, (size_t)waves * (size_t)stride * 4);
    if (st) return st;
    a.fbuf = s.d_fbuf;
    a.wave_stride = stride;
  }
  // counters: [0] the matches found, [1] the task queue
  if (!c->d_list) HIP_TRY(c, hipMalloc((void**)&c->d_list, 2 * sizeof(unsigned long long)));
  if (!c->h_list)
    HIP_TRY(c, hipHostMalloc((void**)&c->h_list, 2 * sizeof(unsigned long long), hipHostMallocDefault));
  a.rows = c->d_list;
  a.queue = c->d_list + 1;
  auto t0 = std::chrono::steady_clock::now();
  if (launch_fill_u64(c->d_list, 2, 0ull, s.stream))
    return fail(c, GPM_E_DEVICE, "fill kernel launch failed");
  HIP_TRY(c, hipEventRecord(s.ev0, s.stream));
  if (launch_list(a, blocks, s.stream)) return fail(c, GPM_E_DEVICE, "listing kernel launch failed");
  HIP_TRY(c, hipEventRecord(s.ev1, s.stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_list, c->d_list, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s.stream));
  HIP_TRY(c, hipStreamSynchronize(s.stream));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, s.ev0, s.ev1));
  c->stats.kernel_ms = ms;
  c->stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *count_out = (uint64_t)c->h_list[0];
  return GPM_OK;
}

gpm_status gpm_count_batch(gpm_ctx* c, int32_t nq, const gpm_query* queries, uint64_t* outs) {
  if (!c || nq < 0 || (nq > 0 && (!queries || !outs))) return GPM_E_INVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  JobPlanSet js;
  std::vector<QueryWork> qs(nq);
  for (int i = 0; i < nq; ++i) {
    gpm_status st = build_query(c, queries[i], js, qs[i]);
    if (st) return st;
  }
  return run_sync(c, js, qs, false, outs);
}

gpm_status gpm_submit(gpm_ctx* c, const gpm_query* q, int64_t* ticket_out) {
  if (!c || !q || !ticket_out) return GPM_E_INVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  if ((int64_t)c->pending.size() >= c->opt_max_pending) return fail(c, GPM_E_BUSY, "pending list full");
  gpm_status st = check_query(c, *q);
  if (st) return st;
  int64_t t = c->next_ticket++;
  c->pending.push_back(Pending{*q, t});
  c->issued.insert(t);
  *ticket_out = t;
  return progress(c);
}

gpm_status gpm_poll(gpm_ctx* c, int64_t ticket, int* done_out, uint64_t* counts_out) {
  if (!c || !done_out) return GPM_E_INVAL;
  *done_out = 0;
  if (!c->issued.count(ticket)) return fail(c, GPM_E_INVAL, "unknown or already collected ticket");
  HIP_TRY(c, hipSetDevice(c->device));
  gpm_status st = progress(c);
  if (st) return st;
  auto it = c->done.find(ticket);
  if (it == c->done.end()) return GPM_OK;
  Done d = std::move(it->second);
  c->done.erase(it);
  c->issued.erase(ticket);
  *done_out = 1;
  if (d.st != GPM_OK) return fail(c, d.st, d.err);
  if (counts_out)
    for (int i = 0; i < 6; ++i) counts_out[i] = d.r[i];
  return GPM_OK;
}

gpm_status gpm_wait(gpm_ctx* c, int64_t ticket, int64_t timeout_ns, uint64_t* counts_out) {
  if (!c) return GPM_E_INVAL;
  auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    int done = 0;
    gpm_status st = gpm_poll(c, ticket, &done, counts_out);
    if (st || done) return st;
    auto el = std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
    if (timeout_ns >= 0 && el >= timeout_ns) return fail(c, GPM_E_TIMEOUT, "wait timed out");
  }
}

gpm_status gpm_serve_state(gpm_ctx* c, gpm_serve_info* out) {
  if (!c || !out) return GPM_E_INVAL;
  gpm_serve_info r{};
  r.pending = (int64_t)c->pending.size();
  r.completed = (int64_t)c->done.size();
  for (int i = 1; i <= kMaxSlots; ++i) {
    r.running += (int64_t)c->slots[i].queries.size();
    r.busy_slots += c->slots[i].busy ? 1 : 0;
  }
  r.frontier_in_use = (int64_t)c->serve_frontier_in_use;
  r.budget = (int64_t)c->budget;
  r.memory_waits = c->serve_memory_waits;
  r.admitted = c->serve_admitted;
  *out = r;
  return GPM_OK;
}

gpm_status gpm_inflight(gpm_ctx* c, int64_t* count_out) {
  if (!c || !count_out) return GPM_E_INVAL;
  int64_t n = (int64_t)c->pending.size() + (int64_t)c->done.size();
  for (auto& s : c->slots) n += (int64_t)s.queries.size();
  *count_out = n;
  return GPM_OK;
}

}  // extern "C"
