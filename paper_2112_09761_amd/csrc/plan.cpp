// Search-plan builder (the paper's pattern analyzer, Sec. 4 "System
// Interface"): matching order, symmetry order and the per-depth set
// operations of the depth-first walk.
#include "plan.h"

#include <algorithm>
#include <cstring>

namespace gpm {

int validate_pattern(const gpm_pattern& p, std::string* err) {
  if (p.k < 1 || p.k > kMaxK) {
    if (err) *err = "pattern: k must be in [1, 8]";
    return GPM_E_PATTERN;
  }
  if (p.n_edges < 0 || p.n_edges > GPM_MAX_PATTERN_EDGES) {
    if (err) *err = "pattern: bad edge count";
    return GPM_E_PATTERN;
  }
  bool adj[kMaxK][kMaxK] = {};
  for (int i = 0; i < p.n_edges; ++i) {
    int a = p.edges[2 * i], b = p.edges[2 * i + 1];
    if (a < 0 || b < 0 || a >= p.k || b >= p.k || a == b) {
      if (err) *err = "pattern: edge endpoint out of range or self loop";
      return GPM_E_PATTERN;
    }
    if (adj[a][b]) {
      if (err) *err = "pattern: duplicate edge";
      return GPM_E_PATTERN;
    }
    adj[a][b] = adj[b][a] = true;
  }
  // connectivity: vertex extension only reaches connected patterns (Sec. 2.2)
  bool seen[kMaxK] = {};
  int stack[kMaxK], top = 0;
  seen[0] = true;
  stack[top++] = 0;
  while (top) {
    int x = stack[--top];
    for (int y = 0; y < p.k; ++y)
      if (adj[x][y] && !seen[y]) {
        seen[y] = true;
        stack[top++] = y;
      }
  }
  for (int i = 0; i < p.k; ++i)
    if (!seen[i]) {
      if (err) *err = "pattern: disconnected";
      return GPM_E_PATTERN;
    }
  return GPM_OK;
}

static void adjacency(const gpm_pattern& p, bool adj[kMaxK][kMaxK]) {
  for (int i = 0; i < kMaxK; ++i)
    for (int j = 0; j < kMaxK; ++j) adj[i][j] = false;
  for (int i = 0; i < p.n_edges; ++i) {
    int a = p.edges[2 * i], b = p.edges[2 * i + 1];
    adj[a][b] = adj[b][a] = true;
  }
}

bool is_clique(const gpm_pattern& p) { return p.n_edges == p.k * (p.k - 1) / 2; }

// All automorphisms of the pattern (k <= 8, so k! <= 40320 candidates).
static std::vector<std::array<int8_t, kMaxK>> automorphisms(int k, bool adj[kMaxK][kMaxK]) {
  std::vector<std::array<int8_t, kMaxK>> out;
  std::array<int8_t, kMaxK> perm{};
  for (int i = 0; i < k; ++i) perm[i] = (int8_t)i;
  do {
    bool ok = true;
    for (int i = 0; i < k && ok; ++i)
      for (int j = i + 1; j < k; ++j)
        if (adj[i][j] != adj[perm[i]][perm[j]]) {
          ok = false;
          break;
        }
    if (ok) out.push_back(perm);
  } while (std::next_permutation(perm.begin(), perm.begin() + k));
  return out;
}

// Greedy connected matching order: start at a vertex of maximum degree, then
// repeatedly take the unmatched vertex with the most matched neighbours
// (ties: higher degree, then lower id).  Every depth > 0 is adjacent to an
// earlier depth, and depth 1 is adjacent to depth 0 (edge-rooted tasks).
static void matching_order(int k, bool adj[kMaxK][kMaxK], int order[kMaxK],
                           uint32_t last = 0) {
  // `last`: vertices kept for the end of the order (in id order)
  int deg[kMaxK] = {};
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) deg[i] += adj[i][j];
  bool used[kMaxK] = {};
  int first = -1;
  for (int i = 0; i < k; ++i)
    if (!((last >> i) & 1u) && (first < 0 || deg[i] > deg[first])) first = i;
  order[0] = first;
  used[first] = true;
  int kp = k - __builtin_popcount(last);
  for (int i = 0, d = kp; i < k; ++i)
    if ((last >> i) & 1u) {
      order[d++] = i;
      used[i] = true;
    }
  for (int d = 1; d < kp; ++d) {
    int best = -1, bc = -1, bd = -1;
    for (int v = 0; v < k; ++v) {
      if (used[v]) continue;
      int c = 0;
      for (int e = 0; e < d; ++e) c += adj[v][order[e]];
      if (c == 0) continue;
      if (c > bc || (c == bc && deg[v] > bd)) {
        best = v;
        bc = c;
        bd = deg[v];
      }
    }
    order[d] = best;
    used[best] = true;
  }
}

// Counting-only pruning (Sec. 5.4 (1), by pattern decomposition): the largest
// set S of r >= 2 pairwise non-adjacent pattern vertices with the same
// neighbours (twins) such that the rest of the pattern is connected and has
// at least two vertices.  Matched last, S's vertices all draw from one
// candidate set C (the same intersection, the same bounds from earlier
// vertices, the same exclusions), so in edge-induced mode the matches that
// extend one prefix number ext * C(|C|, r), ext being the orderings of S
// that its symmetry restrictions allow.  Returns S as a bit mask (0: none).
static uint32_t twin_suffix(int k, bool adj[kMaxK][kMaxK]) {
  uint32_t best = 0;
  int best_r = 1;
  for (int a = 0; a < k; ++a) {
    uint32_t cls = 0;
    for (int b = 0; b < k; ++b) {
      if (adj[a][b]) continue;
      bool same = true;
      for (int x = 0; x < k && same; ++x)
        if (x != a && x != b && adj[a][x] != adj[b][x]) same = false;
      if (same) cls |= 1u << b;   // includes a itself
    }
    // the whole class, or all but one of it, as S
    for (int drop = -1; drop < k; ++drop) {
      uint32_t S = cls;
      if (drop >= 0) {
        if (!((cls >> drop) & 1u)) continue;
        S &= ~(1u << drop);
      }
      const int r = __builtin_popcount(S);
      if (r <= best_r || k - r < 2) continue;
      // the rest connected
      uint32_t rest = ((1u << k) - 1) & ~S;
      int start = __builtin_ctz(rest);
      uint32_t seen = 1u << start, frontier = seen;
      while (frontier) {
        int x = __builtin_ctz(frontier);
        frontier &= frontier - 1;
        for (int y = 0; y < k; ++y)
          if (adj[x][y] && ((rest >> y) & 1u) && !((seen >> y) & 1u)) {
            seen |= 1u << y;
            frontier |= 1u << y;
          }
      }
      if (seen != rest) continue;
      best = S;
      best_r = r;
    }
  }
  return best;
}

int build_plan(const gpm_pattern& p, int mode, bool on_dag, HostPlan* out, std::string* err,
               bool count_only) {
  int st = validate_pattern(p, err);
  if (st) return st;
  HostPlan hp;
  hp.k = p.k;
  hp.mode = mode;
  hp.clique = is_clique(p);
  bool adj[kMaxK][kMaxK];
  adjacency(p, adj);
  auto auts = automorphisms(p.k, adj);
  hp.aut = (int)auts.size();
  const int k = p.k;
  Plan& P = hp.plan;
  std::memset(&P, 0, sizeof(P));
  P.k = k;
  for (int d = 0; d < kMaxK; ++d) P.store_slot[d] = -1;

  if (on_dag) {
    // Cliques on the oriented DAG (Sec. 4.2, graph preprocessing): the orientation already breaks
    // every symmetry, so there are no bounds; depth l intersects the set of
    // depth l-1 with N+(v_{l-1}).
    if (!hp.clique) {
      if (err) *err = "only cliques can run on an oriented (DAG) graph";
      return GPM_E_UNSUPPORTED;
    }
    for (int d = 0; d < k; ++d) hp.order[d] = d;
    P.root_bound = 0;
    int ns = 0;
    for (int l = 2; l < k; ++l) {
      LevelPlan& L = P.lv[l];
      if (l == 2) {
        L.base_buf = -1;
        L.n_int = 2;
        L.int_lv[0] = 0;
        L.int_lv[1] = 1;
      } else {
        L.base_buf = (int8_t)(l - 1);
        L.n_int = 1;
        L.int_lv[0] = (uint8_t)(l - 1);
      }
      if (l < k - 1) {
        L.flags = kLvStore;
        P.store_slot[l] = (int8_t)ns++;
      }
    }
    P.n_store = ns;
    hp.n_buffers = ns;
    *out = hp;
    return GPM_OK;
  }

  const uint32_t suffix =
      (count_only && mode == GPM_EDGE_INDUCED && !hp.clique) ? twin_suffix(k, adj) : 0;
  matching_order(k, adj, hp.order, suffix);
  int depth_of[kMaxK];
  for (int d = 0; d < k; ++d) depth_of[hp.order[d]] = d;

  // Symmetry order by a stabiliser chain (Sec. 2.2 "Symmetry order"; the
  // pattern is built up in matching order and at each step the vertices
  // still symmetric to the new one are ordered below it).  Every orbit
  // element w of u under the stabiliser of the earlier depths lies later in
  // the matching order, so each restriction is v_u > v_w with u earlier.
  std::vector<std::array<int8_t, kMaxK>> G = auts;
  for (int d = 0; d < k; ++d) {
    int u = hp.order[d];
    bool in_orbit[kMaxK] = {};
    for (auto& g : G) in_orbit[g[u]] = true;
    for (int w = 0; w < k; ++w)
      if (w != u && in_orbit[w]) hp.restrictions.push_back({u, w});
    std::vector<std::array<int8_t, kMaxK>> H;
    for (auto& g : G)
      if (g[u] == u) H.push_back(g);
    G.swap(H);
  }

  // less[a][b]: v_a < v_b is implied (by depth), transitively closed
  bool less[kMaxK][kMaxK] = {};
  for (auto& r : hp.restrictions) less[depth_of[r.second]][depth_of[r.first]] = true;
  for (int m = 0; m < k; ++m)
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b)
        if (less[a][m] && less[m][b]) less[a][b] = true;

  uint8_t intm[kMaxK] = {}, subm[kMaxK] = {}, bnd[kMaxK] = {};
  for (int l = 1; l < k; ++l)
    for (int j = 0; j < l; ++j) {
      bool a = adj[hp.order[l]][hp.order[j]];
      if (a) intm[l] |= (uint8_t)(1u << j);
      else if (mode == GPM_VERTEX_INDUCED) subm[l] |= (uint8_t)(1u << j);
    }
  for (auto& r : hp.restrictions) bnd[depth_of[r.second]] |= (uint8_t)(1u << depth_of[r.first]);
  P.root_bound = (bnd[1] & 1u) ? 1 : 0;

  int ns = 0;
  for (int l = 2; l < k; ++l) {
    LevelPlan& L = P.lv[l];
    L.bound_mask = bnd[l];
    // reuse the stored set of an earlier depth j whose constraints are all
    // implied at depth l (the buffer W of Alg. 1, reused across depths)
    int reuse = -1;
    for (int j = l - 1; j >= 2 && reuse < 0; --j) {
      const LevelPlan& J = P.lv[j];
      if (!(J.flags & (kLvStore | kLvSlice))) continue;
      if ((intm[j] & ~intm[l]) || (subm[j] & ~subm[l])) continue;
      bool ok = true;
      for (int r = 0; r < j && ok; ++r)
        if ((bnd[j] >> r) & 1u) ok = less[l][r];
      if (ok) reuse = j;
    }
    uint8_t rem_int = intm[l], rem_sub = subm[l];
    if (reuse >= 0) {
      rem_int &= (uint8_t)~intm[reuse];
      rem_sub &= (uint8_t)~subm[reuse];
      L.base_buf = (int8_t)reuse;
    } else {
      L.base_buf = -1;
    }
    L.n_int = 0;
    for (int j = 0; j < l; ++j)
      if ((rem_int >> j) & 1u) L.int_lv[L.n_int++] = (uint8_t)j;
    L.n_sub = 0;
    for (int j = 0; j < l; ++j)
      if ((rem_sub >> j) & 1u) L.sub_lv[L.n_sub++] = (uint8_t)j;

    // matched vertices that the set algebra does not already remove
    uint8_t excl = 0;
    for (int w = 0; w < l; ++w) {
      if ((intm[l] >> w) & 1u) continue;          // v_w is not in N(v_w)
      if (less[l][w]) continue;                   // v_l < v_w by the bounds
      if (mode == GPM_VERTEX_INDUCED) {
        bool gone = false;
        // in induced mode matched pairs are adjacent exactly as in the pattern
        for (int s = 0; s < l && !gone; ++s)
          if (((subm[l] >> s) & 1u) && adj[hp.order[w]][hp.order[s]]) gone = true;
        for (int b = 0; b < l && !gone; ++b)
          if (((intm[l] >> b) & 1u) && !adj[hp.order[w]][hp.order[b]]) gone = true;
        if (gone) continue;
      }
      excl |= (uint8_t)(1u << w);
    }
    if (reuse >= 0 && (P.lv[reuse].flags & kLvSlice)) excl |= P.lv[reuse].excl_mask;
    L.excl_mask = excl;

    if (l < k - 1) {
      int probes = reuse >= 0 ? L.n_int : L.n_int - 1;
      if (probes == 0 && L.n_sub == 0) {
        L.flags = kLvSlice;
      } else {
        L.flags = kLvStore;
        P.store_slot[l] = (int8_t)ns++;
      }
    }
  }
  P.n_store = ns;
  hp.n_buffers = ns;

  if (suffix) {
    // the leaf at depth kp = k - r stands for depths kp .. k-1; its level
    // (like theirs) intersects the same lists under the same bounds and
    // exclusions from depths below kp
    const int r = __builtin_popcount(suffix);
    const int kp = k - r;
    const uint8_t below = (uint8_t)((1u << kp) - 1);
    bool ok = true;
    for (int l = kp + 1; l < k && ok; ++l)
      ok = (intm[l] & below) == (intm[kp] & below) && !(intm[l] & ~below) &&
           (bnd[l] & below) == (bnd[kp] & below) && subm[l] == 0;
    if (ok) {
      // orderings of the r suffix vertices allowed by their restrictions
      int perm[kMaxK];
      for (int i = 0; i < r; ++i) perm[i] = i;
      int ext = 0;
      do {  // perm[i] = rank of the value at depth kp + i
        bool fine = true;
        for (int a = 0; a < r && fine; ++a)
          for (int b = 0; b < r && fine; ++b)
            if (((bnd[kp + b] >> (kp + a)) & 1u) && !(perm[a] > perm[b])) fine = false;
        ext += fine ? 1 : 0;
      } while (std::next_permutation(perm, perm + r));
      LevelPlan& L = P.lv[kp];
      L.flags = 0;  // count-only
      for (int l = kp; l < kMaxK; ++l) P.store_slot[l] = -1;
      int n2 = 0;
      for (int l = 2; l < kp; ++l) n2 += (P.lv[l].flags & kLvStore) ? 1 : 0;
      P.n_store = n2;
      hp.n_buffers = n2;
      P.k = kp + 1;
      P.leaf_choose = r | (ext << 8);
      hp.choose_r = r;
    }
  }
  *out = hp;
  return GPM_OK;
}

}  // namespace gpm
