// Device code of libgpm: pattern-aware DFS subgraph extension on gfx950.
//
// One persistent launch consumes chunks of root tasks from per-XCD queues
// (work stealing across XCDs when a queue runs dry).  Each task is walked by
// one wave64: all 64 lanes follow the same depth-first walk and share every
// set operation (the paper's warp-centric two-level parallelism, Sec. 5.1,
// mapped to 64-wide wavefronts).  Set intersection / difference / bounding
// (Sec. 6.1) evaluate one element per lane, test membership by binary search
// and compact the survivors with ballot + mbcnt + popcount.  Exact uint64
// counts stay in per-lane registers and are reduced once per job.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>

#include "gpm_internal.h"

namespace gpm {

// ---------------------------------------------------------------------------
// wave-level helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int32_t uni(int32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ int64_t uni64(int64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// number of set bits of m in lanes below this one
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int32_t y = __shfl_up(x, off, 64);
    if (l >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ int64_t wave_incl_scan64(int64_t x) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int64_t y = __shfl_up(x, off, 64);
    if (l >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;  // valid in lane 0
}

// Cross-lane visibility of a wave's own stores before other lanes read them.
__device__ __forceinline__ void wave_sync_mem() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First index i in [0, n) with a[i] >= key (n if none).  Branch-free body:
// the iteration count depends only on n.
template <typename T>
__device__ __forceinline__ int32_t lower_bound(const T* a, int32_t n, int32_t key) {
  if (n <= 0) return 0;
  int32_t base = 0;
  while (n > 1) {
    int32_t half = n >> 1;
    base = (a[base + half] < key) ? base + half : base;
    n -= half;
  }
  return base + (a[base] < key ? 1 : 0);
}

template <typename T>
__device__ __forceinline__ bool member(const T* a, int32_t n, int32_t key) {
  int32_t p = lower_bound(a, n, key);
  return p < n && a[p] == key;
}

// First index i in [0, n) with a[i] > key.
template <typename T, typename K>
__device__ __forceinline__ int32_t upper_bound(const T* a, int32_t n, K key) {
  if (n <= 0) return 0;
  int32_t base = 0;
  while (n > 1) {
    int32_t half = n >> 1;
    base = (a[base + half] <= key) ? base + half : base;
    n -= half;
  }
  return base + (a[base] <= key ? 1 : 0);
}

// First index i in [lo, n) with a[i] >= key, given a[lo - 1] < key (or lo =
// 0): one probe when a[lo] >= key already, else an exponential search from
// lo (the probes stay near lo, where the previous window's slice ended).
__device__ __forceinline__ int32_t gallop_lb(const int32_t* __restrict__ a, int32_t lo,
                                             int32_t n, int32_t key) {
  if (lo >= n || a[lo] >= key) return lo;
  int32_t base = lo;  // a[base] < key
  int32_t step = 1;
  while (base + step < n && a[base + step] < key) {
    base += step;
    step <<= 1;
  }
  const int32_t hi = min(base + step, n);  // a[hi] >= key, or hi == n
  return base + 1 + lower_bound(a + base + 1, hi - base - 1, key);
}

// lower_bound whose first kBstLevels halving steps read their probe values
// from `piv`: the implicit binary search tree's top levels staged in LDS
// (Sec. 6.1: the first levels of the search tree kept in the scratchpad).
// Node t of the tree (1-based heap order: children 2t, 2t + 1) holds the
// value the search meets after the turns spelled by t's bits, so the result
// equals lower_bound's.
constexpr int kBstLevels = 5;
constexpr int kBstNodes = (1 << kBstLevels) - 1;

__device__ __forceinline__ int32_t lower_bound_bst(const int32_t* __restrict__ a, int32_t n,
                                                   int32_t key, const int32_t* piv) {
  if (n <= 0) return 0;
  int32_t base = 0, node = 1;
#pragma unroll
  for (int s = 0; s < kBstLevels; ++s) {
    if (n <= 1) break;
    const int32_t half = n >> 1;
    const bool right = piv[node - 1] < key;
    base = right ? base + half : base;
    node = 2 * node + (right ? 1 : 0);
    n -= half;
  }
  while (n > 1) {
    const int32_t half = n >> 1;
    base = (a[base + half] < key) ? base + half : base;
    n -= half;
  }
  return base + (a[base] < key ? 1 : 0);
}

// Stage the kBstNodes pivots of list a[0, n) (lane t < kBstNodes loads node
// t + 1); nodes the search never reaches are left unset.
__device__ __forceinline__ void bst_stage(const int32_t* __restrict__ a, int32_t n, int32_t* piv) {
  const int p = lane_id();
  if (p < kBstNodes) {
    const int32_t q = p + 1;
    const int lvl = 31 - __clz(q);
    int32_t nn = n, base = 0;
    bool live = true;
    for (int i = lvl - 1; i >= 0 && live; --i) {
      if (nn <= 1) { live = false; break; }
      const int32_t half = nn >> 1;
      if ((q >> i) & 1) base += half;
      nn -= half;
    }
    if (live && nn > 1) piv[p] = a[base + (nn >> 1)];
  }
}

// Instrumented builds only (CE = true): the method's own work, counted the
// same way in every lane (summed over the wave, then divided by 64).
struct ElemCounter {
  uint64_t elems = 0;     // sum over set operations of the bounded operand lengths
  uint64_t fetches = 0;   // neighbour-list reads
  uint64_t written = 0;   // frontier elements stored
  uint64_t words = 0;     // bitmap word operations (AND + popcount of 64 bits),
                          // counted per lane (summed, not divided by 64)
};

// ---------------------------------------------------------------------------
// set operations (Sec. 6.1): one element of the iterated list per lane
// ---------------------------------------------------------------------------

// out = A ∩ B (A iterated, B probed), order of A kept; returns |out|.
template <typename TA, typename TB, typename TO>
__device__ __forceinline__ int32_t intersect_store(const TA* A, int32_t na, const TB* B,
                                                   int32_t nb, TO* out) {
  int32_t total = 0;
  const int l = lane_id();
  for (int32_t ib = 0; ib < na; ib += 64) {
    int32_t i = ib + l;
    bool keep = false;
    int32_t x = 0;
    if (i < na) {
      x = A[i];
      keep = member(B, nb, x);
    }
    uint64_t m = wave_ballot(keep);
    if (keep) out[total + (int32_t)lanes_below(m)] = x;
    total += (int32_t)__popcll(m);
  }
  wave_sync_mem();
  return total;
}

// |A ∩ B| contributed by this lane.
template <typename TA, typename TB>
__device__ __forceinline__ uint32_t intersect_count(const TA* A, int32_t na, const TB* B,
                                                    int32_t nb) {
  uint32_t c = 0;
  const int l = lane_id();
  for (int32_t i = l; i < na; i += 64) c += member(B, nb, (int32_t)A[i]) ? 1u : 0u;
  return c;
}

// ---------------------------------------------------------------------------
// k-clique on the oriented DAG (Sec. 4.2 orientation; Alg. 1 with every level
// an intersection).  Sets F_d of candidates for v_d; the last two vertices
// are counted together as the number of DAG edges inside F_{k-2}.
// ---------------------------------------------------------------------------

// Sum over w in F of |F ∩ N+(w)|.  P is scratch of s + 1 int64 (the prefix of
// the out-degrees over F can pass 2^31 on a caller's DAG with large lists).
template <bool CE, typename TF, typename TP>
__device__ __forceinline__ uint64_t clique_leaf(const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ col,
                                                const TF* F, int32_t s, TP* P,
                                                ElemCounter& ec) {
  const int l = lane_id();
  int64_t running = 0;
  for (int32_t ib = 0; ib < s; ib += 64) {
    int32_t i = ib + l;
    int64_t d = 0;
    if (i < s) {
      int32_t w = F[i];
      d = rp[w + 1] - rp[w];
    }
    int64_t inc = wave_incl_scan64(d);
    if (i < s) P[i + 1] = running + inc;
    running += __shfl(inc, 63, 64);
  }
  if (l == 0) P[0] = 0;
  wave_sync_mem();
  running = uni64(running);
  if (CE) {
    ec.elems += (uint64_t)s * (uint64_t)s + (uint64_t)running;
    ec.fetches += (uint64_t)s;
  }
  uint64_t c = 0;
  for (int64_t tb = 0; tb < running; tb += 64) {
    int64_t t = tb + l;
    if (t < running) {
      // owner i: P[i] <= t < P[i+1]
      int32_t i = upper_bound(P + 1, s, t);
      int32_t w = F[i];
      int32_t x = col[rp[w] + (t - P[i])];
      c += member(F, s, x) ? 1u : 0u;
    }
  }
  return c;
}

// Count k-cliques (k >= 3) whose first two vertices are the DAG edge u->v.
// U = N+(u) (LDS-staged or global), bufs: (k-3) sets of cap ints, P: cap+1
// int64, st: 2*kMaxK ints of wave state.
template <bool CE, typename TU, typename TB>
__device__ __forceinline__ uint64_t clique_edge(const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ col, int k,
                                                const TU* U, int32_t du, int32_t v,
                                                TB* bufs, int64_t* P, int32_t cap,
                                                int32_t* st, ElemCounter& ec) {
  const int32_t* Nv = col + rp[v];
  const int32_t dv = uni((int32_t)(rp[v + 1] - rp[v]));
  if (CE) {
    ec.elems += (uint64_t)du + (uint64_t)dv;
    ec.fetches += 2;
  }
  if (k == 3) return intersect_count(Nv, dv, U, du);
  TB* F2 = bufs;
  int32_t s2 = uni(intersect_store(Nv, dv, U, du, F2));
  if (CE) ec.written += (uint64_t)s2;
  if (s2 < k - 2) return 0;
  if (k == 4) return clique_leaf<CE>(rp, col, F2, s2, P, ec);

  // depths 2 .. k-3 are iterated; F_{k-2} goes to the leaf
  uint64_t c = 0;
  int32_t* sz = st;
  int32_t* ix = st + kMaxK;
  int d = 2;
  if (lane_id() == 0) { sz[2] = s2; ix[2] = 0; }
  wave_sync_mem();
  for (;;) {
    int32_t i = uni(ix[d]);
    int32_t s = uni(sz[d]);
    if (i >= s) {
      if (d == 2) break;
      --d;
      if (lane_id() == 0) ix[d] = ix[d] + 1;
      wave_sync_mem();
      continue;
    }
    TB* Fd = bufs + (size_t)(d - 2) * cap;
    TB* Fn = Fd + cap;
    int32_t w = uni(Fd[i]);
    const int32_t* Nw = col + rp[w];
    int32_t dw = uni((int32_t)(rp[w + 1] - rp[w]));
    int32_t sn;
    // iterate the shorter side; probe LDS-resident F when N+(w) is not much longer
    if (dw <= 4 * s) sn = uni(intersect_store(Nw, dw, Fd, s, Fn));
    else sn = uni(intersect_store(Fd, s, Nw, dw, Fn));
    if (CE) {
      ec.elems += (uint64_t)s + (uint64_t)dw;
      ec.fetches += 1;
      ec.written += (uint64_t)sn;
    }
    if (d + 1 == k - 2) {
      if (sn >= 2) c += clique_leaf<CE>(rp, col, Fn, sn, P, ec);
      if (lane_id() == 0) ix[d] = i + 1;
      wave_sync_mem();
      continue;
    }
    if (sn < k - (d + 1)) {
      if (lane_id() == 0) ix[d] = i + 1;
      wave_sync_mem();
      continue;
    }
    ++d;
    if (lane_id() == 0) { sz[d] = sn; ix[d] = 0; }
    wave_sync_mem();
  }
  return c;
}

// ---------------------------------------------------------------------------
// k-clique by local graph search with bitmaps (Sec. 5.4 (2) and Sec. 6.2):
// for a root u the search stays inside N+(u); its local DAG is stored as one
// bitmap row per vertex of N+(u) (bit j of row i: N+(u)[i] -> N+(u)[j]).
// Triangles, 4-cliques and 5-cliques rooted at u are then popcounts of
// ANDed rows.  One wave per root vertex.
// ---------------------------------------------------------------------------

// position of the r-th (0-based) set bit of x (r < popcount(x))
__device__ __forceinline__ int select64(uint64_t x, int r) {
  int pos = 0;
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    int c = __popcll(x & ((1ull << s) - 1ull));
    if (r >= c) {
      r -= c;
      x >>= s;
      pos += s;
    }
  }
  return pos;
}

// Hash of a local graph's vertex list L (open addressing, linear probing):
// slot = (position << 32) | (vertex + 1), 0 = empty.  lgs_hash_slots(d)
// slots for d vertices keep the load factor at most 1/2.
__device__ __forceinline__ int32_t lgs_hash_bits(int32_t d) {
  return 32 - __clz(2 * d - 1);  // 2^bits = lgs_hash_slots(d) >= 2d
}

__device__ __forceinline__ uint32_t lgs_hash(int32_t x, int32_t bits) {
  return ((uint32_t)x * 0x9E3779B1u) >> (32 - bits);  // Fibonacci hashing
}

template <typename TH>
__device__ __forceinline__ void lgs_hash_put(TH* H, int32_t bits, int32_t x, int32_t pos) {
  const uint32_t mask = (1u << bits) - 1u;
  const unsigned long long e = ((unsigned long long)(uint32_t)pos << 32) | ((uint32_t)x + 1u);
  for (uint32_t s = lgs_hash(x, bits);; s = (s + 1u) & mask)
    if (atomicCAS(&H[s], 0ull, e) == 0ull) return;
}

// Position of x in L, or -1.
template <typename TH>
__device__ __forceinline__ int32_t lgs_hash_get(const TH* H, int32_t bits, int32_t x) {
  const uint32_t mask = (1u << bits) - 1u;
  for (uint32_t s = lgs_hash(x, bits);; s = (s + 1u) & mask) {
    const unsigned long long e = H[s];
    if (e == 0ull) return -1;
    if ((uint32_t)e == (uint32_t)x + 1u) return (int32_t)(e >> 32);
  }
}

// Rows of a local graph: R_i = positions in L of N+(L[i]) ∩ L, for rows
// i = first, first + step, ... (the calling wave owns these rows).  The wave
// scans 64 >> lg rows at once, one per group of 2^lg lanes (lg = 6: one row
// at a time with the whole wave; short out-lists leave most of a wave's
// lanes idle and its rows waiting one memory round trip each, which groups
// of 16 or 8 lanes overlap); a group walks its row's out-list 2^lg elements
// at a time and looks each element up in the hash H of L.  Out-lists are
// sorted, so a row stops at the first batch whose elements all exceed
// max(L).  With BITS the hits are set in R (rows of W words); the number of
// hits is returned either way (per lane).  With `next` (the workgroup path),
// rows are taken from that LDS counter a round at a time instead (first and
// step unused), so waves that drew short rows take more of them.  With SC
// every hit (triangle u, L[i], L[j]) adds 1 to the per-row counters lc[i]
// and lc[j] (edges u-L[i], u-L[j]) and to tri[p], p the DAG position of the
// element (edge L[i]-L[j]).
template <bool CE, bool BITS, bool SC = false, typename TL, typename TH, typename TR,
          typename TC = int32_t>
__device__ __forceinline__ uint64_t lgs_build_rows(const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const TL* L,
                                                   int32_t d, int32_t W, const TH* H,
                                                   int32_t bits, TR* R, int32_t first,
                                                   int32_t step, ElemCounter& ec,
                                                   int32_t* next = nullptr, TC* lc = nullptr,
                                                   unsigned int* tri = nullptr, int32_t lg = 6) {
  constexpr int U = 4;  // batches of a group's lanes whose loads are in flight together
  const int l = lane_id();
  const int32_t GL = 1 << lg;      // lanes per group
  const int32_t G = 64 >> lg;      // rows per round
  const int32_t g = l >> lg;       // this lane's group
  const int32_t q = l & (GL - 1);  // its lane within the group
  const uint64_t gmask = (lg == 6 ? ~0ull : ((1ull << GL) - 1ull)) << (g * GL);
  const int32_t gs = next ? 1 : step;  // row distance between the groups of a round
  const int32_t lmax = uni(L[d - 1]);
  auto take = [&]() -> int32_t {
    int32_t r = 0;
    if (l == 0) r = atomicAdd(next, G);
    return uni(__shfl(r, 0, 64));
  };
  uint64_t hits = 0;
  int32_t ib = next ? take() : first;  // first row of the round (uniform)
  int64_t nb = 0, ne = 0;              // bounds of the group's row, loaded a round ahead
  {
    const int32_t ig = ib + g * gs;
    if (ib < d && ig < d) {
      const int32_t v = L[ig];
      nb = rp[v];
      ne = rp[v + 1];
    }
  }
  while (ib < d) {
    const int32_t i = ib + g * gs;  // this group's row; (b, e) = (0, 0) if i >= d
    const int64_t b = nb, e = ne;
    const int32_t in = next ? take() : ib + G * step;
    nb = 0;
    ne = 0;
    {
      const int32_t ig = in + g * gs;
      if (in < d && ig < d) {
        const int32_t v = L[ig];
        nb = rp[v];
        ne = rp[v + 1];
      }
    }
    if (CE) ec.elems += (uint64_t)(e - b) * (uint64_t)G;  // summed over the lanes / 64
    bool live = b < e;
    for (int64_t pb = b;; pb += (int64_t)GL * U) {
      int32_t x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t p = pb + u * GL + q;
        x[u] = (live && p < e) ? col[p] : INT_MAX;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (x[u] <= lmax) {
          const int32_t j = lgs_hash_get(H, bits, x[u]);
          if (j >= 0) {
            ++hits;
            if (BITS) atomicOr(&R[(size_t)i * W + (j >> 6)], 1ull << (j & 63));
            if (SC) {
              atomicAdd(&lc[i], 1);
              atomicAdd(&lc[j], 1);
              atomicAdd(&tri[pb + u * GL + q], 1u);
            }
          }
        }
      }
      // a row ends at its last element or at the first batch whose elements
      // all exceed max(L) (none further can hit)
      const uint64_t more = wave_ballot(x[U - 1] <= lmax);
      live = live && (more & gmask) != 0ull && pb + (int64_t)GL * U < e;
      if (wave_ballot(live) == 0ull) break;
    }
    ib = in;
  }
  return hits;
}

// Local edges t0 .. t1-1 of a local graph (rows of W words at a stride of
// S, row-size prefix P over its d rows), in order: f(i, j) for each.  The
// first is located through P, each next one as the next bit of the same row
// (a search again only where the row ends).
template <typename TP, typename TR, typename F>
__device__ __forceinline__ void lgs_edge_walk(const TP* P, const TR* R, int32_t d, int32_t W,
                                              int32_t S, int32_t t0, int32_t t1, F&& f) {
  int32_t i = 0, j = 0;
  for (int32_t t = t0; t < t1; ++t) {
    bool found = false;
    if (t > t0) {  // edge t - 1 is (i, j)
      const TR* Rc = R + (size_t)i * S;
      int32_t w = (j + 1) >> 6;
      if (w < W) {
        uint64_t bm = Rc[w] & (~0ull << ((j + 1) & 63));
        while (!bm && ++w < W) bm = Rc[w];
        if (bm) {
          j = w * 64 + __builtin_ctzll(bm);
          found = true;
        }
      }
    }
    if (!found) {
      i = upper_bound(P + 1, d, t);
      int32_t r = t - P[i];
      const TR* Rc = R + (size_t)i * S;
      int32_t w = 0;
      for (;; ++w) {
        const int32_t pc = __popcll(Rc[w]);
        if (r < pc) break;
        r -= pc;
      }
      j = w * 64 + select64(Rc[w], r);
    }
    f(i, j);
  }
}

// L: d ints, P: d + 1 ints, R: d * W uint64 (W = ceil(d / 64)).
// Sub-task `part` of `parts` handles its share of the local edges (i, j), so
// the heaviest roots are spread over several waves (each rebuilds the local
// graph, a small fraction of the root's work).
// 5-clique pair phase of one local graph with W = WC words per row: local
// edges p0 .. p1-1 (enumerated through the row-size prefix P), one per
// thread: this thread takes p0 + first, p0 + first + step, ...
template <bool CE, int WC, bool ORD, typename TP, typename TR>
__device__ __forceinline__ uint64_t lgs_pairs5(const TP* P, const TR* R, int32_t d, int32_t p0,
                                               int32_t p1, int32_t first, int32_t step,
                                               ElemCounter& ec) {
  uint64_t c = 0;
  for (int32_t t = p0 + first; t < p1; t += step) {
    const int32_t i = upper_bound(P + 1, d, t);
    int32_t r = t - P[i];
    const TR* Ri = R + (size_t)i * WC;
    int32_t w = 0;
    for (;; ++w) {
      const int32_t pc = __popcll(Ri[w]);
      if (r < pc) break;
      r -= pc;
    }
    const int32_t j = w * 64 + select64(Ri[w], r);
    const TR* Rj = R + (size_t)j * WC;
    // ordered: R_j (and so M) has bits only above j, R_l only above l
    const int jw = ORD ? ((j + 1) >> 6) : 0;
    uint64_t M[WC];
#pragma unroll
    for (int x = 0; x < WC; ++x) M[x] = (x >= jw) ? (Ri[x] & Rj[x]) : 0ull;
    if (CE) ec.words += (uint64_t)(WC - jw);
    // the pair's count fits 32 bits (|M| * d < 2^22): popcount-accumulate
    uint32_t cp = 0;
    if constexpr (WC <= 16) {
      // both loops unrolled: every word index is static.  Bits are taken from
      // the two 32-bit halves of each word (cheaper find-first and clear), and
      // the row offset within the half-word's block of rows is kept opaque so
      // the row's reads share one base address with small immediate offsets.
#pragma unroll
      for (int x = 0; x < WC; ++x) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          uint32_t m = (uint32_t)(M[x] >> (32 * h));
          const TR* Rxh = R + (size_t)(x * 64 + 32 * h) * WC;
          while (m) {
            uint32_t b = __builtin_ctz(m);
            m &= m - 1u;
            asm("" : "+v"(b));
            // rows < 2^24: the 24-bit multiply is exact and full rate
            const TR* Rl = Rxh + __umul24(b, (uint32_t)WC);
#pragma unroll
            for (int y = ORD ? x : 0; y < WC; ++y) {
              const uint64_t t = M[y] & Rl[y];
              // ordered: row l has bits above l only (see lgs_edge5)
              if (!(ORD && y == x && h == 1)) {
                cp = (uint32_t)__builtin_popcount((uint32_t)t) + cp;
                asm("" : "+v"(cp));
              }
              cp = (uint32_t)__builtin_popcount((uint32_t)(t >> 32)) + cp;
              asm("" : "+v"(cp));
            }
            if (CE) ec.words += (uint64_t)(WC - (ORD ? x : 0));
          }
        }
      }
    } else {
      // wide rows: outer loop over the words of M (reloaded, since dynamic
      // register indexing would go to scratch), inner loop unrolled
      for (int x = jw; x < WC; ++x) {
        uint64_t m = Ri[x] & Rj[x];
        while (m) {
          const int b = __builtin_ctzll(m);
          m &= m - 1ull;
          const TR* Rl = R + (size_t)(x * 64 + b) * WC;
#pragma unroll
          for (int y = 0; y < WC; ++y)
            if (!ORD || y >= x) cp += (uint32_t)__popcll(M[y] & Rl[y]);
          if (CE) ec.words += (uint64_t)(WC - (ORD ? x : 0));
        }
      }
    }
    c += cp;
  }
  return c;
}

// 5-clique count of one local edge (i, j) of an ordered local graph with rows
// of W <= WC words (W == WC except in the wide instance, whose rows are
// narrower than its register array) at a stride of S >= W words:
// Σ_{l ∈ M} |M ∩ R_l|, M = R_i & R_j (bits above j only).
template <int WC>
__device__ __forceinline__ uint32_t lgs_edge5(const unsigned long long* R, int32_t i, int32_t j,
                                              int32_t W, int32_t S) {
  const unsigned long long* Ri = R + (size_t)i * S;
  const unsigned long long* Rj = R + (size_t)j * S;
  const int jw = (j + 1) >> 6;
  uint64_t M[WC];
#pragma unroll
  for (int x = 0; x < WC; ++x) M[x] = (x >= jw && x < W) ? (Ri[x] & Rj[x]) : 0ull;
  uint32_t cp = 0;
#pragma unroll
  for (int x = 0; x < WC; ++x) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t m = (uint32_t)(M[x] >> (32 * h));
      const unsigned long long* Rxh = R + (size_t)(x * 64 + 32 * h) * S;
      while (m) {
        uint32_t b = __builtin_ctz(m);
        m &= m - 1u;
        // opaque row offset: the row's reads share one base address with
        // small immediate offsets
        asm("" : "+v"(b));
        const unsigned long long* Rl = Rxh + __umul24(b, (uint32_t)S);
#pragma unroll
        for (int y = x; y < WC; ++y)
          if (y < W) {
            const uint64_t t = M[y] & Rl[y];
            // row l = x * 64 + 32 * h + b has bits above l only: with l in
            // the upper half of word x, the lower half of t is zero.  Each
            // popcount adds to cp in turn (the empty asm keeps the sum a
            // chain of accumulating popcounts, not a tree of extra adds).
            if (!(y == x && h == 1)) {
              cp = (uint32_t)__builtin_popcount((uint32_t)t) + cp;
              asm("" : "+v"(cp));
            }
            cp = (uint32_t)__builtin_popcount((uint32_t)(t >> 32)) + cp;
            asm("" : "+v"(cp));
          }
      }
    }
  }
  return cp;
}

// The workgroup kernel's 5-clique pair phase with lanes balanced by work:
// each wave takes batches of kSortBatch consecutive local edges (p0 .. p1-1,
// enumerated row by row; the row-size prefix P locates a lane's first
// edge), keys every edge by a
// logarithm of its cost estimate |R_i & R_j| · (words from j's on) — four
// keys per octave, 0..63 — counting-sorts the batch by key in its LDS area
// (ids, cnt), then counts the sorted edges 64 at a time, so that the lanes of
// a round hold edges of similar cost (rows of W words at a stride of S).
// Returns this thread's partial count.
template <int WC>
__device__ __forceinline__ uint64_t lgs_pairs5_sorted(const int32_t* P,
                                                      const unsigned long long* R, int32_t d,
                                                      int32_t W, int32_t S, int32_t p0,
                                                      int32_t p1, int32_t* ids, int32_t* cnt) {
  constexpr int K = kSortBatch / 64;
  const int l = lane_id();
  const int wv = threadIdx.x >> 6;
  uint64_t c = 0;
  for (int32_t base = p0 + wv * kSortBatch; base < p1; base += kBlockWaves * kSortBatch) {
    cnt[l] = 0;
    wave_sync_mem();
    int32_t key[K], pid[K];
    // this lane's K consecutive local edges t0 .. t0 + K - 1: the first found
    // through the row-size prefix, each next one as the next bit of the same
    // row (a search again only where the row ends)
    const int32_t t0 = base + l * K;
    int32_t i = 0, j = 0;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int32_t t = t0 + q;
      key[q] = 64;
      pid[q] = 0;
      if (t < p1) {
        bool found = false;
        if (q > 0) {  // edge t - 1 is (i, j)
          const unsigned long long* Rc = R + (size_t)i * S;
          int32_t w = (j + 1) >> 6;
          if (w < W) {
            uint64_t bm = Rc[w] & (~0ull << ((j + 1) & 63));
            while (!bm && ++w < W) bm = Rc[w];
            if (bm) {
              j = w * 64 + __builtin_ctzll(bm);
              found = true;
            }
          }
        }
        if (!found) {
          i = upper_bound(P + 1, d, t);
          int32_t r = t - P[i];
          const unsigned long long* Rc = R + (size_t)i * S;
          int32_t w = 0;
          for (;; ++w) {
            const int32_t pc = __popcll(Rc[w]);
            if (r < pc) break;
            r -= pc;
          }
          j = w * 64 + select64(Rc[w], r);
        }
        const unsigned long long* Ri = R + (size_t)i * S;
        const unsigned long long* Rj = R + (size_t)j * S;
        const int jw = (j + 1) >> 6;
        int32_t m = 0;
#pragma unroll
        for (int x = 0; x < WC; ++x)
          if (x >= jw && x < W) m += __popcll(Ri[x] & Rj[x]);
        const int32_t v = min(m * (W - jw), 65535);
        key[q] = v < 4 ? v : ((31 - __clz(v)) << 2) | ((v >> (29 - __clz(v))) & 3);
        pid[q] = (i << 16) | j;
        atomicAdd(&cnt[key[q]], 1);
      }
    }
    wave_sync_mem();
    // exclusive prefix over the 64 buckets, one per lane
    const int32_t cb = cnt[l];
    const int32_t incl = wave_incl_scan(cb);
    const int32_t nvalid = uni(__shfl(incl, 63, 64));
    cnt[l] = incl - cb;
    wave_sync_mem();
#pragma unroll
    for (int q = 0; q < K; ++q)
      if (key[q] < 64) ids[atomicAdd(&cnt[key[q]], 1)] = pid[q];
    wave_sync_mem();
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int32_t idx = q * 64 + l;
      if (idx < nvalid) {
        const int32_t e = ids[idx];
        c += lgs_edge5<WC>(R, e >> 16, e & 0xffff, W, S);
      }
    }
    wave_sync_mem();  // the next batch reuses ids and cnt
  }
  return c;
}

template <bool CE, bool SC, typename TL, typename TP, typename TH, typename TR>
__device__ __forceinline__ uint64_t clique_lgs(const int64_t* __restrict__ rp,
                                               const int32_t* __restrict__ col, int k,
                                               int32_t u, int32_t d, int32_t part,
                                               int32_t parts, bool ordered, TL* L, TP* P,
                                               TH* H, TR* R, unsigned int* tri,
                                               ElemCounter& ec, int32_t lg) {
  const int l = lane_id();
  const int32_t W = (d + 63) >> 6;
  // hash of L: at least 2d slots, up to four times as many within the tile's
  // hash area (the slots between H and R, sized for the tile's T >= d)
  int32_t bits = lgs_hash_bits(d);
  {
    const int64_t area = ((const char*)R - (const char*)H) / 8;
    for (int e = 0; e < 2 && (int64_t(1) << (bits + 1)) <= area; ++e) ++bits;
  }
  const int32_t* Nu = col + rp[u];
  for (int32_t i = l; i < d; i += 64) L[i] = Nu[i];
  for (int32_t i = l; i < (1 << bits); i += 64) H[i] = 0ull;
  if (k > 3)
    for (int32_t i = l; i < d * W; i += 64) R[i] = 0ull;
  wave_sync_mem();
  for (int32_t i = l; i < d; i += 64) lgs_hash_put(H, bits, Nu[i], i);
  wave_sync_mem();
  if (CE) {
    ec.elems += (uint64_t)d * (uint64_t)d;
    ec.fetches += (uint64_t)d + 1;
  }
  // k = 3: every hit is a triangle at this root
  if (k == 3) {
    if (part != 0) return 0;
    if constexpr (!SC) {
      return lgs_build_rows<CE, false>(rp, col, L, d, W, H, bits, R, 0, 1, ec, nullptr,
                                       (int32_t*)nullptr, nullptr, lg);
    } else {
      // triangle scatter: P holds the per-row counters (edges u-L[i])
      for (int32_t i = l; i < d; i += 64) P[i] = 0;
      wave_sync_mem();
      lgs_build_rows<CE, false, true>(rp, col, L, d, W, H, bits, R, 0, 1, ec, nullptr, P, tri,
                                      lg);
      wave_sync_mem();
      const int64_t e0 = rp[u];
      for (int32_t i = l; i < d; i += 64)
        if (P[i]) atomicAdd(&tri[e0 + i], (unsigned int)P[i]);
      return 0;
    }
  }
  lgs_build_rows<CE, true>(rp, col, L, d, W, H, bits, R, 0, 1, ec, nullptr, (int32_t*)nullptr,
                          nullptr, lg);
  wave_sync_mem();
  uint64_t c = 0;
  int32_t running;
  // pairs (i, j) with j in row i, enumerated through a prefix over row sizes
  running = 0;
  for (int32_t ib = 0; ib < d; ib += 64) {
    int32_t i = ib + l;
    int32_t pc = 0;
    if (i < d)
      for (int32_t w = 0; w < W; ++w) pc += __popcll(R[(size_t)i * W + w]);
    int32_t inc = wave_incl_scan(pc);
    if (i < d) P[i + 1] = running + inc;
    running += __shfl(inc, 63, 64);
  }
  if (l == 0) P[0] = 0;
  wave_sync_mem();
  const int32_t pairs = uni(running);
  const int32_t p0 = (int32_t)((int64_t)pairs * part / parts);
  const int32_t p1 = (int32_t)((int64_t)pairs * (part + 1) / parts);
  if (k == 4) {
    // each lane a contiguous slice of the local edges, walked row by row
    const int32_t per = (p1 - p0 + 63) >> 6;
    const int32_t t0 = min(p1, p0 + l * per), t1 = min(p1, t0 + per);
    lgs_edge_walk(P, R, d, W, W, t0, t1, [&](int32_t i, int32_t j) {
      const TR* Ri = R + (size_t)i * W;
      const TR* Rj = R + (size_t)j * W;
      // ordered: R_j has bits only above j
      const int32_t x0 = ordered ? ((j + 1) >> 6) : 0;
      uint32_t cp = 0;
      for (int32_t x = x0; x < W; ++x) cp += (uint32_t)__popcll(Ri[x] & Rj[x]);
      c += cp;
      if (CE) ec.words += (uint64_t)(W - x0);
    });
    return c;
  }
  // k = 5: for every local edge (i, j) (one per lane) and every l in
  // M = R_i & R_j add |M & R_l|; M stays in registers.  The word count W is a
  // template constant so the inner loops carry no per-word range checks.
  if (!CE && ordered) {
    switch (W) {
#define GPM_LGS5(WC) \
  case WC:           \
    return c + lgs_pairs5<CE, WC, true>(P, R, d, p0, p1, l, 64, ec);
      // per-wave tiles hold at most 256 vertices (4 words per row); wider
      // rows (roots in HBM) take the generic loop, which keeps the
      // kernel's register count, and so its occupancy, low
      GPM_LGS5(1) GPM_LGS5(2) GPM_LGS5(3) GPM_LGS5(4)
#undef GPM_LGS5
      default: break;
    }
  }
  // lists in arbitrary order (a DAG given by the caller): words recomputed
  for (int32_t tb = p0; tb < p1; tb += 64) {
    const int32_t t = tb + l;
    if (t >= p1) continue;
    const int32_t i = upper_bound(P + 1, d, t);
    int32_t r = t - P[i];
    const TR* Ri = R + (size_t)i * W;
    int32_t w = 0;
    for (;; ++w) {
      const int32_t pc = __popcll(Ri[w]);
      if (r < pc) break;
      r -= pc;
    }
    const int32_t j = w * 64 + select64(Ri[w], r);
    const TR* Rj = R + (size_t)j * W;
    // (instrumented counts follow the ordered path's word ranges)
    const int32_t jw = ordered ? ((j + 1) >> 6) : 0;
    if (CE) ec.words += (uint64_t)(W - jw);
    for (int32_t x = jw; x < W; ++x) {
      uint64_t m = Ri[x] & Rj[x];
      while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1ull;
        const TR* Rl = R + (size_t)(x * 64 + b) * W;
        const int32_t y0 = ordered ? x : 0;
        for (int32_t y = y0; y < W; ++y) c += (uint64_t)__popcll(Ri[y] & Rj[y] & Rl[y]);
        if (CE) ec.words += (uint64_t)(W - y0);
      }
    }
  }
  return c;
}

// ---------------------------------------------------------------------------
// local graphs of large roots: one workgroup of kBlockWaves waves per root
// ---------------------------------------------------------------------------

// Inclusive scan of one value per thread over the workgroup; `total` gets
// the sum.  tmp: kBlockWaves words of LDS.  Contains workgroup barriers.
__device__ __forceinline__ int32_t block_incl_scan(int32_t v, int32_t* tmp, int32_t& total) {
  const int w = threadIdx.x >> 6;
  const int32_t inc = wave_incl_scan(v);
  if (lane_id() == 63) tmp[w] = inc;
  __syncthreads();
  int32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlockWaves; ++i) {
    const int32_t x = tmp[i];
    off += (i < w) ? x : 0;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return off + inc;
}

// The same local-graph search as clique_lgs, for a root u with
// d <= kLgsMaxVertices out-neighbours, with every step spread over the
// workgroup (rows taken by its waves from an LDS counter, per-vertex steps
// two vertices per thread above 1024) and the tile (T = d) in its LDS; with
// Rg the bitmap rows are in that HBM region instead (local graphs whose rows
// do not fit the LDS: L, P and the hash stay in it).  Every thread returns
// its partial count.
template <bool CE, bool HBM>
__device__ __forceinline__ uint64_t clique_lgs_block(const int64_t* __restrict__ rp,
                                     const int32_t* __restrict__ col, int k, int32_t u,
                                     int32_t d, int32_t part, int32_t parts, bool ordered,
                                     int32_t* lds, int32_t* tmp, int32_t* next, int32_t* sort_area,
                                     unsigned int* tri, unsigned long long* Rg, ElemCounter& ec,
                                     int32_t lg) {
  constexpr int NT = kBlockWaves * 64;
  const int tid = threadIdx.x;
  const int wv = tid >> 6;
  const int32_t W = (d + 63) >> 6;
  const int32_t S = HBM ? W : (int32_t)lgs_block_stride_words(W);  // row stride
  // hash of L: at least 2d slots (load factor <= 1/2), up to four times as
  // many where the launch's tile area (all of the LDS below the sort area,
  // sized for its largest root) still holds them beside the rows: most
  // elements of a row's out-list are not in L, and a lookup that misses
  // ends after fewer probes in an emptier table
  int32_t bits = lgs_hash_bits(d);
  {
    const int64_t avail = sort_area - lds;
    const int64_t rows = HBM ? 0 : 2 * (int64_t)d * S;
    for (int e = 0; e < 2; ++e) {
      if (lgs_hash_offset(d) + 2 * (int64_t(1) << (bits + 1)) + rows > avail) break;
      ++bits;
    }
  }
  int32_t* L = lds;
  int32_t* P = lds + d;
  unsigned long long* H = (unsigned long long*)(lds + lgs_hash_offset(d));
  unsigned long long* R =
      HBM ? Rg : (unsigned long long*)(lds + lgs_hash_offset(d) + 2 * (int64_t(1) << bits));
  const int32_t* Nu = col + rp[u];
  for (int32_t i = tid; i < (1 << bits); i += NT) H[i] = 0ull;
  if (k > 3)
    for (int32_t i = tid; i < d * S; i += NT) R[i] = 0ull;
  for (int32_t i = tid; i < d; i += NT) L[i] = Nu[i];
  if (tid == 0) *next = 0;
  __syncthreads();
  for (int32_t i = tid; i < d; i += NT) lgs_hash_put(H, bits, L[i], i);
  __syncthreads();
  if (CE && tid < 64) {
    ec.elems += (uint64_t)d * (uint64_t)d;
    ec.fetches += (uint64_t)d + 1;
  }
  // k = 3: every hit is a triangle at this root
  if (k == 3) {
    if (part != 0) return 0;
    if (!tri)
      return lgs_build_rows<CE, false>(rp, col, L, d, W, H, bits, R, wv, kBlockWaves, ec, next,
                                       (int32_t*)nullptr, nullptr, lg);
    // triangle scatter: P holds the per-row counters (edges u-L[i])
    for (int32_t i = tid; i < d; i += NT) P[i] = 0;
    __syncthreads();
    lgs_build_rows<CE, false, true>(rp, col, L, d, W, H, bits, R, wv, kBlockWaves, ec, next, P,
                                    tri, lg);
    __syncthreads();
    const int64_t e0 = rp[u];
    for (int32_t i = tid; i < d; i += NT)
      if (P[i]) atomicAdd(&tri[e0 + i], (unsigned int)P[i]);
    return 0;
  }
  lgs_build_rows<CE, true>(rp, col, L, d, S, H, bits, R, wv, kBlockWaves, ec, next,
                          (int32_t*)nullptr, nullptr, lg);
  __syncthreads();
  uint64_t c = 0;
  // pairs (i, j) with j in row i, enumerated through a prefix over row sizes
  // (thread t holds rows t * rpt .. t * rpt + rpt - 1)
  const int32_t rpt = (d + NT - 1) / NT;
  int32_t pcr[2] = {0, 0};
  for (int32_t q = 0; q < rpt; ++q) {
    const int32_t i = tid * rpt + q;
    if (i < d)
      for (int32_t w = 0; w < W; ++w) pcr[q] += __popcll(R[(size_t)i * S + w]);
  }
  int32_t pairs = 0;
  const int32_t inc2 = block_incl_scan(pcr[0] + pcr[1], tmp, pairs);
  {
    int32_t run = inc2 - pcr[0] - pcr[1];
    for (int32_t q = 0; q < rpt; ++q) {
      const int32_t i = tid * rpt + q;
      run += pcr[q];
      if (i < d) P[i + 1] = run;
    }
  }
  if (tid == 0) P[0] = 0;
  __syncthreads();
  const int32_t p0 = (int32_t)((int64_t)pairs * part / parts);
  const int32_t p1 = (int32_t)((int64_t)pairs * (part + 1) / parts);
  if (k == 4) {
    // each thread a contiguous slice of the local edges, walked row by row
    const int32_t per = (p1 - p0 + NT - 1) / NT;
    const int32_t t0 = min(p1, p0 + tid * per), t1 = min(p1, t0 + per);
    lgs_edge_walk(P, R, d, W, S, t0, t1, [&](int32_t i, int32_t j) {
      const unsigned long long* Ri = R + (size_t)i * S;
      const unsigned long long* Rj = R + (size_t)j * S;
      const int32_t x0 = ordered ? ((j + 1) >> 6) : 0;
      uint32_t cp = 0;
      for (int32_t x = x0; x < W; ++x) cp += (uint32_t)__popcll(Ri[x] & Rj[x]);
      c += cp;
      if (CE) ec.words += (uint64_t)(W - x0);
    });
    return c;
  }
  if (!CE && ordered) {
    int32_t* ids = sort_area + (size_t)wv * kSortWords;
    int32_t* bcnt = ids + kSortBatch;
    // rows in HBM (local graphs above the LDS tile): one wide instance for
    // every width up to kLgsMaxVertices / 64 words
    if constexpr (HBM) {
      if (W <= kLgsMaxVertices / 64)
        return lgs_pairs5_sorted<kLgsMaxVertices / 64>(P, R, d, W, W, p0, p1, ids, bcnt);
    } else {
    switch (W) {
#define GPM_LGSB5(WC) \
  case WC:            \
    return lgs_pairs5_sorted<WC>(P, R, d, WC, (int32_t)lgs_block_stride_words(WC), p0, p1, \
                                  ids, bcnt);
      GPM_LGSB5(1) GPM_LGSB5(2) GPM_LGSB5(3) GPM_LGSB5(4) GPM_LGSB5(5) GPM_LGSB5(6)
      GPM_LGSB5(7) GPM_LGSB5(8) GPM_LGSB5(9) GPM_LGSB5(10) GPM_LGSB5(11) GPM_LGSB5(12)
      GPM_LGSB5(13) GPM_LGSB5(14) GPM_LGSB5(15) GPM_LGSB5(16)
#undef GPM_LGSB5
      default: break;
    }
    }
  }
  // instrumented or unordered: words recomputed
  for (int32_t t = p0 + tid; t < p1; t += NT) {
    const int32_t i = upper_bound(P + 1, d, t);
    int32_t r = t - P[i];
    const unsigned long long* Ri = R + (size_t)i * S;
    int32_t w = 0;
    for (;; ++w) {
      const int32_t q = __popcll(Ri[w]);
      if (r < q) break;
      r -= q;
    }
    const int32_t j = w * 64 + select64(Ri[w], r);
    const unsigned long long* Rj = R + (size_t)j * S;
    const int32_t jw = ordered ? ((j + 1) >> 6) : 0;
    if (CE) ec.words += (uint64_t)(W - jw);
    for (int32_t x = jw; x < W; ++x) {
      uint64_t m = Ri[x] & Rj[x];
      while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1ull;
        const unsigned long long* Rl = R + (size_t)(x * 64 + b) * S;
        const int32_t y0 = ordered ? x : 0;
        for (int32_t y = y0; y < W; ++y) c += (uint64_t)__popcll(Ri[y] & Rj[y] & Rl[y]);
        if (CE) ec.words += (uint64_t)(W - y0);
      }
    }
  }
  return c;
}

// ---------------------------------------------------------------------------
// generic plan-driven DFS (Alg. 1 generalised by the plan table)
// ---------------------------------------------------------------------------

// How a DFS set operation probes its lists (Sec. 6.1): plain binary search
// in global memory; a merge-path window (for each chunk of 64 base elements,
// the probed list's range between the chunk's first and last element staged
// in LDS when it holds at most kMergeWin elements, and searched there; for a
// lane's own leaf, a galloping merge along each list); or binary search with
// the top kBstLevels of each probed list's search tree in LDS.
struct SetOp {
  int32_t mode;            // kSetopBinary, kSetopMerge, kSetopBst
  int32_t* lds;            // the wave's area: kMergeWin window | kBstNodes pivots per list
  int32_t choose;          // the plan's leaf_choose (counting-only leaf)
};
constexpr int kMergeWin = 256;

struct DfsState {
  int32_t v[kMaxK];        // matched data vertices by depth
  int32_t sz[kMaxK];       // candidate set size by depth
  int32_t ix[kMaxK];       // iteration index by depth
  int32_t pad;
  const int32_t* set[kMaxK];  // candidate set elements by depth
};

// Candidate set of depth `d` (Sec. 2.2 connectivity constraints + symmetry
// bounds; in vertex-induced mode also the non-adjacency constraints).
// STORE: materialise into `out` and return its (uniform) size.
// !STORE: return this lane's share of the set size (count-only leaf).
// Slice levels return the bounded base length and point st.set[d] at it.
template <bool STORE, bool CE>
__device__ __forceinline__ int32_t dfs_level(const int64_t* __restrict__ rp,
                                             const int32_t* __restrict__ col,
                                             const LevelPlan& L, DfsState& st, int d,
                                             int32_t* out, const SetOp& so, ElemCounter& ec) {
  int32_t bound = INT_MAX;
  for (int j = 0; j < d; ++j)
    if ((L.bound_mask >> j) & 1) bound = min(bound, st.v[j]);

  const int32_t* base;
  int32_t blen;
  int base_i = -1;
  if (L.base_buf >= 0) {
    base = st.set[L.base_buf];
    blen = st.sz[L.base_buf];
  } else {
    blen = INT_MAX;
    base = nullptr;
    for (int i = 0; i < L.n_int; ++i) {
      int32_t vj = st.v[L.int_lv[i]];
      int32_t len = (int32_t)(rp[vj + 1] - rp[vj]);
      if (len < blen) { blen = len; base_i = i; base = col + rp[vj]; }
    }
  }
  blen = uni(lower_bound(base, uni(blen), bound));
  const int n_probe = L.n_int - (base_i >= 0 ? 1 : 0);

  if (CE) {
    uint64_t e = (uint64_t)blen;
    for (int i = 0; i < L.n_int; ++i) {
      if (i == base_i) continue;
      int32_t vj = st.v[L.int_lv[i]];
      e += (uint64_t)(rp[vj + 1] - rp[vj]);
    }
    for (int i = 0; i < L.n_sub; ++i) {
      int32_t vj = st.v[L.sub_lv[i]];
      e += (uint64_t)(rp[vj + 1] - rp[vj]);
    }
    ec.elems += e;
    ec.fetches += 1 + n_probe + L.n_sub;
  }

  if (L.flags & kLvSlice) {
    st.set[d] = base;
    return blen;
  }

  if (!STORE && n_probe == 0 && L.n_sub == 0) {
    // size-only leaf: |bounded base| minus the excluded matched vertices in it
    if (lane_id() != 0) return 0;
    int32_t c = blen;
    for (int j = 0; j < d; ++j)
      if ((L.excl_mask >> j) & 1)
        if (st.v[j] < bound && member(base, blen, st.v[j])) --c;
    return c;
  }

  const int l = lane_id();
  int32_t* piv = so.lds + kMergeWin;
  if (so.mode == kSetopBst) {
    // the top of each probed list's search tree, once for the whole level
    int qq = 0;
    for (int q = 0; q < L.n_int; ++q) {
      if (q == base_i) continue;
      const int32_t vj = st.v[L.int_lv[q]];
      bst_stage(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), piv + kBstNodes * qq++);
    }
    for (int q = 0; q < L.n_sub; ++q) {
      const int32_t vj = st.v[L.sub_lv[q]];
      bst_stage(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), piv + kBstNodes * qq++);
    }
    wave_sync_mem();
  }
  int32_t total = 0;
  for (int32_t ib = 0; ib < blen; ib += 64) {
    int32_t i = ib + l;
    bool keep = i < blen;
    int32_t x = keep ? base[i] : 0;
    if (so.mode == kSetopMerge) {
      // each probed list's range between the chunk's first and last element
      const int32_t xf = uni(base[ib]);
      const int32_t xl = uni(base[min(ib + 63, blen - 1)]);
      for (int q = 0; q < L.n_int + L.n_sub; ++q) {
        const bool sub = q >= L.n_int;
        if (!sub && q == base_i) continue;
        const int32_t vj = st.v[sub ? L.sub_lv[q - L.n_int] : L.int_lv[q]];
        const int32_t* N = col + rp[vj];
        const int32_t n = (int32_t)(rp[vj + 1] - rp[vj]);
        const int32_t p0 = uni(lower_bound(N, n, xf));
        const int32_t wl = uni(upper_bound(N, n, xl)) - p0;
        bool m;
        if (wl <= kMergeWin) {
          for (int32_t t = l; t < wl; t += 64) so.lds[t] = N[p0 + t];
          wave_sync_mem();
          m = member(so.lds, wl, x);
          wave_sync_mem();
        } else {
          m = member(N + p0, wl, x);
        }
        keep = keep && (sub ? !m : m);
      }
    } else if (so.mode == kSetopBst) {
      int qq = 0;
      for (int q = 0; q < L.n_int; ++q) {
        if (q == base_i) continue;
        const int32_t vj = st.v[L.int_lv[q]];
        const int32_t* N = col + rp[vj];
        const int32_t n = (int32_t)(rp[vj + 1] - rp[vj]);
        if (keep) {
          const int32_t p = lower_bound_bst(N, n, x, piv + kBstNodes * qq);
          keep = p < n && N[p] == x;
        }
        ++qq;
      }
      for (int q = 0; q < L.n_sub; ++q) {
        const int32_t vj = st.v[L.sub_lv[q]];
        const int32_t* N = col + rp[vj];
        const int32_t n = (int32_t)(rp[vj + 1] - rp[vj]);
        if (keep) {
          const int32_t p = lower_bound_bst(N, n, x, piv + kBstNodes * qq);
          keep = !(p < n && N[p] == x);
        }
        ++qq;
      }
    } else {
      for (int q = 0; q < L.n_int && keep; ++q) {
        if (q == base_i) continue;
        int32_t vj = st.v[L.int_lv[q]];
        const int32_t* N = col + rp[vj];
        keep = member(N, (int32_t)(rp[vj + 1] - rp[vj]), x);
      }
      for (int q = 0; q < L.n_sub && keep; ++q) {
        int32_t vj = st.v[L.sub_lv[q]];
        const int32_t* N = col + rp[vj];
        keep = !member(N, (int32_t)(rp[vj + 1] - rp[vj]), x);
      }
    }
    for (int j = 0; j < d && keep; ++j)
      if ((L.excl_mask >> j) & 1) keep = x != st.v[j];
    if (STORE) {
      uint64_t m = wave_ballot(keep);
      if (keep) out[total + (int32_t)lanes_below(m)] = x;
      total += (int32_t)__popcll(m);
    } else {
      total += keep ? 1 : 0;
    }
  }
  if (STORE) {
    wave_sync_mem();
    st.set[d] = out;
    if (CE) ec.written += (uint64_t)total;
  }
  return total;
}

// C(n, r) mod 2^64 for r <= kMaxK - 2: the factors of r! are divided out of
// the r numerator terms first (r consecutive integers hold them all), so the
// product of what remains is exact modulo 2^64.
__device__ __forceinline__ uint64_t choose_mod64(uint64_t n, int r) {
  if (n < (uint64_t)r) return 0;
  uint64_t t[kMaxK];
#pragma unroll
  for (int i = 0; i < kMaxK; ++i) t[i] = i < r ? n - (uint64_t)i : 1;
  for (int j = 2; j <= r; ++j) {
    int m = j;
    for (int p = 2; p <= 5; ++p)
      while (m % p == 0) {
        m /= p;
#pragma unroll
        for (int i = 0; i < kMaxK; ++i)
          if (i < r && t[i] % (uint64_t)p == 0) {
            t[i] /= (uint64_t)p;
            break;
          }
      }
  }
  uint64_t c = 1;
#pragma unroll
  for (int i = 0; i < kMaxK; ++i) c *= t[i];
  return c;
}

// What a leaf set of size n counts: n, or under counting-only pruning
// (Plan::leaf_choose = r | ext << 8) ext * C(n, r).
__device__ __forceinline__ uint64_t leaf_term(uint64_t n, int32_t choose) {
  if (choose == 0) return n;
  return (uint64_t)(choose >> 8) * choose_mod64(n, choose & 0xff);
}

// Leaf of a wave-wide set operation: the lanes' shares of the set size;
// under counting-only pruning the term of the whole set goes to lane 0.
__device__ __forceinline__ uint64_t leaf_wave(int32_t share, int32_t choose) {
  if (choose == 0) return (uint64_t)share;
  int32_t n = share;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
  return lane_id() == 0 ? leaf_term((uint64_t)n, choose) : 0;
}

__device__ __forceinline__ bool slice_excluded(const LevelPlan& L, const DfsState& st,
                                               int d, int32_t x) {
  for (int j = 0; j < d; ++j)
    if (((L.excl_mask >> j) & 1) && st.v[j] == x) return true;
  return false;
}

// Leaf count of depth d for THIS lane's matched vertices (st.v differs per
// lane), computed serially by the lane.  Returns false -- and counts nothing
// -- when the bounded base set is longer than cap, so that the caller can
// hand that candidate to the wave-wide set operation instead.
template <bool CE>
__device__ __forceinline__ bool leaf_serial(const int64_t* __restrict__ rp,
                                            const int32_t* __restrict__ col,
                                            const LevelPlan& L, const DfsState& st, int d,
                                            int32_t cap, const SetOp& so, uint64_t& count,
                                            ElemCounter& ec) {
  int32_t bound = INT_MAX;
  for (int j = 0; j < d; ++j)
    if ((L.bound_mask >> j) & 1) bound = min(bound, st.v[j]);
  const int32_t* base;
  int32_t blen;
  int base_i = -1;
  if (L.base_buf >= 0) {
    base = st.set[L.base_buf];
    blen = st.sz[L.base_buf];
  } else {
    blen = INT_MAX;
    base = nullptr;
    for (int i = 0; i < L.n_int; ++i) {
      int32_t vj = st.v[L.int_lv[i]];
      int32_t len = (int32_t)(rp[vj + 1] - rp[vj]);
      if (len < blen) { blen = len; base_i = i; base = col + rp[vj]; }
    }
  }
  blen = lower_bound(base, blen, bound);
  const int n_probe = L.n_int - (base_i >= 0 ? 1 : 0);
  if (n_probe == 0 && L.n_sub == 0) {
    int32_t c = blen;
    for (int j = 0; j < d; ++j)
      if ((L.excl_mask >> j) & 1)
        if (st.v[j] < bound && member(base, blen, st.v[j])) --c;
    count += leaf_term((uint64_t)c, so.choose);
    if (CE) { ec.elems += (uint64_t)blen * 64; ec.fetches += 64; }
    return true;
  }
  if (blen > cap) return false;
  uint64_t c = 0;
  if (so.mode == kSetopMerge) {
    // the base ascends, so each probed list is walked once, galloping from
    // where the previous element left it
    int32_t pi[kMaxK], ps[kMaxK];
#pragma unroll
    for (int q = 0; q < kMaxK; ++q) pi[q] = ps[q] = 0;
    for (int32_t i = 0; i < blen; ++i) {
      const int32_t x = base[i];
      bool keep = true;
#pragma unroll
      for (int q = 0; q < kMaxK; ++q) {
        if (q < L.n_int && q != base_i && keep) {
          const int32_t vj = st.v[L.int_lv[q]];
          const int32_t* N = col + rp[vj];
          const int32_t n = (int32_t)(rp[vj + 1] - rp[vj]);
          pi[q] = gallop_lb(N, pi[q], n, x);
          keep = pi[q] < n && N[pi[q]] == x;
        }
      }
#pragma unroll
      for (int q = 0; q < kMaxK; ++q) {
        if (q < L.n_sub && keep) {
          const int32_t vj = st.v[L.sub_lv[q]];
          const int32_t* N = col + rp[vj];
          const int32_t n = (int32_t)(rp[vj + 1] - rp[vj]);
          ps[q] = gallop_lb(N, ps[q], n, x);
          keep = !(ps[q] < n && N[ps[q]] == x);
        }
      }
      for (int j = 0; j < d && keep; ++j)
        if ((L.excl_mask >> j) & 1) keep = x != st.v[j];
      c += keep ? 1u : 0u;
    }
  } else {
    for (int32_t i = 0; i < blen; ++i) {
      const int32_t x = base[i];
      bool keep = true;
      for (int q = 0; q < L.n_int && keep; ++q) {
        if (q == base_i) continue;
        int32_t vj = st.v[L.int_lv[q]];
        keep = member(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), x);
      }
      for (int q = 0; q < L.n_sub && keep; ++q) {
        int32_t vj = st.v[L.sub_lv[q]];
        keep = !member(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), x);
      }
      for (int j = 0; j < d && keep; ++j)
        if ((L.excl_mask >> j) & 1) keep = x != st.v[j];
      c += keep ? 1u : 0u;
    }
  }
  if (CE) {
    uint64_t e = (uint64_t)blen;
    for (int q = 0; q < L.n_int; ++q) {
      if (q == base_i) continue;
      int32_t vj = st.v[L.int_lv[q]];
      e += (uint64_t)(rp[vj + 1] - rp[vj]);
    }
    for (int q = 0; q < L.n_sub; ++q) {
      int32_t vj = st.v[L.sub_lv[q]];
      e += (uint64_t)(rp[vj + 1] - rp[vj]);
    }
    ec.elems += e * 64;
    ec.fetches += (uint64_t)(1 + n_probe + L.n_sub) * 64;
  }
  count += leaf_term(c, so.choose);
  return true;
}

// All leaves below the candidates of depth d = k-2: one candidate per lane
// (leaf_serial); candidates whose leaf set exceeds cap are queued in defq
// and counted with the wave-wide set operation.
template <bool CE>
__device__ uint64_t leaf_bulk(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const Plan& P, int d, DfsState& st, int32_t cap, int32_t* defq,
                              const SetOp& so, ElemCounter& ec) {
  const LevelPlan& Ld = P.lv[d];
  const LevelPlan& L = P.lv[d + 1];
  const int32_t sz = uni(st.sz[d]);
  const int32_t* set = st.set[d];
  const int l = lane_id();
  uint64_t c = 0;
  for (int32_t ib = 0; ib < sz; ib += 64) {
    const int32_t i = ib + l;
    bool act = i < sz;
    int32_t x = act ? set[i] : 0;
    if (act && (Ld.flags & kLvSlice) && slice_excluded(Ld, st, d, x)) act = false;
    bool defer = false;
    if (act) {
      st.v[d] = x;
      uint64_t cnt = 0;
      if (leaf_serial<CE>(rp, col, L, st, d + 1, cap, so, cnt, ec)) c += cnt;
      else defer = true;
    }
    const uint64_t dm = wave_ballot(defer);
    if (dm) {
      if (defer) defq[lanes_below(dm)] = x;
      wave_sync_mem();
      const int nd = (int)__popcll(dm);
      for (int q = 0; q < nd; ++q) {
        st.v[d] = uni(defq[q]);
        c += leaf_wave(dfs_level<false, CE>(rp, col, L, st, d + 1, nullptr, so, ec), so.choose);
      }
      wave_sync_mem();
    }
  }
  return c;
}

// All matches extending the root (v0, v1): the depth-first walk over depths
// 2 .. k-1; depth k-1 is count-only.  Wave-uniform control flow throughout
// except inside leaf_bulk, where each lane owns one last-level candidate.
template <bool CE>
__device__ uint64_t dfs_root(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const Plan& P, int32_t v0, int32_t v1, int32_t* fb,
                             int32_t cap, int32_t leaf_cap, DfsState& st, int32_t* defq,
                             const SetOp& so, ElemCounter& ec) {
  const int k = P.k;
  st.v[0] = v0;
  st.v[1] = v1;
  if (k == 3) return leaf_wave(dfs_level<false, CE>(rp, col, P.lv[2], st, 2, nullptr, so, ec), so.choose);
  uint64_t c = 0;
  int d = 2;
  {
    int32_t* out = fb + (size_t)(P.store_slot[2] < 0 ? 0 : P.store_slot[2]) * cap;
    st.sz[2] = uni(dfs_level<true, CE>(rp, col, P.lv[2], st, 2, out, so, ec));
    st.ix[2] = 0;
  }
  for (;;) {
    if (d == k - 2) {
      if (leaf_cap > 0) {
        c += leaf_bulk<CE>(rp, col, P, d, st, leaf_cap, defq, so, ec);
      } else {
        for (int32_t i = 0; i < st.sz[d]; ++i) {
          int32_t x = uni(st.set[d][i]);
          if ((P.lv[d].flags & kLvSlice) && slice_excluded(P.lv[d], st, d, x)) continue;
          st.v[d] = x;
          c += leaf_wave(dfs_level<false, CE>(rp, col, P.lv[d + 1], st, d + 1, nullptr, so, ec),
                         so.choose);
        }
      }
      if (d == 2) break;
      --d;
      ++st.ix[d];
      continue;
    }
    if (st.ix[d] >= st.sz[d]) {
      if (d == 2) break;
      --d;
      ++st.ix[d];
      continue;
    }
    int32_t x = uni(st.set[d][st.ix[d]]);
    if ((P.lv[d].flags & kLvSlice) && slice_excluded(P.lv[d], st, d, x)) {
      ++st.ix[d];
      continue;
    }
    st.v[d] = x;
    ++d;
    int32_t* out = fb + (size_t)(P.store_slot[d] < 0 ? 0 : P.store_slot[d]) * cap;
    st.sz[d] = uni(dfs_level<true, CE>(rp, col, P.lv[d], st, d, out, so, ec));
    st.ix[d] = 0;
  }
  return c;
}

// ---------------------------------------------------------------------------
// listing (Sec. 2.1: every match is enumerated instead of counted)
// ---------------------------------------------------------------------------

// Rows are staged per wave in LDS and written out in groups: one atomic
// claim of the group's rows on the shared row counter, then a contiguous,
// coalesced copy.  (A claim per 64-candidate batch serialises the whole
// grid on that one counter.)
constexpr int kListStageWords = 2048;   // int32 words of staged rows per wave
constexpr int kListProbeWords = 512;    // per wave: a leaf's probed list, when it fits

// Write the wave's n staged rows (row-major, k words each) to the output and
// empty the stage; rows at or beyond out_cap are counted and dropped.
__device__ __forceinline__ void list_flush(const ListArgs& a, const int32_t* stage, int32_t& n) {
  if (n == 0) return;
  wave_sync_mem();
  unsigned long long first = 0;
  if (lane_id() == 0) first = atomicAdd(a.rows, (unsigned long long)n);
  const int64_t row0 = (int64_t)__shfl(first, 0, 64);
  const int64_t fit = min((int64_t)n, a.out_cap - row0);
  if (fit > 0) {
    int32_t* o = a.out + row0 * a.k;
    const int32_t words = (int32_t)fit * a.k;
    for (int32_t i = lane_id(); i < words; i += 64) o[i] = stage[i];
  }
  n = 0;
  wave_sync_mem();
}

// Stage the rows of the lanes set in m (this lane's row when keep); flush
// once another full batch might not fit.  The stage holds stage_rows rows,
// and n <= stage_rows - 64 holds before every batch.
__device__ __forceinline__ int32_t* stage_row(int32_t* stage, int32_t n, uint64_t m, int k) {
  return stage + (n + (int32_t)lanes_below(m)) * k;
}

// The first probed list of a listing depth (index q0 among the lists to
// intersect, -1 if none), copied to the wave's LDS area when it fits so the
// lanes' binary searches run in LDS instead of as chains of global loads.
__device__ __forceinline__ const int32_t* list_probe_list(const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const LevelPlan& L,
                                                          const DfsState& st, int base_i,
                                                          int32_t* probe, int& q0, int32_t& n0) {
  q0 = -1;
  n0 = 0;
  for (int q = 0; q < L.n_int; ++q)
    if (q != base_i) { q0 = q; break; }
  if (q0 < 0) return nullptr;
  const int32_t v = st.v[L.int_lv[q0]];
  const int32_t* N = col + rp[v];
  n0 = (int32_t)(rp[v + 1] - rp[v]);
  if (n0 > kListProbeWords) return N;
  wave_sync_mem();  // earlier searches are done with the area
  for (int32_t i = lane_id(); i < n0; i += 64) probe[i] = N[i];
  wave_sync_mem();
  return probe;
}

// A stored (or sliced) depth d < k-1 of a listing walk: the candidate set as
// dfs_level<true> forms it, with the leaf's two latency cuts (no search for a
// bound the plan does not have; the first probed list searched in LDS).
__device__ __forceinline__ int32_t list_level(const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ col,
                                              const LevelPlan& L, DfsState& st, int d,
                                              int32_t* out, int32_t* probe) {
  int32_t bound = INT_MAX;
  for (int j = 0; j < d; ++j)
    if ((L.bound_mask >> j) & 1) bound = min(bound, st.v[j]);
  const int32_t* base;
  int32_t blen;
  int base_i = -1;
  if (L.base_buf >= 0) {
    base = st.set[L.base_buf];
    blen = st.sz[L.base_buf];
  } else {
    blen = INT_MAX;
    base = nullptr;
    for (int i = 0; i < L.n_int; ++i) {
      int32_t vj = st.v[L.int_lv[i]];
      int32_t len = (int32_t)(rp[vj + 1] - rp[vj]);
      if (len < blen) { blen = len; base_i = i; base = col + rp[vj]; }
    }
  }
  if (bound != INT_MAX) blen = uni(lower_bound(base, uni(blen), bound));
  if (L.flags & kLvSlice) {
    st.set[d] = base;
    return blen;
  }
  int q0;
  int32_t n0;
  const int32_t* N0 = blen > 0 ? list_probe_list(rp, col, L, st, base_i, probe, q0, n0) : nullptr;
  if (blen <= 0) q0 = -1;
  const int l = lane_id();
  int32_t total = 0;
  for (int32_t ib = 0; ib < blen; ib += 64) {
    const int32_t i = ib + l;
    bool keep = i < blen;
    const int32_t x = keep ? base[i] : 0;
    if (q0 >= 0 && keep) keep = member(N0, n0, x);
    for (int q = 0; q < L.n_int && keep; ++q) {
      if (q == base_i || q == q0) continue;
      int32_t vj = st.v[L.int_lv[q]];
      keep = member(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), x);
    }
    for (int q = 0; q < L.n_sub && keep; ++q) {
      int32_t vj = st.v[L.sub_lv[q]];
      keep = !member(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), x);
    }
    for (int j = 0; j < d && keep; ++j)
      if ((L.excl_mask >> j) & 1) keep = x != st.v[j];
    const uint64_t m = wave_ballot(keep);
    if (keep) out[total + (int32_t)lanes_below(m)] = x;
    total += (int32_t)__popcll(m);
  }
  wave_sync_mem();
  st.set[d] = out;
  return total;
}

// The leaf depth d = k-1 of a listing walk.  Its candidate set is formed as
// dfs_level forms it (bounded base, membership probes, subtractions in
// vertex-induced mode, explicit exclusion of matched vertices), one candidate
// per lane, but is never reduced to a size: every surviving candidate
// completes one match, staged as a row in the caller's vertex ids.
__device__ __forceinline__ void list_leaf(const int64_t* __restrict__ rp,
                                          const int32_t* __restrict__ col, const ListArgs& a,
                                          const LevelPlan& L, const DfsState& st, int d,
                                          int32_t first_hint, int32_t* probe, int32_t* stage,
                                          int32_t& stage_n, int32_t stage_rows) {
  int32_t bound = INT_MAX;
  for (int j = 0; j < d; ++j)
    if ((L.bound_mask >> j) & 1) bound = min(bound, st.v[j]);
  const int32_t* base;
  int32_t blen;
  int base_i = -1;
  if (L.base_buf >= 0) {
    base = st.set[L.base_buf];
    blen = st.sz[L.base_buf];
  } else {
    blen = INT_MAX;
    base = nullptr;
    for (int i = 0; i < L.n_int; ++i) {
      int32_t vj = st.v[L.int_lv[i]];
      int32_t len = (int32_t)(rp[vj + 1] - rp[vj]);
      if (len < blen) { blen = len; base_i = i; base = col + rp[vj]; }
    }
  }
  if (bound != INT_MAX) blen = uni(lower_bound(base, uni(blen), bound));
  // ordered DAG: the leaf set lies in N+(v_{d-1}), above v_{d-1}; skip the
  // sorted base's prefix up to it (first_hint >= 0: its length, known to
  // the caller)
  int32_t first = 0;
  if (a.ordered) first = first_hint >= 0 ? first_hint : uni(lower_bound(base, blen, st.v[d - 1] + 1));
  // the caller's ids of the matched vertices, by depth
  int32_t mv[kMaxK - 1];
#pragma unroll
  for (int j = 0; j < kMaxK - 1; ++j)
    mv[j] = j < d ? (a.ids ? a.ids[st.v[j]] : st.v[j]) : 0;
  const int l = lane_id();
  // the first probed list, copied to the wave's LDS area when it fits: the
  // lanes' binary searches then run in LDS instead of as chains of global loads
  int q0 = -1;
  int32_t n0 = 0;
  const int32_t* N0 = nullptr;
  if (first < blen) N0 = list_probe_list(rp, col, L, st, base_i, probe, q0, n0);
  for (int32_t ib = first; ib < blen; ib += 64) {
    const int32_t i = ib + l;
    bool keep = i < blen;
    const int32_t x = keep ? base[i] : 0;
    if (q0 >= 0 && keep) keep = member(N0, n0, x);
    for (int q = 0; q < L.n_int && keep; ++q) {
      if (q == base_i || q == q0) continue;
      int32_t vj = st.v[L.int_lv[q]];
      keep = member(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), x);
    }
    for (int q = 0; q < L.n_sub && keep; ++q) {
      int32_t vj = st.v[L.sub_lv[q]];
      keep = !member(col + rp[vj], (int32_t)(rp[vj + 1] - rp[vj]), x);
    }
    for (int j = 0; j < d && keep; ++j)
      if ((L.excl_mask >> j) & 1) keep = x != st.v[j];
    const uint64_t m = wave_ballot(keep);
    if (!m) continue;
    if (keep) {
      int32_t* o = stage_row(stage, stage_n, m, a.k);
#pragma unroll
      for (int j = 0; j < kMaxK - 1; ++j)
        if (j < d) o[a.out_col[j]] = mv[j];
      o[a.out_col[d]] = a.ids ? a.ids[x] : x;
    }
    stage_n += (int32_t)__popcll(m);
    if (stage_n > stage_rows - 64) list_flush(a, stage, stage_n);
  }
}

// All matches extending the root (v0, v1), for k >= 3: the walk of dfs_root
// over depths 2 .. k-2 (stored or sliced candidate sets, wave-uniform), with
// the leaf depth emitted by list_leaf.
__device__ void list_root(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const ListArgs& a, int32_t v0, int32_t v1, int32_t* fb,
                          DfsState& st, int32_t* probe, int32_t* stage, int32_t& stage_n,
                          int32_t stage_rows) {
  const Plan& P = a.plan;
  const int k = P.k;
  st.v[0] = v0;
  st.v[1] = v1;
  if (k == 3) {
    list_leaf(rp, col, a, P.lv[2], st, 2, -1, probe, stage, stage_n, stage_rows);
    return;
  }
  int d = 2;
  {
    int32_t* out = fb + (size_t)(P.store_slot[2] < 0 ? 0 : P.store_slot[2]) * a.cap;
    st.sz[2] = uni(list_level(rp, col, P.lv[2], st, 2, out, probe));
    st.ix[2] = 0;
  }
  for (;;) {
    if (d == k - 2) {
      for (int32_t i = 0; i < st.sz[d]; ++i) {
        const int32_t x = uni(st.set[d][i]);
        if ((P.lv[d].flags & kLvSlice) && slice_excluded(P.lv[d], st, d, x)) continue;
        st.v[d] = x;
        // the leaf's base is this depth's set: its prefix up to x is [0, i]
        const int32_t hint = P.lv[d + 1].base_buf == d ? i + 1 : -1;
        list_leaf(rp, col, a, P.lv[d + 1], st, d + 1, hint, probe, stage, stage_n, stage_rows);
      }
      if (d == 2) break;
      --d;
      ++st.ix[d];
      continue;
    }
    if (st.ix[d] >= st.sz[d]) {
      if (d == 2) break;
      --d;
      ++st.ix[d];
      continue;
    }
    const int32_t x = uni(st.set[d][st.ix[d]]);
    if ((P.lv[d].flags & kLvSlice) && slice_excluded(P.lv[d], st, d, x)) {
      ++st.ix[d];
      continue;
    }
    st.v[d] = x;
    ++d;
    int32_t* out = fb + (size_t)(P.store_slot[d] < 0 ? 0 : P.store_slot[d]) * a.cap;
    st.sz[d] = uni(list_level(rp, col, P.lv[d], st, d, out, probe));
    st.ix[d] = 0;
  }
}

// Persistent listing kernel: each wave pops chunks of root tasks from one
// queue counter until the tasks run out.  For k <= 2 a root task is itself a
// match (a vertex, or an edge taken once).
__global__ void __launch_bounds__(kWavesPerBlock * 64) gpm_list(ListArgs a) {
  __shared__ int32_t list_stage[kWavesPerBlock][kListStageWords];
  __shared__ int32_t list_probe[kWavesPerBlock][kListProbeWords];
  const int w = threadIdx.x >> 6;
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + w;
  int32_t* fb = a.fbuf ? a.fbuf + gw * a.wave_stride : nullptr;
  int32_t* stage = list_stage[w];
  const int32_t stage_rows = kListStageWords / a.k;
  int32_t stage_n = 0;
  DfsState st;
  for (;;) {
    unsigned long long c = 0;
    if (lane_id() == 0) c = atomicAdd(a.queue, 1ull);
    c = __shfl(c, 0, 64);
    const int64_t t0 = (int64_t)c * a.chunk;
    if (t0 >= a.n_tasks) break;
    const int64_t t1 = min(t0 + (int64_t)a.chunk, a.n_tasks);
    if (a.k <= 2) {
      for (int64_t tb = t0; tb < t1; tb += 64) {
        const int64_t t = tb + lane_id();
        const bool keep = t < t1;
        const uint64_t m = wave_ballot(keep);
        if (keep) {
          int32_t* o = stage_row(stage, stage_n, m, a.k);
          const int32_t u = a.task_src ? a.task_src[t] : (int32_t)t;
          o[a.out_col[0]] = a.ids ? a.ids[u] : u;
          if (a.k == 2) {
            const int32_t v = a.task_dst[t];
            o[a.out_col[1]] = a.ids ? a.ids[v] : v;
          }
        }
        stage_n += (int32_t)__popcll(m);
        if (stage_n > stage_rows - 64) list_flush(a, stage, stage_n);
      }
      continue;
    }
    for (int64_t t = t0; t < t1; ++t)
      list_root(a.rp, a.col, a, uni(a.task_src[t]), uni(a.task_dst[t]), fb, st, list_probe[w],
                stage, stage_n, stage_rows);
  }
  list_flush(a, stage, stage_n);
}

// ---------------------------------------------------------------------------
// the persistent kernel
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t pop_chunk(unsigned long long* qcnt, const int64_t* qbeg,
                                             int home, uint32_t& dead) {
  for (int i = 0; i < kQueues; ++i) {
    int x = (home + i) & (kQueues - 1);
    if ((dead >> x) & 1u) continue;
    // queue x owns chunks x, x + 8, x + 16, ... (qbeg[kQueues] = chunk count),
    // so heavy and light regions of the task list reach every XCD
    int64_t limit = (qbeg[kQueues] - x + kQueues - 1) / kQueues;
    unsigned long long c = 0;
    if (lane_id() == 0) c = atomicAdd(&qcnt[x * kQueueStride], 1ull);
    c = __shfl(c, 0, 64);
    if ((int64_t)c < limit) return (int64_t)c * kQueues + x;
    dead |= 1u << x;
  }
  return -1;
}

__device__ __forceinline__ int find_job(const int64_t* jbeg, int n_jobs, int64_t c) {
  int lo = 0, hi = n_jobs;  // jbeg[lo] <= c < jbeg[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (jbeg[mid] <= c) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void flush(unsigned long long* results, int slot, uint64_t* acc,
                                      int nf) {
  for (int f = 0; f < nf; ++f) {
    uint64_t s = wave_sum_u64(acc[f]);
    if (lane_id() == 0 && s) atomicAdd(&results[(size_t)slot * kResultFields + f], s);
    acc[f] = 0;
  }
}

// Root tasks [t0, t1) of a local-graph clique job, one wave per root; the
// tile is the wave's LDS area when the root fits it, else its HBM region.
template <bool CE, bool SC>
__device__ __forceinline__ void lgs_tasks(const Job& J, const KernelArgs& a, int32_t* my,
                                          int32_t* fb, int64_t t0, int64_t t1, uint64_t* acc,
                                          ElemCounter& ec) {
  const int64_t* __restrict__ rp = J.rp;
  const int32_t* __restrict__ col = J.col;
  const int k = J.k;
  for (int64_t t = t0; t < t1; ++t) {
    int32_t u = uni(J.task_src[t]);
    int32_t d = uni((int32_t)(rp[u + 1] - rp[u]));
    int32_t part = 0, parts = 1;
    if (J.task_dst) {  // split root: (part, parts) packed as part | parts << 16
      int32_t enc = uni(J.task_dst[t]);
      part = enc & 0xffff;
      parts = enc >> 16;
    }
    // tile layout (lgs_tile_words): L | P | H | R
    if (d <= a.lgs_tile) {
      int32_t* L = my;
      int32_t* Pp = L + a.lgs_tile;
      unsigned long long* H = (unsigned long long*)(my + lgs_hash_offset(a.lgs_tile));
      unsigned long long* R = (unsigned long long*)(my + lgs_rows_offset(a.lgs_tile));
      acc[0] += clique_lgs<CE, SC>(rp, col, k, u, d, part, parts, J.ordered != 0, L, Pp, H, R,
                                   J.tri, ec, a.lgs_lg);
    } else {
      int32_t* L = fb;
      int32_t* Pp = fb + J.cap;
      unsigned long long* H = (unsigned long long*)(fb + lgs_hash_offset(J.cap));
      unsigned long long* R = (unsigned long long*)(fb + lgs_rows_offset(J.cap));
      acc[0] += clique_lgs<CE, SC>(rp, col, k, u, d, part, parts, J.ordered != 0, L, Pp, H, R,
                                   J.tri, ec, a.lgs_lg);
    }
  }
}

template <uint32_t KINDS, bool CE>
__global__ void __launch_bounds__(kWavesPerBlock * 64)
gpm_persistent(KernelArgs a) {
  extern __shared__ int32_t lds[];
  __shared__ int32_t lds_state[kWavesPerBlock][2 * kMaxK];
  __shared__ int32_t dfs_defq[(KINDS & kKindDfs) ? kWavesPerBlock : 1][64];
  __shared__ int32_t dfs_setop[(KINDS & kKindDfs) ? kWavesPerBlock : 1]
                              [(KINDS & kKindDfs) ? kMergeWin + kBstNodes * kMaxK : 1];
  const int w = threadIdx.x >> 6;
  int32_t* my = lds + (size_t)w * a.lds_words;
  int32_t* st_words = lds_state[w];
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + w;
  int32_t* fb = a.fbuf ? a.fbuf + gw * a.wave_stride : nullptr;
  const int home = (int)(blockIdx.x & (kQueues - 1));  // blocks are dealt round-robin to XCDs
  uint32_t dead = 0;
  int cur = -1;
  int cur_slot = 0;
  int nf = 0;
  uint64_t acc[4] = {0, 0, 0, 0};
  ElemCounter ec;
  int32_t cached_u = -1;
  DfsState st;

  for (;;) {
    int64_t c = pop_chunk(a.queue_cnt, a.queue_begin, home, dead);
    if (c < 0) break;
    int j = uni(find_job(a.job_chunk_begin, a.n_jobs, c));
    if (j != cur) {
      if (cur >= 0) flush(a.results, cur_slot, acc, nf);
      cur = j;
      cached_u = -1;
    }
    const Job& J = a.jobs[j];
    const int kind = J.kind;
    cur_slot = J.slot;
    const int64_t t0 = (c - a.job_chunk_begin[j]) * (int64_t)J.chunk;
    const int64_t t1 = min(t0 + (int64_t)J.chunk, J.n_tasks);
    const int64_t* __restrict__ rp = J.rp;
    const int32_t* __restrict__ col = J.col;

    if ((KINDS & kKindClique) && kind == kJobClique) {
      nf = 1;
      const int k = J.k;
      for (int64_t t = t0; t < t1; ++t) {
        int32_t u = uni(J.task_src[t]);
        int32_t v = uni(J.task_dst[t]);
        int32_t du = uni((int32_t)(rp[u + 1] - rp[u]));
        if (J.lds_ok && du <= a.lds_cap) {
          // LDS tile: U | F_2 .. F_{k-2} | (pad to 8 B) | P (int64)
          int32_t* U = my;
          int32_t* bufs = my + a.lds_cap;
          int64_t* P = (int64_t*)(my + ((a.lds_cap + (size_t)(k - 3 > 0 ? k - 3 : 0) * a.lds_cap + 1) & ~(size_t)1));
          if (u != cached_u) {
            const int32_t* Nu = col + rp[u];
            for (int32_t i = lane_id(); i < du; i += 64) U[i] = Nu[i];
            wave_sync_mem();
            cached_u = u;
          }
          acc[0] += clique_edge<CE>(rp, col, k, (const int32_t*)U, du, v, bufs, P, a.lds_cap,
                                    st_words, ec);
        } else {
          const int32_t* U = col + rp[u];
          int32_t* bufs = fb;
          int64_t* P = (int64_t*)(fb + (((size_t)(k - 3 > 0 ? k - 3 : 0) * J.cap + 1) & ~(size_t)1));
          acc[0] += clique_edge<CE>(rp, col, k, U, du, v, bufs, P, J.cap, st_words, ec);
        }
      }
    } else if (((KINDS & kKindCliqueLgs) && kind == kJobCliqueLgs) ||
               ((KINDS & kKindTriScatter) && kind == kJobTriScatter)) {
      nf = 1;
      // the scatter variant is compiled only into instances that take it
      if constexpr ((KINDS & kKindTriScatter) != 0) {
        if (kind == kJobTriScatter)
          lgs_tasks<CE, true>(J, a, my, fb, t0, t1, acc, ec);
        else
          lgs_tasks<CE, false>(J, a, my, fb, t0, t1, acc, ec);
      } else {
        lgs_tasks<CE, false>(J, a, my, fb, t0, t1, acc, ec);
      }
    } else if ((KINDS & kKindDfs) && kind == kJobDfs) {
      nf = 1;
      const Plan& P = a.plans[J.plan];
      for (int64_t t = t0; t < t1; ++t) {
        if (J.vertex_tasks) {
          int32_t v0 = (int32_t)t;
          const int32_t* N0 = col + rp[v0];
          int32_t d0 = uni((int32_t)(rp[v0 + 1] - rp[v0]));
          int32_t end = P.root_bound ? uni(lower_bound(N0, d0, v0)) : d0;
          for (int32_t e = 0; e < end; ++e) {
            int32_t v1 = uni(N0[e]);
            acc[0] += dfs_root<CE>(rp, col, P, v0, v1, fb, J.cap, J.leaf_cap, st,
                                   dfs_defq[w], SetOp{J.setop, dfs_setop[w], P.leaf_choose}, ec);
          }
        } else {
          int32_t v0 = uni(J.task_src[t]);
          int32_t v1 = uni(J.task_dst[t]);
          acc[0] += dfs_root<CE>(rp, col, P, v0, v1, fb, J.cap, J.leaf_cap, st, dfs_defq[w],
                                 SetOp{J.setop, dfs_setop[w], P.leaf_choose},
                                 ec);
        }
      }
    } else if ((KINDS & kKindEdgeTri) && kind == kJobEdgeTri) {
      // per undirected edge e = (u, v), u > v: t_e = |N(u) ∩ N(v)|
      // f0 += t_e (3T in total), f1 += C(t_e, 2) (non-induced diamonds,
      // Alg. 3), f2 += t_e (d_u + d_v - 4) (twice the non-induced tailed
      // triangles), f3 += (d_u - 1)(d_v - 1) (4-paths through e as middle edge
      // plus 3 per triangle)
      nf = 4;
      for (int64_t t = t0; t < t1; ++t) {
        int32_t u = uni(J.task_src[t]);
        int32_t v = uni(J.task_dst[t]);
        int32_t du = uni((int32_t)(rp[u + 1] - rp[u]));
        int32_t dv = uni((int32_t)(rp[v + 1] - rp[v]));
        const int32_t* Nu = col + rp[u];
        const int32_t* Nv = col + rp[v];
        uint32_t part = (du <= dv) ? intersect_count(Nu, du, Nv, dv)
                                   : intersect_count(Nv, dv, Nu, du);
        if (CE) {
          ec.elems += (uint64_t)du + (uint64_t)dv;
          ec.fetches += 2;
        }
        uint64_t te = wave_sum_u64(part);
        te = (uint64_t)__shfl((unsigned long long)te, 0, 64);
        if (lane_id() == 0) {
          acc[0] += te;
          acc[1] += te * (te - (te ? 1 : 0)) / 2;
          acc[2] += te * (uint64_t)((int64_t)du + dv - 4);
          acc[3] += (uint64_t)(du - 1) * (uint64_t)(dv - 1);
        }
      }
    } else if ((KINDS & kKindEdgeTerms) && kind == kJobEdgeTerms) {
      // per DAG edge e = (u, v) with its triangle count t_e (left by the
      // scatter launches, reset here): the same four terms as kJobEdgeTri
      nf = 4;
      for (int64_t e = t0 + lane_id(); e < t1; e += 64) {
        const uint64_t te = J.tri[e];
        if (te) J.tri[e] = 0u;
        const int32_t u = J.task_src[e], v = col[e];
        const uint64_t du = (uint64_t)(J.deg_rp[u + 1] - J.deg_rp[u]);
        const uint64_t dv = (uint64_t)(J.deg_rp[v + 1] - J.deg_rp[v]);
        acc[0] += te;
        acc[1] += te * (te - (te ? 1 : 0)) / 2;
        acc[2] += te * (du + dv - 4);
        acc[3] += (du - 1) * (dv - 1);
      }
    } else if ((KINDS & kKindVertexDeg) && kind == kJobVertexDeg) {
      // f0 += C(d, 2), f1 += C(d, 3) over the chunk's vertices
      nf = 2;
      for (int64_t t = t0 + lane_id(); t < t1; t += 64) {
        uint64_t d = (uint64_t)(rp[t + 1] - rp[t]);
        if (d >= 2) acc[0] += d * (d - 1) / 2;
        if (d >= 3) acc[1] += (uint64_t)((unsigned __int128)d * (d - 1) * (d - 2) / 6);
      }
    }
  }
  if (cur >= 0) flush(a.results, cur_slot, acc, nf);
  if (CE) {
    uint64_t e = wave_sum_u64(ec.elems);
    uint64_t f = wave_sum_u64(ec.fetches);
    uint64_t wr = wave_sum_u64(ec.written);
    uint64_t wo = wave_sum_u64(ec.words);
    if (lane_id() == 0) {
      atomicAdd(&a.counters[0], (unsigned long long)e / 64ull);
      atomicAdd(&a.counters[1], (unsigned long long)f / 64ull);
      atomicAdd(&a.counters[2], (unsigned long long)wr / 64ull);
      atomicAdd(&a.counters[3], (unsigned long long)wo);
    }
  }
}

// Persistent workgroup kernel of the large-root local graphs: wave 0 pops a
// chunk of root tasks from the per-XCD queues and shares it through LDS; the
// whole workgroup then searches each root of the chunk in turn.
template <bool CE>
__global__ void __launch_bounds__(kBlockWaves * 64)
gpm_lgs_block(KernelArgs a) {
  extern __shared__ __attribute__((aligned(16))) int32_t blk_lds[];
  __shared__ int32_t scan_tmp[kBlockWaves];
  __shared__ int32_t row_next;
  __shared__ long long chunk_lds;
  const int home = (int)(blockIdx.x & (kQueues - 1));
  uint32_t dead = 0;
  int cur = -1;
  int cur_slot = 0;
  uint64_t acc[1] = {0};
  ElemCounter ec;
  for (;;) {
    if (threadIdx.x < 64) {
      const int64_t c = pop_chunk(a.queue_cnt, a.queue_begin, home, dead);
      if (lane_id() == 0) chunk_lds = c;
    }
    __syncthreads();
    const int64_t c = uni64(chunk_lds);
    __syncthreads();  // read by every wave before wave 0 pops again
    if (c < 0) break;
    const int j = uni(find_job(a.job_chunk_begin, a.n_jobs, c));
    if (j != cur) {
      if (cur >= 0) flush(a.results, cur_slot, acc, 1);
      cur = j;
    }
    const Job& J = a.jobs[j];
    cur_slot = J.slot;
    const int64_t t0 = (c - a.job_chunk_begin[j]) * (int64_t)J.chunk;
    const int64_t t1 = min(t0 + (int64_t)J.chunk, J.n_tasks);
    for (int64_t t = t0; t < t1; ++t) {
      const int32_t u = uni(J.task_src[t]);
      const int32_t d = uni((int32_t)(J.rp[u + 1] - J.rp[u]));
      int32_t part = 0, parts = 1;
      if (J.task_dst) {
        const int32_t enc = uni(J.task_dst[t]);
        part = enc & 0xffff;
        parts = enc >> 16;
      }
      // the edge-sorting area follows the largest tile of the launch
      // rows in the workgroup's HBM region when the job's local graphs exceed the LDS
      unsigned long long* Rg =
          J.lds_ok ? nullptr
                   : (unsigned long long*)(a.fbuf + (int64_t)blockIdx.x * a.wave_stride);
      if (Rg)
        acc[0] += clique_lgs_block<CE, true>(J.rp, J.col, J.k, u, d, part, parts,
                                             J.ordered != 0, blk_lds, scan_tmp, &row_next,
                                             blk_lds + a.lds_words - kBlockWaves * kSortWords,
                                             J.tri, Rg, ec, a.lgs_lg);
      else
        acc[0] += clique_lgs_block<CE, false>(J.rp, J.col, J.k, u, d, part, parts,
                                              J.ordered != 0, blk_lds, scan_tmp, &row_next,
                                              blk_lds + a.lds_words - kBlockWaves * kSortWords,
                                              J.tri, nullptr, ec, a.lgs_lg);
      __syncthreads();  // the next root reuses the local graph's LDS
    }
  }
  if (cur >= 0) flush(a.results, cur_slot, acc, 1);
  if (CE) {
    uint64_t e = wave_sum_u64(ec.elems);
    uint64_t f = wave_sum_u64(ec.fetches);
    uint64_t wo = wave_sum_u64(ec.words);
    if (lane_id() == 0) {
      atomicAdd(&a.counters[0], (unsigned long long)e / 64ull);
      atomicAdd(&a.counters[1], (unsigned long long)f / 64ull);
      atomicAdd(&a.counters[3], (unsigned long long)wo);
    }
  }
}

// ---------------------------------------------------------------------------
// edge-induced 4-cycles by wedge aggregation in LDS (the counting-only pruning
// of Sec. 5.4 (1) applied to the 4-cycle).  On the graph relabelled by
// ascending (degree, id), every 4-cycle is counted once at its largest vertex
// v together with the vertex w opposite v: with c_w the number of wedges
// v-u-w (u, w < v), the root contributes sum_w C(c_w, 2).  One workgroup
// counts the wedges of one task in a table in its LDS:
//  - direct windows (roots whose endpoints are dense among the ids below
//    them): one counter per endpoint id of a window; each lane keeps its
//    u's list position and end (its cursor, in the workgroup's HBM region)
//    from one window of the task to the next, so a window costs one
//    coalesced cursor read and a short search from the cursor per u;
//  - hash ranges (other roots with many wedges): keys w + 1 with their
//    counts, the root's id ranges in order with cursors as above; a range
//    that meets more distinct keys than kCycHashCap runs again in halves;
//  - hash batches (light roots): keys slot * n + w + 1; a batch that meets
//    more distinct keys than kCycHashCap splits its roots in halves and runs
//    again.
// Every phase leaves the table at zero.
// ---------------------------------------------------------------------------

static_assert(kCycHashCap + kCycWaves * 64 < kCycSlots, "a 4-cycle hash table must never fill");

struct CycShared {
  int64_t S[kCycWaves][64];     // per wave: list start of each lane's slice
  int32_t PF[kCycWaves][64];    // per wave: inclusive prefix of the slice lengths
  int32_t stack[kCycStack][4];  // hash tasks still to run: (r0, r1, x, y)
  int32_t sp;
  uint32_t distinct;            // keys in the table
  int32_t overflow;             // the running hash task split
  long long chunk;
};

__device__ __forceinline__ uint32_t cyc_hash(uint32_t key) {
  return (key * 2654435761u) >> (32 - kCycSlotBits);
}

// One batch of up to 64 slices per wave: lane l holds the slice
// col[start, start + len); the wave takes the slices' elements 64 * kCycEpl at
// a time, kCycEpl consecutive ones per lane: one search of the staged prefix
// finds the slice of a lane's first element, the next ones follow by
// stepping to the next slice when one ends, and their loads are in flight
// together (the kernel is latency-bound; its LDS table allows one workgroup
// per CU, which leaves registers for them); each element goes to sink.
constexpr int kCycEpl = 4;
template <bool CE, typename Sink>
__device__ __forceinline__ void cyc_batch(const int32_t* __restrict__ col, int64_t start,
                                          int32_t len, int64_t* S, int32_t* PF,
                                          ElemCounter& ec, Sink&& sink) {
  const int l = lane_id();
  const int32_t incl = wave_incl_scan(len);
  S[l] = start;
  PF[l] = incl;
  wave_sync_mem();
  const int32_t tot = uni(__shfl(incl, 63, 64));
  for (int32_t tb = 0; tb < tot; tb += 64 * kCycEpl) {
    const int32_t t0 = tb + kCycEpl * l;
    int32_t w[kCycEpl];
#pragma unroll
    for (int j = 0; j < kCycEpl; ++j) w[j] = 0;
    if (t0 < tot) {
      // element t of slice o lies at col[S[o] + t - PF[o - 1]]
      int32_t o = upper_bound(PF, 64, t0);
      int32_t end = PF[o];
      int64_t base = S[o] - (o > 0 ? PF[o - 1] : 0);
#pragma unroll
      for (int j = 0; j < kCycEpl; ++j) {
        const int32_t t = t0 + j;
        if (t < tot) {
          while (t >= end) {  // t < tot = PF[63]: some later slice holds it
            ++o;
            base = S[o] - end;
            end = PF[o];
          }
          w[j] = col[base + t];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kCycEpl; ++j)
      if (t0 + j < tot) sink(w[j]);
  }
  if (CE) ec.elems += (uint64_t)tot;
  wave_sync_mem();
}

// Direct windows a .. a+b-1 of root v (see CycTask).  cursor: two int64
// per lower neighbour: the list position, and the number of list elements
// left with the value of the next one (INT32_MAX past the end) packed as
// rem | next << 32, so that a window the list does not reach is skipped
// without touching the list.
template <bool CE>
__device__ __forceinline__ void cyc_direct(const int64_t* __restrict__ rp,
                                           const int32_t* __restrict__ col, const CycTask& T,
                                           uint32_t* tab, int64_t* cursor, CycShared& sh,
                                           uint64_t& acc, ElemCounter& ec) {
  const int32_t v = T.head;
  const bool c32 = (T.c & kCycWide) != 0;
  const int64_t W = c32 ? kCycWindow / 2 : kCycWindow;
  const int32_t* Nv = col + rp[v];
  const int32_t e = uni(lower_bound(Nv, (int32_t)(rp[v + 1] - rp[v]), v));
  const int wv = (int)(threadIdx.x >> 6);
  const int l = lane_id();
  for (int32_t k = T.a; k < T.a + T.b; ++k) {
    const int64_t wa64 = (int64_t)k * W;
    if (wa64 >= v) break;
    const int32_t wa = (int32_t)wa64;
    const int32_t wb = (int32_t)min(wa64 + W, (int64_t)v);
    for (int32_t ub = wv * 64; ub < e; ub += kCycWaves * 64) {
      const int32_t i = ub + l;
      int64_t start = 0;
      int32_t len = 0;
      if (i < e) {
        // the slice of N(u) in [wa, wb): from the cursor the previous window
        // left (a search at the task's first window), up to wb by galloping
        int64_t pos;
        int32_t rem, nxt;
        const bool first = k == T.a;
        if (first) {
          const int32_t u = Nv[i];
          pos = rp[u];
          const int64_t end = rp[u + 1];
          if (wa > 0) pos += lower_bound(col + pos, (int32_t)(end - pos), wa);
          rem = (int32_t)(end - pos);
          nxt = rem > 0 ? col[pos] : INT32_MAX;
        } else {
          pos = cursor[2 * i];
          const int64_t pk = cursor[2 * i + 1];
          rem = (int32_t)(uint32_t)pk;
          nxt = (int32_t)(pk >> 32);
        }
        if (nxt < wb)  // col[pos] = nxt is in the window
          len = 1 + gallop_lb(col + pos + 1, 0, rem - 1, wb);
        start = pos;
        if (len > 0) {
          pos += len;
          rem -= len;
          nxt = rem > 0 ? col[pos] : INT32_MAX;
        }
        if (first || len > 0) {
          cursor[2 * i] = pos;
          cursor[2 * i + 1] = (int64_t)(uint32_t)rem | ((int64_t)nxt << 32);
        }
      }
      if (CE) ec.fetches += (uint64_t)min(64, e - ub);
      if (c32) {
        cyc_batch<CE>(col, start, len, sh.S[wv], sh.PF[wv], ec,
                      [&](int32_t w) { atomicAdd(&tab[w - wa], 1u); });
      } else {
        cyc_batch<CE>(col, start, len, sh.S[wv], sh.PF[wv], ec, [&](int32_t w) {
          const uint32_t x = (uint32_t)(w - wa);
          atomicAdd(&tab[x >> 1], (x & 1u) ? 0x10000u : 1u);
        });
      }
    }
    __syncthreads();
    // sum_w C(c_w, 2) over the window; the table back to zero
    const int32_t words = c32 ? (wb - wa) : ((wb - wa + 1) >> 1);
    for (int32_t q = (int32_t)threadIdx.x; q < words; q += kCycWaves * 64) {
      const uint32_t x = tab[q];
      if (x) {
        tab[q] = 0;
        if (c32) {
          acc += (uint64_t)x * (uint64_t)(x - 1) / 2;
        } else {
          const uint64_t c0 = x & 0xffffu, c1 = x >> 16;
          acc += c0 * (c0 ? c0 - 1 : 0) / 2 + c1 * (c1 ? c1 - 1 : 0) / 2;
        }
      }
    }
    __syncthreads();
  }
}

// Hash ranges a .. a+b-1 of root v (see CycTask): the ranges in order, each
// lane's list position carried from one range to the next in the cursor; a
// range whose distinct endpoints overflow the table runs again as two halves
// from the same positions.  cursor: three int64 per lower neighbour (list
// position, list end, position after the running range).
template <bool CE>
__device__ __forceinline__ void cyc_ranges(const int64_t* __restrict__ rp,
                                           const int32_t* __restrict__ col,
                                           const int32_t* __restrict__ bounds,
                                           const CycTask& T, uint32_t* tab, int64_t* cursor,
                                           CycShared& sh, uint64_t& acc, ElemCounter& ec) {
  uint32_t* keys = tab;
  uint32_t* cnts = tab + kCycSlots;
  const int32_t v = T.head;
  const int32_t* Nv = col + rp[v];
  const int32_t e = uni(lower_bound(Nv, (int32_t)(rp[v + 1] - rp[v]), v));
  const int wv = (int)(threadIdx.x >> 6);
  const int l = lane_id();
  const int32_t x0 = uni(bounds[T.a]);
  // cursors at the first range's start (thread i*1024 + t keeps lower
  // neighbour i*1024 + t, as in the walk below)
  for (int32_t i = (int32_t)threadIdx.x; i < e; i += kCycWaves * 64) {
    const int32_t u = Nv[i];
    int64_t pos = rp[u];
    const int64_t end = rp[u + 1];
    if (x0 > 0) pos += lower_bound(col + pos, (int32_t)(end - pos), x0);
    cursor[3 * i] = pos;
    cursor[3 * i + 1] = end;
  }
  for (int32_t r = 0; r < T.b; ++r) {
    if (threadIdx.x == 0) {
      sh.stack[0][2] = bounds[T.a + r];
      sh.stack[0][3] = bounds[T.a + r + 1];
      sh.sp = 1;
    }
    __syncthreads();
    for (;;) {
      const int32_t sp = uni(sh.sp);
      if (sp == 0) break;
      const int32_t x = uni(sh.stack[sp - 1][2]);
      const int32_t y = uni(sh.stack[sp - 1][3]);
      __syncthreads();  // every wave has read the entry before it is popped
      if (threadIdx.x == 0) {
        sh.sp = sp - 1;
        sh.distinct = 0;
        sh.overflow = 0;
      }
      __syncthreads();
      for (int32_t ub = wv * 64; ub < e; ub += kCycWaves * 64) {
        if (uni(__hip_atomic_load(&sh.overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)))
          break;
        const int32_t i = ub + l;
        int64_t start = 0;
        int32_t len = 0;
        if (i < e) {
          const int64_t pos = cursor[3 * i];
          const int64_t end = cursor[3 * i + 1];
          len = gallop_lb(col + pos, 0, (int32_t)(end - pos), y);
          start = pos;
          cursor[3 * i + 2] = pos + len;
        }
        if (CE) ec.fetches += (uint64_t)min(64, e - ub);
        cyc_batch<CE>(col, start, len, sh.S[wv], sh.PF[wv], ec, [&](int32_t w) {
          if (__hip_atomic_load(&sh.overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
          const uint32_t key = (uint32_t)w + 1u;
          uint32_t h = cyc_hash(key);
          for (;;) {
            const uint32_t old = atomicCAS(&keys[h], 0u, key);
            if (old == 0u) {
              if (atomicAdd(&sh.distinct, 1u) + 1u > (uint32_t)kCycHashCap)
                __hip_atomic_store(&sh.overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              atomicAdd(&cnts[h], 1u);
              break;
            }
            if (old == key) {
              atomicAdd(&cnts[h], 1u);
              break;
            }
            h = (h + 1u) & (uint32_t)(kCycSlots - 1);
          }
        });
      }
      __syncthreads();
      if (uni(sh.overflow)) {
        // the halves run next, from the same positions (a range of at most
        // kCycHashCap ids cannot overflow, so the halving ends)
        for (int32_t q = (int32_t)threadIdx.x; q < kCycTableWords; q += kCycWaves * 64) tab[q] = 0;
        if (threadIdx.x == 0) {
          const int32_t mid = x + (y - x) / 2;
          int32_t t = sh.sp;
          sh.stack[t][2] = mid; sh.stack[t][3] = y; ++t;
          sh.stack[t][2] = x; sh.stack[t][3] = mid; ++t;
          sh.sp = t;
        }
        __syncthreads();
        continue;
      }
      for (int32_t q = (int32_t)threadIdx.x; q < kCycSlots; q += kCycWaves * 64) {
        if (keys[q]) {
          const uint64_t c = cnts[q];
          acc += c * (c - 1) / 2;
          keys[q] = 0;
          cnts[q] = 0;
        }
      }
      // the range is done: its end positions become the cursors
      for (int32_t i = (int32_t)threadIdx.x; i < e; i += kCycWaves * 64)
        cursor[3 * i] = cursor[3 * i + 2];
      __syncthreads();
    }
    // every wave has seen the empty stack before thread 0 sets up the next
    // range (else a late wave would read the new entry and fall one barrier
    // out of step with the others)
    __syncthreads();
  }
}

// Hash task over roots[r0, r1) with endpoints in [x, y), splitting on overflow.
template <bool CE>
__device__ __forceinline__ void cyc_hash_task(const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ roots, uint32_t n,
                                              const CycTask& T, uint32_t* tab, CycShared& sh,
                                              uint64_t& acc, ElemCounter& ec) {
  uint32_t* keys = tab;
  uint32_t* cnts = tab + kCycSlots;
  const int wv = (int)(threadIdx.x >> 6);
  const int l = lane_id();
  if (threadIdx.x == 0) {
    sh.stack[0][0] = -T.head - 1;
    sh.stack[0][1] = T.a;
    sh.stack[0][2] = T.b;
    sh.stack[0][3] = T.c;
    sh.sp = 1;
  }
  __syncthreads();
  for (;;) {
    const int32_t sp = uni(sh.sp);
    if (sp == 0) break;
    const int32_t r0 = uni(sh.stack[sp - 1][0]);
    const int32_t r1 = uni(sh.stack[sp - 1][1]);
    const int32_t x = uni(sh.stack[sp - 1][2]);
    const int32_t y = uni(sh.stack[sp - 1][3]);
    __syncthreads();  // every wave has read the entry before it is popped
    if (threadIdx.x == 0) {
      sh.sp = sp - 1;
      sh.distinct = 0;
      sh.overflow = 0;
    }
    __syncthreads();
    const int32_t nr = r1 - r0;
    const bool one = nr == 1;
    for (int32_t rr = r0 + (one ? 0 : wv); rr < r1; rr += (one ? 1 : kCycWaves)) {
      if (__hip_atomic_load(&sh.overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
      const int32_t v = uni(roots[rr]);
      const uint32_t base = (uint32_t)(rr - r0) * n + 1u;
      const int32_t hy = min(y, v);
      const int32_t* Nv = col + rp[v];
      const int32_t e = uni(lower_bound(Nv, (int32_t)(rp[v + 1] - rp[v]), v));
      for (int32_t ub = one ? wv * 64 : 0; ub < e; ub += one ? kCycWaves * 64 : 64) {
        if (uni(__hip_atomic_load(&sh.overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)))
          break;
        const int32_t i = ub + l;
        int64_t start = 0;
        int32_t len = 0;
        if (i < e && x < hy) {
          const int32_t u = Nv[i];
          const int64_t s0 = rp[u];
          const int32_t du = (int32_t)(rp[u + 1] - s0);
          const int32_t lo = x == 0 ? 0 : lower_bound(col + s0, du, x);
          len = gallop_lb(col + s0, lo, du, hy) - lo;
          start = s0 + lo;
        }
        if (CE) ec.fetches += (uint64_t)min(64, e - ub);
        cyc_batch<CE>(col, start, len, sh.S[wv], sh.PF[wv], ec, [&](int32_t w) {
          // after a split at most one insert per thread follows: the table
          // never fills (kCycHashCap + 1024 < kCycSlots), so probing ends
          if (__hip_atomic_load(&sh.overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
          const uint32_t key = base + (uint32_t)w;
          uint32_t h = cyc_hash(key);
          for (;;) {
            const uint32_t old = atomicCAS(&keys[h], 0u, key);
            if (old == 0u) {
              if (atomicAdd(&sh.distinct, 1u) + 1u > (uint32_t)kCycHashCap)
                __hip_atomic_store(&sh.overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              atomicAdd(&cnts[h], 1u);
              break;
            }
            if (old == key) {
              atomicAdd(&cnts[h], 1u);
              break;
            }
            h = (h + 1u) & (uint32_t)(kCycSlots - 1);
          }
        });
      }
    }
    __syncthreads();
    if (uni(sh.overflow)) {
      for (int32_t q = (int32_t)threadIdx.x; q < kCycTableWords; q += kCycWaves * 64) tab[q] = 0;
      if (threadIdx.x == 0) {
        // run the halves next (depth <= log2 roots + log2 ids: within kCycStack)
        int32_t t = sh.sp;
        if (nr > 1) {
          const int32_t mid = r0 + nr / 2;
          sh.stack[t][0] = mid; sh.stack[t][1] = r1; sh.stack[t][2] = x; sh.stack[t][3] = y;
          ++t;
          sh.stack[t][0] = r0; sh.stack[t][1] = mid; sh.stack[t][2] = x; sh.stack[t][3] = y;
          ++t;
        } else {
          const int32_t hy = min(y, roots[r0]);
          const int32_t mid = x + (hy - x) / 2;
          sh.stack[t][0] = r0; sh.stack[t][1] = r1; sh.stack[t][2] = mid; sh.stack[t][3] = hy;
          ++t;
          sh.stack[t][0] = r0; sh.stack[t][1] = r1; sh.stack[t][2] = x; sh.stack[t][3] = mid;
          ++t;
        }
        sh.sp = t;
      }
      __syncthreads();
      continue;
    }
    // sum over the keys of C(count, 2); the table back to zero
    for (int32_t q = (int32_t)threadIdx.x; q < kCycSlots; q += kCycWaves * 64) {
      if (keys[q]) {
        const uint64_t c = cnts[q];
        acc += c * (c - 1) / 2;
        keys[q] = 0;
        cnts[q] = 0;
      }
    }
    __syncthreads();
  }
  // every wave has seen the empty stack before the shared state is reused
  __syncthreads();
}

// Persistent workgroup kernel of the 4-cycle tasks: wave 0 pops a chunk of
// tasks from the per-XCD queues and shares it through LDS.
template <bool CE>
__global__ void __launch_bounds__(kCycWaves * 64)
gpm_cycle_block(KernelArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t cyc_tab[];
  __shared__ CycShared sh;
  for (int32_t q = (int32_t)threadIdx.x; q < kCycTableWords; q += kCycWaves * 64) cyc_tab[q] = 0;
  int64_t* cursor = (int64_t*)(a.zbuf + (int64_t)blockIdx.x * a.zstride);
  const int home = (int)(blockIdx.x & (kQueues - 1));
  uint32_t dead = 0;
  int cur = -1;
  int cur_slot = 0;
  uint64_t acc[1] = {0};
  ElemCounter ec;
  for (;;) {
    if (threadIdx.x < 64) {
      const int64_t c = pop_chunk(a.queue_cnt, a.queue_begin, home, dead);
      if (lane_id() == 0) sh.chunk = c;
    }
    __syncthreads();
    const int64_t c = uni64(sh.chunk);
    __syncthreads();  // read by every wave before wave 0 pops again
    if (c < 0) break;
    const int j = uni(find_job(a.job_chunk_begin, a.n_jobs, c));
    if (j != cur) {
      if (cur >= 0) flush(a.results, cur_slot, acc, 1);
      cur = j;
    }
    const Job& J = a.jobs[j];
    cur_slot = J.slot;
    const CycTask* tasks = (const CycTask*)J.task_src;
    const int64_t t0 = (c - a.job_chunk_begin[j]) * (int64_t)J.chunk;
    const int64_t t1 = min(t0 + (int64_t)J.chunk, J.n_tasks);
    for (int64_t t = t0; t < t1; ++t) {
      CycTask T;
      T.head = uni(tasks[t].head);
      T.a = uni(tasks[t].a);
      T.b = uni(tasks[t].b);
      T.c = uni(tasks[t].c);
      if (T.head >= 0 && (T.c & kCycRanges))
        cyc_ranges<CE>(J.rp, J.col, J.bounds, T, cyc_tab, cursor, sh, acc[0], ec);
      else if (T.head >= 0)
        cyc_direct<CE>(J.rp, J.col, T, cyc_tab, cursor, sh, acc[0], ec);
      else
        cyc_hash_task<CE>(J.rp, J.col, J.task_dst, (uint32_t)J.n_vertices, T, cyc_tab, sh,
                          acc[0], ec);
    }
  }
  if (cur >= 0) flush(a.results, cur_slot, acc, 1);
  if (CE) {
    uint64_t e = wave_sum_u64(ec.elems);
    uint64_t f = wave_sum_u64(ec.fetches);
    if (lane_id() == 0) {
      atomicAdd(&a.counters[0], (unsigned long long)e / 64ull);
      atomicAdd(&a.counters[1], (unsigned long long)f / 64ull);
    }
  }
}

__global__ void fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <uint32_t KINDS, bool CE>
static hipError_t launch_t(const KernelArgs& a, int blocks, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((gpm_persistent<KINDS, CE>), dim3(blocks), dim3(kWavesPerBlock * 64),
                     lds, s, a);
  return hipGetLastError();
}

template <bool CE>
static hipError_t launch_kinds(uint32_t kinds, const KernelArgs& a, int blocks, size_t lds,
                               hipStream_t s) {
  switch (kinds) {
    case kKindClique: return launch_t<kKindClique, CE>(a, blocks, lds, s);
    case kKindDfs: return launch_t<kKindDfs, CE>(a, blocks, lds, s);
    case kKindEdgeTri: return launch_t<kKindEdgeTri, CE>(a, blocks, lds, s);
    case kKindVertexDeg: return launch_t<kKindVertexDeg, CE>(a, blocks, lds, s);
    case kKindCliqueLgs: return launch_t<kKindCliqueLgs, CE>(a, blocks, lds, s);
    case kKindEdgeTerms: return launch_t<kKindEdgeTerms, CE>(a, blocks, lds, s);
    case kKindTriScatter: return launch_t<kKindTriScatter, CE>(a, blocks, lds, s);
    case kKindCliqueLgs | kKindClique:
      return launch_t<kKindCliqueLgs | kKindClique, CE>(a, blocks, lds, s);
    default: return launch_t<kKindAll, CE>(a, blocks, lds, s);
  }
}

int launch_persistent(uint32_t kinds, bool count_elems, const KernelArgs& a, int blocks,
                      size_t lds_bytes, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = count_elems ? launch_kinds<true>(kinds, a, blocks, lds_bytes, s)
                             : launch_kinds<false>(kinds, a, blocks, lds_bytes, s);
  return (int)e;
}

int launch_lgs_block(bool count_elems, const KernelArgs& a, int cus, int64_t max_blocks,
                     size_t lds_bytes, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const void* f = count_elems ? (const void*)gpm_lgs_block<true> : (const void*)gpm_lgs_block<false>;
  // room beyond the default dynamic LDS limit
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return (int)e;
  // as many workgroups as can be resident at once (registers and LDS)
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlockWaves * 64, lds_bytes);
  if (e != hipSuccess) return (int)e;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * std::max(per_cu, 1), max_blocks));
  if (count_elems)
    hipLaunchKernelGGL(gpm_lgs_block<true>, dim3((unsigned)blocks), dim3(kBlockWaves * 64), lds_bytes, s, a);
  else
    hipLaunchKernelGGL(gpm_lgs_block<false>, dim3((unsigned)blocks), dim3(kBlockWaves * 64), lds_bytes, s, a);
  return (int)hipGetLastError();
}

static constexpr size_t kCycLdsBytes = (size_t)kCycTableWords * 4;

int cycle_block_grid(int cus, int64_t max_blocks, int* blocks_out) {
  const void* f = (const void*)gpm_cycle_block<false>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCycLdsBytes);
  if (e != hipSuccess) return (int)e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kCycWaves * 64, kCycLdsBytes);
  if (e != hipSuccess) return (int)e;
  *blocks_out = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * std::max(per_cu, 1), max_blocks));
  return 0;
}

int launch_cycle_block(bool count_elems, const KernelArgs& a, int blocks, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const void* f = count_elems ? (const void*)gpm_cycle_block<true> : (const void*)gpm_cycle_block<false>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCycLdsBytes);
  if (e != hipSuccess) return (int)e;
  if (count_elems)
    hipLaunchKernelGGL(gpm_cycle_block<true>, dim3((unsigned)blocks), dim3(kCycWaves * 64), kCycLdsBytes, s, a);
  else
    hipLaunchKernelGGL(gpm_cycle_block<false>, dim3((unsigned)blocks), dim3(kCycWaves * 64), kCycLdsBytes, s, a);
  return (int)hipGetLastError();
}

int launch_list(const ListArgs& a, int blocks, void* stream) {
  hipLaunchKernelGGL(gpm_list, dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

// Device scratch of the allocation-free count (gpm_count_noalloc): job
// table, queue counters, result slots, frontier and counter buffers of one
// synchronous call.  One copy per GPU, loaded with the code object and held
// until the process ends; calls that overlap on one GPU share it.  Host code
// never uses the array's name (a host-side stand-in): its device address
// comes from hipGetSymbolAddress, looked up once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int scratch_address(int device, void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices || !ptr) return (int)hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return (int)e;
    if (cur != device) return (int)hipErrorInvalidDevice;  // the caller makes it current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return 0;
}

int launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, void* stream) {
  if (n <= 0) return 0;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);  // grid-stride beyond
  hipLaunchKernelGGL(fill_u64, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, p, n,
                     v);
  return (int)hipGetLastError();
}

}  // namespace gpm
