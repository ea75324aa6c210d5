// Internal structures shared by the host runtime and the device kernels of
// libgpm (never exposed through include/gpm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gpm {

constexpr int kMaxK = 8;
constexpr int kWavesPerBlock = 4;       // 256-thread workgroups of four wave64s
constexpr int kQueues = 8;              // one task queue per XCD
constexpr int kQueueStride = 16;        // uint64 words between queue counters (128 B)
constexpr int kResultFields = 8;        // uint64 counters per result slot
// Device scratch of the allocation-free count, per GPU (see scratch_address)
constexpr size_t kScratchBytes = size_t(64) << 20;

// One depth of a search plan (Sec. 2.2: the matching order fixes which
// earlier pattern vertices a new vertex must be adjacent to -- its candidate
// set is the intersection of their neighbour lists -- and the symmetry
// order fixes upper bounds).  Depths 0 and 1 are the root task's vertices.
struct LevelPlan {
  uint8_t n_int;           // neighbour lists N(v_j) to intersect, j in int_lv
  uint8_t n_sub;           // neighbour lists to subtract (vertex-induced mode)
  int8_t base_buf;         // >= 2: the candidate set starts from the stored
                           // set of that depth; -1: from the shortest N(v_j)
  uint8_t flags;           // kLvStore / kLvSlice
  uint8_t int_lv[kMaxK];
  uint8_t sub_lv[kMaxK];
  uint8_t bound_mask;      // bit j: v_depth < v_j
  uint8_t excl_mask;       // bit j: v_depth != v_j must be checked explicitly
  uint8_t pad[2];
};

constexpr uint8_t kLvStore = 1;   // materialise into the depth's frontier buffer
constexpr uint8_t kLvSlice = 2;   // the set is a bounded prefix of one list;
                                  // iterate it in place, skipping excl_mask

struct Plan {
  int32_t k;               // depths walked (the leaf is depth k - 1)
  int32_t root_bound;      // 1: root edges (v0, v1) need v1 < v0
  int32_t n_store;         // number of stored depths (frontier buffers)
  int32_t leaf_choose;     // 0: the leaf counts its set; else r | ext << 8:
                           // the leaf set stands for the pattern's last r
                           // vertices (counting-only pruning) and adds
                           // ext * C(|set|, r)
  int8_t store_slot[kMaxK];  // depth -> frontier buffer index, -1 if none
  LevelPlan lv[kMaxK];
};

enum JobKind : int32_t {
  kJobClique = 1,      // k-clique on a DAG, frontiers in LDS or HBM
  kJobDfs = 2,         // generic plan-driven DFS on a symmetric graph
  kJobEdgeTri = 3,     // per-edge triangle counts and the 4-motif edge terms
  kJobVertexDeg = 4,   // per-vertex degree terms
  kJobCliqueLgs = 5,   // k-clique (k = 3..5) by local graph search with bitmaps
  kJobCycleBlock = 6,  // edge-induced 4-cycles by wedge aggregation in LDS, one
                       // workgroup per task (own kernel)
  kJobCliqueLgsBlock = 7,  // k-clique (k = 3..5): the local graph of one large
                           // root shared by a whole workgroup (own kernel)
  kJobEdgeTerms = 8,   // per-edge motif terms from per-edge triangle counts
  kJobTriScatter = 9,  // triangles by local graph search (one wave per root),
                       // each added to its three edges' counters
};

constexpr uint32_t kKindClique = 1u << kJobClique;
constexpr uint32_t kKindDfs = 1u << kJobDfs;
constexpr uint32_t kKindEdgeTri = 1u << kJobEdgeTri;
constexpr uint32_t kKindVertexDeg = 1u << kJobVertexDeg;
constexpr uint32_t kKindCliqueLgs = 1u << kJobCliqueLgs;
constexpr uint32_t kKindCycleBlock = 1u << kJobCycleBlock;
constexpr uint32_t kKindCliqueLgsBlock = 1u << kJobCliqueLgsBlock;
constexpr uint32_t kKindEdgeTerms = 1u << kJobEdgeTerms;
constexpr uint32_t kKindTriScatter = 1u << kJobTriScatter;
// kinds of the per-wave persistent kernel (the workgroup kernel has its own)
constexpr uint32_t kKindAll = kKindClique | kKindDfs | kKindEdgeTri | kKindVertexDeg |
                              kKindCliqueLgs | kKindEdgeTerms |
                              kKindTriScatter;
constexpr int kLgsMaxVertices = 2048;   // local graphs handled by the bitmap kernel
constexpr int kBlockWaves = 16;         // workgroup of the large-root kernel (1024 threads)
constexpr int kLgsBlockMaxVertices = kBlockWaves * 64;  // one vertex per thread in its scans
// The workgroup kernel sorts its 5-clique local edges by cost in batches of
// kSortBatch per wave: an LDS area of kSortBatch ids and 64 bucket counters
// per wave, after the largest tile of the launch.
constexpr int kSortBatch = 512;
constexpr int kSortWords = kSortBatch + 64;
constexpr int kBlockSortWords = kBlockWaves * kSortWords;

// 4-cycle workgroup kernel (kJobCycleBlock): 1024 threads, a table of
// kCycTableWords words of LDS (one workgroup per CU).  Direct windows
// count the endpoints of one id window in 16-bit counters packed two per
// word (kCycWindow ids), or in 32-bit counters (half the ids) for roots with
// 65535 or more lower neighbours.  Hash tasks use the table as keys | counts
// (kCycSlots each); a task stops and splits once kCycHashCap distinct keys
// are in.
constexpr int kCycWaves = 16;
constexpr int kCycSlotBits = 14;
constexpr int kCycSlots = 1 << kCycSlotBits;
constexpr int kCycTableWords = 2 * kCycSlots;
constexpr int kCycWindow = 2 * kCycTableWords;
constexpr int kCycHashCap = kCycSlots * 3 / 4;
constexpr int kCycStack = 64;   // pending split tasks per workgroup

// A task of the 4-cycle kernel, 4 int32 words.
//  head >= 0, c & kCycRanges == 0: direct windows of root v = head: windows
//    a .. a+b-1 (window i covers ids [i*W, (i+1)*W) below v; W = kCycWindow,
//    or kCycWindow / 2 when c & kCycWide: 32-bit counters);
//  head >= 0, c & kCycRanges: hash ranges of root v = head: ranges a .. a+b-1
//    of the job's boundary list (range i covers ids [bd[i], bd[i + 1]));
//  head < 0: hash task over the roots r[-head-1 .. a) of the job's root list
//    (task_dst) with endpoints in [b, c) (and below each root).
constexpr int32_t kCycWide = 1;
constexpr int32_t kCycRanges = 2;
struct CycTask {
  int32_t head;
  int32_t a;
  int32_t b;
  int32_t c;
};

// Set operations of the plan-driven DFS (Sec. 6.1): membership probes by
// binary search in global memory, by a merge-path window of the probed list
// staged in LDS (a galloping merge in a lane's own leaf), or by binary search
// with the top levels of the probed list's search tree in LDS.
constexpr int32_t kSetopBinary = 1;
constexpr int32_t kSetopMerge = 2;
constexpr int32_t kSetopBst = 3;

// One unit of work of a persistent launch: a (graph, pattern plan, range of
// root tasks) triple with its own result slot.
struct Job {
  int32_t kind;
  int32_t k;               // clique size or plan size
  int32_t plan;            // index into the launch's plan table (kJobDfs)
  int32_t slot;            // result slot
  const int64_t* rp;       // graph view: CSR offsets
  const int32_t* col;      //             CSR neighbours
  const int32_t* task_src; // root tasks: edge t is (task_src[t], task_dst[t]);
  const int32_t* task_dst; //   vertex tasks use vertex t and leave these null
  int64_t n_tasks;
  int32_t chunk;           // tasks per queue pop
  int32_t vertex_tasks;    // 1: tasks are root vertices
  int32_t cap;             // frontier capacity in elements (max set size)
  int32_t lds_ok;          // clique job: sets fit the LDS tile
  int32_t leaf_cap;        // DFS job: lane-per-candidate leaves up to this size
  int32_t ordered;         // clique job: out-lists follow the orientation order
                           // (u -> v iff u < v), so local bitmap rows are
                           // upper triangular
  int32_t tri_group;       // > 0: triangle-scatter group.  Its k = 3 local-graph
                           // jobs add 1 per triangle to each of its three edges'
                           // counters (indexed by DAG position) instead of
                           // counting; its kJobEdgeTerms job reads them
  unsigned int* tri;       // the group's per-DAG-edge counters (set at launch;
                           // zero between launches)
  const int64_t* deg_rp;   // kJobEdgeTerms: offsets of the symmetric graph (degrees)
  int32_t n_vertices;      // kJobCycleBlock: vertices of the graph (hash keys)
  int32_t setop;           // kJobDfs: how set operations probe (kSetop*)
  const int32_t* bounds;   // kJobCycleBlock: id boundaries of the hash ranges
};

struct KernelArgs {
  const Job* jobs;
  const int64_t* job_chunk_begin;  // [n_jobs + 1], prefix of chunks per job
  int32_t n_jobs;
  int32_t lds_cap;                 // clique LDS tile (elements per set)
  const Plan* plans;
  const int64_t* queue_begin;      // [kQueues + 1]; [kQueues] = chunk count
  unsigned long long* queue_cnt;   // [kQueues * kQueueStride]
  unsigned long long* results;     // [slots * kResultFields]
  unsigned long long* counters;    // [4]: elements, list fetches (instrumented)
  int32_t* fbuf;                   // HBM frontier buffers
  int64_t wave_stride;             // int32 words of fbuf per wave
  int32_t lds_words;               // int32 words of dynamic LDS per wave
  int32_t lgs_tile;                // local graphs up to this size use LDS
  int32_t lgs_lg;                  // local-graph row build: log2 of the lanes per row (6: a wave)
  int32_t* zbuf;                   // 4-cycle kernel: per-workgroup cursor regions
  int64_t zstride;                 // words of zbuf per workgroup
};

// Local-graph tile of T vertices, in int32 words: L[T] | P[T + 1] | (pad to
// 8 B) | H[lgs_hash_slots(T)] uint64 (hash of L: vertex -> position) |
// R[T * ceil(T / 64)] uint64 (bitmap rows).  A root of d <= T vertices uses
// the first lgs_hash_slots(d) slots of H, or up to four times as many where H
// has them (an emptier table ends lookups that miss sooner).
__host__ __device__ inline int64_t lgs_hash_slots(int64_t d) {
  int64_t s = 2;
  while (s < 2 * d) s <<= 1;  // load factor <= 1/2: every probe sequence meets an empty slot
  return s;
}
__host__ __device__ inline int64_t lgs_hash_offset(int64_t T) { return (2 * T + 2) & ~int64_t(1); }
__host__ __device__ inline int64_t lgs_rows_offset(int64_t T) {
  return lgs_hash_offset(T) + 2 * lgs_hash_slots(T);
}
__host__ __device__ inline int64_t lgs_tile_words(int64_t T) {
  return lgs_rows_offset(T) + 2 * T * ((T + 63) / 64);
}

// The workgroup kernel lays out a root of d vertices as a tile with T = d,
// its bitmap rows padded: a row of W words takes an odd number of words
// (W | 1) where the tile then still fits within that of the largest root,
// W <= kLgsPadWords.  The 64 lanes of a wave read 64 different rows at once;
// with a stride of 2^a * b words (b odd) their first words fall on 2^-a as
// many LDS banks as with an odd stride, so an even stride multiplies the bank
// conflicts of those reads.
constexpr int kLgsPadWords = 13;
__host__ __device__ constexpr int64_t lgs_block_stride_words(int64_t W) {
  return W <= kLgsPadWords ? (W | 1) : W;
}
__host__ __device__ inline int64_t lgs_block_tile_words(int64_t T) {
  return lgs_rows_offset(T) + 2 * T * lgs_block_stride_words((T + 63) / 64);
}

// One listing launch (Sec. 2.1: listing enumerates every match instead of
// counting it): the plan-driven walk of one pattern over one graph view,
// whose leaf depth writes each match as a row of k vertex ids.
struct ListArgs {
  Plan plan;
  const int64_t* rp;         // graph view: CSR offsets
  const int32_t* col;        //             CSR neighbours
  const int32_t* task_src;   // root task t: the edge (task_src[t], task_dst[t]),
  const int32_t* task_dst;   //   or the vertex t when task_src is null (k == 1)
  int64_t n_tasks;
  int32_t chunk;             // root tasks per queue pop
  int32_t cap;               // frontier capacity (elements per stored depth)
  int32_t k;
  int8_t out_col[kMaxK];     // depth -> column of the row (the pattern vertex)
  const int32_t* ids;        // view id -> caller's vertex id; null: identity
  int32_t* out;              // rows [out_cap][k]
  int64_t out_cap;
  unsigned long long* queue;   // next chunk of the root tasks
  unsigned long long* rows;    // matches found (rows claimed)
  int32_t* fbuf;             // frontier buffers: wave_stride words per wave
  int64_t wave_stride;
  int32_t ordered;           // cliques on a DAG whose out-lists lie above their
                             // vertex (u -> v iff u < v): a candidate of depth d
                             // exceeds the vertex of depth d-1
};

// Host-side launchers (kernels.hip).  Return a hipError_t as int.
int launch_persistent(uint32_t kinds, bool count_elems, const KernelArgs& a,
                      int blocks, size_t lds_bytes, void* stream);
int launch_lgs_block(bool count_elems, const KernelArgs& a, int cus, int64_t max_blocks,
                     size_t lds_bytes, void* stream);
// The 4-cycle workgroup kernel; *blocks_out receives the grid size (one
// cursor region of a.zstride words per workgroup in a.zbuf).
int cycle_block_grid(int cus, int64_t max_blocks, int* blocks_out);
int launch_cycle_block(bool count_elems, const KernelArgs& a, int blocks, void* stream);
int launch_list(const ListArgs& a, int blocks, void* stream);
int launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, void* stream);

// Device address of this GPU's copy of the allocation-free count's scratch
// (kScratchBytes); `device` must be the current device.  Returns a hipError_t.
int scratch_address(int device, void** ptr);

}  // namespace gpm
