// Internal declarations shared by the HIP sources of libpkd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/pkd.h"

namespace pkd {

constexpr int kMaxDim = 9;
constexpr int kMaxLambda = 8;
constexpr int kMaxSample = 2048;                 // s = 2^lambda * sigma (LDS of the select and finisher kernels)
constexpr int64_t kCoordLimit = int64_t{1} << 30;   // 32-bit copies, splitters and box bounds
constexpr int64_t kCoordMax = kCoordLimit - 1;
// Exclusive bound of a point's (or query's) coordinates in D dimensions: below
// 2^30, and small enough that D squared differences sum exactly in int64
// (D * (limit - 1)^2 <= 2^63 - 1; only D = 9 is below 2^30).
__host__ __device__ constexpr int64_t coord_limit(int D) {
  return D <= 8 ? kCoordLimit : int64_t{1012333500};
}
static_assert((coord_limit(9) - 1) * (coord_limit(9) - 1) <= INT64_MAX / 9 &&
                  coord_limit(9) * coord_limit(9) > INT64_MAX / 9,
              "the largest bound for nine dimensions");
constexpr int64_t kAllLeft = INT64_MAX;          // splitter that sends every point left
constexpr int kMaxStack = 160;                   // traversal stack of the query kernels

// True while work enqueued on `st` is being captured into a graph: calls then
// only enqueue kernels (no allocation, no event, no readback).
inline bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

// Orders the LDS accesses of one wave: what a lane wrote is seen by every
// lane of the wave after this point.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tree node, 32 bytes.  Subtrees are contiguous slices [off, off+size) of the
// tree's point array (points are kept in in-order leaf order).
struct Node {
  int64_t x;       // interior: splitter coordinate (dim, x); left iff p[dim] < x
  int32_t size;    // number of points in the subtree
  int32_t off;     // first point of the subtree in the point array
  int32_t left;    // interior: left child; leaf: -1
  int32_t right;   // interior: right child; leaf: -1
  int16_t dim;     // interior: 0..D-1; leaf: -1
  int16_t depth;   // depth of the node in the whole tree (sampling salt)
  int32_t pad;
};
static_assert(sizeof(Node) == 32, "node layout");

// A subproblem of the build: the points [start, start+m) of some buffer,
// whose subtree root is to be written into node `slot` at tree depth `depth`.
struct Task {
  int32_t start;
  int32_t m;
  int32_t slot;
  int16_t depth;
  int8_t buf;      // 0: tree array A, 1: twin array B, 2: caller input
  int8_t mode;     // finisher: 0 plain build, 1 heavy leaf (identical points)
};
static_assert(sizeof(Task) == 16, "task layout");

// SplitMix64 finaliser (Steele, Lea & Flood 2014; variant-13 constants of the
// reference splitmix64.c) and the sampling key derived from it.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sample_key(uint64_t seed, int32_t depth, int64_t id) {
  return mix64(mix64(static_cast<uint64_t>(id) ^ seed) + static_cast<uint64_t>(depth + 1) * 0x9E3779B97F4A7C15ULL);
}

// The point buffers a kernel may read or write: 0 and 1 are the tree's two
// arrays (coordinate d of point i at c[b][d*cap[b] + i], id at id[b][i]),
// 2 is a caller-owned input.
struct Bufs {
  int64_t* c[3];
  int64_t* id[3];
  int64_t cap[3];
  int32_t* c32;    // the tree's packed 32-bit coordinates [c32cap][D], point by point (written by the finisher)
  int64_t c32cap;
};

struct Params {
  int D, lambda, phi, sigma, s;   // sigma 0: exact medians at every node (lambda 1, no sampling);
                                  // s is then the size below which the finisher takes over
  int64_t alpha_num, alpha_den;
  uint64_t seed;
  int tile;
  int cand_bias;   // test knob: shifts every candidate threshold (results unchanged)
  int update_events;   // test knob: 0 auto, 1 sorted event lists, 2 per-point arrays (results unchanged)
};

// Workgroups are handed to the 8 XCDs round robin (workgroup b runs on XCD
// b % 8), and each XCD has its own L2.  This maps workgroup b to a work item
// (a sieve tile, a block of spatially ordered queries) so that each XCD takes
// one contiguous range of them: neighbouring items, which share cache lines
// (the ends of bucket runs, the nodes and leaves of nearby queries), then
// meet in the same L2.  Bijective on [0, n) for any n.
__device__ inline int64_t xcd_tile(int64_t b, int64_t n) {
  const int64_t x = b & 7, per = n >> 3, rem = n & 7;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

// Device-side error flags (bitmask in one int).
enum : int {
  kErrRange = 1,
  kErrCandOverflow = 2,
  kErrCandUnderflow = 4,
  kErrNodeOverflow = 8,
  kErrStack = 16,
  kErrInternal = 32,
};

}  // namespace pkd

struct pkd_tree {
  pkd::Params prm;
  int64_t n = 0;          // points stored
  int64_t cap = 0;        // capacity of each point buffer
  int64_t* buf[2] = {nullptr, nullptr};  // buf[cur] holds the tree's points; the other is the twin
  int cur = 0;
  // coordinates of buf[cur] as int32 [cap][D], the D coordinates of a point
  // side by side (coordinates are below 2^30): what the query kernels scan,
  // at half the bytes of the int64 rows and with a leaf's points in few
  // cache lines
  int32_t* c32 = nullptr;
  int64_t c32_cap = 0;
  // the second packed copy an update writes its new layout into (swapped
  // with c32 when the update commits)
  int32_t* c32_twin = nullptr;
  int64_t c32_twin_cap = 0;
  pkd::Node* nodes = nullptr;
  int64_t node_cap = 0;
  int32_t node_count = 0; // node records in use, live or dead (node 0 is the root)
  int32_t compact_mark = 0;  // node_count after the last build or compaction
  int32_t height = 0;      // longest root-leaf path (edges), an upper bound after updates
  int32_t n_trees = 1;     // trees held: their roots are nodes 0 .. n_trees-1
  // copy items the last range report needed (sizes the next one's list)
  mutable int64_t report_items_hint = 0;
  // what the last update rebuilt: subtrees (regions) and their points
  int64_t last_regions = 0, last_rebuilt = 0;
  // bounding boxes of the nodes (int32 [node][lo D, hi D]) while bbox_on:
  // the query kernels then prune with them (recomputed after every update)
  int32_t* bbox = nullptr;
  int64_t bbox_cap = 0;
  bool bbox_on = false;
  // the tree of a graph build plan: its arrays are the ones the captured
  // launches write, so it is never updated, reallocated or freed on its own
  bool plan_owned = false;
};

// A batch build whose launches need no host read: every round's work is
// sized for the most it can hold, counts stay in device memory, so the whole
// build can be captured into a graph and replayed on new points of the same
// trees.  Rare cases the sized launches do not cover (a sampler retry, a
// sample of identical points, more rounds than planned, more node records
// than reserved) are flagged and the build is redone the usual way at finish.
struct pkd_build_plan {
  pkd_tree* T = nullptr;
  std::vector<pkd::Task> roots;    // root tasks (points of tree t at its offset)
  int64_t n = 0;                   // points of all trees
  int rounds = 0;                  // sieve rounds enqueued
  int64_t ns_max = 0, front_max = 0, fin_max = 0, ntiles_max = 0, nchunks_max = 0, cand_len = 0;
  const int64_t* in_c = nullptr;   // the inputs of the last enqueue
  const int64_t* in_id = nullptr;
  // device workspace
  pkd::Task *roots_d = nullptr, *front = nullptr, *next = nullptr, *sieve = nullptr, *fin = nullptr;
  int* ctr = nullptr;              // counters, see the driver
  int64_t *rx = nullptr, *tile_off = nullptr, *chunk_off = nullptr, *tot = nullptr;
  uint8_t* rdim = nullptr;
  int8_t *ext = nullptr, *mode = nullptr, *shift = nullptr, *shift_fix = nullptr;
  int* rootext = nullptr;
  uint64_t* cand_key = nullptr;
  uint32_t *cand_pos = nullptr, *cand_cnt = nullptr, *A = nullptr, *S = nullptr;
  int32_t *B = nullptr, *bsize = nullptr, *bstart = nullptr, *R = nullptr, *res_off = nullptr, *bsum = nullptr;
  int* lists = nullptr;
  std::vector<void*> blocks;       // every block of the workspace
};

// ---- host helpers shared by the sources (defined in pkd_api.hip) -----------
namespace pkd {
// The bounds query launches take from a tree.  Launches captured into a graph
// keep their arguments, so on a build plan's tree (rebuilt by every replay)
// they take the plan's limits: every node record it can hold, and the
// deepest traversal stack.
inline int32_t query_nodes(const pkd_tree* T) {
  return T->plan_owned ? static_cast<int32_t>(T->node_cap) : T->node_count;
}
inline int32_t query_height(const pkd_tree* T) { return T->plan_owned ? kMaxStack - 3 : T->height; }

int hip_status(hipError_t e, const char* what);
#define PKD_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::pkd::hip_status(e_, #call); \
  } while (0)
#define PKD_TRY(call)            \
  do {                           \
    int rc_ = (call);            \
    if (rc_ != PKD_OK) return rc_; \
  } while (0)

int dev_alloc(void** p, size_t bytes, hipStream_t s);
size_t dev_size_class(size_t bytes);   // bytes a dev_alloc of `bytes` actually provides
void dev_free(void* p, hipStream_t s);

inline int kernel_status(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, what);
  return PKD_OK;
}

// Grow-only device array (stream-ordered); need(n, keep) reallocates when
// more than the current capacity is needed, copying the old contents if keep.
template <class T>
struct DArr {
  T* p = nullptr;
  size_t cap = 0;
  hipStream_t st = nullptr;
  explicit DArr(hipStream_t s = nullptr) : st(s) {}
  DArr(const DArr&) = delete;
  DArr& operator=(const DArr&) = delete;
  int need(size_t n, bool keep = false) {
    if (n <= cap && p) return PKD_OK;
    size_t c = n + n / 4 > 256 ? n + n / 4 : 256;
    void* q = nullptr;
    PKD_TRY(dev_alloc(&q, c * sizeof(T), st));
    if (p && keep) PKD_HIP(hipMemcpyAsync(q, p, cap * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (p) dev_free(p, st);
    p = static_cast<T*>(q);
    cap = c;
    return PKD_OK;
  }
  ~DArr() {
    if (p) dev_free(p, st);
  }
};

// Scratch of one segmented sieve pass: tile and chunk layout, tile x bucket
// counts (A), write cursors (B), chunk sums (S), bucket sizes and starts.
struct SieveWork {
  DArr<int64_t> tile_off, chunk_off, tot;
  DArr<int8_t> shift;
  DArr<uint32_t> A, S;
  DArr<int32_t> B, bsize, bstart;
  explicit SieveWork(hipStream_t s)
      : tile_off(s), chunk_off(s), tot(s), shift(s), A(s), S(s), B(s), bsize(s), bstart(s) {}
};

// Exclusive prefix sum of n int32 values: out[i] = in[0] + .. + in[i-1] for
// i in [0, n]; bsum is scratch.
int exscan_i32(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, DArr<int32_t>& bsum);

// Stable LSD radix sort of (key, value) pairs by the low nbits bits of the
// keys (8 bits per pass).  The sorted pairs end either in the input arrays or
// in the work arrays; *kout / *vout point at them.
struct SortWork {
  DArr<uint64_t> k1;
  DArr<uint32_t> v1;
  DArr<int32_t> hist, off, bsum;
  explicit SortWork(hipStream_t st) : k1(st), v1(st), hist(st), off(st), bsum(st) {}
};
int radix_sort_pairs(hipStream_t st, uint64_t* keys, uint32_t* vals, int64_t n, int nbits, SortWork& W,
                     uint64_t** kout, uint32_t** vout);
int bits_for(int64_t v);   // bits needed to write 0 .. v

// The same scan and sort over work arrays the caller provides (nothing is
// allocated): exscan_i32_raw needs bsum [exscan_bsum_need(n)] and n below
// 2^27; the sort needs k1/v1 [n], hist [256 * radix_sort_blocks(n)],
// off [256 * radix_sort_blocks(n) + 1] and bsum [exscan_bsum_need(256 * blocks)].
int64_t exscan_bsum_need(int64_t n);
int exscan_i32_raw(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* bsum);
int64_t radix_sort_blocks(int64_t n);
struct SortBufs {
  uint64_t* k1;
  uint32_t* v1;
  int32_t *hist, *off, *bsum;
};
int radix_sort_pairs_raw(hipStream_t st, uint64_t* keys, uint32_t* vals, int64_t n, int nbits, const SortBufs& B,
                         uint64_t** kout, uint32_t** vout);

// (Re)allocate the packed 32-bit coordinates for the tree's capacity, and
// rewrite them from buf[cur] for all n points.
int ensure_c32(pkd_tree* T, hipStream_t st);
int refresh_c32(pkd_tree* T, hipStream_t st);

// LDS bytes that one workgroup of the skeleton and finisher kernels needs at
// most for D dimensions, sample size s and leaf size phi (both must fit one
// workgroup's LDS, kMaxLdsBytes).
size_t build_lds_need(int D, int s, int phi);
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Tile layout of `ns` tasks (device array): tiles of `tile` points, scan
// chunks; returns the numbers of tiles and chunks and the points covered.
// With known_pts >= 0 (the tasks' points, known to the caller) nothing is
// read back: the numbers returned are upper bounds (pts/tile + ns + 1 tiles),
// and the launches that use them must read the task count on the device.
int sieve_layout(hipStream_t st, const Task* tasks, int ns, int tile, SieveWork& W, int s, int small_max,
                 const int8_t* shift_override, int64_t* ntiles, int64_t* nchunks, int64_t* pts, int cand_bias = 0,
                 int64_t known_pts = -1);
// Count, column-major scan and stable scatter of the tasks' points from
// buffer src to dst through per-task routing skeletons rx/rdim ([ns][2^lambda]).
// Bucket sizes and starts land in W.bsize / W.bstart ([ns][2^lambda]).
// With dns set (the task count in device memory) ntiles and nchunks may be
// upper bounds: the workgroups past the real counts leave.
int sieve_pass(hipStream_t st, int D, int lambda, int tile, const Task* tasks, int ns, const Bufs& bufs, int src,
               int dst, const int64_t* rx, const uint8_t* rdim, const int8_t* mode, SieveWork& W, int64_t ntiles,
               int64_t nchunks, int64_t pts, int check, int* d_flags, const int* dns = nullptr);

// Build the subtrees of the given root tasks into `tree` (whose point buffers
// and node array are set up by the caller).  Points of the tasks live in the
// buffer named by Task::buf; results go to tree->buf[tree->cur].
int build_tasks(pkd_tree* tree, hipStream_t st, const std::vector<Task>& roots,
                const int64_t* in_coords, const int64_t* in_ids, int64_t input_cap);
// The same with the root tasks in device memory (n_roots of them, all in
// buffer src_buf).
int build_tasks_dev(pkd_tree* tree, hipStream_t st, const Task* d_roots, int n_roots, int src_buf,
                    const int64_t* in_coords, const int64_t* in_ids, int64_t input_cap);
int ensure_nodes(pkd_tree* tree, hipStream_t st, int64_t need);

// Tree storage (pkd_api.hip): both point buffers for at least `cap` points;
// release every device array of a tree (the object itself stays); a new tree
// built from caller input (headroom: room for a sixteenth more points);
// exchange the storage of two trees.
int alloc_points(pkd_tree* T, hipStream_t st, int64_t cap);
// Graph build plans (build.hip): workspace sizes and the enqueue of one build.
int plan_size(pkd_build_plan* G);
int plan_enqueue(pkd_build_plan* G, hipStream_t st);
void release(pkd_tree* T, hipStream_t st);
int build_new(const Params& prm, hipStream_t st, const int64_t* coords, const int64_t* ids, int64_t n,
              bool headroom, pkd_tree** out);
void swap_storage(pkd_tree* a, pkd_tree* b);
// Drop the records of dead nodes when they outnumber the rest (update.hip):
// live records keep their order (the roots stay first), links are renumbered.
// Returns PKD_OK also when it skips the compaction (nothing to gain, or no
// memory for the new array); the tree is valid either way.
int compact_nodes(pkd_tree* T, hipStream_t st);

// Bounding boxes of every live node (bbox.hip).
int compute_bbox(pkd_tree* T, hipStream_t st);

// The box of a node: from the stored boxes when there are any, else the
// caller's cell.
template <int D>
__device__ inline void node_box(const int32_t* __restrict__ bbox, int32_t node, int32_t (&lo)[D], int32_t (&hi)[D]) {
#pragma unroll
  for (int d = 0; d < D; ++d) {
    lo[d] = bbox[static_cast<int64_t>(node) * 2 * D + d];
    hi[d] = bbox[static_cast<int64_t>(node) * 2 * D + D + d];
  }
}

// Query launches (query.hip): k-NN and range counts over the trees of a
// handle (tree_of: per query, or null for tree 0); device errors are ORed
// into *flags.
int run_knn(const pkd_tree* T, hipStream_t st, const int64_t* q, const int32_t* tree_of, int64_t nq, int k,
            int64_t* oi, int64_t* od, int* flags);
int run_range(const pkd_tree* T, hipStream_t st, const int64_t* lo, const int64_t* hi, const int32_t* tree_of,
              int64_t nb, int64_t* out, int* flags);
// Range report (report.hip): counts, offsets and (with out_ids) the ids.
int run_range_report(const pkd_tree* T, hipStream_t st, const int64_t* lo, const int64_t* hi, const int32_t* tree_of,
                     int64_t nb, int64_t* offsets, int64_t* out_ids, int64_t cap, int64_t* total);

// A named range for profilers (roctx): shown around the library's calls and
// the rounds of a build in a rocprofv3 trace with --marker-trace.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Per-kernel timing (pkd_profile_*): Prof::begin/end bracket one launch with
// events on its stream; the elapsed time is collected at the next flush.
enum ProfKernel { kProfCount = 0, kProfScatter, kProfSelect, kProfFinish, kProfKnn, kProfRange, kProfReport, kProfN };
struct Prof {
  static bool on();
  static void begin(int kernel, hipStream_t st);
  static void end(int kernel, hipStream_t st, double alg_bytes);
  static void flush();   // after the stream has been synchronized
};
}  // namespace pkd
