/*
 * pkd.h -- C interface of the MI355X (gfx950) Pkd-tree library (libpkd.so).
 *
 * The library builds and maintains a kd-tree over int64 points with the
 * sampling-based multi-level sieve of "Parallel kd-tree with Batch Updates"
 * (Men, Shen, Gu, Sun, SIGMOD 2025):
 *   Build        -- Algorithm 1, Section 3.1
 *   BatchInsert  -- Algorithm 2, Section 4.1
 *   BatchDelete  -- Section 4.2
 *   k-NN, range count, range report -- Section 2 (definitions), Section 5
 *                (traversals)
 * Every step runs in HIP kernels on the GPU; this header holds only plain C
 * types.
 *
 * Conventions for every call
 *   - Return value: PKD_OK (0) or a negative PKD_ERR_* code; pkd_strerror()
 *     names it.  No C++ exception crosses this interface.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is ordered on that stream.  Calls that must report data-dependent
 *     errors (range checks) or that size their own work from device results
 *     synchronize the stream before returning; results are then ready.
 *   - Point sets are structure-of-arrays: `coords` is int64 [dim][n] (row d
 *     holds coordinate d of all points, contiguous), `ids` is int64 [n].  All
 *     point, query and output pointers given to a call are DEVICE pointers
 *     owned by the caller; the library only reads inputs and only writes
 *     outputs during the call's stream work.
 *   - Coordinates (points, queries, box corners) must lie in [0, 2^30), and
 *     point and query coordinates for dim = 9 in [0, 1012333500): squared
 *     distances, sums of dim squared differences, are then exact in int64
 *     (dim * (bound - 1)^2 < 2^63).  Violations return PKD_ERR_RANGE and leave
 *     any tree unchanged.
 *   - Ids are caller-chosen int64 values and must be unique within a tree
 *     (precondition; not checked).
 *   - A tree owns its device storage.  The library takes device memory from
 *     the allocator the caller installed with pkd_set_allocator, else from
 *     its own block cache (hipMalloc'd blocks of rounded sizes, kept after a
 *     free for reuse, a reuse on another stream ordered after the freeing
 *     stream by an event); the cache keeps at most half of device memory.
 *     A tree must not be used by two calls concurrently.
 *   - A mutating call (pkd_batch_insert, pkd_batch_delete) that fails leaves
 *     the tree as it was: it allocates everything it needs, and builds the
 *     subtrees it replaces in memory of its own, before it changes the tree.
 *     (PKD_ERR_HIP from a failing device is the exception: the device state
 *     is then unknown.)
 */
#ifndef PKD_H
#define PKD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PKD_OK 0
#define PKD_ERR_INVALID_ARG (-1)   /* null pointer, negative count, bad parameter */
#define PKD_ERR_RANGE (-2)         /* a coordinate outside its bound (see above) */
#define PKD_ERR_UNSUPPORTED (-3)   /* dim outside 1..9, sample size > 2048, n >= 2^31 */
#define PKD_ERR_OOM (-4)           /* device allocation failed */
#define PKD_ERR_HIP (-5)           /* a HIP runtime call failed */
#define PKD_ERR_CAPACITY (-6)      /* a query needs a deeper traversal stack than built in */
#define PKD_ERR_INTERNAL (-7)      /* an internal consistency check failed */

typedef struct pkd_tree pkd_tree;   /* opaque; device-resident */

/* Parameters that change the tree (Section 5 gives the defaults). */
typedef struct {
  int32_t dim;        /* D, 1..9 */
  int32_t lambda;     /* skeleton levels per sieve round (lambda), 1..8; default 6 */
  int32_t leaf_size;  /* leaf wrap phi: a leaf holds at most phi points unless all
                         its points are identical (heavy leaf); default 32 */
  int32_t oversample; /* sigma; the sample size is s = 2^lambda * sigma <= 2048;
                         default 32 (s = 2048).  0 (with lambda = 1): no sampling --
                         every node is split at the exact median of all its points
                         (the plain construction of Section 3 at every level, the
                         comparison of Section 6.4) */
  int32_t alpha_num;  /* balance parameter alpha = alpha_num / alpha_den with */
  int32_t alpha_den;  /* 0 <= 2*alpha_num <= alpha_den (alpha = 1/2: nothing is ever
                         rebuilt for balance); default 3/10 */
  uint64_t seed;      /* seed of the sampling hash; default 42 */
} pkd_params;

/* Parameters that never change any result (work decomposition only). */
typedef struct {
  int32_t tile_points;      /* points per sieve tile: 1024, 2048 or 4096; default 2048 */
  int32_t cand_shift_bias;  /* test knob, default 0, |bias| <= 4: added to the exponent of
                               every sieving subproblem's sample-candidate threshold, so the
                               sampler's overflow (bias < 0) or underflow (bias > 0) retry
                               runs; the tree never changes */
  int32_t update_events;    /* test knob, default 0: how a batch update places the old
                               points: 0 by the batch's density, 1 always from the sorted
                               update events, 2 always from per-point arrays; the tree
                               never changes */
  int32_t reserved[5];
} pkd_tuning;

/*
 * Device memory supplied by the caller (for example a framework's caching
 * allocator).  alloc returns at least `bytes` bytes of device memory usable in
 * work ordered on `stream` (a hipStream_t as void*), or NULL when it cannot;
 * the library then fails the call with PKD_ERR_OOM.  free returns a block the
 * library no longer needs; work enqueued on `stream` before the free may still
 * use it, so the allocator must not hand it to other streams before that work
 * is done.  Both may be called from any thread that calls into the library,
 * without library locks held.
 */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* stream, void* ctx);
  void* ctx;
} pkd_allocator;

/*
 * Install `a` (copied) as the source of all later device allocations of the
 * library, or go back to the library's block cache with NULL.  Blocks always
 * return to the allocator that made them, so its functions and ctx must stay
 * valid as long as the library holds any block they returned (for example a
 * tree built while it was installed).  Trees may exist while it changes.
 */
int pkd_set_allocator(const pkd_allocator* a);

/* Fill defaults for dimension `dim`. */
void pkd_default_params(pkd_params* p, int32_t dim);
void pkd_default_tuning(pkd_tuning* t);

/*
 * Build (Algorithm 1, Section 3.1).  Builds a tree over the n points
 * (coords: device int64 [dim][n], ids: device int64 [n]); n may be 0.
 * tuning may be NULL (defaults).  On success *out receives a new tree, which
 * the caller releases with pkd_free.  The inputs are not modified and are no
 * longer referenced after the call returns.  Synchronizes `stream`.
 */
int pkd_build(const pkd_params* params, const pkd_tuning* tuning, void* stream,
              const int64_t* coords, const int64_t* ids, int64_t n, pkd_tree** out);

/*
 * BatchInsert (Algorithm 2, Section 4.1).  Inserts m points (device
 * coords [dim][m], ids [m]; ids not yet in the tree).  A node whose two
 * subtrees stay alpha-weight-balanced after the insertion is kept; the topmost
 * node that would become unbalanced is rebuilt from its points and the batch
 * points below it; a leaf that receives points becomes Build(leaf + points).
 * Synchronizes `stream`.
 */
int pkd_batch_insert(pkd_tree* tree, void* stream, const int64_t* coords,
                     const int64_t* ids, int64_t m);

/*
 * BatchDelete (Section 4.2).  Removes, for every batch entry (device
 * coords [dim][m], ids [m]), the stored point with the same id and the same
 * coordinates; entries that match no stored point are ignored, a repeated
 * entry removes once.  Subtrees that become alpha-unbalanced are rebuilt
 * (topmost first) from their remaining points.  *n_deleted (host pointer, may
 * be NULL) receives the number of points removed.  Synchronizes `stream`.
 */
int pkd_batch_delete(pkd_tree* tree, void* stream, const int64_t* coords,
                     const int64_t* ids, int64_t m, int64_t* n_deleted);

/*
 * k-NN (Section 2; depth-first search of Section 5).  For each of the nq
 * queries (device int64 [dim][nq]) writes the min(k, n) stored points with the
 * smallest (squared distance, id) pairs, ascending, into out_ids / out_d2
 * (device int64 [nq][k], row-major); unused slots get -1.  Squared distances
 * are exact int64.  1 <= k <= 128.  Synchronizes `stream`.
 */
int pkd_knn(const pkd_tree* tree, void* stream, const int64_t* queries, int64_t nq,
            int32_t k, int64_t* out_ids, int64_t* out_d2);

/*
 * k-NN that allocates no device memory, for callers that cannot allocate while
 * they run: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Arguments, results and errors as for pkd_knn, with
 * nq <= PKD_KNN_NOALLOC_MAX_QUERIES (larger batches return
 * PKD_ERR_UNSUPPORTED before any work is enqueued).  The scratch pkd_knn takes
 * from the block cache (error flags, Morton keys, radix sort work arrays;
 * 24 bytes per query) comes from one statically allocated device array of
 * 25 MiB + 64 KiB per GPU, held until the process ends.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialized by the caller.  Synchronizes `stream`.
 */
#define PKD_KNN_NOALLOC_MAX_QUERIES 1048576
int pkd_knn_noalloc(const pkd_tree* tree, void* stream, const int64_t* queries, int64_t nq,
                    int32_t k, int64_t* out_ids, int64_t* out_d2);

/*
 * Range count (Section 2; traversal with subtree sizes, Section 5).  For each
 * closed box [lo, hi] (device int64 [dim][nb] each) writes the number of stored
 * points p with lo_d <= p_d <= hi_d in every dimension into out (device int64
 * [nb]); a box with lo_d > hi_d in some dimension counts 0.
 * Synchronizes `stream`.
 */
int pkd_range_count(const pkd_tree* tree, void* stream, const int64_t* lo,
                    const int64_t* hi, int64_t nb, int64_t* out);

/*
 * Range report (Section 2; Section 5: a subtree whose cell lies inside the box
 * is reported whole, a straddling leaf is filtered).  For each closed box j
 * (lo, hi: device int64 [dim][nb]; lo_d > hi_d in some dimension reports
 * nothing) the ids of the stored points in it go to out_ids[offsets[j] ..
 * offsets[j+1]) (device), in no particular order.  offsets (device int64
 * [nb+1]) receives the
 * exclusive prefix sum of the box counts and *total (host) their sum.  With
 * out_ids NULL only offsets and *total are computed (to size the output);
 * if *total > cap nothing is written to out_ids and PKD_ERR_CAPACITY is
 * returned.  Synchronizes `stream`.
 */
int pkd_range_report(const pkd_tree* tree, void* stream, const int64_t* lo, const int64_t* hi,
                     int64_t nb, int64_t* offsets, int64_t* out_ids, int64_t cap, int64_t* total);

/*
 * Batched build of many independent trees in one pass of the segmented
 * pipeline: every sieve round and the finisher run over the subproblems of all
 * trees at once, so the number of launches does not grow with the number of
 * trees.  coords/ids (device) hold the trees' points back to back: tree t owns
 * positions [offsets[t], offsets[t+1]) (offsets: HOST int64 [n_trees+1],
 * offsets[0] = 0, non-decreasing).  All trees share `params`.  The handle holds
 * n_trees trees; each is exactly the tree pkd_build would make of its points.
 * Batch handles answer pkd_knn_batch / pkd_range_count_batch, export one
 * tree at a time and take updates tree by tree (pkd_batch_insert_tree /
 * pkd_batch_delete_tree).
 */
int pkd_build_batch(const pkd_params* params, const pkd_tuning* tuning, void* stream,
                    int32_t n_trees, const int64_t* coords, const int64_t* ids,
                    const int64_t* offsets, pkd_tree** out);

/*
 * BatchInsert / BatchDelete on tree t of a handle (t = 0 for a single tree:
 * pkd_batch_insert / pkd_batch_delete are these with t = 0).  Semantics,
 * arguments and errors as for those calls; the other trees of the handle do
 * not change.
 */
int pkd_batch_insert_tree(pkd_tree* tree, int32_t t, void* stream, const int64_t* coords,
                          const int64_t* ids, int64_t m);
int pkd_batch_delete_tree(pkd_tree* tree, int32_t t, void* stream, const int64_t* coords,
                          const int64_t* ids, int64_t m, int64_t* n_deleted);

/* Number of trees held by a handle (1 for pkd_build). */
int pkd_num_trees(const pkd_tree* tree, int32_t* n_trees);

/*
 * Build plans: the batch build above (Algorithm 1 for every tree) enqueued
 * without any host read, so that one build can be captured into a hipGraph
 * and the graph replayed on new points of the same trees (with query launches
 * captured after it, see pkd_knn_async).  Every sieve round is launched with
 * grids sized for the most work it can hold and reads its counts from device
 * memory; the base cases run in persistent grids that walk their lists.
 *
 * pkd_build_plan_create: params and tuning as for pkd_build (oversample 0,
 *   the exact-median mode, returns PKD_ERR_UNSUPPORTED); n_trees and offsets
 *   (HOST int64 [n_trees+1], as for pkd_build_batch) fix the trees' sizes for
 *   every build of the plan.  Allocates the plan's tree and a workspace sized
 *   for the worst case (about 3 sample-size candidate slots per sieve
 *   subproblem and the node records the rounds can make); synchronizes.
 * pkd_build_plan_enqueue: enqueues one build of the trees over coords / ids
 *   (device, layout of pkd_build_batch) on `stream`: kernel launches only (no
 *   allocation, no host read, no event), so the call may be captured; every
 *   replay rebuilds from what the same buffers then hold.
 * pkd_build_plan_finish: waits for `stream`, checks the build and makes the
 *   plan's tree valid.  Cases the sized launches do not cover (a sampler retry,
 *   a sample of identical points, more rounds than planned, more node records
 *   than reserved) are built again the usual way into the same arrays, with
 *   *redone (optional) set to 1; the tree is the same either way.  Returns
 *   PKD_ERR_RANGE for a coordinate outside its bound (the tree is then empty).
 * pkd_build_plan_tree: the plan's tree, owned by the plan.  It holds the last
 *   finished build until the next enqueue; it answers queries, while updates,
 *   bounding boxes and pkd_free_async return PKD_ERR_INVALID_ARG and pkd_free
 *   does nothing.
 * pkd_build_plan_free: frees the plan and its tree (waits for the device).
 */
typedef struct pkd_build_plan pkd_build_plan;
int pkd_build_plan_create(const pkd_params* params, const pkd_tuning* tuning, int32_t n_trees,
                          const int64_t* offsets, pkd_build_plan** out);
int pkd_build_plan_enqueue(pkd_build_plan* plan, void* stream, const int64_t* coords,
                           const int64_t* ids);
int pkd_build_plan_finish(pkd_build_plan* plan, void* stream, int32_t* redone);
int pkd_build_plan_tree(pkd_build_plan* plan, pkd_tree** tree);
void pkd_build_plan_free(pkd_build_plan* plan);

/*
 * k-NN / range count over the trees of a batch handle: query j runs on tree
 * tree_of[j] (device int32 [nq]; NULL means tree 0).  Other arguments and the
 * output layout as for pkd_knn / pkd_range_count.
 */
int pkd_knn_batch(const pkd_tree* tree, void* stream, const int64_t* queries,
                  const int32_t* tree_of, int64_t nq, int32_t k, int64_t* out_ids,
                  int64_t* out_d2);
int pkd_range_count_batch(const pkd_tree* tree, void* stream, const int64_t* lo,
                          const int64_t* hi, const int32_t* tree_of, int64_t nb,
                          int64_t* out);
int pkd_range_report_batch(const pkd_tree* tree, void* stream, const int64_t* lo,
                           const int64_t* hi, const int32_t* tree_of, int64_t nb,
                           int64_t* offsets, int64_t* out_ids, int64_t cap, int64_t* total);

/*
 * Asynchronous forms of pkd_knn_batch / pkd_range_count_batch for callers that
 * overlap work (a serving loop): the kernel is enqueued on `stream` and the
 * call returns without synchronizing.  Data-dependent errors are ORed into
 * *status (device int32, zeroed by the caller beforehand) instead of being
 * returned: 1 = a coordinate outside its bound, 16 = traversal stack too
 * small, 32 = inconsistent tree or tree index.  Outputs and *status are valid
 * once the stream reaches this point.  The tree must not be modified until then.
 * While `stream` is being captured into a graph (hipStreamBeginCapture) these
 * two calls enqueue kernels only, with no allocation and no event: large
 * batches then skip the spatial ordering of the queries, which changes only
 * the speed.  A sequence of query batches can so be captured once and
 * replayed with new data in the same buffers.
 */
int pkd_knn_async(const pkd_tree* tree, void* stream, const int64_t* queries,
                  const int32_t* tree_of, int64_t nq, int32_t k, int64_t* out_ids,
                  int64_t* out_d2, int32_t* status);
int pkd_range_count_async(const pkd_tree* tree, void* stream, const int64_t* lo,
                          const int64_t* hi, const int32_t* tree_of, int64_t nb,
                          int64_t* out, int32_t* status);

/* Canonical export of tree t of a handle (see pkd_export). */
int pkd_export_tree_sizes(const pkd_tree* tree, int32_t t, int64_t* num_nodes, int64_t* n);
int pkd_export_tree(const pkd_tree* tree, int32_t t, int64_t* rows, int64_t* leaf_ids,
                    int64_t* leaf_coords, int32_t* depths);

/* Number of points (host out). */
int pkd_size(const pkd_tree* tree, int64_t* n);

/* Sizes needed by pkd_export: number of nodes and of points (host outs). */
int pkd_export_sizes(const pkd_tree* tree, int64_t* num_nodes, int64_t* n);

/*
 * Canonical host copy of the tree (a test aid).  HOST buffers:
 *   rows        int64 [num_nodes][4]: pre-order (kind, dim, x, size); kind 0 =
 *               interior node with splitter (dim, x), 1 = leaf (dim -1, x 0)
 *   leaf_ids    int64 [n]: ids of the leaf points, leaves in pre-order, ids
 *               ascending inside each leaf
 *   leaf_coords int64 [dim][n]: their coordinates
 * Any of the three pointers may be NULL.  depths (int32 [num_nodes], may be
 * NULL) receives each node's depth.
 */
int pkd_export(const pkd_tree* tree, int64_t* rows, int64_t* leaf_ids,
               int64_t* leaf_coords, int32_t* depths);

/* Height of the tree (edges on the longest root-leaf path). */
int pkd_height(const pkd_tree* tree, int32_t* height);

/*
 * Kernel timing (diagnostics).  pkd_profile_enable(1) clears and starts
 * per-kernel accounting: every launch of the kernels below is bracketed by HIP
 * events on the stream it runs on; pkd_profile_get(kernel, ...) returns the
 * number of launches, their summed duration in milliseconds and the summed
 * algorithmic bytes (what the method must move: for the sieve count pass 8*D
 * bytes per point, for the scatter pass 2*(8*D+8) bytes per point).
 * kernel: 0 sieve count, 1 sieve scatter, 2 sample select + skeleton,
 * 3 finisher, 4 k-NN, 5 range count, 6 range report (walk and copy; 16 bytes
 * per reported id).  Host outs; any may be NULL.
 */
int pkd_profile_enable(int32_t on);
int pkd_profile_get(int32_t kernel, int64_t* launches, double* total_ms, double* alg_bytes);

/* Release a tree (NULL is ignored).  Waits for all work on the device first. */
void pkd_free(pkd_tree* tree);

/*
 * Release a tree in stream order: its memory is reused only by work ordered
 * after what was enqueued on `stream` before this call; the caller must not
 * have work that uses the tree on other streams still in flight.  Does not
 * synchronize.
 */
int pkd_free_async(pkd_tree* tree, void* stream);

/*
 * Bounding boxes (the Pkd-bb variant of Section 6.3).  With on != 0 the tree
 * computes the tight box of every node's points (2 * dim int32 per node) and
 * keeps it current across updates; range counts, range reports and k-NN with
 * k <= 32 then prune with the boxes instead of the cells derived from the
 * splitters (Section 5).  Results are identical either way; the boxes cost
 * memory and box loads and save visited nodes.  on = 0 drops them.
 * Synchronizes `stream`.
 */
int pkd_set_bbox(pkd_tree* tree, void* stream, int32_t on);

/* The boxes of tree t of a handle in the pre-order of pkd_export: int32
 * [num_nodes][2 * dim] = (lo_0..lo_{D-1}, hi_0..hi_{D-1}); an empty node's
 * box has lo = 2^31-1, hi = -1.  Needs pkd_set_bbox(.., 1).  A test aid. */
int pkd_export_bbox(const pkd_tree* tree, int32_t t, int32_t* boxes);

/*
 * What the last pkd_batch_insert / pkd_batch_delete on the tree rebuilt (a
 * diagnostic; the cost the update theorem of Section 4.3 amortizes): the
 * number of subtrees rebuilt by Build (leaves that received points, and the
 * topmost nodes that became unbalanced) and the points in them.  Host outs;
 * either may be NULL.
 */
int pkd_update_stats(const pkd_tree* tree, int64_t* regions, int64_t* points);

/* Node records the tree holds, live and dead (updates leave the records of
 * replaced nodes dead until a compaction drops them; a diagnostic). */
int pkd_node_slots(const pkd_tree* tree, int64_t* slots);

const char* pkd_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PKD_H */
