// C interface of libpkd: argument checks, tree storage, query launches and the
// canonical export.  See include/pkd.h for the contract of every call.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "pkd_internal.h"

namespace pkd {

int run_knn_static(const pkd_tree* T, hipStream_t st, const int64_t* q, int64_t nq, int k, int64_t* oi,
                   int64_t* od);
int run_insert(pkd_tree* T, int32_t tree, hipStream_t st, const int64_t* coords, const int64_t* ids, int64_t m);
int run_delete(pkd_tree* T, int32_t tree, hipStream_t st, const int64_t* coords, const int64_t* ids, int64_t m,
               int64_t* removed);

int hip_status(hipError_t e, const char* what) {
  if (std::getenv("PKD_VERBOSE")) std::fprintf(stderr, "libpkd: %s failed: %s\n", what, hipGetErrorString(e));
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? PKD_ERR_OOM : PKD_ERR_HIP;
}

namespace {
// Device memory cache.  Builds and updates allocate and free large scratch
// arrays on every call; a tree's buffers come and go with the tree.  Freed
// blocks are kept per size class (sizes rounded up by at most 1/8) with an
// event recorded on the freeing stream: a later request of the same class
// takes the block back (on another stream it first waits for that event),
// so steady-state calls map no new memory (mapping runs at a few tens of GB/s,
// so a fresh tree-sized block costs seconds at 1e9 points).  The cache holds
// at most half of device memory; beyond that the oldest blocks are returned.
struct Cached {
  void* p;
  hipStream_t st;
  hipEvent_t ev;
  uint64_t age;
};

std::mutex g_mu;
std::multimap<size_t, Cached> g_free;        // size class -> freed blocks
std::unordered_map<void*, size_t> g_size;    // live and cached blocks -> size class
size_t g_cached = 0, g_limit = 0;
uint64_t g_clock = 0;

// A caller-installed allocator (pkd_set_allocator) replaces the cache for new
// blocks; every block remembers the allocator that made it, so it goes back
// there even after the caller switched allocators.
bool g_ext_on = false;
pkd_allocator g_ext;
struct ExtBlock {
  pkd_allocator a;
  size_t bytes;
};
std::unordered_map<void*, ExtBlock> g_ext_blocks;

}  // namespace

size_t dev_size_class(size_t b) {
  if (b <= 4096) return 4096;
  const int lg = 63 - __builtin_clzll(static_cast<unsigned long long>(b));
  const size_t unit = size_t{1} << (lg - 3);
  return (b + unit - 1) / unit * unit;
}

namespace {
// Returns one cached block to the device (caller holds g_mu).
void evict(std::multimap<size_t, Cached>::iterator it) {
  (void)hipEventSynchronize(it->second.ev);
  (void)hipEventDestroy(it->second.ev);
  (void)hipFree(it->second.p);
  g_size.erase(it->second.p);
  g_cached -= it->first;
  g_free.erase(it);
}

void evict_oldest_until(size_t limit) {
  while (g_cached > limit && !g_free.empty()) {
    auto old = g_free.begin();
    for (auto it = g_free.begin(); it != g_free.end(); ++it)
      if (it->second.age < old->second.age) old = it;
    evict(old);
  }
}
}  // namespace

int dev_alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  const size_t cls = dev_size_class(bytes);
  pkd_allocator ext;
  bool use_ext = false;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    use_ext = g_ext_on;
    ext = g_ext;
  }
  if (use_ext) {
    // the callback runs without the library's lock held (it may call back
    // into a runtime that takes locks of its own)
    void* q = ext.alloc(cls, static_cast<void*>(s), ext.ctx);
    if (!q) return PKD_ERR_OOM;
    std::lock_guard<std::mutex> lock(g_mu);
    g_ext_blocks[q] = ExtBlock{ext, cls};
    *p = q;
    return PKD_OK;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_limit == 0) {
    size_t free_b = 0, total_b = 0;
    g_limit = hipMemGetInfo(&free_b, &total_b) == hipSuccess && total_b > 0 ? total_b / 2 : (size_t{8} << 30);
  }
  auto range = g_free.equal_range(cls);
  for (auto it = range.first; it != range.second; ++it) {
    if (it->second.st != s && hipStreamWaitEvent(s, it->second.ev, 0) != hipSuccess) continue;
    *p = it->second.p;
    (void)hipEventDestroy(it->second.ev);
    g_cached -= cls;
    g_free.erase(it);
    return PKD_OK;
  }
  hipError_t e = hipMalloc(p, cls);
  if (e != hipSuccess) {
    // out of memory: return every cached block and try once more
    (void)hipGetLastError();
    evict_oldest_until(0);
    e = hipMalloc(p, cls);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_status(e, "device allocation");
  }
  g_size[*p] = cls;
  return PKD_OK;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  {
    ExtBlock blk;
    bool found = false;
    {
      std::lock_guard<std::mutex> lock(g_mu);
      auto it = g_ext_blocks.find(p);
      if (it != g_ext_blocks.end()) {
        blk = it->second;
        g_ext_blocks.erase(it);
        found = true;
      }
    }
    if (found) {
      blk.a.free(p, blk.bytes, static_cast<void*>(s), blk.a.ctx);
      return;
    }
  }
  std::lock_guard<std::mutex> lock(g_mu);
  auto sz = g_size.find(p);
  if (sz == g_size.end()) return;
  hipEvent_t ev;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, s) != hipSuccess) {
    // cannot order a reuse after the last use: wait and return the block
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    g_size.erase(sz);
    return;
  }
  g_free.emplace(sz->second, Cached{p, s, ev, ++g_clock});
  g_cached += sz->second;
  evict_oldest_until(g_limit);
}

// ---- kernel timing -------------------------------------------------------
namespace {
struct ProfState {
  bool on = false;
  int64_t launches[kProfN] = {0};
  double ms[kProfN] = {0};
  double bytes[kProfN] = {0};
  struct Pending {
    int kernel;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> spare;
  hipEvent_t open_ev[kProfN] = {nullptr};
  hipEvent_t get() {
    if (!spare.empty()) {
      hipEvent_t e = spare.back();
      spare.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};
ProfState g_prof;
}  // namespace

bool Prof::on() { return g_prof.on; }
void Prof::begin(int kernel, hipStream_t st) {
  if (!g_prof.on || capturing(st)) return;
  hipEvent_t e = g_prof.get();
  (void)hipEventRecord(e, st);
  g_prof.open_ev[kernel] = e;
}
void Prof::end(int kernel, hipStream_t st, double alg_bytes) {
  if (!g_prof.on || !g_prof.open_ev[kernel]) return;
  hipEvent_t e = g_prof.get();
  (void)hipEventRecord(e, st);
  g_prof.pending.push_back({kernel, g_prof.open_ev[kernel], e, alg_bytes});
  g_prof.open_ev[kernel] = nullptr;
}
void Prof::flush() {
  for (auto& p : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_prof.launches[p.kernel] += 1;
      g_prof.ms[p.kernel] += ms;
      g_prof.bytes[p.kernel] += p.bytes;
    }
    g_prof.spare.push_back(p.a);
    g_prof.spare.push_back(p.b);
  }
  g_prof.pending.clear();
}

int ensure_nodes(pkd_tree* T, hipStream_t st, int64_t need) {
  if (need <= T->node_cap) return PKD_OK;
  if (need >= INT32_MAX) return PKD_ERR_UNSUPPORTED;
  int64_t cap = std::max<int64_t>(need + need / 4, 1024);
  cap = std::min<int64_t>(cap, INT32_MAX - 1);
  void* q = nullptr;
  PKD_TRY(dev_alloc(&q, sizeof(Node) * cap, st));
  if (T->nodes && T->node_count > 0)
    PKD_HIP(hipMemcpyAsync(q, T->nodes, sizeof(Node) * T->node_count, hipMemcpyDeviceToDevice, st));
  dev_free(T->nodes, st);
  T->nodes = static_cast<Node*>(q);
  T->node_cap = cap;
  return PKD_OK;
}

int check_params(const pkd_params* p, const pkd_tuning* t, Params* out) {
  if (!p) return PKD_ERR_INVALID_ARG;
  if (p->dim < 1 || p->dim > kMaxDim) return PKD_ERR_UNSUPPORTED;
  if (p->lambda < 1 || p->lambda > kMaxLambda || p->leaf_size < 1 || p->oversample < 0) return PKD_ERR_INVALID_ARG;
  // oversample 0: exact medians at every node, one level per round (no sampling)
  if (p->oversample == 0 && p->lambda != 1) return PKD_ERR_INVALID_ARG;
  if (p->alpha_den <= 0 || p->alpha_num < 0 || 2 * static_cast<int64_t>(p->alpha_num) > p->alpha_den)
    return PKD_ERR_INVALID_ARG;
  int64_t s = p->oversample == 0 ? kMaxSample : static_cast<int64_t>(p->oversample) << p->lambda;
  if (s > kMaxSample) return PKD_ERR_UNSUPPORTED;
  if (build_lds_need(p->dim, static_cast<int>(s), p->leaf_size) > kMaxLdsBytes) return PKD_ERR_UNSUPPORTED;
  int tile = t ? t->tile_points : 2048;
  if (tile != 1024 && tile != 2048 && tile != 4096) return PKD_ERR_INVALID_ARG;
  const int bias = t ? t->cand_shift_bias : 0;
  if (bias < -4 || bias > 4) return PKD_ERR_INVALID_ARG;
  const int events = t ? t->update_events : 0;
  if (events < 0 || events > 2) return PKD_ERR_INVALID_ARG;
  out->D = p->dim;
  out->lambda = p->lambda;
  out->phi = p->leaf_size;
  out->sigma = p->oversample;
  out->s = static_cast<int>(s);
  out->alpha_num = p->alpha_num;
  out->alpha_den = p->alpha_den;
  out->seed = p->seed;
  out->tile = tile;
  out->cand_bias = bias;
  out->update_events = events;
  return PKD_OK;
}

// Allocate both point buffers of the tree with capacity `cap`.
// Point buffers for at least `cap` points; the capacity is whatever the
// rounded allocation holds.
int alloc_points(pkd_tree* T, hipStream_t st, int64_t cap) {
  cap = std::max<int64_t>(cap, 1);
  const size_t per = sizeof(int64_t) * static_cast<size_t>(T->prm.D + 1);
  const size_t bytes = dev_size_class(per * static_cast<size_t>(cap));
  cap = static_cast<int64_t>(bytes / per);
  void* a = nullptr;
  void* b = nullptr;
  PKD_TRY(dev_alloc(&a, bytes, st));
  int rc = dev_alloc(&b, bytes, st);
  if (rc != PKD_OK) {
    dev_free(a, st);
    return rc;
  }
  T->buf[0] = static_cast<int64_t*>(a);
  T->buf[1] = static_cast<int64_t*>(b);
  T->cap = cap;
  T->cur = 0;
  return PKD_OK;
}

void release(pkd_tree* T, hipStream_t st) {
  if (!T) return;
  dev_free(T->buf[0], st);
  dev_free(T->buf[1], st);
  dev_free(T->nodes, st);
  dev_free(T->c32, st);
  dev_free(T->c32_twin, st);
  dev_free(T->bbox, st);
  T->bbox = nullptr;
  T->bbox_cap = 0;
  T->buf[0] = T->buf[1] = nullptr;
  T->nodes = nullptr;
  T->c32 = T->c32_twin = nullptr;
  T->c32_cap = T->c32_twin_cap = 0;
  T->node_cap = 0;
  T->node_count = 0;
}

void swap_storage(pkd_tree* a, pkd_tree* b) {
  std::swap(a->n, b->n);
  std::swap(a->cap, b->cap);
  std::swap(a->buf[0], b->buf[0]);
  std::swap(a->buf[1], b->buf[1]);
  std::swap(a->cur, b->cur);
  std::swap(a->c32, b->c32);
  std::swap(a->c32_cap, b->c32_cap);
  std::swap(a->c32_twin, b->c32_twin);
  std::swap(a->c32_twin_cap, b->c32_twin_cap);
  std::swap(a->nodes, b->nodes);
  std::swap(a->node_cap, b->node_cap);
  std::swap(a->node_count, b->node_count);
  std::swap(a->compact_mark, b->compact_mark);
  std::swap(a->height, b->height);
  std::swap(a->n_trees, b->n_trees);
  std::swap(a->last_regions, b->last_regions);
  std::swap(a->last_rebuilt, b->last_rebuilt);
}

int write_empty_root(pkd_tree* T, hipStream_t st) {
  Node nd;
  std::memset(&nd, 0, sizeof(nd));
  nd.left = nd.right = -1;
  nd.dim = -1;
  PKD_HIP(hipMemcpyAsync(T->nodes, &nd, sizeof(nd), hipMemcpyHostToDevice, st));
  PKD_HIP(hipStreamSynchronize(st));
  T->node_count = 1;
  T->height = 0;
  return PKD_OK;
}

int flags_alloc(int** f, hipStream_t st) {
  PKD_TRY(dev_alloc(reinterpret_cast<void**>(f), sizeof(int) * 4, st));
  PKD_HIP(hipMemsetAsync(*f, 0, sizeof(int) * 4, st));
  return PKD_OK;
}

int flags_check(int* f, hipStream_t st) {
  int h = 0;
  PKD_HIP(hipMemcpyAsync(&h, f, sizeof(int), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));
  dev_free(f, st);
  if (h & kErrRange) return PKD_ERR_RANGE;
  if (h & kErrStack) return PKD_ERR_CAPACITY;
  if (h) return PKD_ERR_INTERNAL;
  return PKD_OK;
}

int build_new(const Params& prm, hipStream_t st, const int64_t* coords, const int64_t* ids, int64_t n,
              bool headroom, pkd_tree** out) {
  *out = nullptr;
  pkd_tree* T = new pkd_tree;
  T->prm = prm;
  // room for later inserts: a sixteenth more than the points (plus what the
  // rounded allocation holds), so moderate batches never reallocate
  int rc = alloc_points(T, st, headroom ? n + n / 16 : n);
  if (rc == PKD_OK) rc = ensure_nodes(T, st, std::max<int64_t>(1024, n / 8));
  if (rc == PKD_OK) {
    if (n == 0) {
      rc = write_empty_root(T, st);
    } else {
      T->node_count = 1;
      T->height = 0;
      Task root;
      root.start = 0;
      root.m = static_cast<int32_t>(n);
      root.slot = 0;
      root.depth = 0;
      root.buf = 2;
      root.mode = 0;
      rc = build_tasks(T, st, std::vector<Task>{root}, coords, ids, n);
    }
  }
  if (rc != PKD_OK) {
    release(T, st);
    (void)hipStreamSynchronize(st);
    delete T;
    return rc;
  }
  T->n = n;
  T->compact_mark = T->node_count;
  *out = T;
  return PKD_OK;
}

}  // namespace pkd

using namespace pkd;

extern "C" {

void pkd_default_params(pkd_params* p, int32_t dim) {
  if (!p) return;
  p->dim = dim;
  p->lambda = 6;
  p->leaf_size = 32;
  p->oversample = 32;
  p->alpha_num = 3;
  p->alpha_den = 10;
  p->seed = 42;
}

void pkd_default_tuning(pkd_tuning* t) {
  if (!t) return;
  std::memset(t, 0, sizeof(*t));
  t->tile_points = 2048;
}

int pkd_build(const pkd_params* params, const pkd_tuning* tuning, void* stream, const int64_t* coords,
              const int64_t* ids, int64_t n, pkd_tree** out) {
  TraceRange tr("pkd_build");
  if (!out) return PKD_ERR_INVALID_ARG;
  *out = nullptr;
  Params prm;
  PKD_TRY(check_params(params, tuning, &prm));
  if (n < 0 || (n > 0 && (!coords || !ids))) return PKD_ERR_INVALID_ARG;
  if (n >= INT32_MAX) return PKD_ERR_UNSUPPORTED;
  return build_new(prm, static_cast<hipStream_t>(stream), coords, ids, n, true, out);
}

int pkd_knn_batch(const pkd_tree* tree, void* stream, const int64_t* queries, const int32_t* tree_of, int64_t nq,
                  int32_t k, int64_t* out_ids, int64_t* out_d2) {
  TraceRange tr("pkd_knn");
  if (!tree || nq < 0 || k < 1 || k > 128) return PKD_ERR_INVALID_ARG;
  if (nq == 0) return PKD_OK;
  if (!queries || !out_ids || !out_d2) return PKD_ERR_INVALID_ARG;
  if (!tree_of && tree->n_trees < 1) return PKD_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* f = nullptr;
  PKD_TRY(flags_alloc(&f, st));
  Prof::begin(kProfKnn, st);
  int rc = run_knn(tree, st, queries, tree_of, nq, k, out_ids, out_d2, f);
  Prof::end(kProfKnn, st, 0.0);
  int rc2 = flags_check(f, st);
  return rc != PKD_OK ? rc : rc2;
}

int pkd_knn_async(const pkd_tree* tree, void* stream, const int64_t* queries, const int32_t* tree_of, int64_t nq,
                  int32_t k, int64_t* out_ids, int64_t* out_d2, int32_t* status) {
  if (!tree || nq < 0 || k < 1 || k > 128 || !status) return PKD_ERR_INVALID_ARG;
  if (nq == 0) return PKD_OK;
  if (!queries || !out_ids || !out_d2) return PKD_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Prof::begin(kProfKnn, st);
  int rc = run_knn(tree, st, queries, tree_of, nq, k, out_ids, out_d2, reinterpret_cast<int*>(status));
  Prof::end(kProfKnn, st, 0.0);
  return rc;
}

int pkd_range_count_async(const pkd_tree* tree, void* stream, const int64_t* lo, const int64_t* hi,
                          const int32_t* tree_of, int64_t nb, int64_t* out, int32_t* status) {
  if (!tree || nb < 0 || !status) return PKD_ERR_INVALID_ARG;
  if (nb == 0) return PKD_OK;
  if (!lo || !hi || !out) return PKD_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Prof::begin(kProfRange, st);
  int rc = run_range(tree, st, lo, hi, tree_of, nb, out, reinterpret_cast<int*>(status));
  Prof::end(kProfRange, st, 0.0);
  return rc;
}

int pkd_knn(const pkd_tree* tree, void* stream, const int64_t* queries, int64_t nq, int32_t k, int64_t* out_ids,
            int64_t* out_d2) {
  return pkd_knn_batch(tree, stream, queries, nullptr, nq, k, out_ids, out_d2);
}

int pkd_knn_noalloc(const pkd_tree* tree, void* stream, const int64_t* queries, int64_t nq, int32_t k,
                    int64_t* out_ids, int64_t* out_d2) {
  if (!tree || nq < 0 || k < 1 || k > 128) return PKD_ERR_INVALID_ARG;
  if (nq == 0) return PKD_OK;
  if (!queries || !out_ids || !out_d2) return PKD_ERR_INVALID_ARG;
  if (nq > PKD_KNN_NOALLOC_MAX_QUERIES) return PKD_ERR_UNSUPPORTED;
  return run_knn_static(tree, static_cast<hipStream_t>(stream), queries, nq, k, out_ids, out_d2);
}

int pkd_range_count_batch(const pkd_tree* tree, void* stream, const int64_t* lo, const int64_t* hi,
                          const int32_t* tree_of, int64_t nb, int64_t* out) {
  TraceRange tr("pkd_range_count");
  if (!tree || nb < 0) return PKD_ERR_INVALID_ARG;
  if (nb == 0) return PKD_OK;
  if (!lo || !hi || !out) return PKD_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* f = nullptr;
  PKD_TRY(flags_alloc(&f, st));
  Prof::begin(kProfRange, st);
  int rc = run_range(tree, st, lo, hi, tree_of, nb, out, f);
  Prof::end(kProfRange, st, 0.0);
  int rc2 = flags_check(f, st);
  return rc != PKD_OK ? rc : rc2;
}

int pkd_range_count(const pkd_tree* tree, void* stream, const int64_t* lo, const int64_t* hi, int64_t nb,
                    int64_t* out) {
  return pkd_range_count_batch(tree, stream, lo, hi, nullptr, nb, out);
}

int pkd_range_report_batch(const pkd_tree* tree, void* stream, const int64_t* lo, const int64_t* hi,
                           const int32_t* tree_of, int64_t nb, int64_t* offsets, int64_t* out_ids, int64_t cap,
                           int64_t* total) {
  TraceRange tr("pkd_range_report");
  if (total) *total = 0;
  if (!tree || nb < 0 || cap < 0 || !total) return PKD_ERR_INVALID_ARG;
  if (nb > 0 && (!lo || !hi)) return PKD_ERR_INVALID_ARG;
  if (!offsets) return PKD_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (nb == 0) {
    const int64_t zero = 0;
    PKD_HIP(hipMemcpyAsync(offsets, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
    PKD_HIP(hipStreamSynchronize(st));
    return PKD_OK;
  }
  return run_range_report(tree, st, lo, hi, tree_of, nb, offsets, out_ids, cap, total);
}

int pkd_range_report(const pkd_tree* tree, void* stream, const int64_t* lo, const int64_t* hi, int64_t nb,
                     int64_t* offsets, int64_t* out_ids, int64_t cap, int64_t* total) {
  return pkd_range_report_batch(tree, stream, lo, hi, nullptr, nb, offsets, out_ids, cap, total);
}

int pkd_build_batch(const pkd_params* params, const pkd_tuning* tuning, void* stream, int32_t n_trees,
                    const int64_t* coords, const int64_t* ids, const int64_t* offsets, pkd_tree** out) {
  TraceRange tr("pkd_build_batch");
  if (!out) return PKD_ERR_INVALID_ARG;
  *out = nullptr;
  Params prm;
  PKD_TRY(check_params(params, tuning, &prm));
  if (n_trees < 1 || !offsets || offsets[0] != 0) return PKD_ERR_INVALID_ARG;
  for (int32_t t = 0; t < n_trees; ++t)
    if (offsets[t + 1] < offsets[t]) return PKD_ERR_INVALID_ARG;
  const int64_t n = offsets[n_trees];
  if (n > 0 && (!coords || !ids)) return PKD_ERR_INVALID_ARG;
  if (n >= INT32_MAX || n_trees >= INT32_MAX / 2) return PKD_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  pkd_tree* T = new pkd_tree;
  T->prm = prm;
  T->n_trees = n_trees;
  int rc = alloc_points(T, st, n);
  if (rc == PKD_OK) rc = ensure_nodes(T, st, std::max<int64_t>(1024, n / 8 + n_trees));
  std::vector<Task> roots;
  if (rc == PKD_OK) {
    // every root starts as an empty leaf; non-empty trees overwrite theirs
    std::vector<Node> empty(n_trees);
    for (int32_t t = 0; t < n_trees; ++t) {
      std::memset(&empty[t], 0, sizeof(Node));
      empty[t].left = empty[t].right = -1;
      empty[t].dim = -1;
      empty[t].off = static_cast<int32_t>(offsets[t]);
      if (offsets[t + 1] > offsets[t]) {
        Task r;
        r.start = static_cast<int32_t>(offsets[t]);
        r.m = static_cast<int32_t>(offsets[t + 1] - offsets[t]);
        r.slot = t;
        r.depth = 0;
        r.buf = 2;
        r.mode = 0;
        roots.push_back(r);
      }
    }
    int e = hipMemcpyAsync(T->nodes, empty.data(), sizeof(Node) * n_trees, hipMemcpyHostToDevice, st) == hipSuccess
                ? PKD_OK : PKD_ERR_HIP;
    if (e == PKD_OK) e = hipStreamSynchronize(st) == hipSuccess ? PKD_OK : PKD_ERR_HIP;
    rc = e;
    T->node_count = n_trees;
    T->height = 0;
  }
  if (rc == PKD_OK && !roots.empty()) rc = build_tasks(T, st, roots, coords, ids, n);
  if (rc != PKD_OK) {
    release(T, st);
    (void)hipStreamSynchronize(st);
    delete T;
    return rc;
  }
  T->n = n;
  T->compact_mark = T->node_count;
  *out = T;
  return PKD_OK;
}

// ------------------------------------------------ graph build plans
namespace {
int plan_block(pkd_build_plan* G, void** p, size_t elem, int64_t count) {
  void* q = nullptr;
  PKD_TRY(dev_alloc(&q, elem * static_cast<size_t>(std::max<int64_t>(count, 1)), nullptr));
  G->blocks.push_back(q);
  *p = q;
  return PKD_OK;
}
#define PKD_PLAN_ALLOC(G, field, count) \
  plan_block((G), reinterpret_cast<void**>(&(G)->field), sizeof(*(G)->field), (count))

void plan_release(pkd_build_plan* G) {
  (void)hipDeviceSynchronize();
  for (void* q : G->blocks) dev_free(q, nullptr);
  G->blocks.clear();
  if (G->T) {
    release(G->T, nullptr);
    delete G->T;
    G->T = nullptr;
  }
  (void)hipDeviceSynchronize();
}
}  // namespace

int pkd_build_plan_create(const pkd_params* params, const pkd_tuning* tuning, int32_t n_trees, const int64_t* offsets,
                          pkd_build_plan** out) {
  TraceRange tr("pkd_build_plan_create");
  if (!out) return PKD_ERR_INVALID_ARG;
  *out = nullptr;
  Params prm;
  PKD_TRY(check_params(params, tuning, &prm));
  if (n_trees < 1 || !offsets || offsets[0] != 0) return PKD_ERR_INVALID_ARG;
  for (int32_t t = 0; t < n_trees; ++t)
    if (offsets[t + 1] < offsets[t]) return PKD_ERR_INVALID_ARG;
  const int64_t n = offsets[n_trees];
  if (n >= INT32_MAX || n_trees >= INT32_MAX / 2) return PKD_ERR_UNSUPPORTED;
  pkd_build_plan* G = new pkd_build_plan;
  G->n = n;
  G->T = new pkd_tree;
  pkd_tree* T = G->T;
  T->prm = prm;
  T->n_trees = n_trees;
  T->plan_owned = true;
  std::vector<Node> empty(n_trees);
  for (int32_t t = 0; t < n_trees; ++t) {
    std::memset(&empty[t], 0, sizeof(Node));
    empty[t].left = empty[t].right = -1;
    empty[t].dim = -1;
    empty[t].off = static_cast<int32_t>(offsets[t]);
    if (offsets[t + 1] > offsets[t]) {
      Task r;
      r.start = static_cast<int32_t>(offsets[t]);
      r.m = static_cast<int32_t>(offsets[t + 1] - offsets[t]);
      r.slot = t;
      r.depth = 0;
      r.buf = 2;
      r.mode = 0;
      G->roots.push_back(r);
    }
  }
  const int D = prm.D;
  const int64_t NB = int64_t{1} << prm.lambda;
  int rc = alloc_points(T, nullptr, std::max<int64_t>(n, 1));
  if (rc == PKD_OK) rc = ensure_c32(T, nullptr);
  if (rc == PKD_OK) rc = plan_size(G);   // also sizes the node array
  if (rc == PKD_OK)
    rc = hipMemcpy(T->nodes, empty.data(), sizeof(Node) * n_trees, hipMemcpyHostToDevice) == hipSuccess
             ? PKD_OK : PKD_ERR_HIP;
  const int64_t nb = (G->fin_max + 2047) / 2048 + 2;
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, roots_d, static_cast<int64_t>(G->roots.size()));
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, front, G->front_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, next, G->front_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, sieve, G->ns_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, fin, G->fin_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, ctr, 64);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, rx, G->ns_max * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, tile_off, G->ns_max + 1);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, chunk_off, G->ns_max + 1);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, tot, 2);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, rdim, G->ns_max * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, ext, G->ns_max * 2 * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, mode, G->ns_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, shift, G->ns_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, shift_fix, G->ns_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, rootext, G->ns_max);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, cand_key, G->cand_len);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, cand_pos, G->cand_len);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, cand_cnt, G->ns_max * 32);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, A, G->ntiles_max * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, B, G->ntiles_max * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, S, G->nchunks_max * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, bsize, G->ns_max * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, bstart, G->ns_max * NB);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, R, G->fin_max + 1);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, res_off, G->fin_max + 1);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, bsum, nb);
  if (rc == PKD_OK) rc = PKD_PLAN_ALLOC(G, lists, 8 * G->fin_max);
  if (rc == PKD_OK && !G->roots.empty())
    rc = hipMemcpy(G->roots_d, G->roots.data(), sizeof(Task) * G->roots.size(), hipMemcpyHostToDevice) == hipSuccess
             ? PKD_OK : PKD_ERR_HIP;
  if (rc == PKD_OK) rc = hipDeviceSynchronize() == hipSuccess ? PKD_OK : PKD_ERR_HIP;
  (void)D;
  T->n = n;                    // fixed for the plan: the trees' sizes
  T->node_count = n_trees;     // the roots, until the first build is finished
  T->compact_mark = n_trees;
  if (rc != PKD_OK) {
    plan_release(G);
    delete G;
    return rc;
  }
  *out = G;
  return PKD_OK;
}

int pkd_build_plan_enqueue(pkd_build_plan* plan, void* stream, const int64_t* coords, const int64_t* ids) {
  TraceRange tr("pkd_build_plan_enqueue");
  if (!plan) return PKD_ERR_INVALID_ARG;
  if (plan->n > 0 && (!coords || !ids)) return PKD_ERR_INVALID_ARG;
  plan->in_c = coords;
  plan->in_id = ids;
  return plan_enqueue(plan, static_cast<hipStream_t>(stream));
}

int pkd_build_plan_finish(pkd_build_plan* plan, void* stream, int32_t* redone) {
  TraceRange tr("pkd_build_plan_finish");
  if (redone) *redone = 0;
  if (!plan) return PKD_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  pkd_tree* T = plan->T;
  int h[8] = {0};
  PKD_HIP(hipMemcpyAsync(h, plan->ctr, sizeof(h), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));
  const int flags = h[4];
  if (flags & kErrRange) {
    T->node_count = T->n_trees;   // no tree: the roots only (as created)
    return PKD_ERR_RANGE;
  }
  // any other flag but an internal error alone marks a case the sized
  // launches do not cover (the rounds after it may then have found empty
  // buckets too): the usual build redoes it and reports its own errors
  if (flags == kErrInternal) {
    T->node_count = T->n_trees;
    return PKD_ERR_INTERNAL;
  }
  if (flags) {
    // a case the sized launches do not cover: build the usual way, then copy
    // the result into the plan's arrays (their addresses are the captured ones)
    pkd_tree* Z = nullptr;
    pkd_params p;
    pkd_default_params(&p, T->prm.D);
    p.lambda = T->prm.lambda;
    p.leaf_size = T->prm.phi;
    p.oversample = T->prm.sigma;
    p.alpha_num = T->prm.alpha_num;
    p.alpha_den = T->prm.alpha_den;
    p.seed = T->prm.seed;
    pkd_tuning tu;
    pkd_default_tuning(&tu);
    tu.tile_points = T->prm.tile;
    tu.cand_shift_bias = T->prm.cand_bias;
    tu.update_events = T->prm.update_events;
    std::vector<int64_t> offs(static_cast<size_t>(T->n_trees) + 1, 0);
    {
      // offsets from the roots (empty trees hold no task)
      std::vector<int64_t> sizes(T->n_trees, 0);
      for (const Task& r : plan->roots) sizes[r.slot] = r.m;
      for (int32_t t = 0; t < T->n_trees; ++t) offs[t + 1] = offs[t] + sizes[t];
    }
    PKD_TRY(pkd_build_batch(&p, &tu, stream, T->n_trees, plan->in_c, plan->in_id, offs.data(), &Z));
    int rc = PKD_OK;
    if (Z->node_count > T->node_cap) rc = PKD_ERR_CAPACITY;
    const int D = T->prm.D;
    if (rc == PKD_OK && Z->node_count > 0)
      rc = hipMemcpyAsync(T->nodes, Z->nodes, sizeof(Node) * Z->node_count, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? PKD_OK : PKD_ERR_HIP;
    for (int d = 0; d <= D && rc == PKD_OK && plan->n > 0; ++d)
      rc = hipMemcpyAsync(T->buf[T->cur] + static_cast<int64_t>(d) * T->cap, Z->buf[Z->cur] + static_cast<int64_t>(d) * Z->cap,
                          sizeof(int64_t) * plan->n, hipMemcpyDeviceToDevice, st) == hipSuccess ? PKD_OK : PKD_ERR_HIP;
    if (rc == PKD_OK && plan->n > 0)
      rc = hipMemcpyAsync(T->c32, Z->c32, sizeof(int32_t) * D * plan->n, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? PKD_OK : PKD_ERR_HIP;
    if (rc == PKD_OK) {
      T->node_count = Z->node_count;
      T->height = Z->height;
    }
    if (rc == PKD_OK) rc = hipStreamSynchronize(st) == hipSuccess ? PKD_OK : PKD_ERR_HIP;
    pkd_free(Z);
    if (rc != PKD_OK) return rc;
    if (redone) *redone = 1;
  } else {
    T->node_count = h[3];
    T->height = h[6];
  }
  T->compact_mark = T->node_count;
  return PKD_OK;
}

int pkd_build_plan_tree(pkd_build_plan* plan, pkd_tree** tree) {
  if (!plan || !tree) return PKD_ERR_INVALID_ARG;
  *tree = plan->T;
  return PKD_OK;
}

void pkd_build_plan_free(pkd_build_plan* plan) {
  if (!plan) return;
  plan_release(plan);
  delete plan;
}

int pkd_num_trees(const pkd_tree* tree, int32_t* n_trees) {
  if (!tree || !n_trees) return PKD_ERR_INVALID_ARG;
  *n_trees = tree->n_trees;
  return PKD_OK;
}

int pkd_batch_insert_tree(pkd_tree* tree, int32_t t, void* stream, const int64_t* coords, const int64_t* ids,
                          int64_t m) {
  TraceRange tr("pkd_batch_insert");
  if (!tree || m < 0 || t < 0 || t >= tree->n_trees || tree->plan_owned) return PKD_ERR_INVALID_ARG;
  if (m == 0) return PKD_OK;
  if (!coords || !ids) return PKD_ERR_INVALID_ARG;
  if (tree->n + m >= INT32_MAX) return PKD_ERR_UNSUPPORTED;
  return run_insert(tree, t, static_cast<hipStream_t>(stream), coords, ids, m);
}

int pkd_batch_insert(pkd_tree* tree, void* stream, const int64_t* coords, const int64_t* ids, int64_t m) {
  return pkd_batch_insert_tree(tree, 0, stream, coords, ids, m);
}

int pkd_batch_delete_tree(pkd_tree* tree, int32_t t, void* stream, const int64_t* coords, const int64_t* ids,
                          int64_t m, int64_t* n_deleted) {
  TraceRange tr("pkd_batch_delete");
  if (n_deleted) *n_deleted = 0;
  if (!tree || m < 0 || t < 0 || t >= tree->n_trees || tree->plan_owned) return PKD_ERR_INVALID_ARG;
  if (m == 0) return PKD_OK;
  if (!coords || !ids) return PKD_ERR_INVALID_ARG;
  if (m >= INT32_MAX) return PKD_ERR_UNSUPPORTED;
  int64_t removed = 0;
  int rc = run_delete(tree, t, static_cast<hipStream_t>(stream), coords, ids, m, &removed);
  if (rc == PKD_OK && n_deleted) *n_deleted = removed;
  return rc;
}

int pkd_batch_delete(pkd_tree* tree, void* stream, const int64_t* coords, const int64_t* ids, int64_t m,
                     int64_t* n_deleted) {
  return pkd_batch_delete_tree(tree, 0, stream, coords, ids, m, n_deleted);
}

int pkd_size(const pkd_tree* tree, int64_t* n) {
  if (!tree || !n) return PKD_ERR_INVALID_ARG;
  *n = tree->n;
  return PKD_OK;
}

int pkd_height(const pkd_tree* tree, int32_t* h) {
  if (!tree || !h) return PKD_ERR_INVALID_ARG;
  *h = tree->height;
  return PKD_OK;
}

namespace {
int copy_host(const pkd_tree* T, std::vector<Node>& nodes, std::vector<int64_t>& pts) {
  nodes.resize(T->node_count);
  const int D = T->prm.D;
  pts.resize(static_cast<size_t>(D + 1) * T->n);
  PKD_HIP(hipDeviceSynchronize());
  PKD_HIP(hipMemcpy(nodes.data(), T->nodes, sizeof(Node) * T->node_count, hipMemcpyDeviceToHost));
  for (int d = 0; d <= D; ++d)
    if (T->n > 0)
      PKD_HIP(hipMemcpy(pts.data() + static_cast<size_t>(d) * T->n, T->buf[T->cur] + static_cast<int64_t>(d) * T->cap,
                        sizeof(int64_t) * T->n, hipMemcpyDeviceToHost));
  return PKD_OK;
}

// Pre-order walk from a root; returns the node count or -1 when the stored
// links do not form a tree.
int64_t walk(const std::vector<Node>& nodes, int32_t root, std::vector<int32_t>* order) {
  std::vector<int32_t> stack{root};
  int64_t count = 0;
  while (!stack.empty()) {
    int32_t t = stack.back();
    stack.pop_back();
    if (t < 0 || t >= static_cast<int32_t>(nodes.size()) || count > static_cast<int64_t>(nodes.size())) return -1;
    ++count;
    if (order) order->push_back(t);
    if (nodes[t].left >= 0) {
      stack.push_back(nodes[t].right);
      stack.push_back(nodes[t].left);
    }
  }
  return count;
}
}  // namespace

int pkd_export_tree_sizes(const pkd_tree* tree, int32_t t, int64_t* num_nodes, int64_t* n) {
  if (!tree || !num_nodes || !n || t < 0 || t >= tree->n_trees) return PKD_ERR_INVALID_ARG;
  std::vector<Node> nodes(tree->node_count);
  PKD_HIP(hipDeviceSynchronize());
  PKD_HIP(hipMemcpy(nodes.data(), tree->nodes, sizeof(Node) * tree->node_count, hipMemcpyDeviceToHost));
  int64_t c = walk(nodes, t, nullptr);
  if (c < 0) return PKD_ERR_INTERNAL;
  *num_nodes = c;
  *n = nodes[t].size;
  return PKD_OK;
}

int pkd_export_sizes(const pkd_tree* tree, int64_t* num_nodes, int64_t* n) {
  return pkd_export_tree_sizes(tree, 0, num_nodes, n);
}

int pkd_export_tree(const pkd_tree* tree, int32_t t, int64_t* rows, int64_t* leaf_ids, int64_t* leaf_coords,
                    int32_t* depths) {
  if (!tree || t < 0 || t >= tree->n_trees) return PKD_ERR_INVALID_ARG;
  std::vector<Node> nodes;
  std::vector<int64_t> pts;
  PKD_TRY(copy_host(tree, nodes, pts));
  std::vector<int32_t> order;
  if (walk(nodes, t, &order) < 0) return PKD_ERR_INTERNAL;
  const int D = tree->prm.D;
  const int64_t N = tree->n;          // points of all trees (host copy layout)
  const int64_t n = nodes[t].size;    // points of tree t
  int64_t at = 0;
  std::vector<int64_t> idx;
  for (size_t r = 0; r < order.size(); ++r) {
    const Node& nd = nodes[order[r]];
    const bool leaf = nd.left < 0;
    if (rows) {
      rows[4 * r + 0] = leaf ? 1 : 0;
      rows[4 * r + 1] = leaf ? -1 : nd.dim;
      rows[4 * r + 2] = leaf ? 0 : nd.x;
      rows[4 * r + 3] = nd.size;
    }
    if (depths) depths[r] = nd.depth;
    if (!leaf) continue;
    if (nd.off < 0 || static_cast<int64_t>(nd.off) + nd.size > N || at + nd.size > n) return PKD_ERR_INTERNAL;
    idx.resize(nd.size);
    for (int32_t i = 0; i < nd.size; ++i) idx[i] = nd.off + i;
    const int64_t* id = pts.data() + static_cast<size_t>(D) * N;
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return id[a] < id[b]; });
    for (int32_t i = 0; i < nd.size; ++i) {
      if (leaf_ids) leaf_ids[at + i] = id[idx[i]];
      if (leaf_coords)
        for (int d = 0; d < D; ++d) leaf_coords[static_cast<int64_t>(d) * n + at + i] = pts[static_cast<size_t>(d) * N + idx[i]];
    }
    at += nd.size;
  }
  return at == n ? PKD_OK : PKD_ERR_INTERNAL;
}

int pkd_export(const pkd_tree* tree, int64_t* rows, int64_t* leaf_ids, int64_t* leaf_coords, int32_t* depths) {
  return pkd_export_tree(tree, 0, rows, leaf_ids, leaf_coords, depths);
}

int pkd_profile_enable(int32_t on) {
  Prof::flush();
  g_prof.on = on != 0;
  for (int k = 0; k < kProfN; ++k) {
    g_prof.launches[k] = 0;
    g_prof.ms[k] = 0;
    g_prof.bytes[k] = 0;
  }
  return PKD_OK;
}

int pkd_profile_get(int32_t kernel, int64_t* launches, double* total_ms, double* alg_bytes) {
  if (kernel < 0 || kernel >= kProfN) return PKD_ERR_INVALID_ARG;
  Prof::flush();
  if (launches) *launches = g_prof.launches[kernel];
  if (total_ms) *total_ms = g_prof.ms[kernel];
  if (alg_bytes) *alg_bytes = g_prof.bytes[kernel];
  return PKD_OK;
}

void pkd_free(pkd_tree* tree) {
  if (!tree || tree->plan_owned) return;   // a plan's tree goes with its plan
  (void)hipDeviceSynchronize();
  release(tree, nullptr);
  (void)hipDeviceSynchronize();
  delete tree;
}

int pkd_free_async(pkd_tree* tree, void* stream) {
  if (!tree) return PKD_OK;
  if (tree->plan_owned) return PKD_ERR_INVALID_ARG;
  // every block goes back with an event on `stream`: its next user waits for
  // the work enqueued on `stream` before this call
  release(tree, static_cast<hipStream_t>(stream));
  delete tree;
  return PKD_OK;
}

int pkd_set_allocator(const pkd_allocator* a) {
  if (a && (!a->alloc || !a->free)) return PKD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  g_ext_on = a != nullptr;
  if (a) g_ext = *a;
  return PKD_OK;
}

int pkd_set_bbox(pkd_tree* tree, void* stream, int32_t on) {
  if (!tree || tree->plan_owned) return PKD_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!on) {
    tree->bbox_on = false;
    dev_free(tree->bbox, st);
    tree->bbox = nullptr;
    tree->bbox_cap = 0;
    return PKD_OK;
  }
  PKD_TRY(compute_bbox(tree, st));
  tree->bbox_on = true;
  return PKD_OK;
}

int pkd_export_bbox(const pkd_tree* tree, int32_t t, int32_t* boxes) {
  if (!tree || !boxes || t < 0 || t >= tree->n_trees) return PKD_ERR_INVALID_ARG;
  if (!tree->bbox_on) return PKD_ERR_INVALID_ARG;
  const int D = tree->prm.D;
  std::vector<Node> nodes(tree->node_count);
  std::vector<int32_t> bb(static_cast<size_t>(tree->node_count) * 2 * D);
  PKD_HIP(hipDeviceSynchronize());
  PKD_HIP(hipMemcpy(nodes.data(), tree->nodes, sizeof(Node) * tree->node_count, hipMemcpyDeviceToHost));
  PKD_HIP(hipMemcpy(bb.data(), tree->bbox, sizeof(int32_t) * bb.size(), hipMemcpyDeviceToHost));
  std::vector<int32_t> order;
  if (walk(nodes, t, &order) < 0) return PKD_ERR_INTERNAL;
  for (size_t r = 0; r < order.size(); ++r)
    for (int c = 0; c < 2 * D; ++c) boxes[r * 2 * D + c] = bb[static_cast<size_t>(order[r]) * 2 * D + c];
  return PKD_OK;
}

int pkd_update_stats(const pkd_tree* tree, int64_t* regions, int64_t* points) {
  if (!tree) return PKD_ERR_INVALID_ARG;
  if (regions) *regions = tree->last_regions;
  if (points) *points = tree->last_rebuilt;
  return PKD_OK;
}

int pkd_node_slots(const pkd_tree* tree, int64_t* slots) {
  if (!tree || !slots) return PKD_ERR_INVALID_ARG;
  *slots = tree->node_count;
  return PKD_OK;
}

const char* pkd_strerror(int code) {
  switch (code) {
    case PKD_OK: return "ok";
    case PKD_ERR_INVALID_ARG: return "invalid argument";
    case PKD_ERR_RANGE: return "coordinate outside [0, 2^30)";
    case PKD_ERR_UNSUPPORTED: return "unsupported size or dimension";
    case PKD_ERR_OOM: return "device out of memory";
    case PKD_ERR_HIP: return "HIP runtime error";
    case PKD_ERR_CAPACITY: return "traversal stack capacity exceeded";
    case PKD_ERR_INTERNAL: return "internal consistency check failed";
  }
  return "unknown error";
}

}  // extern "C"
