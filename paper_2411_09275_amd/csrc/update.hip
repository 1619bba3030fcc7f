// Batch updates on the GPU: BatchInsert (Algorithm 2, Section 4.1) and
// BatchDelete (Section 4.2).
//
//   route     the batch is sieved through skeletons fetched from the tree (the
//             top lambda levels below each routing node), one sieve round per
//             lambda levels, with the build's count/scan/scatter kernels, until
//             every batch point sits in the slice of the leaf it belongs to;
//             the batch ends up in the tree's in-order.
//   match     (delete) each entry finds the stored point of its leaf with the
//             same id and coordinates; absent entries drop out, and of the
//             entries naming one point the first claims it.
//   decide    the rounds are replayed top-down with exact counts (inserted
//             points, or points actually removed): a touched node that stays
//             alpha-balanced keeps its splitter and takes its new size; the
//             topmost one that does not becomes a rebuild region and nothing
//             below it is visited; an inserted-into leaf is rebuilt.
//   relayout  the tree keeps its points packed in in-order: the regions sorted
//             by old end (with the batch points each adds) and the sorted
//             removed positions give every surviving point and node its new
//             offset (a batch dense in the tree uses per-point arrays
//             instead); old points, batch points and survivors move in one
//             pass.
//   rebuild   all regions are rebuilt by one segmented Build (Algorithm 1),
//             each at the depth of the node it replaces.
#include <algorithm>
#include <cstring>

#include "pkd_internal.h"

namespace pkd {

namespace {

constexpr int kUBlock = 256;

struct Res {      // a routed slice of the batch that ends at a leaf
  int32_t node, start, count, buf;
};

struct Region {   // a node to rebuild (old range [a, b), batch slice [s, e))
  int32_t node, depth, a, b, s, e, new_start, new_size;
};

template <int D>
__global__ void k_validate(const int64_t* coords, int64_t m, int* flags) {
  bool bad = false;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    for (int d = 0; d < D; ++d) bad |= static_cast<uint64_t>(coords[d * m + i]) >= static_cast<uint64_t>(coord_limit(D));
  if (bad) atomicOr(flags, kErrRange);
}

// Kernels that work per routing subproblem give each subproblem one wave and
// put several waves in a workgroup: a late routing round can hold hundreds of
// thousands of subproblems with a handful of points each, and one workgroup
// per subproblem would be bound by workgroup dispatch.
constexpr int kWaves = 4;

// Skeleton of the top lambda levels below each routing node, in heap order:
// hn[v] is the tree node at heap position v (-1 below a leaf); interior
// positions above level lambda route by their splitter, the rest send left.
__global__ void __launch_bounds__(64 * kWaves) k_fetch_skeleton(const Task* tasks, int ns, const Node* nodes,
                                                                int lambda, int64_t* rx, uint8_t* rdim,
                                                                int32_t* hn_out) {
  const int NB = 1 << lambda, nheap = 2 << lambda;
  __shared__ int32_t hn_w[kWaves][2 << kMaxLambda];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sig = blockIdx.x * kWaves + w;
  const bool active = sig < ns;
  int32_t* hn = hn_w[w];
  for (int v = lane; v < nheap; v += 64) hn[v] = -1;
  __syncthreads();
  if (active && lane == 0) hn[1] = tasks[sig].slot;
  __syncthreads();
  for (int l = 0; l < lambda; ++l) {
    if (active) {
      for (int v = (1 << l) + lane; v < (2 << l); v += 64) {
        const int32_t u = hn[v];
        int64_t x = kAllLeft;
        uint8_t d = 0;
        if (u >= 0) {
          const Node nd = nodes[u];
          if (nd.left >= 0) {
            x = nd.x;
            d = static_cast<uint8_t>(nd.dim);
            hn[2 * v] = nd.left;
            hn[2 * v + 1] = nd.right;
          }
        }
        rx[static_cast<int64_t>(sig) * NB + v] = x;
        rdim[static_cast<int64_t>(sig) * NB + v] = d;
      }
    }
    __syncthreads();
  }
  if (active)
    for (int v = lane; v < nheap; v += 64) hn_out[static_cast<int64_t>(sig) * nheap + v] = hn[v];
}

// Buckets that end at a leaf are resolved; buckets at an interior node of
// level lambda become the next round's routing tasks.  Two passes: count the
// outcomes per subproblem, then (after an exclusive scan over subproblems)
// write them at fixed places, so there is no contended counter and the order
// of tasks and resolved slices follows the subproblems.
struct Outcome {
  int32_t u, start, size;
  int level;
  bool go_on, leaf_end;
};

__device__ inline Outcome route_outcome(const Node* nodes, int lambda, const int32_t* hn, const int32_t* bsize_t,
                                        const int32_t* bstart_t, int v) {
  const int NB = 1 << lambda, nheap = 2 << lambda;
  Outcome o{-1, 0, 0, 0, false, false};
  if (v < 1 || v >= nheap) return o;
  o.u = hn[v];
  if (o.u < 0) return o;
  o.level = 31 - __clz(v);
  // external: the skeleton's last level, or a leaf above it (whose children
  // the fetched skeleton left empty)
  if (o.level == lambda || hn[2 * v] < 0) {
    const int label = (v << (lambda - o.level)) - NB;
    o.size = bsize_t[label];
    o.start = bstart_t[label];
    if (o.size > 0) {
      o.leaf_end = o.level < lambda || nodes[o.u].left < 0;
      o.go_on = !o.leaf_end;
    }
  }
  return o;
}

__global__ void __launch_bounds__(64 * kWaves) k_route_count(const Task* tasks, int ns, const Node* nodes, int lambda,
                                                             const int32_t* hn_all, const int32_t* bsize,
                                                             const int32_t* bstart, int32_t* n_go, int32_t* n_leaf) {
  const int NB = 1 << lambda, nheap = 2 << lambda;
  const int lane = threadIdx.x & 63;
  const int sig = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (sig >= ns) return;
  const int32_t* hn = hn_all + static_cast<int64_t>(sig) * nheap;
  int go = 0, leaf = 0;
  for (int base = 0; base < nheap; base += 64) {
    const Outcome o = route_outcome(nodes, lambda, hn, bsize + static_cast<int64_t>(sig) * NB,
                                    bstart + static_cast<int64_t>(sig) * NB, base + lane);
    go += __popcll(__ballot(o.go_on));
    leaf += __popcll(__ballot(o.leaf_end));
  }
  if (lane == 0) {
    n_go[sig] = go;
    n_leaf[sig] = leaf;
  }
  (void)tasks;
}

__global__ void __launch_bounds__(64 * kWaves) k_route_emit(const Task* tasks, int ns, const Node* nodes, int lambda,
                                                            const int32_t* hn_all, const int32_t* bsize,
                                                            const int32_t* bstart, int dst, const int32_t* off_go,
                                                            const int32_t* off_leaf, int res_base, Task* next,
                                                            int32_t* child_idx, Res* res) {
  const int NB = 1 << lambda, nheap = 2 << lambda;
  const int lane = threadIdx.x & 63;
  const int sig = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (sig >= ns) return;
  const unsigned long long lt = (1ULL << lane) - 1;
  const Task q = tasks[sig];
  const int32_t* hn = hn_all + static_cast<int64_t>(sig) * nheap;
  int go_at = off_go[sig], leaf_at = res_base + off_leaf[sig];
  for (int base = 0; base < nheap; base += 64) {
    const int v = base + lane;
    const Outcome o = route_outcome(nodes, lambda, hn, bsize + static_cast<int64_t>(sig) * NB,
                                    bstart + static_cast<int64_t>(sig) * NB, v);
    const unsigned long long mg = __ballot(o.go_on);
    const unsigned long long ml = __ballot(o.leaf_end);
    if (v >= 1 && v < nheap) {
      int32_t child = -1;
      if (o.go_on) {
        const int at = go_at + __popcll(mg & lt);
        Task c;
        c.start = o.start;
        c.m = o.size;
        c.slot = o.u;
        c.depth = static_cast<int16_t>(q.depth + o.level);
        c.buf = static_cast<int8_t>(dst);
        c.mode = 0;
        next[at] = c;
        child = at;
      }
      child_idx[static_cast<int64_t>(sig) * nheap + v] = child;
      if (o.leaf_end) res[leaf_at + __popcll(ml & lt)] = Res{o.u, o.start, o.size, dst};
    }
    go_at += __popcll(mg);
    leaf_at += __popcll(ml);
  }
}

// ---- routing rounds with many small subproblems: one stable radix sort of
// the batch by (subproblem start, bucket label) gives the order the tiled
// sieve gives (stable by position inside each subproblem) without a tile,
// a scan and a workgroup per subproblem.
__global__ void __launch_bounds__(64 * kWaves) k_task_fill(const Task* tasks, int ns, int32_t* task_of) {
  const int sig = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (sig >= ns) return;
  const Task t = tasks[sig];
  for (int i = threadIdx.x & 63; i < t.m; i += 64) task_of[t.start + i] = sig;
}

template <int D>
__global__ void k_route_keys(const int64_t* X, int64_t xcap, int64_t m, const int32_t* task_of, const Task* tasks,
                             const int64_t* rx, const uint8_t* rdim, int lambda, uint64_t* key, uint32_t* val) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (p >= m) return;
  const int32_t t = task_of[p];
  uint64_t k;
  if (t < 0) {
    k = static_cast<uint64_t>(p) << lambda;   // not routed this round: keeps its own place in the order
  } else {
    const int NB = 1 << lambda;
    const int64_t* sx = rx + static_cast<int64_t>(t) * NB;
    const uint8_t* sd = rdim + static_cast<int64_t>(t) * NB;
    int64_t c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) c[d] = X[d * xcap + p];
    int v = 1;
    for (int l = 0; l < lambda; ++l) {
      const int d = sd[v];
      const int64_t x = sx[v];
      int ge = 0;
#pragma unroll
      for (int e = 0; e < D; ++e) ge |= (d == e) & (c[e] >= x);
      v = 2 * v + ge;
    }
    k = (static_cast<uint64_t>(tasks[t].start) << lambda) | static_cast<uint64_t>(v - NB);
  }
  key[p] = k;
  val[p] = static_cast<uint32_t>(p);
}

__device__ inline int64_t lower_bound_u64(const uint64_t* a, int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Sorted item i of a subproblem starting at P goes to P + (i - first item of
// that subproblem); the last item of each (subproblem, bucket) run records the
// bucket size.
template <int D>
__global__ void k_route_place(const uint64_t* ks, const uint32_t* vs, int64_t m, const int32_t* task_of, int lambda,
                              Bufs wb, int src, int dst, int32_t* bsize) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= m) return;
  const uint64_t key = ks[i];
  const uint32_t p = vs[i];
  const int32_t t = task_of[p];
  if (t < 0) return;
  const uint64_t P = key >> lambda;
  const int64_t out = static_cast<int64_t>(P) + (i - lower_bound_u64(ks, m, P << lambda));
#pragma unroll
  for (int d = 0; d < D; ++d) wb.c[dst][d * wb.cap[dst] + out] = wb.c[src][d * wb.cap[src] + p];
  wb.id[dst][out] = wb.id[src][p];
  if (i == m - 1 || ks[i + 1] != key) {
    const int64_t run = lower_bound_u64(ks, m, key);
    bsize[static_cast<int64_t>(t) * (1 << lambda) + static_cast<int>(key & ((1u << lambda) - 1))] =
        static_cast<int32_t>(i - run + 1);
  }
}

__global__ void __launch_bounds__(64 * kWaves) k_route_bstart(const Task* tasks, int ns, int lambda,
                                                              const int32_t* bsize, int32_t* bstart) {
  const int sig = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (sig >= ns) return;
  const int lane = threadIdx.x & 63;
  const int NB = 1 << lambda;
  // exclusive scan of the bucket sizes from the subproblem's start
  int32_t carry = tasks[sig].start;
  for (int base = 0; base < NB; base += 64) {
    const int j = base + lane;
    const int32_t x = j < NB ? bsize[static_cast<int64_t>(sig) * NB + j] : 0;
    int32_t incl = x;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (j < NB) bstart[static_cast<int64_t>(sig) * NB + j] = carry + incl - x;
    carry += __shfl(incl, 63);
  }
}

// Copy every resolved slice into one buffer (same positions) and record the
// leaf of each batch position.
__global__ void __launch_bounds__(64 * kWaves) k_gather(const Res* res, int nres, int D, Bufs wb, int64_t* out,
                                                        int64_t m, int32_t* leaf_of) {
  const int rid = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (rid >= nres) return;
  const Res r = res[rid];
  for (int i = threadIdx.x & 63; i < r.count; i += 64) {
    const int64_t p = r.start + i;
    for (int d = 0; d < D; ++d) out[d * m + p] = wb.c[r.buf][d * wb.cap[r.buf] + p];
    out[D * m + p] = wb.id[r.buf][p];
    leaf_of[p] = r.node;
  }
}

// Delete: each batch entry looks in its leaf for the stored point with the
// same id and coordinates and notes its position (n when there is none).
template <int D>
__global__ void k_match(const int64_t* batch, int64_t m, const int32_t* leaf_of, const Node* nodes, const int64_t* X,
                        int64_t cap, int64_t n, uint64_t* pos, uint32_t* entry) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (p >= m) return;
  int64_t c[D];
  for (int d = 0; d < D; ++d) c[d] = batch[d * m + p];
  const int64_t id = batch[D * m + p];
  const Node nd = nodes[leaf_of[p]];
  const int64_t* ids = X + static_cast<int64_t>(D) * cap;
  int64_t at = n;
  for (int64_t i = nd.off; i < static_cast<int64_t>(nd.off) + nd.size; ++i) {
    if (ids[i] != id) continue;
    bool same = true;
    for (int d = 0; d < D; ++d) same &= X[d * cap + i] == c[d];
    if (!same) continue;
    at = i;
    break;
  }
  pos[p] = static_cast<uint64_t>(at);
  entry[p] = static_cast<uint32_t>(p);
}

// After the positions are sorted: the first entry of each matched position
// claims it (repeated entries of one point drop out), weight 1 for the claim.
__global__ void k_claim(const uint64_t* pos, const uint32_t* entry, int64_t m, int64_t n, int32_t* claim,
                        int32_t* weight) {
  for (int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; j < m;
       j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int32_t c = pos[j] < static_cast<uint64_t>(n) && (j == 0 || pos[j] != pos[j - 1]) ? 1 : 0;
    claim[j] = c;
    weight[entry[j]] = c;
  }
}

// The claimed positions, ascending and without repeats.
__global__ void k_removed_list(const uint64_t* pos, const int32_t* claim, const int32_t* at, int64_t m,
                               uint64_t* removed) {
  for (int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; j < m;
       j += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (claim[j]) removed[at[j]] = pos[j];
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = v;
}

// Replay of one routing round, top-down, with exact counts.  cnt(v) is the
// weight of the batch slice below heap position v (1 per inserted point, 1 per
// point actually removed); a killed task lies below a region.
// The decisions run twice per round: apply = 0 only counts the regions and the
// recorded sizes each subproblem adds (rcount[sig], scount[sig]) and writes
// nothing else; after exclusive scans (roff, soff), apply = 1 makes the same
// decisions and writes subproblem sig's regions at n_regions + roff[sig] and
// its sizes at n_sizes + soff[sig] onwards, in a fixed order.  (A counter
// shared by all waves serialized tens of millions of atomics when a batch
// touched millions of nodes.)
__host__ __device__ inline size_t decide_lds_per_wave(int lambda) {
  return (static_cast<size_t>(2 << lambda) * (7 * sizeof(int32_t) + 1) + 15) & ~size_t{15};
}

__global__ void __launch_bounds__(64 * kWaves) k_decide(const Task* tasks, int ns, int lambda, const int32_t* hn_all,
                                                        const int32_t* bsize, const int32_t* bstart,
                                                        const int32_t* child_idx, const int8_t* killed,
                                                        int8_t* killed_next, const int32_t* M, const Node* nodes,
                                                        int64_t an, int64_t ad, int insert, Region* regions,
                                                        const int* n_regions, int apply, int32_t* rcount,
                                                        const int32_t* roff, int2* sizes, const int* n_sizes,
                                                        int32_t* scount, const int32_t* soff) {
  const int NB = 1 << lambda, nheap = 2 << lambda;
  // per wave: cnt, s0, sz, and the touched nodes' size, offset, depth and
  // left child's size [nheap] int32, alive [nheap] bytes (dynamic LDS, sized
  // for this lambda)
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sig = blockIdx.x * kWaves + w;
  const bool active = sig < ns && !killed[sig];
  if (!active) {
    // every wave works in its own LDS slice and synchronizes only itself
    if (!apply && lane == 0 && sig < ns) rcount[sig] = scount[sig] = 0;
    return;
  }
  unsigned char* mine = smem + static_cast<size_t>(w) * decide_lds_per_wave(lambda);
  int32_t* cnt = reinterpret_cast<int32_t*>(mine);
  int32_t* s0 = cnt + nheap;
  int32_t* sz = s0 + nheap;
  int32_t* t_size = sz + nheap;
  int32_t* t_off = t_size + nheap;
  int32_t* t_depth = t_off + nheap;
  int32_t* t_lsize = t_depth + nheap;   // left child's size; -1: a leaf
  uint8_t* alive = reinterpret_cast<uint8_t*>(t_lsize + nheap);
  const int32_t* hn = hn_all + static_cast<int64_t>(sig) * nheap;
  for (int j = lane; j < NB; j += 64) {
    const int32_t st = bstart[static_cast<int64_t>(sig) * NB + j];
    const int32_t n = bsize[static_cast<int64_t>(sig) * NB + j];
    s0[NB + j] = st;
    sz[NB + j] = n;
    cnt[NB + j] = M[st + n] - M[st];
  }
  for (int v = lane; v < nheap; v += 64) alive[v] = v == 1 ? 1 : 0;
  wave_sync();
  for (int l = lambda - 1; l >= 0; --l) {
    for (int v = (1 << l) + lane; v < (2 << l); v += 64) {
      cnt[v] = cnt[2 * v] + cnt[2 * v + 1];
      sz[v] = sz[2 * v] + sz[2 * v + 1];
      s0[v] = s0[2 * v];
    }
    wave_sync();
  }
  // the records of every node the batch reaches, loaded together (the walk
  // below would otherwise wait on two dependent loads per level)
  for (int v = 1 + lane; v < nheap; v += 64) {
    const int32_t u = hn[v];
    if (u >= 0 && cnt[v] != 0) {
      const Node nd = nodes[u];
      t_size[v] = nd.size;
      t_off[v] = nd.off;
      t_depth[v] = nd.depth;
      const int lev = 31 - __clz(v);
      t_lsize[v] = nd.left < 0 ? -1 : (lev < lambda ? nodes[nd.left].size : 0);
    }
  }
  wave_sync();
  int added = 0;   // regions this wave has added so far (uniform)
  int sized = 0;   // sizes this wave has recorded so far (uniform)
  const int32_t base = apply ? *n_regions + roff[sig] : 0;
  const int32_t sbase = apply ? *n_sizes + soff[sig] : 0;
  for (int l = 0; l <= lambda; ++l) {
    {
      // a level without a live node ends the walk: nodes below it are
      // reached only through live ones
      bool any = false;
      for (int v = (1 << l) + lane; v < (2 << l); v += 64) any |= alive[v] != 0;
      if (__ballot(any) == 0) break;
      // every lane runs every step (the ballot keeps `added` uniform)
      for (int v0 = 1 << l; v0 < (2 << l); v0 += 64) {
        const int v = v0 + lane;
        const bool in = v < (2 << l);
        const int32_t u = in ? hn[v] : -1;
        bool add = false;   // node u becomes a region to rebuild
        bool setsz = false; // node u keeps its place and takes size newsz
        int32_t newsz = 0;
        Region reg{};
        if (in && alive[v] && u >= 0 && cnt[v] != 0) {
          const int32_t nsize = t_size[v], noff = t_off[v], ndepth = t_depth[v], lsize = t_lsize[v];
          const int sign = insert ? 1 : -1;
          if (lsize < 0) {
            if (insert) {
              add = true;
              reg = Region{u, ndepth, noff, noff + nsize, s0[v], s0[v] + sz[v], 0, 0};
            } else {
              setsz = true;
              newsz = nsize - cnt[v];
            }
          } else if (l == lambda) {
            if (apply) killed_next[child_idx[static_cast<int64_t>(sig) * nheap + v]] = 0;
          } else {
            const int64_t n2 = static_cast<int64_t>(nsize) + sign * cnt[v];
            const int64_t l2 = static_cast<int64_t>(lsize) + sign * cnt[2 * v];
            const bool bal = n2 > 0 && (ad - 2 * an) * n2 <= 2 * ad * l2 && 2 * ad * l2 <= (ad + 2 * an) * n2;
            if (bal) {
              setsz = true;
              newsz = static_cast<int32_t>(n2);
              alive[2 * v] = alive[2 * v + 1] = 1;
            } else {
              add = true;
              reg = Region{u, ndepth, noff, noff + nsize, s0[v], s0[v] + sz[v], 0, 0};
            }
          }
        }
        // new sizes are recorded, not written: the tree changes only once the
        // whole update has its memory (commit)
        const unsigned long long sm = __ballot(setsz);
        if (apply && setsz) sizes[sbase + sized + __popcll(sm & ((1ULL << lane) - 1))] = make_int2(u, newsz);
        sized += __popcll(sm);
        const unsigned long long rm = __ballot(add);
        if (apply && add) regions[base + added + __popcll(rm & ((1ULL << lane) - 1))] = reg;
        added += __popcll(rm);
      }
    }
    wave_sync();
  }
  if (!apply && lane == 0) {
    rcount[sig] = added;
    scount[sig] = sized;
  }
}

__global__ void k_add_regions(int* n_regions, const int32_t* roff, int* n_sizes, const int32_t* soff, int ns) {
  *n_regions += roff[ns];
  *n_sizes += soff[ns];
}

// ---- where the old points go.  A batch that is small against the tree is
// described by two sorted event lists instead of per-point arrays (which cost
// O(n) fills and a prefix sum over the whole tree at every batch, however
// small): the rebuild regions ordered by their old end b (an insert adds a
// region's batch points there; a region's own points are left to the
// rebuild), and for a delete the ascending positions of the removed points.
// A table per chunk of kEvChunk old positions holds how many events lie below
// the chunk, so a lookup searches only the chunk's own events.  A batch whose
// events are dense in the tree (more than one per kDenseRatio positions)
// takes per-point arrays instead: region marks, and the prefix sum of the
// batch points noted at region ends or of the removal flags.
constexpr int64_t kEvChunk = 4096;
constexpr int64_t kDenseRatio = 32;

struct EvView {
  const uint64_t* rkey;   // [R] 2 b + (region empty), ascending: at equal ends a non-empty region comes first
  const uint32_t* rk;     // [R] the region of sorted entry j
  const int32_t* gx;      // [R + 1] insert: batch points of the sorted entries below j
  const int32_t* rc;      // [nch + 1] entries whose end lies below c kEvChunk
  const uint64_t* dp;     // [nd] delete: removed positions, ascending
  const int32_t* dc;      // [nch + 1] removed positions below c kEvChunk
  int32_t R, nd;
  int dense;              // per-point arrays instead of the lists:
  const int32_t* S;       //   [n + 2] insert: batch points at region ends below o; delete: removed below o
  const int32_t* regid;   //   [n] the region holding o, or -1
  const int32_t* delflag; //   [n] delete: o is removed
};

// Index of the first a[lo .. hi) that is >= x (hi if none); a ascending.
__device__ inline int32_t first_not_below(const uint64_t* a, int32_t lo, int32_t hi, uint64_t x) {
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Regions whose old end lies below x, for 0 <= x <= n (event lists only).
__device__ inline int32_t ends_below(const EvView& ev, int64_t x) {
  const int64_t c = x / kEvChunk;
  return first_not_below(ev.rkey, ev.rc[c], ev.rc[c + 1], static_cast<uint64_t>(x) << 1);
}

// Batch points of the regions whose old end lies below x, for 0 <= x <= n.
__device__ inline int32_t growth_below(const EvView& ev, int64_t x) {
  return ev.dense ? ev.S[x] : ev.gx[ends_below(ev, x)];
}

// Removed positions below x, for 0 <= x <= n.
__device__ inline int32_t removed_below(const EvView& ev, int64_t x) {
  if (ev.dense) return ev.S[x];
  const int64_t c = x / kEvChunk;
  return first_not_below(ev.dp, ev.dc[c], ev.dc[c + 1], static_cast<uint64_t>(x));
}

// The region holding old position o (0 <= o < n), or -1.  In the lists the
// first entry ending after o is the only candidate: regions are disjoint, and
// an empty region (an empty tree of a batch handle) sits at a boundary
// between trees, never strictly inside another region.
__device__ inline int32_t region_at(const EvView& ev, const Region* regions, int64_t o) {
  if (ev.dense) return ev.regid[o];
  const int32_t u = ends_below(ev, o + 1);
  if (u >= ev.R) return -1;
  const int32_t k = static_cast<int32_t>(ev.rk[u]);
  return regions[k].a <= o ? k : -1;
}

// Whether old position o (0 <= o < n) is removed; *below = removed below o.
__device__ inline bool removed_at(const EvView& ev, int64_t o, int32_t* below) {
  if (ev.dense) {
    *below = ev.S[o];
    return ev.delflag[o] != 0;
  }
  const int32_t j = removed_below(ev, o);
  *below = j;
  return j < ev.nd && ev.dp[j] == static_cast<uint64_t>(o);
}

// Per-point arrays of a dense batch: the region of every old position, and
// (insert) each region's batch points noted at its end.  Grid (regions, y):
// the y blocks of a region share its range.
__global__ void k_region_mark(const Region* regions, int32_t* regid, int32_t* at_end) {
  const Region r = regions[blockIdx.x];
  const int64_t stride = static_cast<int64_t>(gridDim.y) * blockDim.x;
  for (int64_t o = r.a + static_cast<int64_t>(blockIdx.y) * blockDim.x + threadIdx.x; o < r.b; o += stride)
    regid[o] = blockIdx.x;
  if (at_end && blockIdx.y == 0 && threadIdx.x == 0) atomicAdd(at_end + r.b, r.e - r.s);
}

// Removal flags of a dense delete from the sorted removed positions.
__global__ void k_mark_removed(const uint64_t* dp, int32_t nd, int32_t* flag) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nd; j += gridDim.x * blockDim.x) flag[dp[j]] = 1;
}

// Sort keys of the regions by old end.
__global__ void k_region_keys(const Region* regions, int n_regions, uint64_t* key, uint32_t* val) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_regions; k += gridDim.x * blockDim.x) {
    const Region r = regions[k];
    key[k] = (static_cast<uint64_t>(r.b) << 1) | (r.a == r.b ? 1u : 0u);
    val[k] = static_cast<uint32_t>(k);
  }
}

// Batch points of the sorted regions (the insert's growth at each end).
__global__ void k_region_growth(const Region* regions, const uint32_t* rk, int n_regions, int32_t* g) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_regions; j += gridDim.x * blockDim.x) {
    const Region r = regions[rk[j]];
    g[j] = r.e - r.s;
  }
}

// Chunk table of an ascending key list: out[c] = keys below c kEvChunk << shift.
__global__ void k_chunk_table(const uint64_t* keys, int32_t cnt, int shift, int64_t nch, int32_t* out) {
  for (int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; c <= nch;
       c += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[c] = first_not_below(keys, 0, cnt, static_cast<uint64_t>(c * kEvChunk) << shift);
}

// New places of the old points outside every region: insert: o plus the batch
// points of the regions ending at or before o; delete: o minus the removed
// points before o.  The packed 32-bit coordinates go to the new layout's own
// array.  Points of regions are left to the rebuild.  One workgroup per chunk
// of kEvChunk positions; the chunk's events (the region entries ending in it
// and the first one after it, the removed positions in it) are staged in LDS
// when they fit, so a point's lookup is a short search there (a dense batch
// reads its per-point arrays).
constexpr int kEvStage = 512;

template <int D>
__global__ void __launch_bounds__(256) k_relayout(const int64_t* X, int64_t xcap, int64_t n, EvView ev,
                                                  const Region* regions, int insert, int64_t* Y, int64_t ycap,
                                                  int32_t* C32) {
  __shared__ uint64_t s_key[kEvStage];
  __shared__ int32_t s_a[kEvStage];
  __shared__ int32_t s_g[kEvStage];
  __shared__ uint64_t s_dp[kEvStage];
  const int64_t c = blockIdx.x;
  const int64_t o0 = c * kEvChunk;
  const int64_t o1 = o0 + kEvChunk < n ? o0 + kEvChunk : n;
  if (o0 >= o1) return;
  // o in the chunk: the first entry ending after o lies in [r0, r1], the
  // removed positions below o number d0 + (those of [d0, d1) below o)
  const bool lists = !ev.dense;
  const int32_t r0 = lists ? ev.rc[c] : 0, r1 = lists ? ev.rc[c + 1] : 0;
  const int32_t d0 = lists && !insert ? ev.dc[c] : 0, d1 = lists && !insert ? ev.dc[c + 1] : 0;
  const int32_t nr = r1 - r0, nd = d1 - d0;
  const bool staged = lists && nr < kEvStage && nd <= kEvStage;
  if (staged) {
    const int32_t na = (r1 < ev.R ? nr + 1 : nr);
    for (int i = threadIdx.x; i <= nr; i += blockDim.x) {
      if (i < nr) s_key[i] = ev.rkey[r0 + i];
      if (i < na) s_a[i] = regions[ev.rk[r0 + i]].a;
      if (insert) s_g[i] = ev.gx[r0 + i];
    }
    for (int i = threadIdx.x; i < nd; i += blockDim.x) s_dp[i] = ev.dp[d0 + i];
  }
  __syncthreads();
  for (int64_t o = o0 + threadIdx.x; o < o1; o += blockDim.x) {
    int32_t u = 0, j = 0;   // u: first entry ending after o; j: removed positions below o
    bool removed = false;
    if (staged) {
      int32_t lo = 0, hi = nr;
      const uint64_t x = static_cast<uint64_t>(o + 1) << 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (s_key[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      if (r0 + lo < ev.R && s_a[lo] <= o) continue;
      u = lo;
      if (!insert) {
        int32_t l2 = 0, h2 = nd;
        while (l2 < h2) {
          const int32_t mid = (l2 + h2) >> 1;
          if (s_dp[mid] < static_cast<uint64_t>(o)) l2 = mid + 1;
          else h2 = mid;
        }
        removed = l2 < nd && s_dp[l2] == static_cast<uint64_t>(o);
        j = d0 + l2;
      }
    } else if (lists) {
      u = ends_below(ev, o + 1);
      if (u < ev.R && regions[ev.rk[u]].a <= o) continue;
      if (!insert) removed = removed_at(ev, o, &j);
    } else {
      if (ev.regid[o] >= 0) continue;
      if (!insert) removed = removed_at(ev, o, &j);
    }
    int64_t dst;
    if (insert) {
      dst = o + (staged ? s_g[u] : (lists ? ev.gx[u] : ev.S[o + 1]));
    } else {
      if (removed) continue;
      dst = o - j;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t v = X[d * xcap + o];
      Y[d * ycap + dst] = v;
      C32[dst * D + d] = static_cast<int32_t>(v);
    }
    Y[D * ycap + dst] = X[D * xcap + o];
  }
}

// New offsets of the surviving nodes.  Live node ranges nest like the tree,
// so a node whose first point lies inside a region and that is deeper than
// the region's node is below it: it dies (the rebuilt subtree replaces it).
// Returns the node's new offset, -1 to leave it, -2 to mark it dead.
__device__ inline int64_t node_new_off(const Node& nd, int32_t t, const EvView& ev, const Region* regions,
                                       int insert, int64_t n_old) {
  if (nd.pad != 0) return -1;   // dead since an earlier update
  if (nd.off < 0 || nd.off > n_old) return -1;
  const bool inside = nd.off < n_old;
  // in the lists one lookup serves both the region test and an insert's
  // shift: the first entry ending after the node's first point
  int32_t u = 0;
  if (!ev.dense && (insert || inside)) u = ends_below(ev, inside ? nd.off + 1 : nd.off);
  if (inside && nd.size > 0) {
    int32_t k = -1;
    if (ev.dense) {
      k = ev.regid[nd.off];
    } else if (u < ev.R) {
      const int32_t c = static_cast<int32_t>(ev.rk[u]);
      if (regions[c].a <= nd.off) k = c;
    }
    if (k >= 0) {
      const Region r = regions[k];
      if (r.node == t) return -1;        // overwritten by its rebuilt subtree
      if (nd.depth > r.depth) return -2;
    }
  }
  if (insert) return nd.off + (ev.dense ? ev.S[inside ? nd.off + 1 : nd.off] : ev.gx[u]);
  return nd.off - removed_below(ev, nd.off);
}

// Four nodes per thread, their records loaded together (coalesced across the
// wave) and their lookups done before any store, so a thread has four chains
// of dependent loads in flight rather than one.
constexpr int kNodesPerThread = 4;

__global__ void __launch_bounds__(256) k_node_update(Node* nodes, int32_t n_nodes, EvView ev, const Region* regions,
                                                     int insert, int64_t n_old) {
  const int64_t S = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t0 < n_nodes;
       t0 += S * kNodesPerThread) {
    Node nd[kNodesPerThread];
#pragma unroll
    for (int i = 0; i < kNodesPerThread; ++i) {
      const int64_t t = t0 + i * S;
      if (t < n_nodes) nd[i] = nodes[t];
      else nd[i].pad = 1;
    }
    int64_t no[kNodesPerThread];
#pragma unroll
    for (int i = 0; i < kNodesPerThread; ++i)
      no[i] = node_new_off(nd[i], static_cast<int32_t>(t0 + i * S), ev, regions, insert, n_old);
#pragma unroll
    for (int i = 0; i < kNodesPerThread; ++i) {
      const int64_t t = t0 + i * S;
      if (no[i] == -2) nodes[t].pad = 1;
      else if (no[i] >= 0) nodes[t].off = static_cast<int32_t>(no[i]);
    }
  }
}

__global__ void k_region_final(Region* regions, int n_regions, EvView ev, int insert, int32_t* new_size,
                               int32_t* old_size) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_regions; k += gridDim.x * blockDim.x) {
    Region& r = regions[k];
    if (insert) {
      // batch points are placed at region ends; for a region with old points
      // the end lies after its start, for an empty one (an empty tree of a
      // batch handle) on it, and its own batch points are not before it
      r.new_start = r.a + growth_below(ev, r.a < r.b ? r.a + 1 : r.a);
      r.new_size = (r.b - r.a) + (r.e - r.s);
    } else {
      const int32_t before = removed_below(ev, r.a);
      r.new_start = r.a - before;
      r.new_size = (r.b - r.a) - (removed_below(ev, r.b) - before);
    }
    new_size[k] = r.new_size;
    old_size[k] = r.b - r.a;
  }
}

// Root task of every region's rebuild (its points at comp[k] in the packed
// gather, its subtree at the region node's depth) and the int64 offsets.
__global__ void k_region_roots(const Region* regions, int n_regions, const int32_t* comp32, int64_t* comp,
                               Task* roots) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= n_regions; k += gridDim.x * blockDim.x) {
    comp[k] = comp32[k];
    if (k == n_regions) continue;
    Task t;
    t.start = comp32[k];
    t.m = regions[k].new_size;
    t.slot = k;
    t.depth = static_cast<int16_t>(regions[k].depth);
    t.buf = 2;
    t.mode = 0;
    roots[k] = t;
  }
}

// Work over the regions' points is spread by points, not by regions (their
// sizes are skewed: many leaves and a few large subtrees): each workgroup
// takes kFlatChunk consecutive entries q of a per-region prefix sum P (region
// k owns P[k] .. P[k+1]-1), finds the regions of its first and last entry by
// binary search, and each thread then searches only that range.
constexpr int kFlatChunk = 2048;

// The last index in [lo, hi) whose P is <= q (P[lo] <= q).  An empty region
// shares its P with the next one and is never chosen over it.
__device__ inline int last_at_or_below(const int32_t* P, int lo, int hi, int64_t q) {
  while (hi - lo > 1) {
    const int mid = lo + ((hi - lo) >> 1);
    if (P[mid] <= q) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ inline void chunk_regions(const int32_t* P, int nreg, int64_t q0, int64_t q1, int* k0, int* k1) {
  __shared__ int s_k[2];
  if (threadIdx.x == 0) s_k[0] = last_at_or_below(P, 0, nreg, q0);
  if (threadIdx.x == 1) s_k[1] = last_at_or_below(P, 0, nreg, q1 - 1);
  __syncthreads();
  *k0 = s_k[0];
  *k1 = s_k[1];
}

// The points of every region after the update, packed region after region
// (region k from comp[k]) as the input of the rebuild: the old points of the
// region that survive, then (insert) its batch points.  Insert: P = comp and
// entry q is output position q; delete: P is the prefix of the regions' old
// sizes and entry q an old point, placed among the survivors.
template <int D>
__global__ void __launch_bounds__(256) k_gather_regions(const Region* regions, int n_regions, const int32_t* P,
                                                        int64_t total, const int32_t* comp, const int64_t* X,
                                                        int64_t xcap, EvView ev, const int64_t* batch, int64_t m,
                                                        int insert, int64_t* cin, int64_t ccap) {
  const int64_t q0 = static_cast<int64_t>(blockIdx.x) * kFlatChunk;
  if (q0 >= total) return;
  const int64_t q1 = q0 + kFlatChunk < total ? q0 + kFlatChunk : total;
  int k0, k1;
  chunk_regions(P, n_regions, q0, q1, &k0, &k1);
  for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    const int k = last_at_or_below(P, k0, k1 + 1, q);
    const Region r = regions[k];
    const int64_t local = q - P[k];
    if (insert) {
      const int64_t nold = r.b - r.a;
      if (local < nold) {
        const int64_t o = r.a + local;
#pragma unroll
        for (int d = 0; d <= D; ++d) cin[d * ccap + q] = X[d * xcap + o];
      } else {
        const int64_t i = r.s + (local - nold);
#pragma unroll
        for (int d = 0; d <= D; ++d) cin[d * ccap + q] = batch[d * m + i];
      }
    } else {
      const int64_t o = r.a + local;
      int32_t j;
      if (removed_at(ev, o, &j)) continue;
      const int64_t at = comp[k] + (o - j) - r.new_start;
#pragma unroll
      for (int d = 0; d <= D; ++d) cin[d * ccap + at] = X[d * xcap + o];
    }
  }
}

// ---- commit: the kernels below run only after every allocation of the
// update has succeeded, so a failed update never reaches them.
__global__ void k_apply_sizes(Node* nodes, const int2* sizes, const int* n_sizes) {
  const int n = *n_sizes;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    nodes[sizes[i].x].size = sizes[i].y;
}

__device__ inline int region_of(const int64_t* comp, int nreg, int64_t p) {
  int lo = 0, hi = nreg;   // last region whose packed range starts at or before p
  while (hi - lo > 1) {
    const int mid = lo + ((hi - lo) >> 1);
    if (comp[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// Rebuilt points back from the packed rebuild (region k from comp[k]) to
// their regions' ranges, spread by points as in the gather.
template <int D>
__global__ void __launch_bounds__(256) k_scatter_back(const Region* regions, const int32_t* comp, int nreg,
                                                      int64_t total, const int64_t* Z, int64_t zcap, int64_t* Y,
                                                      int64_t ycap, int32_t* C32) {
  const int64_t q0 = static_cast<int64_t>(blockIdx.x) * kFlatChunk;
  if (q0 >= total) return;
  const int64_t q1 = q0 + kFlatChunk < total ? q0 + kFlatChunk : total;
  int k0, k1;
  chunk_regions(comp, nreg, q0, q1, &k0, &k1);
  for (int64_t p = q0 + threadIdx.x; p < q1; p += blockDim.x) {
    const int k = last_at_or_below(comp, k0, k1 + 1, p);
    const int64_t dst = regions[k].new_start + (p - comp[k]);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t v = Z[d * zcap + p];
      Y[d * ycap + dst] = v;
      C32[dst * D + d] = static_cast<int32_t>(v);
    }
    Y[D * ycap + dst] = Z[D * zcap + p];
  }
}

// A node of the rebuild as a node of the tree: rebuild node j >= nreg goes to
// base + j - nreg, rebuild root r to the region's node; offsets move from the
// packed range to the region's range.
__device__ inline Node translate(Node nd, const Region* regions, const int64_t* comp, int nreg, int region,
                                 int32_t base) {
  if (nd.pad != 0) return nd;
  if (nd.left >= 0) {
    nd.left = base + (nd.left - nreg);
    nd.right = base + (nd.right - nreg);
  }
  const int r = region >= 0 ? region : region_of(comp, nreg, nd.off);
  nd.off = static_cast<int32_t>(regions[r].new_start + (nd.off - comp[r]));
  return nd;
}

__global__ void k_append_nodes(Node* nodes, int32_t base, const Node* tmp, int32_t tmp_count, const Region* regions,
                               const int64_t* comp, int nreg) {
  for (int32_t j = nreg + blockIdx.x * blockDim.x + threadIdx.x; j < tmp_count; j += gridDim.x * blockDim.x)
    nodes[base + (j - nreg)] = translate(tmp[j], regions, comp, nreg, -1, base);
}

__global__ void k_copy_roots(Node* nodes, int32_t base, const Node* tmp, const Region* regions, const int64_t* comp,
                             int nreg) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nreg; r += gridDim.x * blockDim.x)
    nodes[regions[r].node] = translate(tmp[r], regions, comp, nreg, r, base);
}

// After an update the stored boxes (if any) are recomputed; a tree that
// cannot get the memory for them drops them (queries then derive the cells
// from the splitters, with the same results).
void refresh_boxes(pkd_tree* T, hipStream_t st) {
  if (T->bbox_on && compute_bbox(T, st) != PKD_OK) {
    T->bbox_on = false;
    dev_free(T->bbox, st);
    T->bbox = nullptr;
    T->bbox_cap = 0;
  }
}

int fill(hipStream_t st, int32_t* a, int64_t n, int32_t v) {
  if (n <= 0) return PKD_OK;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>(4096, (n + 255) / 256));
  hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(256), 0, st, a, n, v);
  return kernel_status("k_fill_i32");
}

struct RoundSave {
  DArr<Task> tasks;
  DArr<int32_t> hn, bsize, bstart, child;
  int ns = 0;
  int lambda = 0;   // levels this round descends
  explicit RoundSave(hipStream_t s) : tasks(s), hn(s), bsize(s), bstart(s), child(s) {}
};

// Rounds with at least this many subproblems route by one sort of the batch
// instead of the tiled sieve (which needs a tile and a workgroup per
// subproblem, however few points it holds).
constexpr int kSortRouteMin = 512;

struct SortRoute {
  DArr<int32_t> task_of;
  DArr<uint64_t> keys;
  DArr<uint32_t> vals;
  SortWork sort;
  explicit SortRoute(hipStream_t s) : task_of(s), keys(s), vals(s), sort(s) {}
};

// One routing round by sort: the points of the ns tasks move from buffer src
// to dst grouped by bucket (stable), bsize/bstart ([ns][2^lambda]) as the
// sieve pass would leave them.
template <int D>
int route_by_sort(hipStream_t st, const Task* tasks, int ns, int64_t m, const Bufs& wb, int src, int dst,
                  const int64_t* rx, const uint8_t* rdim, int lambda, SortRoute& W, int32_t* bsize,
                  int32_t* bstart) {
  const int NB = 1 << lambda;
  PKD_TRY(W.task_of.need(m));
  PKD_TRY(W.keys.need(m));
  PKD_TRY(W.vals.need(m));
  PKD_TRY(fill(st, W.task_of.p, m, -1));
  hipLaunchKernelGGL(k_task_fill, dim3((ns + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, st, tasks, ns, W.task_of.p);
  PKD_TRY(kernel_status("k_task_fill"));
  const unsigned g = static_cast<unsigned>((m + 255) / 256);
  hipLaunchKernelGGL(k_route_keys<D>, dim3(g), dim3(256), 0, st, wb.c[src], wb.cap[src], m, W.task_of.p, tasks, rx,
                     rdim, lambda, W.keys.p, W.vals.p);
  PKD_TRY(kernel_status("k_route_keys"));
  uint64_t* ks = nullptr;
  uint32_t* vs = nullptr;
  PKD_TRY(radix_sort_pairs(st, W.keys.p, W.vals.p, m, bits_for(m - 1) + lambda, W.sort, &ks, &vs));
  PKD_TRY(fill(st, bsize, static_cast<int64_t>(ns) * NB, 0));
  hipLaunchKernelGGL(k_route_place<D>, dim3(g), dim3(256), 0, st, ks, vs, m, W.task_of.p, lambda, wb, src, dst, bsize);
  PKD_TRY(kernel_status("k_route_place"));
  hipLaunchKernelGGL(k_route_bstart, dim3((ns + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, st, tasks, ns, lambda,
                     bsize, bstart);
  return kernel_status("k_route_bstart");
}

template <int D>
int update_d(pkd_tree* T, int32_t tree, hipStream_t st, const int64_t* coords, const int64_t* ids, int64_t m,
             bool insert, int64_t* removed) {
  const Params& P = T->prm;
  const int lambda = P.lambda, NB = 1 << lambda, nheap = 2 << lambda;
  const int64_t n = T->n;
  Node root{};
  DArr<int> flags(st);
  PKD_TRY(flags.need(8));
  PKD_HIP(hipMemsetAsync(flags.p, 0, sizeof(int) * 8, st));
  {
    const unsigned g = static_cast<unsigned>(std::min<int64_t>(4096, (m + 255) / 256));
    hipLaunchKernelGGL(k_validate<D>, dim3(g), dim3(256), 0, st, coords, m, flags.p);
    PKD_TRY(kernel_status("k_validate"));
    int h = 0;
    PKD_HIP(hipMemcpyAsync(&h, flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
    // the tree's root (node `tree`: the trees of a handle have their roots
    // first) comes back with the same wait
    if (!(insert && n == 0 && T->n_trees == 1))   // (that insert is a fresh build)
      PKD_HIP(hipMemcpyAsync(&root, T->nodes + tree, sizeof(Node), hipMemcpyDeviceToHost, st));
    PKD_HIP(hipStreamSynchronize(st));
    if (h & kErrRange) return PKD_ERR_RANGE;
  }
  if (insert && n == 0 && T->n_trees == 1) {
    // inserting into the empty tree is Build(P) at the root: built as a new
    // tree whose storage replaces the tree's only once it is complete
    pkd_tree* fresh = nullptr;
    PKD_TRY(build_new(T->prm, st, coords, ids, m, 1, &fresh));
    swap_storage(T, fresh);
    release(fresh, st);
    delete fresh;
    T->last_regions = 1;
    T->last_rebuilt = m;
    refresh_boxes(T, st);
    return PKD_OK;
  }

  // ---- route the batch to the leaves
  DArr<int64_t> wb0(st), wb1(st), wf(st), rx(st);
  DArr<uint8_t> rdim(st);
  DArr<int8_t> mode(st);
  DArr<Task> cur(st), nxt(st);
  DArr<Res> res(st);
  DArr<int> ctr(st);
  DArr<int32_t> leaf_of(st), Mw(st), M(st), bsum(st), n_go(st), n_leaf(st), off_go(st), off_leaf(st);
  PKD_TRY(wb0.need(static_cast<size_t>(D + 1) * m));
  PKD_TRY(wb1.need(static_cast<size_t>(D + 1) * m));
  PKD_TRY(wf.need(static_cast<size_t>(D + 1) * m));
  PKD_HIP(hipMemcpyAsync(wb0.p, coords, sizeof(int64_t) * D * m, hipMemcpyDeviceToDevice, st));
  PKD_HIP(hipMemcpyAsync(wb0.p + static_cast<int64_t>(D) * m, ids, sizeof(int64_t) * m, hipMemcpyDeviceToDevice, st));
  Bufs wb;
  wb.c[0] = wb0.p;
  wb.id[0] = wb0.p + static_cast<int64_t>(D) * m;
  wb.c[1] = wb1.p;
  wb.id[1] = wb1.p + static_cast<int64_t>(D) * m;
  wb.c[2] = wb.id[2] = nullptr;
  wb.cap[0] = wb.cap[1] = m;
  wb.cap[2] = 0;
  PKD_TRY(ctr.need(8));
  PKD_HIP(hipMemsetAsync(ctr.p, 0, sizeof(int) * 8, st));
  int* d_regions = ctr.p + 2;
  PKD_TRY(res.need(static_cast<size_t>(m) + 1));

  std::vector<RoundSave*> rounds;
  struct Cleanup {
    std::vector<RoundSave*>& r;
    ~Cleanup() {
      for (auto* x : r) delete x;
    }
  } cleanup{rounds};
  int nres = 0;
  if (root.left < 0) {
    Res r0{tree, 0, static_cast<int32_t>(m), 0};
    PKD_HIP(hipMemcpyAsync(res.p, &r0, sizeof(Res), hipMemcpyHostToDevice, st));
    nres = 1;
  } else {
    PKD_TRY(cur.need(1));
    Task t0{0, static_cast<int32_t>(m), tree, root.depth, 0, 0};
    PKD_HIP(hipMemcpyAsync(cur.p, &t0, sizeof(Task), hipMemcpyHostToDevice, st));
    int ns = 1, src = 0;
    int depth_r = root.depth;   // depth of this round's subproblem roots
    SieveWork W(st);
    SortRoute SR(st);
    while (ns > 0) {
      // every round descends at least one level of a tree no higher than T->height
      if (static_cast<int64_t>(rounds.size()) > T->height + 4) return PKD_ERR_INTERNAL;
      // lambda levels per round, fewer where the tree ends sooner (a round's
      // per-subproblem arrays have 2^levels entries, and the last rounds hold
      // the most subproblems)
      const int lr = std::max(1, std::min(lambda, T->height - depth_r));
      const int NBr = 1 << lr, nheapr = 2 << lr;
      RoundSave* R = new RoundSave(st);
      rounds.push_back(R);
      R->ns = ns;
      R->lambda = lr;
      PKD_TRY(R->tasks.need(ns));
      PKD_HIP(hipMemcpyAsync(R->tasks.p, cur.p, sizeof(Task) * ns, hipMemcpyDeviceToDevice, st));
      PKD_TRY(rx.need(static_cast<size_t>(ns) * NBr));
      PKD_TRY(rdim.need(static_cast<size_t>(ns) * NBr));
      PKD_TRY(mode.need(ns));
      PKD_TRY(R->hn.need(static_cast<size_t>(ns) * nheapr));
      PKD_TRY(R->child.need(static_cast<size_t>(ns) * nheapr));
      PKD_HIP(hipMemsetAsync(mode.p, 0, ns, st));
      hipLaunchKernelGGL(k_fetch_skeleton, dim3((ns + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, st, cur.p, ns,
                         T->nodes, lr, rx.p, rdim.p, R->hn.p);
      PKD_TRY(kernel_status("k_fetch_skeleton"));
      const int dst = 1 - src;
      PKD_TRY(R->bsize.need(static_cast<size_t>(ns) * NBr));
      PKD_TRY(R->bstart.need(static_cast<size_t>(ns) * NBr));
      if (ns >= kSortRouteMin) {
        PKD_TRY(route_by_sort<D>(st, cur.p, ns, m, wb, src, dst, rx.p, rdim.p, lr, SR, R->bsize.p,
                                 R->bstart.p));
      } else {
        int64_t ntiles = 0, nchunks = 0, pts = 0;
        PKD_TRY(sieve_layout(st, cur.p, ns, P.tile, W, P.s, 0, nullptr, &ntiles, &nchunks, &pts));
        PKD_TRY(sieve_pass(st, D, lr, P.tile, cur.p, ns, wb, src, dst, rx.p, rdim.p, mode.p, W, ntiles, nchunks,
                           pts, 0, flags.p));
        PKD_HIP(hipMemcpyAsync(R->bsize.p, W.bsize.p, sizeof(int32_t) * ns * NBr, hipMemcpyDeviceToDevice, st));
        PKD_HIP(hipMemcpyAsync(R->bstart.p, W.bstart.p, sizeof(int32_t) * ns * NBr, hipMemcpyDeviceToDevice, st));
      }
      PKD_TRY(nxt.need(static_cast<size_t>(ns) * NBr));
      PKD_TRY(n_go.need(ns));
      PKD_TRY(n_leaf.need(ns));
      PKD_TRY(off_go.need(ns + 1));
      PKD_TRY(off_leaf.need(ns + 1));
      const unsigned gw = static_cast<unsigned>((ns + kWaves - 1) / kWaves);
      hipLaunchKernelGGL(k_route_count, dim3(gw), dim3(64 * kWaves), 0, st, cur.p, ns, T->nodes, lr, R->hn.p,
                         R->bsize.p, R->bstart.p, n_go.p, n_leaf.p);
      PKD_TRY(kernel_status("k_route_count"));
      PKD_TRY(exscan_i32(st, n_go.p, off_go.p, ns, bsum));
      PKD_TRY(exscan_i32(st, n_leaf.p, off_leaf.p, ns, bsum));
      int h[2];
      PKD_HIP(hipMemcpyAsync(&h[0], off_go.p + ns, sizeof(int), hipMemcpyDeviceToHost, st));
      PKD_HIP(hipMemcpyAsync(&h[1], off_leaf.p + ns, sizeof(int), hipMemcpyDeviceToHost, st));
      hipLaunchKernelGGL(k_route_emit, dim3(gw), dim3(64 * kWaves), 0, st, cur.p, ns, T->nodes, lr, R->hn.p,
                         R->bsize.p, R->bstart.p, dst, off_go.p, off_leaf.p, nres, nxt.p, R->child.p, res.p);
      PKD_TRY(kernel_status("k_route_emit"));
      PKD_HIP(hipStreamSynchronize(st));
      ns = h[0];
      nres += h[1];
      depth_r += lr;
      std::swap(cur.p, nxt.p);
      std::swap(cur.cap, nxt.cap);
      src = dst;
    }
  }
  PKD_TRY(leaf_of.need(m));
  if (nres > 0)
    hipLaunchKernelGGL(k_gather, dim3((nres + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, st, res.p, nres, D, wb,
                       wf.p, m, leaf_of.p);
  PKD_TRY(kernel_status("k_gather"));

  // ---- weights: 1 per inserted point, 1 per point actually removed
  const int64_t* X = T->buf[T->cur];
  PKD_TRY(Mw.need(m + 1));
  PKD_TRY(M.need(m + 1));
  // the chunk tables of the event lists cover old positions 0 .. n
  const int64_t nch = n / kEvChunk + 1;
  const unsigned gch = static_cast<unsigned>(std::min<int64_t>(4096, (nch + 256) / 256));
  DArr<uint64_t> dpos(st);
  DArr<int32_t> dtab(st);
  int64_t n_removed = 0;
  if (insert) {
    PKD_TRY(fill(st, Mw.p, m, 1));
  } else {
    // removed positions: matched, sorted, repeats dropped
    DArr<uint64_t> pos(st);
    DArr<uint32_t> ent(st);
    DArr<int32_t> claim(st), at(st);
    SortWork SW(st);
    PKD_TRY(pos.need(m));
    PKD_TRY(ent.need(m));
    PKD_TRY(claim.need(m));
    PKD_TRY(at.need(m + 1));
    PKD_TRY(dpos.need(m));
    hipLaunchKernelGGL(k_match<D>, dim3(static_cast<unsigned>((m + 255) / 256)), dim3(256), 0, st, wf.p, m,
                       leaf_of.p, T->nodes, X, T->cap, n, pos.p, ent.p);
    PKD_TRY(kernel_status("k_match"));
    uint64_t* ks = nullptr;
    uint32_t* vs = nullptr;
    PKD_TRY(radix_sort_pairs(st, pos.p, ent.p, m, bits_for(n), SW, &ks, &vs));
    const unsigned gm = static_cast<unsigned>(std::min<int64_t>(4096, (m + 255) / 256));
    hipLaunchKernelGGL(k_claim, dim3(gm), dim3(256), 0, st, ks, vs, m, n, claim.p, Mw.p);
    PKD_TRY(kernel_status("k_claim"));
    PKD_TRY(exscan_i32(st, claim.p, at.p, m, bsum));
    hipLaunchKernelGGL(k_removed_list, dim3(gm), dim3(256), 0, st, ks, claim.p, at.p, m, dpos.p);
    PKD_TRY(kernel_status("k_removed_list"));
  }
  PKD_TRY(exscan_i32(st, Mw.p, M.p, m, bsum));
  if (!insert) {
    int32_t tot = 0;
    PKD_HIP(hipMemcpyAsync(&tot, M.p + m, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PKD_HIP(hipStreamSynchronize(st));
    n_removed = tot;
    *removed = tot;
    if (tot == 0) {   // nothing to do
      T->last_regions = T->last_rebuilt = 0;
      return PKD_OK;
    }
  }

  // ---- decide, round by round, top-down.  Nothing is written to the tree
  // until the commit below: new sizes and regions are recorded in scratch.
  DArr<Region> regions(st);
  DArr<int2> sizes(st);
  DArr<int8_t> killed(st), killed_next(st);
  DArr<int32_t> rcount(st), roff(st), scount(st), soff(st);
  PKD_TRY(regions.need(static_cast<size_t>(m) + 1));
  {
    size_t most = 2;
    for (auto* R : rounds) most += static_cast<size_t>(R->ns) * (2 << R->lambda);
    PKD_TRY(sizes.need(most));
  }
  int* d_sizes = ctr.p + 3;
  if (rounds.empty()) {
    // the root is a leaf
    if (insert) {
      Region r{tree, root.depth, root.off, root.off + root.size, 0, static_cast<int32_t>(m), 0, 0};
      PKD_HIP(hipMemcpyAsync(regions.p, &r, sizeof(Region), hipMemcpyHostToDevice, st));
      int one = 1;
      PKD_HIP(hipMemcpyAsync(d_regions, &one, sizeof(int), hipMemcpyHostToDevice, st));
    } else {
      const int2 sz = make_int2(tree, root.size - static_cast<int32_t>(n_removed));
      PKD_HIP(hipMemcpyAsync(sizes.p, &sz, sizeof(int2), hipMemcpyHostToDevice, st));
      int one = 1;
      PKD_HIP(hipMemcpyAsync(d_sizes, &one, sizeof(int), hipMemcpyHostToDevice, st));
    }
  } else {
    PKD_TRY(killed.need(1));
    PKD_HIP(hipMemsetAsync(killed.p, 0, 1, st));
    for (size_t r = 0; r < rounds.size(); ++r) {
      RoundSave* R = rounds[r];
      const int nn = r + 1 < rounds.size() ? rounds[r + 1]->ns : 0;
      PKD_TRY(killed_next.need(static_cast<size_t>(nn) + 1));
      PKD_HIP(hipMemsetAsync(killed_next.p, 1, nn + 1, st));
      PKD_TRY(rcount.need(static_cast<size_t>(R->ns) + 1));
      PKD_TRY(roff.need(static_cast<size_t>(R->ns) + 1));
      PKD_TRY(scount.need(static_cast<size_t>(R->ns) + 1));
      PKD_TRY(soff.need(static_cast<size_t>(R->ns) + 1));
      for (int apply = 0; apply < 2; ++apply) {
        hipLaunchKernelGGL(k_decide, dim3((R->ns + kWaves - 1) / kWaves), dim3(64 * kWaves),
                           kWaves * decide_lds_per_wave(R->lambda), st, R->tasks.p, R->ns, R->lambda, R->hn.p,
                           R->bsize.p,
                           R->bstart.p, R->child.p, killed.p, killed_next.p, M.p, T->nodes, P.alpha_num, P.alpha_den,
                           insert ? 1 : 0, regions.p, d_regions, apply, rcount.p, roff.p, sizes.p, d_sizes,
                           scount.p, soff.p);
        PKD_TRY(kernel_status("k_decide"));
        if (apply == 0) {
          PKD_TRY(exscan_i32(st, rcount.p, roff.p, R->ns, bsum));
          PKD_TRY(exscan_i32(st, scount.p, soff.p, R->ns, bsum));
        }
      }
      hipLaunchKernelGGL(k_add_regions, dim3(1), dim3(1), 0, st, d_regions, roff.p, d_sizes, soff.p, R->ns);
      PKD_TRY(kernel_status("k_add_regions"));
      std::swap(killed.p, killed_next.p);
      std::swap(killed.cap, killed_next.cap);
    }
  }
  int n_regions = 0;
  PKD_HIP(hipMemcpyAsync(&n_regions, d_regions, sizeof(int), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));

  // ---- new layout of the packed point array, written into the twin buffer
  // (or fresh buffers when the capacity grows) and a second packed 32-bit
  // copy: the tree's own arrays stay as they are until the commit
  const int64_t n_new = insert ? n + m : n - n_removed;
  int64_t* Xold = T->buf[T->cur];
  const int64_t old_cap = T->cap;
  int64_t new_cap = T->cap;
  struct Owned {   // device blocks this update allocated; freed unless committed
    hipStream_t st;
    void* p[3] = {nullptr, nullptr, nullptr};
    ~Owned() {
      for (void* q : p) dev_free(q, st);
    }
  } own{st};
  int64_t* Ynew = T->buf[1 - T->cur];
  int64_t* fresh_twin = nullptr;
  if (n_new > T->cap) {
    new_cap = std::max<int64_t>(n_new, T->cap + T->cap / 2);
    const size_t bytes = sizeof(int64_t) * static_cast<size_t>(D + 1) * new_cap;
    PKD_TRY(dev_alloc(&own.p[0], bytes, st));
    PKD_TRY(dev_alloc(&own.p[1], bytes, st));
    Ynew = static_cast<int64_t*>(own.p[0]);
    fresh_twin = static_cast<int64_t*>(own.p[1]);
  }
  int32_t* c32_new = T->c32_twin;
  if (!c32_new || T->c32_twin_cap != new_cap) {
    PKD_TRY(dev_alloc(&own.p[2], sizeof(int32_t) * static_cast<size_t>(D) * static_cast<size_t>(new_cap), st));
    c32_new = static_cast<int32_t*>(own.p[2]);
  }
  // the update's events: sorted lists with chunk tables for a batch that is
  // small against the tree, per-point arrays for a dense one
  const bool dense = P.update_events == 0 ? (static_cast<int64_t>(n_regions) + n_removed) * kDenseRatio > n
                                          : P.update_events == 2;
  DArr<uint64_t> rkey(st);
  DArr<uint32_t> rval(st);
  DArr<int32_t> rtab(st), growth(st), gx(st), S(st), regid(st), flag(st);
  SortWork RW(st);
  EvView ev{};
  ev.R = n_regions;
  ev.nd = static_cast<int32_t>(n_removed);
  ev.dp = dpos.p;
  ev.dense = dense ? 1 : 0;
  if (dense) {
    PKD_TRY(S.need(n + 2));
    PKD_TRY(regid.need(n + 1));
    PKD_TRY(flag.need(n + 2));
    PKD_TRY(fill(st, regid.p, n + 1, -1));
    PKD_TRY(fill(st, flag.p, n + 2, 0));
    // region ranges share out over y blocks in proportion to the points per region
    const unsigned rym = static_cast<unsigned>(
        std::min<int64_t>(1024, std::max<int64_t>(1, (n + m) / (std::max(n_regions, 1) * int64_t{8192}))));
    if (n_regions > 0)
      hipLaunchKernelGGL(k_region_mark, dim3(n_regions, rym), dim3(256), 0, st, regions.p, regid.p,
                         insert ? flag.p : nullptr);
    PKD_TRY(kernel_status("k_region_mark"));
    if (insert) {
      PKD_TRY(exscan_i32(st, flag.p, S.p, n + 1, bsum));   // S[o] = batch points noted at ends below o
    } else {
      if (n_removed > 0)
        hipLaunchKernelGGL(k_mark_removed, dim3(static_cast<unsigned>(std::min<int64_t>(4096, (n_removed + 255) / 256))),
                           dim3(256), 0, st, dpos.p, static_cast<int32_t>(n_removed), flag.p);
      PKD_TRY(kernel_status("k_mark_removed"));
      PKD_TRY(exscan_i32(st, flag.p, S.p, n, bsum));       // S[o] = removed points below o
    }
    ev.S = S.p;
    ev.regid = regid.p;
    ev.delflag = flag.p;
  } else {
    // the regions ordered by old end, their chunk table and (insert) the
    // batch points placed before each end; the removed positions' table
    PKD_TRY(rtab.need(static_cast<size_t>(nch) + 1));
    PKD_TRY(gx.need(static_cast<size_t>(n_regions) + 1));
    ev.rc = rtab.p;
    ev.gx = gx.p;
    if (n_regions > 0) {
      PKD_TRY(rkey.need(n_regions));
      PKD_TRY(rval.need(n_regions));
      const unsigned gr = static_cast<unsigned>(std::min<int64_t>(4096, (n_regions + 255) / 256));
      hipLaunchKernelGGL(k_region_keys, dim3(gr), dim3(256), 0, st, regions.p, n_regions, rkey.p, rval.p);
      PKD_TRY(kernel_status("k_region_keys"));
      uint64_t* ks = nullptr;
      uint32_t* vs = nullptr;
      PKD_TRY(radix_sort_pairs(st, rkey.p, rval.p, n_regions, bits_for(2 * n + 1), RW, &ks, &vs));
      ev.rkey = ks;
      ev.rk = vs;
      if (insert) {
        PKD_TRY(growth.need(n_regions));
        hipLaunchKernelGGL(k_region_growth, dim3(gr), dim3(256), 0, st, regions.p, vs, n_regions, growth.p);
        PKD_TRY(kernel_status("k_region_growth"));
        PKD_TRY(exscan_i32(st, growth.p, gx.p, n_regions, bsum));
      }
    } else {
      PKD_TRY(fill(st, gx.p, 1, 0));
    }
    hipLaunchKernelGGL(k_chunk_table, dim3(gch), dim3(256), 0, st, ev.rkey, n_regions, 1, nch, rtab.p);
    PKD_TRY(kernel_status("k_chunk_table"));
    if (!insert) {
      PKD_TRY(dtab.need(static_cast<size_t>(nch) + 1));
      hipLaunchKernelGGL(k_chunk_table, dim3(gch), dim3(256), 0, st, dpos.p, static_cast<int32_t>(n_removed), 0, nch,
                         dtab.p);
      PKD_TRY(kernel_status("k_chunk_table"));
      ev.dc = dtab.p;
    }
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_relayout<D>, dim3(static_cast<unsigned>(nch)), dim3(256), 0, st, Xold, old_cap, n, ev,
                       regions.p, insert ? 1 : 0, Ynew, new_cap, c32_new);
    PKD_TRY(kernel_status("k_relayout"));
  }
  // region sizes and places after the update, their packed offsets in the
  // rebuild's input (comp) and the rebuild's root tasks, all on the device
  DArr<int32_t> rsize(st), comp32(st), osize(st), ocomp32(st);
  DArr<int64_t> dcomp(st), cin(st);
  DArr<Task> roots(st);
  int32_t R_pts32 = 0, R_old32 = 0;
  if (n_regions > 0) {
    PKD_TRY(rsize.need(static_cast<size_t>(n_regions) + 1));
    PKD_TRY(osize.need(static_cast<size_t>(n_regions) + 1));
    PKD_TRY(ocomp32.need(static_cast<size_t>(n_regions) + 1));
    PKD_TRY(comp32.need(static_cast<size_t>(n_regions) + 1));
    PKD_TRY(dcomp.need(static_cast<size_t>(n_regions) + 1));
    PKD_TRY(roots.need(static_cast<size_t>(n_regions)));
    const unsigned gr = static_cast<unsigned>(std::min<int64_t>(65536, (n_regions + 256) / 256));
    hipLaunchKernelGGL(k_region_final, dim3(gr), dim3(256), 0, st, regions.p, n_regions, ev, insert ? 1 : 0,
                       rsize.p, osize.p);
    PKD_TRY(kernel_status("k_region_final"));
    PKD_TRY(exscan_i32(st, rsize.p, comp32.p, n_regions, bsum));
    if (!insert) {
      PKD_TRY(exscan_i32(st, osize.p, ocomp32.p, n_regions, bsum));
      PKD_HIP(hipMemcpyAsync(&R_old32, ocomp32.p + n_regions, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    hipLaunchKernelGGL(k_region_roots, dim3(gr), dim3(256), 0, st, regions.p, n_regions, comp32.p, dcomp.p,
                       roots.p);
    PKD_TRY(kernel_status("k_region_roots"));
    PKD_HIP(hipMemcpyAsync(&R_pts32, comp32.p + n_regions, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  }
  int n_sizes = 0;
  PKD_HIP(hipMemcpyAsync(&n_sizes, d_sizes, sizeof(int), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));

  // ---- rebuild every region (one segmented Build, Algorithm 1) into a
  // temporary tree: roots 0 .. n_regions-1, each at its node's depth, over the
  // regions' points packed back to back
  struct TmpTree {
    pkd_tree* t = nullptr;
    hipStream_t st;
    ~TmpTree() {
      if (t) {
        release(t, st);
        delete t;
      }
    }
  } tmp{nullptr, st};
  const int64_t R_pts = R_pts32;
  int32_t appended = 0;
  if (n_regions > 0) {
    tmp.t = new pkd_tree;
    tmp.t->prm = T->prm;
    tmp.t->n_trees = n_regions;
    PKD_TRY(alloc_points(tmp.t, st, R_pts));
    PKD_TRY(ensure_nodes(tmp.t, st, std::max<int64_t>(1024, n_regions + R_pts / 8)));
    PKD_TRY(cin.need(static_cast<size_t>(D + 1) * std::max<int64_t>(R_pts, 1)));
    const int64_t ccap = std::max<int64_t>(R_pts, 1);
    // entries of the gather: the output positions (insert) or the regions'
    // old points (delete)
    const int64_t gtot = insert ? R_pts : static_cast<int64_t>(R_old32);
    if (R_pts > 0 && gtot > 0)
      hipLaunchKernelGGL(k_gather_regions<D>, dim3(static_cast<unsigned>((gtot + kFlatChunk - 1) / kFlatChunk)),
                         dim3(256), 0, st, regions.p, n_regions, insert ? comp32.p : ocomp32.p, gtot, comp32.p, Xold,
                         old_cap, ev, wf.p, m, insert ? 1 : 0, cin.p, ccap);
    PKD_TRY(kernel_status("k_gather_regions"));
    tmp.t->node_count = n_regions;
    tmp.t->height = 0;
    PKD_TRY(build_tasks_dev(tmp.t, st, roots.p, n_regions, 2, cin.p, cin.p + static_cast<int64_t>(D) * ccap, ccap));
    tmp.t->n = R_pts;
    appended = tmp.t->node_count - n_regions;
    if (static_cast<int64_t>(T->node_count) + appended >= INT32_MAX) return PKD_ERR_UNSUPPORTED;
    PKD_TRY(ensure_nodes(T, st, static_cast<int64_t>(T->node_count) + appended));
  }

  // ---- commit (kernels only; every allocation above has succeeded)
  if (n_sizes > 0)
    hipLaunchKernelGGL(k_apply_sizes, dim3(std::min(1024, (n_sizes + 255) / 256)), dim3(256), 0, st, T->nodes,
                       sizes.p, d_sizes);
  PKD_TRY(kernel_status("k_apply_sizes"));
  if (T->node_count > 0) {
    const unsigned g = static_cast<unsigned>(
        std::min<int64_t>(65536, (T->node_count + 256 * kNodesPerThread - 1) / (256 * kNodesPerThread)));
    hipLaunchKernelGGL(k_node_update, dim3(g), dim3(256), 0, st, T->nodes, T->node_count, ev, regions.p,
                       insert ? 1 : 0, n);
    PKD_TRY(kernel_status("k_node_update"));
  }
  if (n_regions > 0) {
    pkd_tree* Z = tmp.t;
    if (R_pts > 0) {
      hipLaunchKernelGGL(k_scatter_back<D>, dim3(static_cast<unsigned>((R_pts + kFlatChunk - 1) / kFlatChunk)),
                         dim3(256), 0, st, regions.p, comp32.p, n_regions, R_pts, Z->buf[Z->cur], Z->cap, Ynew,
                         new_cap, c32_new);
      PKD_TRY(kernel_status("k_scatter_back"));
    }
    const int32_t base = T->node_count;
    if (appended > 0) {
      const unsigned g = static_cast<unsigned>(std::min<int64_t>(65536, (appended + 255) / 256));
      hipLaunchKernelGGL(k_append_nodes, dim3(g), dim3(256), 0, st, T->nodes, base, Z->nodes, Z->node_count,
                         regions.p, dcomp.p, n_regions);
      PKD_TRY(kernel_status("k_append_nodes"));
    }
    hipLaunchKernelGGL(k_copy_roots, dim3((n_regions + 255) / 256), dim3(256), 0, st, T->nodes, base, Z->nodes,
                       regions.p, dcomp.p, n_regions);
    PKD_TRY(kernel_status("k_copy_roots"));
    T->node_count = base + appended;
    T->height = std::max(T->height, Z->height);
  }
  PKD_HIP(hipStreamSynchronize(st));
  // the new arrays become the tree's; the old ones its twins
  if (fresh_twin) {
    dev_free(T->buf[0], st);
    dev_free(T->buf[1], st);
    T->buf[0] = Ynew;
    T->buf[1] = fresh_twin;
    own.p[0] = own.p[1] = nullptr;
    T->cur = 0;
    T->cap = new_cap;
  } else {
    T->cur = 1 - T->cur;
  }
  if (own.p[2]) {
    dev_free(T->c32_twin, st);
    own.p[2] = nullptr;
  }
  std::swap(T->c32, c32_new);
  T->c32_twin = c32_new;
  T->c32_twin_cap = T->c32_cap;
  T->c32_cap = new_cap;
  T->n = n_new;
  T->last_regions = n_regions;
  T->last_rebuilt = R_pts;
  // reclaim the records of replaced nodes once they outnumber the rest
  // (optional: a tree that cannot get the memory keeps them)
  (void)compact_nodes(T, st);
  refresh_boxes(T, st);
  return PKD_OK;
}

// ---- node compaction: live records move down in order, links renumbered
__global__ void k_live_flags(const Node* nodes, int32_t n, int32_t* live) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    live[i] = nodes[i].pad == 0 ? 1 : 0;
}

__global__ void k_compact(const Node* src, int32_t n, const int32_t* newid, Node* dst) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    Node nd = src[i];
    if (nd.pad != 0) continue;
    if (nd.left >= 0 && nd.left < n && nd.right >= 0 && nd.right < n) {
      nd.left = newid[nd.left];
      nd.right = newid[nd.right];
    }
    dst[newid[i]] = nd;
  }
}

}  // namespace

int compact_nodes(pkd_tree* T, hipStream_t st) {
  const int32_t n = T->node_count;
  if (n < 2 * std::max<int32_t>(T->compact_mark, 1024)) return PKD_OK;
  DArr<int32_t> live(st), newid(st), bsum(st);
  if (live.need(n) != PKD_OK || newid.need(static_cast<size_t>(n) + 1) != PKD_OK) return PKD_OK;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>(65536, (n + 255) / 256));
  hipLaunchKernelGGL(k_live_flags, dim3(g), dim3(256), 0, st, T->nodes, n, live.p);
  PKD_TRY(kernel_status("k_live_flags"));
  if (exscan_i32(st, live.p, newid.p, n, bsum) != PKD_OK) return PKD_OK;
  int32_t total = 0;
  PKD_HIP(hipMemcpyAsync(&total, newid.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));
  if (total < T->n_trees || total > n) return PKD_ERR_INTERNAL;
  const int64_t cap = std::max<int64_t>(1024, static_cast<int64_t>(total) + total / 4);
  void* q = nullptr;
  if (dev_alloc(&q, sizeof(Node) * cap, st) != PKD_OK) return PKD_OK;
  hipLaunchKernelGGL(k_compact, dim3(g), dim3(256), 0, st, T->nodes, n, newid.p, static_cast<Node*>(q));
  const int rc = kernel_status("k_compact");
  if (rc != PKD_OK) {
    dev_free(q, st);
    return rc;
  }
  dev_free(T->nodes, st);
  T->nodes = static_cast<Node*>(q);
  T->node_cap = cap;
  T->node_count = total;
  T->compact_mark = total;
  return PKD_OK;
}

int run_insert(pkd_tree* T, int32_t tree, hipStream_t st, const int64_t* coords, const int64_t* ids, int64_t m) {
  int64_t dummy = 0;
  switch (T->prm.D) {
    case 1: return update_d<1>(T, tree, st, coords, ids, m, true, &dummy);
    case 2: return update_d<2>(T, tree, st, coords, ids, m, true, &dummy);
    case 3: return update_d<3>(T, tree, st, coords, ids, m, true, &dummy);
    case 4: return update_d<4>(T, tree, st, coords, ids, m, true, &dummy);
    case 5: return update_d<5>(T, tree, st, coords, ids, m, true, &dummy);
    case 6: return update_d<6>(T, tree, st, coords, ids, m, true, &dummy);
    case 7: return update_d<7>(T, tree, st, coords, ids, m, true, &dummy);
    case 8: return update_d<8>(T, tree, st, coords, ids, m, true, &dummy);
    case 9: return update_d<9>(T, tree, st, coords, ids, m, true, &dummy);
  }
  return PKD_ERR_UNSUPPORTED;
}

int run_delete(pkd_tree* T, int32_t tree, hipStream_t st, const int64_t* coords, const int64_t* ids, int64_t m,
               int64_t* removed) {
  *removed = 0;
  switch (T->prm.D) {
    case 1: return update_d<1>(T, tree, st, coords, ids, m, false, removed);
    case 2: return update_d<2>(T, tree, st, coords, ids, m, false, removed);
    case 3: return update_d<3>(T, tree, st, coords, ids, m, false, removed);
    case 4: return update_d<4>(T, tree, st, coords, ids, m, false, removed);
    case 5: return update_d<5>(T, tree, st, coords, ids, m, false, removed);
    case 6: return update_d<6>(T, tree, st, coords, ids, m, false, removed);
    case 7: return update_d<7>(T, tree, st, coords, ids, m, false, removed);
    case 8: return update_d<8>(T, tree, st, coords, ids, m, false, removed);
    case 9: return update_d<9>(T, tree, st, coords, ids, m, false, removed);
  }
  return PKD_ERR_UNSUPPORTED;
}

}  // namespace pkd
