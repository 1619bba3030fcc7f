// Range report (Section 2 query; Section 5: a subtree whose cell lies inside
// the box is reported whole, a leaf that straddles it is filtered).  Subtrees
// are contiguous slices of the tree's point array (in-order leaf order), so
// flattening a contained subtree is a contiguous copy of its ids.
//
//   walk    one wave per box finds the box's contained subtrees and the hits
//           of its straddling leaves (lanes descend independently, the wave
//           handles what they found together) and records them as copy
//           items with their positions inside the box; the box's count is
//           the total
//   scan    an exclusive scan of the counts places each box's output
//   copy    one wave per item
// The ids of a box land in its range in no particular order.
#include <algorithm>

#include "pkd_internal.h"

namespace pkd {

namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 4096;     // ids per copy record


__device__ inline void wave_sync_r() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- int64 exclusive prefix sum: out[i] = in[0] + .. + in[i-1], out[n] = total
constexpr int kScanPer = 2048;

__global__ void __launch_bounds__(kBlock) k_scan64_blocks(const int64_t* in, int64_t n, int64_t* bsum) {
  __shared__ int64_t part[kBlock];
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kScanPer;
  int64_t s = 0;
  for (int64_t i = b0 + threadIdx.x; i < min<int64_t>(n, b0 + kScanPer); i += kBlock) s += in[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = part[0];
}

// exclusive scan of nb block sums by one workgroup (runs of nb/256 per thread)
__global__ void __launch_bounds__(kBlock) k_scan64_sums(int64_t* bsum, int64_t nb) {
  __shared__ int64_t tot[kBlock];
  const int tid = threadIdx.x;
  const int64_t per = (nb + kBlock - 1) / kBlock;
  const int64_t b = tid * per, e = min(nb, b + per);
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += bsum[i];
  tot[tid] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int t = 0; t < kBlock; ++t) {
      const int64_t x = tot[t];
      tot[t] = run;
      run += x;
    }
  }
  __syncthreads();
  int64_t run = tot[tid];
  for (int64_t i = b; i < e; ++i) {
    const int64_t x = bsum[i];
    bsum[i] = run;
    run += x;
  }
}

__global__ void __launch_bounds__(kBlock) k_scan64_apply(const int64_t* in, int64_t n, const int64_t* bsum,
                                                         int64_t* out) {
  __shared__ int64_t tsum[kBlock];
  const int tid = threadIdx.x;
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kScanPer;
  constexpr int per = kScanPer / kBlock;
  int64_t v[per];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    const int64_t i = b0 + tid * per + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  tsum[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int o = 1; o < kBlock; o <<= 1) {
    const int64_t y = tid >= o ? tsum[tid - o] : 0;
    __syncthreads();
    tsum[tid] += y;
    __syncthreads();
  }
  int64_t run = bsum[blockIdx.x] + tsum[tid] - s;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    const int64_t i = b0 + tid * per + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == kBlock - 1) out[n] = run;
}

int exscan_i64(hipStream_t st, const int64_t* in, int64_t* out, int64_t n, DArr<int64_t>& bsum) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanPer - 1) / kScanPer);
  PKD_TRY(bsum.need(nb + 1));
  hipLaunchKernelGGL(k_scan64_blocks, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, st, in, n, bsum.p);
  PKD_TRY(kernel_status("k_scan64_blocks"));
  hipLaunchKernelGGL(k_scan64_sums, dim3(1), dim3(kBlock), 0, st, bsum.p, nb);
  PKD_TRY(kernel_status("k_scan64_sums"));
  hipLaunchKernelGGL(k_scan64_apply, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, st, in, n, bsum.p, out);
  return kernel_status("k_scan64_apply");
}

// ---- walk: one wave per box.  Lanes hold cells of the box: first a
// breadth-first expansion over the lanes (while the next level fits in 64
// lanes), then a depth-first walk per lane with a private stack.  The walk
// alternates between a descent loop (every lane advances until it holds a
// contained subtree or a straddling leaf, or has nothing left) and a joint
// loop in which the whole wave handles the held pieces one after another: a
// contained subtree becomes copy items of at most kChunk ids, a straddling
// leaf is tested 64 points at a time (coalesced) and its hits become an item
// with a hit mask.  Every item carries its position inside the box's output;
// the box's count is where the positions end.
struct Item {
  int32_t box;
  int32_t src;    // first position in the tree's point array
  int32_t len;    // ids covered (mask == 0: all of them)
  int32_t rel;    // first output position inside the box
  uint64_t mask;  // leaf chunk: bit i set = point src + i is in the box
};

template <int D>
__device__ inline bool point_in(const int32_t* __restrict__ C32, int64_t cap, int64_t i, const int32_t (&lo)[D],
                                const int32_t (&hi)[D]) {
  bool in = true;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int32_t v = C32[i * D + d];
    in &= v >= lo[d] && v <= hi[d];
  }
  return in;
}

struct Held {      // a piece a lane holds for the joint loop
  int32_t src, len;
  bool leaf;       // straddling leaf (else a contained subtree or heavy leaf)
};

// Item slots of one wave: taken from the global list kSlotBlock at a time
// (one atomic per block instead of one per item; a single counter hit by
// every item serializes); slots a wave does not fill become empty items.
constexpr int kSlotBlock = 256;
struct Slots {
  unsigned long long at = 0, end = 0;   // wave-uniform
};

__device__ inline void mark_empty(Item* items, int64_t item_cap, unsigned long long a, unsigned long long e) {
  const int lane = threadIdx.x & 63;
  for (unsigned long long r = a + lane; r < e; r += 64)
    if (r < static_cast<unsigned long long>(item_cap)) items[r] = Item{0, 0, 0, 0, 0};
}

__device__ inline unsigned long long take_slots(Slots& S, int k, Item* items, unsigned long long* n_items,
                                                int64_t item_cap) {
  if (S.at + k > S.end) {
    mark_empty(items, item_cap, S.at, S.end);
    const unsigned long long want = k > kSlotBlock ? static_cast<unsigned long long>(k) : kSlotBlock;
    unsigned long long a = 0;
    if ((threadIdx.x & 63) == 0) a = atomicAdd(n_items, want);
    a = __shfl(a, 0);
    S.at = a;
    S.end = a + want;
  }
  const unsigned long long r = S.at;
  S.at += k;
  return r;
}

// Joint loop: the wave handles every held piece; pos (wave-uniform) is the
// box's output position so far.
template <int D>
__device__ inline void handle_held(bool has, const Held& h, int box, const int32_t* __restrict__ C32, int64_t cap,
                                   const int32_t (&lo)[D], const int32_t (&hi)[D], int64_t& pos, Item* items,
                                   unsigned long long* n_items, int64_t item_cap, Slots& S) {
  const int lane = threadIdx.x & 63;
  unsigned long long hm = __ballot(has);
  while (hm) {
    const int l = __ffsll(static_cast<long long>(hm)) - 1;
    hm &= hm - 1;
    const int32_t src = __shfl(h.src, l), len = __shfl(h.len, l);
    const bool leaf = __shfl(static_cast<int>(h.leaf), l) != 0;
    if (!leaf) {
      const int nrec = (len + kChunk - 1) / kChunk;
      const unsigned long long at = take_slots(S, nrec, items, n_items, item_cap);
      for (int r = lane; r < nrec; r += 64)
        if (at + r < static_cast<unsigned long long>(item_cap))
          items[at + r] = Item{box, src + r * kChunk, min(kChunk, len - r * kChunk),
                               static_cast<int32_t>(pos + static_cast<int64_t>(r) * kChunk), 0};
      pos += len;
      continue;
    }
    for (int32_t c0 = 0; c0 < len; c0 += 64) {
      const int32_t i = c0 + lane;
      const bool in = i < len && point_in<D>(C32, cap, src + i, lo, hi);
      const unsigned long long m = __ballot(in);
      if (m) {
        const unsigned long long at = take_slots(S, 1, items, n_items, item_cap);
        if (lane == 0 && at < static_cast<unsigned long long>(item_cap))
          items[at] = Item{box, src + c0, min(64, len - c0), static_cast<int32_t>(pos), m};
        pos += __popcll(m);
      }
    }
  }
}

// What one cell contributes: returns 1 if the lane now holds a piece, 2 if
// the cell is a straddling interior node (children to visit), 0 otherwise.
template <int D>
__device__ inline int classify(const Node& nd, bool inside, const int32_t* __restrict__ C32, int64_t cap,
                               const int32_t (&lo)[D], const int32_t (&hi)[D], int phi, int64_t n_pts, Held* h,
                               int* fail) {
  const bool leaf = nd.left < 0;
  if (!leaf && !inside) return 2;
  if (nd.off < 0 || nd.size < 0 || static_cast<int64_t>(nd.off) + nd.size > n_pts) {
    *fail |= kErrInternal;
    return 0;
  }
  if (nd.size == 0) return 0;
  // a leaf larger than phi holds identical points: one decides for all
  if (inside || (nd.size > phi && point_in<D>(C32, cap, nd.off, lo, hi))) {
    *h = Held{nd.off, nd.size, false};
    return 1;
  }
  if (nd.size > phi) return 0;
  *h = Held{nd.off, nd.size, true};
  return 1;
}

template <int D, int SD>
__global__ void __launch_bounds__(kBlock) k_report_walk(const Node* __restrict__ nodes,
                                                        const int32_t* __restrict__ C32, int64_t cap,
                                                        const int64_t* __restrict__ Lo,
                                                        const int64_t* __restrict__ Hi, int64_t nb,
                                                        const int32_t* tree_of, int32_t n_trees, int phi,
                                                        int32_t n_nodes, int64_t n_pts, int64_t* counts, Item* items,
                                                        unsigned long long* n_items, int64_t item_cap,
                                                        unsigned long long* next_box, int* flags,
                                                        const int32_t* __restrict__ bbox) {
  constexpr int WPB = kBlock / 64;
  constexpr int EW = 1 + 2 * D;   // words of a frontier cell: node, lo[D], hi[D]
  __shared__ int32_t frontier[WPB][64 * EW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t* F = frontier[wave];
  Slots S;
  // a resident set of waves takes boxes from a counter (boxes differ in cost
  // by orders of magnitude), so item slots are shared by all boxes of a wave
  while (true) {
    unsigned long long jj = 0;
    if (lane == 0) jj = atomicAdd(next_box, 1ULL);
    const int64_t j = static_cast<int64_t>(__shfl(jj, 0));
    if (j >= nb) break;
    int32_t lo[D], hi[D];
    bool bad = false, none = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t l = Lo[d * nb + j], u = Hi[d * nb + j];
      bad |= static_cast<uint64_t>(l) >= static_cast<uint64_t>(kCoordLimit);
      bad |= static_cast<uint64_t>(u) >= static_cast<uint64_t>(kCoordLimit);
      none |= l > u;
      lo[d] = static_cast<int32_t>(l);
      hi[d] = static_cast<int32_t>(u);
    }
    if (bad) {
      if (lane == 0) atomicOr(flags, kErrRange);
      continue;
    }
    const int32_t root = tree_of ? tree_of[j] : 0;
    if (static_cast<uint32_t>(root) >= static_cast<uint32_t>(n_trees)) {
      if (lane == 0) atomicOr(flags, kErrInternal);
      continue;
    }
    int64_t pos = 0;
    bool have = lane == 0 && !none;
    int32_t node = root, clo[D], chi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      clo[d] = 0;
      chi[d] = static_cast<int32_t>(kCoordMax);
    }
    if (bbox) node_box<D>(bbox, root, clo, chi);
    int fail = 0;
    int32_t steps = 0;
    Node nd;
    // breadth-first expansion over the lanes
    while (true) {
      bool expand = false, holds = false;
      Held h{0, 0, false};
      if (have) {
        bool inside = true, disjoint = false;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          disjoint |= chi[d] < lo[d] || clo[d] > hi[d];
          inside &= clo[d] >= lo[d] && chi[d] <= hi[d];
        }
        if (static_cast<uint32_t>(node) >= static_cast<uint32_t>(n_nodes)) {
          fail |= kErrInternal;
        } else if (!disjoint) {
          nd = nodes[node];
          const int c = classify<D>(nd, inside, C32, cap, lo, hi, phi, n_pts, &h, &fail);
          holds = c == 1;
          expand = c == 2;
        }
        have = false;
      }
      handle_held<D>(holds, h, static_cast<int>(j), C32, cap, lo, hi, pos, items, n_items, item_cap, S);
      const unsigned long long em = __ballot(expand);
      const int total = 2 * __popcll(em);
      // a valid tree has at most n_nodes levels: the bound only stops a corrupt one
      if (total == 0 || total > 64 || ++steps > n_nodes) {
        have = expand;   // cells whose children are still to be visited: walked below
        break;
      }
      if (expand) {
        const int at = 2 * __popcll(em & ((1ULL << lane) - 1));
        int32_t* l = F + at * EW;        // left child: hi[dim] = x - 1
        int32_t* r = F + (at + 1) * EW;  // right child: lo[dim] = x
        l[0] = nd.left;
        r[0] = nd.right;
        if (bbox) {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            l[1 + d] = bbox[static_cast<int64_t>(nd.left) * 2 * D + d];
            l[1 + D + d] = bbox[static_cast<int64_t>(nd.left) * 2 * D + D + d];
            r[1 + d] = bbox[static_cast<int64_t>(nd.right) * 2 * D + d];
            r[1 + D + d] = bbox[static_cast<int64_t>(nd.right) * 2 * D + D + d];
          }
        } else {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            l[1 + d] = clo[d];
            l[1 + D + d] = (nd.dim == d) ? static_cast<int32_t>(nd.x - 1) : chi[d];
            r[1 + d] = (nd.dim == d) ? static_cast<int32_t>(nd.x) : clo[d];
            r[1 + D + d] = chi[d];
          }
        }
      }
      wave_sync_r();
      have = lane < total;
      if (have) {
        const int32_t* e = F + lane * EW;
        node = e[0];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          clo[d] = e[1 + d];
          chi[d] = e[1 + D + d];
        }
      }
      wave_sync_r();
    }
    // depth-first walk below the cells that still straddle: descent loop and
    // joint loop in turn
    struct Ent {
      int32_t node;
      int32_t clo[D], chi[D];
    };
    Ent stk[SD];
    int sp = 0;
    if (have) {
      if (bbox) {
        node_box<D>(bbox, nd.right, stk[0].clo, stk[0].chi);
        node_box<D>(bbox, nd.left, stk[1].clo, stk[1].chi);
      } else {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          stk[0].clo[d] = (nd.dim == d) ? static_cast<int32_t>(nd.x) : clo[d];
          stk[0].chi[d] = chi[d];
          stk[1].clo[d] = clo[d];
          stk[1].chi[d] = (nd.dim == d) ? static_cast<int32_t>(nd.x - 1) : chi[d];
        }
      }
      stk[0].node = nd.right;
      stk[1].node = nd.left;
      sp = 2;
    }
    int32_t visits = 0;
    bool done = sp == 0;
    while (true) {
      bool holds = false;
      Held h{0, 0, false};
#pragma unroll 1
      while (true) {
        const bool want = !done && !holds;
        if (__ballot(want) == 0) break;
        if (!want) continue;
        if (sp == 0) {
          done = true;
          continue;
        }
        --sp;
        const int32_t v = stk[sp].node;
        if (static_cast<uint32_t>(v) >= static_cast<uint32_t>(n_nodes) || ++visits > n_nodes) {
          fail |= kErrInternal;
          done = true;
          continue;
        }
        int32_t a[D], b[D];
        bool inside = true, disjoint = false;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          a[d] = stk[sp].clo[d];
          b[d] = stk[sp].chi[d];
          disjoint |= b[d] < lo[d] || a[d] > hi[d];
          inside &= a[d] >= lo[d] && b[d] <= hi[d];
        }
        if (disjoint) continue;
        const Node w = nodes[v];
        const int c = classify<D>(w, inside, C32, cap, lo, hi, phi, n_pts, &h, &fail);
        if (c == 1) {
          holds = true;
          continue;
        }
        if (c == 0) continue;
        if (sp + 2 > SD) {
          fail |= kErrStack;
          done = true;
          continue;
        }
        if (bbox) {
          node_box<D>(bbox, w.right, stk[sp].clo, stk[sp].chi);
          node_box<D>(bbox, w.left, stk[sp + 1].clo, stk[sp + 1].chi);
        } else {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            stk[sp].clo[d] = (w.dim == d) ? static_cast<int32_t>(w.x) : a[d];
            stk[sp].chi[d] = b[d];
            stk[sp + 1].clo[d] = a[d];
            stk[sp + 1].chi[d] = (w.dim == d) ? static_cast<int32_t>(w.x - 1) : b[d];
          }
        }
        stk[sp].node = w.right;
        stk[sp + 1].node = w.left;
        sp += 2;
      }
      if (__ballot(holds) == 0) break;
      handle_held<D>(holds, h, static_cast<int>(j), C32, cap, lo, hi, pos, items, n_items, item_cap, S);
    }
    const unsigned long long fm = __ballot(fail != 0);
    if (fm) {
      if (fail) atomicOr(flags, fail);
      continue;
    }
    if (lane == 0) counts[j] = pos;
  }
  mark_empty(items, item_cap, S.at, S.end);
}

// One wave per item: copy a contained run of ids, or a leaf chunk's hits in
// order of their bits.
__global__ void __launch_bounds__(kBlock) k_report_copy(const Item* items, const unsigned long long* n_items,
                                                        int64_t item_cap, const int64_t* offsets,
                                                        const int64_t* __restrict__ ids, int64_t* __restrict__ out) {
  const int64_t n = min(static_cast<int64_t>(*n_items), item_cap);
  const int lane = threadIdx.x & 63;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBlock / 64);
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6); r < n; r += waves) {
    const Item it = items[r];
    int64_t* dst = out + offsets[it.box] + it.rel;
    if (it.mask == 0) {
      for (int i = lane; i < it.len; i += 64) dst[i] = ids[it.src + i];
    } else if ((it.mask >> lane) & 1) {
      dst[__popcll(it.mask & ((1ULL << lane) - 1))] = ids[it.src + lane];
    }
  }
}

// workgroups of the walk: enough resident waves to fill the chip
constexpr int64_t kWalkBlocks = 2048;

template <int D>
int report_walk_d(const pkd_tree* T, hipStream_t st, const int64_t* lo, const int64_t* hi, const int32_t* tree_of,
                  int64_t nb, int64_t* counts, Item* items, unsigned long long* n_items, int64_t item_cap,
                  unsigned long long* next_box, int* flags) {
  const int64_t need = (nb + kBlock / 64 - 1) / (kBlock / 64);
  const dim3 g(static_cast<unsigned>(std::min<int64_t>(need, kWalkBlocks)));
#define PKD_WALK(SD)                                                                                              \
  hipLaunchKernelGGL((k_report_walk<D, SD>), g, dim3(kBlock), 0, st, T->nodes, T->c32, T->cap, lo, hi, nb,       \
                     tree_of, T->n_trees, T->prm.phi, T->node_count, T->n, counts, items, n_items, item_cap,    \
                     next_box, flags, T->bbox_on ? T->bbox : nullptr);
  if (T->height + 3 <= 48) {
    PKD_WALK(48)
  } else if (T->height + 3 <= kMaxStack) {
    PKD_WALK(kMaxStack)
  } else {
    return PKD_ERR_CAPACITY;
  }
#undef PKD_WALK
  return kernel_status("k_report_walk");
}

int read_flags(int* f, hipStream_t st) {
  int h = 0;
  PKD_HIP(hipMemcpyAsync(&h, f, sizeof(int), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));
  if (h & kErrRange) return PKD_ERR_RANGE;
  if (h & kErrStack) return PKD_ERR_CAPACITY;
  if (h) return PKD_ERR_INTERNAL;
  return PKD_OK;
}

}  // namespace

int run_range_report(const pkd_tree* T, hipStream_t st, const int64_t* lo, const int64_t* hi, const int32_t* tree_of,
                     int64_t nb, int64_t* offsets, int64_t* out_ids, int64_t cap, int64_t* total) {
  DArr<int> flags(st);
  DArr<int64_t> cnt(st), bsum(st);
  DArr<unsigned long long> nitems(st);
  DArr<Item> items(st);
  PKD_TRY(flags.need(4));
  PKD_TRY(cnt.need(nb));
  PKD_TRY(nitems.need(2));   // [0] item slots taken, [1] next box of the walk
  // the item list of the previous call sizes this one's (a second walk runs
  // only when the list overflows, with the exact size)
  int64_t item_cap = std::max<int64_t>(T->report_items_hint, std::max<int64_t>(int64_t{1} << 20, 64 * nb));
  unsigned long long used = 0;
  Prof::begin(kProfReport, st);
  for (int attempt = 0; attempt < 2; ++attempt) {
    PKD_TRY(items.need(item_cap));
    PKD_HIP(hipMemsetAsync(flags.p, 0, sizeof(int) * 4, st));
    PKD_HIP(hipMemsetAsync(nitems.p, 0, 2 * sizeof(unsigned long long), st));
    int rc = PKD_ERR_UNSUPPORTED;
    switch (T->prm.D) {
#define PKD_RW(DD)                                                                                        \
  case DD:                                                                                                \
    rc = report_walk_d<DD>(T, st, lo, hi, tree_of, nb, cnt.p, items.p, nitems.p, item_cap, nitems.p + 1, flags.p); \
    break;
      PKD_RW(1) PKD_RW(2) PKD_RW(3) PKD_RW(4) PKD_RW(5) PKD_RW(6) PKD_RW(7) PKD_RW(8) PKD_RW(9)
#undef PKD_RW
    }
    PKD_TRY(rc);
    PKD_TRY(exscan_i64(st, cnt.p, offsets, nb, bsum));
    PKD_HIP(hipMemcpyAsync(total, offsets + nb, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PKD_HIP(hipMemcpyAsync(&used, nitems.p, sizeof(used), hipMemcpyDeviceToHost, st));
    PKD_TRY(read_flags(flags.p, st));
    if (used <= static_cast<unsigned long long>(item_cap)) break;
    if (attempt == 1) return PKD_ERR_INTERNAL;
    // waves take boxes dynamically, so the slots a run leaves empty vary from
    // run to run: a slot is left empty only when a group of items larger than
    // what is left of a wave's block arrives (fewer empties than items), or
    // at a wave's end (less than a block), so this always suffices
    item_cap = 2 * static_cast<int64_t>(used) + kWalkBlocks * (kBlock / 64) * kSlotBlock;
  }
  T->report_items_hint = static_cast<int64_t>(used) + static_cast<int64_t>(used) / 4 +
                         kWalkBlocks * (kBlock / 64) * kSlotBlock;
  if (!out_ids) return PKD_OK;
  if (*total > cap) return PKD_ERR_CAPACITY;
  if (used > 0) {
    const int64_t* ids = T->buf[T->cur] + static_cast<int64_t>(T->prm.D) * T->cap;
    const unsigned g = static_cast<unsigned>(std::min<unsigned long long>((used + 3) / 4, 1u << 20));
    hipLaunchKernelGGL(k_report_copy, dim3(g), dim3(kBlock), 0, st, items.p, nitems.p, item_cap, offsets, ids,
                       out_ids);
    PKD_TRY(kernel_status("k_report_copy"));
  }
  Prof::end(kProfReport, st, 16.0 * static_cast<double>(*total));
  PKD_HIP(hipStreamSynchronize(st));
  return PKD_OK;
}

}  // namespace pkd
