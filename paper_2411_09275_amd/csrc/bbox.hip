// Bounding boxes of the tree's nodes (the Pkd-bb variant of Section 6.3):
// the Pkd-tree keeps no boxes and derives each node's cell from the splitters
// on the way down; with boxes on, every live node also stores the tight box
// of its points (int32 [node][lo 0..D-1, hi 0..D-1]) and the query kernels
// prune and decide containment with it.  Results are the same either way;
// the boxes trade memory and box loads for fewer visited nodes.
//
// The boxes are computed bottom-up: live nodes are sorted by depth, deepest
// first (the library's radix sort), and each depth is one launch: a leaf
// reduces its slice of the packed coordinates, an interior node joins its
// children's boxes.  An empty node's box is empty (lo = 2^31-1, hi = -1).
#include <algorithm>

#include "pkd_internal.h"

namespace pkd {

namespace {

constexpr int kHistLds = 4096;   // depth histograms up to this many levels are gathered in LDS first

__global__ void k_bb_keys(const Node* nodes, int32_t n, int32_t maxdepth, uint64_t* key, uint32_t* val,
                          int32_t* hist) {
  __shared__ int32_t h[kHistLds];
  const bool lds = maxdepth + 1 < kHistLds;
  if (lds)
    for (int i = threadIdx.x; i <= maxdepth; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const Node nd = nodes[i];
    // dead records sort last (key maxdepth + 1) and are never processed
    const int32_t lvl = nd.pad != 0 ? maxdepth + 1 : maxdepth - min<int32_t>(nd.depth, maxdepth);
    key[i] = static_cast<uint64_t>(lvl);
    val[i] = static_cast<uint32_t>(i);
    if (nd.pad == 0) atomicAdd(lds ? h + lvl : hist + lvl, 1);
  }
  __syncthreads();
  if (lds)
    for (int i = threadIdx.x; i <= maxdepth; i += blockDim.x)
      if (h[i]) atomicAdd(hist + i, h[i]);
}

template <int D>
__global__ void k_bb_level(const Node* nodes, const uint32_t* order, int32_t count, const int32_t* C32, int64_t cap,
                           int32_t* bbox) {
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < count; r += gridDim.x * blockDim.x) {
    const int32_t v = static_cast<int32_t>(order[r]);
    const Node nd = nodes[v];
    int32_t lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      lo[d] = INT32_MAX;
      hi[d] = -1;
    }
    if (nd.left >= 0) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        lo[d] = min(bbox[static_cast<int64_t>(nd.left) * 2 * D + d], bbox[static_cast<int64_t>(nd.right) * 2 * D + d]);
        hi[d] = max(bbox[static_cast<int64_t>(nd.left) * 2 * D + D + d],
                    bbox[static_cast<int64_t>(nd.right) * 2 * D + D + d]);
      }
    } else {
      // a leaf of more than phi points holds identical points; the loop over
      // all of them gives the same box
      for (int32_t i = 0; i < nd.size; ++i) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int32_t c = C32[(static_cast<int64_t>(nd.off) + i) * D + d];
          lo[d] = min(lo[d], c);
          hi[d] = max(hi[d], c);
        }
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      bbox[static_cast<int64_t>(v) * 2 * D + d] = lo[d];
      bbox[static_cast<int64_t>(v) * 2 * D + D + d] = hi[d];
    }
  }
}

template <int D>
int compute_bbox_d(pkd_tree* T, hipStream_t st) {
  const int32_t n = T->node_count;
  if (!T->bbox || T->bbox_cap < T->node_cap) {
    void* p = nullptr;
    PKD_TRY(dev_alloc(&p, sizeof(int32_t) * 2 * D * static_cast<size_t>(T->node_cap), st));
    dev_free(T->bbox, st);
    T->bbox = static_cast<int32_t*>(p);
    T->bbox_cap = T->node_cap;
  }
  if (n == 0) return PKD_OK;
  // depths of live nodes are at most the tree's height (trees of a batch
  // handle all have their roots at depth 0)
  const int32_t maxdepth = std::max<int32_t>(T->height, 0);
  DArr<uint64_t> key(st);
  DArr<uint32_t> val(st);
  DArr<int32_t> hist(st), start(st), bsum(st);
  SortWork W(st);
  PKD_TRY(key.need(n));
  PKD_TRY(val.need(n));
  PKD_TRY(hist.need(static_cast<size_t>(maxdepth) + 2));
  PKD_TRY(start.need(static_cast<size_t>(maxdepth) + 3));
  PKD_HIP(hipMemsetAsync(hist.p, 0, sizeof(int32_t) * (maxdepth + 2), st));
  const unsigned g = static_cast<unsigned>(std::min<int64_t>(2048, (n + 255) / 256));
  hipLaunchKernelGGL(k_bb_keys, dim3(g), dim3(256), 0, st, T->nodes, n, maxdepth, key.p, val.p, hist.p);
  PKD_TRY(kernel_status("k_bb_keys"));
  uint64_t* ks = nullptr;
  uint32_t* vs = nullptr;
  PKD_TRY(radix_sort_pairs(st, key.p, val.p, n, bits_for(maxdepth + 1), W, &ks, &vs));
  PKD_TRY(exscan_i32(st, hist.p, start.p, maxdepth + 2, bsum));
  std::vector<int32_t> hs(static_cast<size_t>(maxdepth) + 3);
  PKD_HIP(hipMemcpyAsync(hs.data(), start.p, sizeof(int32_t) * (maxdepth + 3), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));
  for (int32_t lvl = 0; lvl <= maxdepth; ++lvl) {   // level 0 holds the deepest nodes
    const int32_t count = hs[lvl + 1] - hs[lvl];
    if (count <= 0) continue;
    const unsigned gl = static_cast<unsigned>(std::min<int64_t>(65536, (count + 255) / 256));
    hipLaunchKernelGGL(k_bb_level<D>, dim3(gl), dim3(256), 0, st, T->nodes, vs + hs[lvl], count, T->c32, T->c32_cap,
                       T->bbox);
    PKD_TRY(kernel_status("k_bb_level"));
  }
  PKD_HIP(hipStreamSynchronize(st));
  return PKD_OK;
}

}  // namespace

int compute_bbox(pkd_tree* T, hipStream_t st) {
  switch (T->prm.D) {
    case 1: return compute_bbox_d<1>(T, st);
    case 2: return compute_bbox_d<2>(T, st);
    case 3: return compute_bbox_d<3>(T, st);
    case 4: return compute_bbox_d<4>(T, st);
    case 5: return compute_bbox_d<5>(T, st);
    case 6: return compute_bbox_d<6>(T, st);
    case 7: return compute_bbox_d<7>(T, st);
    case 8: return compute_bbox_d<8>(T, st);
    case 9: return compute_bbox_d<9>(T, st);
  }
  return PKD_ERR_UNSUPPORTED;
}

}  // namespace pkd
