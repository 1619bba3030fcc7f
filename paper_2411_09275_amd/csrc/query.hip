// k-NN and range-count queries on a built Pkd-tree (Section 2 definitions,
// Section 5 traversals).  One lane per query; the subspace of a node is not
// stored but derived on the way down from the splitters (no bounding boxes,
// Section 5).
#include "pkd_internal.h"

namespace pkd {

int dev_alloc(void** p, size_t bytes, hipStream_t s);

namespace {

constexpr int kQBlock = 256;

__device__ inline bool pair_less(int64_t d2, int64_t id, int64_t cd2, int64_t cid) {
  return d2 < cd2 || (d2 == cd2 && id < cid);
}

// Exact k nearest (squared distance, id) pairs, k <= KM, candidates kept as a
// sorted array in registers.  The first KM-k slots hold sentinels that are
// smaller than any real pair, so the k-th best is always slot KM-1.
// Depth-first: the nearer child first; the farther child is stacked with the
// lower bound of its subspace (squared distance from q to the cell, updated
// incrementally in the split dimension) and skipped when that bound exceeds
// the current k-th distance (strictly: an equal distance may still win on id).
template <int D, int KM, int SD>
__global__ void __launch_bounds__(kQBlock) k_knn(const Node* __restrict__ nodes, const int64_t* __restrict__ X,
                                                 int64_t cap, const int64_t* __restrict__ ids,
                                                 const int64_t* __restrict__ Qry, int64_t nq, int k,
                                                 int64_t* __restrict__ out_ids, int64_t* __restrict__ out_d2,
                                                 int* flags, const int32_t* tree_of, int32_t n_trees,
                                                 int32_t n_nodes, int64_t n_pts) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kQBlock + threadIdx.x;
  if (j >= nq) return;
  int64_t q[D];
  bool bad = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    q[d] = Qry[d * nq + j];
    bad |= static_cast<uint64_t>(q[d]) >= static_cast<uint64_t>(kCoordLimit);
  }
  if (bad) {
    atomicOr(flags, kErrRange);
    return;
  }
  int64_t bd[KM], bi[KM];
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    bd[i] = (i < KM - k) ? -1 : INT64_MAX;
    bi[i] = (i < KM - k) ? INT64_MIN : INT64_MAX;
  }

  struct Ent {
    int32_t node;
    int32_t depth;
    int32_t off[D];
    int64_t lb;
  };
  // the trees of a handle have their roots at nodes 0 .. n_trees-1; an empty
  // tree's root is a leaf of size 0
  const int32_t root = tree_of ? tree_of[j] : 0;
  if (static_cast<uint32_t>(root) >= static_cast<uint32_t>(n_trees)) {
    atomicOr(flags, kErrInternal);
    return;
  }
  Ent stk[SD];
  stk[0].node = root;
  stk[0].depth = 0;
  stk[0].lb = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) stk[0].off[d] = 0;
  int sp = 1;
  while (sp > 0) {
    --sp;
    int32_t node = stk[sp].node;
    int32_t depth = stk[sp].depth;
    int64_t lb = stk[sp].lb;
    int32_t off[D];
#pragma unroll
    for (int d = 0; d < D; ++d) off[d] = stk[sp].off[d];
    if (lb > bd[KM - 1]) continue;
    while (true) {
      // the links of a valid tree stay inside the node array and no path is
      // longer than the stack: anything else stops this lane with an error
      if (static_cast<uint32_t>(node) >= static_cast<uint32_t>(n_nodes) || depth >= SD) {
        atomicOr(flags, kErrInternal);
        return;
      }
      const Node nd = nodes[node];
      if (nd.left < 0) {
        const int64_t e = static_cast<int64_t>(nd.off) + nd.size;
        if (nd.off < 0 || nd.size < 0 || e > n_pts) {
          atomicOr(flags, kErrInternal);
          return;
        }
        for (int64_t i = nd.off; i < e; ++i) {
          int64_t d2 = 0;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const int64_t diff = X[d * cap + i] - q[d];
            d2 += diff * diff;
          }
          if (d2 <= bd[KM - 1]) {
            const int64_t id = ids[i];
            if (pair_less(d2, id, bd[KM - 1], bi[KM - 1])) {
#pragma unroll
              for (int t = KM - 1; t > 0; --t) {
                const bool shift = pair_less(d2, id, bd[t - 1], bi[t - 1]);
                const bool here = !shift && pair_less(d2, id, bd[t], bi[t]);
                bd[t] = shift ? bd[t - 1] : (here ? d2 : bd[t]);
                bi[t] = shift ? bi[t - 1] : (here ? id : bi[t]);
              }
              const bool first = pair_less(d2, id, bd[0], bi[0]);
              bd[0] = first ? d2 : bd[0];
              bi[0] = first ? id : bi[0];
            }
          }
        }
        break;
      }
      int64_t qd = q[0];
      int32_t od = off[0];
#pragma unroll
      for (int d = 1; d < D; ++d) {
        qd = (nd.dim == d) ? q[d] : qd;
        od = (nd.dim == d) ? off[d] : od;
      }
      const bool go_left = qd < nd.x;
      const int32_t near = go_left ? nd.left : nd.right;
      const int32_t far = go_left ? nd.right : nd.left;
      const int64_t fo = go_left ? nd.x - qd : qd - nd.x + 1;   // distance to the far cell in this dim
      const int64_t flb = lb - static_cast<int64_t>(od) * od + fo * fo;
      if (flb <= bd[KM - 1]) {
        if (sp >= SD) {
          atomicOr(flags, kErrStack);
          return;
        }
        stk[sp].node = far;
        stk[sp].depth = depth + 1;
        stk[sp].lb = flb;
#pragma unroll
        for (int d = 0; d < D; ++d) stk[sp].off[d] = (nd.dim == d) ? static_cast<int32_t>(fo) : off[d];
        ++sp;
      }
      node = near;
      ++depth;
    }
  }
  for (int i = 0; i < k; ++i) {
    // slot KM-k+i holds the i-th nearest; unfilled slots are +inf
    int64_t cd = bd[0], ci = bi[0];
#pragma unroll
    for (int t = 1; t < KM; ++t) {
      cd = (t == KM - k + i) ? bd[t] : cd;
      ci = (t == KM - k + i) ? bi[t] : ci;
    }
    const bool have = cd != INT64_MAX;
    out_d2[j * k + i] = have ? cd : -1;
    out_ids[j * k + i] = have ? ci : -1;
  }
}

// Range count: a node whose cell lies inside the box contributes its stored
// subtree size; a disjoint cell contributes nothing; leaves are scanned.
template <int D, int SD>
__global__ void __launch_bounds__(kQBlock) k_range(const Node* __restrict__ nodes, const int64_t* __restrict__ X,
                                                   int64_t cap, const int64_t* __restrict__ Lo,
                                                   const int64_t* __restrict__ Hi, int64_t nb, int64_t* out,
                                                   int* flags, const int32_t* tree_of, int32_t n_trees, int phi,
                                                   int32_t n_nodes, int64_t n_pts) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kQBlock + threadIdx.x;
  if (j >= nb) return;
  int64_t lo[D], hi[D];
  bool bad = false, none = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    lo[d] = Lo[d * nb + j];
    hi[d] = Hi[d * nb + j];
    bad |= static_cast<uint64_t>(lo[d]) >= static_cast<uint64_t>(kCoordLimit);
    bad |= static_cast<uint64_t>(hi[d]) >= static_cast<uint64_t>(kCoordLimit);
    none |= lo[d] > hi[d];
  }
  if (bad) {
    atomicOr(flags, kErrRange);
    return;
  }
  int64_t count = 0;
  struct Ent {
    int32_t node;
    int32_t depth;
    int32_t clo[D], chi[D];
  };
  Ent stk[SD];
  int sp = 0;
  const int32_t root = tree_of ? tree_of[j] : 0;
  if (static_cast<uint32_t>(root) >= static_cast<uint32_t>(n_trees)) {
    atomicOr(flags, kErrInternal);
    return;
  }
  if (!none) {
    stk[0].node = root;
    stk[0].depth = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      stk[0].clo[d] = 0;
      stk[0].chi[d] = static_cast<int32_t>(kCoordMax);
    }
    sp = 1;
  }
  while (sp > 0) {
    --sp;
    const int32_t node = stk[sp].node;
    const int32_t depth = stk[sp].depth;
    if (static_cast<uint32_t>(node) >= static_cast<uint32_t>(n_nodes) || depth >= SD) {
      atomicOr(flags, kErrInternal);
      return;
    }
    int32_t clo[D], chi[D];
    bool inside = true, disjoint = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      clo[d] = stk[sp].clo[d];
      chi[d] = stk[sp].chi[d];
      disjoint |= chi[d] < lo[d] || clo[d] > hi[d];
      inside &= clo[d] >= lo[d] && chi[d] <= hi[d];
    }
    if (disjoint) continue;
    const Node nd = nodes[node];
    if (inside) {
      count += nd.size;
      continue;
    }
    if (nd.left < 0) {
      if (nd.off < 0 || nd.size < 0 || static_cast<int64_t>(nd.off) + nd.size > n_pts) {
        atomicOr(flags, kErrInternal);
        return;
      }
      // a leaf larger than phi holds identical points: test one of them
      const int64_t e = nd.size > phi ? static_cast<int64_t>(nd.off) + 1 : static_cast<int64_t>(nd.off) + nd.size;
      int64_t c = 0;
      for (int64_t i = nd.off; i < e; ++i) {
        bool in = true;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int64_t v = X[d * cap + i];
          in &= v >= lo[d] && v <= hi[d];
        }
        c += in ? 1 : 0;
      }
      count += nd.size > phi ? c * nd.size : c;
      continue;
    }
    if (sp + 2 > SD) {
      atomicOr(flags, kErrStack);
      return;
    }
    // right child: lo[dim] = x; left child: hi[dim] = x - 1
#pragma unroll
    for (int d = 0; d < D; ++d) {
      stk[sp].clo[d] = (nd.dim == d) ? static_cast<int32_t>(nd.x) : clo[d];
      stk[sp].chi[d] = chi[d];
      stk[sp + 1].clo[d] = clo[d];
      stk[sp + 1].chi[d] = (nd.dim == d) ? static_cast<int32_t>(nd.x - 1) : chi[d];
    }
    stk[sp].node = nd.right;
    stk[sp + 1].node = nd.left;
    stk[sp].depth = depth + 1;
    stk[sp + 1].depth = depth + 1;
    sp += 2;
  }
  out[j] = count;
}

template <int D, int SD>
void launch_knn(int km, dim3 g, hipStream_t st, const Node* nodes, const int64_t* X, int64_t cap,
                const int64_t* ids, const int64_t* q, int64_t nq, int k, int64_t* oi, int64_t* od, int* flags,
                const int32_t* tree_of, int32_t n_trees, int32_t n_nodes, int64_t n_pts) {
#define PKD_KNN_CASE(KM) \
  case KM:               \
    hipLaunchKernelGGL((k_knn<D, KM, SD>), g, dim3(kQBlock), 0, st, nodes, X, cap, ids, q, nq, k, oi, od, flags, \
                       tree_of, n_trees, n_nodes, n_pts); \
    break;
  switch (km) {
    PKD_KNN_CASE(1)
    PKD_KNN_CASE(2)
    PKD_KNN_CASE(4)
    PKD_KNN_CASE(8)
    PKD_KNN_CASE(16)
    PKD_KNN_CASE(32)
    PKD_KNN_CASE(64)
    PKD_KNN_CASE(128)
  }
#undef PKD_KNN_CASE
}

template <int D>
int knn_d(const pkd_tree* T, hipStream_t st, const int64_t* q, const int32_t* tree_of, int64_t nq, int k,
          int64_t* oi, int64_t* od, int* flags) {
  int km = 1;
  while (km < k) km <<= 1;
  const dim3 g(static_cast<unsigned>((nq + kQBlock - 1) / kQBlock));
  const int64_t* X = T->buf[T->cur];
  const int64_t* ids = X + static_cast<int64_t>(D) * T->cap;
  if (T->height + 2 <= 48)
    launch_knn<D, 48>(km, g, st, T->nodes, X, T->cap, ids, q, nq, k, oi, od, flags, tree_of, T->n_trees,
                      T->node_count, T->n);
  else if (T->height + 2 <= 96)
    launch_knn<D, 96>(km, g, st, T->nodes, X, T->cap, ids, q, nq, k, oi, od, flags, tree_of, T->n_trees,
                      T->node_count, T->n);
  else if (T->height + 2 <= kMaxStack)
    launch_knn<D, kMaxStack>(km, g, st, T->nodes, X, T->cap, ids, q, nq, k, oi, od, flags, tree_of, T->n_trees,
                             T->node_count, T->n);
  else
    return PKD_ERR_CAPACITY;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "k_knn");
  return PKD_OK;
}

template <int D>
int range_d(const pkd_tree* T, hipStream_t st, const int64_t* lo, const int64_t* hi, const int32_t* tree_of,
            int64_t nb, int64_t* out, int* flags) {
  const dim3 g(static_cast<unsigned>((nb + kQBlock - 1) / kQBlock));
  const int64_t* X = T->buf[T->cur];
  if (T->height + 3 <= 48)
    hipLaunchKernelGGL((k_range<D, 48>), g, dim3(kQBlock), 0, st, T->nodes, X, T->cap, lo, hi, nb, out, flags, tree_of,
                       T->n_trees, T->prm.phi, T->node_count, T->n);
  else if (T->height + 3 <= kMaxStack)
    hipLaunchKernelGGL((k_range<D, kMaxStack>), g, dim3(kQBlock), 0, st, T->nodes, X, T->cap, lo, hi, nb, out, flags,
                       tree_of, T->n_trees, T->prm.phi, T->node_count, T->n);
  else
    return PKD_ERR_CAPACITY;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "k_range");
  return PKD_OK;
}

}  // namespace

int run_knn(const pkd_tree* T, hipStream_t st, const int64_t* q, const int32_t* tree_of, int64_t nq, int k,
            int64_t* oi, int64_t* od, int* flags) {
  switch (T->prm.D) {
    case 1: return knn_d<1>(T, st, q, tree_of, nq, k, oi, od, flags);
    case 2: return knn_d<2>(T, st, q, tree_of, nq, k, oi, od, flags);
    case 3: return knn_d<3>(T, st, q, tree_of, nq, k, oi, od, flags);
    case 4: return knn_d<4>(T, st, q, tree_of, nq, k, oi, od, flags);
    case 5: return knn_d<5>(T, st, q, tree_of, nq, k, oi, od, flags);
    case 6: return knn_d<6>(T, st, q, tree_of, nq, k, oi, od, flags);
    case 7: return knn_d<7>(T, st, q, tree_of, nq, k, oi, od, flags);
  }
  return PKD_ERR_UNSUPPORTED;
}

int run_range(const pkd_tree* T, hipStream_t st, const int64_t* lo, const int64_t* hi, const int32_t* tree_of,
              int64_t nb, int64_t* out, int* flags) {
  switch (T->prm.D) {
    case 1: return range_d<1>(T, st, lo, hi, tree_of, nb, out, flags);
    case 2: return range_d<2>(T, st, lo, hi, tree_of, nb, out, flags);
    case 3: return range_d<3>(T, st, lo, hi, tree_of, nb, out, flags);
    case 4: return range_d<4>(T, st, lo, hi, tree_of, nb, out, flags);
    case 5: return range_d<5>(T, st, lo, hi, tree_of, nb, out, flags);
    case 6: return range_d<6>(T, st, lo, hi, tree_of, nb, out, flags);
    case 7: return range_d<7>(T, st, lo, hi, tree_of, nb, out, flags);
  }
  return PKD_ERR_UNSUPPORTED;
}

}  // namespace pkd
