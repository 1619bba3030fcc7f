// k-NN and range-count queries on a built Pkd-tree (Section 2 definitions,
// Section 5 traversals).  k-NN with k <= 32 and large batches of range counts
// run one lane per query; k-NN with larger k and smaller batches of range
// counts run one wave per query.  The subspace of a node is not stored but
// derived on the way down from the splitters (no bounding boxes, Section 5).
#include <algorithm>
#include <mutex>

#include "pkd_internal.h"

namespace pkd {

namespace {

constexpr int kQBlock = 256;

__device__ inline bool pair_less(int64_t d2, int64_t id, int64_t cd2, int64_t cid) {
  return d2 < cd2 || (d2 == cd2 && id < cid);
}

// Exact k nearest (squared distance, id) pairs for k <= 32, one lane per
// query: k <= KM (10 for k = 9, 10, else a power of two up to 32), candidates kept as a
// sorted array in registers.  The first KM-k slots hold sentinels that are
// smaller than any real pair, so the k-th best is always slot KM-1.
// Depth-first: the nearer child first; the farther child is stacked with the
// lower bound of its subspace (squared distance from q to the cell, updated
// incrementally in the split dimension) and skipped when that bound exceeds
// the current k-th distance (strictly: an equal distance may still win on id).
// The lanes of a wave alternate between two loops: every lane descends until
// it holds a leaf (or has nothing left), then all scan their leaves together,
// so a leaf scan is paid once per round rather than once per node step.
// Coordinates lie in [0, 2^30): differences fit 32 bits, and the leaves are
// scanned in the tree's packed 32-bit copy of its coordinates.
constexpr int kLeafBatch = 4;

template <int D, int KM, int SD>
__global__ void __launch_bounds__(kQBlock) __attribute__((amdgpu_waves_per_eu(KM == 16 ? 3 : (KM == 32 ? 2 : 1)))) k_knn(const Node* __restrict__ nodes, const int32_t* __restrict__ C32,
                                                 int64_t cap, const int64_t* __restrict__ ids,
                                                 const int64_t* __restrict__ Qry, int64_t nq, int k,
                                                 int64_t* __restrict__ out_ids, int64_t* __restrict__ out_d2,
                                                 int* flags, const int32_t* tree_of, int32_t n_trees,
                                                 int32_t n_nodes, int64_t n_pts, const uint32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ bbox) {
  const int64_t j0 = static_cast<int64_t>(blockIdx.x) * kQBlock + threadIdx.x;
  if (j0 >= nq) return;
  const int64_t j = perm ? static_cast<int64_t>(perm[j0]) : j0;   // lanes of a wave take nearby queries
  int32_t q[D];
  bool bad = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int64_t v = Qry[d * nq + j];
    bad |= static_cast<uint64_t>(v) >= static_cast<uint64_t>(coord_limit(D));
    q[d] = static_cast<int32_t>(v);
  }
  if (bad) {
    atomicOr(flags, kErrRange);
    return;
  }
  // the k best pairs sorted in registers; slots 0..KM-k-1 hold sentinels
  // smaller than any pair
  constexpr int KR = KM;
  int64_t bd[KR], bi[KR];
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    bd[i] = (i < KM - k) ? -1 : INT64_MAX;
    bi[i] = (i < KM - k) ? INT64_MIN : INT64_MAX;
  }

  // a stacked cell: its node and its per-dimension distances from q; the
  // lower bound is their sum of squares, recomputed when the entry is taken
  struct Ent {
    int32_t node;
    int32_t off[D];
  };
  // the trees of a handle have their roots at nodes 0 .. n_trees-1; an empty
  // tree's root is a leaf of size 0
  const int32_t root = tree_of ? tree_of[j] : 0;
  if (static_cast<uint32_t>(root) >= static_cast<uint32_t>(n_trees)) {
    atomicOr(flags, kErrInternal);
    return;
  }
  // a node is stacked at most once per level of the current path, so a valid
  // tree never needs more than its height
  Ent stk[SD];
  int sp = 0;
  int32_t node = root;      // node being descended, -1: take the next stacked one
  int64_t lb = 0;
  int32_t off[D];
  // per-dimension distance from q to a box (0 inside its range)
  auto box_off = [&](int32_t v, int32_t (&o)[D]) -> int64_t {
    int64_t s2 = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int32_t lo = bbox[static_cast<int64_t>(v) * 2 * D + d], hi = bbox[static_cast<int64_t>(v) * 2 * D + D + d];
      o[d] = q[d] < lo ? lo - q[d] : (q[d] > hi ? q[d] - hi : 0);
      s2 += static_cast<int64_t>(o[d]) * o[d];
    }
    return s2;
  };
#pragma unroll
  for (int d = 0; d < D; ++d) off[d] = 0;
  if (bbox) lb = box_off(root, off);
  int32_t leaf_off = 0, leaf_size = 0;
  bool have_leaf = false, done = false;
  int fail_bits = 0;
  int32_t visits = 0;
  while (true) {
    // descend: one pop or one node step per iteration, until every lane holds
    // a leaf or is finished
#pragma unroll 1
    while (true) {
      const bool want = !done && !have_leaf;
      if (__ballot(want) == 0) break;
      if (!want) continue;
      if (node < 0) {
        if (sp == 0) {
          done = true;
          continue;
        }
        --sp;
        node = stk[sp].node;
        lb = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          off[d] = stk[sp].off[d];
          lb += static_cast<int64_t>(off[d]) * off[d];
        }
        if (lb > bd[KR - 1]) {
          node = -1;
          continue;
        }
      }
      // the links of a valid tree stay inside the node array and a traversal
      // visits every node at most once: anything else stops this lane
      if (static_cast<uint32_t>(node) >= static_cast<uint32_t>(n_nodes) || ++visits > n_nodes) {
        fail_bits = kErrInternal;
        done = true;
        continue;
      }
      const Node nd = nodes[node];
      if (nd.left < 0) {
        if (nd.off < 0 || nd.size < 0 || static_cast<int64_t>(nd.off) + nd.size > n_pts) {
          fail_bits = kErrInternal;
          done = true;
          continue;
        }
        leaf_off = nd.off;
        leaf_size = nd.size;
        have_leaf = true;
        node = -1;
        continue;
      }
      int32_t qd = q[0], od = off[0];
#pragma unroll
      for (int d = 1; d < D; ++d) {
        qd = (nd.dim == d) ? q[d] : qd;
        od = (nd.dim == d) ? off[d] : od;
      }
      const bool go_left = qd < nd.x;
      const int32_t near = go_left ? nd.left : nd.right;
      const int32_t far = go_left ? nd.right : nd.left;
      if (bbox) {
        // both children by their own boxes: the far one is stacked, the near
        // one descended, each only while its bound can still win
        int32_t fo_[D];
        const int64_t fl = box_off(far, fo_);
        if (fl <= bd[KR - 1]) {
          if (sp >= SD) {
            fail_bits = kErrStack;
            done = true;
            continue;
          }
          stk[sp].node = far;
#pragma unroll
          for (int d = 0; d < D; ++d) stk[sp].off[d] = fo_[d];
          ++sp;
        }
        lb = box_off(near, off);
        node = lb > bd[KR - 1] ? -1 : near;
        continue;
      }
      // distance to the far cell in this dimension (the splitter is a stored
      // coordinate, so it fits 32 bits)
      const int64_t fo = go_left ? nd.x - qd : static_cast<int64_t>(qd) - nd.x + 1;
      const int64_t flb = lb - static_cast<int64_t>(od) * od + fo * fo;
      if (flb <= bd[KR - 1]) {
        if (sp >= SD) {
          fail_bits = kErrStack;
          done = true;
          continue;
        }
        stk[sp].node = far;
#pragma unroll
        for (int d = 0; d < D; ++d) stk[sp].off[d] = (nd.dim == d) ? static_cast<int32_t>(fo) : off[d];
        ++sp;
      }
      node = near;
    }
    if (__ballot(have_leaf) == 0) break;
    if (have_leaf) {
      auto consider = [&](int64_t d2, int64_t i) {
        if (d2 <= bd[KR - 1]) {
          const int64_t id = ids[i];
          if (pair_less(d2, id, bd[KR - 1], bi[KR - 1])) {
            // drop the worst, then bubble the new pair down
            bd[KR - 1] = d2;
            bi[KR - 1] = id;
#pragma unroll
            for (int t = KR - 1; t > 0; --t) {
              const bool sw = pair_less(bd[t], bi[t], bd[t - 1], bi[t - 1]);
              const int64_t x0 = bd[t - 1], y0 = bi[t - 1];
              bd[t - 1] = sw ? bd[t] : x0;
              bi[t - 1] = sw ? bi[t] : y0;
              bd[t] = sw ? x0 : bd[t];
              bi[t] = sw ? y0 : bi[t];
            }
          }
        }
      };
      const int64_t e = static_cast<int64_t>(leaf_off) + leaf_size;
      int64_t i = leaf_off;
      // LB points' coordinates are loaded before the first is tested, so
      // their loads are in flight together (more of them when the list is
      // short and registers are free)
      constexpr int LB = KM <= 4 ? 2 * kLeafBatch : kLeafBatch;
#pragma unroll 1
      for (; i + LB <= e; i += LB) {
        int64_t d2[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) d2[u] = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            const int32_t diff = C32[(i + u) * D + d] - q[d];
            d2[u] += static_cast<int64_t>(diff) * diff;
          }
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) consider(d2[u], i + u);
      }
#pragma unroll 1
      for (; i < e; ++i) {
        int64_t d2 = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int32_t diff = C32[i * D + d] - q[d];
          d2 += static_cast<int64_t>(diff) * diff;
        }
        consider(d2, i);
      }
      have_leaf = false;
    }
  }
  if (fail_bits) {
    atomicOr(flags, fail_bits);
    return;
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

// --------------------------------------------------------- k-NN, larger k
// k = 33..128: one wave answers one query.  The wave walks a single
// path (every lane takes the same branch, so nothing diverges), its 64 lanes
// scan a leaf's points together, and the k best pairs are one sorted list in
// the wave's LDS.  A leaf's accepted pairs are sorted across the wave by a
// bitonic network and merged into the list (each pair's new place is its own
// index plus its rank in the other sorted sequence).  Traversal order, the
// pruning bound and the tie rule are those of k_knn, so the results are the
// same (the k best pairs are unique).
struct WaveKnnLayout {
  size_t ld0, li0, ld1, li1, cd, ci, stk, end;   // byte offsets inside one wave's slice
  __host__ __device__ WaveKnnLayout(int D, int SD, int k) {
    size_t o = 0;
    ld0 = o; o += sizeof(int64_t) * k;
    li0 = o; o += sizeof(int64_t) * k;
    ld1 = o; o += sizeof(int64_t) * k;
    li1 = o; o += sizeof(int64_t) * k;
    cd = o;  o += sizeof(int64_t) * 64;
    ci = o;  o += sizeof(int64_t) * 64;
    stk = o; o += sizeof(int32_t) * SD * (1 + D);
    end = (o + 15) & ~size_t{15};
  }
};

__device__ inline int64_t shfl_xor_i64(int64_t v, int mask) {
  const int lo = __shfl_xor(static_cast<int>(static_cast<uint32_t>(v)), mask);
  const int hi = __shfl_xor(static_cast<int>(static_cast<uint64_t>(v) >> 32), mask);
  return static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo));
}

// Ascending bitonic sort of one (d2, id) pair per lane across the wave.
__device__ inline void wave_sort_pairs(int64_t& d2, int64_t& id) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int j = size >> 1; j > 0; j >>= 1) {
      const int64_t od = shfl_xor_i64(d2, j), oi = shfl_xor_i64(id, j);
      const bool keep_min = ((lane & j) == 0) == ((lane & size) == 0);
      const bool take = keep_min ? pair_less(od, oi, d2, id) : pair_less(d2, id, od, oi);
      d2 = take ? od : d2;
      id = take ? oi : id;
    }
  }
}

constexpr int kFewPairs = 4;   // a leaf adding at most this many pairs skips the sort

template <int D, int SD>
__global__ void __launch_bounds__(kQBlock) k_knn_wave(const Node* __restrict__ nodes, const int32_t* __restrict__ C32,
                                                      int64_t cap, const int64_t* __restrict__ ids,
                                                      const int64_t* __restrict__ Qry, int64_t nq, int k,
                                                      int64_t* __restrict__ out_ids, int64_t* __restrict__ out_d2,
                                                      int* flags, const int32_t* tree_of, int32_t n_trees,
                                                      int32_t n_nodes, int64_t n_pts, const uint32_t* __restrict__ perm) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int WPB = kQBlock / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const WaveKnnLayout lay(D, SD, k);
  unsigned char* mine = smem + wave * lay.end;
  int64_t* Ld[2] = {reinterpret_cast<int64_t*>(mine + lay.ld0), reinterpret_cast<int64_t*>(mine + lay.ld1)};
  int64_t* Li[2] = {reinterpret_cast<int64_t*>(mine + lay.li0), reinterpret_cast<int64_t*>(mine + lay.li1)};
  int64_t* Cd = reinterpret_cast<int64_t*>(mine + lay.cd);
  int64_t* Ci = reinterpret_cast<int64_t*>(mine + lay.ci);
  int32_t* stk = reinterpret_cast<int32_t*>(mine + lay.stk);   // [SD][1 + D]: node, then offsets
  const int64_t waves = static_cast<int64_t>(gridDim.x) * WPB;
  for (int64_t j0 = static_cast<int64_t>(blockIdx.x) * WPB + wave; j0 < nq; j0 += waves) {
    const int64_t j = perm ? static_cast<int64_t>(perm[j0]) : j0;
    int32_t q[D];
    bool bad = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t v = Qry[d * nq + j];
      bad |= static_cast<uint64_t>(v) >= static_cast<uint64_t>(coord_limit(D));
      q[d] = static_cast<int32_t>(v);
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
    int cur = 0;
    for (int e = lane; e < k; e += 64) {
      Ld[0][e] = INT64_MAX;
      Li[0][e] = INT64_MAX;
    }
    wave_sync();
    int64_t wd = INT64_MAX, wi = INT64_MAX;   // the k-th best pair so far
    int sp = 0;
    int32_t node = root;
    int64_t lb = 0;
    int32_t off[D];
#pragma unroll
    for (int d = 0; d < D; ++d) off[d] = 0;
    int32_t visits = 0;
    int fail_bits = 0;
    while (true) {
      if (node < 0) {
        if (sp == 0) break;
        --sp;
        node = stk[sp * (1 + D)];
        lb = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          off[d] = stk[sp * (1 + D) + 1 + d];
          lb += static_cast<int64_t>(off[d]) * off[d];
        }
        if (lb > wd) {
          node = -1;
          continue;
        }
      }
      if (static_cast<uint32_t>(node) >= static_cast<uint32_t>(n_nodes) || ++visits > n_nodes) {
        fail_bits = kErrInternal;
        break;
      }
      const Node nd = nodes[node];
      if (nd.left < 0) {
        if (nd.off < 0 || nd.size < 0 || static_cast<int64_t>(nd.off) + nd.size > n_pts) {
          fail_bits = kErrInternal;
          break;
        }
        const int64_t e = static_cast<int64_t>(nd.off) + nd.size;
        for (int64_t b = nd.off; b < e; b += 64) {
          const int64_t i = b + lane;
          int64_t d2 = INT64_MAX, id = INT64_MAX;
          bool acc = false;
          if (i < e) {
            int64_t s = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
              const int32_t diff = C32[i * D + d] - q[d];
              s += static_cast<int64_t>(diff) * diff;
            }
            if (s <= wd) {
              const int64_t x = ids[i];
              if (pair_less(s, x, wd, wi)) {
                acc = true;
                d2 = s;
                id = x;
              }
            }
          }
          const unsigned long long am = __ballot(acc);
          if (am == 0) continue;
          const int c = __popcll(am);
          const int nx = cur ^ 1;
          if (c <= kFewPairs) {
            // few pairs: no sort.  They are compacted to slots 0..c-1; every
            // list entry moves up by the pairs below it, and pair u lands
            // after the list entries not above it and the pairs before it
            // (ties: list entries first, then pairs by slot).  k <= 128, so
            // lane l holds list entries l and l + 64.
            if (acc) {
              const int r = __popcll(am & ((1ULL << lane) - 1));
              Cd[r] = d2;
              Ci[r] = id;
            }
            wave_sync();
            int64_t pd[kFewPairs], pi[kFewPairs];
#pragma unroll
            for (int u = 0; u < kFewPairs; ++u) {
              pd[u] = u < c ? Cd[u] : INT64_MAX;
              pi[u] = u < c ? Ci[u] : INT64_MAX;
            }
            int mypos = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int t = lane + 64 * h;
              const bool have = t < k;
              const int64_t xd = have ? Ld[cur][t] : INT64_MAX, xi = have ? Li[cur][t] : INT64_MAX;
              int below = 0;
#pragma unroll
              for (int u = 0; u < kFewPairs; ++u) below += (u < c && pair_less(pd[u], pi[u], xd, xi)) ? 1 : 0;
              if (have && t + below < k) {
                Ld[nx][t + below] = xd;
                Li[nx][t + below] = xi;
              }
#pragma unroll
              for (int u = 0; u < kFewPairs; ++u) {
                if (u < c) {
                  const int n_le = __popcll(__ballot(have && !pair_less(pd[u], pi[u], xd, xi)));
                  mypos += lane == u ? n_le : 0;
                }
              }
            }
            if (lane < c) {
              int64_t sd = pd[0], si = pi[0];
#pragma unroll
              for (int u = 1; u < kFewPairs; ++u) {
                sd = lane == u ? pd[u] : sd;
                si = lane == u ? pi[u] : si;
              }
              int before = 0;
#pragma unroll
              for (int u = 0; u < kFewPairs; ++u)
                before += (u < c && (pair_less(pd[u], pi[u], sd, si) || (u < lane && pd[u] == sd && pi[u] == si)))
                              ? 1 : 0;
              if (mypos + before < k) {
                Ld[nx][mypos + before] = sd;
                Li[nx][mypos + before] = si;
              }
            }
            wave_sync();
            cur = nx;
            wd = Ld[cur][k - 1];
            wi = Li[cur][k - 1];
            continue;
          }
          wave_sort_pairs(d2, id);   // the c accepted pairs come first
          Cd[lane] = d2;
          Ci[lane] = id;
          wave_sync();
          for (int t = lane; t < k; t += 64) {
            // list entry t moves up by the candidates below it
            const int64_t xd = Ld[cur][t], xi = Li[cur][t];
            int lo = 0, hi = c;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (pair_less(Cd[mid], Ci[mid], xd, xi)) lo = mid + 1; else hi = mid;
            }
            if (t + lo < k) {
              Ld[nx][t + lo] = xd;
              Li[nx][t + lo] = xi;
            }
          }
          if (lane < c) {
            // candidate `lane` goes after every list entry not above it
            int lo = 0, hi = k;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (pair_less(d2, id, Ld[cur][mid], Li[cur][mid])) hi = mid; else lo = mid + 1;
            }
            if (lane + lo < k) {
              Ld[nx][lane + lo] = d2;
              Li[nx][lane + lo] = id;
            }
          }
          wave_sync();
          cur = nx;
          wd = Ld[cur][k - 1];
          wi = Li[cur][k - 1];
        }
        node = -1;
        continue;
      }
      int32_t qd = q[0], od = off[0];
#pragma unroll
      for (int d = 1; d < D; ++d) {
        qd = (nd.dim == d) ? q[d] : qd;
        od = (nd.dim == d) ? off[d] : od;
      }
      const bool go_left = qd < nd.x;
      const int32_t near = go_left ? nd.left : nd.right;
      const int32_t far = go_left ? nd.right : nd.left;
      const int64_t fo = go_left ? nd.x - qd : static_cast<int64_t>(qd) - nd.x + 1;
      const int64_t flb = lb - static_cast<int64_t>(od) * od + fo * fo;
      if (flb <= wd) {
        if (sp >= SD) {
          fail_bits = kErrStack;
          break;
        }
        stk[sp * (1 + D)] = far;
#pragma unroll
        for (int d = 0; d < D; ++d) stk[sp * (1 + D) + 1 + d] = (nd.dim == d) ? static_cast<int32_t>(fo) : off[d];
        ++sp;
      }
      node = near;
    }
    if (fail_bits) {
      if (lane == 0) atomicOr(flags, fail_bits);
      wave_sync();
      continue;
    }
    for (int t = lane; t < k; t += 64) {
      const int64_t cd = Ld[cur][t];
      const bool have = cd != INT64_MAX;
      out_d2[j * k + t] = have ? cd : -1;
      out_ids[j * k + t] = have ? Li[cur][t] : -1;
    }
    wave_sync();   // the next query rewrites the list
  }
}

// Range count: a node whose cell lies inside the box contributes its stored
// subtree size; a disjoint cell contributes nothing; leaves are scanned.  As
// in k-NN, the lanes descend until each holds a leaf that straddles its box,
// then scan those leaves together.  range_walk counts the box's points in the
// subtree of one starting cell per lane (start = false: nothing to count);
// every lane of the wave calls it.
// Points among [off, off+n) of the packed coordinates that lie in the box;
// kLeafBatch points' loads are issued before the first is tested.
template <int D>
__device__ inline int64_t count_in_box(const int32_t* __restrict__ C32, int64_t cap, int64_t off, int64_t n,
                                       const int32_t (&lo)[D], const int32_t (&hi)[D]) {
  const int64_t e = off + n;
  int64_t c = 0, i = off;
#pragma unroll 1
  for (; i + kLeafBatch <= e; i += kLeafBatch) {
    bool in[kLeafBatch];
#pragma unroll
    for (int u = 0; u < kLeafBatch; ++u) in[u] = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
      for (int u = 0; u < kLeafBatch; ++u) {
        const int32_t v = C32[(i + u) * D + d];
        in[u] &= v >= lo[d] && v <= hi[d];
      }
    }
#pragma unroll
    for (int u = 0; u < kLeafBatch; ++u) c += in[u] ? 1 : 0;
  }
#pragma unroll 1
  for (; i < e; ++i) {
    bool in = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int32_t v = C32[i * D + d];
      in &= v >= lo[d] && v <= hi[d];
    }
    c += in ? 1 : 0;
  }
  return c;
}

template <int D, int SD>
__device__ int64_t range_walk(const Node* __restrict__ nodes, const int32_t* __restrict__ C32, int64_t cap,
                              const int32_t (&lo)[D], const int32_t (&hi)[D], int phi, int32_t n_nodes,
                              int64_t n_pts, bool start, int32_t node0, const int32_t (&clo0)[D],
                              const int32_t (&chi0)[D], int* fail_out, const int32_t* __restrict__ bbox) {
  int64_t count = 0;
  struct Ent {
    int32_t node;
    int32_t clo[D], chi[D];
  };
  Ent stk[SD];
  int sp = 0;
  if (start) {
    stk[0].node = node0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      stk[0].clo[d] = clo0[d];
      stk[0].chi[d] = chi0[d];
    }
    sp = 1;
  }
  int32_t leaf_off = 0, leaf_size = 0;
  bool have_leaf = false, done = false;
  int fail_bits = 0;
  int32_t visits = 0;
  while (true) {
#pragma unroll 1
    while (true) {
      const bool want = !done && !have_leaf;
      if (__ballot(want) == 0) break;
      if (!want) continue;
      if (sp == 0) {
        done = true;
        continue;
      }
      --sp;
      const int32_t node = stk[sp].node;
      if (static_cast<uint32_t>(node) >= static_cast<uint32_t>(n_nodes) || ++visits > n_nodes) {
        fail_bits = kErrInternal;
        done = true;
        continue;
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
          fail_bits = kErrInternal;
          done = true;
          continue;
        }
        leaf_off = nd.off;
        leaf_size = nd.size;
        have_leaf = true;
        continue;
      }
      if (sp + 2 > SD) {
        fail_bits = kErrStack;
        done = true;
        continue;
      }
      if (bbox) {
        // the children's own boxes
        node_box<D>(bbox, nd.right, stk[sp].clo, stk[sp].chi);
        node_box<D>(bbox, nd.left, stk[sp + 1].clo, stk[sp + 1].chi);
      } else {
        // right child: lo[dim] = x; left child: hi[dim] = x - 1
#pragma unroll
        for (int d = 0; d < D; ++d) {
          stk[sp].clo[d] = (nd.dim == d) ? static_cast<int32_t>(nd.x) : clo[d];
          stk[sp].chi[d] = chi[d];
          stk[sp + 1].clo[d] = clo[d];
          stk[sp + 1].chi[d] = (nd.dim == d) ? static_cast<int32_t>(nd.x - 1) : chi[d];
        }
      }
      stk[sp].node = nd.right;
      stk[sp + 1].node = nd.left;
      sp += 2;
    }
    if (__ballot(have_leaf) == 0) break;
    if (have_leaf) {
      // a leaf larger than phi holds identical points: test one of them
      const int64_t c = count_in_box<D>(C32, cap, leaf_off, leaf_size > phi ? 1 : leaf_size, lo, hi);
      count += leaf_size > phi ? c * leaf_size : c;
      have_leaf = false;
    }
  }
  *fail_out |= fail_bits;
  return count;
}

// Reads box j; false (and the error flagged) if a corner is out of range.
template <int D>
__device__ inline bool load_box(const int64_t* __restrict__ Lo, const int64_t* __restrict__ Hi, int64_t nb, int64_t j,
                                int32_t (&lo)[D], int32_t (&hi)[D], bool* none) {
  bool bad = false;
  *none = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int64_t l = Lo[d * nb + j], h = Hi[d * nb + j];
    bad |= static_cast<uint64_t>(l) >= static_cast<uint64_t>(kCoordLimit);
    bad |= static_cast<uint64_t>(h) >= static_cast<uint64_t>(kCoordLimit);
    *none |= l > h;
    lo[d] = static_cast<int32_t>(l);
    hi[d] = static_cast<int32_t>(h);
  }
  return !bad;
}

// One lane per box (large batches).
template <int D, int SD>
__global__ void __launch_bounds__(kQBlock) k_range(const Node* __restrict__ nodes, const int32_t* __restrict__ C32,
                                                   int64_t cap, const int64_t* __restrict__ Lo,
                                                   const int64_t* __restrict__ Hi, int64_t nb, int64_t* out,
                                                   int* flags, const int32_t* tree_of, int32_t n_trees, int phi,
                                                   int32_t n_nodes, int64_t n_pts, const uint32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ bbox) {
  const int64_t j0 = static_cast<int64_t>(blockIdx.x) * kQBlock + threadIdx.x;
  if (j0 >= nb) return;
  const int64_t j = perm ? static_cast<int64_t>(perm[j0]) : j0;
  int32_t lo[D], hi[D];
  bool none;
  if (!load_box<D>(Lo, Hi, nb, j, lo, hi, &none)) {
    atomicOr(flags, kErrRange);
    return;
  }
  const int32_t root = tree_of ? tree_of[j] : 0;
  if (static_cast<uint32_t>(root) >= static_cast<uint32_t>(n_trees)) {
    atomicOr(flags, kErrInternal);
    return;
  }
  int32_t clo[D], chi[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    clo[d] = 0;
    chi[d] = static_cast<int32_t>(kCoordMax);
  }
  if (bbox) node_box<D>(bbox, root, clo, chi);
  int fail_bits = 0;
  const int64_t count = range_walk<D, SD>(nodes, C32, cap, lo, hi, phi, n_nodes, n_pts, !none, root, clo, chi,
                                          &fail_bits, bbox);
  if (fail_bits) {
    atomicOr(flags, fail_bits);
    return;
  }
  out[j] = count;
}

constexpr int64_t kRangeWaveMax = int64_t{1} << 20;

// One wave per box (smaller batches, where one lane per box would leave most
// of the chip idle and the largest box's walk would set the time).  The wave
// first expands the box's straddling cells breadth-first, one cell per lane,
// while the next level still fits in 64 lanes (contained cells add their
// size, leaves are scanned, disjoint cells drop out); then every lane walks
// the subtree of its cell with range_walk, and the lane counts are summed.
template <int D, int SD>
__global__ void __launch_bounds__(kQBlock) k_range_wave(const Node* __restrict__ nodes,
                                                        const int32_t* __restrict__ C32, int64_t cap,
                                                        const int64_t* __restrict__ Lo,
                                                        const int64_t* __restrict__ Hi, int64_t nb, int64_t* out,
                                                        int* flags, const int32_t* tree_of, int32_t n_trees, int phi,
                                                        int32_t n_nodes, int64_t n_pts,
                                                        const uint32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ bbox) {
  constexpr int WPB = kQBlock / 64;
  constexpr int EW = 1 + 2 * D;   // words of a frontier cell: node, lo[D], hi[D]
  __shared__ int32_t frontier[WPB][64 * EW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t* F = frontier[wave];
  const int64_t waves = static_cast<int64_t>(gridDim.x) * WPB;
  for (int64_t j0 = static_cast<int64_t>(blockIdx.x) * WPB + wave; j0 < nb; j0 += waves) {
    const int64_t j = perm ? static_cast<int64_t>(perm[j0]) : j0;
    int32_t lo[D], hi[D];
    bool none;
    if (!load_box<D>(Lo, Hi, nb, j, lo, hi, &none)) {
      if (lane == 0) atomicOr(flags, kErrRange);
      continue;
    }
    const int32_t root = tree_of ? tree_of[j] : 0;
    if (static_cast<uint32_t>(root) >= static_cast<uint32_t>(n_trees)) {
      if (lane == 0) atomicOr(flags, kErrInternal);
      continue;
    }
    // this lane's cell
    bool have = lane == 0 && !none;
    int32_t node = root, clo[D], chi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      clo[d] = 0;
      chi[d] = static_cast<int32_t>(kCoordMax);
    }
    if (bbox) node_box<D>(bbox, root, clo, chi);
    int64_t count = 0;
    int fail_bits = 0;
    int32_t steps = 0;
    while (true) {
      bool expand = false;
      Node nd;
      if (have) {
        bool inside = true, disjoint = false;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          disjoint |= chi[d] < lo[d] || clo[d] > hi[d];
          inside &= clo[d] >= lo[d] && chi[d] <= hi[d];
        }
        if (static_cast<uint32_t>(node) >= static_cast<uint32_t>(n_nodes)) {
          fail_bits = kErrInternal;
          have = false;
        } else if (disjoint) {
          have = false;
        } else {
          nd = nodes[node];
          if (inside) {
            count += nd.size;
            have = false;
          } else if (nd.left < 0) {
            if (nd.off < 0 || nd.size < 0 || static_cast<int64_t>(nd.off) + nd.size > n_pts) {
              fail_bits = kErrInternal;
            } else {
              const int64_t c = count_in_box<D>(C32, cap, nd.off, nd.size > phi ? 1 : nd.size, lo, hi);
              count += nd.size > phi ? c * nd.size : c;
            }
            have = false;
          } else {
            expand = true;
          }
        }
      }
      const unsigned long long em = __ballot(expand);
      const int total = 2 * __popcll(em);
      // a valid tree has at most n_nodes levels: the bound only stops a
      // corrupt one
      if (total == 0 || total > 64 || ++steps > n_nodes) break;
      if (expand) {
        const int at = 2 * __popcll(em & ((1ULL << lane) - 1));
        int32_t* r = F + at * EW;        // right child: lo[dim] = x
        int32_t* l = F + (at + 1) * EW;  // left child: hi[dim] = x - 1
        r[0] = nd.right;
        l[0] = nd.left;
        if (bbox) {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            r[1 + d] = bbox[static_cast<int64_t>(nd.right) * 2 * D + d];
            r[1 + D + d] = bbox[static_cast<int64_t>(nd.right) * 2 * D + D + d];
            l[1 + d] = bbox[static_cast<int64_t>(nd.left) * 2 * D + d];
            l[1 + D + d] = bbox[static_cast<int64_t>(nd.left) * 2 * D + D + d];
          }
        } else {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            r[1 + d] = (nd.dim == d) ? static_cast<int32_t>(nd.x) : clo[d];
            r[1 + D + d] = chi[d];
            l[1 + d] = clo[d];
            l[1 + D + d] = (nd.dim == d) ? static_cast<int32_t>(nd.x - 1) : chi[d];
          }
        }
      }
      wave_sync();
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
      wave_sync();
    }
    // the remaining cells (more than 64 children wanted): one subtree walk per lane
    count += range_walk<D, SD>(nodes, C32, cap, lo, hi, phi, n_nodes, n_pts, have, node, clo, chi, &fail_bits,
                               bbox);
    const unsigned long long fm = __ballot(fail_bits != 0);
    if (fm) {
      if (fail_bits) atomicOr(flags, fail_bits);
      continue;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) count += shfl_xor_i64(count, o);
    if (lane == 0) out[j] = count;
  }
}

// ------------------------------------------------ spatial order of queries
// A batch of queries is processed in Morton order (bits of the coordinates
// interleaved, most significant first, below the tree id of a batch handle):
// the lanes of a wave then walk neighbouring paths of the tree, which keeps
// them converged and their node and leaf loads in cache.  Results still go to
// each query's own row.  The order comes from a stable LSD radix sort
// (radix_sort_pairs).
constexpr int64_t kOrderMinQueries = 16384;  // smaller batches keep their order

template <int D>
__global__ void k_morton(const int64_t* __restrict__ Q, int64_t nq, const int32_t* __restrict__ tree_of, int bpd,
                         uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nq) return;
  uint64_t c[D];
#pragma unroll
  for (int d = 0; d < D; ++d) c[d] = static_cast<uint64_t>(Q[d * nq + j]) & static_cast<uint64_t>(kCoordMax);
  uint64_t code = tree_of ? static_cast<uint64_t>(static_cast<uint32_t>(tree_of[j])) : 0;
  for (int b = 29; b > 29 - bpd; --b)
#pragma unroll
    for (int d = 0; d < D; ++d) code = (code << 1) | ((c[d] >> b) & 1);
  key[j] = code;
  val[j] = static_cast<uint32_t>(j);
}

struct QueryOrder {
  DArr<uint64_t> k0;
  DArr<uint32_t> v0;
  SortWork sort;
  explicit QueryOrder(hipStream_t st) : k0(st), v0(st), sort(st) {}
};

// Fills *perm with the queries in Morton order, or leaves it null for small
// batches.  Stream-ordered, no host synchronisation.
// Bits of position per dimension and key bits of the Morton order.
template <int D>
void morton_bits(int64_t nq, const int32_t* tree_of, int32_t n_trees, int* bpd_out, int* nbits_out) {
  const int tb = tree_of ? bits_for(n_trees - 1) : 0;
  // about 64 cells per wave of queries: log2(nq) + 6 bits of position
  int bpd = (bits_for(nq) + 6 + D - 1) / D;
  bpd = std::min(bpd, std::min(30, (64 - tb) / D));
  *bpd_out = bpd;
  *nbits_out = tb + D * bpd;
}

template <int D>
int order_queries(hipStream_t st, const int64_t* Q, int64_t nq, const int32_t* tree_of, int32_t n_trees,
                  QueryOrder& W, const uint32_t** perm) {
  *perm = nullptr;
  // under graph capture the queries run in input order: the order would need
  // sort buffers, and it changes only the speed, never a result
  if (nq < kOrderMinQueries || capturing(st)) return PKD_OK;
  int bpd = 0, nbits = 0;
  morton_bits<D>(nq, tree_of, n_trees, &bpd, &nbits);
  PKD_TRY(W.k0.need(nq));
  PKD_TRY(W.v0.need(nq));
  hipLaunchKernelGGL(k_morton<D>, dim3(static_cast<unsigned>((nq + 255) / 256)), dim3(256), 0, st, Q, nq, tree_of,
                     bpd, W.k0.p, W.v0.p);
  PKD_TRY(kernel_status("k_morton"));
  uint64_t* ks = nullptr;
  uint32_t* vs = nullptr;
  PKD_TRY(radix_sort_pairs(st, W.k0.p, W.v0.p, nq, nbits, W.sort, &ks, &vs));
  *perm = vs;
  return PKD_OK;
}

template <int D, int SD>
void launch_knn(int km, dim3 g, hipStream_t st, const Node* nodes, const int32_t* X, int64_t cap,
                const int64_t* ids, const int64_t* q, int64_t nq, int k, int64_t* oi, int64_t* od, int* flags,
                const int32_t* tree_of, int32_t n_trees, int32_t n_nodes, int64_t n_pts, const uint32_t* perm,
                const int32_t* bbox) {
#define PKD_KNN_CASE(KM) \
  case KM:               \
    hipLaunchKernelGGL((k_knn<D, KM, SD>), g, dim3(kQBlock), 0, st, nodes, X, cap, ids, q, nq, k, oi, od, flags, \
                       tree_of, n_trees, n_nodes, n_pts, perm, bbox); \
    break;
  switch (km) {
    PKD_KNN_CASE(1)
    PKD_KNN_CASE(2)
    PKD_KNN_CASE(4)
    PKD_KNN_CASE(8)
    PKD_KNN_CASE(10)
    PKD_KNN_CASE(16)
    PKD_KNN_CASE(32)
    default: {
      // k > 32: one wave per query (measured faster than a persistent grid
      // sized to the resident workgroups: the dispatcher balances the uneven
      // query costs); the kernel still strides if the grid is capped
      const size_t lds = (kQBlock / 64) * WaveKnnLayout(D, SD, k).end;
      const int64_t need = (nq + kQBlock / 64 - 1) / (kQBlock / 64);
      const dim3 gw(static_cast<unsigned>(std::min<int64_t>(need, INT32_MAX)));
      hipLaunchKernelGGL((k_knn_wave<D, SD>), gw, dim3(kQBlock), lds, st, nodes, X, cap, ids, q, nq, k, oi, od,
                         flags, tree_of, n_trees, n_nodes, n_pts, perm);
    }
  }
#undef PKD_KNN_CASE
}

// Launches the k-NN kernel for the queries in the order `perm` (null: as given).
template <int D>
int knn_launch(const pkd_tree* T, hipStream_t st, const int64_t* q, const int32_t* tree_of, int64_t nq, int k,
               int64_t* oi, int64_t* od, int* flags, const uint32_t* perm) {
  int km = 1;
  while (km < k) km <<= 1;
  if (k == 9 || k == 10) km = 10;   // the common k = 10 without six idle slots
  const dim3 g(static_cast<unsigned>((nq + kQBlock - 1) / kQBlock));
  const int32_t* X = T->c32;
  const int64_t* ids = T->buf[T->cur] + static_cast<int64_t>(D) * T->cap;
  // stored boxes prune the one-lane kernel (k <= 32); the one-wave kernel
  // keeps the cells derived from the splitters (same results)
  const int32_t* bb = T->bbox_on ? T->bbox : nullptr;
  if (query_height(T) + 2 <= 32)
    launch_knn<D, 32>(km, g, st, T->nodes, X, T->cap, ids, q, nq, k, oi, od, flags, tree_of, T->n_trees,
                      query_nodes(T), T->n, perm, bb);
  else if (query_height(T) + 2 <= 64)
    launch_knn<D, 64>(km, g, st, T->nodes, X, T->cap, ids, q, nq, k, oi, od, flags, tree_of, T->n_trees,
                      query_nodes(T), T->n, perm, bb);
  else if (query_height(T) + 2 <= kMaxStack)
    launch_knn<D, kMaxStack>(km, g, st, T->nodes, X, T->cap, ids, q, nq, k, oi, od, flags, tree_of, T->n_trees,
                             query_nodes(T), T->n, perm, bb);
  else
    return PKD_ERR_CAPACITY;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "k_knn");
  return PKD_OK;
}

template <int D>
int knn_d(const pkd_tree* T, hipStream_t st, const int64_t* q, const int32_t* tree_of, int64_t nq, int k,
          int64_t* oi, int64_t* od, int* flags) {
  QueryOrder W(st);
  const uint32_t* perm = nullptr;
  PKD_TRY(order_queries<D>(st, q, nq, tree_of, T->n_trees, W, &perm));
  return knn_launch<D>(T, st, q, tree_of, nq, k, oi, od, flags, perm);
}

template <int D>
int range_d(const pkd_tree* T, hipStream_t st, const int64_t* lo, const int64_t* hi, const int32_t* tree_of,
            int64_t nb, int64_t* out, int* flags) {
  QueryOrder W(st);
  const uint32_t* perm = nullptr;
  PKD_TRY(order_queries<D>(st, lo, nb, tree_of, T->n_trees, W, &perm));   // boxes by their low corner
  const int32_t* X = T->c32;
  const int32_t* bb = T->bbox_on ? T->bbox : nullptr;
  // below kRangeWaveMax boxes one lane per box would fill too little of the chip
  const bool per_wave = nb < kRangeWaveMax;
  const int64_t per_block = per_wave ? kQBlock / 64 : kQBlock;
  const dim3 g(static_cast<unsigned>(std::min<int64_t>((nb + per_block - 1) / per_block, INT32_MAX)));
#define PKD_RANGE(SD)                                                                                             \
  if (per_wave)                                                                                                   \
    hipLaunchKernelGGL((k_range_wave<D, SD>), g, dim3(kQBlock), 0, st, T->nodes, X, T->cap, lo, hi, nb, out, flags, \
                       tree_of, T->n_trees, T->prm.phi, query_nodes(T), T->n, perm, bb);                            \
  else                                                                                                            \
    hipLaunchKernelGGL((k_range<D, SD>), g, dim3(kQBlock), 0, st, T->nodes, X, T->cap, lo, hi, nb, out, flags,      \
                       tree_of, T->n_trees, T->prm.phi, query_nodes(T), T->n, perm, bb);
  if (query_height(T) + 3 <= 48) {
    PKD_RANGE(48)
  } else if (query_height(T) + 3 <= kMaxStack) {
    PKD_RANGE(kMaxStack)
  } else {
    return PKD_ERR_CAPACITY;
  }
#undef PKD_RANGE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "k_range");
  return PKD_OK;
}

// ------------------------------------------------ allocation-free k-NN
// pkd_knn_static takes every scratch array of pkd_knn (error flags, Morton
// keys and the radix sort's work arrays) from one statically allocated device
// array instead of the block cache.  Layout for nq queries, each part aligned
// to 256 bytes.
struct StaticLayout {
  size_t flags, k0, v0, k1, v1, hist, off, bsum, end;
  explicit StaticLayout(int64_t nq) {
    const int64_t nblk = radix_sort_blocks(std::max<int64_t>(nq, 1));
    size_t at = 0;
    auto take = [&at](size_t bytes) {
      const size_t here = at;
      at = (at + bytes + 255) & ~size_t{255};
      return here;
    };
    flags = take(4 * sizeof(int));
    k0 = take(sizeof(uint64_t) * nq);
    v0 = take(sizeof(uint32_t) * nq);
    k1 = take(sizeof(uint64_t) * nq);
    v1 = take(sizeof(uint32_t) * nq);
    hist = take(sizeof(int32_t) * 256 * nblk);
    off = take(sizeof(int32_t) * (256 * nblk + 1));
    bsum = take(sizeof(int32_t) * exscan_bsum_need(256 * nblk));
    end = at;
  }
};

__global__ void k_clear_i32(int32_t* a, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = 0;
}

template <int D>
int knn_static_d(const pkd_tree* T, hipStream_t st, const int64_t* q, int64_t nq, int k, int64_t* oi, int64_t* od,
                 unsigned char* base, const StaticLayout& L) {
  int* flags = reinterpret_cast<int*>(base + L.flags);
  const uint32_t* perm = nullptr;
  if (nq >= kOrderMinQueries) {
    int bpd = 0, nbits = 0;
    morton_bits<D>(nq, nullptr, T->n_trees, &bpd, &nbits);
    uint64_t* k0 = reinterpret_cast<uint64_t*>(base + L.k0);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(base + L.v0);
    hipLaunchKernelGGL(k_morton<D>, dim3(static_cast<unsigned>((nq + 255) / 256)), dim3(256), 0, st, q, nq,
                       nullptr, bpd, k0, v0);
    PKD_TRY(kernel_status("k_morton"));
    SortBufs B{reinterpret_cast<uint64_t*>(base + L.k1), reinterpret_cast<uint32_t*>(base + L.v1),
               reinterpret_cast<int32_t*>(base + L.hist), reinterpret_cast<int32_t*>(base + L.off),
               reinterpret_cast<int32_t*>(base + L.bsum)};
    uint64_t* ks = nullptr;
    uint32_t* vs = nullptr;
    PKD_TRY(radix_sort_pairs_raw(st, k0, v0, nq, nbits, B, &ks, &vs));
    perm = vs;
  }
  return knn_launch<D>(T, st, q, nullptr, nq, k, oi, od, flags, perm);
}

}  // namespace

// The array itself; host code never passes its name to a kernel, only the
// per-device address that hipGetSymbolAddress returns for it.
constexpr int64_t kStaticMaxQueries = PKD_KNN_NOALLOC_MAX_QUERIES;
constexpr size_t kStaticScratchBytes = (size_t{25} << 20) + (size_t{64} << 10);   // 25 MiB + 64 KiB
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {nullptr};

// The array's address on the current device (looked up once per device).
int static_scratch(unsigned char** out) {
  int dev = 0;
  PKD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PKD_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    PKD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return PKD_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return PKD_OK;
}
}  // namespace

int run_knn_static(const pkd_tree* T, hipStream_t st, const int64_t* q, int64_t nq, int k, int64_t* oi,
                   int64_t* od) {
  if (nq > kStaticMaxQueries) return PKD_ERR_UNSUPPORTED;
  const StaticLayout L(nq);
  if (L.end > kStaticScratchBytes) return PKD_ERR_INTERNAL;
  unsigned char* base = nullptr;
  PKD_TRY(static_scratch(&base));
  int* flags = reinterpret_cast<int*>(base + L.flags);
  hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(64), 0, st, flags, 4);
  PKD_TRY(kernel_status("k_clear_i32"));
  int rc = PKD_ERR_UNSUPPORTED;
  switch (T->prm.D) {
    case 1: rc = knn_static_d<1>(T, st, q, nq, k, oi, od, base, L); break;
    case 2: rc = knn_static_d<2>(T, st, q, nq, k, oi, od, base, L); break;
    case 3: rc = knn_static_d<3>(T, st, q, nq, k, oi, od, base, L); break;
    case 4: rc = knn_static_d<4>(T, st, q, nq, k, oi, od, base, L); break;
    case 5: rc = knn_static_d<5>(T, st, q, nq, k, oi, od, base, L); break;
    case 6: rc = knn_static_d<6>(T, st, q, nq, k, oi, od, base, L); break;
    case 7: rc = knn_static_d<7>(T, st, q, nq, k, oi, od, base, L); break;
    case 8: rc = knn_static_d<8>(T, st, q, nq, k, oi, od, base, L); break;
    case 9: rc = knn_static_d<9>(T, st, q, nq, k, oi, od, base, L); break;
  }
  if (rc != PKD_OK) return rc;
  int h = 0;
  PKD_HIP(hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));
  if (h & kErrRange) return PKD_ERR_RANGE;
  if (h & kErrStack) return PKD_ERR_CAPACITY;
  if (h) return PKD_ERR_INTERNAL;
  return PKD_OK;
}

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
    case 8: return knn_d<8>(T, st, q, tree_of, nq, k, oi, od, flags);
    case 9: return knn_d<9>(T, st, q, tree_of, nq, k, oi, od, flags);
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
    case 8: return range_d<8>(T, st, lo, hi, tree_of, nb, out, flags);
    case 9: return range_d<9>(T, st, lo, hi, tree_of, nb, out, flags);
  }
  return PKD_ERR_UNSUPPORTED;
}

}  // namespace pkd
