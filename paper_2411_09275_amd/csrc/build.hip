// Build of a Pkd-tree on the GPU: Algorithm 1 of the paper (Section 3.1),
// re-planned for gfx950.
//
// One sieve round processes every live subproblem of a recursion level at once
// (segmented launches), so the GPU sees one large grid per step:
//   candidates  -- hash-key prefilter of each subproblem's ids (sampling)
//   select      -- bottom-s sample by (key, id) with an LDS radix select, then
//                  the lambda-level skeleton on the sample (LDS presorted build)
//   count       -- per tile: walk the skeleton, 2^lambda-bin LDS histogram
//   scan        -- exclusive prefix sum of the tile x bucket counts in
//                  column-major order, segmented by subproblem
//   scatter     -- stable, LDS-staged, coalesced distribution of coordinates
//                  and ids into the twin buffer (buffers swap every round
//                  instead of copying back, Section 5)
//   emit        -- skeleton nodes become tree nodes; buckets become the next
//                  round's subproblems (>= s points) or finisher tasks
// Subproblems below s = 2^lambda*sigma points are finished by the plain
// construction in LDS, one workgroup per subproblem.
#include <algorithm>
#include <cstring>

#include "pkd_internal.h"

namespace pkd {

namespace {

constexpr int kBlock = 256;
constexpr int kChunkTiles = 64;      // tiles per scan chunk

__device__ inline uint32_t lane_id() { return threadIdx.x & 63; }

// Wave-aggregated append: every lane with `take` gets a distinct slot of
// *counter; one atomic per wave.
__device__ inline int wave_append(bool take, int* counter) {
  const unsigned long long mask = __ballot(take);
  if (mask == 0) return -1;
  const int leader = __ffsll(static_cast<long long>(mask)) - 1;
  int base = 0;
  if (lane_id() == static_cast<uint32_t>(leader)) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return take ? base + static_cast<int>(__popcll(mask & ((1ULL << lane_id()) - 1))) : -1;
}

// wave_append for a whole workgroup: one counter update per workgroup (one
// per wave serializes on the counter when tens of thousands of waves append).
// Every thread of the workgroup calls it.
__device__ inline int block_append(bool take, int* counter) {
  __shared__ int wc[16];
  __shared__ int base;
  const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  const unsigned long long m = __ballot(take);
  const int rank = static_cast<int>(__popcll(m & ((1ULL << (threadIdx.x & 63)) - 1)));
  if ((threadIdx.x & 63) == 0) wc[wave] = static_cast<int>(__popcll(m));
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < nw; ++w) {
      const int x = wc[w];
      wc[w] = run;
      run += x;
    }
    base = run ? atomicAdd(counter, run) : 0;
  }
  __syncthreads();
  const int at = take ? base + wc[wave] + rank : -1;
  __syncthreads();   // the next call reuses wc and base
  return at;
}

template <int D>
__device__ inline int64_t pick(const int64_t (&c)[D], int d) {
  int64_t v = c[0];
#pragma unroll
  for (int e = 1; e < D; ++e) v = (d == e) ? c[e] : v;
  return v;
}

// Bucket label of a point: lambda steps down the heap-ordered skeleton.  Nodes
// that are external above level lambda carry the all-left splitter, so every
// walk takes exactly lambda steps and ends at the leftmost depth-lambda
// position below its external node.
template <int D>
__device__ inline int route(const int64_t (&c)[D], const int64_t* sx, const uint8_t* sdim, int lambda) {
  int v = 1;
  for (int l = 0; l < lambda; ++l) {
    // compare every coordinate and keep the one of the split dimension (no
    // dynamic register indexing)
    const int d = sdim[v];
    const int64_t x = sx[v];
    int ge = 0;
#pragma unroll
    for (int e = 0; e < D; ++e) ge |= (d == e) & (c[e] >= x);
    v = 2 * v + ge;
  }
  return v - (1 << lambda);
}


__device__ inline int find_owner(const int64_t* off, int n, int64_t t) {
  // largest s with off[s] <= t
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Candidate threshold exponent: keys below 2^(64-t) are candidates, so that a
// subproblem of m points keeps about m/2^t in [1.25 s, 2.5 s) of them.
__host__ __device__ inline int cand_shift(int64_t m, int s) {
  int t = 0;
  while (4 * m >= 5 * static_cast<int64_t>(s) * (int64_t{2} << t) && t < 62) ++t;
  return t;
}

// A count the host passes (eager launches, sized exactly) or, when `d` is
// set, the one in device memory (launches enqueued without host reads, sized
// for the largest count; blocks past the count return at once).
__device__ inline int dev_count(const int* d, int h) { return d ? *d : h; }

// ---------------------------------------------------------------- classify
// With sieve_pts set, the points of the sieve tasks are added up there.
__global__ void k_classify(const Task* front, int n_front, int s, Task* sieve, int* n_sieve, Task* fin,
                           int* n_fin, const int* dn = nullptr, unsigned long long* sieve_pts = nullptr) {
  n_front = dev_count(dn, n_front);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < n_front;
  Task t{};
  if (ok) t = front[i];
  const int a = block_append(ok && t.m >= s, n_sieve);
  const int b = block_append(ok && t.m < s, n_fin);
  if (a >= 0) sieve[a] = t;
  if (b >= 0) fin[b] = t;
  if (sieve_pts && a >= 0) atomicAdd(sieve_pts, static_cast<unsigned long long>(t.m));
}

// ------------------------------------------------------------ tile layout
// Single workgroup: exclusive prefix sums of tiles and chunks per subproblem.
__global__ void k_tile_scan(const Task* sp, int ns, int tile, int64_t* tile_off, int64_t* chunk_off,
                            int8_t* shift, int s, int small_max, const int8_t* shift_override, int64_t* total_pts,
                            int cand_bias, const int* dns = nullptr) {
  ns = dev_count(dns, ns);
  __shared__ int64_t part_t[1024], part_c[1024];
  __shared__ unsigned long long pts;
  if (threadIdx.x == 0) pts = 0;
  __syncthreads();
  int tid = threadIdx.x, nt = blockDim.x;
  int per = (ns + nt - 1) / nt;
  int b = tid * per, e = min(ns, b + per);
  int64_t st = 0, sc = 0;
  for (int i = b; i < e; ++i) {
    int64_t tiles = (sp[i].m + tile - 1) / tile;
    st += tiles;
    sc += (tiles + kChunkTiles - 1) / kChunkTiles;
  }
  part_t[tid] = st;
  part_c[tid] = sc;
  {
    unsigned long long mine = 0;
    for (int i = b; i < e; ++i) mine += static_cast<unsigned long long>(sp[i].m);
    atomicAdd(&pts, mine);
  }
  __syncthreads();
  if (tid == 0) {
    *total_pts = static_cast<int64_t>(pts);
    int64_t a = 0, c = 0;
    for (int i = 0; i < nt; ++i) {
      int64_t x = part_t[i], y = part_c[i];
      part_t[i] = a;
      part_c[i] = c;
      a += x;
      c += y;
    }
    tile_off[ns] = a;
    chunk_off[ns] = c;
  }
  __syncthreads();
  st = part_t[tid];
  sc = part_c[tid];
  for (int i = b; i < e; ++i) {
    tile_off[i] = st;
    chunk_off[i] = sc;
    int64_t tiles = (sp[i].m + tile - 1) / tile;
    st += tiles;
    sc += (tiles + kChunkTiles - 1) / kChunkTiles;
    int sh = sp[i].m <= small_max ? 0 : max(0, cand_shift(sp[i].m, s) + cand_bias);
    if (shift_override && shift_override[i] >= 0) sh = shift_override[i];
    shift[i] = static_cast<int8_t>(sh);
  }
}

// Candidates of the sample of every subproblem that sieves this round: the
// points whose key is at most the subproblem's threshold (Section 3: the
// sample is the s points of smallest key).  One tile per workgroup; the tile's
// candidates are counted first and take their slots with one atomic, so the
// counters (one per 128-byte line) see one update per tile.
constexpr int kCntStride = 32;   // uint32 counters, one per cache line

template <int ITER>
__global__ void __launch_bounds__(kBlock) k_candidates(const Task* sp, int ns, const int64_t* tile_off, Bufs bufs,
                                                       int src, uint64_t seed, const int8_t* shift, int small_max,
                                                       uint64_t* cand_key, uint32_t* cand_pos, uint32_t* cand_cnt,
                                                       int cap, const int* dns = nullptr) {
  constexpr int kWaves = kBlock / 64;
  __shared__ int sig_sh;
  __shared__ uint32_t wcnt[ITER][kWaves];
  __shared__ uint32_t gbase;
  const int64_t t = blockIdx.x;
  ns = dev_count(dns, ns);
  if (dns && t >= tile_off[ns]) return;
  const int tid = threadIdx.x, wave = tid >> 6;
  const uint32_t lane = lane_id();
  if (tid == 0) sig_sh = find_owner(tile_off, ns, t);
  __syncthreads();
  const int sig = sig_sh;
  const Task q = sp[sig];
  if (q.m <= small_max) return;
  const int sh = shift[sig];
  const uint64_t thr = sh == 0 ? ~0ULL : (~0ULL >> sh);   // key <= thr  <=>  key < 2^(64-sh)
  const int64_t lo = (t - tile_off[sig]) * (kBlock * ITER);
  const int64_t hi = min<int64_t>(lo + kBlock * ITER, q.m);
  const int64_t* ids = bufs.id[src] + q.start;
  uint64_t key[ITER];
  unsigned long long mask[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int64_t i = lo + it * kBlock + tid;
    key[it] = i < hi ? sample_key(seed, q.depth, ids[i]) : ~0ULL;
    mask[it] = __ballot(i < hi && key[it] <= thr);
    if (lane == 0) wcnt[it][wave] = static_cast<uint32_t>(__popcll(mask[it]));
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int it = 0; it < ITER; ++it)
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t x = wcnt[it][w];
        wcnt[it][w] = run;
        run += x;
      }
    gbase = run ? atomicAdd(cand_cnt + static_cast<int64_t>(sig) * kCntStride, run) : 0;
  }
  __syncthreads();
  uint64_t* kout = cand_key + static_cast<int64_t>(sig) * cap;
  uint32_t* pout = cand_pos + static_cast<int64_t>(sig) * cap;
  const unsigned long long lt = (1ULL << lane) - 1;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    if ((mask[it] >> lane) & 1) {
      const uint32_t k = gbase + wcnt[it][wave] + static_cast<uint32_t>(__popcll(mask[it] & lt));
      if (k < static_cast<uint32_t>(cap)) {
        kout[k] = key[it];
        pout[k] = static_cast<uint32_t>(lo + it * kBlock + tid);
      }
    }
  }
}

// ---------------------------------------------------- LDS presorted kd build
// Shared pieces of the skeleton kernel and the finisher kernel.  Points are
// held in LDS as 30-bit coordinates; O[d] lists the points sorted by
// coordinate d (ties by index).  A node owns the same position range [a, a+L)
// in every O[d], so its widest dimension and its upper median are read
// directly, and a split is a stable partition of each O[d] by the side flag.

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int mask) {
  const int lo = __shfl_xor(static_cast<int>(static_cast<uint32_t>(v)), mask);
  const int hi = __shfl_xor(static_cast<int>(v >> 32), mask);
  return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

constexpr uint16_t kNone = 0xFFFF;   // "no segment"

// Bitonic sort of 64*NPL 64-bit keys held by one wave, ascending; lane l
// holds elements l*NPL .. l*NPL+NPL-1.  Partners closer than NPL are in the
// same lane, the others one shuffle away.
template <int NPL>
__device__ void wave_bitonic(uint64_t (&k)[NPL]) {
  constexpr int N = 64 * NPL;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int j = size >> 1; j > 0; j >>= 1) {
      if (j < NPL) {
#pragma unroll
        for (int r = 0; r < NPL; ++r) {
          const int pr = r ^ j;
          if (pr > r) {
            const bool up = size < NPL ? (r & size) == 0 : ((lane * NPL) & size) == 0;
            const uint64_t a = k[r], b = k[pr];
            const bool sw = (a > b) == up;
            k[r] = sw ? b : a;
            k[pr] = sw ? a : b;
          }
        }
      } else {
        const bool keep_min = (((lane * NPL) & j) == 0) == (((lane * NPL) & size) == 0);
#pragma unroll
        for (int r = 0; r < NPL; ++r) {
          const uint64_t o = shfl_xor_u64(k[r], j / NPL);
          const bool take = (o < k[r]) == keep_min;
          k[r] = take ? o : k[r];
        }
      }
    }
  }
}

// Stable partition, in place, of one sorted order Od (positions 0..m-1, held
// by one wave) inside the segments that split: flagged points go to the left
// part.  The rank of a point among the flagged ones before it comes from
// ballots; segF[k] records that rank at the first position of segment k.
// Every thread of the block calls this (it holds a block barrier); only
// `active` waves touch Od.
template <int NPL>
__device__ void wave_partition(bool active, uint16_t* Od, int m, const uint16_t* seg_of_pt, const uint8_t* splits,
                               const uint16_t* segA, const uint16_t* segNL, const uint8_t* flag, uint16_t* segF) {
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = (1ULL << lane) - 1;
  // Positions are taken in chunks of CH rows.  Every load is unconditional,
  // on an index kept inside its array (positions below 64*NPL, the row
  // length; segment 0 standing in where there is none), so the loads of a
  // chunk issue back to back with no branches; values of positions >= m are
  // dropped afterwards.
  constexpr int CH = NPL < 2 ? NPL : 2;
  // per position: point | rank << 16, and segment | side << 16 (kNone: stays)
  uint32_t pe[NPL], ks[NPL];
  if (active) {
    int run = 0;
#pragma unroll
    for (int r0 = 0; r0 < NPL; r0 += CH) {
      uint32_t e[CH], k[CH], sp[CH], fg[CH], sa[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int p = (r0 + c) * 64 + lane;
        const uint32_t v = Od[p];
        e[c] = p < m ? v : 0u;
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int p = (r0 + c) * 64 + lane;
        const uint32_t v = seg_of_pt[e[c]];
        k[c] = p < m ? v : static_cast<uint32_t>(kNone);
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const uint32_t kc = k[c] == kNone ? 0u : k[c];
        sp[c] = splits[kc];
        fg[c] = flag[e[c]];
        sa[c] = segA[kc];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int r = r0 + c, p = r * 64 + lane;
        const bool spl = (k[c] != kNone) & (sp[c] != 0);
        const bool f = spl & (fg[c] != 0);
        const unsigned long long mask = __ballot(f);
        const int F = run + __popcll(mask & lt);
        run += __popcll(mask);
        if (spl & (p == static_cast<int>(sa[c]))) segF[k[c]] = static_cast<uint16_t>(F);
        pe[r] = e[c] | (static_cast<uint32_t>(F) << 16);
        ks[r] = spl ? (k[c] | (f ? 0x10000u : 0u)) : static_cast<uint32_t>(kNone);
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int r0 = 0; r0 < NPL; r0 += CH) {
      uint32_t a[CH], fb[CH], nl[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const uint32_t k = ks[r0 + c] & 0xFFFFu;
        const uint32_t kc = k == kNone ? 0u : k;
        a[c] = segA[kc];
        fb[c] = segF[kc];
        nl[c] = segNL[kc];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int r = r0 + c, p = r * 64 + lane;
        if (p < m) {
          int np = p;
          if ((ks[r] & 0xFFFFu) != kNone) {
            const int lrank = static_cast<int>(pe[r] >> 16) - static_cast<int>(fb[c]);
            np = (ks[r] >> 16) ? static_cast<int>(a[c]) + lrank
                               : static_cast<int>(a[c]) + static_cast<int>(nl[c]) + (p - static_cast<int>(a[c]) - lrank);
          }
          Od[np] = static_cast<uint16_t>(pe[r] & 0xFFFFu);
        }
      }
    }
  }
}

// Split rule of a node that owns positions [a, a+L) (L >= 1): widest
// dimension (max - min, lowest index on ties), upper median v[floor(L/2)],
// moved to the next larger distinct value if it equals the minimum.
// Returns false when the node has zero width in every dimension.
template <int D>
__device__ bool lds_split_rule(const uint32_t* C, const uint16_t* O, int P, int a, int L, int* od, uint32_t* ox,
                               int* onl) {
  int best = -1;
  uint32_t bw = 0;
  for (int d = 0; d < D; ++d) {
    uint32_t lo = C[d * P + O[d * P + a]];
    uint32_t hi = C[d * P + O[d * P + a + L - 1]];
    if (hi - lo > bw) {   // strict: the lowest index wins ties
      bw = hi - lo;
      best = d;
    }
  }
  if (best < 0) return false;
  const uint32_t* Cd = C + best * P;
  const uint16_t* Od = O + best * P;
  const uint32_t mn = Cd[Od[a]];
  uint32_t x = Cd[Od[a + L / 2]];
  int nl;
  if (x == mn) {
    // the next larger distinct value: first position with value > mn
    int lo = a, hi = a + L - 1;   // Cd[Od[hi]] > mn since the width is positive
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Cd[Od[mid]] > mn) hi = mid; else lo = mid + 1;
    }
    x = Cd[Od[lo]];
    nl = lo - a;
  } else if (Cd[Od[a + L / 2 - 1]] < x) {
    nl = L / 2;   // no copy of x before the median position
  } else {
    // copies of x before the median: first position with value >= x
    int lo = a, hi = a + L / 2;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Cd[Od[mid]] < x) lo = mid + 1; else hi = mid;
    }
    nl = lo - a;
  }
  *od = best;
  *ox = x;
  *onl = nl;
  return true;
}

// LDS layouts (byte offsets), computed identically on host and device.  The
// 8-byte arrays come first so every array is naturally aligned.
__host__ __device__ inline int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}
__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~size_t{7}; }

// The select phase's tie and histogram arrays (kSelScratch bytes) live in
// the C region, which is written only after them; the sample positions share
// their region with the orders O, which are written only after the positions
// have been read.
constexpr size_t kSelScratch = 256 * (sizeof(int64_t) + sizeof(uint32_t) + sizeof(uint32_t));

struct SkelLayout {
  size_t C, pos, O, node_of, segF, flag, end;
  __host__ __device__ SkelLayout(int D, int P) {
    size_t o = 0;
    const size_t c_bytes = sizeof(uint32_t) * D * P;
    C = o;        o += c_bytes > kSelScratch ? c_bytes : kSelScratch;
    const size_t pos_bytes = sizeof(uint32_t) * P, o_bytes = sizeof(uint16_t) * D * P;
    pos = o;
    O = o;        o += pos_bytes > o_bytes ? pos_bytes : o_bytes;
    node_of = o;  o += sizeof(uint16_t) * P;
    segF = o;     o += sizeof(uint16_t) * D * (2 << kMaxLambda);
    flag = o;     o += P;
    end = align8(o);
  }
};

struct FinLayout {
  size_t C, O, seg, flag, lA0, lA1, lL0, lL1, lN0, lN1, sxs, snl, srank, segF, sdm, ssplit, end;
  int MS;   // segments per level: splitting segments hold > phi points each
  __host__ __device__ FinLayout(int D, int P, int phi) {
    MS = min(P, 2 * P / (phi + 1) + 2);
    size_t o = 0;
    lN0 = o;    o += sizeof(int32_t) * MS;
    lN1 = o;    o += sizeof(int32_t) * MS;
    sxs = o;    o += sizeof(uint32_t) * MS;
    C = o;      o += sizeof(uint32_t) * D * P;
    O = o;      o += sizeof(uint16_t) * D * P;
    seg = o;    o += sizeof(uint16_t) * P;
    lA0 = o;    o += sizeof(uint16_t) * MS;
    lA1 = o;    o += sizeof(uint16_t) * MS;
    lL0 = o;    o += sizeof(uint16_t) * MS;
    lL1 = o;    o += sizeof(uint16_t) * MS;
    snl = o;    o += sizeof(uint16_t) * MS;
    srank = o;  o += sizeof(uint16_t) * MS;
    segF = o;   o += sizeof(uint16_t) * D * MS;
    flag = o;   o += P;
    sdm = o;    o += MS;
    ssplit = o; o += MS;
    end = align8(o);
  }
};

// ------------------------------------------------- select sample + skeleton
// One workgroup of D waves per sieve subproblem.  Phase 1 finds the s
// smallest (key, id) among the candidates by a radix select over the 64-bit
// keys (ties by id), reading the candidates from global memory (they stay in
// L2 across the passes).  Phase 2 gathers the sample's coordinates and builds
// the lambda-level skeleton; wave d keeps the sample sorted by coordinate d
// and partitions that order as the skeleton nodes split.
struct SelectOut {
  int64_t* rx;        // [ns][2^lambda] splitters in routing form
  uint8_t* rdim;      // [ns][2^lambda]
  int8_t* ext;        // [ns][2^(lambda+1)] external flags (reachable nodes only)
  int* root_ext_list; // subproblems whose skeleton root is external
  int* n_root_ext;
  int8_t* shift_fix;  // retry: corrected threshold exponent per subproblem (-1 = ok)
  int* flags;
};

template <int D, int NPL>
__global__ void __launch_bounds__(64 * D) k_select_skeleton(const Task* sp, int ns, Bufs bufs, int src,
                                                              uint64_t seed, int s, int lambda,
                                                              const int8_t* shift, int small_max,
                                                              const uint64_t* cand_key, const uint32_t* cand_pos,
                                                              const uint32_t* cand_cnt, int cap, SelectOut out,
                                                              const int* dns = nullptr) {
  constexpr int NT = 64 * D;
  constexpr int P = 64 * NPL;   // padded stride of the per-dimension arrays (>= s)
  extern __shared__ __align__(16) unsigned char smem[];
  const int sig = blockIdx.x;
  if (dns && sig >= *dns) return;
  const Task q = sp[sig];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t* ids = bufs.id[src] + q.start;
  const int64_t* X = bufs.c[src];
  const int64_t xcap = bufs.cap[src];
  const SkelLayout lay(D, P);
  uint32_t* C = reinterpret_cast<uint32_t*>(smem + lay.C);
  uint32_t* sampPos = reinterpret_cast<uint32_t*>(smem + lay.pos);
  uint16_t* O = reinterpret_cast<uint16_t*>(smem + lay.O);
  uint16_t* node_of = reinterpret_cast<uint16_t*>(smem + lay.node_of);
  uint16_t* segF = reinterpret_cast<uint16_t*>(smem + lay.segF);
  uint8_t* flag = smem + lay.flag;

  int64_t* tie_id = reinterpret_cast<int64_t*>(smem + lay.C);   // [256]; phase 1 only (see SkelLayout)
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem + lay.C + 256 * sizeof(int64_t));
  uint32_t* tie_pos = hist + 256;
  __shared__ int sh_c, sh_done, sh_pass, sh_need, sh_cnt, sh_bad, sh_tie_n;
  __shared__ uint64_t sh_prefix, sh_T;

  // ---- phase 1: the s smallest keys
  if (tid == 0) {
    int c;
    if (q.m <= small_max) {
      c = q.m;
    } else {
      c = static_cast<int>(cand_cnt[static_cast<int64_t>(sig) * kCntStride]);
    }
    sh_c = c;
    sh_bad = 0;
    if (q.m > small_max && (c > cap || c < s)) {
      // retry with a threshold that keeps more (underflow) or fewer (overflow)
      int sh0 = shift[sig];
      out.shift_fix[sig] = static_cast<int8_t>(c > cap ? sh0 + 1 : max(0, sh0 - 1));
      atomicOr(out.flags, c > cap ? kErrCandOverflow : kErrCandUnderflow);
      sh_bad = 1;
    }
    sh_done = 0;
    sh_pass = 0;
    sh_need = s;
    sh_prefix = 0;
    sh_cnt = 0;
    sh_tie_n = 0;
  }
  __syncthreads();
  if (sh_bad) return;
  const int c = sh_c;
  // small subproblems sample from all their points: keys are computed on the fly
  const bool small = q.m <= small_max;
  const uint64_t* kin = cand_key + static_cast<int64_t>(sig) * cap;
  const uint32_t* pin = cand_pos + static_cast<int64_t>(sig) * cap;
  for (int pass = 0; pass < 8; ++pass) {
    for (int i = tid; i < 256; i += NT) hist[i] = 0;
    __syncthreads();
    const int shv = 56 - 8 * pass;
    const uint64_t prefix = sh_prefix;
    for (int i = tid; i < c; i += NT) {
      const uint64_t k = small ? sample_key(seed, q.depth, ids[i]) : kin[i];
      const bool match = pass == 0 || (k >> (64 - 8 * pass)) == prefix;
      if (match) atomicAdd(&hist[(k >> shv) & 255], 1u);
    }
    __syncthreads();
    if (wave == 0) {
      // first bin whose inclusive running count reaches `need` (bin 255 if
      // none); lane l scans bins 4l .. 4l+3
      const uint32_t need = static_cast<uint32_t>(sh_need);
      uint32_t h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) h[j] = hist[4 * lane + j];
      const uint32_t tot = h[0] + h[1] + h[2] + h[3];
      uint32_t incl = tot;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      const uint32_t excl = incl - tot;
      int b = -1;
      uint32_t cum = 0;
      if (excl < need && incl >= need) {
        uint32_t run = excl;
        for (int j = 0; j < 4; ++j) {
          if (run + h[j] >= need) {
            b = 4 * lane + j;
            cum = run;
            break;
          }
          run += h[j];
        }
      }
      const unsigned long long found = __ballot(b >= 0);
      if (!found && lane == 63) {
        b = 255;
        cum = incl - h[3];
      }
      if (b >= 0) {
        const uint32_t hb = hist[b];
        if (cum + hb == need) {
          sh_done = 1;
          sh_pass = pass;
          sh_T = (prefix << 8) | static_cast<uint64_t>(b);
        } else {
          sh_need = static_cast<int>(need - cum);
          sh_prefix = (prefix << 8) | static_cast<uint64_t>(b);
        }
      }
    }
    __syncthreads();
    if (sh_done) break;
  }
  if (sh_done) {
    const int bits = 8 * (sh_pass + 1);
    const uint64_t T = sh_T;
    for (int i = tid; i < c; i += NT) {
      const uint64_t k = small ? sample_key(seed, q.depth, ids[i]) : kin[i];
      if ((k >> (64 - bits)) <= T) {
        const int at = atomicAdd(&sh_cnt, 1);
        if (at < s) sampPos[at] = small ? static_cast<uint32_t>(i) : pin[i];
      }
    }
  } else {
    // All 64 key bits fixed: sh_prefix is the s-th smallest key K*; take the
    // keys below it and the sh_need smallest ids among those equal to it.
    const uint64_t Ks = sh_prefix;
    for (int i = tid; i < c; i += NT) {
      const uint64_t k = small ? sample_key(seed, q.depth, ids[i]) : kin[i];
      const uint32_t pos = small ? static_cast<uint32_t>(i) : pin[i];
      if (k < Ks) {
        const int at = atomicAdd(&sh_cnt, 1);
        if (at < s) sampPos[at] = pos;
      } else if (k == Ks) {
        const int at = atomicAdd(&sh_tie_n, 1);
        if (at < 256) {
          tie_pos[at] = pos;
          tie_id[at] = ids[pos];
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      const int nt = min(sh_tie_n, 256);
      if (sh_tie_n > 256) atomicOr(out.flags, kErrInternal);
      for (int r = 0; r < sh_need; ++r) {
        int best = -1;
        for (int j = 0; j < nt; ++j)
          if (tie_pos[j] != 0xFFFFFFFFu && (best < 0 || tie_id[j] < tie_id[best])) best = j;
        if (best < 0) break;
        const int at = sh_cnt++;
        if (at < s) sampPos[at] = tie_pos[best];
        tie_pos[best] = 0xFFFFFFFFu;
      }
    }
  }
  __syncthreads();
  if (sh_cnt != s) {
    if (tid == 0) atomicOr(out.flags, kErrInternal);
    return;
  }

  // ---- phase 2: skeleton on the sample
  __shared__ uint16_t segA[2 << kMaxLambda], segL[2 << kMaxLambda], segNL[2 << kMaxLambda];
  __shared__ uint8_t live[2 << kMaxLambda], splits[2 << kMaxLambda], sdim[1 << kMaxLambda];
  __shared__ uint32_t sx[1 << kMaxLambda];
  for (int i = tid; i < s; i += NT) {
    const int64_t pos = q.start + static_cast<int64_t>(sampPos[i]);
#pragma unroll
    for (int d = 0; d < D; ++d) C[d * P + i] = static_cast<uint32_t>(X[d * xcap + pos]);
    node_of[i] = 1;
  }
  const int nheap = 2 << lambda;
  for (int v = tid; v < nheap; v += NT) {
    live[v] = 0;
    splits[v] = 0;
  }
  __syncthreads();
  {
    // wave d: the sample ordered by (coordinate d, index)
    uint64_t k[NPL];
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int e = lane * NPL + r;
      k[r] = e < s ? (static_cast<uint64_t>(C[wave * P + e]) << 16) | static_cast<uint64_t>(e) : ~0ULL;
    }
    wave_bitonic<NPL>(k);
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int e = lane * NPL + r;
      if (e < s) O[wave * P + e] = static_cast<uint16_t>(k[r] & 0xFFFF);
    }
  }
  if (tid == 0) {
    live[1] = 1;
    segA[1] = 0;
    segL[1] = static_cast<uint16_t>(s);
  }
  __syncthreads();
  for (int level = 0; level < lambda; ++level) {
    const int v0 = 1 << level, v1 = 2 << level;
    for (int v = v0 + tid; v < v1; v += NT) {
      splits[v] = 0;
      if (!live[v]) continue;
      int d, nl;
      uint32_t x;
      if (lds_split_rule<D>(C, O, P, segA[v], segL[v], &d, &x, &nl) && nl > 0 && nl < segL[v]) {
        splits[v] = 1;
        sdim[v] = static_cast<uint8_t>(d);
        sx[v] = x;
        segNL[v] = static_cast<uint16_t>(nl);
        live[2 * v] = live[2 * v + 1] = 1;
        segA[2 * v] = segA[v];
        segL[2 * v] = static_cast<uint16_t>(nl);
        segA[2 * v + 1] = static_cast<uint16_t>(segA[v] + nl);
        segL[2 * v + 1] = static_cast<uint16_t>(segL[v] - nl);
      }
    }
    __syncthreads();
    if (level + 1 == lambda) break;   // the orders are not read after the last level
    for (int e = tid; e < s; e += NT) {
      const int v = node_of[e];
      flag[e] = splits[v] ? (C[sdim[v] * P + e] < sx[v] ? 1 : 0) : 0;
    }
    __syncthreads();
    wave_partition<NPL>(true, O + wave * P, s, node_of, splits, segA, segNL, flag, segF + wave * (2 << kMaxLambda));
    __syncthreads();
    for (int e = tid; e < s; e += NT) {
      const int v = node_of[e];
      if (splits[v]) node_of[e] = static_cast<uint16_t>(2 * v + (flag[e] ? 0 : 1));
    }
    __syncthreads();
  }
  // routing form: interior nodes keep (dim, x); everything else sends left
  const int NB = 1 << lambda;
  int64_t* rx = out.rx + static_cast<int64_t>(sig) * NB;
  uint8_t* rd = out.rdim + static_cast<int64_t>(sig) * NB;
  int8_t* ex = out.ext + static_cast<int64_t>(sig) * nheap;
  for (int v = tid; v < nheap; v += NT) {
    const bool interior = v < NB && live[v] && splits[v];
    if (v < NB) {
      rx[v] = interior ? static_cast<int64_t>(sx[v]) : kAllLeft;
      rd[v] = interior ? sdim[v] : 0;
    }
    ex[v] = (live[v] && !interior) ? 1 : 0;
  }
  if (tid == 0 && !splits[1]) {
    const int k = atomicAdd(out.n_root_ext, 1);
    out.root_ext_list[k] = sig;
  }
}

// ------------------------------------------------------------------ count
template <int D>
__global__ void __launch_bounds__(kBlock) k_count(const Task* sp, int ns, const int64_t* tile_off, int tile,
                                                  Bufs bufs, int src, const int64_t* rx, const uint8_t* rdim,
                                                  const int8_t* mode, int lambda, uint32_t* A, int check,
                                                  int* flags, const int* dns = nullptr) {
  __shared__ int64_t sx[1 << kMaxLambda];
  __shared__ uint8_t sd[1 << kMaxLambda];
  __shared__ uint32_t hist[1 << kMaxLambda];
  __shared__ int sig_sh;
  const int NB = 1 << lambda;
  const int64_t t = blockIdx.x;
  ns = dev_count(dns, ns);
  if (dns && t >= tile_off[ns]) return;
  if (threadIdx.x == 0) sig_sh = find_owner(tile_off, ns, t);
  for (int j = threadIdx.x; j < NB; j += kBlock) hist[j] = 0;
  __syncthreads();
  const int sig = sig_sh;
  const Task q = sp[sig];
  if (mode[sig] == 1) {   // heavy leaf: nothing moves
    for (int j = threadIdx.x; j < NB; j += kBlock) A[t * NB + j] = 0;
    return;
  }
  for (int j = threadIdx.x; j < NB; j += kBlock) {
    sx[j] = rx[static_cast<int64_t>(sig) * NB + j];
    sd[j] = rdim[static_cast<int64_t>(sig) * NB + j];
  }
  __syncthreads();
  const int64_t lo = q.start + (t - tile_off[sig]) * tile;
  const int64_t hi = min<int64_t>(lo + tile, static_cast<int64_t>(q.start) + q.m);
  const int64_t* X = bufs.c[src];
  const int64_t cap = bufs.cap[src];
  bool bad = false;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    int64_t c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      c[d] = X[d * cap + i];
      bad |= static_cast<uint64_t>(c[d]) >= static_cast<uint64_t>(coord_limit(D));
    }
    atomicAdd(&hist[route<D>(c, sx, sd, lambda)], 1u);
  }
  if (check && bad) atomicOr(flags, kErrRange);
  __syncthreads();
  for (int j = threadIdx.x; j < NB; j += kBlock) A[t * NB + j] = hist[j];
}

// ------------------------------------------------------------------- scan
// Column sums of each chunk of kChunkTiles tiles.
__global__ void k_chunk_sum(const int64_t* chunk_off, const int64_t* tile_off, int ns, int lambda,
                            const uint32_t* A, uint32_t* S, const int* dns = nullptr) {
  __shared__ int sig_sh;
  __shared__ uint32_t part[kBlock];
  const int NB = 1 << lambda;
  const int64_t c = blockIdx.x;
  ns = dev_count(dns, ns);
  if (dns && c >= chunk_off[ns]) return;
  if (threadIdx.x == 0) sig_sh = find_owner(chunk_off, ns, c);
  __syncthreads();
  const int sig = sig_sh;
  const int64_t t0 = tile_off[sig] + (c - chunk_off[sig]) * kChunkTiles;
  const int64_t t1 = min<int64_t>(t0 + kChunkTiles, tile_off[sig + 1]);
  const int j = threadIdx.x % NB, lane = threadIdx.x / NB, lanes = kBlock / NB;
  uint32_t acc = 0;
  for (int64_t t = t0 + lane; t < t1; t += lanes) acc += A[t * NB + j];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < NB) {
    uint32_t s = 0;
    for (int l = 0; l < lanes; ++l) s += part[l * NB + threadIdx.x];
    S[c * NB + threadIdx.x] = s;
  }
}

// Per subproblem: exclusive prefix of the chunk sums over chunks (per bucket),
// bucket sizes and bucket starts (prefix over buckets, offset by the start).
__global__ void k_sp_scan(const Task* sp, const int64_t* chunk_off, int lambda, uint32_t* S, int32_t* bsize,
                          int32_t* bstart, const int* dns = nullptr) {
  __shared__ uint32_t part[kBlock];
  __shared__ uint32_t tot[1 << kMaxLambda];
  const int NB = 1 << lambda;
  const int sig = blockIdx.x;
  if (dns && sig >= *dns) return;
  const int64_t c0 = chunk_off[sig], c1 = chunk_off[sig + 1];
  const int j = threadIdx.x % NB, lane = threadIdx.x / NB, lanes = kBlock / NB;
  const int64_t nc = c1 - c0;
  const int64_t per = (nc + lanes - 1) / lanes;
  const int64_t b = c0 + lane * per, e = min(c1, b + per);
  uint32_t acc = 0;
  for (int64_t c = b; c < e; ++c) acc += S[c * NB + j];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < NB) {
    uint32_t run = 0;
    for (int l = 0; l < lanes; ++l) {
      uint32_t x = part[l * NB + threadIdx.x];
      part[l * NB + threadIdx.x] = run;
      run += x;
    }
    tot[threadIdx.x] = run;
  }
  __syncthreads();
  uint32_t run = part[threadIdx.x];
  for (int64_t c = b; c < e; ++c) {
    uint32_t x = S[c * NB + j];
    S[c * NB + j] = run;
    run += x;
  }
  if (threadIdx.x == 0) {
    int32_t at = sp[sig].start;
    for (int k = 0; k < NB; ++k) {
      bsize[static_cast<int64_t>(sig) * NB + k] = static_cast<int32_t>(tot[k]);
      bstart[static_cast<int64_t>(sig) * NB + k] = at;
      at += static_cast<int32_t>(tot[k]);
    }
  }
}

// B[t][j] = bucket start + prefix over earlier chunks + prefix over earlier
// tiles of the chunk: the write cursor of tile t for bucket j.
__global__ void k_apply(const int64_t* chunk_off, const int64_t* tile_off, int ns, int lambda, const uint32_t* A,
                        const uint32_t* S, const int32_t* bstart, int32_t* B, const int* dns = nullptr) {
  __shared__ int sig_sh;
  const int NB = 1 << lambda;
  const int64_t c = blockIdx.x;
  ns = dev_count(dns, ns);
  if (dns && c >= chunk_off[ns]) return;
  if (threadIdx.x == 0) sig_sh = find_owner(chunk_off, ns, c);
  __syncthreads();
  const int sig = sig_sh;
  const int64_t t0 = tile_off[sig] + (c - chunk_off[sig]) * kChunkTiles;
  const int64_t t1 = min<int64_t>(t0 + kChunkTiles, tile_off[sig + 1]);
  for (int j = threadIdx.x; j < NB; j += kBlock) {
    int32_t run = bstart[static_cast<int64_t>(sig) * NB + j] + static_cast<int32_t>(S[c * NB + j]);
    for (int64_t t = t0; t < t1; ++t) {
      B[t * NB + j] = run;
      run += static_cast<int32_t>(A[t * NB + j]);
    }
  }
}

// ---------------------------------------------------------------- scatter
// Same walk as route() on 32-bit values: the coordinates were range-checked
// (below 2^30) and the all-left splitter becomes 0xFFFFFFFF, above every one.
template <int D>
__device__ inline int route32(const uint32_t (&c)[D], const uint32_t* sx, const uint8_t* sdim, int lambda) {
  int v = 1;
  for (int l = 0; l < lambda; ++l) {
    const int d = sdim[v];
    const uint32_t x = sx[v];
    int ge = 0;
#pragma unroll
    for (int e = 0; e < D; ++e) ge |= (d == e) & (c[e] >= x);
    v = 2 * v + ge;
  }
  return v - (1 << lambda);
}

// LDS of one scatter workgroup, sized for 2^lambda buckets.
struct ScatterLayout {
  size_t stage, sx, cur, cnt, ls, sd, slab, end;
  __host__ __device__ ScatterLayout(int T, int lambda) {
    const int NB = 1 << lambda, NCH = T / 64;
    size_t o = 0;
    stage = o; o += sizeof(int64_t) * T;
    sx = o;    o += sizeof(uint32_t) * NB;
    cur = o;   o += sizeof(int32_t) * NB;
    cnt = o;   o += sizeof(uint16_t) * NCH * NB;
    ls = o;    o += sizeof(uint16_t) * (NB + 2);
    sd = o;    o += NB;
    slab = o;  o += T;
    end = (o + 15) & ~size_t{15};
  }
};

// Stable distribution of one tile.  Each wave ranks its 64 consecutive points
// among equal labels with ballots; chunk counts are scanned in LDS; every
// array (D coordinates, then ids) is staged in LDS in bucket order and written
// out as contiguous runs.
template <int D, int PPT>
__global__ void __launch_bounds__(kBlock) k_scatter(const Task* sp, int ns, const int64_t* tile_off, Bufs bufs,
                                                    int src, int dst, const int64_t* rx, const uint8_t* rdim,
                                                    const int8_t* mode, int lambda, const int32_t* B,
                                                    const int* dns = nullptr) {
  constexpr int T = kBlock * PPT;
  constexpr int NCH = T / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const ScatterLayout lay(T, lambda);
  int64_t* stage = reinterpret_cast<int64_t*>(smem + lay.stage);
  uint32_t* sx = reinterpret_cast<uint32_t*>(smem + lay.sx);
  int32_t* cur = reinterpret_cast<int32_t*>(smem + lay.cur);
  uint16_t* cnt = reinterpret_cast<uint16_t*>(smem + lay.cnt);   // [NCH][NB]
  uint16_t* ls = reinterpret_cast<uint16_t*>(smem + lay.ls);
  uint8_t* sd = smem + lay.sd;
  uint8_t* slab = smem + lay.slab;
  __shared__ int sig_sh;
  const int NB = 1 << lambda;
  int64_t ntiles = gridDim.x;
  if (dns) {
    // the grid is sized for the most tiles a round can have: the blocks past
    // this round's tiles leave, the others map as in an exact grid
    ns = *dns;
    ntiles = tile_off[ns];
    if (static_cast<int64_t>(blockIdx.x) >= ntiles) return;
  }
  const int64_t t = xcd_tile(blockIdx.x, ntiles);
  const int tid = threadIdx.x;
  if (tid == 0) sig_sh = find_owner(tile_off, ns, t);
  for (int i = tid; i < NCH * NB; i += kBlock) cnt[i] = 0;
  __syncthreads();
  const int sig = sig_sh;
  if (mode[sig] == 1) return;
  const Task q = sp[sig];
  for (int j = tid; j < NB; j += kBlock) {
    const int64_t x = rx[static_cast<int64_t>(sig) * NB + j];
    sx[j] = x == kAllLeft ? 0xFFFFFFFFu : static_cast<uint32_t>(x);
    sd[j] = rdim[static_cast<int64_t>(sig) * NB + j];
    cur[j] = B[t * NB + j];
  }
  __syncthreads();
  const int64_t lo = q.start + (t - tile_off[sig]) * T;
  const int len = static_cast<int>(min<int64_t>(T, static_cast<int64_t>(q.start) + q.m - lo));
  const int64_t* X = bufs.c[src];
  const int64_t cap = bufs.cap[src];
  const uint32_t lane = lane_id();
  const int wave = tid >> 6;
  const unsigned long long lt = (1ULL << lane) - 1;
  // coordinates were range-checked before this pass: 30-bit values fit 32 bits
  uint32_t val[PPT][D];
  int64_t idv[PPT];   // ids are loaded with the coordinates so all loads are in flight together
  int lr[PPT];        // label << 8 | rank among equal labels of the wave
  const int64_t* Iin = bufs.id[src];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = k * kBlock + tid;
    const bool ok = li < len;
    idv[k] = ok ? Iin[lo + li] : 0;
#pragma unroll
    for (int d = 0; d < D; ++d) val[k][d] = ok ? static_cast<uint32_t>(X[d * cap + lo + li]) : 0u;
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = k * kBlock + tid;
    const bool ok = li < len;
    const int label = ok ? route32<D>(val[k], sx, sd, lambda) : 0;
    unsigned long long peers = __ballot(ok);
    for (int b = 0; b < lambda; ++b) {
      unsigned long long m = __ballot((label >> b) & 1);
      peers &= ((label >> b) & 1) ? m : ~m;
    }
    lr[k] = (label << 8) | __popcll(peers & lt);
    const int ch = k * (kBlock / 64) + wave;
    if (ok && (peers & lt) == 0) cnt[ch * NB + label] = static_cast<uint16_t>(__popcll(peers));
  }
  __syncthreads();
  for (int j = tid; j < NB; j += kBlock) {
    uint16_t run = 0;
    for (int ch = 0; ch < NCH; ++ch) {
      uint16_t x = cnt[ch * NB + j];
      cnt[ch * NB + j] = run;
      run += x;
    }
    ls[j] = run;   // total of bucket j in this tile, scanned below
  }
  __syncthreads();
  if (tid == 0) {
    uint16_t run = 0;
    for (int j = 0; j < NB; ++j) {
      uint16_t x = ls[j];
      ls[j] = run;
      run += x;
    }
    ls[NB] = run;
  }
  __syncthreads();
  int lpos[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = k * kBlock + tid;
    const int ch = k * (kBlock / 64) + wave;
    lpos[k] = -1;
    if (li < len) {
      const int label = lr[k] >> 8;
      lpos[k] = ls[label] + cnt[ch * NB + label] + (lr[k] & 0xFF);
      slab[lpos[k]] = static_cast<uint8_t>(label);
    }
  }
  __syncthreads();
  int64_t* Y = bufs.c[dst];
  const int64_t ycap = bufs.cap[dst];
  int64_t* Iout = bufs.id[dst];
#pragma unroll
  for (int a = 0; a <= D; ++a) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (lpos[k] >= 0) stage[lpos[k]] = a < D ? static_cast<int64_t>(val[k][a < D ? a : 0]) : idv[k];
    }
    __syncthreads();
    int64_t* out = a < D ? Y + a * ycap : Iout;
    for (int p = tid; p < len; p += kBlock) {
      const int j = slab[p];
      out[cur[j] + (p - ls[j])] = stage[p];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------- emit
// Skeleton nodes of each subproblem become tree nodes; its buckets become
// tasks of the next round.  One workgroup of 64 threads per subproblem; the
// heap is processed level by level.
// Four subproblems per workgroup, one per wave: the waves reserve their node
// slots and their next-front entries with one counter update per workgroup
// each (one update per subproblem serialized on the two counters when
// thousands of subproblems emit at once).
constexpr int kEmitWaves = 4;

// Per wave: `count` items to reserve on `counter`; returns the wave's first
// slot.  Every thread of the workgroup calls it.
__device__ inline int block_reserve(int wave, int count, int* counter) {
  __shared__ int wcnt[kEmitWaves], wbase[kEmitWaves];
  if ((threadIdx.x & 63) == 0) wcnt[wave] = count;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kEmitWaves; ++w) {
      wbase[w] = t;
      t += wcnt[w];
    }
    const int b = t > 0 ? atomicAdd(counter, t) : 0;
    for (int w = 0; w < kEmitWaves; ++w) wbase[w] += b;
  }
  __syncthreads();
  return wbase[wave];
}

__global__ void __launch_bounds__(64 * kEmitWaves) k_emit(const Task* sp, int ns, int lambda, const int64_t* rx,
                                                          const uint8_t* rdim, const int8_t* ext, const int8_t* mode,
                                                          const int32_t* bsize, const int32_t* bstart, int dst,
                                                          Node* nodes, int* node_count, Task* front, int* n_front,
                                                          Task* fin, int* n_fin, int* flags,
                                                          const int* dns = nullptr) {
  ns = dev_count(dns, ns);
  if (static_cast<int>(blockIdx.x) * kEmitWaves >= ns) return;   // the whole workgroup has nothing
  const int NB = 1 << lambda;
  const int nheap = 2 << lambda;
  constexpr int H = 2 << kMaxLambda;
  __shared__ int32_t size_[kEmitWaves][H], off_[kEmitWaves][H], idx_[kEmitWaves][H];
  __shared__ uint8_t reach_[kEmitWaves][H], exs_[kEmitWaves][H];
  const int wave = threadIdx.x >> 6, tid = threadIdx.x & 63;
  int32_t* size = size_[wave];
  int32_t* off = off_[wave];
  int32_t* idx = idx_[wave];
  uint8_t* reach = reach_[wave];
  uint8_t* exs = exs_[wave];
  const int sig = blockIdx.x * kEmitWaves + wave;
  // a wave emits unless it has no subproblem or a heavy leaf of identical
  // points (one finisher task, data staying where it is)
  bool active = sig < ns;
  Task q{};
  if (active) {
    q = sp[sig];
    if (mode[sig] == 1) {
      if (tid == 0) {
        Task h = q;
        h.mode = 1;
        fin[atomicAdd(n_fin, 1)] = h;
      }
      active = false;
    }
  }
  if (active) {
    const int8_t* ex = ext + static_cast<int64_t>(sig) * nheap;
    for (int v = tid; v < nheap; v += 64) exs[v] = ex[v];
    for (int j = tid; j < NB; j += 64) {
      size[NB + j] = bsize[static_cast<int64_t>(sig) * NB + j];
      off[NB + j] = bstart[static_cast<int64_t>(sig) * NB + j];
    }
    wave_sync();
    for (int l = lambda - 1; l >= 0; --l) {
      for (int v = (1 << l) + tid; v < (2 << l); v += 64) {
        size[v] = size[2 * v] + size[2 * v + 1];
        off[v] = off[2 * v];
      }
      wave_sync();
    }
    if (tid == 0) reach[1] = 1;
    wave_sync();
    for (int l = 1; l <= lambda; ++l) {
      for (int v = (1 << l) + tid; v < (2 << l); v += 64) reach[v] = reach[v >> 1] && !exs[v >> 1];
      wave_sync();
    }
  }
  // rank the reachable heap nodes other than the root in heap order
  const int per = (nheap + 63) / 64;
  const int b = tid * per, e = min(nheap, b + per);
  int cnt = 0;
  if (active)
    for (int v = max(b, 2); v < e; ++v) cnt += reach[v];
  int incl = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (tid >= o) incl += y;
  }
  const int nbase = block_reserve(wave, __shfl(incl, 63), node_count);
  // external (next-round) nodes of this subproblem, counted per wave
  int n_ext = 0;
  if (active) {
    for (int base = 0; base < nheap; base += 64) {
      const int v = base + tid;
      n_ext += __popcll(__ballot(v >= 1 && v < nheap && reach[v] && exs[v]));
    }
  }
  const int fbase = block_reserve(wave, n_ext, n_front);
  if (!active) return;
  int r = nbase + incl - cnt;
  for (int v = max(b, 2); v < e; ++v)
    if (reach[v]) idx[v] = r++;
  if (tid == 0) idx[1] = q.slot;
  wave_sync();
  const int64_t* sxv = rx + static_cast<int64_t>(sig) * NB;
  const uint8_t* sdv = rdim + static_cast<int64_t>(sig) * NB;
  const unsigned long long lt = (1ULL << tid) - 1;
  int fpos = fbase;
  for (int base = 0; base < nheap; base += 64) {
    const int v = base + tid;
    const bool live = v >= 1 && v < nheap && reach[v];
    const bool interior = live && !exs[v];
    const bool external = live && exs[v];
    if (interior) {
      const int level = 31 - __clz(v);
      Node nd;
      nd.x = sxv[v];
      nd.size = size[v];
      nd.off = off[v];
      nd.left = idx[2 * v];
      nd.right = idx[2 * v + 1];
      nd.dim = sdv[v];
      nd.depth = static_cast<int16_t>(q.depth + level);
      nd.pad = 0;
      nodes[idx[v]] = nd;
    }
    const unsigned long long em = __ballot(external);
    if (external) {
      const int level = 31 - __clz(v);
      if (size[v] <= 0) atomicOr(flags, kErrInternal);
      Task c;
      c.start = off[v];
      c.m = size[v];
      c.slot = idx[v];
      c.depth = static_cast<int16_t>(q.depth + level);
      c.buf = static_cast<int8_t>(dst);
      c.mode = 0;
      front[fpos + __popcll(em & lt)] = c;
    }
    fpos += __popcll(em);
  }
}

// ---------------------------------------------------------------- finisher
// Plain construction of a subproblem of m < s points (Section 3: median split
// on the widest dimension, one level at a time) in LDS, one workgroup of D
// waves per subproblem: wave d sorts dimension d and keeps that order
// partitioned as the nodes split.  P >= m is the padded size of the launch's
// class (64 * NPL).
// Node slots: each task owns a reserved range [res_base + res_off[i],
// res_base + res_off[i+1]) sized for distinct coordinates; a task that needs
// more (duplicates) takes the rest from the shared overflow counter.
// One task (every thread of the workgroup calls it).
template <int D, int NPL>
__device__ __forceinline__ void finish_task(int ti, const Task* tasks, int P, Bufs bufs, int final_buf, int phi,
                                            Node* nodes, int* overflow_ctr, int64_t node_cap, int* height,
                                            int* flags, const int32_t* res_off, int32_t res_base) {
  constexpr int NT = 64 * D;
  extern __shared__ __align__(16) unsigned char smem[];
  const Task q = tasks[ti];
  const int m = q.m;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const FinLayout lay(D, P, phi);
  uint32_t* C = reinterpret_cast<uint32_t*>(smem + lay.C);
  uint16_t* O = reinterpret_cast<uint16_t*>(smem + lay.O);
  uint16_t* seg = reinterpret_cast<uint16_t*>(smem + lay.seg);
  uint8_t* flag = smem + lay.flag;
  // the two levels' segment lists lie back to back (list 1 = list 0 + MS);
  // they are addressed by offset from smem, not through a table of
  // pointers, which the compiler turned into flat (non-LDS) accesses
  uint16_t* const lA0 = reinterpret_cast<uint16_t*>(smem + lay.lA0);
  uint16_t* const lL0 = reinterpret_cast<uint16_t*>(smem + lay.lL0);
  int32_t* const lN0 = reinterpret_cast<int32_t*>(smem + lay.lN0);
  const int MS = lay.MS;
  uint32_t* sxs = reinterpret_cast<uint32_t*>(smem + lay.sxs);
  uint16_t* snl = reinterpret_cast<uint16_t*>(smem + lay.snl);
  uint16_t* srank = reinterpret_cast<uint16_t*>(smem + lay.srank);
  uint16_t* segF = reinterpret_cast<uint16_t*>(smem + lay.segF);
  uint8_t* sdm = smem + lay.sdm;
  uint8_t* ssplit = smem + lay.ssplit;
  __shared__ int sh_nlist, sh_nsplit, sh_base, sh_over, sh_maxdepth, sh_next, sh_more;
  const int res_end = res_base + res_off[ti + 1];

  const int src = q.buf;
  const int64_t* X = bufs.c[src];
  const int64_t xcap = bufs.cap[src];
  bool bad = false;
  for (int i = tid; i < m; i += NT) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t v = X[d * xcap + q.start + i];
      bad |= static_cast<uint64_t>(v) >= static_cast<uint64_t>(coord_limit(D));
      C[d * P + i] = static_cast<uint32_t>(v);
    }
    seg[i] = 0;
  }
  if (bad) atomicOr(flags, kErrRange);
  if (tid == 0) {
    sh_nlist = 1;
    sh_over = 0;
    sh_maxdepth = 0;
    sh_next = res_base + res_off[ti];
    lA0[0] = 0;
    lL0[0] = static_cast<uint16_t>(m);
    lN0[0] = q.slot;
  }
  __syncthreads();
  if (m > phi) {
    // wave d: the points ordered by (coordinate d, index)
    uint64_t k[NPL];
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int e = lane * NPL + r;
      k[r] = e < m ? (static_cast<uint64_t>(C[wave * P + e]) << 16) | static_cast<uint64_t>(e) : ~0ULL;
    }
    wave_bitonic<NPL>(k);
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int e = lane * NPL + r;
      if (e < m) O[wave * P + e] = static_cast<uint16_t>(k[r] & 0xFFFF);
    }
  } else {
    for (int i = tid; i < m; i += NT) O[i] = static_cast<uint16_t>(i);
  }
  __syncthreads();
  int cur = 0;
  int depth = q.depth;
  while (true) {
    const int nl = sh_nlist;
    if (nl == 0) break;
    if (tid == 0) sh_more = 0;
    __syncthreads();
    // decide every segment of this level
    for (int k = tid; k < nl; k += NT) {
      const int a = (lA0 + cur * MS)[k], L = (lL0 + cur * MS)[k];
      int d = 0, nleft = 0;
      uint32_t x = 0;
      bool split = L > phi && lds_split_rule<D>(C, O, P, a, L, &d, &x, &nleft);
      if (split && (nleft <= 0 || nleft >= L)) {
        atomicOr(flags, kErrInternal);
        split = false;
      }
      ssplit[k] = split ? 1 : 0;
      if (split) {
        sdm[k] = static_cast<uint8_t>(d);
        sxs[k] = x;
        snl[k] = static_cast<uint16_t>(nleft);
        if (nleft > phi || L - nleft > phi) sh_more = 1;   // a child splits again
      } else {
        // leaf (at most phi points, or a heavy leaf of identical points)
        Node nd;
        nd.x = 0;
        nd.size = L;
        nd.off = q.start + a;
        nd.left = -1;
        nd.right = -1;
        nd.dim = -1;
        nd.depth = static_cast<int16_t>(depth);
        nd.pad = 0;
        const int32_t at = (lN0 + cur * MS)[k];
        if (at < node_cap) nodes[at] = nd;
        atomicMax(&sh_maxdepth, depth);
      }
    }
    __syncthreads();
    if (wave == 0) {
      // ranks of the splitting segments among themselves (ballot prefix)
      const unsigned long long lt = (1ULL << lane) - 1;
      int r = 0;
      for (int base = 0; base < nl; base += 64) {
        const int k = base + lane;
        const bool spl = k < nl && ssplit[k];
        const unsigned long long mk = __ballot(spl);
        if (k < nl) srank[k] = static_cast<uint16_t>(r + __popcll(mk & lt));
        r += __popcll(mk);
      }
      if (lane == 0) {
        sh_nsplit = r;
        int b = 0;
        if (r > 0) {
          if (sh_next + 2 * r <= res_end) {
            b = sh_next;
            sh_next += 2 * r;
          } else {
            b = atomicAdd(overflow_ctr, 2 * r);
          }
        }
        if (static_cast<int64_t>(b) + 2 * r > node_cap) sh_over = 1;
        sh_base = b;
      }
    }
    __syncthreads();
    const int nsplit = sh_nsplit;
    const int nbase = sh_base;
    const bool over = sh_over != 0;
    const int nxt = cur ^ 1;
    for (int k = tid; k < nl; k += NT) {
      if (!ssplit[k]) continue;
      const int a = (lA0 + cur * MS)[k], L = (lL0 + cur * MS)[k], r = srank[k];
      const int cl = nbase + 2 * r, cr = cl + 1;
      if (!over && (lN0 + cur * MS)[k] < node_cap) {
        Node nd;
        nd.x = sxs[k];
        nd.size = L;
        nd.off = q.start + a;
        nd.left = cl;
        nd.right = cr;
        nd.dim = sdm[k];
        nd.depth = static_cast<int16_t>(depth);
        nd.pad = 0;
        nodes[(lN0 + cur * MS)[k]] = nd;
      }
      (lA0 + nxt * MS)[2 * r] = static_cast<uint16_t>(a);
      (lL0 + nxt * MS)[2 * r] = snl[k];
      (lN0 + nxt * MS)[2 * r] = cl;
      (lA0 + nxt * MS)[2 * r + 1] = static_cast<uint16_t>(a + snl[k]);
      (lL0 + nxt * MS)[2 * r + 1] = static_cast<uint16_t>(L - snl[k]);
      (lN0 + nxt * MS)[2 * r + 1] = cr;
    }
    if (nsplit == 0) break;
    // side flags of the points of splitting segments
    for (int e = tid; e < m; e += NT) {
      const int k = seg[e];
      flag[e] = (k != kNone && ssplit[k]) ? (C[sdm[k] * P + e] < sxs[k] ? 1 : 0) : 0;
    }
    __syncthreads();
    // wave d partitions order d; on the last splitting level only the order
    // that is written out (dimension 0) matters
    const bool active = wave < (sh_more ? D : 1);
    wave_partition<NPL>(active, O + wave * P, m, seg, ssplit, (lA0 + cur * MS), snl, flag, segF + wave * MS);
    __syncthreads();
    for (int e = tid; e < m; e += NT) {
      const int k = seg[e];
      if (k == kNone) continue;
      seg[e] = ssplit[k] ? static_cast<uint16_t>(2 * srank[k] + (flag[e] ? 0 : 1)) : kNone;
    }
    if (tid == 0) sh_nlist = 2 * nsplit;
    __syncthreads();
    cur = nxt;
    ++depth;
  }
  __syncthreads();
  // reserved slots this task did not use become dead records
  for (int i = sh_next + tid; i < res_end; i += NT) {
    if (i >= node_cap) break;
    Node dead;
    dead.x = 0;
    dead.size = 0;
    dead.off = 0;
    dead.left = dead.right = -1;
    dead.dim = -1;
    dead.depth = 0;
    dead.pad = 1;
    nodes[i] = dead;
  }
  if (sh_over) {
    if (tid == 0) atomicOr(flags, kErrNodeOverflow);
    return;
  }
  if (tid == 0 && sh_maxdepth > *reinterpret_cast<volatile int*>(height)) atomicMax(height, sh_maxdepth);
  // ids are gathered into registers before any is written: the source and
  // destination arrays may be the same
  constexpr int PER = (64 * NPL + NT - 1) / NT;
  const int64_t* Isrc = bufs.id[src] + q.start;
  int64_t idv[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int p = r * NT + tid;
    idv[r] = p < m ? Isrc[O[p]] : 0;
  }
  __syncthreads();
  int64_t* Y = bufs.c[final_buf];
  const int64_t ycap = bufs.cap[final_buf];
  int64_t* Iout = bufs.id[final_buf] + q.start;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int p = r * NT + tid;
    if (p < m) {
      const int e = O[p];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        Y[d * ycap + q.start + p] = static_cast<int64_t>(C[d * P + e]);
        bufs.c32[(static_cast<int64_t>(q.start) + p) * D + d] = static_cast<int32_t>(C[d * P + e]);
      }
      Iout[p] = idv[r];
    }
  }
}

template <int D, int NPL>
__global__ void __launch_bounds__(64 * D) __attribute__((amdgpu_waves_per_eu(NPL <= 8 ? 8 : 1))) k_finish(const Task* tasks, const int* list, int P, Bufs bufs, int final_buf,
                                                     int phi, Node* nodes, int* overflow_ctr, int64_t node_cap,
                                                     int* height, int* flags, const int32_t* res_off,
                                                     int32_t res_base, const int* count = nullptr,
                                                     const int* res_base_d = nullptr) {
  // with `count` set (launches sized for the most tasks the class can hold)
  // the blocks past the class's count leave, and the reservation base is the
  // one in device memory
  if (count) {
    if (static_cast<int>(blockIdx.x) >= *count) return;
    res_base = *res_base_d;
  }
  finish_task<D, NPL>(list[blockIdx.x], tasks, P, bufs, final_buf, phi, nodes, overflow_ctr, node_cap, height, flags,
                      res_off, res_base);
}

// Persistent form for launches enqueued without host reads: a fixed grid
// walks the class list up to its count in device memory; the base of the
// node reservations is read from device memory too.
template <int D, int NPL>
__global__ void __launch_bounds__(64 * D) __attribute__((amdgpu_waves_per_eu(NPL <= 8 ? 8 : 1))) k_finish_persist(const Task* tasks, const int* list, const int* count, int P, Bufs bufs,
                                                     int final_buf, int phi, Node* nodes, int* overflow_ctr,
                                                     int64_t node_cap, int* height, int* flags,
                                                     const int32_t* res_off, const int* res_base) {
  const int n = *count;
  const int32_t base = *res_base;
  for (int b = blockIdx.x; b < n; b += gridDim.x) {
    // the layout and everything derived from (P, phi) are recomputed per
    // task: hoisted out of the loop they stayed live and spilled
    int P_t = P, phi_t = phi;
    asm volatile("" : "+s"(P_t), "+s"(phi_t));
    finish_task<D, NPL>(list[b], tasks, P_t, bufs, final_buf, phi_t, nodes, overflow_ctr, node_cap, height, flags,
                        res_off, base);
    __syncthreads();   // the next task reuses the LDS
  }
}

// Heavy leaf of identical points found by the sieve (m may exceed any LDS
// size): copy the points into the tree array and write one leaf.
// With `dn` set the launch covers n_fin slots of which the first *dn are
// tasks; the others get 0.
__global__ void k_fin_reserve(const Task* fin, int n_fin, int phi, int32_t* R, const int* dn = nullptr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_fin) return;
  if (dn && i >= *dn) {
    R[i] = 0;
    return;
  }
  const Task t = fin[i];
  // a plain build of m distinct points with leaves of at most phi points has
  // at most about 2m/(phi+1) leaves, so fewer than 4m/(phi+1)+4 nodes below the root
  R[i] = (t.mode == 1 || t.m <= phi) ? 0 : 4 * t.m / (phi + 1) + 4;
}

// With `count` set, a fixed grid walks the list up to *count.
__global__ void k_finish_heavy(const Task* tasks, const int* list, int D, Bufs bufs, int final_buf, Node* nodes,
                               int* height, const int* count = nullptr) {
  const int n = count ? *count : static_cast<int>(gridDim.x);
  for (int b = blockIdx.x; b < n; b += gridDim.x) {
    const Task q = tasks[list[b]];
    const int src = q.buf;
    for (int64_t i = threadIdx.x; i < q.m; i += blockDim.x) {
      for (int d = 0; d < D; ++d) {
        const int64_t v = bufs.c[src][d * bufs.cap[src] + q.start + i];
        if (src != final_buf) bufs.c[final_buf][d * bufs.cap[final_buf] + q.start + i] = v;
        bufs.c32[(static_cast<int64_t>(q.start) + i) * D + d] = static_cast<int32_t>(v);
      }
      if (src != final_buf) bufs.id[final_buf][q.start + i] = bufs.id[src][q.start + i];
    }
    if (threadIdx.x == 0) {
      Node nd;
      nd.x = 0;
      nd.size = q.m;
      nd.off = q.start;
      nd.left = -1;
      nd.right = -1;
      nd.dim = -1;
      nd.depth = q.depth;
      nd.pad = 0;
      nodes[q.slot] = nd;
      atomicMax(height, static_cast<int>(q.depth));
    }
  }
}

// Sort finisher tasks into classes by padded size (64, 128, ..., 4096) and
// heavy leaves (class 7).
__global__ void k_bin_finish(const Task* fin, int n_fin, int* lists, int stride, int* counts, const int* dn = nullptr) {
  n_fin = dev_count(dn, n_fin);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < n_fin;
  int cls = -1;
  if (ok) {
    const Task t = fin[i];
    cls = 7;
    if (t.mode == 0) {
      cls = 0;
      while ((64 << cls) < t.m) ++cls;
    }
  }
  // one counter update per class and workgroup (one per wave serialized
  // tens of thousands of atomics on each of the 8 counters)
  __shared__ int wcnt[8][16];
  __shared__ int wbase[8];
  const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  const unsigned long long below = (1ULL << (threadIdx.x & 63)) - 1;
  int rank = 0;
  for (int c = 0; c < 8; ++c) {
    const unsigned long long m = __ballot(cls == c);
    if (cls == c) rank = static_cast<int>(__popcll(m & below));
    if ((threadIdx.x & 63) == 0) wcnt[c][wave] = static_cast<int>(__popcll(m));
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int c = threadIdx.x;
    int run = 0;
    for (int w = 0; w < nw; ++w) {
      const int x = wcnt[c][w];
      wcnt[c][w] = run;
      run += x;
    }
    wbase[c] = run ? atomicAdd(counts + c, run) : 0;
  }
  __syncthreads();
  if (cls >= 0) lists[cls * stride + wbase[cls] + wcnt[cls][wave] + rank] = i;
}

// ------------------------------------------- segmented exact split
// For every subproblem of a list at once (the rounds of the exact-median
// construction, or the subproblems whose sample was entirely identical): the
// split rule on all of the subproblem's points.  Per-dimension min and max;
// the widest dimension, lowest index on ties (none: all points identical, a
// heavy leaf); the upper median v[floor(m/2)] on it by a radix selection
// (digits of 8, 8, 8 and 6 bits of the 30-bit coordinates, one counting pass
// each); if that equals the minimum, the next larger distinct value.  The
// result is written as a skeleton whose root splits and whose two children
// are external (buckets 0 and 2^(lambda-1)).
template <int D>
__global__ void __launch_bounds__(kBlock) k_seg_minmax(const Task* sp, int ns, const int64_t* tile_off, int tile,
                                                       Bufs bufs, int src, unsigned long long* mn,
                                                       unsigned long long* mx) {
  __shared__ int sig_sh;
  const int64_t t = blockIdx.x;
  if (threadIdx.x == 0) sig_sh = find_owner(tile_off, ns, t);
  __syncthreads();
  const int sig = sig_sh;
  const Task q = sp[sig];
  const int64_t lo = q.start + (t - tile_off[sig]) * tile;
  const int64_t hi = min<int64_t>(lo + tile, static_cast<int64_t>(q.start) + q.m);
  const int64_t* X = bufs.c[src];
  const int64_t cap = bufs.cap[src];
  unsigned long long a[D], b[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    a[d] = ~0ULL;
    b[d] = 0;
  }
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const unsigned long long v = static_cast<unsigned long long>(X[d * cap + i]);
      a[d] = v < a[d] ? v : a[d];
      b[d] = v > b[d] ? v : b[d];
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long x = __shfl_xor(a[d], o), y = __shfl_xor(b[d], o);
      a[d] = x < a[d] ? x : a[d];
      b[d] = y > b[d] ? y : b[d];
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(mn + static_cast<int64_t>(sig) * D + d, a[d]);
      atomicMax(mx + static_cast<int64_t>(sig) * D + d, b[d]);
    }
  }
}

__global__ void k_seg_init(int ns, int D, unsigned long long* mn, unsigned long long* mx, unsigned long long* above,
                           unsigned int* hist) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < static_cast<int64_t>(ns) * 256;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    hist[i] = 0;
    if (i < static_cast<int64_t>(ns) * D) {
      mn[i] = ~0ULL;
      mx[i] = 0;
    }
    if (i < ns) above[i] = ~0ULL;
  }
}

__global__ void k_seg_pick(const Task* sp, int ns, int D, const unsigned long long* mn, const unsigned long long* mx,
                           int32_t* sdim, int64_t* rank, unsigned long long* prefix) {
  const int sig = blockIdx.x * blockDim.x + threadIdx.x;
  if (sig >= ns) return;
  int best = -1;
  unsigned long long bw = 0;
  for (int d = 0; d < D; ++d) {
    const unsigned long long w = mx[static_cast<int64_t>(sig) * D + d] - mn[static_cast<int64_t>(sig) * D + d];
    if (w > bw) {
      bw = w;
      best = d;
    }
  }
  sdim[sig] = best;   // -1: every point identical
  rank[sig] = sp[sig].m / 2;
  prefix[sig] = 0;
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_seg_hist(const Task* sp, int ns, const int64_t* tile_off, int tile,
                                                     Bufs bufs, int src, const int32_t* sdim,
                                                     const unsigned long long* prefix, int pshift, int dshift,
                                                     int dmask, unsigned int* hist) {
  __shared__ unsigned int h[256];
  __shared__ int sig_sh;
  const int64_t t = blockIdx.x;
  if (threadIdx.x == 0) sig_sh = find_owner(tile_off, ns, t);
  for (int i = threadIdx.x; i < 256; i += kBlock) h[i] = 0;
  __syncthreads();
  const int sig = sig_sh;
  const int d = sdim[sig];
  if (d < 0) return;
  const Task q = sp[sig];
  const int64_t lo = q.start + (t - tile_off[sig]) * tile;
  const int64_t hi = min<int64_t>(lo + tile, static_cast<int64_t>(q.start) + q.m);
  const int64_t* Xd = bufs.c[src] + d * bufs.cap[src];
  const unsigned long long pre = prefix[sig];
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    const unsigned long long v = static_cast<unsigned long long>(Xd[i]);
    if (pshift >= 64 || (v >> pshift) == pre) atomicAdd(&h[(v >> dshift) & dmask], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += kBlock)
    if (h[i]) atomicAdd(hist + static_cast<int64_t>(sig) * 256 + i, h[i]);
}

__global__ void k_seg_digit(int ns, const int32_t* sdim, unsigned int* hist, int nbins, int bits, int64_t* rank,
                            unsigned long long* prefix) {
  const int sig = blockIdx.x * blockDim.x + threadIdx.x;
  if (sig >= ns || sdim[sig] < 0) return;
  unsigned int* hs = hist + static_cast<int64_t>(sig) * 256;
  int64_t r = rank[sig];
  int b = 0;
  for (; b < nbins - 1; ++b) {
    if (r < static_cast<int64_t>(hs[b])) break;
    r -= hs[b];
  }
  rank[sig] = r;
  prefix[sig] = (prefix[sig] << bits) | static_cast<unsigned long long>(b);
  for (int i = 0; i < 256; ++i) hs[i] = 0;
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_seg_min_above(const Task* sp, int ns, const int64_t* tile_off, int tile,
                                                          Bufs bufs, int src, const int32_t* sdim,
                                                          const unsigned long long* mn,
                                                          const unsigned long long* prefix,
                                                          unsigned long long* above) {
  __shared__ int sig_sh;
  const int64_t t = blockIdx.x;
  if (threadIdx.x == 0) sig_sh = find_owner(tile_off, ns, t);
  __syncthreads();
  const int sig = sig_sh;
  const int d = sdim[sig];
  if (d < 0) return;
  const unsigned long long v0 = mn[static_cast<int64_t>(sig) * D + d];
  if (prefix[sig] != v0) return;   // the median already exceeds the minimum
  const Task q = sp[sig];
  const int64_t lo = q.start + (t - tile_off[sig]) * tile;
  const int64_t hi = min<int64_t>(lo + tile, static_cast<int64_t>(q.start) + q.m);
  const int64_t* Xd = bufs.c[src] + d * bufs.cap[src];
  unsigned long long best = ~0ULL;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    const unsigned long long v = static_cast<unsigned long long>(Xd[i]);
    if (v > v0 && v < best) best = v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(best, o);
    best = x < best ? x : best;
  }
  if ((threadIdx.x & 63) == 0 && best != ~0ULL) atomicMin(above + sig, best);
}

// The split as a skeleton row of subproblem map[i] (or i): root splits,
// children 2 and 3 external; mode 1 (heavy leaf) when all points are equal.
__global__ void k_seg_finish(int ns, int D, int lambda, const int* map, const int32_t* sdim,
                             const unsigned long long* mn, const unsigned long long* prefix,
                             const unsigned long long* above, int64_t* rx, uint8_t* rdim, int8_t* ext, int8_t* mode) {
  const int i = blockIdx.x;
  const int sig = map ? map[i] : i;
  const int NB = 1 << lambda, nheap = 2 << lambda;
  const int d = sdim[i];
  unsigned long long x = prefix[i];
  if (d >= 0 && x == mn[static_cast<int64_t>(i) * D + d]) x = above[i];
  for (int v = threadIdx.x; v < nheap; v += blockDim.x) {
    if (v < NB) {
      rx[static_cast<int64_t>(sig) * NB + v] = (v == 1 && d >= 0) ? static_cast<int64_t>(x) : kAllLeft;
      rdim[static_cast<int64_t>(sig) * NB + v] = (v == 1 && d >= 0) ? static_cast<uint8_t>(d) : 0;
    }
    ext[static_cast<int64_t>(sig) * nheap + v] = (v == 2 || v == 3) ? 1 : 0;
  }
  if (threadIdx.x == 0) mode[sig] = d >= 0 ? 2 : 1;
}

__global__ void k_gather_tasks(const Task* all, const int* list, int n, Task* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = all[list[i]];
}

// ------------------------------------------------------------ host helpers
template <class K>
int allow_lds(K kernel, size_t bytes) {
  PKD_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(bytes)));
  return PKD_OK;
}

template <int D>
size_t select_lds_bytes(int s) {
  return SkelLayout(D, std::max(64, next_pow2(s))).end;
}

template <int D>
size_t finish_lds_bytes(int P, int phi) {
  return FinLayout(D, P, phi).end;
}

// Scratch of the segmented exact split.
struct ExactWork {
  DArr<Task> sub;
  DArr<unsigned long long> mn, mx, prefix, above;
  DArr<int64_t> rank;
  DArr<int32_t> sdim;
  DArr<unsigned int> hist;
  SieveWork W;
  explicit ExactWork(hipStream_t s) : sub(s), mn(s), mx(s), prefix(s), above(s), rank(s), sdim(s), hist(s), W(s) {}
};

// The split rule on all points of ns subproblems at once (tasks: device;
// list: optional device indices of the subproblems within `tasks`, whose rows
// of rx / rdim / ext / mode receive the result).
template <int D>
int seg_exact_split(hipStream_t st, const Task* tasks, const int* list, int ns, int tile, int lambda, int s,
                    const Bufs& bufs, int src, int64_t* rx, uint8_t* rdim, int8_t* ext, int8_t* mode, ExactWork& E) {
  if (ns <= 0) return PKD_OK;
  const Task* sub = tasks;
  if (list) {
    PKD_TRY(E.sub.need(ns));
    hipLaunchKernelGGL(k_gather_tasks, dim3((ns + 255) / 256), dim3(256), 0, st, tasks, list, ns, E.sub.p);
    PKD_TRY(kernel_status("k_gather_tasks"));
    sub = E.sub.p;
  }
  int64_t ntiles = 0, nchunks = 0, pts = 0;
  PKD_TRY(sieve_layout(st, sub, ns, tile, E.W, s, 0, nullptr, &ntiles, &nchunks, &pts));
  PKD_TRY(E.mn.need(static_cast<size_t>(ns) * D));
  PKD_TRY(E.mx.need(static_cast<size_t>(ns) * D));
  PKD_TRY(E.prefix.need(ns));
  PKD_TRY(E.above.need(ns));
  PKD_TRY(E.rank.need(ns));
  PKD_TRY(E.sdim.need(ns));
  PKD_TRY(E.hist.need(static_cast<size_t>(ns) * 256));
  const unsigned gi = static_cast<unsigned>(std::min<int64_t>(65536, (static_cast<int64_t>(ns) * 256 + 255) / 256));
  hipLaunchKernelGGL(k_seg_init, dim3(gi), dim3(256), 0, st, ns, D, E.mn.p, E.mx.p, E.above.p, E.hist.p);
  PKD_TRY(kernel_status("k_seg_init"));
  const dim3 gt(static_cast<unsigned>(ntiles));
  if (ntiles > 0) {
    hipLaunchKernelGGL(k_seg_minmax<D>, gt, dim3(kBlock), 0, st, sub, ns, E.W.tile_off.p, tile, bufs, src, E.mn.p,
                       E.mx.p);
    PKD_TRY(kernel_status("k_seg_minmax"));
  }
  const unsigned gs = static_cast<unsigned>((ns + 255) / 256);
  hipLaunchKernelGGL(k_seg_pick, dim3(gs), dim3(256), 0, st, sub, ns, D, E.mn.p, E.mx.p, E.sdim.p, E.rank.p,
                     E.prefix.p);
  PKD_TRY(kernel_status("k_seg_pick"));
  const int shifts[4] = {22, 14, 6, 0};
  const int bits[4] = {8, 8, 8, 6};
  for (int pass = 0; pass < 4; ++pass) {
    const int pshift = pass == 0 ? 64 : shifts[pass] + bits[pass];
    if (ntiles > 0) {
      hipLaunchKernelGGL(k_seg_hist<D>, gt, dim3(kBlock), 0, st, sub, ns, E.W.tile_off.p, tile, bufs, src, E.sdim.p,
                         E.prefix.p, pshift, shifts[pass], (1 << bits[pass]) - 1, E.hist.p);
      PKD_TRY(kernel_status("k_seg_hist"));
    }
    hipLaunchKernelGGL(k_seg_digit, dim3(gs), dim3(256), 0, st, ns, E.sdim.p, E.hist.p, 1 << bits[pass], bits[pass],
                       E.rank.p, E.prefix.p);
    PKD_TRY(kernel_status("k_seg_digit"));
  }
  if (ntiles > 0) {
    hipLaunchKernelGGL(k_seg_min_above<D>, gt, dim3(kBlock), 0, st, sub, ns, E.W.tile_off.p, tile, bufs, src,
                       E.sdim.p, E.mn.p, E.prefix.p, E.above.p);
    PKD_TRY(kernel_status("k_seg_min_above"));
  }
  hipLaunchKernelGGL(k_seg_finish, dim3(ns), dim3(64), 0, st, ns, D, lambda, list, E.sdim.p, E.mn.p, E.prefix.p,
                     E.above.p, rx, rdim, ext, mode);
  return kernel_status("k_seg_finish");
}

template <int D>
int build_tasks_d(pkd_tree* T, hipStream_t st, const Task* roots, int n_roots, bool roots_on_device, int src_buf,
                  const int64_t* in_c, const int64_t* in_id, int64_t in_cap) {
  const Params& P = T->prm;
  const int NB = 1 << P.lambda;
  const int nheap = 2 << P.lambda;
  const int s = P.s;
  const int tile = P.tile;
  const int cap = 3 * s;            // candidate capacity per subproblem
  const int small_max = 3 * s;      // subproblems up to this size sample from all points
  const int F = T->cur;             // final buffer
  Bufs bufs;
  for (int b = 0; b < 2; ++b) {
    bufs.c[b] = T->buf[b];
    bufs.id[b] = T->buf[b] ? T->buf[b] + static_cast<int64_t>(D) * T->cap : nullptr;
    bufs.cap[b] = T->cap;
  }
  bufs.c[2] = const_cast<int64_t*>(in_c);
  bufs.id[2] = const_cast<int64_t*>(in_id);
  bufs.cap[2] = in_cap;
  PKD_TRY(ensure_c32(T, st));
  bufs.c32 = T->c32;
  bufs.c32cap = T->c32_cap;

  DArr<Task> front(st), next(st), sieve(st), fin(st);
  DArr<int64_t> rx(st);
  DArr<uint32_t> cand_cnt(st), cand_pos(st);
  DArr<uint64_t> cand_key(st);
  DArr<uint8_t> rdim(st);
  DArr<int8_t> ext(st), mode(st), shift_fix(st);
  DArr<int> ctr(st), lists(st), rootext(st);
  SieveWork W(st);
  ExactWork EW(st);

  // counters: 0 n_sieve, 1 n_fin, 2 n_next, 3 node_count, 4 flags, 5 n_root_ext, 6 height, 7 spare
  PKD_TRY(ctr.need(16));
  int hc[16] = {0};
  hc[3] = T->node_count;
  hc[6] = T->height;
  PKD_HIP(hipMemcpyAsync(ctr.p, hc, sizeof(hc), hipMemcpyHostToDevice, st));
  int* d_nsieve = ctr.p + 0;
  int* d_nfin = ctr.p + 1;
  int* d_nnext = ctr.p + 2;
  int* d_nodes = ctr.p + 3;
  int* d_flags = ctr.p + 4;
  int* d_nrootext = ctr.p + 5;
  int* d_height = ctr.p + 6;
  // slots 8-9 (during the rounds): the points of the round's sieve tasks
  unsigned long long* d_spts = reinterpret_cast<unsigned long long*>(ctr.p + 8);
  auto read_pts = [&]() {
    unsigned long long v = 0;
    std::memcpy(&v, hc + 8, sizeof(v));
    return static_cast<int64_t>(v);
  };

  int n_front = n_roots;
  PKD_TRY(front.need(n_front));
  if (n_front > 0)
    PKD_HIP(hipMemcpyAsync(front.p, roots, sizeof(Task) * n_front,
                           roots_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  int src = n_roots == 0 ? 2 : src_buf;
  int dst = 1 - F;
  int n_fin = 0;
  int node_count = T->node_count;
  bool first = true;

  int rounds = 0;
  static const char* const kRoundNames[] = {"sieve round 1", "sieve round 2", "sieve round 3", "sieve round 4",
                                             "sieve round 5", "sieve round 6", "sieve round 7", "sieve round 8+"};
  bool classified = false;   // the front was classified with the last round's emit
  while (n_front > 0) {
    if (++rounds > 200) return PKD_ERR_INTERNAL;   // every round shrinks every subproblem
    TraceRange tr(kRoundNames[std::min(rounds, 8) - 1]);
    if (!classified) {
      PKD_TRY(fin.need(static_cast<size_t>(n_fin) + n_front + 1, true));
      PKD_TRY(sieve.need(n_front));
      PKD_HIP(hipMemsetAsync(d_nsieve, 0, sizeof(int), st));
      PKD_HIP(hipMemsetAsync(d_spts, 0, sizeof(unsigned long long), st));
      hipLaunchKernelGGL(k_classify, dim3((n_front + 255) / 256), dim3(256), 0, st, front.p, n_front, s, sieve.p,
                         d_nsieve, fin.p, d_nfin, static_cast<const int*>(nullptr), d_spts);
      PKD_TRY(kernel_status("k_classify"));
      PKD_HIP(hipMemcpyAsync(hc, ctr.p, sizeof(int) * 10, hipMemcpyDeviceToHost, st));
      PKD_HIP(hipStreamSynchronize(st));
      if (hc[4] & kErrRange) return PKD_ERR_RANGE;
      if (hc[4] & kErrInternal) return PKD_ERR_INTERNAL;
    }
    classified = false;
    const int ns = hc[0];
    const int64_t sieve_pts = read_pts();   // points of this round's sieve tasks
    n_fin = hc[1];
    node_count = hc[3];
    T->node_count = node_count;   // nodes that a growth of the node array must keep
    if (ns == 0) break;

    // tile layout and candidate thresholds
    PKD_TRY(shift_fix.need(ns));
    PKD_TRY(mode.need(ns));
    PKD_HIP(hipMemsetAsync(shift_fix.p, 0xFF, ns, st));
    PKD_HIP(hipMemsetAsync(mode.p, 0, ns, st));
    const int8_t* override_p = nullptr;
    int64_t ntiles = 0, nchunks = 0, round_pts = 0;
    // the tile layout is not read back: its launches take bounds from the
    // round's points and read the task count on the device
    bool bounded = false;
    PKD_TRY(rx.need(static_cast<size_t>(ns) * NB));
    PKD_TRY(rdim.need(static_cast<size_t>(ns) * NB));
    PKD_TRY(ext.need(static_cast<size_t>(ns) * nheap));
    PKD_TRY(rootext.need(ns));
    PKD_TRY(cand_cnt.need(static_cast<size_t>(ns) * kCntStride));
    for (int attempt = 0; P.sigma > 0; ++attempt) {
      PKD_TRY(sieve_layout(st, sieve.p, ns, tile, W, s, small_max, override_p, &ntiles, &nchunks, &round_pts,
                           P.cand_bias, sieve_pts));
      bounded = true;
      PKD_TRY(cand_key.need(static_cast<size_t>(ns) * cap));
      PKD_TRY(cand_pos.need(static_cast<size_t>(ns) * cap));
      PKD_HIP(hipMemsetAsync(cand_cnt.p, 0, sizeof(uint32_t) * kCntStride * ns, st));
#define PKD_CAND(ITER)                                                                                            \
  hipLaunchKernelGGL((k_candidates<ITER>), dim3(static_cast<unsigned>(ntiles)), dim3(kBlock), 0, st, sieve.p, ns, \
                     W.tile_off.p, bufs, src, P.seed, W.shift.p, small_max, cand_key.p, cand_pos.p, cand_cnt.p, cap, \
                     d_nsieve)
      if (tile == 1024) PKD_CAND(4);
      else if (tile == 2048) PKD_CAND(8);
      else PKD_CAND(16);
#undef PKD_CAND
      PKD_TRY(kernel_status("k_candidates"));
      SelectOut so{rx.p, rdim.p, ext.p, rootext.p, d_nrootext, shift_fix.p, d_flags};
      PKD_HIP(hipMemsetAsync(d_nrootext, 0, sizeof(int), st));
      size_t lds = select_lds_bytes<D>(s);
      Prof::begin(kProfSelect, st);
      const int p2 = std::max(64, next_pow2(s));
#define PKD_SEL(NPL)                                                                                              \
  {                                                                                                               \
    PKD_TRY(allow_lds(k_select_skeleton<D, NPL>, lds));                                                           \
    hipLaunchKernelGGL((k_select_skeleton<D, NPL>), dim3(ns), dim3(64 * D), lds, st, sieve.p, ns, bufs, src, P.seed, \
                       s, P.lambda, W.shift.p, small_max, cand_key.p, cand_pos.p, cand_cnt.p, cap, so);           \
  }
      if (p2 <= 64) PKD_SEL(1)
      else if (p2 <= 128) PKD_SEL(2)
      else if (p2 <= 256) PKD_SEL(4)
      else if (p2 <= 512) PKD_SEL(8)
      else if (p2 <= 1024) PKD_SEL(16)
      else PKD_SEL(32)
#undef PKD_SEL
      Prof::end(kProfSelect, st, 0.0);
      PKD_TRY(kernel_status("k_select_skeleton"));
      PKD_HIP(hipMemcpyAsync(hc, ctr.p, sizeof(int) * 8, hipMemcpyDeviceToHost, st));
      PKD_HIP(hipStreamSynchronize(st));
      if (hc[4] & kErrInternal) return PKD_ERR_INTERNAL;
      if (!(hc[4] & (kErrCandOverflow | kErrCandUnderflow))) break;
      if (attempt > 8) return PKD_ERR_INTERNAL;
      int clear = hc[4] & ~(kErrCandOverflow | kErrCandUnderflow);
      PKD_HIP(hipMemcpyAsync(d_flags, &clear, sizeof(int), hipMemcpyHostToDevice, st));
      override_p = shift_fix.p;
    }
    if (P.sigma == 0) {
      // exact medians, one level per round (no sampling): the split rule on
      // all points of every subproblem
      PKD_TRY(seg_exact_split<D>(st, sieve.p, nullptr, ns, tile, P.lambda, s, bufs, src, rx.p, rdim.p, ext.p,
                                 mode.p, EW));
      PKD_TRY(sieve_layout(st, sieve.p, ns, tile, W, s, small_max, nullptr, &ntiles, &nchunks, &round_pts,
                           P.cand_bias));
      bounded = false;
    } else if (hc[5] > 0) {
      // subproblems whose sample was entirely identical (rare): the split
      // rule on all their points
      PKD_TRY(seg_exact_split<D>(st, sieve.p, rootext.p, hc[5], tile, P.lambda, s, bufs, src, rx.p, rdim.p, ext.p,
                                 mode.p, EW));
    }
    // sieve: count, column-major scan, stable scatter
    PKD_TRY(sieve_pass(st, D, P.lambda, tile, sieve.p, ns, bufs, src, dst, rx.p, rdim.p, mode.p, W, ntiles, nchunks,
                       round_pts, first && src == 2 ? 1 : 0, d_flags, bounded ? d_nsieve : nullptr));
    // nodes and next round's tasks
    PKD_TRY(ensure_nodes(T, st, static_cast<int64_t>(node_count) + static_cast<int64_t>(ns) * nheap));
    // the emit adds at most one heavy leaf per subproblem to the finisher's
    // list and at most 2^lambda tasks per subproblem to the next front; the
    // next front is classified right after, reading its count on the device,
    // so one host read ends the round
    const int64_t next_max = static_cast<int64_t>(ns) * NB;
    PKD_TRY(next.need(static_cast<size_t>(next_max)));
    PKD_TRY(fin.need(static_cast<size_t>(n_fin) + ns + next_max + 1, true));
    PKD_HIP(hipMemsetAsync(d_nnext, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_emit, dim3((ns + kEmitWaves - 1) / kEmitWaves), dim3(64 * kEmitWaves), 0, st, sieve.p, ns,
                       P.lambda, rx.p, rdim.p, ext.p, mode.p,
                       W.bsize.p, W.bstart.p, dst, T->nodes, d_nodes, next.p, d_nnext, fin.p, d_nfin, d_flags);
    PKD_TRY(kernel_status("k_emit"));
    PKD_TRY(sieve.need(static_cast<size_t>(next_max)));
    PKD_HIP(hipMemsetAsync(d_nsieve, 0, sizeof(int), st));
    PKD_HIP(hipMemsetAsync(d_spts, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_classify, dim3(static_cast<unsigned>((next_max + 255) / 256)), dim3(256), 0, st, next.p,
                       static_cast<int>(next_max), s, sieve.p, d_nsieve, fin.p, d_nfin, d_nnext, d_spts);
    PKD_TRY(kernel_status("k_classify"));
    PKD_HIP(hipMemcpyAsync(hc, ctr.p, sizeof(int) * 10, hipMemcpyDeviceToHost, st));
    PKD_HIP(hipStreamSynchronize(st));
    if (hc[4] & kErrRange) return PKD_ERR_RANGE;
    if (hc[4] & kErrInternal) return PKD_ERR_INTERNAL;
    n_front = hc[2];
    n_fin = hc[1];
    node_count = hc[3];
    T->node_count = node_count;
    classified = true;
    std::swap(front.p, next.p);
    std::swap(front.cap, next.cap);
    src = dst;
    dst = (dst == F) ? 1 - F : F;
    first = false;
  }

  // finisher over every small subproblem, by size class
  if (n_fin > 0) {
    TraceRange tr("finisher");
    PKD_TRY(lists.need(static_cast<size_t>(8) * n_fin + 8));
    int* d_counts = ctr.p + 8;
    PKD_HIP(hipMemsetAsync(d_counts, 0, sizeof(int) * 8, st));
    hipLaunchKernelGGL(k_bin_finish, dim3((n_fin + 1023) / 1024), dim3(1024), 0, st, fin.p, n_fin, lists.p, n_fin,
                       d_counts);
    PKD_TRY(kernel_status("k_bin_finish"));
    // node slots: a reserved range per task from a prefix sum of size bounds
    DArr<int32_t> R(st), res_off(st), bsum(st);
    PKD_TRY(R.need(n_fin + 1));
    PKD_TRY(res_off.need(n_fin + 1));
    hipLaunchKernelGGL(k_fin_reserve, dim3((n_fin + 255) / 256), dim3(256), 0, st, fin.p, n_fin, P.phi, R.p);
    PKD_TRY(kernel_status("k_fin_reserve"));
    PKD_TRY(exscan_i32(st, R.p, res_off.p, n_fin, bsum));
    // one host read for the total reservation (into spare slot 7) and the
    // class counts (slots 8-15)
    PKD_HIP(hipMemcpyAsync(ctr.p + 7, res_off.p + n_fin, sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    int hf[9];
    PKD_HIP(hipMemcpyAsync(hf, ctr.p + 7, sizeof(hf), hipMemcpyDeviceToHost, st));
    PKD_HIP(hipStreamSynchronize(st));
    const int32_t reserved = hf[0];
    int counts[8];
    for (int c = 0; c < 8; ++c) counts[c] = hf[1 + c];
    const int base_nodes = node_count;
    T->node_count = base_nodes;   // the finisher's nodes are rewritten on a retry
    int64_t want = static_cast<int64_t>(base_nodes) + reserved + 1024;
    for (int attempt = 0; attempt < 3; ++attempt) {
      PKD_TRY(ensure_nodes(T, st, want));
      int zero_flags = 0;
      const int ovf_start = base_nodes + reserved;
      PKD_HIP(hipMemcpyAsync(d_nodes, &ovf_start, sizeof(int), hipMemcpyHostToDevice, st));
      PKD_HIP(hipMemcpyAsync(d_flags, &zero_flags, sizeof(int), hipMemcpyHostToDevice, st));
      for (int cls = 0; cls < 7; ++cls) {
        if (counts[cls] == 0) continue;
        const int Pc = 64 << cls;
        size_t lds = finish_lds_bytes<D>(Pc, P.phi);
        Prof::begin(kProfFinish, st);
        // one workgroup of D waves per subproblem, 64*NPL = P keys per wave
#define PKD_FIN(NPL)                                                                                              \
  {                                                                                                               \
    PKD_TRY(allow_lds(k_finish<D, NPL>, lds));                                                                    \
    hipLaunchKernelGGL((k_finish<D, NPL>), dim3(counts[cls]), dim3(64 * D), lds, st, fin.p, lists.p + cls * n_fin, \
                       Pc, bufs, F, P.phi, T->nodes, d_nodes, T->node_cap, d_height, d_flags, res_off.p,          \
                       base_nodes);                                                                               \
  }
        switch (cls) {
          case 0: PKD_FIN(1) break;
          case 1: PKD_FIN(2) break;
          case 2: PKD_FIN(4) break;
          case 3: PKD_FIN(8) break;
          case 4: PKD_FIN(16) break;
          case 5: PKD_FIN(32) break;
          default: return PKD_ERR_INTERNAL;   // base cases hold fewer than s <= 2048 points
        }
#undef PKD_FIN
        Prof::end(kProfFinish, st, 0.0);
        PKD_TRY(kernel_status("k_finish"));
      }
      if (counts[7] > 0) {
        hipLaunchKernelGGL(k_finish_heavy, dim3(counts[7]), dim3(256), 0, st, fin.p, lists.p + 7 * n_fin, D, bufs, F,
                           T->nodes, d_height);
        PKD_TRY(kernel_status("k_finish_heavy"));
      }
      PKD_HIP(hipMemcpyAsync(hc, ctr.p, sizeof(int) * 8, hipMemcpyDeviceToHost, st));
      PKD_HIP(hipStreamSynchronize(st));
      if (hc[4] & kErrRange) return PKD_ERR_RANGE;
      if (hc[4] & kErrInternal) return PKD_ERR_INTERNAL;
      node_count = hc[3];
      if (!(hc[4] & kErrNodeOverflow)) break;
      if (attempt == 2) return PKD_ERR_INTERNAL;
      want = node_count;   // the counter kept counting: the exact need
    }
  }
  T->node_count = node_count;
  T->height = hc[6];
  return PKD_OK;
}

template <int D>
int sieve_pass_d(hipStream_t st, int lambda, int tile, const Task* tasks, int ns, const Bufs& bufs, int src, int dst,
                 const int64_t* rx, const uint8_t* rdim, const int8_t* mode, SieveWork& W, int64_t ntiles,
                 int64_t nchunks, int64_t pts, int check, int* d_flags, const int* dns) {
  const int NB = 1 << lambda;
  PKD_TRY(W.A.need(static_cast<size_t>(ntiles) * NB));
  PKD_TRY(W.B.need(static_cast<size_t>(ntiles) * NB));
  PKD_TRY(W.S.need(static_cast<size_t>(nchunks) * NB));
  PKD_TRY(W.bsize.need(static_cast<size_t>(ns) * NB));
  PKD_TRY(W.bstart.need(static_cast<size_t>(ns) * NB));
  Prof::begin(kProfCount, st);
  hipLaunchKernelGGL(k_count<D>, dim3(static_cast<unsigned>(ntiles)), dim3(kBlock), 0, st, tasks, ns, W.tile_off.p,
                     tile, bufs, src, rx, rdim, mode, lambda, W.A.p, check, d_flags, dns);
  Prof::end(kProfCount, st, 8.0 * D * static_cast<double>(pts));
  PKD_TRY(kernel_status("k_count"));
  // an out-of-range coordinate of caller input is flagged by k_count and
  // reported at the round's end, before the tree is used: routing compares
  // coordinates with splitters, so every later step stays in bounds
  hipLaunchKernelGGL(k_chunk_sum, dim3(static_cast<unsigned>(nchunks)), dim3(kBlock), 0, st, W.chunk_off.p,
                     W.tile_off.p, ns, lambda, W.A.p, W.S.p, dns);
  PKD_TRY(kernel_status("k_chunk_sum"));
  hipLaunchKernelGGL(k_sp_scan, dim3(ns), dim3(kBlock), 0, st, tasks, W.chunk_off.p, lambda, W.S.p, W.bsize.p,
                     W.bstart.p, dns);
  PKD_TRY(kernel_status("k_sp_scan"));
  hipLaunchKernelGGL(k_apply, dim3(static_cast<unsigned>(nchunks)), dim3(kBlock), 0, st, W.chunk_off.p, W.tile_off.p,
                     ns, lambda, W.A.p, W.S.p, W.bstart.p, W.B.p, dns);
  PKD_TRY(kernel_status("k_apply"));
  Prof::begin(kProfScatter, st);
#define PKD_SCATTER(PPT)                                                                                          \
  {                                                                                                               \
    const size_t lds = ScatterLayout(kBlock * (PPT), lambda).end;                                               \
    PKD_TRY(allow_lds(k_scatter<D, PPT>, lds));                                                                   \
    hipLaunchKernelGGL((k_scatter<D, PPT>), dim3(static_cast<unsigned>(ntiles)), dim3(kBlock), lds, st, tasks, ns, \
                       W.tile_off.p, bufs, src, dst, rx, rdim, mode, lambda, W.B.p, dns);                          \
  }
  if (tile == 2048)
    PKD_SCATTER(8)
  else if (tile == 1024)
    PKD_SCATTER(4)
  else
    PKD_SCATTER(16)
#undef PKD_SCATTER
  Prof::end(kProfScatter, st, 2.0 * (8.0 * D + 8.0) * static_cast<double>(pts));
  PKD_TRY(kernel_status("k_scatter"));
  return PKD_OK;
}

}  // namespace

// ------------------------------------------------ int32 exclusive prefix sum
constexpr int kScanThreads = 256;
// Exclusive prefix sums over int32 arrays: block sums, one-workgroup scan of
// the block sums, then the per-block pass (the last alone for inputs of one
// block).  out[i] = sum in[0..i), out[n] = total.
constexpr int kScanBlock = 2048;

__global__ void k_scan_blocks(const int32_t* in, int64_t n, int32_t* bsum) {
  __shared__ int32_t part[kScanThreads];
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kScanBlock;
  int32_t s = 0;
  for (int64_t i = b0 + threadIdx.x; i < min<int64_t>(n, b0 + kScanBlock); i += kScanThreads) s += in[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = kScanThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = part[0];
}

__global__ void __launch_bounds__(1024) k_scan_sums(int32_t* bsum, int64_t nb) {
  // exclusive scan of the block sums: each thread sums a contiguous run, the
  // 1024 run totals are scanned by wave shuffles (16 waves, then their totals)
  __shared__ int32_t wtot[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b = tid * per, e = min(nb, b + per);
  int32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += bsum[i];
  int32_t incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  if (w == 0) {
    const int32_t x = lane < 16 ? wtot[lane] : 0;
    int32_t wi = x;
    for (int o = 1; o < 16; o <<= 1) {
      const int32_t y = __shfl_up(wi, o);
      if (lane >= o) wi += y;
    }
    if (lane < 16) wtot[lane] = wi - x;
  }
  __syncthreads();
  int32_t run = wtot[w] + incl - s;
  for (int64_t i = b; i < e; ++i) {
    const int32_t x = bsum[i];
    bsum[i] = run;
    run += x;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int32_t* in, int64_t n, const int32_t* bsum,
                                                            int32_t* out) {
  __shared__ int32_t vals[kScanBlock];
  __shared__ int32_t wtot[kScanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kScanBlock;
  const int len = static_cast<int>(min<int64_t>(kScanBlock, n - b0));
  for (int i = tid; i < kScanBlock; i += kScanThreads) vals[i] = i < len ? in[b0 + i] : 0;
  __syncthreads();
  constexpr int per = kScanBlock / kScanThreads;
  int32_t s = 0;
  for (int k = 0; k < per; ++k) s += vals[tid * per + k];
  // exclusive scan of the per-thread sums: shuffles inside each wave, then
  // the wave totals
  int32_t incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  int32_t before = bsum ? bsum[blockIdx.x] : 0;   // no block sums: a single block
  for (int j = 0; j < w; ++j) before += wtot[j];
  int32_t run = before + incl - s;
  for (int k = 0; k < per; ++k) {
    const int i = tid * per + k;
    if (i < len) out[b0 + i] = run;
    run += vals[i];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == kScanThreads - 1) out[n] = run;
}

// Up to this many block sums are scanned by the one-workgroup kernel; more
// (inputs above 2^27) are scanned by this same three-pass scheme, in place.
constexpr int64_t kScanSumsMax = int64_t{1} << 16;

int64_t exscan_bsum_need(int64_t n) { return std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock) + 1; }

int exscan_i32_raw(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* bsum) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
  if (nb > kScanSumsMax) return PKD_ERR_INTERNAL;   // callers with larger inputs use exscan_i32
  if (nb == 1) {   // one block scans it all (most scans of an update are this small)
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, st, in, n, static_cast<const int32_t*>(nullptr),
                       out);
    return kernel_status("k_scan_apply");
  }
  hipLaunchKernelGGL(k_scan_blocks, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, st, in, n, bsum);
  PKD_TRY(kernel_status("k_scan_blocks"));
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, bsum, nb);
  PKD_TRY(kernel_status("k_scan_sums"));
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, st, in, n, bsum, out);
  return kernel_status("k_scan_apply");
}

int exscan_i32(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, DArr<int32_t>& bsum) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
  PKD_TRY(bsum.need(nb + 1));
  if (nb <= kScanSumsMax) return exscan_i32_raw(st, in, out, n, bsum.p);
  hipLaunchKernelGGL(k_scan_blocks, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, st, in, n, bsum.p);
  PKD_TRY(kernel_status("k_scan_blocks"));
  DArr<int32_t> b2(st);
  PKD_TRY(exscan_i32(st, bsum.p, bsum.p, nb, b2));   // each block reads its range before writing it
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, st, in, n, bsum.p, out);
  PKD_TRY(kernel_status("k_scan_apply"));
  return PKD_OK;
}


// ------------------------------------------------ LSD radix sort of pairs
// Stable sort of (uint64 key, uint32 value) pairs by the low `nbits` bits of
// the key, 8 bits per pass: per-tile digit counts, one exclusive scan over
// (digit, tile), and a scatter that ranks equal digits inside each tile with
// ballots (chunks of 64 consecutive items in order, so equal keys keep their
// order).
namespace {
constexpr int kRsTile = 2048;   // 256 threads x 8 items

__global__ void __launch_bounds__(256) k_rs_count(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                  int32_t* __restrict__ hist, int64_t nblk) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kRsTile;
  for (int i = threadIdx.x; i < kRsTile; i += 256)
    if (b0 + i < n) atomicAdd(&h[(key[b0 + i] >> shift) & 255], 1u);
  __syncthreads();
  hist[static_cast<int64_t>(threadIdx.x) * nblk + blockIdx.x] = static_cast<int32_t>(h[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    int64_t n, int shift, const int32_t* __restrict__ off,
                                                    int64_t nblk, uint64_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout) {
  constexpr int PER = kRsTile / 256, NCH = kRsTile / 64;   // chunks of 64 consecutive items
  __shared__ uint16_t cnt[NCH][256];
  __shared__ int32_t base[256];
  const int tid = threadIdx.x, wave = tid >> 6;
  const uint32_t lane = tid & 63;
  const unsigned long long lt = (1ULL << lane) - 1;
  for (int i = tid; i < NCH * 256; i += 256) (&cnt[0][0])[i] = 0;
  base[tid] = off[static_cast<int64_t>(tid) * nblk + blockIdx.x];
  __syncthreads();
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kRsTile;
  uint64_t kk[PER];
  uint32_t vv[PER];
  int dig[PER], rank[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t i = b0 + k * 256 + tid;
    const bool ok = i < n;
    kk[k] = ok ? kin[i] : 0;
    vv[k] = ok ? vin[i] : 0;
    const int d = static_cast<int>((kk[k] >> shift) & 255);
    unsigned long long peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    dig[k] = d;
    rank[k] = __popcll(peers & lt);
    if (ok && (peers & lt) == 0) cnt[k * 4 + wave][d] = static_cast<uint16_t>(__popcll(peers));
  }
  __syncthreads();
  {
    uint16_t run = 0;
    for (int ch = 0; ch < NCH; ++ch) {
      const uint16_t x = cnt[ch][tid];
      cnt[ch][tid] = run;
      run += x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t i = b0 + k * 256 + tid;
    if (i < n) {
      const int64_t pos = static_cast<int64_t>(base[dig[k]]) + cnt[k * 4 + wave][dig[k]] + rank[k];
      kout[pos] = kk[k];
      vout[pos] = vv[k];
    }
  }
}

}  // namespace

namespace {
template <int D>
__global__ void k_make_c32(const int64_t* X, int64_t cap, int64_t n, int32_t* c32) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
#pragma unroll
    for (int d = 0; d < D; ++d) c32[i * D + d] = static_cast<int32_t>(X[d * cap + i]);
}
}  // namespace

int ensure_c32(pkd_tree* T, hipStream_t st) {
  if (T->c32 && T->c32_cap == T->cap) return PKD_OK;
  dev_free(T->c32, st);
  T->c32 = nullptr;
  T->c32_cap = 0;
  void* p = nullptr;
  PKD_TRY(dev_alloc(&p, sizeof(int32_t) * static_cast<size_t>(T->prm.D) * static_cast<size_t>(T->cap), st));
  T->c32 = static_cast<int32_t*>(p);
  T->c32_cap = T->cap;
  return PKD_OK;
}

int refresh_c32(pkd_tree* T, hipStream_t st) {
  PKD_TRY(ensure_c32(T, st));
  if (T->n == 0) return PKD_OK;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>(65536, (T->n + 255) / 256));
  switch (T->prm.D) {
#define PKD_C32(DD) \
  case DD: hipLaunchKernelGGL(k_make_c32<DD>, dim3(g), dim3(256), 0, st, T->buf[T->cur], T->cap, T->n, T->c32); break;
    PKD_C32(1) PKD_C32(2) PKD_C32(3) PKD_C32(4) PKD_C32(5) PKD_C32(6) PKD_C32(7) PKD_C32(8) PKD_C32(9)
#undef PKD_C32
    default: return PKD_ERR_UNSUPPORTED;
  }
  return kernel_status("k_make_c32");
}

int bits_for(int64_t v) {
  int b = 0;
  while (b < 63 && (int64_t{1} << b) <= v) ++b;
  return b;
}

int64_t radix_sort_blocks(int64_t n) { return (n + kRsTile - 1) / kRsTile; }

namespace {
// The passes of the sort over caller-provided work arrays: k1/v1 [n],
// hist [256 * nblk], off [256 * nblk + 1]; the scans of the digit counts take
// their block sums from `scan` (DArr) or, when it is null, from bsum_raw.
int radix_passes(hipStream_t st, uint64_t* keys, uint32_t* vals, int64_t n, int nbits, uint64_t* k1, uint32_t* v1,
                 int32_t* hist, int32_t* off, DArr<int32_t>* scan, int32_t* bsum_raw, uint64_t** kout,
                 uint32_t** vout) {
  const int passes = (nbits + 7) / 8;
  const int64_t nblk = radix_sort_blocks(n);
  uint64_t* ka = keys;
  uint64_t* kb = k1;
  uint32_t* va = vals;
  uint32_t* vb = v1;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_rs_count, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, st, ka, n, 8 * p, hist, nblk);
    PKD_TRY(kernel_status("k_rs_count"));
    if (scan) PKD_TRY(exscan_i32(st, hist, off, 256 * nblk, *scan));
    else PKD_TRY(exscan_i32_raw(st, hist, off, 256 * nblk, bsum_raw));
    hipLaunchKernelGGL(k_rs_scatter, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, st, ka, va, n, 8 * p, off,
                       nblk, kb, vb);
    PKD_TRY(kernel_status("k_rs_scatter"));
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  *kout = ka;
  *vout = va;
  return PKD_OK;
}
}  // namespace

int radix_sort_pairs(hipStream_t st, uint64_t* keys, uint32_t* vals, int64_t n, int nbits, SortWork& W,
                     uint64_t** kout, uint32_t** vout) {
  *kout = keys;
  *vout = vals;
  if (n <= 1 || nbits <= 0) return PKD_OK;
  const int64_t nblk = radix_sort_blocks(n);
  PKD_TRY(W.k1.need(n));
  PKD_TRY(W.v1.need(n));
  PKD_TRY(W.hist.need(static_cast<size_t>(256) * nblk));
  PKD_TRY(W.off.need(static_cast<size_t>(256) * nblk + 1));
  return radix_passes(st, keys, vals, n, nbits, W.k1.p, W.v1.p, W.hist.p, W.off.p, &W.bsum, nullptr, kout, vout);
}

int radix_sort_pairs_raw(hipStream_t st, uint64_t* keys, uint32_t* vals, int64_t n, int nbits, const SortBufs& B,
                         uint64_t** kout, uint32_t** vout) {
  *kout = keys;
  *vout = vals;
  if (n <= 1 || nbits <= 0) return PKD_OK;
  return radix_passes(st, keys, vals, n, nbits, B.k1, B.v1, B.hist, B.off, nullptr, B.bsum, kout, vout);
}

int sieve_layout(hipStream_t st, const Task* tasks, int ns, int tile, SieveWork& W, int s, int small_max,
                 const int8_t* shift_override, int64_t* ntiles, int64_t* nchunks, int64_t* pts, int cand_bias,
                 int64_t known_pts) {
  PKD_TRY(W.tile_off.need(ns + 1));
  PKD_TRY(W.chunk_off.need(ns + 1));
  PKD_TRY(W.shift.need(ns));
  PKD_TRY(W.tot.need(4));
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, tasks, ns, tile, W.tile_off.p, W.chunk_off.p, W.shift.p,
                     s, small_max, shift_override, W.tot.p + 2, cand_bias);
  PKD_TRY(kernel_status("k_tile_scan"));
  if (known_pts >= 0) {
    // a task of m points has ceil(m/tile) tiles; a chunk holds kChunkTiles
    *ntiles = known_pts / tile + ns + 1;
    *nchunks = *ntiles / kChunkTiles + ns + 1;
    *pts = known_pts;
    return PKD_OK;
  }
  PKD_HIP(hipMemcpyAsync(W.tot.p, W.tile_off.p + ns, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  PKD_HIP(hipMemcpyAsync(W.tot.p + 1, W.chunk_off.p + ns, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  int64_t tot[3];
  PKD_HIP(hipMemcpyAsync(tot, W.tot.p, sizeof(tot), hipMemcpyDeviceToHost, st));
  PKD_HIP(hipStreamSynchronize(st));
  *ntiles = tot[0];
  *nchunks = tot[1];
  *pts = tot[2];
  return PKD_OK;
}

int sieve_pass(hipStream_t st, int D, int lambda, int tile, const Task* tasks, int ns, const Bufs& bufs, int src,
               int dst, const int64_t* rx, const uint8_t* rdim, const int8_t* mode, SieveWork& W, int64_t ntiles,
               int64_t nchunks, int64_t pts, int check, int* d_flags, const int* dns) {
  switch (D) {
#define PKD_SIEVE_CASE(DD) \
  case DD: return sieve_pass_d<DD>(st, lambda, tile, tasks, ns, bufs, src, dst, rx, rdim, mode, W, ntiles, nchunks, pts, check, d_flags, dns);
    PKD_SIEVE_CASE(1)
    PKD_SIEVE_CASE(2)
    PKD_SIEVE_CASE(3)
    PKD_SIEVE_CASE(4)
    PKD_SIEVE_CASE(5)
    PKD_SIEVE_CASE(6)
    PKD_SIEVE_CASE(7)
    PKD_SIEVE_CASE(8)
    PKD_SIEVE_CASE(9)
#undef PKD_SIEVE_CASE
  }
  return PKD_ERR_UNSUPPORTED;
}

size_t build_lds_need(int D, int s, int phi) {
  const int P = std::max(64, next_pow2(s));   // the largest finisher class holds fewer than s points
  return std::max(SkelLayout(D, P).end, FinLayout(D, P, phi).end);
}

namespace {
int build_tasks_any(pkd_tree* T, hipStream_t st, const Task* roots, int n_roots, bool on_device, int src_buf,
                    const int64_t* in_c, const int64_t* in_id, int64_t input_cap) {
  switch (T->prm.D) {
#define PKD_BT(DD) \
  case DD: return build_tasks_d<DD>(T, st, roots, n_roots, on_device, src_buf, in_c, in_id, input_cap);
    PKD_BT(1) PKD_BT(2) PKD_BT(3) PKD_BT(4) PKD_BT(5) PKD_BT(6) PKD_BT(7) PKD_BT(8) PKD_BT(9)
#undef PKD_BT
    default: return PKD_ERR_UNSUPPORTED;
  }
}
}  // namespace

int build_tasks(pkd_tree* T, hipStream_t st, const std::vector<Task>& roots, const int64_t* in_c,
                const int64_t* in_id, int64_t input_cap) {
  return build_tasks_any(T, st, roots.data(), static_cast<int>(roots.size()), false,
                         roots.empty() ? 2 : roots[0].buf, in_c, in_id, input_cap);
}

// ------------------------------------------------ graph build plans
namespace {
// Counter slots of a plan (G->ctr).
enum : int {
  kGSieve = 0, kGFin = 1, kGNext = 2, kGNodes = 3, kGFlags = 4, kGRootExt = 5, kGHeight = 6, kGFront = 7,
  kGClass = 8,      // 8 class counts of the finisher
  kGBase = 16,      // node records before the finisher (base of its reservations)
  kGSlots = 32
};
constexpr int kErrPlan = 64;   // flag: the sized launches did not cover this input

// The roots of the non-empty trees form the first front; node records
// 0 .. n_slots-1 are the trees' roots.
__global__ void k_plan_start(int* ctr, int n_roots, int n_slots, const Task* roots, Task* front) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_roots) front[i] = roots[i];
  if (i < kGSlots) ctr[i] = i == kGNodes ? n_slots : (i == kGFront ? n_roots : 0);
}

// Before a round: the round's append counters start at zero.
__global__ void k_plan_round(int* ctr) {
  if (threadIdx.x == 0) {
    ctr[kGSieve] = 0;
    ctr[kGNext] = 0;
    ctr[kGRootExt] = 0;
  }
}

// After a round: the buckets become the next front; a sample of identical
// points needs the exact split the sized launches do not make.
__global__ void k_plan_round_end(int* ctr) {
  if (threadIdx.x == 0) {
    ctr[kGFront] = ctr[kGNext];
    if (ctr[kGRootExt] > 0) ctr[kGFlags] |= kErrPlan;
  }
}

// After the last round: no subproblem may be left for another round.
__global__ void k_plan_rounds_done(int* ctr) {
  if (threadIdx.x == 0 && ctr[kGSieve] > 0) ctr[kGFlags] |= kErrPlan;
}

// The finisher's node reservations start after the records made so far.
__global__ void k_plan_fin_base(int* ctr, const int32_t* res_off, int64_t fin_max) {
  if (threadIdx.x == 0) {
    ctr[kGBase] = ctr[kGNodes];
    ctr[kGNodes] = ctr[kGNodes] + res_off[fin_max];
  }
}

__global__ void k_fill_u8(uint8_t* a, int64_t n, uint8_t v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = v;
}
__global__ void k_fill_u32(uint32_t* a, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = v;
}

unsigned grid_for(int64_t n, int block) {
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, INT32_MAX)));
}

template <int D>
int plan_enqueue_d(pkd_build_plan* G, hipStream_t st) {
  pkd_tree* T = G->T;
  const Params& P = T->prm;
  const int NB = 1 << P.lambda;
  const int nheap = 2 << P.lambda;
  const int s = P.s;
  const int tile = P.tile;
  const int cap = 3 * s;
  const int small_max = 3 * s;
  const int F = T->cur;
  const int n_roots = static_cast<int>(G->roots.size());
  Bufs bufs;
  for (int b = 0; b < 2; ++b) {
    bufs.c[b] = T->buf[b];
    bufs.id[b] = T->buf[b] + static_cast<int64_t>(D) * T->cap;
    bufs.cap[b] = T->cap;
  }
  bufs.c[2] = const_cast<int64_t*>(G->in_c);
  bufs.id[2] = const_cast<int64_t*>(G->in_id);
  bufs.cap[2] = G->n;
  bufs.c32 = T->c32;
  bufs.c32cap = T->c32_cap;
  int* ctr = G->ctr;
  int* d_flags = ctr + kGFlags;

  hipLaunchKernelGGL(k_plan_start, dim3(grid_for(std::max(n_roots, static_cast<int>(kGSlots)), 256)), dim3(256), 0, st,
                     ctr, n_roots, T->n_trees, G->roots_d, G->front);
  PKD_TRY(kernel_status("k_plan_start"));
  Task* front = G->front;
  Task* next = G->next;
  int src = 2, dst = 1 - F;
  const size_t sel_lds = select_lds_bytes<D>(s);
  const int p2 = std::max(64, next_pow2(s));
  // bounds of round r: at most n/s sieve subproblems, and at most
  // 2^lambda times as many tasks as the round before (the roots in round 0)
  int64_t front_r = n_roots;
  for (int r = 0; r < G->rounds; ++r) {
    TraceRange tr("planned sieve round");
    const int64_t ns_r = std::min<int64_t>(G->ns_max, front_r);
    const int64_t ntiles_r = std::min<int64_t>(G->ntiles_max, G->n / tile + ns_r + 1);
    const int64_t nchunks_r = std::min<int64_t>(G->nchunks_max, ntiles_r / kChunkTiles + ns_r + 1);
    hipLaunchKernelGGL(k_plan_round, dim3(1), dim3(64), 0, st, ctr);
    hipLaunchKernelGGL(k_classify, dim3(grid_for(front_r, 256)), dim3(256), 0, st, front,
                       static_cast<int>(front_r), s, G->sieve, ctr + kGSieve, G->fin, ctr + kGFin, ctr + kGFront);
    PKD_TRY(kernel_status("k_classify"));
    const int* dns = ctr + kGSieve;
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, G->sieve, 0, tile, G->tile_off, G->chunk_off,
                       G->shift, s, small_max, static_cast<const int8_t*>(nullptr), G->tot, P.cand_bias, dns);
    PKD_TRY(kernel_status("k_tile_scan"));
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(ns_r, 256)), dim3(256), 0, st,
                       reinterpret_cast<uint8_t*>(G->shift_fix), ns_r, static_cast<uint8_t>(0xFF));
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(ns_r, 256)), dim3(256), 0, st, reinterpret_cast<uint8_t*>(G->mode),
                       ns_r, static_cast<uint8_t>(0));
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(ns_r * kCntStride, 256)), dim3(256), 0, st, G->cand_cnt,
                       ns_r * kCntStride, 0u);
    PKD_TRY(kernel_status("k_fill"));
    const unsigned gt = static_cast<unsigned>(ntiles_r);
    if (tile == 1024)
      hipLaunchKernelGGL((k_candidates<4>), dim3(gt), dim3(kBlock), 0, st, G->sieve, 0, G->tile_off, bufs, src, P.seed,
                         G->shift, small_max, G->cand_key, G->cand_pos, G->cand_cnt, cap, dns);
    else if (tile == 2048)
      hipLaunchKernelGGL((k_candidates<8>), dim3(gt), dim3(kBlock), 0, st, G->sieve, 0, G->tile_off, bufs, src, P.seed,
                         G->shift, small_max, G->cand_key, G->cand_pos, G->cand_cnt, cap, dns);
    else
      hipLaunchKernelGGL((k_candidates<16>), dim3(gt), dim3(kBlock), 0, st, G->sieve, 0, G->tile_off, bufs, src,
                         P.seed, G->shift, small_max, G->cand_key, G->cand_pos, G->cand_cnt, cap, dns);
    PKD_TRY(kernel_status("k_candidates"));
    SelectOut so{G->rx, G->rdim, G->ext, G->rootext, ctr + kGRootExt, G->shift_fix, d_flags};
    const unsigned gs = static_cast<unsigned>(ns_r);
#define PKD_PSEL(NPL)                                                                                             \
  {                                                                                                               \
    PKD_TRY(allow_lds(k_select_skeleton<D, NPL>, sel_lds));                                                       \
    hipLaunchKernelGGL((k_select_skeleton<D, NPL>), dim3(gs), dim3(64 * D), sel_lds, st, G->sieve, 0, bufs, src,   \
                       P.seed, s, P.lambda, G->shift, small_max, G->cand_key, G->cand_pos, G->cand_cnt, cap, so,  \
                       dns);                                                                                      \
  }
    if (p2 <= 64) PKD_PSEL(1)
    else if (p2 <= 128) PKD_PSEL(2)
    else if (p2 <= 256) PKD_PSEL(4)
    else if (p2 <= 512) PKD_PSEL(8)
    else if (p2 <= 1024) PKD_PSEL(16)
    else PKD_PSEL(32)
#undef PKD_PSEL
    PKD_TRY(kernel_status("k_select_skeleton"));
    // sieve: count, column-major scan, stable scatter
    hipLaunchKernelGGL(k_count<D>, dim3(gt), dim3(kBlock), 0, st, G->sieve, 0, G->tile_off, tile, bufs, src, G->rx,
                       G->rdim, G->mode, P.lambda, G->A, r == 0 ? 1 : 0, d_flags, dns);
    PKD_TRY(kernel_status("k_count"));
    const unsigned gc = static_cast<unsigned>(nchunks_r);
    hipLaunchKernelGGL(k_chunk_sum, dim3(gc), dim3(kBlock), 0, st, G->chunk_off, G->tile_off, 0, P.lambda, G->A,
                       G->S, dns);
    PKD_TRY(kernel_status("k_chunk_sum"));
    hipLaunchKernelGGL(k_sp_scan, dim3(gs), dim3(kBlock), 0, st, G->sieve, G->chunk_off, P.lambda, G->S, G->bsize,
                       G->bstart, dns);
    PKD_TRY(kernel_status("k_sp_scan"));
    hipLaunchKernelGGL(k_apply, dim3(gc), dim3(kBlock), 0, st, G->chunk_off, G->tile_off, 0, P.lambda, G->A, G->S,
                       G->bstart, G->B, dns);
    PKD_TRY(kernel_status("k_apply"));
#define PKD_PSCATTER(PPT)                                                                                         \
  {                                                                                                               \
    const size_t lds = ScatterLayout(kBlock * (PPT), P.lambda).end;                                              \
    PKD_TRY(allow_lds(k_scatter<D, PPT>, lds));                                                                   \
    hipLaunchKernelGGL((k_scatter<D, PPT>), dim3(gt), dim3(kBlock), lds, st, G->sieve, 0, G->tile_off, bufs, src,  \
                       dst, G->rx, G->rdim, G->mode, P.lambda, G->B, dns);                                        \
  }
    if (tile == 2048)
      PKD_PSCATTER(8)
    else if (tile == 1024)
      PKD_PSCATTER(4)
    else
      PKD_PSCATTER(16)
#undef PKD_PSCATTER
    PKD_TRY(kernel_status("k_scatter"));
    hipLaunchKernelGGL(k_emit, dim3((gs + kEmitWaves - 1) / kEmitWaves), dim3(64 * kEmitWaves), 0, st, G->sieve, 0,
                       P.lambda, G->rx, G->rdim, G->ext, G->mode,
                       G->bsize, G->bstart, dst, T->nodes, ctr + kGNodes, next, ctr + kGNext, G->fin, ctr + kGFin,
                       d_flags, dns);
    PKD_TRY(kernel_status("k_emit"));
    hipLaunchKernelGGL(k_plan_round_end, dim3(1), dim3(64), 0, st, ctr);
    front_r = std::min<int64_t>(G->front_max, ns_r << P.lambda);
    std::swap(front, next);
    src = dst;
    dst = (dst == F) ? 1 - F : F;
  }
  // the front left after the last round goes to the finisher; nothing may
  // still need a sieve round
  hipLaunchKernelGGL(k_plan_round, dim3(1), dim3(64), 0, st, ctr);
  hipLaunchKernelGGL(k_classify, dim3(grid_for(front_r, 256)), dim3(256), 0, st, front, static_cast<int>(front_r), s,
                     G->sieve, ctr + kGSieve, G->fin, ctr + kGFin, ctr + kGFront);
  hipLaunchKernelGGL(k_plan_rounds_done, dim3(1), dim3(64), 0, st, ctr);
  PKD_TRY(kernel_status("k_plan_rounds_done"));

  // finisher over every small subproblem, by size class, in persistent grids
  TraceRange tr("planned finisher");
  const int fin_max = static_cast<int>(G->fin_max);
  hipLaunchKernelGGL(k_bin_finish, dim3(grid_for(fin_max, 1024)), dim3(1024), 0, st, G->fin, fin_max, G->lists,
                     fin_max, ctr + kGClass, ctr + kGFin);
  PKD_TRY(kernel_status("k_bin_finish"));
  hipLaunchKernelGGL(k_fin_reserve, dim3(grid_for(fin_max, 256)), dim3(256), 0, st, G->fin, fin_max, P.phi, G->R,
                     ctr + kGFin);
  PKD_TRY(kernel_status("k_fin_reserve"));
  PKD_TRY(exscan_i32_raw(st, G->R, G->res_off, fin_max, G->bsum));
  hipLaunchKernelGGL(k_plan_fin_base, dim3(1), dim3(64), 0, st, ctr, G->res_off, G->fin_max);
  PKD_TRY(kernel_status("k_plan_fin_base"));
  for (int cls = 0; cls < 6; ++cls) {
    const int Pc = 64 << cls;
    if (Pc / 2 >= s) break;   // classes above the sample size hold no task
    const size_t lds = finish_lds_bytes<D>(Pc, P.phi);
    // a task of class cls >= 1 holds more than Pc/2 points, so the class has
    // at most n/(Pc/2+1) tasks: one workgroup each, as in the eager build
    // (blocks past the count leave at once).  Class 0 (up to 64 points, with
    // no such bound) runs in a persistent grid that walks its list.
    const unsigned gf = static_cast<unsigned>(std::min<int64_t>(G->fin_max, 8192));
    const unsigned gb = static_cast<unsigned>(std::min<int64_t>(G->fin_max, G->n / (Pc / 2 + 1) + 1));
#define PKD_PFIN(NPL)                                                                                             \
  {                                                                                                               \
    if (cls == 0) {                                                                                               \
      PKD_TRY(allow_lds(k_finish_persist<D, NPL>, lds));                                                          \
      hipLaunchKernelGGL((k_finish_persist<D, NPL>), dim3(gf), dim3(64 * D), lds, st, G->fin,                     \
                         G->lists + cls * fin_max, ctr + kGClass + cls, Pc, bufs, F, P.phi, T->nodes,             \
                         ctr + kGNodes, T->node_cap, ctr + kGHeight, d_flags, G->res_off, ctr + kGBase);          \
    } else {                                                                                                      \
      PKD_TRY(allow_lds(k_finish<D, NPL>, lds));                                                                  \
      hipLaunchKernelGGL((k_finish<D, NPL>), dim3(gb), dim3(64 * D), lds, st, G->fin, G->lists + cls * fin_max,  \
                         Pc, bufs, F, P.phi, T->nodes, ctr + kGNodes, T->node_cap, ctr + kGHeight, d_flags,       \
                         G->res_off, 0, ctr + kGClass + cls, ctr + kGBase);                                       \
    }                                                                                                             \
  }
    switch (cls) {
      case 0: PKD_PFIN(1) break;
      case 1: PKD_PFIN(2) break;
      case 2: PKD_PFIN(4) break;
      case 3: PKD_PFIN(8) break;
      case 4: PKD_PFIN(16) break;
      case 5: PKD_PFIN(32) break;
    }
#undef PKD_PFIN
    PKD_TRY(kernel_status("k_finish_persist"));
  }
  hipLaunchKernelGGL(k_finish_heavy, dim3(static_cast<unsigned>(std::min<int64_t>(G->fin_max, 4096))), dim3(256), 0,
                     st, G->fin, G->lists + 7 * fin_max, D, bufs, F, T->nodes, ctr + kGHeight, ctr + kGClass + 7);
  return kernel_status("k_finish_heavy");
}
}  // namespace

int plan_size(pkd_build_plan* G) {
  const Params& P = G->T->prm;
  if (P.sigma == 0) return PKD_ERR_UNSUPPORTED;   // exact medians split by host-sized passes
  const int s = P.s;
  const int64_t NB = int64_t{1} << P.lambda;
  const int64_t nheap = int64_t{2} << P.lambda;
  int64_t m_max = 0;
  for (const Task& t : G->roots) m_max = std::max<int64_t>(m_max, t.m);
  // rounds: every round divides a subproblem by about 2^lambda; the plan
  // allows for buckets twice the expected size and one round more
  int R = 0;
  for (double m = static_cast<double>(m_max); m >= s; m /= static_cast<double>(NB) / 2.0) ++R;
  if (R > 0) ++R;
  G->rounds = R;
  const int64_t n = G->n, nt = G->T->n_trees;
  const int64_t sigma = std::max<int64_t>(1, s / NB);
  G->ns_max = n / s + 1;                                       // sieve subproblems hold at least s points
  G->front_max = std::max<int64_t>(nt, n / sigma + 1);          // at most 2^lambda buckets per subproblem
  G->fin_max = std::min<int64_t>(n + 1, nt + static_cast<int64_t>(R + 1) * (n / sigma + 1)) + 1;
  G->ntiles_max = n / P.tile + G->ns_max + 1;
  G->nchunks_max = G->ntiles_max / kChunkTiles + G->ns_max + 1;
  G->cand_len = G->ns_max * 3 * s;
  const int64_t nodes = nt + static_cast<int64_t>(R) * G->ns_max * nheap + 4 * (n / (P.phi + 1)) + 4 * G->fin_max +
                        1024;
  if (nodes >= INT32_MAX || G->fin_max >= INT32_MAX / 8 || G->front_max >= INT32_MAX) return PKD_ERR_UNSUPPORTED;
  if ((G->fin_max + kScanBlock - 1) / kScanBlock > kScanSumsMax) return PKD_ERR_UNSUPPORTED;
  PKD_TRY(ensure_nodes(G->T, nullptr, nodes));
  return PKD_OK;
}

int plan_enqueue(pkd_build_plan* G, hipStream_t st) {
  switch (G->T->prm.D) {
#define PKD_PE(DD) \
  case DD: return plan_enqueue_d<DD>(G, st);
    PKD_PE(1) PKD_PE(2) PKD_PE(3) PKD_PE(4) PKD_PE(5) PKD_PE(6) PKD_PE(7) PKD_PE(8) PKD_PE(9)
#undef PKD_PE
    default: return PKD_ERR_UNSUPPORTED;
  }
}

int build_tasks_dev(pkd_tree* T, hipStream_t st, const Task* d_roots, int n_roots, int src_buf,
                    const int64_t* in_c, const int64_t* in_id, int64_t input_cap) {
  return build_tasks_any(T, st, d_roots, n_roots, true, src_buf, in_c, in_id, input_cap);
}

}  // namespace pkd
