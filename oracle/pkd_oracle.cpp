// Sequential CPU oracle for the Pkd-tree hot path.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's CPU
// baseline leg may load this library.  It shares no code, header, table or
// helper with the GPU library: everything below is written from the paper
// ("Parallel kd-tree with Batch Updates", Men, Shen, Gu, Sun, SIGMOD 2025) and
// from the readings listed in the design notes, in the paper's order and
// notation, with no blocking, fusion or reordering beyond what the text states.
//
// What it computes
//   * Build(P)        -- Algorithm 1 (Section 3.1): sample 2^lambda*sigma points,
//                        build a lambda-level skeleton on the sample, sieve P into
//                        the 2^lambda buckets (stable), recurse per bucket; below
//                        2^lambda*sigma points use the plain construction.
//   * BatchInsert     -- Algorithm 2 (Section 4.1), node by node: keep a node whose
//                        two subtrees stay weight-balanced after insertion, rebuild
//                        the topmost one that does not; a leaf becomes
//                        Build(leaf u batch).
//   * BatchDelete     -- Section 4.2, two rounds: sieve the batch to the leaves and
//                        drop absent points, then rebuild the topmost subtrees that
//                        are unbalanced under the exact new sizes.
//   * k-NN, range count, range report -- Section 2 (query definitions) and
//                        Section 5 (DFS with on-the-fly subspaces, subtree sizes for
//                        counts, flattened subtrees for reports).  The brute force
//                        functions are the plain definitions themselves.
//   * instrumentation  -- per-query work of the k-NN search (nodes read, leaves and
//                        points scanned; the counts Appendix H reports) and what
//                        each batch update rebuilt (the cost that the update
//                        theorem of Section 4.3 amortizes).  Neither changes a
//                        result.
//
// Readings where the paper is silent (all integer, so results are exact):
//   split side: coordinate < x goes left, the rest right (Section 2);
//   split dim: widest max-min stretch, lowest index on ties; split value: upper
//     median v[floor(m/2)] of the sorted coordinates, moved up to the next larger
//     distinct value when it equals the minimum (both sides non-empty);
//   leaf: at most phi points; more than phi identical points form a heavy leaf
//     (Appendix C) that keeps every point and id;
//   sample: the s = 2^lambda*sigma points with the smallest (key, id), key =
//     SplitMix64-mix(SplitMix64-mix(id ^ seed) + (h+1)*golden) with h the depth of
//     the subtree root in the whole tree (uniform, without replacement, and
//     independent of the array order);
//   skeleton: a node whose sample subset has zero width in every dimension is
//     external; an external node above level lambda takes the leftmost
//     depth-lambda bucket label below it; if the skeleton root itself is external
//     (sample all identical, set not) one exact split of the whole set is made;
//   balance: n' > 0 and (den-2num)*n' <= 2*den*l' <= (den+2num)*n', alpha=num/den;
//     subtrees that receive no batch point (insert) or lose no point (delete) are
//     left untouched; a rebuild at node t uses depth(t) for the sampling salt.
//
// Layout at the C boundary: coordinates are int64 [D][n] (structure of arrays),
// ids int64 [n]; coordinates and query coordinates lie in [0, 2^30).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

namespace {

struct Params {
  int D;
  int lambda;
  int phi;
  int sigma;
  int64_t alpha_num;
  int64_t alpha_den;
  uint64_t seed;
};

// --- Sampling key ----------------------------------------------------------
// SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014; the variant-13 mixing
// constants of Vigna's reference splitmix64.c).
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

const uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

uint64_t sample_key(uint64_t seed, int64_t h, int64_t id) {
  uint64_t a = mix64(static_cast<uint64_t>(id) ^ seed);
  return mix64(a + static_cast<uint64_t>(h + 1) * kGolden);
}

// --- Point store -------------------------------------------------------------
struct Store {
  int D = 0;
  std::vector<int64_t> c;   // coordinates of point i at c[i*D + d]
  std::vector<int64_t> id;
  int64_t coord(int64_t i, int d) const { return c[static_cast<size_t>(i) * D + d]; }
  int64_t add(const int64_t* coords, int64_t stride, int64_t j, int64_t pid) {
    for (int d = 0; d < D; ++d) c.push_back(coords[d * stride + j]);
    id.push_back(pid);
    return static_cast<int64_t>(id.size()) - 1;
  }
};

struct Node {
  bool leaf = true;
  int dim = -1;
  int64_t x = 0;
  int64_t size = 0;
  int depth = 0;
  int left = -1, right = -1;
  bool plain = false;        // interior node made by one exact split (not a skeleton node)
  std::vector<int64_t> pts;  // leaf only: point handles, in their stable order
};

// What the last batch update rebuilt (for the amortized-cost check of the
// update theorem, Section 4.3): interior subtrees rebuilt because they became
// unbalanced, leaves rebuilt because they received points, and kept interior
// nodes whose size changed.
struct UpdateLog {
  int64_t interior_rebuilds = 0, interior_points = 0;
  int64_t leaf_rebuilds = 0, leaf_points = 0;
  int64_t kept = 0;
};

struct Tree {
  Params p;
  Store st;
  std::vector<Node> nodes;
  int root = -1;
  UpdateLog log;
};

using Set = std::vector<int64_t>;  // a sequence of point handles

// --- Split rule (Section 2) -----------------------------------------------
bool all_identical(const Store& st, const Set& Q) {
  for (size_t i = 1; i < Q.size(); ++i)
    for (int d = 0; d < st.D; ++d)
      if (st.coord(Q[i], d) != st.coord(Q[0], d)) return false;
  return true;
}

// Widest dimension (max - min), lowest index on ties.
int widest_dim(const Store& st, const Set& Q) {
  int best = 0;
  int64_t best_w = -1;
  for (int d = 0; d < st.D; ++d) {
    int64_t lo = st.coord(Q[0], d), hi = lo;
    for (int64_t q : Q) {
      lo = std::min(lo, st.coord(q, d));
      hi = std::max(hi, st.coord(q, d));
    }
    if (hi - lo > best_w) {
      best_w = hi - lo;
      best = d;
    }
  }
  return best;
}

// Upper median of the sorted coordinates on d; if it equals the minimum take
// the next larger distinct value so that both sides are non-empty.
// Precondition: Q has positive width on d.
int64_t split_value(const Store& st, const Set& Q, int d) {
  std::vector<int64_t> v;
  v.reserve(Q.size());
  for (int64_t q : Q) v.push_back(st.coord(q, d));
  std::sort(v.begin(), v.end());
  int64_t x = v[v.size() / 2];
  if (x == v[0]) x = *std::upper_bound(v.begin(), v.end(), v[0]);
  return x;
}

// --- Skeleton on the sample (Section 3.1, Algorithm 1) ----------------------
struct Skeleton {
  int lambda = 0;
  std::vector<int> dim;          // heap index 1 .. 2^lambda - 1
  std::vector<int64_t> x;
  std::vector<char> external;    // heap index 1 .. 2^(lambda+1) - 1
};

int level_of(int v) {
  int l = 0;
  while (v > 1) {
    v >>= 1;
    ++l;
  }
  return l;
}

void skeleton_rec(const Store& st, Skeleton& sk, int v, const Set& S) {
  if (level_of(v) == sk.lambda || all_identical(st, S)) {
    sk.external[v] = 1;
    return;
  }
  int d = widest_dim(st, S);
  int64_t x = split_value(st, S, d);
  sk.dim[v] = d;
  sk.x[v] = x;
  Set L, R;
  for (int64_t q : S) (st.coord(q, d) < x ? L : R).push_back(q);
  skeleton_rec(st, sk, 2 * v, L);
  skeleton_rec(st, sk, 2 * v + 1, R);
}

Skeleton build_skeleton(const Store& st, const Set& S, int lambda) {
  Skeleton sk;
  sk.lambda = lambda;
  sk.dim.assign(1u << lambda, -1);
  sk.x.assign(1u << lambda, 0);
  sk.external.assign(2u << lambda, 0);
  skeleton_rec(st, sk, 1, S);
  return sk;
}

// Bucket label of a point: walk down until an external node; its label is the
// leftmost depth-lambda heap position below it, minus 2^lambda.
int route(const Store& st, const Skeleton& sk, int64_t q) {
  int v = 1;
  while (!sk.external[v]) v = 2 * v + (st.coord(q, sk.dim[v]) >= sk.x[v] ? 1 : 0);
  int l = level_of(v);
  return (v << (sk.lambda - l)) - (1 << sk.lambda);
}

// Uniform sample of s points without replacement: the s smallest (key, id).
Set take_sample(const Tree& T, const Set& Q, int h, size_t s) {
  std::vector<std::pair<uint64_t, int64_t>> keyed;
  keyed.reserve(Q.size());
  for (size_t i = 0; i < Q.size(); ++i) keyed.push_back({sample_key(T.p.seed, h, T.st.id[Q[i]]), static_cast<int64_t>(i)});
  auto less = [&](const std::pair<uint64_t, int64_t>& a, const std::pair<uint64_t, int64_t>& b) {
    if (a.first != b.first) return a.first < b.first;
    return T.st.id[Q[a.second]] < T.st.id[Q[b.second]];
  };
  std::sort(keyed.begin(), keyed.end(), less);
  Set S;
  for (size_t i = 0; i < s; ++i) S.push_back(Q[keyed[i].second]);
  return S;
}

// --- Build (Algorithm 1) -------------------------------------------------------
int new_leaf(Tree& T, const Set& Q, int h) {
  Node n;
  n.leaf = true;
  n.size = static_cast<int64_t>(Q.size());
  n.depth = h;
  n.pts = Q;
  T.nodes.push_back(std::move(n));
  return static_cast<int>(T.nodes.size()) - 1;
}

int new_interior(Tree& T, int d, int64_t x, int h) {
  Node n;
  n.leaf = false;
  n.dim = d;
  n.x = x;
  n.depth = h;
  T.nodes.push_back(std::move(n));
  return static_cast<int>(T.nodes.size()) - 1;
}

int build(Tree& T, const Set& Q, int h);

// One exact split of Q by the split rule, children built recursively.  This is
// the plain construction's step (Section 3) and also the fallback when the
// sample of a large set is all identical.
int split_node(Tree& T, const Set& Q, int h) {
  int d = widest_dim(T.st, Q);
  int64_t x = split_value(T.st, Q, d);
  Set L, R;
  for (int64_t q : Q) (T.st.coord(q, d) < x ? L : R).push_back(q);
  int me = new_interior(T, d, x, h);
  T.nodes[me].plain = true;
  int l = build(T, L, h + 1);
  int r = build(T, R, h + 1);
  T.nodes[me].left = l;
  T.nodes[me].right = r;
  T.nodes[me].size = T.nodes[l].size + T.nodes[r].size;
  return me;
}

// Turn the skeleton (heap node v, at tree depth h) into tree nodes; external
// nodes become Build(bucket, depth) recursively.
int emit(Tree& T, const Skeleton& sk, std::vector<Set>& R, int v, int h) {
  if (sk.external[v]) {
    int l = level_of(v);
    int label = (v << (sk.lambda - l)) - (1 << sk.lambda);
    return build(T, R[label], h);
  }
  int me = new_interior(T, sk.dim[v], sk.x[v], h);
  int l = emit(T, sk, R, 2 * v, h + 1);
  int r = emit(T, sk, R, 2 * v + 1, h + 1);
  T.nodes[me].left = l;
  T.nodes[me].right = r;
  T.nodes[me].size = T.nodes[l].size + T.nodes[r].size;
  return me;
}

int build(Tree& T, const Set& Q, int h) {
  const Params& p = T.p;
  const size_t s = static_cast<size_t>(p.sigma) << p.lambda;
  if (Q.size() <= static_cast<size_t>(p.phi)) return new_leaf(T, Q, h);
  if (all_identical(T.st, Q)) return new_leaf(T, Q, h);      // heavy leaf
  if (Q.size() < s) return split_node(T, Q, h);               // plain construction
  if (p.sigma == 0) return split_node(T, Q, h);               // no sampling: exact medians everywhere
  Set S = take_sample(T, Q, h, s);
  Skeleton sk = build_skeleton(T.st, S, p.lambda);
  if (sk.external[1]) return split_node(T, Q, h);             // degenerate sample
  // Sieve: a stable distribution of Q into the 2^lambda buckets.
  std::vector<Set> R(static_cast<size_t>(1) << p.lambda);
  for (int64_t q : Q) R[route(T.st, sk, q)].push_back(q);
  return emit(T, sk, R, 1, h);
}

// --- Tree helpers --------------------------------------------------------------
void collect(const Tree& T, int t, Set& out) {
  const Node& n = T.nodes[t];
  if (n.leaf) {
    out.insert(out.end(), n.pts.begin(), n.pts.end());
    return;
  }
  collect(T, n.left, out);
  collect(T, n.right, out);
}

bool balanced(const Params& p, int64_t l, int64_t n) {
  if (n <= 0) return false;
  int64_t lo = (p.alpha_den - 2 * p.alpha_num) * n;
  int64_t mid = 2 * p.alpha_den * l;
  int64_t hi = (p.alpha_den + 2 * p.alpha_num) * n;
  return lo <= mid && mid <= hi;
}

bool goes_left(const Tree& T, const Node& n, int64_t q) { return T.st.coord(q, n.dim) < n.x; }

// --- BatchInsert (Algorithm 2, node by node) ----------------------------------
int insert_rec(Tree& T, int t, const Set& P, int h) {
  if (P.empty()) return t;
  if (T.nodes[t].leaf) {
    Set all = T.nodes[t].pts;
    all.insert(all.end(), P.begin(), P.end());
    T.log.leaf_rebuilds += 1;
    T.log.leaf_points += static_cast<int64_t>(all.size());
    return build(T, all, h);
  }
  Set PL, PR;
  for (int64_t q : P) (goes_left(T, T.nodes[t], q) ? PL : PR).push_back(q);
  int64_t n_after = T.nodes[t].size + static_cast<int64_t>(P.size());
  int64_t l_after = T.nodes[T.nodes[t].left].size + static_cast<int64_t>(PL.size());
  if (!balanced(T.p, l_after, n_after)) {
    Set all;
    collect(T, t, all);
    all.insert(all.end(), P.begin(), P.end());
    T.log.interior_rebuilds += 1;
    T.log.interior_points += static_cast<int64_t>(all.size());
    return build(T, all, h);
  }
  T.log.kept += 1;
  int l = insert_rec(T, T.nodes[t].left, PL, h + 1);
  int r = insert_rec(T, T.nodes[t].right, PR, h + 1);
  T.nodes[t].left = l;
  T.nodes[t].right = r;
  T.nodes[t].size = n_after;
  return t;
}

// --- BatchDelete (Section 4.2, two rounds) ------------------------------------
int64_t count_marked(const Tree& T, int t, const std::vector<char>& marked, std::vector<int64_t>& del) {
  const Node& n = T.nodes[t];
  int64_t c = 0;
  if (n.leaf) {
    for (int64_t q : n.pts) c += marked[q];
  } else {
    c = count_marked(T, n.left, marked, del) + count_marked(T, n.right, marked, del);
  }
  del[t] = c;
  return c;
}

int delete_rec(Tree& T, int t, const std::vector<char>& marked, const std::vector<int64_t>& del, int h) {
  if (del[t] == 0) return t;
  if (T.nodes[t].leaf) {
    Set keep;
    for (int64_t q : T.nodes[t].pts)
      if (!marked[q]) keep.push_back(q);
    if (keep.empty()) return build(T, keep, h);   // only reachable at the root
    T.nodes[t].pts = keep;
    T.nodes[t].size = static_cast<int64_t>(keep.size());
    return t;
  }
  int64_t n_after = T.nodes[t].size - del[t];
  int64_t l_after = T.nodes[T.nodes[t].left].size - del[T.nodes[t].left];
  if (!balanced(T.p, l_after, n_after)) {
    Set all, keep;
    collect(T, t, all);
    for (int64_t q : all)
      if (!marked[q]) keep.push_back(q);
    T.log.interior_rebuilds += 1;
    T.log.interior_points += static_cast<int64_t>(keep.size());
    return build(T, keep, h);
  }
  T.log.kept += 1;
  int l = delete_rec(T, T.nodes[t].left, marked, del, h + 1);
  int r = delete_rec(T, T.nodes[t].right, marked, del, h + 1);
  T.nodes[t].left = l;
  T.nodes[t].right = r;
  T.nodes[t].size = n_after;
  return t;
}

// --- Queries -------------------------------------------------------------------
int64_t sqdist(const Store& st, int64_t p, const int64_t* q, int64_t qs, int64_t j) {
  int64_t s = 0;
  for (int d = 0; d < st.D; ++d) {
    int64_t diff = st.coord(p, d) - q[d * qs + j];
    s += diff * diff;
  }
  return s;
}

using Cand = std::pair<int64_t, int64_t>;  // (squared distance, id)

struct KnnState {
  const Tree* T;
  const int64_t* q;
  int64_t qs, j;
  size_t k;
  std::vector<Cand> best;  // sorted ascending, at most k entries
  // work of the search (the per-query counts of Appendix H): nodes whose
  // record is read (not pruned), leaves scanned, points scanned in them
  int64_t nodes = 0, leaves = 0, points = 0;
  void offer(int64_t p) {
    Cand c{sqdist(T->st, p, q, qs, j), T->st.id[p]};
    if (best.size() == k && !(c < best.back())) return;
    best.insert(std::upper_bound(best.begin(), best.end(), c), c);
    if (best.size() > k) best.pop_back();
  }
  // Prune only when the cell is strictly farther than the current k-th pair.
  bool prune(int64_t lb) const { return best.size() == k && lb > best.back().first; }
};

// Lower bound on the squared distance from q to the cell [lo, hi].
int64_t cell_bound(const KnnState& S, const std::vector<int64_t>& lo, const std::vector<int64_t>& hi) {
  int64_t s = 0;
  for (size_t d = 0; d < lo.size(); ++d) {
    int64_t v = S.q[d * S.qs + S.j];
    int64_t off = v < lo[d] ? lo[d] - v : (v > hi[d] ? v - hi[d] : 0);
    s += off * off;
  }
  return s;
}

// Depth-first search: nearer child first, the other child pruned by the bound
// of its subspace, computed on the fly from the splitters (Section 5).
void knn_rec(KnnState& S, int t, std::vector<int64_t>& lo, std::vector<int64_t>& hi) {
  const Node& n = S.T->nodes[t];
  if (S.prune(cell_bound(S, lo, hi))) return;
  S.nodes += 1;
  if (n.leaf) {
    S.leaves += 1;
    S.points += static_cast<int64_t>(n.pts.size());
    for (int64_t p : n.pts) S.offer(p);
    return;
  }
  int d = n.dim;
  bool left_first = S.q[d * S.qs + S.j] < n.x;
  for (int pass = 0; pass < 2; ++pass) {
    bool go_left = (pass == 0) == left_first;
    int64_t save_lo = lo[d], save_hi = hi[d];
    if (go_left) hi[d] = n.x - 1; else lo[d] = n.x;
    knn_rec(S, go_left ? n.left : n.right, lo, hi);
    lo[d] = save_lo;
    hi[d] = save_hi;
  }
}

const int64_t kCoordMax = (int64_t{1} << 30) - 1;

int64_t range_rec(const Tree& T, int t, std::vector<int64_t>& clo, std::vector<int64_t>& chi,
                  const int64_t* lo, const int64_t* hi, int64_t bs, int64_t j) {
  const Node& n = T.nodes[t];
  int D = T.st.D;
  bool inside = true;
  for (int d = 0; d < D; ++d) {
    if (chi[d] < lo[d * bs + j] || clo[d] > hi[d * bs + j]) return 0;   // disjoint
    if (clo[d] < lo[d * bs + j] || chi[d] > hi[d * bs + j]) inside = false;
  }
  if (inside) return n.size;   // the subtree size answers a contained cell
  if (n.leaf) {
    int64_t c = 0;
    for (int64_t p : n.pts) {
      bool in = true;
      for (int d = 0; d < D; ++d) {
        int64_t v = T.st.coord(p, d);
        if (v < lo[d * bs + j] || v > hi[d * bs + j]) in = false;
      }
      c += in;
    }
    return c;
  }
  int64_t total = 0;
  int d = n.dim;
  int64_t save = chi[d];
  chi[d] = n.x - 1;
  if (clo[d] <= chi[d]) total += range_rec(T, n.left, clo, chi, lo, hi, bs, j);
  chi[d] = save;
  save = clo[d];
  clo[d] = n.x;
  total += range_rec(T, n.right, clo, chi, lo, hi, bs, j);
  clo[d] = save;
  return total;
}

// Range report (Section 5): the points of a closed box.  A cell inside the box
// contributes its whole subtree (flattened); a leaf that straddles the box
// contributes the points that lie in it; disjoint cells nothing.  Points are
// appended in the tree's in-order.
void range_report_rec(const Tree& T, int t, std::vector<int64_t>& clo, std::vector<int64_t>& chi,
                      const int64_t* lo, const int64_t* hi, int64_t bs, int64_t j, std::vector<int64_t>& out) {
  const Node& n = T.nodes[t];
  int D = T.st.D;
  bool inside = true;
  for (int d = 0; d < D; ++d) {
    if (chi[d] < lo[d * bs + j] || clo[d] > hi[d * bs + j]) return;   // disjoint
    if (clo[d] < lo[d * bs + j] || chi[d] > hi[d * bs + j]) inside = false;
  }
  if (inside) {
    Set all;
    collect(T, t, all);
    for (int64_t p : all) out.push_back(T.st.id[p]);
    return;
  }
  if (n.leaf) {
    for (int64_t p : n.pts) {
      bool in = true;
      for (int d = 0; d < D; ++d) {
        int64_t v = T.st.coord(p, d);
        if (v < lo[d * bs + j] || v > hi[d * bs + j]) in = false;
      }
      if (in) out.push_back(T.st.id[p]);
    }
    return;
  }
  int d = n.dim;
  int64_t save = chi[d];
  chi[d] = n.x - 1;
  if (clo[d] <= chi[d]) range_report_rec(T, n.left, clo, chi, lo, hi, bs, j, out);
  chi[d] = save;
  save = clo[d];
  clo[d] = n.x;
  range_report_rec(T, n.right, clo, chi, lo, hi, bs, j, out);
  clo[d] = save;
}

// --- Canonical export (pre-order) -----------------------------------------------
void export_rec(const Tree& T, int t, std::vector<int64_t>& rows, std::vector<int64_t>& leaf_pts) {
  const Node& n = T.nodes[t];
  rows.push_back(n.leaf ? 1 : 0);
  rows.push_back(n.leaf ? -1 : n.dim);
  rows.push_back(n.leaf ? 0 : n.x);
  rows.push_back(n.size);
  if (n.leaf) {
    Set s = n.pts;
    std::sort(s.begin(), s.end(), [&](int64_t a, int64_t b) { return T.st.id[a] < T.st.id[b]; });
    leaf_pts.insert(leaf_pts.end(), s.begin(), s.end());
    return;
  }
  export_rec(T, n.left, rows, leaf_pts);
  export_rec(T, n.right, rows, leaf_pts);
}

int height_rec(const Tree& T, int t) {
  const Node& n = T.nodes[t];
  if (n.leaf) return 0;
  return 1 + std::max(height_rec(T, n.left), height_rec(T, n.right));
}

int64_t count_nodes(const Tree& T, int t) {
  const Node& n = T.nodes[t];
  return n.leaf ? 1 : 1 + count_nodes(T, n.left) + count_nodes(T, n.right);
}

Params make_params(int D, int lambda, int phi, int sigma, int64_t an, int64_t ad, uint64_t seed) {
  Params p;
  p.D = D;
  p.lambda = lambda;
  p.phi = phi;
  p.sigma = sigma;
  p.alpha_num = an;
  p.alpha_den = ad;
  p.seed = seed;
  return p;
}

}  // namespace

// =============================== C interface ===================================
extern "C" {

struct orc_tree {
  Tree t;
};

uint64_t orc_mix64(uint64_t z) { return mix64(z); }

int orc_balanced(int64_t l, int64_t n, int64_t alpha_num, int64_t alpha_den) {
  Params p = make_params(1, 1, 1, 1, alpha_num, alpha_den, 0);
  return balanced(p, l, n) ? 1 : 0;
}
uint64_t orc_sample_key(uint64_t seed, int64_t h, int64_t id) { return sample_key(seed, h, id); }

// Build(P) with its root at depth h of an enclosing tree (h salts the samples;
// a rebuild of a node at depth h is Build of its points at depth h).
orc_tree* orc_build_at(int D, int lambda, int phi, int sigma, int64_t alpha_num, int64_t alpha_den,
                       uint64_t seed, const int64_t* coords, const int64_t* ids, int64_t n, int h) {
  orc_tree* o = new orc_tree;
  o->t.p = make_params(D, lambda, phi, sigma, alpha_num, alpha_den, seed);
  o->t.st.D = D;
  Set Q;
  for (int64_t j = 0; j < n; ++j) Q.push_back(o->t.st.add(coords, n, j, ids[j]));
  o->t.root = build(o->t, Q, h);
  return o;
}

orc_tree* orc_build(int D, int lambda, int phi, int sigma, int64_t alpha_num, int64_t alpha_den,
                    uint64_t seed, const int64_t* coords, const int64_t* ids, int64_t n) {
  return orc_build_at(D, lambda, phi, sigma, alpha_num, alpha_den, seed, coords, ids, n, 0);
}

// What the last orc_insert / orc_delete rebuilt: out[0] interior subtrees
// rebuilt, out[1] their points, out[2] leaves rebuilt, out[3] their points,
// out[4] kept interior nodes that the batch reached.
void orc_update_log(const orc_tree* o, int64_t* out) {
  const UpdateLog& L = o->t.log;
  out[0] = L.interior_rebuilds;
  out[1] = L.interior_points;
  out[2] = L.leaf_rebuilds;
  out[3] = L.leaf_points;
  out[4] = L.kept;
}

void orc_free(orc_tree* o) { delete o; }

int64_t orc_size(const orc_tree* o) { return o->t.nodes[o->t.root].size; }
int64_t orc_num_nodes(const orc_tree* o) { return count_nodes(o->t, o->t.root); }
int orc_height(const orc_tree* o) { return height_rec(o->t, o->t.root); }

void orc_insert(orc_tree* o, const int64_t* coords, const int64_t* ids, int64_t m) {
  Set P;
  for (int64_t j = 0; j < m; ++j) P.push_back(o->t.st.add(coords, m, j, ids[j]));
  o->t.log = UpdateLog();
  o->t.root = insert_rec(o->t, o->t.root, P, 0);
}

// Returns the number of points removed.  A batch entry removes the stored point
// with the same id and the same coordinates in the leaf its coordinates route
// to; entries that match nothing are ignored, and a repeated entry removes once.
int64_t orc_delete(orc_tree* o, const int64_t* coords, const int64_t* ids, int64_t m) {
  Tree& T = o->t;
  int D = T.st.D;
  std::vector<char> marked(T.st.id.size(), 0);
  int64_t removed = 0;
  for (int64_t j = 0; j < m; ++j) {
    int t = T.root;
    while (!T.nodes[t].leaf) {
      const Node& n = T.nodes[t];
      t = coords[n.dim * m + j] < n.x ? n.left : n.right;
    }
    for (int64_t q : T.nodes[t].pts) {
      if (T.st.id[q] != ids[j] || marked[q]) continue;
      bool same = true;
      for (int d = 0; d < D; ++d) same = same && T.st.coord(q, d) == coords[d * m + j];
      if (same) {
        marked[q] = 1;
        ++removed;
        break;
      }
    }
  }
  std::vector<int64_t> del(T.nodes.size(), 0);
  T.log = UpdateLog();
  count_marked(T, T.root, marked, del);
  T.root = delete_rec(T, T.root, marked, del, 0);
  return removed;
}

void orc_knn(const orc_tree* o, const int64_t* q, int64_t nq, int k, int64_t* out_ids, int64_t* out_d2) {
  const Tree& T = o->t;
  for (int64_t j = 0; j < nq; ++j) {
    KnnState S{&T, q, nq, j, static_cast<size_t>(k), {}};
    std::vector<int64_t> lo(T.st.D, 0), hi(T.st.D, kCoordMax);
    knn_rec(S, T.root, lo, hi);
    for (int i = 0; i < k; ++i) {
      bool have = i < static_cast<int>(S.best.size());
      out_d2[j * k + i] = have ? S.best[i].first : -1;
      out_ids[j * k + i] = have ? S.best[i].second : -1;
    }
  }
}

// The same queries split into `threads` contiguous ranges, each answered by
// orc_knn on its own thread (for timing the oracle on all host cores; the
// per-query search is unchanged).
void orc_knn_threads(const orc_tree* o, const int64_t* q, int64_t nq, int k, int64_t* out_ids, int64_t* out_d2,
                     int threads) {
  if (threads < 1) threads = 1;
  const int64_t per = (nq + threads - 1) / threads;
  std::vector<std::vector<int64_t>> qs(threads);
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) {
    const int64_t a = std::min<int64_t>(nq, t * per), b = std::min<int64_t>(nq, a + per);
    if (a >= b) break;
    // the query block as its own [D][b-a] array
    const int D = o->t.st.D;
    qs[t].resize(static_cast<size_t>(D) * (b - a));
    for (int d = 0; d < D; ++d)
      for (int64_t j = a; j < b; ++j) qs[t][d * (b - a) + (j - a)] = q[d * nq + j];
    pool.emplace_back([o, &qs, t, a, b, k, out_ids, out_d2]() {
      orc_knn(o, qs[t].data(), b - a, k, out_ids + a * k, out_d2 + a * k);
    });
  }
  for (auto& th : pool) th.join();
}

// Per-query work of the k-NN search: nodes read (not pruned), leaves scanned
// and points scanned in them.
void orc_knn_visits(const orc_tree* o, const int64_t* q, int64_t nq, int k, int64_t* nodes, int64_t* leaves,
                    int64_t* points) {
  const Tree& T = o->t;
  for (int64_t j = 0; j < nq; ++j) {
    KnnState S{&T, q, nq, j, static_cast<size_t>(k), {}};
    std::vector<int64_t> lo(T.st.D, 0), hi(T.st.D, kCoordMax);
    knn_rec(S, T.root, lo, hi);
    nodes[j] = S.nodes;
    leaves[j] = S.leaves;
    points[j] = S.points;
  }
}

void orc_range_count(const orc_tree* o, const int64_t* lo, const int64_t* hi, int64_t nb, int64_t* out) {
  const Tree& T = o->t;
  for (int64_t j = 0; j < nb; ++j) {
    std::vector<int64_t> clo(T.st.D, 0), chi(T.st.D, kCoordMax);
    out[j] = range_rec(T, T.root, clo, chi, lo, hi, nb, j);
  }
}

// Range report: box j's point ids, in the tree's in-order, written from
// out_ids[off[j]] on (off: prefix sums of the box counts, which the caller
// takes from orc_range_count).
void orc_range_report(const orc_tree* o, const int64_t* lo, const int64_t* hi, int64_t nb, const int64_t* off,
                      int64_t* out_ids) {
  const Tree& T = o->t;
  std::vector<int64_t> ids;
  for (int64_t j = 0; j < nb; ++j) {
    std::vector<int64_t> clo(T.st.D, 0), chi(T.st.D, kCoordMax);
    ids.clear();
    range_report_rec(T, T.root, clo, chi, lo, hi, nb, j, ids);
    std::copy(ids.begin(), ids.end(), out_ids + off[j]);
  }
}

// Pre-order export.  rows: [num_nodes][4] = (kind 0 interior / 1 leaf, dim or -1,
// x or 0, size).  leaf_ids/leaf_coords: the points of the leaves in pre-order,
// ids ascending inside each leaf; coords as [D][size].
void orc_export(const orc_tree* o, int64_t* rows, int64_t* leaf_ids, int64_t* leaf_coords) {
  const Tree& T = o->t;
  std::vector<int64_t> r, pts;
  export_rec(T, T.root, r, pts);
  std::memcpy(rows, r.data(), r.size() * sizeof(int64_t));
  int64_t n = static_cast<int64_t>(pts.size());
  for (int64_t i = 0; i < n; ++i) {
    leaf_ids[i] = T.st.id[pts[i]];
    for (int d = 0; d < T.st.D; ++d) leaf_coords[d * n + i] = T.st.coord(pts[i], d);
  }
}

// Node depths and plain-split flags in pre-order (depths for checking the
// sampling salts of rebuilt nodes; the flag marks interior nodes made by one
// exact split rather than taken from a skeleton).
void orc_export_depths(const orc_tree* o, int32_t* depths, int8_t* plain) {
  const Tree& T = o->t;
  std::vector<int> stack{T.root};
  int64_t i = 0;
  while (!stack.empty()) {
    int t = stack.back();
    stack.pop_back();
    plain[i] = T.nodes[t].plain ? 1 : 0;
    depths[i++] = T.nodes[t].depth;
    if (!T.nodes[t].leaf) {
      stack.push_back(T.nodes[t].right);
      stack.push_back(T.nodes[t].left);
    }
  }
}

// ---- Building blocks, exposed so that tests can pin them individually ----------

// The sample of a set: handles (positions 0..n-1) of the s smallest (key, id).
void orc_sample(uint64_t seed, int64_t h, const int64_t* ids, int64_t n, int64_t s, int64_t* out_pos) {
  Tree T;
  T.p = make_params(1, 1, 1, 1, 3, 10, seed);
  T.st.D = 1;
  int64_t zero = 0;
  Set Q;
  for (int64_t j = 0; j < n; ++j) Q.push_back(T.st.add(&zero, 0, 0, ids[j]));
  Set S = take_sample(T, Q, static_cast<int>(h), static_cast<size_t>(s));
  for (int64_t i = 0; i < s; ++i) out_pos[i] = S[i];
}

// Split rule on a point set: writes the dimension and value; returns 0, or -1
// when the set has zero width in every dimension (no split exists).
int orc_split_rule(int D, const int64_t* coords, int64_t n, int* out_dim, int64_t* out_x) {
  Store st;
  st.D = D;
  Set Q;
  for (int64_t j = 0; j < n; ++j) Q.push_back(st.add(coords, n, j, j));
  if (n < 1 || all_identical(st, Q)) return -1;
  *out_dim = widest_dim(st, Q);
  *out_x = split_value(st, Q, *out_dim);
  return 0;
}

// Skeleton of lambda levels on a sample.  Heap arrays of length 2^lambda
// (index 0 unused): dim (-1 where not an interior node), x; ext of length
// 2^(lambda+1): 1 at external nodes.
void orc_skeleton(int D, int lambda, const int64_t* coords, int64_t n, int32_t* out_dim, int64_t* out_x,
                  int8_t* out_ext) {
  Store st;
  st.D = D;
  Set S;
  for (int64_t j = 0; j < n; ++j) S.push_back(st.add(coords, n, j, j));
  Skeleton sk = build_skeleton(st, S, lambda);
  for (int v = 0; v < (1 << lambda); ++v) {
    out_dim[v] = sk.external[v] || v == 0 ? -1 : sk.dim[v];
    out_x[v] = sk.x[v];
  }
  for (int v = 0; v < (2 << lambda); ++v) out_ext[v] = sk.external[v];
}

// Sieve of a point set through a skeleton given by heap arrays (as produced by
// orc_skeleton): labels per point, and the stable order (positions).
void orc_sieve(int D, int lambda, const int32_t* sk_dim, const int64_t* sk_x, const int8_t* sk_ext,
               const int64_t* coords, int64_t n, int32_t* out_label, int64_t* out_order) {
  Store st;
  st.D = D;
  for (int64_t j = 0; j < n; ++j) st.add(coords, n, j, j);
  Skeleton sk;
  sk.lambda = lambda;
  sk.dim.assign(sk_dim, sk_dim + (1 << lambda));
  sk.x.assign(sk_x, sk_x + (1 << lambda));
  sk.external.assign(sk_ext, sk_ext + (2 << lambda));
  std::vector<Set> R(static_cast<size_t>(1) << lambda);
  for (int64_t j = 0; j < n; ++j) {
    out_label[j] = route(st, sk, j);
    R[out_label[j]].push_back(j);
  }
  int64_t i = 0;
  for (const Set& b : R)
    for (int64_t q : b) out_order[i++] = q;
}

// The root skeleton of Build(P) for a large P (sample, then skeleton), so that a
// full-size GPU tree can be checked at its top levels without a full oracle run.
void orc_root_skeleton(int D, int lambda, int sigma, uint64_t seed, int64_t h, const int64_t* coords,
                       const int64_t* ids, int64_t n, int32_t* out_dim, int64_t* out_x, int8_t* out_ext) {
  int64_t s = static_cast<int64_t>(sigma) << lambda;
  std::vector<std::pair<uint64_t, int64_t>> keyed(n);
  for (int64_t j = 0; j < n; ++j) keyed[j] = {sample_key(seed, h, ids[j]), ids[j]};
  std::vector<int64_t> pos(n);
  std::iota(pos.begin(), pos.end(), 0);
  std::nth_element(pos.begin(), pos.begin() + (s - 1), pos.end(),
                   [&](int64_t a, int64_t b) { return keyed[a] < keyed[b]; });
  std::vector<int64_t> samp(static_cast<size_t>(D) * s);
  for (int64_t i = 0; i < s; ++i)
    for (int d = 0; d < D; ++d) samp[d * s + i] = coords[d * n + pos[i]];
  orc_skeleton(D, lambda, samp.data(), s, out_dim, out_x, out_ext);
}

// Brute force, the plain definitions (Section 2): k smallest (d^2, id) pairs,
// ascending, padded with -1; closed-box counts.
void orc_brute_knn(int D, const int64_t* coords, const int64_t* ids, int64_t n, const int64_t* q, int64_t nq,
                   int k, int64_t* out_ids, int64_t* out_d2) {
  std::vector<Cand> all(n);
  for (int64_t j = 0; j < nq; ++j) {
    for (int64_t i = 0; i < n; ++i) {
      int64_t s = 0;
      for (int d = 0; d < D; ++d) {
        int64_t diff = coords[d * n + i] - q[d * nq + j];
        s += diff * diff;
      }
      all[i] = {s, ids[i]};
    }
    int64_t kk = std::min<int64_t>(k, n);
    std::partial_sort(all.begin(), all.begin() + kk, all.end());
    for (int i = 0; i < k; ++i) {
      out_d2[j * k + i] = i < kk ? all[i].first : -1;
      out_ids[j * k + i] = i < kk ? all[i].second : -1;
    }
  }
}

void orc_brute_range_count(int D, const int64_t* coords, int64_t n, const int64_t* lo, const int64_t* hi,
                           int64_t nb, int64_t* out) {
  for (int64_t j = 0; j < nb; ++j) {
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) {
      bool in = true;
      for (int d = 0; d < D; ++d) {
        int64_t v = coords[d * n + i];
        if (v < lo[d * nb + j] || v > hi[d * nb + j]) in = false;
      }
      c += in;
    }
    out[j] = c;
  }
}

}  // extern "C"
