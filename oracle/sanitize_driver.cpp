// Drives every entry point of the CPU oracle on small seeded inputs, for a
// build with AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure: tests/test_oracle_sanitize.py compiles and runs it).  Exits
// non-zero when a result breaks a basic invariant; the sanitizers report
// memory and undefined-behaviour errors themselves.
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
struct orc_tree;
orc_tree* orc_build(int, int, int, int, int64_t, int64_t, uint64_t, const int64_t*, const int64_t*, int64_t);
orc_tree* orc_build_at(int, int, int, int, int64_t, int64_t, uint64_t, const int64_t*, const int64_t*, int64_t, int);
void orc_free(orc_tree*);
int64_t orc_size(const orc_tree*);
int64_t orc_num_nodes(const orc_tree*);
int orc_height(const orc_tree*);
void orc_insert(orc_tree*, const int64_t*, const int64_t*, int64_t);
int64_t orc_delete(orc_tree*, const int64_t*, const int64_t*, int64_t);
void orc_update_log(const orc_tree*, int64_t*);
void orc_knn(const orc_tree*, const int64_t*, int64_t, int, int64_t*, int64_t*);
void orc_knn_threads(const orc_tree*, const int64_t*, int64_t, int, int64_t*, int64_t*, int);
void orc_knn_visits(const orc_tree*, const int64_t*, int64_t, int, int64_t*, int64_t*, int64_t*);
void orc_range_count(const orc_tree*, const int64_t*, const int64_t*, int64_t, int64_t*);
void orc_range_report(const orc_tree*, const int64_t*, const int64_t*, int64_t, const int64_t*, int64_t*);
void orc_export(const orc_tree*, int64_t*, int64_t*, int64_t*);
void orc_export_depths(const orc_tree*, int32_t*, int8_t*);
void orc_brute_knn(int, const int64_t*, const int64_t*, int64_t, const int64_t*, int64_t, int, int64_t*, int64_t*);
void orc_brute_range_count(int, const int64_t*, int64_t, const int64_t*, const int64_t*, int64_t, int64_t*);
}

namespace {
uint64_t state = 0x1234567;
int64_t rnd(int64_t hi) {   // a 64-bit LCG (Knuth's MMIX constants); modulo bias is irrelevant here
  state = state * 6364136223846793005ULL + 1442695040888963407ULL;
  return static_cast<int64_t>((state >> 17) % static_cast<uint64_t>(hi));
}

int check(bool ok, const char* what) {
  if (!ok) std::fprintf(stderr, "sanitize driver: %s\n", what);
  return ok ? 0 : 1;
}

int run(int D, int64_t n, int64_t span, int lambda, int phi, int sigma) {
  int bad = 0;
  std::vector<int64_t> c(D * n), id(n);
  for (int64_t j = 0; j < n; ++j) {
    id[j] = j * 3 + 1;
    for (int d = 0; d < D; ++d) c[d * n + j] = j % 7 == 0 ? 5 : rnd(span);   // duplicates as well
  }
  orc_tree* T = orc_build(D, lambda, phi, sigma, 3, 10, 42, c.data(), id.data(), n);
  bad += check(orc_size(T) == n, "size after build");
  const int64_t N = orc_num_nodes(T);
  std::vector<int64_t> rows(4 * N), lid(n), lc(D * n);
  orc_export(T, rows.data(), lid.data(), lc.data());
  std::vector<int32_t> dep(N);
  std::vector<int8_t> pl(N);
  orc_export_depths(T, dep.data(), pl.data());
  // insert, delete (absent, mismatched and repeated entries), rebuild log
  const int64_t m = n / 3 + 1;
  std::vector<int64_t> bc(D * m), bi(m);
  for (int64_t j = 0; j < m; ++j) {
    bi[j] = 10'000'000 + j;
    for (int d = 0; d < D; ++d) bc[d * m + j] = rnd(span);
  }
  orc_insert(T, bc.data(), bi.data(), m);
  bad += check(orc_size(T) == n + m, "size after insert");
  int64_t log[5];
  orc_update_log(T, log);
  std::vector<int64_t> dc(D * m), di(m);
  for (int64_t j = 0; j < m; ++j) {
    const int64_t k = (j * 2) % n;
    di[j] = j % 5 == 0 ? -7 : id[k];
    for (int d = 0; d < D; ++d) dc[d * m + j] = c[d * n + k] + (j % 11 == 0 ? 1 : 0);
  }
  const int64_t removed = orc_delete(T, dc.data(), di.data(), m);
  bad += check(removed >= 0 && removed <= m && orc_size(T) == n + m - removed, "size after delete");
  // queries against brute force on the current set
  std::vector<int64_t> cur_c, cur_i;
  {
    const int64_t M = orc_size(T), NN = orc_num_nodes(T);
    std::vector<int64_t> r2(4 * NN), i2(M), c2(D * M);
    orc_export(T, r2.data(), i2.data(), c2.data());
    cur_c = c2;
    cur_i = i2;
  }
  const int64_t M = static_cast<int64_t>(cur_i.size());
  const int64_t nq = 50;
  std::vector<int64_t> q(D * nq);
  for (auto& v : q) v = rnd(span);
  for (int k : {1, 7, 40}) {
    std::vector<int64_t> a(nq * k), b(nq * k), e(nq * k), f(nq * k), g(nq * k), h(nq * k);
    orc_knn(T, q.data(), nq, k, a.data(), b.data());
    orc_knn_threads(T, q.data(), nq, k, g.data(), h.data(), 3);
    orc_brute_knn(D, cur_c.data(), cur_i.data(), M, q.data(), nq, k, e.data(), f.data());
    bad += check(a == e && b == f && a == g && b == h, "k-NN against brute force");
    std::vector<int64_t> vn(nq), vl(nq), vp(nq);
    orc_knn_visits(T, q.data(), nq, k, vn.data(), vl.data(), vp.data());
  }
  std::vector<int64_t> lo(D * nq), hi(D * nq), cnt(nq), bcnt(nq);
  for (int64_t j = 0; j < nq; ++j)
    for (int d = 0; d < D; ++d) {
      lo[d * nq + j] = rnd(span);
      hi[d * nq + j] = lo[d * nq + j] + rnd(span / 2 + 1) - (j == 3 ? span : 0);   // one inverted box
    }
  orc_range_count(T, lo.data(), hi.data(), nq, cnt.data());
  orc_brute_range_count(D, cur_c.data(), M, lo.data(), hi.data(), nq, bcnt.data());
  bad += check(cnt == bcnt, "range count against brute force");
  std::vector<int64_t> off(nq + 1, 0);
  for (int64_t j = 0; j < nq; ++j) off[j + 1] = off[j] + cnt[j];
  std::vector<int64_t> rep(off[nq] + 1);
  orc_range_report(T, lo.data(), hi.data(), nq, off.data(), rep.data());
  orc_free(T);
  // a rebuild at depth and an empty tree
  orc_tree* U = orc_build_at(D, lambda, phi, sigma, 3, 10, 7, c.data(), id.data(), n, 5);
  orc_free(U);
  orc_tree* E = orc_build(D, lambda, phi, sigma, 3, 10, 42, c.data(), id.data(), 0);
  bad += check(orc_size(E) == 0, "empty tree");
  orc_insert(E, bc.data(), bi.data(), m);
  orc_free(E);
  return bad;
}
}  // namespace

int main() {
  int bad = 0;
  bad += run(2, 3000, 1000000, 6, 32, 32);
  bad += run(3, 5000, 200, 3, 4, 4);      // many ties, small skeletons and leaves
  bad += run(1, 2500, 1 << 29, 2, 8, 8);
  bad += run(3, 4000, 100000, 1, 32, 0);  // exact medians
  std::fprintf(stderr, "sanitize driver: %s\n", bad ? "FAILED" : "ok");
  return bad ? 1 : 0;
}
