// Host sanitizer driver for the CPU-side C and C++ sources: the oracle
// (oracle/oracle.c) and the input generators (graphgen/graphgen.cpp) are
// compiled with AddressSanitizer and UndefinedBehaviorSanitizer (no
// recovery) and exercised on small graphs of every family.  Any invalid
// access, leak or undefined operation aborts the run with a report; the
// driver also checks a few results against each other, so that it cannot
// pass by computing nothing.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
struct gg_csr;
int32_t gg_n(const gg_csr* g);
int64_t gg_m(const gg_csr* g);
void gg_copy(const gg_csr* g, int64_t* row_ptr, int32_t* col, int32_t* w);
void gg_free(gg_csr* g);
gg_csr* gg_grid(int32_t R, int32_t C, int32_t wlo, int32_t whi, uint64_t seed);
gg_csr* gg_road(int32_t side, double p_keep, double lr_frac, int32_t lr_radius, uint64_t seed);
gg_csr* gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, int32_t wlo, int32_t whi,
                uint64_t seed);
gg_csr* gg_rgg(int32_t n, double mean_degree, uint64_t seed, int32_t* xs, int32_t* ys);
void gg_grid_heuristic(int32_t side, int32_t target, int32_t* h);
void gg_uniform(uint64_t seed, uint64_t stream, int64_t count, uint64_t k, int64_t* out);

int oracle_dijkstra(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t src,
                    int64_t* dist);
int oracle_bellman_ford(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t src,
                        int64_t* dist);
int oracle_bfs_reach(int32_t n, const int64_t* row_ptr, const int32_t* col, int32_t src, uint8_t* reached);
int oracle_canonical_pred(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t src,
                          const int64_t* dist, int32_t* pred);
int64_t oracle_to_i32(int32_t n, const int64_t* d64, int32_t* d32);
int64_t oracle_ppsp(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t src,
                    int32_t dst);
int64_t oracle_astar(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t src,
                     int32_t dst, const int32_t* hh, int64_t* expanded);
uint32_t oracle_check(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w, int32_t src,
                      const int32_t* dist, const int32_t* pred);
int oracle_dijkstra_f64(int32_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t src,
                        double* dist);
int oracle_dijkstra_f32(int32_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t src,
                        double* dist);
int oracle_tree_real(int32_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t src,
                     const double* dist, int use_f32, int32_t* pred, int32_t* pred_edge);
int oracle_subtree_grad(int32_t n, int64_t m, const double* dist, const int32_t* pred, const int32_t* pred_edge,
                        const double* upstream, double* grad_w);
int oracle_kcore(int32_t n, const int64_t* row_ptr, const int32_t* col, int32_t* core);
}

namespace {

struct G {
  int32_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col, w;
};

G take(gg_csr* h) {
  if (!h) {
    std::fprintf(stderr, "generator returned null\n");
    std::exit(2);
  }
  G g;
  g.n = gg_n(h);
  const int64_t m = gg_m(h);
  g.rp.resize((size_t)g.n + 1);
  g.col.resize((size_t)(m > 0 ? m : 1));
  g.w.resize((size_t)(m > 0 ? m : 1));
  gg_copy(h, g.rp.data(), g.col.data(), g.w.data());
  g.col.resize((size_t)m);
  g.w.resize((size_t)m);
  gg_free(h);
  return g;
}

int fails = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++fails;
  }
}

void exercise(const G& g, const char* name, bool small) {
  const int32_t n = g.n;
  const int64_t m = (int64_t)g.col.size();
  int64_t pick[2];
  gg_uniform(7, 101, 2, (uint64_t)n, pick);
  const int32_t src = (int32_t)pick[0], dst = (int32_t)pick[1];
  std::vector<int64_t> d((size_t)n), bf((size_t)n);
  expect(oracle_dijkstra(n, g.rp.data(), g.col.data(), g.w.data(), src, d.data()) == 0, "dijkstra");
  if (small) {
    expect(oracle_bellman_ford(n, g.rp.data(), g.col.data(), g.w.data(), src, bf.data()) >= 0, "bellman-ford");
    expect(d == bf, "dijkstra == bellman-ford");
  }
  std::vector<uint8_t> reach((size_t)n);
  expect(oracle_bfs_reach(n, g.rp.data(), g.col.data(), src, reach.data()) == 0, "bfs");
  std::vector<int32_t> pred((size_t)n), d32((size_t)n);
  expect(oracle_canonical_pred(n, g.rp.data(), g.col.data(), g.w.data(), src, d.data(), pred.data()) == 0, "pred");
  expect(oracle_to_i32(n, d.data(), d32.data()) == 0, "no overflow");
  expect(oracle_check(n, g.rp.data(), g.col.data(), g.w.data(), src, d32.data(), pred.data()) == 0, "certificate");
  const int64_t pp = oracle_ppsp(n, g.rp.data(), g.col.data(), g.w.data(), src, dst);
  const int64_t want = d32[dst] == INT32_MAX ? -1 : (int64_t)d32[dst];
  expect(pp == want, "ppsp == dijkstra");
  std::vector<int32_t> h0((size_t)n, 0);
  int64_t expanded = 0;
  expect(oracle_astar(n, g.rp.data(), g.col.data(), g.w.data(), src, dst, h0.data(), &expanded) == want,
         "astar(h=0) == dijkstra");
  // real-valued paths: weights as floats, then the tree and its gradient
  std::vector<float> wf((size_t)m);
  for (int64_t e = 0; e < m; ++e) wf[(size_t)e] = (float)g.w[(size_t)e] + 0.25f;
  std::vector<double> d64((size_t)n), d32f((size_t)n);
  expect(oracle_dijkstra_f64(n, g.rp.data(), g.col.data(), wf.data(), src, d64.data()) == 0, "f64");
  expect(oracle_dijkstra_f32(n, g.rp.data(), g.col.data(), wf.data(), src, d32f.data()) == 0, "f32");
  std::vector<int32_t> tp((size_t)n), te((size_t)n);
  expect(oracle_tree_real(n, g.rp.data(), g.col.data(), wf.data(), src, d64.data(), 0, tp.data(), te.data()) == 0,
         "tree");
  std::vector<double> up((size_t)n, 1.0), gw((size_t)(m > 0 ? m : 1));
  expect(oracle_subtree_grad(n, m, d64.data(), tp.data(), te.data(), up.data(), gw.data()) == 0, "subtree grad");
  std::vector<int32_t> core((size_t)n);
  expect(oracle_kcore(n, g.rp.data(), g.col.data(), core.data()) == 0, "kcore");
  std::printf("%s: n=%d m=%lld src=%d dist[dst]=%lld ok\n", name, n, (long long)m, src, (long long)want);
}

}  // namespace

int main() {
  exercise(take(gg_grid(12, 9, 1, 100, 0)), "grid 12x9", true);
  exercise(take(gg_road(48, 0.75, 0.001, 64, 0)), "road 48", true);
  exercise(take(gg_road(256, 0.75, 0.001, 64, 0)), "road 256", false);
  exercise(take(gg_rmat(10, 16, 0.57, 0.19, 0.19, 1, 1000, 0)), "rmat 10", false);
  std::vector<int32_t> xs(3000), ys(3000);
  exercise(take(gg_rgg(3000, 6.0, 5, xs.data(), ys.data())), "rgg 3000", false);
  std::vector<int32_t> h(64 * 64);
  gg_grid_heuristic(64, 100, h.data());
  expect(h[100] == 0 && h[0] == (int32_t)std::floor(10.0 * std::sqrt(1.0 + 36.0 * 36.0)), "heuristic");
  if (fails) return 1;
  std::printf("sanitized run ok\n");
  return 0;
}
