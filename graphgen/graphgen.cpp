// Seeded synthetic graph generators (host C++, OpenMP).
//
// This module only produces inputs: directed CSR graphs (rows sorted by
// destination, no self-loops, no duplicate edges) and per-vertex A*
// heuristics.  It holds none of the shortest-path arithmetic; both the CPU
// oracle's tests and the GPU path's tests and benchmark draw their inputs
// from here.
//
// Randomness is counter-based: every value is a pure function of
// (seed, stream, index) through SplitMix64, so generation is deterministic
// for any thread count.
//
//   sm64(x)           : SplitMix64 finaliser (Steele, Lea, Flood 2014)
//   draw(seed,st,i)   = sm64(sm64(sm64(seed) + st) + i)
//   u01(x)            = (x >> 11) * 2^-53                       in [0,1)
//   uint_below(x, k)  = ((x >> 32) * k) >> 32                   in [0,k)
//
// Generators
//   gg_grid : R x C 4-neighbour grid, every edge kept, int weights
//             uniform in [wlo, whi) per undirected edge.
//   gg_road : side x side 4-neighbour grid, each undirected edge kept with
//             probability p; weight llround(10 * len * U(1,2)); plus
//             round(lr_frac * kept) long-range undirected edges to a partner
//             within Chebyshev distance lr_radius (unit grid steps and
//             off-grid partners are re-drawn), weight
//             max(llround(10 * len * U(1,2)), ceil(10 * len)), so that the
//             heuristic floor(10 * euclid) is consistent.
//   gg_rmat : Graph500-style R-MAT (no noise), 2^scale vertices,
//             edge_factor * 2^scale draws, random vertex relabelling,
//             self-loops dropped, symmetrised and deduplicated; int weight
//             uniform in [wlo, whi) per undirected pair.
//   gg_rgg  : random geometric graph, integer coordinates in [0, 2^20)^2,
//             radius for a requested mean degree, weight
//             max(1, llround(euclid length)).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t sm64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}
inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t i) {
  return sm64(sm64(sm64(seed) + stream) + i);
}
inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
inline uint64_t uint_below(uint64_t x, uint64_t k) { return ((x >> 32) * k) >> 32; }
inline int32_t uniform_int(uint64_t x, int32_t lo, int32_t hi) {
  return lo + (int32_t)uint_below(x, (uint64_t)(hi - lo));
}

// Random streams (documented draw order).
enum : uint64_t {
  S_KEEP = 1,   // grid edge kept?            index: grid edge id
  S_W = 2,      // grid edge weight           index: grid edge id
  S_LR_V = 3,   // long-range anchor vertex   index: j*1024 + attempt
  S_LR_D = 4,   // long-range offset          index: j*1024 + attempt
  S_LR_W = 5,   // long-range weight          index: lo*n + hi
  S_RMAT = 6,   // R-MAT quadrant choices     index: draw*8 + k
  S_PERM = 7,   // R-MAT relabelling          index: Fisher-Yates step
  S_RMAT_W = 8, // R-MAT weight               index: lo*n + hi
  S_RGG_X = 9,  // RGG x coordinate           index: vertex
  S_RGG_Y = 10, // RGG y coordinate           index: vertex
};

struct Csr {
  int32_t n;
  int64_t m;
  int64_t* row_ptr;
  int32_t* col;
  int32_t* w;
};

// Builds a CSR from per-row packed (dst << 32 | weight) entries that were
// scattered into rows unsorted: sorts each row by destination, drops
// duplicates (keeping the smallest weight, so the result does not depend on
// scatter order) and compacts.
Csr* finish_rows(int32_t n, std::vector<int64_t>& start, std::vector<uint64_t>& packed) {
  std::vector<int64_t> keep(n);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; ++v) {
    uint64_t* b = packed.data() + start[v];
    uint64_t* e = packed.data() + start[v + 1];
    std::sort(b, e);
    int64_t k = 0;
    for (uint64_t* p = b; p < e; ++p) {
      if (k > 0 && (b[k - 1] >> 32) == (*p >> 32)) continue;  // same dst: first (min weight) wins
      b[k++] = *p;
    }
    keep[v] = k;
  }
  Csr* g = (Csr*)std::calloc(1, sizeof(Csr));
  g->n = n;
  g->row_ptr = (int64_t*)std::malloc(sizeof(int64_t) * ((size_t)n + 1));
  g->row_ptr[0] = 0;
  for (int32_t v = 0; v < n; ++v) g->row_ptr[v + 1] = g->row_ptr[v] + keep[v];
  g->m = g->row_ptr[n];
  g->col = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(g->m, 1));
  g->w = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(g->m, 1));
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; ++v) {
    const uint64_t* b = packed.data() + start[v];
    int64_t o = g->row_ptr[v];
    for (int64_t k = 0; k < keep[v]; ++k) {
      g->col[o + k] = (int32_t)(b[k] >> 32);
      g->w[o + k] = (int32_t)(uint32_t)(b[k] & 0xffffffffULL);
    }
  }
  return g;
}

inline uint64_t pack(int32_t dst, int32_t w) {
  return ((uint64_t)(uint32_t)dst << 32) | (uint64_t)(uint32_t)w;
}

// Undirected edge lists -> symmetric CSR.
Csr* build_symmetric(int32_t n, const std::vector<int32_t>& a, const std::vector<int32_t>& b,
                     const std::vector<int32_t>& w) {
  const size_t E = a.size();
  std::vector<std::atomic<int64_t>> deg(n);
  for (int32_t v = 0; v < n; ++v) deg[v].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (size_t i = 0; i < E; ++i) {
    if (a[i] == b[i]) continue;
    deg[a[i]].fetch_add(1, std::memory_order_relaxed);
    deg[b[i]].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> start((size_t)n + 1);
  start[0] = 0;
  for (int32_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v].load(std::memory_order_relaxed);
  std::vector<std::atomic<int64_t>> cur(n);
  for (int32_t v = 0; v < n; ++v) cur[v].store(start[v], std::memory_order_relaxed);
  std::vector<uint64_t> packed((size_t)start[n]);
#pragma omp parallel for schedule(static)
  for (size_t i = 0; i < E; ++i) {
    if (a[i] == b[i]) continue;
    packed[cur[a[i]].fetch_add(1, std::memory_order_relaxed)] = pack(b[i], w[i]);
    packed[cur[b[i]].fetch_add(1, std::memory_order_relaxed)] = pack(a[i], w[i]);
  }
  return finish_rows(n, start, packed);
}

}  // namespace

extern "C" {

typedef Csr gg_csr;

int32_t gg_n(const gg_csr* g) { return g->n; }
int64_t gg_m(const gg_csr* g) { return g->m; }

// Copies the CSR arrays out (caller-owned buffers of n+1, m and m entries).
void gg_copy(const gg_csr* g, int64_t* row_ptr, int32_t* col, int32_t* w) {
  std::memcpy(row_ptr, g->row_ptr, sizeof(int64_t) * ((size_t)g->n + 1));
  if (g->m > 0) {
    std::memcpy(col, g->col, sizeof(int32_t) * (size_t)g->m);
    std::memcpy(w, g->w, sizeof(int32_t) * (size_t)g->m);
  }
}

void gg_free(gg_csr* g) {
  if (!g) return;
  std::free(g->row_ptr);
  std::free(g->col);
  std::free(g->w);
  std::free(g);
}

// Full R x C 4-neighbour grid.  Vertex (r, c) has id r*C + c.  Undirected
// edge ids: horizontal (r,c)-(r,c+1) -> r*(C-1)+c, then vertical
// (r,c)-(r+1,c) -> R*(C-1) + r*C + c.  Weight uniform in [wlo, whi).
gg_csr* gg_grid(int32_t R, int32_t C, int32_t wlo, int32_t whi, uint64_t seed) {
  if (R <= 0 || C <= 0 || whi <= wlo) return nullptr;
  const int64_t H = (int64_t)R * (C - 1), V = (int64_t)(R - 1) * C;
  std::vector<int32_t> a(H + V), b(H + V), w(H + V);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < H + V; ++e) {
    int32_t r, c, r2, c2;
    if (e < H) { r = (int32_t)(e / (C - 1)); c = (int32_t)(e % (C - 1)); r2 = r; c2 = c + 1; }
    else { int64_t f = e - H; r = (int32_t)(f / C); c = (int32_t)(f % C); r2 = r + 1; c2 = c; }
    a[e] = r * C + c;
    b[e] = r2 * C + c2;
    w[e] = uniform_int(draw(seed, S_W, (uint64_t)e), wlo, whi);
  }
  return build_symmetric(R * C, a, b, w);
}

// Road-like percolated grid with long-range shortcuts (see file header).
gg_csr* gg_road(int32_t side, double p_keep, double lr_frac, int32_t lr_radius, uint64_t seed) {
  if (side < 2 || lr_radius < 1) return nullptr;
  const int64_t S = side;
  const int64_t n = S * S;
  if (n > INT32_MAX) return nullptr;
  const int64_t H = S * (S - 1), Vt = (S - 1) * S, G = H + Vt;
  std::vector<uint8_t> kept(G);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < G; ++e) kept[e] = u01(draw(seed, S_KEEP, (uint64_t)e)) < p_keep;
  int64_t nk = 0;
  for (int64_t e = 0; e < G; ++e) nk += kept[e];
  const int64_t L = std::llround(lr_frac * (double)nk);
  std::vector<int32_t> a(nk + L), b(nk + L), w(nk + L);
  // Compact kept grid edges in edge-id order.
  std::vector<int64_t> slot(G);
  int64_t k = 0;
  for (int64_t e = 0; e < G; ++e) { slot[e] = k; k += kept[e]; }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < G; ++e) {
    if (!kept[e]) continue;
    int64_t r, c, r2, c2;
    if (e < H) { r = e / (S - 1); c = e % (S - 1); r2 = r; c2 = c + 1; }
    else { int64_t f = e - H; r = f / S; c = f % S; r2 = r + 1; c2 = c; }
    const int64_t i = slot[e];
    a[i] = (int32_t)(r * S + c);
    b[i] = (int32_t)(r2 * S + c2);
    w[i] = (int32_t)std::llround(10.0 * 1.0 * (1.0 + u01(draw(seed, S_W, (uint64_t)e))));
  }
  const int64_t span = 2 * (int64_t)lr_radius + 1;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < L; ++j) {
    for (int64_t att = 0;; ++att) {
      const uint64_t key = (uint64_t)j * 1024 + (uint64_t)att;
      const int64_t v0 = (int64_t)uint_below(draw(seed, S_LR_V, key), (uint64_t)n);
      const uint64_t d = draw(seed, S_LR_D, key);
      const int64_t dx = (int64_t)uint_below(d, (uint64_t)span) - lr_radius;
      const int64_t dy = (int64_t)uint_below(d << 32, (uint64_t)span) - lr_radius;
      const int64_t r0 = v0 / S, c0 = v0 % S, r1 = r0 + dy, c1 = c0 + dx;
      if (std::llabs(dx) + std::llabs(dy) <= 1) continue;          // no self-loops or grid steps
      if (r1 < 0 || r1 >= S || c1 < 0 || c1 >= S) continue;        // stays on the grid
      const int64_t v1 = r1 * S + c1;
      const int64_t lo = std::min(v0, v1), hi = std::max(v0, v1);
      const double len = std::sqrt((double)(dx * dx + dy * dy));
      const double u = 1.0 + u01(draw(seed, S_LR_W, (uint64_t)lo * (uint64_t)n + (uint64_t)hi));
      int64_t wt = std::llround(10.0 * len * u);
      const int64_t floor_w = (int64_t)std::ceil(10.0 * len);
      if (wt < floor_w) wt = floor_w;
      a[nk + j] = (int32_t)lo;
      b[nk + j] = (int32_t)hi;
      w[nk + j] = (int32_t)wt;
      break;
    }
  }
  return build_symmetric((int32_t)n, a, b, w);
}

// Graph500-style R-MAT.  Each of edge_factor * 2^scale draws picks one of
// four quadrants per level with probabilities (a, b, c, 1-a-b-c), high bit
// first, using one 16-bit uniform per level.  Vertex ids are then relabelled
// by a seeded Fisher-Yates permutation.
gg_csr* gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, int32_t wlo,
                int32_t whi, uint64_t seed) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || whi <= wlo) return nullptr;
  const int64_t n = (int64_t)1 << scale;
  const int64_t D = (int64_t)edge_factor * n;
  std::vector<int32_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    const int64_t j = (int64_t)uint_below(draw(seed, S_PERM, (uint64_t)i), (uint64_t)(i + 1));
    std::swap(perm[i], perm[j]);
  }
  const uint32_t ta = (uint32_t)std::llround(a * 65536.0);
  const uint32_t tb = (uint32_t)std::llround((a + b) * 65536.0);
  const uint32_t tc = (uint32_t)std::llround((a + b + c) * 65536.0);
  auto edge = [&](int64_t i, int32_t& u, int32_t& v) {
    uint32_t su = 0, sv = 0;
    uint64_t bits = 0;
    for (int32_t lvl = 0; lvl < scale; ++lvl) {
      if ((lvl & 3) == 0) bits = draw(seed, S_RMAT, (uint64_t)i * 8 + (uint64_t)(lvl >> 2));
      const uint32_t r = (uint32_t)(bits & 0xffff);
      bits >>= 16;
      const uint32_t bit = 1u << (scale - 1 - lvl);
      if (r < ta) {
      } else if (r < tb) {
        sv |= bit;
      } else if (r < tc) {
        su |= bit;
      } else {
        su |= bit;
        sv |= bit;
      }
    }
    u = perm[su];
    v = perm[sv];
  };
  std::vector<std::atomic<int64_t>> deg(n);
  for (int64_t v = 0; v < n; ++v) deg[v].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < D; ++i) {
    int32_t u, v;
    edge(i, u, v);
    if (u == v) continue;
    deg[u].fetch_add(1, std::memory_order_relaxed);
    deg[v].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> start((size_t)n + 1);
  start[0] = 0;
  for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v].load(std::memory_order_relaxed);
  std::vector<std::atomic<int64_t>> cur(n);
  for (int64_t v = 0; v < n; ++v) cur[v].store(start[v], std::memory_order_relaxed);
  std::vector<uint64_t> packed((size_t)start[n]);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < D; ++i) {
    int32_t u, v;
    edge(i, u, v);
    if (u == v) continue;
    const int64_t lo = std::min(u, v), hi = std::max(u, v);
    const int32_t wt = uniform_int(draw(seed, S_RMAT_W, (uint64_t)lo * (uint64_t)n + (uint64_t)hi), wlo, whi);
    packed[cur[u].fetch_add(1, std::memory_order_relaxed)] = pack(v, wt);
    packed[cur[v].fetch_add(1, std::memory_order_relaxed)] = pack(u, wt);
  }
  return finish_rows((int32_t)n, start, packed);
}

// Random geometric graph on n points with integer coordinates in
// [0, 2^20)^2; u and v are joined when their Euclidean distance is at most
// r = 2^20 * sqrt(mean_degree / (n * pi)).  Weight max(1, llround(len)).
// Points are bucketed on a square cell grid of side >= r.
gg_csr* gg_rgg(int32_t n, double mean_degree, uint64_t seed, int32_t* xs, int32_t* ys) {
  if (n < 1 || mean_degree <= 0) return nullptr;
  const double side = 1048576.0;
  const double r = side * std::sqrt(mean_degree / ((double)n * M_PI));
  std::vector<int32_t> x(n), y(n);
  for (int32_t i = 0; i < n; ++i) {
    x[i] = (int32_t)uint_below(draw(seed, S_RGG_X, (uint64_t)i), 1u << 20);
    y[i] = (int32_t)uint_below(draw(seed, S_RGG_Y, (uint64_t)i), 1u << 20);
  }
  if (xs) std::memcpy(xs, x.data(), sizeof(int32_t) * n);
  if (ys) std::memcpy(ys, y.data(), sizeof(int32_t) * n);
  int64_t cells = std::max<int64_t>(1, (int64_t)(side / std::max(r, 1.0)));
  if (cells > 4096) cells = 4096;
  const double cw = side / (double)cells;
  std::vector<std::vector<int32_t>> bucket((size_t)(cells * cells));
  for (int32_t i = 0; i < n; ++i) {
    int64_t cx = std::min<int64_t>(cells - 1, (int64_t)(x[i] / cw));
    int64_t cy = std::min<int64_t>(cells - 1, (int64_t)(y[i] / cw));
    bucket[(size_t)(cy * cells + cx)].push_back(i);
  }
  std::vector<int32_t> ea, eb, ew;
  const double r2 = r * r;
  for (int32_t i = 0; i < n; ++i) {
    int64_t cx = std::min<int64_t>(cells - 1, (int64_t)(x[i] / cw));
    int64_t cy = std::min<int64_t>(cells - 1, (int64_t)(y[i] / cw));
    for (int64_t yy = std::max<int64_t>(0, cy - 1); yy <= std::min<int64_t>(cells - 1, cy + 1); ++yy)
      for (int64_t xx = std::max<int64_t>(0, cx - 1); xx <= std::min<int64_t>(cells - 1, cx + 1); ++xx)
        for (int32_t j : bucket[(size_t)(yy * cells + xx)]) {
          if (j <= i) continue;
          const double dx = (double)x[i] - x[j], dy = (double)y[i] - y[j];
          const double d2 = dx * dx + dy * dy;
          if (d2 > r2) continue;
          ea.push_back(i);
          eb.push_back(j);
          ew.push_back((int32_t)std::max<int64_t>(1, std::llround(std::sqrt(d2))));
        }
  }
  return build_symmetric(n, ea, eb, ew);
}

// A* heuristic on a side x side grid graph with vertex (r, c) at id
// r*side + c: h[v] = floor(10 * euclid(v, target)).
void gg_grid_heuristic(int32_t side, int32_t target, int32_t* h) {
  const int64_t S = side, n = S * S;
  const int64_t rt = target / S, ct = target % S;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    const double dr = (double)(v / S - rt), dc = (double)(v % S - ct);
    h[v] = (int32_t)std::floor(10.0 * std::sqrt(dr * dr + dc * dc));
  }
}

// Uniform draws in [0, k) for picking sources / targets: out[i] =
// uint_below(draw(seed, stream, i), k).
void gg_uniform(uint64_t seed, uint64_t stream, int64_t count, uint64_t k, int64_t* out) {
  for (int64_t i = 0; i < count; ++i) out[i] = (int64_t)uint_below(draw(seed, stream, (uint64_t)i), k);
}

}  // extern "C"
