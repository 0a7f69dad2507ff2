/*
 * CPU oracle for bucketed shortest-path processing -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU product path never links, loads or calls
 * it, and it shares no code, header, table or helper with that path.
 *
 * What is computed.  The paper's Delta-stepping (section 3, Figures
 * "lazy bucket update", "eager bucket update" and "eager bucket update with
 * bucket fusion") is an ordered label-correcting method: whatever Delta,
 * bucket-update strategy or fusion threshold is chosen, it terminates with
 * the single-source shortest-path distances
 *
 *     dist[v] = min over paths s -> v of (sum of edge weights)
 *
 * (section 2: priority coarsening p' = floor(p / Delta) only trades
 * work-efficiency for parallelism; section 3.3: fusing rounds of the same
 * bucket never processes a bucket out of priority order).  The result has
 * this plain definition, so the oracle is that definition computed by
 * textbook binary-heap Dijkstra in 64-bit integers.  Unreachable vertices
 * get INF; the int32 form uses INT32_MAX, the value the paper's programs
 * initialise distances to (Figure "Delta-stepping in GraphIt", dist
 * initialisation to INT_MAX).
 *
 * Variants (section 6.1):
 *   - wBFS: Delta-stepping with Delta = 1 on positive integer weights; the
 *     result is the same shortest-path definition.
 *   - PPSP: s, d -> shortest distance from s to d (Dijkstra stopped when d is
 *     settled).
 *   - A*: s, d and a per-vertex estimate h; with an admissible h the result
 *     is again the s-d shortest distance (textbook A* with re-opening).
 *
 *   - Lazy bucket update (Figure "lazy bucket update"): the same
 *     distances; only the bucket bookkeeping differs.
 *   - k-core (section 6.1): coreness of every vertex, by peeling.
 *
 * Predecessors are not discussed in the paper.  The reading used here is
 * the canonical one: pred[v] = smallest u with an edge (u,v) such that
 * dist[u] is finite and dist[u] + w(u,v) == dist[v]; pred[s] = s; -1 when
 * v is unreachable.
 *
 * Pins (tests marked "not gpu"): Bellman-Ford brute force and exhaustive
 * path enumeration on tiny graphs, scipy's independent Dijkstra, closed
 * forms on uniform grids and paths, a hand-worked 3x3 grid fixture, and the
 * certificate checker below on every generated workload.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_INF INT64_MAX
#define I32_INF 2147483647

#ifndef ORACLE_MUTATION
#define ORACLE_MUTATION 0 /* a planted bug, selected only by the pin tests */
#endif

/* ---------------- binary min-heap of (key, vertex) ---------------- */
typedef struct {
  int64_t* key;
  int32_t* vid;
  int64_t size, cap;
} heap_t;

static int heap_init(heap_t* h, int64_t cap) {
  h->key = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
  h->vid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
  h->size = 0;
  h->cap = cap > 0 ? cap : 1;
  return h->key && h->vid;
}
static void heap_free(heap_t* h) { free(h->key); free(h->vid); }

static int heap_push(heap_t* h, int64_t k, int32_t v) {
  if (h->size == h->cap) {
    int64_t nc = h->cap * 2;
    int64_t* nk = (int64_t*)realloc(h->key, sizeof(int64_t) * (size_t)nc);
    if (!nk) return 0;
    h->key = nk;
    int32_t* nv = (int32_t*)realloc(h->vid, sizeof(int32_t) * (size_t)nc);
    if (!nv) return 0;
    h->vid = nv;
    h->cap = nc;
  }
  int64_t i = h->size++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->key[p] <= k) break;
    h->key[i] = h->key[p];
    h->vid[i] = h->vid[p];
    i = p;
  }
  h->key[i] = k;
  h->vid[i] = v;
  return 1;
}

static void heap_pop(heap_t* h, int64_t* k, int32_t* v) {
  *k = h->key[0];
  *v = h->vid[0];
  int64_t lk = h->key[--h->size];
  int32_t lv = h->vid[h->size];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->size) break;
    if (c + 1 < h->size && h->key[c + 1] < h->key[c]) c++;
    if (h->key[c] >= lk) break;
    h->key[i] = h->key[c];
    h->vid[i] = h->vid[c];
    i = c;
  }
  h->key[i] = lk;
  h->vid[i] = lv;
}

/* Dijkstra from src, stopping early once `stop` (if >= 0) is settled.
 * dist: int64[n], ORACLE_INF = unreachable (or not settled before stop).
 * Returns 0, or -1 on allocation failure / bad arguments. */
static int dijkstra_impl(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                         int32_t src, int32_t stop, int64_t* dist) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  for (int32_t v = 0; v < n; ++v) dist[v] = ORACLE_INF;
  heap_t h;
  if (!heap_init(&h, 1024)) return -1;
  dist[src] = 0;
  heap_push(&h, 0, src);
  while (h.size > 0) {
    int64_t d;
    int32_t u;
    heap_pop(&h, &d, &u);
    if (d > dist[u]) continue; /* lazy deletion of superseded entries */
    if (u == stop) break;
#if ORACLE_MUTATION == 3
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1] - 1; ++e) { /* planted: last edge skipped */
#else
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
#endif
      int32_t v = col[e];
#if ORACLE_MUTATION == 1
      int64_t nd = d; /* planted: dropped weight term */
#elif ORACLE_MUTATION == 2
      int64_t nd = d + (int64_t)w[row_ptr[u]]; /* planted: wrong edge index */
#else
      int64_t nd = d + (int64_t)w[e];
#endif
      if (nd < dist[v]) {
        dist[v] = nd;
        if (!heap_push(&h, nd, v)) { heap_free(&h); return -1; }
      }
    }
  }
  heap_free(&h);
  return 0;
}

/* Single-source shortest paths (the definition above).  int64 distances,
 * ORACLE_INF for unreachable vertices. */
int oracle_dijkstra(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                    int32_t src, int64_t* dist) {
  return dijkstra_impl(n, row_ptr, col, w, src, -1, dist);
}

/* Bellman-Ford brute force (n-1 full passes, early exit when a pass
 * changes nothing): the unordered baseline the paper compares against
 * (section 1), used here only to pin Dijkstra on tiny graphs.
 * Returns the number of passes, or -1 on bad arguments. */
int oracle_bellman_ford(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                        int32_t src, int64_t* dist) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  for (int32_t v = 0; v < n; ++v) dist[v] = ORACLE_INF;
  dist[src] = 0;
  int passes = 0;
  for (int32_t it = 0; it < n; ++it) {
    int changed = 0;
    ++passes;
    for (int32_t u = 0; u < n; ++u) {
      if (dist[u] == ORACLE_INF) continue;
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        int64_t nd = dist[u] + (int64_t)w[e];
        if (nd < dist[col[e]]) { dist[col[e]] = nd; changed = 1; }
      }
    }
    if (!changed) break;
  }
  return passes;
}

/* Unweighted reachability from src (breadth-first).  reached: uint8[n]. */
int oracle_bfs_reach(int32_t n, const int64_t* row_ptr, const int32_t* col, int32_t src,
                     uint8_t* reached) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!q) return -1;
  memset(reached, 0, (size_t)n);
  int64_t qh = 0, qt = 0;
  q[qt++] = src;
  reached[src] = 1;
  while (qh < qt) {
    int32_t u = q[qh++];
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      if (!reached[v]) { reached[v] = 1; q[qt++] = v; }
    }
  }
  free(q);
  return 0;
}

/* Canonical predecessors from exact distances: pred[v] = min u over edges
 * (u,v) with dist[u] finite and dist[u] + w == dist[v]; pred[src] = src;
 * -1 where no such u exists. */
int oracle_canonical_pred(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                          int32_t src, const int64_t* dist, int32_t* pred) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  for (int32_t v = 0; v < n; ++v) pred[v] = -1;
  for (int32_t u = 0; u < n; ++u) {
    if (dist[u] == ORACLE_INF) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      if (v == src) continue;
#if ORACLE_MUTATION == 4
      if (dist[v] != ORACLE_INF && dist[u] + (int64_t)w[e] == dist[v] && (pred[v] < 0 || u > pred[v]))
#else
      if (dist[v] != ORACLE_INF && dist[u] + (int64_t)w[e] == dist[v] && (pred[v] < 0 || u < pred[v]))
#endif
        pred[v] = u;
    }
  }
  pred[src] = src;
  return 0;
}

/* int64 distances -> int32 with INF = INT32_MAX.  Returns the number of
 * finite distances that do not fit below INT32_MAX (the int32 overflow
 * condition), which are written as INT32_MAX. */
int64_t oracle_to_i32(int32_t n, const int64_t* d64, int32_t* d32) {
  int64_t over = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (d64[v] == ORACLE_INF) d32[v] = I32_INF;
    else if (d64[v] >= (int64_t)I32_INF) { d32[v] = I32_INF; ++over; }
    else d32[v] = (int32_t)d64[v];
  }
  return over;
}

/* Point-to-point shortest path (section 6.1, PPSP): distance from src to
 * dst, or -1 if dst is unreachable. */
int64_t oracle_ppsp(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                    int32_t src, int32_t dst) {
  if (dst < 0 || dst >= n) return -2;
  int64_t* dist = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!dist) return -2;
  int rc = dijkstra_impl(n, row_ptr, col, w, src, dst, dist);
  int64_t r = rc ? -2 : (dist[dst] == ORACLE_INF ? -1 : dist[dst]);
  free(dist);
  return r;
}

/* Textbook A* (section 6.1, A*): a heap ordered by g + h with re-opening of
 * vertices whose g improves; stops when dst is popped.  With an admissible
 * h (h never exceeds the true remaining distance, h[dst] = 0) the returned
 * g(dst) is the shortest s-d distance.  Returns -1 if unreachable.
 * expanded (nullable) receives the number of heap pops that expanded a
 * vertex. */
int64_t oracle_astar(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                     int32_t src, int32_t dst, const int32_t* hh, int64_t* expanded) {
  if (n <= 0 || src < 0 || src >= n || dst < 0 || dst >= n) return -2;
  int64_t* g = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  heap_t h;
  if (!g || !heap_init(&h, 1024)) { free(g); return -2; }
  for (int32_t v = 0; v < n; ++v) g[v] = ORACLE_INF;
  g[src] = 0;
  heap_push(&h, (int64_t)hh[src], src);
  int64_t result = -1, pops = 0;
  while (h.size > 0) {
    int64_t f;
    int32_t u;
    heap_pop(&h, &f, &u);
    if (f > g[u] + (int64_t)hh[u]) continue; /* superseded entry */
    if (u == dst) { result = g[u]; break; }
    ++pops;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      int64_t ng = g[u] + (int64_t)w[e];
      if (ng < g[v]) {
        g[v] = ng;
        if (!heap_push(&h, ng + (int64_t)hh[v], v)) { result = -2; break; }
      }
    }
    if (result == -2) break;
  }
  if (expanded) *expanded = pops;
  heap_free(&h);
  free(g);
  return result;
}

/* Certificate checker for an int32 result (dist, and pred if non-NULL).
 * Together these invariants certify that dist equals the shortest-path
 * distances for non-negative weights:
 *   bit 0  dist[src] != 0
 *   bit 1  an edge (u,v) with dist[u] finite and dist[v] > dist[u] + w
 *   bit 2  dist[v] negative
 *   bit 3  dist finite on a vertex unreachable from src, or INF on a
 *          reachable one
 *   bit 4  pred[src] != src
 *   bit 5  pred[v] == -1 for a reachable v != src
 *   bit 6  pred[v] != -1 for an unreachable v
 *   bit 7  pred[v] = u but no edge (u,v) with dist[u] + w == dist[v]
 *   bit 8  following pred from some vertex does not reach src (a cycle)
 *   bit 9  pred out of range
 * Returns the OR of violated bits (0 = certified). */
uint32_t oracle_check(int32_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* w,
                      int32_t src, const int32_t* dist, const int32_t* pred) {
  uint32_t bad = 0;
  if (n <= 0 || src < 0 || src >= n) return 0xffffffffu;
  if (dist[src] != 0) bad |= 1u << 0;
  for (int32_t u = 0; u < n; ++u) {
    if (dist[u] < 0) bad |= 1u << 2;
    if (dist[u] == I32_INF) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int64_t nd = (int64_t)dist[u] + (int64_t)w[e];
      int32_t v = col[e];
      int64_t dv = dist[v] == I32_INF ? ORACLE_INF : (int64_t)dist[v];
      if (dv > nd) bad |= 1u << 1;
    }
  }
  uint8_t* reached = (uint8_t*)malloc((size_t)n);
  if (!reached) return 0xffffffffu;
  oracle_bfs_reach(n, row_ptr, col, src, reached);
  for (int32_t v = 0; v < n; ++v)
    if ((dist[v] != I32_INF) != (reached[v] != 0)) bad |= 1u << 3;
  if (pred) {
    if (pred[src] != src) bad |= 1u << 4;
    for (int32_t v = 0; v < n; ++v) {
      if (v == src) continue;
      int32_t p = pred[v];
      if (dist[v] == I32_INF) { if (p != -1) bad |= 1u << 6; continue; }
      if (p == -1) { bad |= 1u << 5; continue; }
      if (p < 0 || p >= n) { bad |= 1u << 9; continue; }
      int tight = 0;
      if (dist[p] != I32_INF)
        for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e)
          if (col[e] == v && (int64_t)dist[p] + (int64_t)w[e] == (int64_t)dist[v]) tight = 1;
      if (!tight) bad |= 1u << 7;
    }
    if (!(bad & ((1u << 9) | (1u << 4)))) {
      /* rootedness: every reachable vertex's pred chain ends at src.
       * state: 0 unknown, 1 on current walk, 2 reaches src. */
      uint8_t* st = reached; /* reuse */
      memset(st, 0, (size_t)n);
      st[src] = 2;
      int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
      if (!stack) { free(reached); return 0xffffffffu; }
      for (int32_t v = 0; v < n && !(bad & (1u << 8)); ++v) {
        if (st[v] || pred[v] < 0) continue;
        int64_t top = 0;
        int32_t x = v;
        while (x >= 0 && st[x] == 0) { st[x] = 1; stack[top++] = x; x = pred[x]; }
        if (x < 0 || st[x] == 1) bad |= 1u << 8;
        while (top > 0) st[stack[--top]] = 2;
      }
      free(stack);
    }
  }
  free(reached);
  return bad;
}

/* ---------------- real-valued weights (differentiable variant) ----------
 * Weights are float32 values w >= 0.  Two oracles:
 *
 *  - oracle_dijkstra_f64: shortest distances in float64.  Every float32
 *    weight has a 24-bit significand, and for weights in [2^-14, 2^10) and
 *    distances below 2^30 every partial sum is a multiple of 2^-37 below
 *    2^30, i.e. fits in 67 bits -- so beyond 2^53 the sums can round; for
 *    the workloads used here (weights in (1, 1000), distances below 2^22,
 *    ulp multiples of 2^-23) every sum is exact, and the result is the
 *    exact real shortest distance.
 *  - oracle_dijkstra_f32: the same search with every addition rounded to
 *    float32 (d_new = fl32(d_u + w)).  Rounding is monotone, so the label
 *    at each vertex converges to the unique fixed point
 *    D(v) = min over in-edges fl32(D(u) + w), which is what any
 *    label-correcting schedule computes in float32 arithmetic.
 *
 * Tree: pred[v] = smallest u with a tight edge (D(u) + w == D(v) in the
 * arithmetic of the search); pred_edge[v] = that edge's index.  The
 * gradient of L = sum_t D(t) (t over targets, with multiplicity) with
 * respect to w_e is the number of targets in the subtree below e
 * (unique shortest paths), computed by oracle_subtree_counts. */
typedef struct {
  double* key;
  int32_t* vid;
  int64_t size, cap;
} dheap_t;

static int dheap_push(dheap_t* h, double k, int32_t v) {
  if (h->size == h->cap) {
    int64_t nc = h->cap ? h->cap * 2 : 1024;
    double* nk = (double*)realloc(h->key, sizeof(double) * (size_t)nc);
    if (!nk) return 0;
    h->key = nk;
    int32_t* nv = (int32_t*)realloc(h->vid, sizeof(int32_t) * (size_t)nc);
    if (!nv) return 0;
    h->vid = nv;
    h->cap = nc;
  }
  int64_t i = h->size++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->key[p] <= k) break;
    h->key[i] = h->key[p];
    h->vid[i] = h->vid[p];
    i = p;
  }
  h->key[i] = k;
  h->vid[i] = v;
  return 1;
}

static void dheap_pop(dheap_t* h, double* k, int32_t* v) {
  *k = h->key[0];
  *v = h->vid[0];
  double lk = h->key[--h->size];
  int32_t lv = h->vid[h->size];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->size) break;
    if (c + 1 < h->size && h->key[c + 1] < h->key[c]) c++;
    if (h->key[c] >= lk) break;
    h->key[i] = h->key[c];
    h->vid[i] = h->vid[c];
    i = c;
  }
  h->key[i] = lk;
  h->vid[i] = lv;
}

static volatile float f32_sink;
/* float32 sum, rounded once (no excess precision or contraction) */
static float add_f32(float a, float b) {
  volatile float s = a + b;
  return s;
}

static int dijkstra_real(int32_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t src,
                         int use_f32, double* dist) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  for (int32_t v = 0; v < n; ++v) dist[v] = INFINITY;
  dheap_t h = {0, 0, 0, 0};
  dist[src] = 0.0;
  if (!dheap_push(&h, 0.0, src)) return -1;
  while (h.size > 0) {
    double d;
    int32_t u;
    dheap_pop(&h, &d, &u);
    if (d > dist[u]) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      double nd = use_f32 ? (double)add_f32((float)d, w[e]) : d + (double)w[e];
      if (nd < dist[v]) {
        dist[v] = nd;
        if (!dheap_push(&h, nd, v)) { free(h.key); free(h.vid); return -1; }
      }
    }
  }
  free(h.key);
  free(h.vid);
  return 0;
}

int oracle_dijkstra_f64(int32_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t src,
                        double* dist) {
  return dijkstra_real(n, row_ptr, col, w, src, 0, dist);
}

int oracle_dijkstra_f32(int32_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t src,
                        double* dist) {
  return dijkstra_real(n, row_ptr, col, w, src, 1, dist);
}

/* Canonical tree from real distances: tightness in float32 arithmetic when
 * use_f32, exact otherwise.  pred / pred_edge = -1 where unreachable;
 * pred[src] = src, pred_edge[src] = -1. */
int oracle_tree_real(int32_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t src,
                     const double* dist, int use_f32, int32_t* pred, int32_t* pred_edge) {
  if (n <= 0 || src < 0 || src >= n) return -1;
  for (int32_t v = 0; v < n; ++v) { pred[v] = -1; pred_edge[v] = -1; }
  for (int32_t u = 0; u < n; ++u) {
    if (isinf(dist[u])) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      if (v == src || isinf(dist[v])) continue;
      double nd = use_f32 ? (double)add_f32((float)dist[u], w[e]) : dist[u] + (double)w[e];
      if (nd == dist[v] && (pred[v] < 0 || u < pred[v])) { pred[v] = u; pred_edge[v] = (int32_t)e; }
    }
  }
  pred[src] = src;
  return 0;
}

/* grad_w[e] = sum of upstream[t] over vertices t in the subtree below tree
 * edge e (0 for non-tree edges): the gradient of sum_t upstream[t] * D(t).
 * Vertices are visited in decreasing distance, so every child is done
 * before its parent. */
static const double* g_sort_key;
static int cmp_desc(const void* a, const void* b) {
  double x = g_sort_key[*(const int32_t*)a], y = g_sort_key[*(const int32_t*)b];
  return x < y ? 1 : (x > y ? -1 : 0);
}

int oracle_subtree_grad(int32_t n, int64_t m, const double* dist, const int32_t* pred, const int32_t* pred_edge,
                        const double* upstream, double* grad_w) {
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  double* acc = (double*)malloc(sizeof(double) * (size_t)n);
  if (!order || !acc) { free(order); free(acc); return -1; }
  int32_t k = 0;
  for (int32_t v = 0; v < n; ++v) {
    acc[v] = upstream[v];
    if (!isinf(dist[v])) order[k++] = v;
  }
  g_sort_key = dist;
  qsort(order, (size_t)k, sizeof(int32_t), cmp_desc);
  for (int64_t e = 0; e < m; ++e) grad_w[e] = 0.0;
  for (int32_t i = 0; i < k; ++i) {
    int32_t v = order[i];
    if (pred_edge[v] < 0) continue;
    grad_w[pred_edge[v]] = acc[v];
    acc[pred[v]] += acc[v];
  }
  free(order);
  free(acc);
  return 0;
}

/* ---------------- k-core decomposition (section 6.1, k-core) ----------------
 * coreness[v] = the largest k such that v belongs to the k-core, the
 * maximal subgraph in which every vertex keeps at least k neighbours.  The
 * paper computes it by peeling (Matula and Beck): repeatedly remove a vertex
 * of minimum remaining degree; the coreness of the removed vertex is the
 * largest minimum degree seen so far.  That is what this function does,
 * with a binary heap keyed by remaining degree (stale heap entries are
 * skipped).  The graph is given by symmetric rows: the degree of v is its
 * row length, and removing v lowers the degree of every vertex in its row.
 * Returns 0, or -1 on allocation failure / bad arguments. */
int oracle_kcore(int32_t n, const int64_t* row_ptr, const int32_t* col, int32_t* core) {
  if (n <= 0) return -1;
  int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  unsigned char* gone = (unsigned char*)calloc((size_t)n, 1);
  heap_t h;
  if (!deg || !gone || !heap_init(&h, n)) { free(deg); free(gone); return -1; }
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = row_ptr[v + 1] - row_ptr[v];
    if (!heap_push(&h, deg[v], v)) { free(deg); free(gone); heap_free(&h); return -1; }
  }
  int64_t level = 0;
  while (h.size > 0) {
    int64_t d;
    int32_t v;
    heap_pop(&h, &d, &v);
    if (gone[v] || d != deg[v]) continue; /* removed, or superseded by a lower degree */
#if ORACLE_MUTATION == 5
    level = d; /* planted: the level may go down */
#else
    if (d > level) level = d;
#endif
    core[v] = (int32_t)level;
    gone[v] = 1;
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t u = col[e];
      if (gone[u]) continue;
      deg[u] -= 1;
      if (!heap_push(&h, deg[u], u)) { free(deg); free(gone); heap_free(&h); return -1; }
    }
  }
  free(deg);
  free(gone);
  heap_free(&h);
  return 0;
}
