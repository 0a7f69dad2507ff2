// og_bench: native driver for the benchmark workloads through the C ABI.
//
// Generates the seeded road-like grid (or R-MAT) with libgraphgen, uploads
// it, and runs single-source queries (distances + canonical predecessors)
// with og_sssp, or k-core decompositions with og_kcore, timing each call's
// phases with the library's HIP events.  It exists so that profilers can be
// attached to a plain native process; the Python benchmark (bench.py) runs
// the same workloads, sources and schedules.
//
//   og_bench [--graph road|rmat] [--side 4096] [--scale 24] [--delta 512]
//            [--steps 8] [--warmup 2] [--update fused|unfused|lazy]
//            [--engine persistent|host|graph] [--window K] [--kcore]
//            [--direction push|pull|hybrid]   (pull and hybrid need --update lazy)
//            [--bins]   (degree-binned load balancing)
//            [--split [--keep]]   (light/heavy edge split; --keep reuses the
//                                  split copy across the calls)
//            [--blocks [--block-size N]]   (LDS-resident vertex blocks, the
//                                  blocked copy kept across the calls)
//            [--batch N]   (each step: one og_sssp_batch call over the first N
//                           sources)
//            [--copy-calibration]
//
// --copy-calibration instead runs a plain copy kernel over 1 GiB three
// times, to scale hardware byte counters against a kernel of known traffic.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "og.h"

extern "C" {
// libgraphgen (graphgen/graphgen.cpp)
void* gg_road(int32_t side, double p_keep, double lr_frac, int32_t lr_radius, uint64_t seed);
void* gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, int32_t wlo, int32_t whi,
             uint64_t seed);
int32_t gg_n(const void* g);
int64_t gg_m(const void* g);
void gg_copy(const void* g, int64_t* row_ptr, int32_t* col, int32_t* w);
void gg_free(void* g);
void gg_uniform(uint64_t seed, uint64_t stream, int64_t count, uint64_t k, int64_t* out);
}

namespace {

constexpr uint64_t kStreamSources = 101;  // graphgen.STREAM_SOURCES

#define CHECK(x)                                                                       \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      std::fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
      std::exit(1);                                                                    \
    }                                                                                  \
  } while (0)

__global__ void copy_kernel(const int4* __restrict__ a, int4* __restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

int copy_calibration() {
  const size_t bytes = (size_t)1 << 30;
  int4 *a = nullptr, *b = nullptr;
  CHECK(hipMalloc(&a, bytes));
  CHECK(hipMalloc(&b, bytes));
  CHECK(hipMemset(a, 1, bytes));
  for (int i = 0; i < 3; ++i) hipLaunchKernelGGL(copy_kernel, dim3(8192), dim3(256), 0, 0, a, b, bytes / 16);
  CHECK(hipDeviceSynchronize());
  std::printf("{\"copy_kernel_bytes_read_per_launch\": %zu, \"bytes_written_per_launch\": %zu, \"launches\": 3}\n",
              bytes, bytes);
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  int side = 4096, scale = 24, delta = 512, steps = 8, warmup = 2, nsrc = 8, window = 0;
  int update = OG_EAGER_WITH_FUSION, engine = OG_ENGINE_PERSISTENT;
  bool rmat = false, kcore = false;
  uint32_t direction = 0;
  bool bins = false, split = false, keep = false, blocks = false;
  int block_size = 0, batch = 0;
  for (int i = 1; i < argc; ++i) {
    auto next = [&](void) -> const char* {
      if (i + 1 >= argc) { std::fprintf(stderr, "missing value for %s\n", argv[i]); std::exit(2); }
      return argv[++i];
    };
    if (!std::strcmp(argv[i], "--side")) side = std::atoi(next());
    else if (!std::strcmp(argv[i], "--delta")) delta = std::atoi(next());
    else if (!std::strcmp(argv[i], "--steps")) steps = std::atoi(next());
    else if (!std::strcmp(argv[i], "--warmup")) warmup = std::atoi(next());
    else if (!std::strcmp(argv[i], "--scale")) scale = std::atoi(next());
    else if (!std::strcmp(argv[i], "--window")) window = std::atoi(next());
    else if (!std::strcmp(argv[i], "--kcore")) kcore = true;
    else if (!std::strcmp(argv[i], "--graph")) rmat = !std::strcmp(next(), "rmat");
    else if (!std::strcmp(argv[i], "--update")) {
      const char* u = next();
      update = !std::strcmp(u, "unfused") ? OG_EAGER_NO_FUSION
               : !std::strcmp(u, "lazy")  ? OG_LAZY_UPDATE
                                          : OG_EAGER_WITH_FUSION;
    } else if (!std::strcmp(argv[i], "--engine")) {
      const char* e = next();
      engine = !std::strcmp(e, "host") ? OG_ENGINE_HOST_ROUNDS
               : !std::strcmp(e, "graph") ? OG_ENGINE_GRAPH_ROUNDS
                                          : OG_ENGINE_PERSISTENT;
    }
    else if (!std::strcmp(argv[i], "--direction")) {
      const char* d = next();
      direction = !std::strcmp(d, "pull") ? OG_FLAG_DENSE_PULL : !std::strcmp(d, "hybrid") ? OG_FLAG_HYBRID_DIRECTION : 0u;
    }
    else if (!std::strcmp(argv[i], "--bins")) bins = true;
    else if (!std::strcmp(argv[i], "--split")) split = true;
    else if (!std::strcmp(argv[i], "--keep")) keep = true;
    else if (!std::strcmp(argv[i], "--blocks")) blocks = true;
    else if (!std::strcmp(argv[i], "--block-size")) block_size = std::atoi(next());
    else if (!std::strcmp(argv[i], "--batch")) batch = std::atoi(next());
    else if (!std::strcmp(argv[i], "--copy-calibration")) return copy_calibration();
    else { std::fprintf(stderr, "unknown argument %s\n", argv[i]); return 2; }
  }

  if (batch < 0 || (batch > 0 && kcore)) {
    std::fprintf(stderr, "--batch needs N >= 1 and no --kcore\n");
    return 2;
  }
  if (batch > nsrc) nsrc = batch;
  // road: as graphgen.road(side, seed=0); rmat: as graphgen.rmat(scale, 16, seed=0), w in [1, 1000)
  void* h = rmat ? gg_rmat(scale, 16, 0.57, 0.19, 0.19, 1, 1000, 0) : gg_road(side, 0.75, 0.001, 64, 0);
  if (!h) { std::fprintf(stderr, "graph generation failed\n"); return 1; }
  const int32_t n = gg_n(h);
  const int64_t m = gg_m(h);
  std::vector<int64_t> row_ptr((size_t)n + 1);
  std::vector<int32_t> col((size_t)m), w((size_t)m);
  gg_copy(h, row_ptr.data(), col.data(), w.data());
  gg_free(h);
  // sources: uniform over vertices of out-degree >= 1 (same draw as graphgen.pick_sources)
  std::vector<int64_t> cand;
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] > row_ptr[v]) cand.push_back(v);
  std::vector<int64_t> pick(nsrc);
  gg_uniform(rmat ? 2 : 1, kStreamSources, nsrc, cand.size(), pick.data());
  std::vector<int32_t> srcs(nsrc);
  for (int i = 0; i < nsrc; ++i) srcs[i] = (int32_t)cand[pick[i]];

  int64_t* d_rp;
  int32_t *d_col, *d_w, *d_dist, *d_pred;
  CHECK(hipMalloc(&d_rp, sizeof(int64_t) * ((size_t)n + 1)));
  CHECK(hipMalloc(&d_col, sizeof(int32_t) * (size_t)m));
  CHECK(hipMalloc(&d_w, sizeof(int32_t) * (size_t)m));
  const size_t nout = (size_t)n * (size_t)(batch > 0 ? batch : 1);
  CHECK(hipMalloc(&d_dist, sizeof(int32_t) * nout));
  CHECK(hipMalloc(&d_pred, sizeof(int32_t) * nout));
  CHECK(hipMemcpy(d_rp, row_ptr.data(), sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
  CHECK(hipMemcpy(d_col, col.data(), sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(d_w, w.data(), sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));

  og_graph g{n, m, d_rp, d_col, d_w};
  og_schedule s;
  og_default_schedule(&s);
  s.delta = delta;
  s.update = update;
  s.engine = engine;
  s.flags = OG_FLAG_TIMING | direction | (bins ? OG_FLAG_DEGREE_BINS : 0u) | (split ? OG_FLAG_LIGHT_HEAVY : 0u) |
            (split && keep ? OG_FLAG_KEEP_SPLIT : 0u) | (blocks ? OG_FLAG_VERTEX_BLOCKS | OG_FLAG_KEEP_BLOCKS : 0u);
  if (block_size > 0) s.block_size = block_size;
  if (window > 0) s.window_buckets = window;
  const size_t wsb = kcore ? og_workspace_bytes_kcore(&g, &s)
                    : batch > 0 ? og_workspace_bytes_batch(&g, &s, batch)
                                : og_workspace_bytes(&g, &s);
  void* ws = nullptr;
  CHECK(hipMalloc(&ws, wsb));
  hipStream_t stream;
  CHECK(hipStreamCreate(&stream));

  double eng = 0, pred = 0, tot_e = 0, rounds = 0;
  for (int i = 0; i < warmup + steps; ++i) {
    og_stats st;
    const og_status rc = kcore       ? og_kcore(&g, &s, d_dist, ws, wsb, &st, stream)
                         : batch > 0 ? og_sssp_batch(&g, srcs.data(), batch, &s, d_dist, d_pred, ws, wsb, &st, stream)
                                     : og_sssp(&g, srcs[i % nsrc], &s, d_dist, d_pred, ws, wsb, &st, stream);
    if (rc != OG_OK) {
      std::fprintf(stderr, "%s failed: %s\n", kcore ? "og_kcore" : batch > 0 ? "og_sssp_batch" : "og_sssp",
                   og_status_string(rc));
      return 1;
    }
    if (i >= warmup) {
      eng += st.engine_ms;
      pred += st.pred_ms;
      tot_e += (double)st.reached_edges;
      rounds += (double)st.rounds;
      if (batch > 0)
        std::fprintf(stderr, "step %d batch of %d: engine %.3f ms pred %.3f ms rounds %lld\n", i - warmup, batch,
                     st.engine_ms, st.pred_ms, (long long)st.rounds);
      else
        std::fprintf(stderr, "step %d src %d: engine %.3f ms pred %.3f ms rounds %lld\n", i - warmup,
                     srcs[i % nsrc], st.engine_ms, st.pred_ms, (long long)st.rounds);
    }
  }
  std::printf("{\"graph\": \"%s\", \"call\": \"%s\", \"batch\": %d, \"n\": %d, \"m\": %lld, \"delta\": %d, \"update\": %d, "
              "\"engine\": %d, \"direction\": %u, \"steps\": %d, \"engine_ms\": %.4f, \"pred_ms\": %.4f, \"rounds\": %.1f, "
              "\"reached_edges\": %.0f}\n",
              rmat ? "rmat" : "road", kcore ? "og_kcore" : batch > 0 ? "og_sssp_batch" : "og_sssp", batch, n, (long long)m, delta, update, engine, direction, steps,
              eng / steps, pred / steps, rounds / steps, tot_e / steps);
  if (og_release() != OG_OK) {
    std::fprintf(stderr, "og_release failed\n");
    return 1;
  }
  CHECK(hipStreamDestroy(stream));
  CHECK(hipFree(ws));
  CHECK(hipFree(d_rp));
  CHECK(hipFree(d_col));
  CHECK(hipFree(d_w));
  CHECK(hipFree(d_dist));
  CHECK(hipFree(d_pred));
  return 0;
}
