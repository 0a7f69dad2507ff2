/*
 * og.h -- ordered (bucketed) shortest-path processing on MI355X (gfx950).
 *
 * A C ABI over hand-written HIP kernels for Delta-stepping with eager
 * bucket updates and bucket fusion, as described in "Optimizing Ordered
 * Graph Algorithms with GraphIt" (CGO 2020):
 *   - section 2: priority coarsening, bucket index = floor(priority / Delta);
 *   - section 3.2: eager bucket update (each worker inserts improved
 *     vertices into its own buckets; the smallest non-empty bucket across
 *     workers is processed next);
 *   - section 3.3: bucket fusion (a worker keeps processing its local copy
 *     of the current bucket, without a global synchronisation, while it is
 *     non-empty and smaller than a threshold);
 *   - section 6.1: SSSP, wBFS (Delta fixed to 1), PPSP (stop on entering
 *     bucket i with i*Delta >= best distance to the target found so far)
 *     and A* (priority = distance so far + per-vertex estimate).
 * The schedule fields mirror the scheduling-language table of section 4.2
 * (configApplyPriorityUpdate, ...Delta, configBucketFusionThreshold,
 * configNumBuckets); the traversal direction (configApplyDirection) is a
 * schedule flag.  Also: the lazy bucket update (section 3.1) and k-core
 * decomposition (section 6.1), batched queries, and a float32 variant with
 * a backward pass.
 *
 * Conventions
 *   - Every array argument is DEVICE memory owned by the caller, except
 *     og_stats and the og_graph / og_schedule structs themselves, which are
 *     host memory.  The library allocates nothing: scratch space is the
 *     caller's workspace buffer, sized by og_workspace_bytes().
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it.  Unless OG_FLAG_ASYNC is set the call waits
 *     for the stream before returning and reports the device-side status.
 *   - Graphs are directed CSR: the out-edges of v are col[row_ptr[v] ..
 *     row_ptr[v+1]) with weights w[...].  An undirected graph stores both
 *     directions.  Weights are int32 >= 0.  A negative weight on an edge the
 *     search examines is reported as OG_ERR_NEGATIVE_WEIGHT (outputs then
 *     undefined); OG_FLAG_VALIDATE checks every weight before running.
 *     Column indices must lie in [0, n) and row_ptr must run from 0 to m
 *     without decreasing: a malformed graph is undefined behaviour unless
 *     OG_FLAG_VALIDATE is set, which checks the structure first and then
 *     returns OG_ERR_INVALID_ARG with nothing else run.
 *   - Distances are int32 with INF = INT32_MAX for unreachable vertices.  A
 *     finite path length that does not fit below INT32_MAX is reported as
 *     OG_ERR_OVERFLOW (the outputs are then undefined).
 *   - Predecessors (optional, may be NULL) follow a canonical rule, so they
 *     are unique: pred[v] = the smallest u with an edge (u,v) and
 *     dist[u] + w(u,v) == dist[v]; pred[src] = src; -1 if v is unreachable.
 *   - Calls on one workspace must not overlap; distinct workspaces may run
 *     concurrently on distinct streams.
 */
#ifndef OG_H
#define OG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t og_status;
#define OG_OK 0
#define OG_ERR_INVALID_ARG (-1)     /* bad argument; nothing was launched       */
#define OG_ERR_NEGATIVE_WEIGHT (-2) /* an edge weight < 0 was found             */
#define OG_ERR_OVERFLOW (-3)        /* a path length reached INT32_MAX          */
#define OG_ERR_WORKSPACE (-4)       /* ws_bytes too small, a queue filled up or
                                       the queue pool ran empty;
                                       og_stats.queue_needed tells how many
                                       entries per queue would have been used,
                                       og_stats.pool_needed how many pool
                                       entries were in use                     */
#define OG_ERR_HIP (-5)             /* a HIP runtime call failed                */
#define OG_ERR_ROUND_LIMIT (-6)     /* schedule.max_rounds reached              */
#define OG_ERR_INTERNAL (-7)        /* an internal consistency check failed
                                       (a library bug; no memory was touched
                                       out of bounds)                           */

/* Schedule flags. */
#define OG_FLAG_VALIDATE 1u /* check the CSR structure and the weights' signs
                               before running (waits for the check, also with
                               OG_FLAG_ASYNC)                                 */
#define OG_FLAG_ASYNC 2u    /* do not wait; read the status later with
                               og_read_stats() after synchronising the stream */
#define OG_FLAG_TIMING 4u   /* time the phases with HIP events recorded on the
                               stream (ignored with OG_FLAG_ASYNC)            */
#define OG_FLAG_LIGHT_HEAVY 8u /* light/heavy edge split (Meyer and Sanders'
                               Delta-stepping; the paper relaxes every edge):
                               rounds relax only light edges (w < Delta); the
                               heavy edges of the vertices settled in a bucket
                               are relaxed once, in one extra round when the
                               bucket is finished.  int32 weights and eager
                               updates only (og_sssp_f32 and a lazy schedule
                               return OG_ERR_INVALID_ARG); the workspace holds
                               a split copy of the rows.  og_kcore ignores it. */
#define OG_FLAG_DENSE_PULL 16u /* traversal direction DensePull (section 4.2,
                               configApplyDirection; combined with lazy updates
                               as in section 5.1): every round first marks its
                               frontier in a dense per-vertex array, then each
                               vertex that can still improve reads its own row
                               as its in-edges and takes the best offer of the
                               marked neighbours, with no atomic operation on
                               the destination.  Requires OG_LAZY_UPDATE and a
                               SYMMETRIC graph (each edge (u, v, w) has a
                               reverse (v, u, w); with OG_FLAG_VALIDATE this is
                               checked, by a 64-bit hash of the edge multiset,
                               and a failure returns OG_ERR_INVALID_ARG).
                               int32 weights (og_sssp_f32 returns
                               OG_ERR_INVALID_ARG).  Applies to og_kcore too
                               (a vertex counts its peeled neighbours).  The
                               workspace holds the frontier marks (8 bytes
                               per vertex; og_kcore: one bit) and a list of
                               slices of the rows longer than 8192 edges.    */
#define OG_FLAG_HYBRID_DIRECTION 32u /* SparsePush-DensePull: as
                               OG_FLAG_DENSE_PULL, but a round pulls only when
                               its input holds more than n/20 entries (the
                               frontier's edges, estimated as its size times the
                               mean degree, exceed m/20) and pushes otherwise.
                               Same requirements; not together with
                               OG_FLAG_DENSE_PULL.                            */
#define OG_FLAG_KEEP_SPLIT 128u /* with OG_FLAG_LIGHT_HEAVY: reuse the split
                               copy of the rows that the previous split call on
                               this workspace built, when it was for the same
                               graph arrays, sizes and Delta (the library keeps
                               a record per workspace; any other call on the
                               workspace drops it, and a mismatch rebuilds).
                               The caller promises that the graph's contents
                               have not changed since.  Ignored without
                               OG_FLAG_LIGHT_HEAVY.                           */
#define OG_FLAG_DEGREE_BINS 64u /* degree-binned load balancing: within each
                               batch of queue entries, a vertex of at most
                               schedule.bin_thread edges gets a fixed group of
                               4 lanes, one edge each (no scan, no search),
                               one of at most schedule.bin_wave edges one
                               wavefront, 64 edges at a time, and larger ones
                               the whole workgroup (a block scan spreads their
                               edges over all lanes, the default for every
                               vertex without this flag).  int32 and float32
                               weights (og_sssp_f32); not together with
                               OG_FLAG_LIGHT_HEAVY or a pull direction;
                               og_kcore ignores it.                           */

#define OG_FLAG_VERTEX_BLOCKS 256u /* bucket fusion at the granularity of a
                               vertex block (section 3.3: a worker keeps
                               processing its share of the current bucket
                               without a global synchronisation).  The library
                               groups the vertices into compact blocks (cells
                               of a hop-distance Voronoi partition from sampled
                               seeds; about schedule.block_size vertices each,
                               at most 4,096 vertices and 12,288 internal
                               edges); a workgroup that takes a block holds its
                               distances and internal edges (weights below
                               65,536) in LDS and drains the block's part of
                               the current bucket there, with LDS atomics; only
                               edges that leave the block update dist in HBM.
                               A block improved across its boundary in the
                               current bucket is queued for any idle workgroup
                               within the same round.  Meant for graphs with
                               locality, such as road networks.  int32 weights,
                               og_sssp / og_wbfs / og_ppsp / og_sssp_multi
                               only (a batch or an A* estimate returns
                               OG_ERR_INVALID_ARG), update
                               OG_EAGER_WITH_FUSION and the persistent engine
                               (else OG_ERR_INVALID_ARG), not together with
                               OG_FLAG_LIGHT_HEAVY, OG_FLAG_DEGREE_BINS or a
                               pull direction.  The workspace holds the blocked
                               copy (about 20 bytes per vertex and 16 per edge),
                               per-query block state and the build's
                               temporaries (about 60 bytes per vertex); building
                               the copy waits on the stream, also with
                               OG_FLAG_ASYNC.  og_kcore ignores it.            */
#define OG_FLAG_KEEP_BLOCKS 512u /* with OG_FLAG_VERTEX_BLOCKS: reuse the
                               blocked copy that the previous block call on this
                               workspace built, when it was for the same graph
                               arrays, sizes and block_size (as
                               OG_FLAG_KEEP_SPLIT; the caller promises that the
                               graph's contents have not changed since).       */

/* Priority-update strategies (section 4.2, configApplyPriorityUpdate). */
#define OG_EAGER_NO_FUSION 0
#define OG_EAGER_WITH_FUSION 1
#define OG_LAZY_UPDATE 2 /* section 3.1: a round only records which vertices
                            changed (each once, by a flag); after a device-wide
                            barrier each of them is filed once into the bucket
                            of its final priority.  Two barriers per round, no
                            fusion.  For og_kcore the recorded change is a
                            count of lost neighbours (constant-sum reduction,
                            section 5.1).                                     */

/* Engines. */
#define OG_ENGINE_PERSISTENT 0 /* one cooperative launch, device-wide barrier
                                  between rounds (default; with teams, each
                                  team's barrier between its own rounds)     */
#define OG_ENGINE_HOST_ROUNDS 1 /* one kernel launch per round (with teams:
                                  one round of every team not yet done)      */
#define OG_ENGINE_GRAPH_ROUNDS 2 /* as _HOST_ROUNDS, the launches replayed from
                                   one executable hipGraph of 32 rounds, kept
                                   per host thread while the call's kernel,
                                   grid and arguments stay the same          */

/* Borrowed view of a directed CSR graph (device arrays). */
typedef struct og_graph {
  int32_t n;               /* vertices, >= 1                                  */
  int64_t m;               /* directed edges, row_ptr[n]                      */
  const int64_t* row_ptr;  /* [n+1], row_ptr[0] = 0, non-decreasing           */
  const int32_t* col;      /* [m], destinations in [0, n)                     */
  const int32_t* w;        /* [m], weights >= 0                               */
} og_graph;

/* How to run (section 4.2).  Zero fields take the defaults documented here;
 * og_default_schedule() fills them in explicitly. */
typedef struct og_schedule {
  int32_t delta;            /* Delta >= 1: bucket = floor(priority/Delta)     */
  int32_t update;           /* OG_EAGER_WITH_FUSION (default), ..._NO_FUSION
                               or OG_LAZY_UPDATE                              */
  int32_t fusion_threshold; /* a workgroup keeps processing its local current
                               bucket while it holds fewer entries than this
                               (0 = 1024; capped at the LDS queue, 1024)      */
  int32_t window_buckets;   /* buckets materialised at once, 2..64 (0 = 16);
                               later ones wait in an overflow ("far") queue   */
  int32_t engine;           /* OG_ENGINE_PERSISTENT (default), _HOST_ROUNDS or
                               _GRAPH_ROUNDS                                  */
  int32_t max_rounds;       /* stop with OG_ERR_ROUND_LIMIT after this many
                               rounds (0 = unlimited)                         */
  int32_t workgroups;       /* workgroups to launch (0 = all co-resident)     */
  uint32_t flags;           /* OG_FLAG_*                                      */
  int64_t queue_capacity;   /* entries per global queue (0 = n + m/8; og_kcore:
                               2n + m/8)                                      */
  int32_t bin_thread;       /* OG_FLAG_DEGREE_BINS: largest degree relaxed by
                               one lane (0 = 4; at most 4)                    */
  int32_t bin_wave;         /* OG_FLAG_DEGREE_BINS: largest degree relaxed by
                               one wavefront (0 = 64; below bin_thread: no
                               wavefront bin)                                 */
  int32_t block_size;       /* OG_FLAG_VERTEX_BLOCKS: mean block size the
                               partition aims at, in vertices (0 = 2048; at
                               most 4096)                                     */
  int64_t queue_pool;       /* entries shared by all global queues, drawn in
                               chunks of 4096 as the queues grow and returned
                               when a queue has been consumed (0 = twice
                               queue_capacity plus one chunk per queue); with
                               teams, each team draws from an equal share.
                               An empty pool (or share) ends the call with
                               OG_ERR_WORKSPACE                               */
  int32_t teams;            /* batched calls of the eager push engine: teams
                               of workgroups (workgroup b in team b mod
                               teams), each with the queries q with q mod
                               teams = team, its own queues, pool share and
                               rounds: a team synchronises only its own
                               workgroups and takes its own bucket
                               decisions.  The hardware deals consecutive
                               workgroups to the 8 XCDs in turn, so with 8
                               teams each XCD serves its own queries.  0 =
                               8; at most 8, one per query and one per
                               workgroup.  Other calls, OG_LAZY_UPDATE and
                               the split, pull and block variants run one
                               team                                           */
} og_schedule;

/* Per-call counters (host struct). */
typedef struct og_stats {
  og_status status;
  int32_t workgroups;       /* workgroups launched                            */
  int64_t rounds;           /* rounds (bucket decisions); with teams, the
                               most rounds one team took                      */
  int64_t buckets;          /* distinct buckets processed, summed over teams  */
  int64_t relaxations;      /* edges examined                                 */
  int64_t improvements;     /* successful atomic minimum updates              */
  int64_t pushes_local;     /* entries appended to an LDS (fused) queue       */
  int64_t pushes_global;    /* entries appended to a global queue             */
  int64_t far_pushes;       /* of which went to the overflow queue            */
  int64_t reached_vertices; /* dist < INF (computed when pred or stats given) */
  int64_t reached_edges;    /* sum of out-degrees of reached vertices         */
  int64_t queue_needed;     /* largest queue fill requested, in entries       */
  double init_ms;           /* OG_FLAG_TIMING: initialisation kernel          */
  double engine_ms;         /* OG_FLAG_TIMING: bucket engine (all rounds)     */
  double pred_ms;           /* OG_FLAG_TIMING: predecessor / counting pass    */
  int64_t batches;          /* batches of up to 256 entries processed, summed
                               over workgroups                                */
  int64_t chain;            /* sum over rounds of the most batches any one
                               workgroup processed in that round (the engine's
                               critical path in batch steps); with teams, the
                               largest team's sum                             */
  int64_t barriers;         /* device-wide synchronisations: one per round, two
                               with OG_LAZY_UPDATE; with teams, the most one
                               team took (each synchronises its own)          */
  int64_t blocks;           /* OG_FLAG_VERTEX_BLOCKS: blocks of the copy (the
                               activations of blocks are counted in batches)  */
  double prep_ms;           /* OG_FLAG_VERTEX_BLOCKS with OG_FLAG_TIMING: time
                               to build the blocked copy (0 when kept)        */
  int64_t pool_needed;      /* most queue-pool entries in use at once (whole
                               chunks; with teams: the most one team held
                               times the team count, the pool whose equal
                               shares hold every team's peak; after
                               OG_ERR_WORKSPACE: the demand up to the
                               failure)                                       */
} og_stats;

/* Library version, (major << 16) | minor. */
int32_t og_version(void);

/* Human-readable name of a status code (static string). */
const char* og_status_string(og_status s);

/* Overwrites every field of *s with the defaults (delta 1, fusion on,
 * threshold 1024, 16 window buckets, persistent engine, no limits, degree
 * bins 4 / 64, blocks of 2048 vertices). */
og_status og_default_schedule(og_schedule* s);

/* Workspace bytes og_sssp & co. need for this graph and schedule (0 if the
 * arguments are invalid).  Aligned to 256 bytes. */
size_t og_workspace_bytes(const og_graph* g, const og_schedule* s);

/* Single-source shortest paths by Delta-stepping (sections 3.2, 3.3).
 *   src      : source vertex in [0, n)
 *   dist     : [n] output distances
 *   pred     : [n] output canonical predecessors, or NULL
 *   ws       : device workspace of ws_bytes >= og_workspace_bytes(g, s)
 *   stats    : host counters, or NULL
 * Returns OG_OK or an error code (see above). */
og_status og_sssp(const og_graph* g, int32_t src, const og_schedule* s, int32_t* dist, int32_t* pred,
                  void* ws, size_t ws_bytes, og_stats* stats, void* stream);

/* Weighted BFS (section 6.1): og_sssp with Delta forced to 1; intended for
 * positive integer weights in [1, log n). */
og_status og_wbfs(const og_graph* g, int32_t src, const og_schedule* s, int32_t* dist, int32_t* pred,
                  void* ws, size_t ws_bytes, og_stats* stats, void* stream);

/* Point-to-point shortest path (section 6.1): stops before processing a
 * bucket i with i*Delta >= dist[dst].  Only dist[dst] and the predecessor
 * chain from dst back to src are defined on return (other entries hold
 * upper bounds).  dist[dst] = INT32_MAX if dst is unreachable. */
og_status og_ppsp(const og_graph* g, int32_t src, int32_t dst, const og_schedule* s, int32_t* dist,
                  int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats, void* stream);

/* A* (section 6.1): as og_ppsp, but a vertex v reached at distance d is
 * bucketed by floor((d + h[v]) / Delta).  h ([n], device, int32 >= 0) must
 * be admissible (never above the true remaining distance to dst, so
 * h[dst] = 0) for dist[dst] to be exact. */
og_status og_astar(const og_graph* g, int32_t src, int32_t dst, const int32_t* h, const og_schedule* s,
                   int32_t* dist, int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats,
                   void* stream);

/* ---- Several queries in one launch ------------------------------------
 * Query q works on its own copy of the graph (virtual vertex q * n + v);
 * all queries share one bucket sequence, so a single persistent launch
 * serves the whole batch.  One launch holds up to Q = min(1024,
 * (2^31 - 2) / n) queries (virtual ids are int32); a batch of more (up to
 * 2^20 queries) runs as consecutive launches of up to Q queries on the same
 * workspace, each on its own slice of dist, pred and h, with the counters
 * summed (not with OG_FLAG_ASYNC or OG_FLAG_VERTEX_BLOCKS:
 * OG_ERR_INVALID_ARG).  srcs and dsts are HOST arrays of nq base vertex ids;
 * dist and pred are DEVICE arrays of nq * n entries, query q's results at
 * [q * n, (q + 1) * n) (pred holds base vertex ids).  The workspace must
 * hold og_workspace_bytes_batch(), sized for min(nq, Q) queries. */
size_t og_workspace_bytes_batch(const og_graph* g, const og_schedule* s, int32_t nq);

/* nq independent single-source queries (og_sssp semantics per query). */
og_status og_sssp_batch(const og_graph* g, const int32_t* srcs, int32_t nq, const og_schedule* s, int32_t* dist,
                        int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats, void* stream);

/* nq point-to-point queries (og_ppsp semantics per query): the launch stops
 * before a bucket i with i*Delta >= dist of every query's target. */
og_status og_ppsp_batch(const og_graph* g, const int32_t* srcs, const int32_t* dsts, int32_t nq,
                        const og_schedule* s, int32_t* dist, int32_t* pred, void* ws, size_t ws_bytes,
                        og_stats* stats, void* stream);

/* nq A* queries (og_astar semantics per query); h is a DEVICE array of
 * nq * n estimates, query q's at [q * n, (q + 1) * n). */
og_status og_astar_batch(const og_graph* g, const int32_t* srcs, const int32_t* dsts, int32_t nq, const int32_t* h,
                         const og_schedule* s, int32_t* dist, int32_t* pred, void* ws, size_t ws_bytes,
                         og_stats* stats, void* stream);

/* Multi-source shortest paths: dist[v] = min over the nsrc sources (HOST
 * array) of the shortest distance to v; pred[src] = src for every source.
 * Many disjoint graphs stored as one block-diagonal CSR, one source each,
 * are solved in one launch this way.  Workspace: og_workspace_bytes_multi(). */
size_t og_workspace_bytes_multi(const og_graph* g, const og_schedule* s, int32_t nsrc);
og_status og_sssp_multi(const og_graph* g, const int32_t* srcs, int32_t nsrc, const og_schedule* s, int32_t* dist,
                        int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats, void* stream);

/* ---- Real-valued weights (the differentiable variant) ------------------
 * The same engine on float32 distances: every relaxation computes
 * fl32(dist[u] + w) (round to nearest), so the result is the unique fixed
 * point D(v) = min over in-edges fl32(D(u) + w(u,v)), D(src) = 0, whatever
 * the schedule; unreachable vertices get +inf.  Weights must be finite and
 * >= 0 (a NaN, infinite or negative weight is OG_ERR_NEGATIVE_WEIGHT); a sum
 * that reaches +inf is OG_ERR_OVERFLOW.  Delta is the bucket width
 * (bucket = floor(d / Delta)).  Predecessors follow the canonical rule with
 * float32 tightness (fl32(D(u) + w) == D(v)); pred_edge[v] (optional, needs
 * pred) is the CSR index of the tree edge pred[v] -> v, -1 for the source
 * and unreachable vertices. */
typedef struct og_graph_f32 {
  int32_t n;
  int64_t m;
  const int64_t* row_ptr;  /* [n+1] */
  const int32_t* col;      /* [m], rows sorted by destination */
  const float* w;          /* [m] */
} og_graph_f32;

size_t og_workspace_bytes_f32(const og_graph_f32* g, const og_schedule* s);

og_status og_sssp_f32(const og_graph_f32* g, int32_t src, const og_schedule* s, float* dist, int32_t* pred,
                      int32_t* pred_edge, void* ws, size_t ws_bytes, og_stats* stats, void* stream);

/* Backward pass: given the tree of an og_sssp_f32 call and an upstream
 * gradient grad_dist[v] = dL/dD(v) (DEVICE, n floats), writes
 * grad_w[e] = dL/dw_e (DEVICE, m floats): for the tree edge e into v, the
 * sum of grad_dist over v's subtree (accumulated in float64, then rounded);
 * 0 for every other edge.  This is the derivative of the distances when
 * shortest paths are unique.  Stream-ordered, no synchronisation.
 * Workspace: og_backward_workspace_bytes(n) bytes, 256-byte aligned. */
size_t og_backward_workspace_bytes(int32_t n);
og_status og_sssp_backward_f32(const og_graph_f32* g, const int32_t* pred, const int32_t* pred_edge,
                               const float* grad_dist, float* grad_w, void* ws, size_t ws_bytes, void* stream);

/* ---- k-core decomposition (section 6.1, k-core) ------------------------
 * core[v] = the coreness of v: the largest k such that v lies in a subgraph
 * whose every vertex keeps at least k neighbours.  The graph must be
 * undirected (both directions stored); the degree of v is its row length
 * and w may be NULL (weights are not read).  Vertices are peeled in
 * increasing order of remaining degree, one bucket per degree value (Delta
 * is not used: the order is strict, section 2).  core is also the priority
 * vector during the call.  update:
 *   OG_LAZY_UPDATE (recommended): a round counts, per neighbour, how many of
 *     its neighbours were peeled (one atomic increment each) and then lowers
 *     each counted neighbour's degree once by that count, clamped at the
 *     current level (the constant-sum reduction of section 5.1);
 *   OG_EAGER_NO_FUSION / OG_EAGER_WITH_FUSION: every peeled edge lowers the
 *     neighbour's degree by one at once (compare-and-swap, clamped at the
 *     current level) and files it in its new bucket.
 * Workspace: og_workspace_bytes_kcore(). */
size_t og_workspace_bytes_kcore(const og_graph* g, const og_schedule* s);
og_status og_kcore(const og_graph* g, const og_schedule* s, int32_t* core, void* ws, size_t ws_bytes,
                   og_stats* stats, void* stream);

/* Reads the status and counters of the last call made with workspace ws
 * (device) into *stats (host); used after an OG_FLAG_ASYNC call once the
 * stream has been synchronised.  Blocking copy on stream. */
og_status og_read_stats(const void* ws, og_stats* stats, void* stream);

/* ---- A call that allocates nothing -------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * og_sssp_noalloc is og_sssp with the workspace taken from a fixed device
 * array inside the library, OG_SCRATCH_BYTES (32 MiB) per device, present
 * from the library's load on that device until the process ends.  The
 * caller still owns dist and pred.  It calls no hipMalloc / hipFree and
 * creates no HIP object, so OG_FLAG_TIMING and OG_ENGINE_GRAPH_ROUNDS are
 * rejected (OG_ERR_INVALID_ARG); a graph and schedule whose
 * og_workspace_bytes() exceed OG_SCRATCH_BYTES return OG_ERR_WORKSPACE
 * with nothing launched (a smaller schedule.queue_capacity or queue_pool
 * shrinks the need).  Every call on one device uses the same array and leaves its
 * contents behind (each call initialises what it reads): calls that
 * overlap in time on one device race and must not be made.  Results are
 * those of og_sssp. */
#define OG_SCRATCH_BYTES ((size_t)32 << 20)
og_status og_sssp_noalloc(const og_graph* g, int32_t src, const og_schedule* s, int32_t* dist, int32_t* pred,
                          og_stats* stats, void* stream);

/* Releases what the library keeps per host thread between calls: the HIP
 * events of OG_FLAG_TIMING and the executable round graph of
 * OG_ENGINE_GRAPH_ROUNDS (both are recreated on demand by a later call).
 * Waits for the current device first.  Call it on each thread that made
 * calls before that thread or the process ends, while the HIP runtime is
 * still up (profilers attached to the process finalise in exit handlers).
 * Returns OG_OK, or OG_ERR_HIP if a HIP call failed. */
og_status og_release(void);

#ifdef __cplusplus
}
#endif

#endif /* OG_H */
