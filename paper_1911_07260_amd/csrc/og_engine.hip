// Delta-stepping with eager bucket updates and bucket fusion on gfx950.
//
// Paper mapping ("Optimizing Ordered Graph Algorithms with GraphIt"):
//   - A "thread" of the eager algorithm (section 3.2) is a workgroup here.
//     Its thread-local buckets are an LDS ring holding the local copy of the
//     current bucket; later buckets go to device-wide bucket queues (a
//     window of K materialised buckets plus an overflow "far" queue, the
//     same idea as keeping only a few buckets materialised in section 5.1).
//   - A round processes the round's input list (the current bucket) split
//     across workgroups; every relaxation is a 32-bit atomic minimum on dist
//     (section 3, Dist[e.dst] = min(...)), and an improved vertex is inserted
//     at once into the bucket of its new priority floor(d / Delta) (eager
//     update, section 2 coarsening).
//   - Bucket fusion (section 3.3): after its share of the round input, a
//     workgroup keeps draining its LDS current-bucket ring with no global
//     synchronisation while the ring holds fewer entries than the fusion
//     threshold; a larger local bucket is published to the global list for
//     the next round, which redistributes it over all workgroups.
//   - The global minimum-bucket selection (section 3.2, getGlobalMinBucket;
//     section 5.2, cross-thread minimum) is done once per round by the last
//     workgroup to arrive at the device-wide barrier (in a batched launch
//     split into teams: by the last of the team, at the team's barrier).
//   - Stale entries are never removed from queues: entries carry (v, d) and
//     are skipped when d > dist[v] (insert without delete).
//
// Several queries run in one launch over "virtual vertices": query q's copy
// of base vertex v is q * n + v, with its own slot in dist (and pred) and the
// base CSR shared by all copies.  A batch of single-source queries on one
// graph is the disjoint union of q copies with one source each; a
// multi-source query (one copy, several sources at distance 0) covers many
// disjoint graphs stored as one block-diagonal CSR.  The queries of one team
// of workgroups (below) share its bucket sequence and advance together
// through its rounds; different teams run their rounds independently.
//
// The same round structure carries the other schedules and algorithms, each
// as its own template instantiation so that adding one leaves the machine
// code of the others unchanged:
//   - IntW: integer distances (SSSP, wBFS with Delta = 1, PPSP with its
//     early exit, A* with the estimate added to the bucket key).
//   - FloatW: FP32 distances for the differentiable pass; the bucket of a
//     float key is floor(d / Delta) on the float value.
//   - CoreW: k-core (section 6.1) with the degree as priority and Delta = 1;
//     peeling a vertex lowers its neighbours' degrees, clamped at the core
//     value being peeled.
//   - SplitW: integer distances with light and heavy edges kept apart; light
//     edges are relaxed in the ordinary rounds, heavy edges once per finished
//     bucket.
//   - Lazy update (section 3.1; its schedules in section 5.1): changed
//     vertices are collected once per round, with a flag to drop
//     duplicates, and filed by their final priority after a second
//     device-wide barrier.
// Rounds run inside one persistent cooperative kernel, or one launch per
// round from the host, or as rounds replayed from a captured hipGraph.
//
// Correctness does not depend on the cache coherence of plain loads of
// dist: dist only decreases during a call, a plain load returns some past
// value (>= the current one), and every decision that matters is taken on
// the return value of the device-scope atomic minimum or on the distance
// carried in the queue entry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "og.h"

namespace og {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kLq = 1024;  // LDS ring entries (power of two)
constexpr int kKmax = 64;
constexpr int kDefaultK = 16;
constexpr int kDefaultThreshold = 1024;
constexpr int kGroup = 16;  // workgroups per first-level barrier counter
constexpr int kMaxWg = 4096;
constexpr int kMaxGroups = kMaxWg / kGroup;
constexpr int kFlags = 64;  // release flags, one per 128-byte line
constexpr int kMaxQueries = 1024;    // queries in one launch
constexpr int kMaxBatch = 1 << 20;  // queries in one batch call (in launches of at most kMaxQueries)
constexpr size_t kCtlBytes = 131072;
// A batched launch splits its workgroups into teams: workgroup b serves team
// b % teams, which owns the queries q with q % teams == team, a set of bucket
// lists, a share of the queue pool and a control state of its own.  A team's
// workgroups synchronise only with each other and the team takes its own
// bucket decisions, so no team waits for another's rounds.  The hardware
// deals consecutive workgroups to the XCDs in turn, so with 8 teams each
// XCD's L2 holds the working set of its own queries only.  Every vertex a
// team files belongs to one of its queries (edges stay within a query's copy
// of the graph), so a team's lists, LDS rings and pushes never mix teams.
constexpr int kMaxTeams = 8;
// The global bucket lists (K window slots, 2 spill lists, 2 far lists) draw
// fixed-size chunks from a pool, each team from an equal share of its own:
// list L's position p lives in the chunk its table names for p / kChunk.  A
// list's chunks go back to its team's share when the list is consumed.
constexpr int kChunkLog = 12;
constexpr unsigned kChunk = 1u << kChunkLog;  // entries per chunk (32 KB)
constexpr int kNoChunk = -1;    // table entry: chunk not taken yet
constexpr int kLostChunk = -2;  // table entry: the pool was empty (the call fails)
constexpr unsigned kChunkSpinLimit = 1u << 20;  // polls before a missing chunk is an internal error
constexpr unsigned kNoBucket = 0xffffffffu;
constexpr int kInf = INT_MAX;
constexpr int kPeeled = INT_MAX;  // k-core mark of a peeled vertex (above every generation)

enum : int { kInWin = 0, kInSpill = 1, kInFar = 2, kInHeavy = 3 };
// Direction of the rounds of a pull instantiation.  The hybrid pulls when
// the round input holds more than n / kPullDiv entries: the frontier's edges
// estimated as its size times the mean degree, against m / kPullDiv.
enum : int { kPullNever = 0, kPullAlways = 1, kPullHybrid = 2 };
constexpr unsigned kPullDiv = 20;
// A pull round expands rows of up to kLongRow edges inside 256-vertex
// batches; longer rows are cut into slices of kSlice edges that are handed
// out to workgroups like the batches.  Slices per graph are at most
// m / kSlice + m / kLongRow + 1.
constexpr int kLongRow = 8192;
constexpr int kSlice = 2048;
__host__ __device__ inline unsigned long long slice_cap(long long m) {
  return (unsigned long long)(m / kSlice + m / kLongRow + 1);
}
// The predecessor pass leaves rows longer than kPredLong edges out of its
// per-wavefront vertex chunks and hands them out in slices of kPredSlice
// edges, so that a hub's row does not keep one wavefront busy long after
// the rest.  Slices per copy of the graph: at most m / kPredSlice + m /
// kPredLong + 1.
constexpr int kPredLong = 1024;
constexpr int kPredSlice = 2048;
constexpr int kPredIlp = 4;  // groups of 64 edges whose loads a wavefront keeps in flight
// Edges per lane whose loads and atomics the engine keeps in flight in a
// batch of more than one workgroup's worth of edges.
constexpr int kEdgeIlp = 2;
constexpr int kPredParDeg = 8;  // mean degree from which the parity filter is used
__host__ __device__ inline unsigned long long pred_slice_cap(long long m, int reps) {
  return (unsigned long long)reps * (unsigned long long)(m / kPredSlice + m / kPredLong + 1);
}
// Light/heavy split: a settled vertex whose heavy part has more than
// kHeavySlice edges is filed for the heavy round as one entry per slice of
// kHeavySlice edges, (v, slice), so that the slices of a hub are spread over
// workgroups; any other vertex as (v, -1), its whole heavy part.  A heavy
// list then holds at most n + m / kHeavySlice entries per copy.
constexpr int kHeavySlice = 4096;
__host__ __device__ inline long long heavy_cap(long long nv, long long m, int reps) {
  return nv + (long long)reps * (m / kHeavySlice) + 1;
}
// Light/heavy split: LDS ring entries carry a vertex's light-edge count with
// this bit set when the vertex also has heavy edges.
constexpr int kHeavyBit = 1 << 30;
constexpr int kDegMask = kHeavyBit - 1;
// Degree bins: the lane bin holds vertices of up to kBinLane edges, each
// edge on a fixed slot of its own.
constexpr int kBinLane = 4;
constexpr int kDefaultBinWave = 64;
enum : int {
  kStRelax, kStImprove, kStPushLocal, kStPushGlobal, kStFar, kStBatches, kStReachedV, kStReachedE, kStCount
};

// Every counter that many workgroups update sits on its own 128-byte line.
struct alignas(128) Word {
  unsigned v;
};
struct alignas(128) Word64 {
  unsigned long long v;
};

// State chosen by the bucket decision for a team's next round.
struct alignas(128) Control {
  unsigned cur;       // current bucket
  unsigned in_kind;   // round input: window slot / spill list / far list
  unsigned in_index;
  unsigned done;
  unsigned spill_out;  // spill list receiving current-bucket pushes
  unsigned far_in;     // far list holding pending overflow entries
  unsigned win_hi;     // buckets >= win_hi go to the far list
  unsigned round;
  unsigned buckets;
  unsigned epoch;    // the team's barriers completed
  unsigned far_gen;  // generation of the pending far list (k-core filing)
  unsigned hout;     // light/heavy split: heavy list receiving settled vertices
  unsigned hgen;     // light/heavy split: generation of that list (heavy rounds so far)
  unsigned pull;     // direction of this round: 1 = dense pull (pull instantiations)
};

// A team's bucket lists: the fill of each, the smallest bucket filed in
// each far list, and the team's share of the round input.
struct TeamQ {
  Word in_count;  // entries of the team's round input list
  Word in_head;   // dynamic chunk cursor into a large round input
  Word win_tail[kKmax];
  Word spill_tail[2];
  Word far_tail[2];
  Word far_min[2];
};

// Device-side control block at the start of the workspace.  Every team
// runs rounds of its own: its control state, barrier counters, release
// flags, bucket lists and share of the queue pool are its own (a launch of
// one team uses entry 0 of each).
struct Ctl {
  Control tc[kMaxTeams];
  Word status;
  Word live;  // teams not done yet (status and live are adjacent: the host-driven engine polls both)
  Word teams;
  Word bar_root[kMaxTeams];
  Word bar_grp[kMaxGroups + 2 * kMaxTeams];  // each team's first-level counters, kGroup workgroups each
  Word flag[kFlags];  // release flags, kFlags / teams per team: the round number now allowed to start
  TeamQ tq[kMaxTeams];
  Word round_max_batches[kMaxTeams];  // most batches one of the team's workgroups ran in its current round
  Word buf_tail;                      // lazy update: entries in the change buffer
  Word64 need;
  Word64 st[kStCount];
  Word64 chain[kMaxTeams];  // per team: sum over its rounds of round_max_batches
  Word heavy_tail[2];  // light/heavy split: settled vertices per heavy list
  Word big_rows;       // light/heavy split: rows left to the wavefront split pass
  Word64 sym;          // symmetry checksum of OG_FLAG_VALIDATE with a pull direction
  Word slices;         // pull direction: row slices listed per copy of the graph
  Word64 pred_slices;  // predecessor pass: slices of long rows listed
  Word free_top[kMaxTeams];   // free chunks on each team's stack
  Word pool_peak[kMaxTeams];  // most of the team's chunks taken at once (sampled at each bucket decision)
  Word blk_out;        // vertex blocks: work items of the round not yet finished
  Word blk_head;       // vertex blocks: ring positions taken
  Word blk_tail;       // vertex blocks: ring positions filled
};
static_assert(sizeof(Ctl) <= kCtlBytes, "control block too large");

struct Args {
  const long long* row_ptr;
  const int* col;
  const int* w;
  int* dist;     // [n] virtual vertices
  const int* h;  // [n] A* estimate or nullptr
  int n;         // virtual vertices = reps * nbase
  int nbase;     // vertices of the base graph
  int reps;      // copies (queries)
  const int* srcs;  // [nsrc] virtual source ids (query table)
  int nsrc;
  const int* tgts;  // [reps] virtual target ids, or nullptr (no early exit)
  unsigned delta;
  int shift;  // log2(delta) when delta is a power of two, else -1
  int K;      // window buckets (power of two)
  unsigned cap;  // entries one list may hold
  int fused;
  unsigned threshold;
  unsigned max_rounds;
  int nwg;
  int teams;  // workgroup teams (1, or up to kMaxTeams in a batched launch)
  Ctl* ctl;
  int2* pool;         // [pool_chunks * kChunk] entries of every global list
  int* ctab;          // [teams * (K + 4) * tchunks] chunk of each list position / kChunk
  int* fstack;        // [pool_chunks] free chunks: team t's stack at team_lo(t) (its bottom free_top[t] entries)
  unsigned pool_chunks;
  unsigned tchunks;   // table entries per list: ceil(cap / kChunk)
  int lazy;       // lazy bucket update: record changes, file them after a barrier
  int* aux;       // [n] lazy: change flag (SSSP) or lost-neighbour count (k-core)
  int* buf;       // [buf_cap] lazy: vertices changed this round, each once
  unsigned buf_cap;
  int* mark;      // [n] k-core: kPeeled once peeled, else the newest far-list
                  // generation the vertex was filed in
  // light/heavy split (SplitW only)
  const int* ecol;    // [m] the rows' light edges first, then the heavy ones
  const int* ew;      // [m] their weights
  const int* lsplit;  // [nbase] light edges per row
  unsigned* hmark;    // [n] 1 + the generation of the last heavy list holding the vertex
  int2* heavy;        // 2 lists of hcap (v, slice) entries: vertices settled in a bucket
  unsigned hcap;
  long long m;
  int bin_thread;    // degree bins (BinW): lane bin up to this degree (<= kBinLane)
  int bin_wave;      // degree bins (BinW): wavefront bin up to this degree
  int pull;          // direction: kPullNever, kPullAlways or kPullHybrid
  int2* front;       // [n] pull, SSSP: (round stamp, distance) of the round's frontier vertices
  unsigned* fbits;   // [ceil(n / 32)] pull, k-core: bitmap of the vertices peeled in the round
  const int2* slices;  // pull: (base vertex, slice index) of every long row's slices
  // vertex blocks (BlockW only); a block's vertices occupy positions
  // bstart[b] .. bstart[b+1] of the blocked order
  const int* bstart;     // [nb + 1]
  const int4* bmeta;     // [nb] first position, vertices, first internal edge, internal edges
  const int* verts;      // [n] vertex at each position
  const int* blk_of;     // [n] block of each vertex
  const int* irow;       // [n + 1] internal edges of each position (offsets into iedge)
  const int* xrow;       // [n + 1] leaving edges of each position (offsets into xcol / xw / xblk)
  const unsigned* iedge;  // internal edges: local target | weight << 16
  const int* xcol;       // leaving edges: target vertex
  const int* xw;         //                weight
  const int* xblk;       //                target's block
  int* brel;             // [n] per position: the distance at which the vertex's edges were last relaxed
  unsigned* bstate;      // [nb] kBlkDirty / kBlkOwned
  unsigned long long* ring;  // [ring_mask + 1] queue of dirty blocks: (position << 32) | (block + 1),
                             // or (position << 32) once taken
  unsigned ring_mask;
  int nb;
};

// Per-thread event counts, 32 bits each (registers are what limits the
// persistent kernels' occupancy); round_barrier adds them to the 64-bit
// totals before any can pass 2^31.
struct Counters {
  unsigned relax = 0, improve = 0, push_local = 0, push_global = 0, far = 0, batches = 0;
  unsigned round_batches = 0;
};

struct Smem {
  int4 lq[kLq];        // local current bucket: (v, d, base row start, out-degree)
  int bstart[kBlock];  // batch: base row start, degree offset, distance, vertex,
  int boff[kBlock];    //        virtual offset of the vertex's copy
  int bd[kBlock];
  int bv[kBlock];
  int bvo[kBlock];
  int tb[kMaxQueries];  // per-query bound: current dist of the target
  int wsum[kWaves];
  unsigned lq_head, lq_tail, bhead;
  int mode, nb;
  unsigned gbase;
  int exhausted;
  int last;
  // snapshot of the control block for this round
  unsigned cur, in_count, win_hi, round, epoch, far_stamp;
  int in_kind, in_index, done, spill_out, far_out;
  int team, team_rank, team_size;  // this workgroup's team, its index in it, the team's workgroups
  int hout;       // light/heavy split
  unsigned hgen;  // light/heavy split
  int pull;       // this round pulls
  int flat_any;   // degree bins: the batch has rows for the workgroup bin (0 between batches)
};

// ------------------------------------------------- device-coherent access
// Data that one workgroup writes and another reads in a later round goes
// through device-scope (write-through / cache-bypassing) stores and loads,
// so a round boundary needs no cache write-back or invalidation: only the
// writer's completion wait before it arrives at the barrier.
__device__ __forceinline__ unsigned ld_dev(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int2 ld_entry(const int2* q, size_t i) {
  const unsigned long long x =
      __hip_atomic_load(reinterpret_cast<const unsigned long long*>(q + i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int)(unsigned)(x & 0xffffffffull), (int)(unsigned)(x >> 32));
}
__device__ __forceinline__ void st_entry(int2* q, size_t i, int v, int d) {
  const unsigned long long x = (unsigned long long)(unsigned)v | ((unsigned long long)(unsigned)d << 32);
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(q + i), x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until this wavefront's vector memory operations (stores and
// atomics included) have completed; also a compiler memory barrier.
__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }
__device__ __forceinline__ unsigned long long lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// query (copy) of a virtual vertex
__device__ __forceinline__ int query_of(const Args& a, int v) {
  return a.reps == 1 ? 0 : (int)((unsigned)v / (unsigned)a.nbase);
}

__device__ __forceinline__ unsigned sat_add(unsigned x, unsigned y) {
  return x > 0xffffffffu - y ? 0xffffffffu : x + y;
}

__device__ __forceinline__ void set_status(Ctl* c, int st) {
  atomicCAS(reinterpret_cast<int*>(&c->status.v), 0, st);
}

// Distance arithmetic.  Distances are stored as int32 bit patterns so that
// one 32-bit atomic minimum serves both kinds: non-negative int32 values, or
// non-negative float32 values (whose bit patterns order like the floats,
// with +inf = 0x7f800000 as the unreachable label).
struct IntW {
  static constexpr int kInfBits = INT_MAX;
  static constexpr bool kSplit = false;
  // process_batch takes batches of more than kBlock edges kEdgeIlp edges
  // per lane at a time (relax_wide); the plain int32 engine does without,
  // as the extra registers cost it a wavefront per SIMD on the road graphs
  static constexpr bool kWide = false;
  static constexpr bool kCore = false;
  static constexpr bool kPull = false;
  static constexpr bool kBin = false;
  static constexpr bool kBlocks = false;
  // nd = d + w; false (and a status) for a negative weight or a sum that
  // reaches INT32_MAX
  __device__ static bool add(const Args& a, int d, int wraw, int* nd) {
    if (wraw < 0) {
      set_status(a.ctl, OG_ERR_NEGATIVE_WEIGHT);
      return false;
    }
    const unsigned sum = (unsigned)d + (unsigned)wraw;
    if (sum >= (unsigned)INT_MAX) {
      set_status(a.ctl, OG_ERR_OVERFLOW);
      return false;
    }
    *nd = (int)sum;
    return true;
  }
  __device__ static bool tight(int du, int wraw, int dv) { return (unsigned)du + (unsigned)wraw == (unsigned)dv; }
  // the bit pattern dist[v] has when the edge is tight
  __device__ static unsigned cand(int du, int wraw) { return (unsigned)du + (unsigned)wraw; }
  // priority of vertex v at distance d: d, or d + h[v] for A*
  __device__ static unsigned key(const Args& a, int v, int d) {
    return a.h ? (unsigned)d + (unsigned)a.h[v] : (unsigned)d;  // both < 2^31: no wrap
  }
  __device__ static unsigned bucket(const Args& a, unsigned key) {
    return a.shift >= 0 ? (key >> a.shift) : (key / a.delta);
  }
};

struct FloatW {
  static constexpr int kInfBits = 0x7f800000;  // +inf
  static constexpr bool kSplit = false;
  static constexpr bool kWide = true;
  static constexpr bool kCore = false;
  static constexpr bool kPull = false;
  static constexpr bool kBin = false;
  static constexpr bool kBlocks = false;
  __device__ static bool add(const Args& a, int d, int wraw, int* nd) {
    const float w = __int_as_float(wraw);
    if (!(w >= 0.0f) || w == __int_as_float(kInfBits)) {  // negative, NaN or infinite
      set_status(a.ctl, OG_ERR_NEGATIVE_WEIGHT);
      return false;
    }
    const float sum = __fadd_rn(__int_as_float(d), w);
    if (sum == __int_as_float(kInfBits)) {
      set_status(a.ctl, OG_ERR_OVERFLOW);
      return false;
    }
    *nd = __float_as_int(sum);
    return true;
  }
  __device__ static bool tight(int du, int wraw, int dv) {
    return __fadd_rn(__int_as_float(du), __int_as_float(wraw)) == __int_as_float(dv);
  }
  // the bit pattern dist[v] has when the edge is tight (distances are never
  // -0, so equal values have equal bits)
  __device__ static unsigned cand(int du, int wraw) {
    return (unsigned)__float_as_int(__fadd_rn(__int_as_float(du), __int_as_float(wraw)));
  }
  __device__ static unsigned key(const Args&, int, int d) { return (unsigned)d; }
  // floor(d / Delta): the float64 quotient of two float32 values never
  // rounds across an integer, so this is the exact floor
  __device__ static unsigned bucket(const Args& a, unsigned key) {
    const double q = floor((double)__int_as_float((int)key) / (double)a.delta);
    return q >= 4294967294.0 ? 4294967294u : (unsigned)q;
  }
};

// k-core: the priority of a vertex is its remaining degree (the "dist"
// array is the priority vector), one bucket per value; no weights.
struct CoreW : IntW {
  static constexpr bool kCore = true;
};

// Light/heavy split (Meyer and Sanders' Delta-stepping; the paper relaxes
// every edge): int32 distances, rounds relax the light edges (w < Delta)
// only, and the heavy edges of the vertices settled in a bucket are relaxed
// once, in one extra round when the bucket is finished.  A separate
// instantiation, so the other engines' code is not touched by it.
struct SplitW : IntW {
  static constexpr bool kSplit = true;
  static constexpr bool kWide = true;
  __device__ static bool light(const Args& a, int wraw) { return wraw < (int)a.delta; }
};

// Direction optimisation with lazy updates (section 4.2, DensePull and the
// SparsePush-DensePull hybrid; section 5.1: no atomics on the destination).
// A pull round first marks its frontier in a dense per-vertex array; after a
// device-wide barrier every vertex that can still improve reads its own row
// as its in-edges (the graph is symmetric) and takes the best value offered
// by marked neighbours.  Separate instantiations of the int32 and k-core
// engines.
struct PullW : IntW {
  static constexpr bool kPull = true;
};
struct CorePullW : CoreW {
  static constexpr bool kPull = true;
};

// Degree-binned load balancing: within a batch, a vertex of at most
// bin_thread edges (<= kBinLane) is relaxed by kBinLane lanes of fixed
// slots, one of at most bin_wave edges by its wavefront, and larger ones by
// the whole workgroup (the flat expansion of the other instantiations).
// int32 distances.
struct BinW : IntW {
  static constexpr bool kBin = true;
};
struct BinFloatW : FloatW {
  static constexpr bool kBin = true;
};

// LDS-resident vertex blocks (bucket fusion at block granularity): the
// vertices are grouped into compact blocks of at most kBcap vertices whose
// distances, processed labels and internal edges a workgroup holds in LDS;
// a block's part of the current bucket is drained there with LDS atomics,
// and only edges leaving the block touch dist in HBM.  int32 distances.
struct BlockW : IntW {
  static constexpr bool kBlocks = true;
};

// List ids: team t's window slots t(K+4) + 0 .. K-1, spill lists + K, K+1,
// far lists + K+2, K+3.
__device__ __forceinline__ int list_of(const Args& a, int team, int kind, int index) {
  return team * (a.K + 4) + (kind == kInWin ? index : (kind == kInSpill ? a.K + index : a.K + 2 + index));
}
__device__ __forceinline__ unsigned* chunk_slot(const Args& a, int list, unsigned pos) {
  return reinterpret_cast<unsigned*>(a.ctab) + (size_t)list * a.tchunks + (pos >> kChunkLog);
}

// Entry pos of a list, written before the last device-wide barrier (so its
// chunk is in the table); a chunk the pool could not supply reads as no
// entry (the call has already failed).
__device__ __forceinline__ int2 load_at(const Args& a, int list, unsigned pos) {
  const int ch = (int)ld_dev(chunk_slot(a, list, pos));
  if (ch < 0) return make_int2(-1, 0);
  return ld_entry(a.pool, (size_t)ch * kChunk + (pos & (kChunk - 1)));
}

// Team t's share of the pool: chunks team_lo(t) .. team_lo(t + 1) - 1, and
// the same positions of the free stack.
__device__ __host__ __forceinline__ unsigned team_lo(unsigned chunks, int teams, int t) {
  return (unsigned)(((unsigned long long)t * chunks) / (unsigned)teams);
}

// Stores (v, d) at position pos (< cap) of a list.  The writer of a chunk's
// first position takes a chunk from its team's stack for it; writers of the
// chunk's other positions wait until the table names it (that writer
// reserved its position earlier and does not wait on anything).  False when
// the team's share was empty (OG_ERR_WORKSPACE is set).
__device__ bool store_at(const Args& a, int list, unsigned pos, int v, int d) {
  unsigned* slot = chunk_slot(a, list, pos);
  if ((pos & (kChunk - 1)) == 0) {
    const int t = list / (a.K + 4);
    const unsigned lo = team_lo(a.pool_chunks, a.teams, t);
    const int size = (int)(team_lo(a.pool_chunks, a.teams, t + 1) - lo);
    const int top = atomicSub(reinterpret_cast<int*>(&a.ctl->free_top[t].v), 1) - 1;
    int ch = kLostChunk;
    if (top >= 0 && top < size) ch = (int)ld_dev(reinterpret_cast<const unsigned*>(a.fstack) + lo + top);
    else set_status(a.ctl, OG_ERR_WORKSPACE);
    st_dev(slot, (unsigned)ch);
  }
  int ch;
  for (unsigned spin = 0; (ch = (int)ld_dev(slot)) == kNoChunk; ++spin) {
    if (spin == kChunkSpinLimit) {
      set_status(a.ctl, OG_ERR_INTERNAL);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (ch < 0) return false;
  st_entry(a.pool, (size_t)ch * kChunk + (pos & (kChunk - 1)), v, d);
  return true;
}

// Block-wide exclusive prefix sum of x; *total receives the sum.  The
// per-wave totals are reused only after the caller's next barrier.
__device__ int block_excl_scan(int x, Smem& s, int* total) {
  const int lane = (int)lane_id(), wid = threadIdx.x / kWave;
  int v = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) s.wsum[wid] = v;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    int t = s.wsum[i];
    pre += i < wid ? t : 0;
    tot += t;
  }
  *total = tot;
  return pre + v - x;
}

// Wave-cooperative append of (v, d) entries to global queues.  Targets:
// 0..K-1 window slots, K = this round's spill list, K+1 = far list.  All 64
// lanes must call it together.  One atomic per wavefront and target reserves
// the slots.  A full window slot or spill list falls back to the far list;
// a full far list sets OG_ERR_WORKSPACE and drops the entry.
template <class S>
__device__ void wave_push_global(const Args& a, const S& s, Counters& c, bool has, int tgt, int v, int d,
                                 unsigned b) {
  Ctl* ctl = a.ctl;
  const int K = a.K;
  if (a.teams > 1 && has && query_of(a, v) % a.teams != s.team) {  // another team's vertex: a library bug
    set_status(ctl, OG_ERR_INTERNAL);
    has = false;
  }
  for (;;) {
    const unsigned long long m = __ballot(has);
    if (m == 0) break;
    const int leader = __ffsll((long long)m) - 1;
    const int t = __shfl(tgt, leader);
    const bool mine = has && tgt == t;
    const unsigned long long mm = __ballot(mine);
    TeamQ& q = ctl->tq[s.team];
    unsigned* tail;
    int list;
    if (t < K) {
      tail = &q.win_tail[t].v;
      list = list_of(a, s.team, kInWin, t);
    } else if (t == K) {
      tail = &q.spill_tail[s.spill_out].v;
      list = list_of(a, s.team, kInSpill, s.spill_out);
    } else {
      tail = &q.far_tail[s.far_out].v;
      list = list_of(a, s.team, kInFar, s.far_out);
    }
    unsigned base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(tail, (unsigned)__popcll(mm));
    base = __shfl(base, leader);
    if (mine) {
      const unsigned pos = base + (unsigned)__popcll(mm & lanemask_lt());
      if (pos < a.cap && pos >= base) {
        if (store_at(a, list, pos, v, d)) {
          c.push_global++;
          if (t == K + 1) {
            c.far++;
            atomicMin(&q.far_min[s.far_out].v, b);
          }
        }
        has = false;
      } else if (t == K + 1) {
        set_status(ctl, OG_ERR_WORKSPACE);
        has = false;
      } else {
        tgt = K + 1;
      }
    }
  }
}

// Lazy update: appends the lanes' vertices to the change buffer (one atomic
// per wavefront).  Each vertex is appended at most once per round (the
// caller holds its flag), so the buffer never exceeds n entries.
__device__ void wave_append_buf(const Args& a, bool has, int v) {
  const unsigned long long m = __ballot(has);
  if (m == 0) return;
  const int leader = __ffsll((long long)m) - 1;
  unsigned base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(&a.ctl->buf_tail.v, (unsigned)__popcll(m));
  base = __shfl(base, leader);
  if (has) {
    const unsigned pos = base + (unsigned)__popcll(m & lanemask_lt());
    if (pos < a.buf_cap) st_dev(reinterpret_cast<unsigned*>(a.buf) + pos, (unsigned)v);
    else set_status(a.ctl, OG_ERR_WORKSPACE);
  }
}

// Light/heavy split: files the lanes' vertices (processed in the current
// bucket, with heavy edges) in the pending heavy list, each at most once per
// list (the generation stamp in hmark).  The stamp is per list, not per
// bucket: with an A* estimate a heavy edge can lead back into the current
// bucket, so a vertex whose heavy edges were relaxed in the bucket's heavy
// round can improve again and must be filed again.  nheavy: the heavy
// part's length when known (more than kHeavySlice: one entry per slice),
// else -1.  One atomic per wavefront.
__device__ void wave_append_heavy(const Args& a, const Smem& s, bool has, int v, int nheavy) {
  const unsigned stamp = s.hgen + 1u;
  if (has) has = atomicMax(&a.hmark[v], stamp) < stamp;
  if (__ballot(has) == 0) return;
  const int nsl = !has ? 0 : (nheavy > kHeavySlice ? (nheavy + kHeavySlice - 1) / kHeavySlice : 1);
  const int lane = (int)lane_id();
  int inc = nsl;  // inclusive scan of the entry counts over the wavefront
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  const int total = __shfl(inc, kWave - 1);
  unsigned base = 0;
  if (lane == 0) base = atomicAdd(&a.ctl->heavy_tail[s.hout].v, (unsigned)total);
  base = __shfl(base, 0);
  const unsigned first = base + (unsigned)(inc - nsl);
  for (int k = 0; k < nsl; ++k) {
    const unsigned pos = first + (unsigned)k;
    if (pos < a.hcap) st_entry(a.heavy + (size_t)s.hout * a.hcap, pos, v, nsl > 1 ? k : -1);
    else set_status(a.ctl, OG_ERR_WORKSPACE);
  }
}

// Routes one improved vertex per lane: the current bucket goes to the LDS
// ring when fusing, together with its CSR row so the next hop needs no row
// lookup (falling back to the spill list when the ring is full); later
// buckets go to their window slot or the far list.
__device__ void route_push(const Args& a, Smem& s, Counters& c, bool has, int v, int d, unsigned b, int r0,
                           int deg) {
  const unsigned cur = s.cur;
  const bool local = has && a.fused && b == cur;
  const unsigned long long m = __ballot(local);
  if (m) {
    const int leader = __ffsll((long long)m) - 1;
    unsigned base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(&s.lq_tail, (unsigned)__popcll(m));
    base = __shfl(base, leader);
    if (local) {
      const unsigned pos = base + (unsigned)__popcll(m & lanemask_lt());
      if (pos - s.lq_head < (unsigned)kLq) {
        s.lq[pos & (kLq - 1)] = make_int4(v, d, r0, deg);
        c.push_local++;
        has = false;
      }
    }
  }
  int tgt = 0;
  if (has) tgt = b == cur ? a.K : (b < s.win_hi ? (int)(b & (unsigned)(a.K - 1)) : a.K + 1);
  wave_push_global(a, s, c, has, tgt, v, d, b);
}

// The edge loop of process_batch for a batch of more than kBlock edges
// (throughput-bound: every edge is filtered by a plain load of dist[u]).
// Each lane takes kEdgeIlp edges per step and keeps their loads, filter
// reads and atomics in flight together; the improved vertices are then
// filed as by process_batch.  The batch arrays (boff, bstart, bd, bv, bvo)
// are in place.
template <class W>
__device__ void relax_wide(const Args& a, Smem& s, Counters& c, bool from_lds, int total, int nb, unsigned cur) {
  const int tid = threadIdx.x;
  for (int base = 0; base < total; base += kBlock * kEdgeIlp) {
    int u[kEdgeIlp], ub[kEdgeIlp], wt[kEdgeIlp], ds[kEdgeIlp], dn[kEdgeIlp], cu[kEdgeIlp], old[kEdgeIlp];
    unsigned nd[kEdgeIlp], b[kEdgeIlp];
    bool go[kEdgeIlp];
#pragma unroll
    for (int j = 0; j < kEdgeIlp; ++j) {  // edge loads
      const int e = base + j * kBlock + tid;
      go[j] = e < total;
      u[j] = ub[j] = wt[j] = ds[j] = dn[j] = 0;
      if (go[j]) {
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s.boff[mid] <= e) lo = mid;
          else hi = mid - 1;
        }
        const int edge = s.bstart[lo] + (e - s.boff[lo]);
        ds[j] = s.bd[lo];
        ub[j] = W::kSplit ? a.ecol[edge] : a.col[edge];
        wt[j] = W::kSplit ? a.ew[edge] : a.w[edge];
        dn[j] = from_lds ? a.dist[s.bv[lo]] : ds[j];
        u[j] = ub[j] + s.bvo[lo];
      }
    }
#pragma unroll
    for (int j = 0; j < kEdgeIlp; ++j) {  // new distances, then the filter reads
      nd[j] = b[j] = 0;
      cu[j] = 0;
      if (go[j]) {
        c.relax++;
        int ndi = 0;
        go[j] = ds[j] <= dn[j] && W::add(a, ds[j], wt[j], &ndi);
        if (go[j]) {
          nd[j] = (unsigned)ndi;
          const unsigned key = W::key(a, u[j], ndi);
          go[j] = !(a.tgts && key >= (unsigned)s.tb[query_of(a, u[j])]);  // cannot improve the target
          b[j] = W::bucket(a, key);
          if (b[j] < cur) b[j] = cur;  // only an inconsistent A* estimate gets here
          if (go[j]) cu[j] = a.dist[u[j]];
        }
      }
    }
    long long q0[kEdgeIlp], q1[kEdgeIlp];
    int ql[kEdgeIlp];
#pragma unroll
    for (int j = 0; j < kEdgeIlp; ++j) {  // the atomics (with the chased rows)
      q0[j] = q1[j] = 0;
      ql[j] = 0;
      old[j] = 0;
      go[j] = go[j] && (int)nd[j] < cu[j];
      if (go[j]) {
        if (a.fused && b[j] == cur) {
          q0[j] = a.row_ptr[ub[j]];
          q1[j] = a.row_ptr[ub[j] + 1];
          if constexpr (W::kSplit) ql[j] = a.lsplit[ub[j]];
        }
        old[j] = atomicMin(&a.dist[u[j]], (int)nd[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < kEdgeIlp; ++j) {  // file the improved vertices
      const bool has = go[j] && (int)nd[j] < old[j];
      int r0 = 0, rdeg = 0;
      if (has) {
        c.improve++;
        r0 = (int)q0[j];
        rdeg = (int)(q1[j] - q0[j]);
        if constexpr (W::kSplit) rdeg = ql[j] | (rdeg > ql[j] ? kHeavyBit : 0);
      }
      if (a.lazy) {
        const bool first = has && atomicExch(&a.aux[u[j]], 1) == 0;
        wave_append_buf(a, first, u[j]);
      } else {
        route_push(a, s, c, has, u[j], (int)nd[j], b[j], r0, rdeg);
      }
    }
  }
}

// Relaxes the out-edges of one batch of up to kBlock entries; lane i holds
// entry i (v < 0: none).  Edges of the batch are spread evenly over the
// workgroup (flat expansion with a binary search over degree offsets), so a
// high-degree vertex is shared by all lanes.
//
// from_lds: entries come from the local ring and carry their CSR row.  The
// staleness check (d > dist[v]) is then made per edge, with the dist load
// issued together with the edge loads; a small batch then needs two
// dependent global round trips per hop (edge loads, then the atomic
// together with the next vertex's row).  Otherwise (a global list) the row
// is looked up per entry.
//
// SplitW (light/heavy split): an ordinary round relaxes a vertex's light
// edges and files the vertex (once per bucket) for the bucket's heavy round;
// the heavy round (input kind kInHeavy) relaxes the heavy part of each filed
// vertex's row at its final distance.  Rows and list entries are checked on
// this path: a violated bound is OG_ERR_INTERNAL, never an access.
template <class W>
__device__ void process_batch(const Args& a, Smem& s, Counters& c, int4 ent, bool from_lds) {
  const int tid = threadIdx.x;
  const int v = ent.x;
  // a heavy-round entry uses the vertex's final distance
  const int d = W::kSplit && v >= 0 && !from_lds && s.in_kind == kInHeavy
                    ? (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + v)
                    : ent.y;
  int deg = 0, start = 0, voff = 0, nheavy = -1;
  bool repush = false, settle = false;
  unsigned rb = 0;
  if (v >= 0) {
    const int vb = a.reps == 1 ? v : (int)((unsigned)v % (unsigned)a.nbase);
    voff = v - vb;
    if (from_lds) {
      start = ent.z;
      if constexpr (W::kSplit) {
        deg = ent.w & kDegMask;
        settle = (ent.w & kHeavyBit) != 0;
      } else {
        deg = ent.w;
      }
    } else if (W::kSplit && s.in_kind == kInHeavy) {
      // the bucket is finished: the heavy part of the vertex's row, or its
      // slice ent.y
      const long long r0 = a.row_ptr[vb];
      const long long r1 = a.row_ptr[vb + 1];
      const int l = a.lsplit[vb];
      start = (int)r0 + l;
      deg = (int)(r1 - r0) - l;
      if (ent.y >= 0) {
        const long long skip = (long long)ent.y * kHeavySlice;
        start += (int)(skip < deg ? skip : deg);
        deg = skip < deg ? (deg - (int)skip < kHeavySlice ? deg - (int)skip : kHeavySlice) : -1;
      }
    } else {
      // issued together: the staleness check does not delay the row lookup
      const int cv = a.dist[v];
      const long long r0 = a.row_ptr[vb];
      const long long r1 = a.row_ptr[vb + 1];
      int l = 0;
      if constexpr (W::kSplit) l = a.lsplit[vb];
      const unsigned key = W::key(a, v, d);
      bool live = d <= cv;
      if (live) {
        rb = W::bucket(a, key);
        if (rb > s.cur) {
          repush = true;  // a far-list entry that belongs to a later bucket
          live = false;
        }
      }
      if (live && a.tgts && key >= (unsigned)s.tb[query_of(a, v)]) live = false;  // cannot improve the target
      if (live) {
        start = (int)r0;
        if constexpr (W::kSplit) {
          deg = l;
          settle = (int)(r1 - r0) > l;
          nheavy = (int)(r1 - r0) - l;
        } else {
          deg = (int)(r1 - r0);
        }
      }
    }
    if constexpr (W::kSplit) {
      if ((unsigned)v >= (unsigned)a.n || start < 0 || deg < 0 || (long long)start + deg > a.m) {
        set_status(a.ctl, OG_ERR_INTERNAL);
        deg = 0;
        settle = false;
        repush = false;
      }
    }
  }
  {
    int tgt = 0;
    if (repush) tgt = rb < s.win_hi ? (int)(rb & (unsigned)(a.K - 1)) : a.K + 1;
    wave_push_global(a, s, c, repush, tgt, v, d, rb);
  }
  if constexpr (W::kSplit) wave_append_heavy(a, s, settle, v, nheavy);  // heavy edges wait for the bucket's end
  int total;
  const int off = block_excl_scan(deg, s, &total);
  s.boff[tid] = off;
  s.bstart[tid] = start;
  s.bd[tid] = d;
  s.bv[tid] = v;
  s.bvo[tid] = voff;
  __syncthreads();
  const int nb = s.nb;
  const unsigned cur = s.cur;
  // A plain load of dist[u] skips atomics that cannot succeed.  It costs a
  // dependent round trip, so a small locally chased batch of one query
  // (latency-bound, one pass over its edges) goes straight to the atomic;
  // larger batches and batched launches (throughput-bound) filter.
  const bool prefilter = !from_lds || total > kBlock || a.reps > 1;
  if constexpr (W::kWide) {
    if (total > kBlock) {
      relax_wide<W>(a, s, c, from_lds, total, nb, cur);
      return;
    }
  }
  for (int base = 0; base < total; base += kBlock) {
    const int e = base + tid;
    bool has = false;
    int u = 0, r0 = 0, rdeg = 0;
    unsigned nd = 0, b = 0;
    if (e < total) {
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.boff[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      const int edge = s.bstart[lo] + (e - s.boff[lo]);
      const int dsrc = s.bd[lo];
      const int ub = W::kSplit ? a.ecol[edge] : a.col[edge];
      const int wt = W::kSplit ? a.ew[edge] : a.w[edge];
      const int dnow = from_lds ? a.dist[s.bv[lo]] : dsrc;
      u = ub + s.bvo[lo];
      c.relax++;
      int ndi = 0;
      if (dsrc <= dnow && W::add(a, dsrc, wt, &ndi)) {
        nd = (unsigned)ndi;
        const unsigned key = W::key(a, u, ndi);
        bool go = !(a.tgts && key >= (unsigned)s.tb[query_of(a, u)]);  // cannot improve the target
        if (go && prefilter) go = (int)nd < a.dist[u];
        if (go) {
          b = W::bucket(a, key);
          if (b < cur) b = cur;  // only an inconsistent A* estimate gets here
          long long q0 = 0, q1 = 0;
          int ql = 0;
          const bool chase = a.fused && b == cur;
          if (chase) {  // the next hop's row, fetched alongside the atomic
            q0 = a.row_ptr[ub];
            q1 = a.row_ptr[ub + 1];
            if constexpr (W::kSplit) ql = a.lsplit[ub];
          }
          const int old = atomicMin(&a.dist[u], (int)nd);
          if ((int)nd < old) {
            c.improve++;
            has = true;
            r0 = (int)q0;
            rdeg = (int)(q1 - q0);
            if constexpr (W::kSplit) rdeg = ql | (rdeg > ql ? kHeavyBit : 0);
          }
        }
      }
    }
    if (a.lazy) {
      // record the change once per round; its bucket is filed after the round
      const bool first = has && atomicExch(&a.aux[u], 1) == 0;
      wave_append_buf(a, first, u);
    } else {
      route_push(a, s, c, has, u, (int)nd, b, r0, rdeg);
    }
  }
}

// One edge of the binned routine (the same steps as the edge loop of
// process_batch): u = ub + voff, entry distance dsrc, the vertex's current
// distance dnow (the per-edge staleness check of ring entries).  Returns
// whether the atomic minimum improved u; *nd, *b, *r0, *rdeg as for
// route_push.
template <class W>
__device__ __forceinline__ bool relax_edge(const Args& a, const Smem& s, Counters& c, int ub, int wt, int dsrc,
                                           int dnow, int u, bool prefilter, unsigned* nd, unsigned* b, int* r0,
                                           int* rdeg) {
  c.relax++;
  int ndi = 0;
  if (!(dsrc <= dnow && W::add(a, dsrc, wt, &ndi))) return false;
  *nd = (unsigned)ndi;
  const unsigned key = W::key(a, u, ndi);
  bool go = !(a.tgts && key >= (unsigned)s.tb[query_of(a, u)]);  // cannot improve the target
  if (go && prefilter) go = ndi < a.dist[u];
  if (!go) return false;
  unsigned bk = W::bucket(a, key);
  if (bk < s.cur) bk = s.cur;  // only an inconsistent A* estimate gets here
  *b = bk;
  long long q0 = 0, q1 = 0;
  if (a.fused && bk == s.cur) {  // the next hop's row, fetched alongside the atomic
    q0 = a.row_ptr[ub];
    q1 = a.row_ptr[ub + 1];
  }
  const int old = atomicMin(&a.dist[u], ndi);
  if (ndi >= old) return false;
  c.improve++;
  *r0 = (int)q0;
  *rdeg = (int)(q1 - q0);
  return true;
}

// Files the lanes' improved vertices (all 64 lanes call it together): lazy
// update records them, eager update routes them.
__device__ __forceinline__ void finish_edges(const Args& a, Smem& s, Counters& c, bool has, int u, unsigned nd,
                                             unsigned b, int r0, int rdeg) {
  if (a.lazy) {
    const bool first = has && atomicExch(&a.aux[u], 1) == 0;
    wave_append_buf(a, first, u);
  } else {
    route_push(a, s, c, has, u, (int)nd, b, r0, rdeg);
  }
}

// process_batch with degree bins (BinW).  The entry checks are those of
// process_batch.  Then:
//   - lane bin (degree <= bin_thread): kBinLane lanes per vertex, one edge
//     each, found by a division instead of a scan and a search;
//   - wavefront bin (degree <= bin_wave): each wavefront takes the bin's
//     vertices of its own 64 lanes (no workgroup barrier) and relaxes each
//     row 64 edges at a time;
//   - workgroup bin: the remaining rows are expanded over the workgroup by
//     a block scan and a binary search, as in process_batch.
template <class W>
__device__ void process_batch_binned(const Args& a, Smem& s, Counters& c, int4 ent, bool from_lds, int nb,
                                     unsigned new_head, bool advance) {
  const int tid = threadIdx.x;
  const int v = ent.x;
  const int d = ent.y;
  int deg = 0, start = 0, voff = 0;
  bool repush = false;
  unsigned rb = 0;
  if (v >= 0) {
    const int vb = a.reps == 1 ? v : (int)((unsigned)v % (unsigned)a.nbase);
    voff = v - vb;
    if (from_lds) {
      start = ent.z;
      deg = ent.w;
    } else {
      const int cv = a.dist[v];
      const long long r0 = a.row_ptr[vb];
      const long long r1 = a.row_ptr[vb + 1];
      const unsigned key = W::key(a, v, d);
      bool live = d <= cv;
      if (live) {
        rb = W::bucket(a, key);
        if (rb > s.cur) {
          repush = true;  // a far-list entry that belongs to a later bucket
          live = false;
        }
      }
      if (live && a.tgts && key >= (unsigned)s.tb[query_of(a, v)]) live = false;  // cannot improve the target
      if (live) {
        start = (int)r0;
        deg = (int)(r1 - r0);
      }
    }
  }
  {
    int tgt = 0;
    if (repush) tgt = rb < s.win_hi ? (int)(rb & (unsigned)(a.K - 1)) : a.K + 1;
    wave_push_global(a, s, c, repush, tgt, v, d, rb);
  }
  const int lane_max = a.bin_thread < kBinLane ? a.bin_thread : kBinLane;
  const bool in_lane = deg > 0 && deg <= lane_max;
  const bool in_wave = deg > lane_max && deg <= a.bin_wave;
  // The plain-load filter (an atomic only where dist[u] still looks larger)
  // is used for global entries, and for every entry of a batched launch:
  // with several queries in flight the device-scope atomics queue at the
  // memory side and dropping the hopeless ones pays; for one query the
  // filter's extra dependent load only lengthens the ring's chain.
  const bool prefilter = !from_lds || a.reps > 1;
  // Ring entries get their staleness check per edge: the vertex's current
  // distance is loaded together with the edge (global entries were checked
  // above).

  // lane bin: kBinLane lanes per vertex, slot e = kBinLane * (entry index)
  // + k holds edge k of that entry (no scan, no search), so every edge of
  // the bin is in flight at once.  The batch arrays hold every entry's row
  // start, distance, vertex and offset for all three bins; boff holds the
  // lane bin's degrees (a wavefront-bin entry: minus its degree).
  const int dflat = in_lane || in_wave ? 0 : deg;
  s.bstart[tid] = start;
  s.boff[tid] = in_lane ? deg : (in_wave ? -deg : 0);
  s.bd[tid] = d;
  s.bv[tid] = v;
  s.bvo[tid] = voff;
  // whether any row is left to the workgroup bin: set by the wavefronts
  // that have one before the barrier, read at the workgroup bin, cleared
  // after the next barrier (nothing writes it in between)
  if (__ballot(dflat > 0) && lane_id() == 0) s.flat_any = 1;
  __syncthreads();
  // a batch taken from the ring by every lane alike: its entries are consumed
  // only now, when every lane has read the ring pointers
  if (advance && tid == 0) s.lq_head = new_head;
  {
    const int slots = nb * kBinLane;
    for (int base = 0; base < slots; base += kBlock) {
      const int e = base + tid;
      const int j = e / kBinLane, k = e % kBinLane;
      bool has = false;
      int u = 0, r0 = 0, rdeg = 0;
      unsigned nd = 0, b = 0;
      if (e < slots && k < s.boff[j]) {
        const int edge = s.bstart[j] + k;
        const int ubk = a.col[edge];
        const int wk = a.w[edge];
        const int dn = from_lds ? a.dist[s.bv[j]] : s.bd[j];
        u = ubk + s.bvo[j];
        has = relax_edge<W>(a, s, c, ubk, wk, s.bd[j], dn, u, prefilter, &nd, &b, &r0, &rdeg);
      }
      finish_edges(a, s, c, has, u, nd, b, r0, rdeg);
    }
  }

  // wavefront bin: the wavefront takes the bin's vertices of its own 64
  // lanes one at a time, each vertex's fields read once into scalar
  // registers (no further workgroup barrier)
  {
    const int wbase = (tid / kWave) * kWave;
    unsigned long long wm = __ballot(in_wave);
    while (wm) {
      const int j = wbase + __ffsll((long long)wm) - 1;
      wm &= wm - 1;
      const int e0 = __builtin_amdgcn_readfirstlane(s.bstart[j]);
      const int dg = -__builtin_amdgcn_readfirstlane(s.boff[j]);
      const int dj = __builtin_amdgcn_readfirstlane(s.bd[j]);
      const int vj = __builtin_amdgcn_readfirstlane(s.bv[j]);
      const int vo = __builtin_amdgcn_readfirstlane(s.bvo[j]);
      for (int it = 0; it < dg; it += kWave) {
        const int k = it + (int)lane_id();
        unsigned nd = 0, b = 0;
        int r0 = 0, rdeg = 0, u = 0;
        bool has = false;
        if (k < dg) {
          const int ubk = a.col[e0 + k];
          const int wk = a.w[e0 + k];
          const int dn = from_lds ? a.dist[vj] : dj;
          u = ubk + vo;
          has = relax_edge<W>(a, s, c, ubk, wk, dj, dn, u, prefilter, &nd, &b, &r0, &rdeg);
        }
        finish_edges(a, s, c, has, u, nd, b, r0, rdeg);
      }
    }
  }

  // workgroup bin: flat expansion of the remaining rows
  if (!s.flat_any) return;
  int total;
  const int off = block_excl_scan(dflat, s, &total);  // its barrier also ends the lane bin's use of the arrays
  if (tid == 0) s.flat_any = 0;  // every lane has read it before that barrier
  if (total == 0) return;
  s.boff[tid] = off;  // row start, distance, vertex and offset are in place from the lane bin
  __syncthreads();
  for (int base = 0; base < total; base += kBlock) {
    const int e = base + tid;
    bool has = false;
    int u = 0, r0 = 0, rdeg = 0;
    unsigned nd = 0, b = 0;
    if (e < total) {
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.boff[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      const int edge = s.bstart[lo] + (e - s.boff[lo]);
      const int dsrc = s.bd[lo];
      const int ubk = a.col[edge];
      const int wk = a.w[edge];
      const int dn = from_lds ? a.dist[s.bv[lo]] : dsrc;
      u = ubk + s.bvo[lo];
      has = relax_edge<W>(a, s, c, ubk, wk, dsrc, dn, u, !from_lds || total > kBlock || a.reps > 1, &nd, &b,
                          &r0, &rdeg);
    }
    finish_edges(a, s, c, has, u, nd, b, r0, rdeg);
  }
}

// k-core filing of vertex u at priority p (> the current level, or equal to
// it for the current bucket).  A priority at or beyond the window goes to
// the far list only if u is not already filed in that list (the far list is
// re-read by current priority when it is redistributed), so it holds each
// vertex at most once; far_min still records p.  A peeled vertex (mark
// kPeeled, above every generation) is never filed there again.
__device__ void route_core(const Args& a, Smem& s, Counters& c, bool has, int u, int p, int r0, int deg) {
  if (has && (unsigned)p >= s.win_hi) {
    atomicMin(&a.ctl->tq[s.team].far_min[s.far_out].v, (unsigned)p);
    if (atomicMax(&a.mark[u], (int)s.far_stamp) >= (int)s.far_stamp) has = false;
  }
  route_push(a, s, c, has, u, p, (unsigned)p, r0, deg);
}

// k-core frontier batch (section 6.1 peeling at level k = current bucket).
// An entry (v, p) is live when v is not yet peeled and its current degree
// equals k; the peel mark (kPeeled) makes each vertex peel once even if it
// was filed more than once.  An entry whose vertex now has a larger
// degree (a far-list entry being redistributed) is filed by that degree.
// Every edge of a peeled vertex lowers the neighbour's degree if it is above
// k: lazily (count it; the change is applied once after the round) or
// eagerly (compare-and-swap one lower, never below k, and file it).
__device__ void process_batch_core(const Args& a, Smem& s, Counters& c, int4 ent, bool from_lds) {
  const int tid = threadIdx.x;
  const unsigned cur = s.cur;
  const int v = ent.x;
  int deg = 0, start = 0, now = 0;
  bool refile = false;
  if (v >= 0) {
    now = (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + v);
    const int mk = (int)ld_dev(reinterpret_cast<const unsigned*>(a.mark) + v);
    if (mk != kPeeled) {
      if ((unsigned)now == cur) {
        if (atomicExch(&a.mark[v], kPeeled) != kPeeled) {  // peel v at level cur
          if (from_lds) {
            start = ent.z;
            deg = ent.w;
          } else {
            const long long r0 = a.row_ptr[v];
            start = (int)r0;
            deg = (int)(a.row_ptr[v + 1] - r0);
          }
        }
      } else if ((unsigned)now > cur) {
        refile = true;
      }
    }
  }
  route_core(a, s, c, refile, v, now, 0, 0);
  int total;
  const int off = block_excl_scan(deg, s, &total);
  s.boff[tid] = off;
  s.bstart[tid] = start;
  __syncthreads();
  const int nb = s.nb;
  for (int base = 0; base < total; base += kBlock) {
    const int e = base + tid;
    bool has = false;
    int u = 0, nd = 0, r0 = 0, rdeg = 0;
    if (e < total) {
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.boff[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      u = a.col[s.bstart[lo] + (e - s.boff[lo])];
      c.relax++;
      int du = a.dist[u];  // a past value: never below the current one
      if (du > (int)cur) {
        if (a.lazy) {
          has = atomicAdd(&a.aux[u], 1) == 0;  // first count of u this round
        } else {
          while (du > (int)cur) {
            const int old = atomicCAS(&a.dist[u], du, du - 1);
            if (old == du) {
              has = true;
              nd = du - 1;
              break;
            }
            du = old;
          }
          if (has) {
            c.improve++;
            if (a.fused && (unsigned)nd == cur) {
              const long long q0 = a.row_ptr[u];
              r0 = (int)q0;
              rdeg = (int)(a.row_ptr[u + 1] - q0);
            }
          }
        }
      }
    }
    if (a.lazy) wave_append_buf(a, has, u);
    else route_core(a, s, c, has, u, nd, r0, rdeg);
  }
}

// Second phase of a lazy round (section 3.1, reduce the buffered updates and
// file them in bulk): every vertex recorded in the change buffer is filed
// once, by its final priority.  SSSP: the final distance's bucket.  k-core
// (constant-sum reduction, section 5.1): the degree drops by the number of
// peeled neighbours counted in the round, clamped at the current level.
template <class W>
__device__ void run_flush(const Args& a, Smem& s, Counters& c) {
  if constexpr (W::kPull && W::kCore) {
    if (s.pull) {  // the pull phase is over: clear the bitmap of peeled vertices
      const unsigned words = ((unsigned)a.n + 31u) / 32u;
      for (unsigned i = blockIdx.x * (unsigned)kBlock + threadIdx.x; i < words; i += (unsigned)a.nwg * kBlock)
        st_dev(a.fbits + i, 0u);
    }
  }
  const unsigned cnt0 = ld_dev(&a.ctl->buf_tail.v);
  const unsigned cnt = cnt0 < a.buf_cap ? cnt0 : a.buf_cap;
  const unsigned cur = s.cur;
  for (unsigned base = blockIdx.x * (unsigned)kBlock; base < cnt; base += (unsigned)a.nwg * kBlock) {
    const unsigned i = base + threadIdx.x;
    bool has = false;
    int u = 0, d = 0;
    unsigned b = 0;
    if (i < cnt) {
      u = (int)ld_dev(reinterpret_cast<const unsigned*>(a.buf) + i);
      if constexpr (W::kCore) {
        const int k = atomicExch(&a.aux[u], 0);
        const int now = (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + u);
        if (now > (int)cur) {
          d = now - k > (int)cur ? now - k : (int)cur;
          st_dev(reinterpret_cast<unsigned*>(a.dist) + u, (unsigned)d);
          has = true;
          c.improve++;
        }
      } else {
        st_dev(reinterpret_cast<unsigned*>(a.aux) + u, 0u);
        d = (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + u);
        b = W::bucket(a, W::key(a, u, d));
        if (b < cur) b = cur;
        has = true;
      }
    }
    if constexpr (W::kCore) {
      route_core(a, s, c, has, u, d, 0, 0);
    } else {
      int tgt = 0;
      if (has) tgt = b == cur ? a.K : (b < s.win_hi ? (int)(b & (unsigned)(a.K - 1)) : a.K + 1);
      wave_push_global(a, s, c, has, tgt, u, d, b);
    }
  }
}

// Publishes the LDS ring (the local current bucket) to the global spill
// list so the next round spreads it over all workgroups (section 3.3: a
// local bucket at or above the threshold is copied to the global bucket).
__device__ void publish_local(const Args& a, Smem& s, Counters& c) {
  const int tid = threadIdx.x;
  const unsigned h = s.lq_head, cnt = s.lq_tail - s.lq_head;
  if (tid == 0) s.gbase = atomicAdd(&a.ctl->tq[s.team].spill_tail[s.spill_out].v, cnt);
  __syncthreads();
  const unsigned gb = s.gbase;
  const int list = list_of(a, s.team, kInSpill, s.spill_out);
  for (unsigned i0 = 0; i0 < cnt; i0 += kBlock) {
    const unsigned i = i0 + tid;
    bool spill_far = false;
    int4 e = make_int4(0, 0, 0, 0);
    if (i < cnt) {
      e = s.lq[(h + i) & (kLq - 1)];
      const unsigned pos = gb + i;
      if (pos < a.cap && pos >= gb) {
        if (store_at(a, list, pos, e.x, e.y)) c.push_global++;
      } else {
        spill_far = true;
      }
    }
    wave_push_global(a, s, c, spill_far, a.K + 1, e.x, e.y, s.cur);
  }
  __syncthreads();
  if (tid == 0) s.lq_head = s.lq_tail = 0;
}

// Thread 0 takes the workgroup's next share of its team's round input:
// an input that fits in one batch per workgroup of the team is split
// statically (the team's b-th workgroup takes the b-th slice, no atomics);
// a larger one is handed out in kBlock chunks through the team's cursor.
// Sets s.mode = 2 with s.nb entries from s.gbase, or s.exhausted.
template <class S>
__device__ void take_input(const Args& a, S& s) {
  const unsigned count = s.in_count, tsize = (unsigned)s.team_size;
  const bool fixed = count <= tsize * (unsigned)kBlock;
  const unsigned per = fixed ? (count + tsize - 1) / tsize : (unsigned)kBlock;
  unsigned base;
  if (fixed) {
    base = (unsigned)s.team_rank * per;
    s.exhausted = 1;
  } else {
    base = atomicAdd(&a.ctl->tq[s.team].in_head.v, (unsigned)kBlock);
  }
  if (base < count) {
    s.mode = 2;
    const unsigned left = count - base;
    s.nb = (int)(left < per ? left : per);
    s.gbase = base;
  } else {
    s.exhausted = 1;
  }
}

// One round: the round input list, then (fused) the local current bucket.
// A round input that fits in one batch per workgroup is split statically
// (workgroup b takes the b-th slice, no atomics); a larger one is handed
// out in kBlock chunks through an atomic cursor.
template <class W>
__device__ void run_round(const Args& a, Smem& s, Counters& c) {
  const int tid = threadIdx.x;
  // the round input: a heavy list (light/heavy split) or a pooled list
  const int2* hin = W::kSplit && s.in_kind == kInHeavy ? a.heavy + (size_t)s.in_index * a.hcap : nullptr;
  if (tid == 0) {
    s.lq_head = s.lq_tail = 0;
    s.exhausted = 0;
  }
  for (;;) {
    // (ring pushes of the previous batch are complete: end-of-batch barrier)
    __syncthreads();
    if (tid == 0) {
      if (s.lq_tail - s.lq_head > (unsigned)kLq) s.lq_tail = s.lq_head + kLq;  // burned reservations
      const unsigned lsize = s.lq_tail - s.lq_head;
      s.mode = 0;
      if (lsize > 0 && lsize >= a.threshold) {
        s.mode = 3;
      } else if (lsize > 0) {
        s.mode = 1;
        s.nb = (int)(lsize < (unsigned)kBlock ? lsize : (unsigned)kBlock);
        s.bhead = s.lq_head;
        s.lq_head += (unsigned)s.nb;  // entries are read before any push of this batch
      } else if (!s.exhausted) {
        take_input(a, s);
      }
    }
    __syncthreads();
    const int mode = s.mode;
    if (mode == 0) break;
    if (mode == 3) {
      publish_local(a, s, c);
      continue;
    }
    if (a.tgts) {
      for (int q = tid; q < a.reps; q += kBlock) s.tb[q] = a.dist[a.tgts[q]];
      __syncthreads();
    }
    int4 ent = make_int4(-1, 0, 0, 0);
    if (tid < s.nb) {
      if (mode == 1) {
        ent = s.lq[(s.bhead + tid) & (kLq - 1)];
      } else {
        const unsigned pos = s.gbase + (unsigned)tid;
        const int2 e = hin ? ld_entry(hin, pos) : load_at(a, list_of(a, s.team, s.in_kind, s.in_index), pos);
        ent = make_int4(e.x, e.y, 0, 0);
      }
    }
    if constexpr (W::kCore) process_batch_core(a, s, c, ent, mode == 1);
    else process_batch<W>(a, s, c, ent, mode == 1);
    c.batches++;
    c.round_batches++;
  }
}

// Direction of a round whose input holds `count` entries (1 = pull).
__device__ __forceinline__ unsigned pull_round(const Args& a, unsigned count) {
  return a.pull == kPullAlways || (a.pull == kPullHybrid && count > (unsigned)a.n / kPullDiv) ? 1u : 0u;
}

// Frontier of a pull round, written in the mark phase and read with one
// device-scope load per edge in the pull phase.  SSSP: (round stamp,
// distance) per vertex; stamps are unique within a call, so nothing is
// cleared between rounds.  k-core needs membership only: a bitmap (n / 8
// bytes), cleared in the filing phase of each pull round.
__device__ __forceinline__ int pull_stamp(const Smem& s) { return (int)s.round + 1; }
__device__ __forceinline__ void mark_peeled(const Args& a, int v) {
  atomicOr(&a.fbits[(unsigned)v >> 5], 1u << ((unsigned)v & 31u));
}

// First phase of a pull round: the live entries of the round input (entry
// distance equal to the vertex's current one, bucket not later than the
// current one) are marked in the frontier array with the round's stamp and
// their distance; an entry of a later bucket (a far round) is filed there;
// stale entries are dropped.  k-core: a live entry is a vertex not yet
// peeled whose degree equals the current level; it is peeled here and set
// in the bitmap.
template <class W>
__device__ void run_mark(const Args& a, Smem& s, Counters& c) {
  const int in_list = list_of(a, s.team, s.in_kind, s.in_index);
  const unsigned count = s.in_count;
  const unsigned cur = s.cur;
  const int stamp = pull_stamp(s);
  for (unsigned base = (unsigned)s.team_rank * (unsigned)kBlock; base < count;
       base += (unsigned)s.team_size * kBlock) {
    const unsigned i = base + threadIdx.x;
    bool later = false;
    int v = 0, d = 0;
    unsigned rb = 0;
    const int2 e = i < count ? load_at(a, in_list, i) : make_int2(-1, 0);
    if (e.x >= 0) {
      v = e.x;
      d = e.y;
      const int now = (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + v);
      if constexpr (W::kCore) {
        if ((int)ld_dev(reinterpret_cast<const unsigned*>(a.mark) + v) != kPeeled) {
          if ((unsigned)now == cur) {
            if (atomicExch(&a.mark[v], kPeeled) != kPeeled) mark_peeled(a, v);
          } else if ((unsigned)now > cur) {
            later = true;
            d = now;
          }
        }
      } else if (d == now) {
        rb = W::bucket(a, W::key(a, v, d));
        if (rb > cur) later = true;
        else st_entry(a.front, (size_t)v, stamp, d);
      }
    }
    if constexpr (W::kCore) {
      route_core(a, s, c, later, v, d, 0, 0);
    } else {
      int tgt = 0;
      if (later) tgt = rb < s.win_hi ? (int)(rb & (unsigned)(a.K - 1)) : a.K + 1;
      wave_push_global(a, s, c, later, tgt, v, d, rb);
    }
  }
}

// Whether vertex v (current value dv) can still improve in a pull round.
// SSSP: every frontier distance is at least cur * Delta, so a vertex at or
// below it cannot (not so with an A* estimate in the bucket key).  k-core:
// a vertex not peeled whose degree is above the current level.
template <class W>
__device__ __forceinline__ bool pull_open(const Args& a, unsigned cur, int v, int dv) {
  if constexpr (W::kCore) {
    return dv > (int)cur && (int)ld_dev(reinterpret_cast<const unsigned*>(a.mark) + v) != kPeeled;
  } else {
    const unsigned long long lo = a.h ? 0ull : (unsigned long long)cur * a.delta;
    return (unsigned long long)(unsigned)dv > lo;
  }
}

// Up to kPullIlp edges of a pull round per lane, their loads issued
// together: the columns, then the neighbours' frontier entries, then the
// weights of the frontier neighbours.  offer[k]: the best value edge k
// brings (SSSP: the neighbour's marked distance plus the weight, kInf if
// none; k-core: 1 for a peeled neighbour, else 0).
constexpr int kPullIlp = 2;
template <class W>
__device__ __forceinline__ void pull_edges(const Args& a, Counters& c, int stamp, const int (&edge)[kPullIlp],
                                           const int (&voff)[kPullIlp], const bool (&ok)[kPullIlp],
                                           int (&offer)[kPullIlp]) {
  int u[kPullIlp];
#pragma unroll
  for (int k = 0; k < kPullIlp; ++k) u[k] = ok[k] ? a.col[edge[k]] + voff[k] : 0;
  int2 f[kPullIlp];
#pragma unroll
  for (int k = 0; k < kPullIlp; ++k) {
    if constexpr (W::kCore)
      f[k] = make_int2(ok[k] ? (int)((ld_dev(a.fbits + ((unsigned)u[k] >> 5)) >> ((unsigned)u[k] & 31u)) & 1u) : 0, 0);
    else
      f[k] = ok[k] ? ld_entry(a.front, (size_t)u[k]) : make_int2(0, 0);
  }
#pragma unroll
  for (int k = 0; k < kPullIlp; ++k) {
    const bool hit = ok[k] && f[k].x == (W::kCore ? 1 : stamp);
    offer[k] = W::kCore ? 0 : kInf;
    if (hit) {
      c.relax++;
      if constexpr (W::kCore) {
        offer[k] = 1;
      } else {
        int nd = 0;
        if (W::add(a, f[k].y, a.w[edge[k]], &nd)) offer[k] = nd;
      }
    }
  }
}

// Appends one vertex to the change buffer (a single lane).
__device__ __forceinline__ void append_buf_one(const Args& a, int v) {
  const unsigned pos = atomicAdd(&a.ctl->buf_tail.v, 1u);
  if (pos < a.buf_cap) st_dev(reinterpret_cast<unsigned*>(a.buf) + pos, (unsigned)v);
  else set_status(a.ctl, OG_ERR_WORKSPACE);
}

// A slice of up to kSlice edges of one long row, by the whole workgroup:
// the offers are reduced over the workgroup and combined into the vertex
// with one atomic (several slices share the row), the vertex recorded in
// the change buffer by the first slice that changes it (the lazy flag).
template <class W>
__device__ void pull_slice(const Args& a, Smem& s, Counters& c, unsigned item) {
  const int tid = threadIdx.x;
  const unsigned cur = s.cur;
  const unsigned per = ld_dev(&a.ctl->slices.v);  // > 0: item is a slice
  const unsigned q = item / per;
  const int2 sl = a.slices[item - q * per];
  const int vb = sl.x;
  const int v = (int)q * a.nbase + vb;
  if (tid == 0) {
    const int dv = (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + v);
    s.mode = pull_open<W>(a, cur, v, dv) ? 1 : 0;
    s.nb = dv;
  }
  __syncthreads();
  if (!s.mode) return;
  const int dv = s.nb;
  const long long r0 = a.row_ptr[vb] + (long long)sl.y * kSlice;
  const long long rend = a.row_ptr[vb + 1];
  const long long r1 = rend - r0 < kSlice ? rend : r0 + kSlice;
  const int stamp = pull_stamp(s);
  int best = W::kCore ? 0 : dv;
  for (int k0 = 0; k0 < kSlice / kBlock; k0 += kPullIlp) {
    int edge[kPullIlp], voff[kPullIlp], offer[kPullIlp];
    bool ok[kPullIlp];
#pragma unroll
    for (int k = 0; k < kPullIlp; ++k) {
      const long long e = r0 + (long long)(k0 + k) * kBlock + tid;
      ok[k] = e < r1;
      edge[k] = ok[k] ? (int)e : 0;
      voff[k] = v - vb;
    }
    pull_edges<W>(a, c, stamp, edge, voff, ok, offer);
#pragma unroll
    for (int k = 0; k < kPullIlp; ++k) best = W::kCore ? best + offer[k] : (offer[k] < best ? offer[k] : best);
  }
  // workgroup reduction: sum (k-core) or minimum (SSSP)
  for (int o = 32; o >= 1; o >>= 1) {
    const int y = __shfl_xor(best, o);
    best = W::kCore ? best + y : (y < best ? y : best);
  }
  if (lane_id() == 0) s.wsum[tid / kWave] = best;
  __syncthreads();
  if (tid == 0) {
    int r = s.wsum[0];
    for (int i = 1; i < kWaves; ++i) r = W::kCore ? r + s.wsum[i] : (s.wsum[i] < r ? s.wsum[i] : r);
    if constexpr (W::kCore) {
      if (r > 0 && atomicAdd(&a.aux[v], r) == 0) append_buf_one(a, v);
    } else if (r < dv) {
      const int old = atomicMin(&a.dist[v], r);
      if (r < old) {
        c.improve++;
        if (atomicExch(&a.aux[v], 1) == 0) append_buf_one(a, v);
      }
    }
  }
}

// Second phase of a pull round.  Work items are handed out one at a time
// through the chunk cursor: first the slices of the long rows (every copy
// of the graph), then batches of kBlock vertices.  In a batch, a vertex
// that can still improve and whose row has at most kLongRow edges has its
// row expanded over the workgroup; the frontier neighbours' offers are
// combined per vertex in LDS (minimum of distance + weight; k-core: the
// number of peeled neighbours).  Only the vertex's own lane writes its
// result, so the destination needs no atomic: a lowered distance is stored,
// a k-core count is left for the filing phase, and the vertex is recorded
// in the change buffer.
template <class W>
__device__ void run_pull(const Args& a, Smem& s, Counters& c) {
  const int tid = threadIdx.x;
  const unsigned cur = s.cur;
  const unsigned nsl = ld_dev(&a.ctl->slices.v) * (unsigned)a.reps;  // at most slice_cap(m) per copy
  const unsigned nvb = ((unsigned)a.n + kBlock - 1) / kBlock;
  const int stamp = pull_stamp(s);
  for (;;) {
    __syncthreads();  // the previous item's shared state is no longer read
    if (tid == 0) s.gbase = atomicAdd(&a.ctl->tq[s.team].in_head.v, 1u);
    __syncthreads();
    const unsigned item = s.gbase;
    if (item >= nsl + nvb) break;
    c.batches++;
    c.round_batches++;
    if (item < nsl) {
      pull_slice<W>(a, s, c, item);
      continue;
    }
    const unsigned base = (item - nsl) * (unsigned)kBlock;
    const int nb = (unsigned)a.n - base < (unsigned)kBlock ? (int)((unsigned)a.n - base) : kBlock;
    const int v = (int)base + tid;
    int deg = 0, start = 0, voff = 0, dv = 0;
    if (tid < nb) {
      const int vb = a.reps == 1 ? v : (int)((unsigned)v % (unsigned)a.nbase);
      voff = v - vb;
      dv = (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + v);
      const long long r0 = a.row_ptr[vb];
      const int len = (int)(a.row_ptr[vb + 1] - r0);
      if (len <= kLongRow && pull_open<W>(a, cur, v, dv)) {
        start = (int)r0;
        deg = len;
      }
    }
    int total;
    const int off = block_excl_scan(deg, s, &total);
    s.boff[tid] = off;
    s.bstart[tid] = start;
    s.bvo[tid] = voff;
    s.bd[tid] = W::kCore ? 0 : dv;
    __syncthreads();
    for (int eb = 0; eb < total; eb += kPullIlp * kBlock) {
      int edge[kPullIlp], voff[kPullIlp], slot[kPullIlp], offer[kPullIlp];
      bool ok[kPullIlp];
#pragma unroll
      for (int k = 0; k < kPullIlp; ++k) {
        const int e = eb + k * kBlock + tid;
        ok[k] = e < total;
        int lo_i = 0, hi_i = nb - 1;
        while (ok[k] && lo_i < hi_i) {
          const int mid = (lo_i + hi_i + 1) >> 1;
          if (s.boff[mid] <= e) lo_i = mid;
          else hi_i = mid - 1;
        }
        slot[k] = lo_i;
        edge[k] = ok[k] ? s.bstart[lo_i] + (e - s.boff[lo_i]) : 0;
        voff[k] = s.bvo[lo_i];
      }
      pull_edges<W>(a, c, stamp, edge, voff, ok, offer);
#pragma unroll
      for (int k = 0; k < kPullIlp; ++k) {
        if constexpr (W::kCore) {
          if (offer[k]) atomicAdd(&s.bd[slot[k]], offer[k]);
        } else {
          if (offer[k] < s.bd[slot[k]]) atomicMin(&s.bd[slot[k]], offer[k]);
        }
      }
    }
    __syncthreads();
    bool changed = false;
    if (deg > 0) {
      const int r = s.bd[tid];
      if constexpr (W::kCore) {
        if (r > 0) {
          st_dev(reinterpret_cast<unsigned*>(a.aux) + v, (unsigned)r);
          changed = true;
        }
      } else if (r < dv) {
        st_dev(reinterpret_cast<unsigned*>(a.dist) + v, (unsigned)r);
        c.improve++;
        changed = true;
      }
    }
    wave_append_buf(a, changed, v);
  }
}

// run_round for the degree-binned instantiation.  After the loop's barrier
// every lane reads the ring pointers; when they call for a batch from the
// ring (non-empty, below the fusion threshold, no burned reservations),
// every lane takes the same batch without a second barrier, and the ring's
// head is advanced after the batch's first barrier.  Any other case takes
// the decision of thread 0 as in run_round.  The rule reads nothing that
// thread 0 changes before that decision, except a clamp of the tail that
// leads every lane to the same (thread-0) branch, so the lanes never take
// different barrier sequences.
template <class W>
__device__ void run_round_binned(const Args& a, Smem& s, Counters& c) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    s.lq_head = s.lq_tail = 0;
    s.exhausted = 0;
  }
  for (;;) {
    // (ring pushes of the previous batch are complete: end-of-batch barrier)
    __syncthreads();
    const unsigned h = s.lq_head, t = s.lq_tail;
    const unsigned lsize = t - h;
    int mode, nb;
    unsigned bhead = 0;
    const bool lane_ring = lsize > 0 && lsize <= (unsigned)kLq && lsize < a.threshold;
    if (lane_ring) {
      mode = 1;
      nb = (int)(lsize < (unsigned)kBlock ? lsize : (unsigned)kBlock);
      bhead = h;
    } else {
      if (tid == 0) {
        if (s.lq_tail - s.lq_head > (unsigned)kLq) s.lq_tail = s.lq_head + kLq;  // burned reservations
        const unsigned ls = s.lq_tail - s.lq_head;
        s.mode = 0;
        if (ls > 0 && ls >= a.threshold) {
          s.mode = 3;
        } else if (ls > 0) {  // not reached: the lanes take such a batch themselves
          s.mode = 1;
          s.nb = (int)(ls < (unsigned)kBlock ? ls : (unsigned)kBlock);
          s.bhead = s.lq_head;
          s.lq_head += (unsigned)s.nb;
        } else if (!s.exhausted) {
          take_input(a, s);
        }
      }
      __syncthreads();
      mode = s.mode;
      nb = s.nb;
      bhead = s.bhead;
    }
    if (mode == 0) break;
    if (mode == 3) {
      publish_local(a, s, c);
      continue;
    }
    if (a.tgts) {
      for (int q = tid; q < a.reps; q += kBlock) s.tb[q] = a.dist[a.tgts[q]];
      __syncthreads();
    }
    int4 ent = make_int4(-1, 0, 0, 0);
    if (tid < nb) {
      if (mode == 1) {
        ent = s.lq[(bhead + tid) & (kLq - 1)];
      } else {
        const int2 e = load_at(a, list_of(a, s.team, s.in_kind, s.in_index), s.gbase + (unsigned)tid);
        ent = make_int4(e.x, e.y, 0, 0);
      }
    }
    process_batch_binned<W>(a, s, c, ent, mode == 1, nb, bhead + (unsigned)nb, lane_ring);
    c.batches++;
    c.round_batches++;
  }
}

// Bucket decision of one team, executed by wave 0 of the team's last
// workgroup to finish a round, while the team's other workgroups wait
// (persistent engine) or have exited (host-driven engine); other teams run
// their own rounds meanwhile.  Chooses the team's next round input:
//   1. far entries of the current bucket (overflow, or the initial sources),
//   2. the window slot of the current bucket (after such a far round),
//   3. the spill list: the same bucket needs another round,
//   4. otherwise the next non-empty bucket (section 3.2: smallest bucket
//      across workers), or stop (nothing left, or PPSP / A*: that bucket's
//      lower bound i*Delta already reaches every target of the team's
//      queries).
// The round's control values come from the deciding workgroup's snapshot
// (taken at the round's start; only the decision changes them), so the
// loads below do not wait on one another.
template <class W, class S>
__device__ void decide(const Args& a, const S& snap) {
  Ctl* c = a.ctl;
  const int lane = (int)lane_id();
  const int K = a.K;
  const int T = a.teams;
  const int t0 = snap.team;
  TeamQ& tq = c->tq[t0];
  Control& tc = c->tc[t0];
  const unsigned cur = snap.cur;
  const int in_kind = snap.in_kind, in_index = snap.in_index;
  const unsigned round = snap.round + 1;
  const unsigned win_hi = snap.win_hi;
  int status = (int)ld_dev(&c->status.v);
  const int far_in = in_kind == kInFar ? 1 - in_index : snap.far_out;
  const int so = snap.spill_out;
  // the pending spill and far lists: fill, smallest far bucket
  const unsigned spill_raw = ld_dev(&tq.spill_tail[so].v);
  const unsigned far_raw = ld_dev(&tq.far_tail[far_in].v);
  const unsigned fm = ld_dev(&tq.far_min[far_in].v);  // (read whether or not the list is empty)
  const unsigned fmin = far_raw ? fm : kNoBucket;
  const unsigned need_l = spill_raw > far_raw ? spill_raw : far_raw;
  unsigned hout = 0, heavy_raw = 0;
  if constexpr (W::kSplit) {
    hout = (unsigned)snap.hout;
    heavy_raw = ld_dev(&c->heavy_tail[hout].v);
  }
  // window occupancy, lane j looks at bucket cur + j
  unsigned wraw = 0;
  bool nonempty = false;
  if (lane < K) {
    const unsigned slot = (cur + (unsigned)lane) & (unsigned)(K - 1);
    const bool consumed = in_kind == kInWin && (int)slot == in_index;
    if (!consumed) wraw = ld_dev(&tq.win_tail[slot].v);
    const unsigned bk = cur + (unsigned)lane;
    nonempty = wraw > 0 && bk >= cur && bk < win_hi;
  }
  unsigned long long need_w = wraw;
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long y = __shfl_xor(need_w, o);
    need_w = need_w > y ? need_w : y;
  }
  // largest current distance among the team's targets (INF while one is
  // unreached)
  unsigned tmax = 0;
  if (a.tgts)
    for (int q = t0 + lane * T; q < a.reps; q += kWave * T) {
      const unsigned dt = (unsigned)__hip_atomic_load(&a.dist[a.tgts[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      tmax = dt > tmax ? dt : tmax;
    }
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned y = __shfl_xor(tmax, o);
    tmax = y > tmax ? y : tmax;
  }
  const unsigned slot_cur_cnt = __shfl(wraw, 0);
  const unsigned long long ne = __ballot(nonempty) & ~1ull;  // buckets after cur
  // The consumed input list's chunks go back to the team's stack (every
  // lane takes a share of the chunk table).  After a failure the call ends
  // and the pool is rebuilt by the next one.
  if (!(W::kSplit && in_kind == kInHeavy)) {
    const unsigned lo = team_lo(a.pool_chunks, T, t0);
    const unsigned size = team_lo(a.pool_chunks, T, t0 + 1) - lo;
    int top = (int)ld_dev(&c->free_top[t0].v);
    if (lane == 0) {
      const unsigned taken = (unsigned)((int)size - top);
      if (taken > ld_dev(&c->pool_peak[t0].v)) st_dev(&c->pool_peak[t0].v, taken);
    }
    if (status == 0) {
      // the list's fill is the team's input size of this round (it takes no
      // entries while it is the input)
      const unsigned used = snap.in_count;
      const unsigned nch = (used + kChunk - 1) >> kChunkLog;
      unsigned* tab = chunk_slot(a, list_of(a, t0, in_kind, in_index), 0);
      bool bad = top < 0 || (unsigned)top + nch > size;
      for (unsigned j = (unsigned)lane; j < nch && !bad; j += kWave) {
        const int ch = (int)ld_dev(tab + j);
        if (ch < (int)lo || ch >= (int)(lo + size)) {
          bad = true;
        } else {
          st_dev(reinterpret_cast<unsigned*>(a.fstack) + lo + top + j, (unsigned)ch);
          st_dev(tab + j, (unsigned)kNoChunk);
        }
      }
      if (__ballot(bad)) {
        status = OG_ERR_INTERNAL;  // a chunk table disagrees with its list's fill
        if (lane == 0) set_status(c, status);
      } else if (lane == 0) {
        st_dev(&c->free_top[t0].v, (unsigned)(top + (int)nch));
      }
    }
  }
  if (lane != 0) return;
  // the consumed input list is empty again
  if (in_kind == kInWin) st_dev(&tq.win_tail[in_index].v, 0);
  else if (in_kind == kInSpill) st_dev(&tq.spill_tail[in_index].v, 0);
  else if (!(W::kSplit && in_kind == kInHeavy)) {
    st_dev(&tq.far_tail[in_index].v, 0);
    st_dev(&tq.far_min[in_index].v, kNoBucket);
  }
  st_dev(&tq.in_head.v, 0);
  if (W::kSplit && in_kind == kInHeavy) st_dev(&c->heavy_tail[in_index].v, 0);
  st_dev(&c->buf_tail.v, 0);
  // a consumed far list hands its role to the other one (next generation;
  // the snapshot's far_stamp is the generation plus that one)
  st_dev(&tc.far_gen, snap.far_stamp);
  {
    const unsigned rm = __hip_atomic_exchange(&c->round_max_batches[t0].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicAdd(&c->chain[t0].v, (unsigned long long)rm);
  }
  {
    const unsigned long long nd = need_w > need_l ? need_w : need_l;
    __hip_atomic_fetch_max(&c->need.v, nd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  auto clampcap = [&](unsigned x) { return x < a.cap ? x : a.cap; };
  unsigned done = 0;
  unsigned ncur = cur, count = 0, buckets = ld_dev(&tc.buckets), nwin_hi = win_hi;
  int nkind = kInWin, nindex = 0, nspill_out = so;
  unsigned nhout = hout;
  if (status != 0) {
    done = 1;
  } else if (a.max_rounds && round >= a.max_rounds) {
    set_status(c, OG_ERR_ROUND_LIMIT);
    done = 1;
  } else if (far_raw && fmin <= cur) {
    nkind = kInFar;
    nindex = far_in;
    count = clampcap(far_raw);
  } else if (slot_cur_cnt) {
    nkind = kInWin;
    nindex = (int)(cur & (unsigned)(K - 1));
    count = clampcap(slot_cur_cnt);
  } else if (spill_raw) {
    nkind = kInSpill;
    nindex = so;
    nspill_out = 1 - so;
    count = clampcap(spill_raw);
  } else if (W::kSplit && heavy_raw) {
    // the current bucket is finished: relax the heavy edges of the vertices
    // settled in it (later buckets, or with an A* estimate possibly this one
    // again); later filings go to the other list, a new generation
    nkind = kInHeavy;
    nindex = (int)hout;
    nhout = 1u - hout;
    count = heavy_raw < a.hcap ? heavy_raw : a.hcap;
  } else {
    const unsigned wnext = ne ? cur + (unsigned)(__ffsll((long long)ne) - 1) : kNoBucket;
    const unsigned next = wnext < fmin ? wnext : fmin;
    if (next == kNoBucket) {
      done = 1;
    } else if (a.tgts && tmax != (unsigned)kInf &&
               (unsigned long long)next * a.delta >= (unsigned long long)tmax) {
      done = 1;
    } else {
      ncur = next;
      buckets++;
      if (fmin == next) {
        nkind = kInFar;
        nindex = far_in;
        count = clampcap(far_raw);
      } else {
        nkind = kInWin;
        nindex = (int)(next & (unsigned)(K - 1));
        count = clampcap(ld_dev(&tq.win_tail[nindex].v));
      }
      nwin_hi = sat_add(next, (unsigned)K);
    }
  }
  st_dev(&tq.in_count.v, done ? 0u : count);
  st_dev(&tc.cur, ncur);
  st_dev(&tc.in_kind, (unsigned)nkind);
  st_dev(&tc.in_index, (unsigned)nindex);
  st_dev(&tc.spill_out, (unsigned)nspill_out);
  st_dev(&tc.far_in, (unsigned)far_in);
  st_dev(&tc.win_hi, nwin_hi);
  st_dev(&tc.buckets, buckets);
  if constexpr (W::kSplit) {
    if (nhout != hout) st_dev(&tc.hgen, snap.hgen + 1u);
    st_dev(&tc.hout, nhout);
  }
  if constexpr (W::kPull) st_dev(&tc.pull, done ? 0u : pull_round(a, count));
  if constexpr (W::kBlocks) {
    st_dev(&c->blk_out.v, (unsigned)a.nwg);  // one input-scan token per workgroup
    st_dev(&c->blk_head.v, 0u);              // ring positions restart
    st_dev(&c->blk_tail.v, 0u);
  }
  st_dev(&tc.done, done);
  st_dev(&tc.round, round);
  if (done) atomicSub(&c->live.v, 1u);  // (a team decides done once: its workgroups stop)
}

// The workgroup's team (thread 0, once at the start of a kernel).
template <class S>
__device__ void init_team(const Args& a, S& s) {
  s.team = (int)blockIdx.x % a.teams;
  s.team_rank = (int)blockIdx.x / a.teams;
  s.team_size = (a.nwg - s.team + a.teams - 1) / a.teams;
}

template <class W, class S>
__device__ void load_control(const Args& a, S& s) {
  Ctl* c = a.ctl;
  const Control& tc = c->tc[s.team];
  s.cur = ld_dev(&tc.cur);
  s.in_kind = (int)ld_dev(&tc.in_kind);
  s.in_index = (int)ld_dev(&tc.in_index);
  s.in_count = ld_dev(&c->tq[s.team].in_count.v);
  s.win_hi = ld_dev(&tc.win_hi);
  s.spill_out = (int)ld_dev(&tc.spill_out);
  s.round = ld_dev(&tc.round);
  const int far_in = (int)ld_dev(&tc.far_in);
  s.far_out = s.in_kind == kInFar ? 1 - far_in : far_in;
  s.far_stamp = ld_dev(&tc.far_gen) + (s.in_kind == kInFar ? 1u : 0u);
  s.epoch = ld_dev(&tc.epoch);
  if constexpr (W::kSplit) {
    s.hout = (int)ld_dev(&tc.hout);
    s.hgen = ld_dev(&tc.hgen);
  }
  if constexpr (W::kPull) s.pull = (int)ld_dev(&tc.pull);
  s.done = ld_dev(&tc.done) || ld_dev(&c->status.v) != 0;
}

// Synchronisation of a team's workgroups (device-wide when one team runs).
// Every wavefront waits for its own stores and atomics to complete; thread 0
// of each workgroup then arrives on its group's counter (kGroup workgroups
// of the team per counter, each on its own cache line), the last of a group
// arrives on the team's root counter, and the team's last workgroup (with
// decide_next: after taking the team's bucket decision with wave 0)
// publishes the team's new barrier count on its kFlags / teams release
// flags.  With wait_others (the persistent engine) every other workgroup of
// the team spins on one of those flags; the host-driven engine ends the
// kernel instead.
__device__ void flush_counters(const Args& a, Counters& c);

template <class W, class S>
__device__ void round_barrier(const Args& a, S& s, Counters& c, bool wait_others, bool decide_next) {
  Ctl* ctl = a.ctl;
  // a wavefront whose 32-bit counts near 2^31 adds them to the totals now
  if (__ballot((c.relax | c.improve | c.push_local | c.push_global | c.far | c.batches) >= 0x80000000u))
    flush_counters(a, c);
  if (threadIdx.x == 0) atomicMax(&ctl->round_max_batches[s.team].v, c.round_batches);
  c.round_batches = 0;
  wait_vm();
  __syncthreads();
  if (threadIdx.x == 0) {
    // the team's groups: counters team * gstride .. team * gstride + ngrp - 1
    const int gstride = ((a.nwg + a.teams - 1) / a.teams + kGroup - 1) / kGroup;
    const int g = s.team_rank / kGroup;
    const int ngrp = (s.team_size + kGroup - 1) / kGroup;
    const int gsize = g == ngrp - 1 ? s.team_size - g * kGroup : kGroup;
    const int grp = s.team * gstride + g;
    bool last = false;
    const unsigned p = atomicAdd(&ctl->bar_grp[grp].v, 1u);
    if (p == (unsigned)gsize - 1) {
      (void)atomicExch(&ctl->bar_grp[grp].v, 0u);
      const unsigned q = atomicAdd(&ctl->bar_root[s.team].v, 1u);
      if (q == (unsigned)ngrp - 1) {
        (void)atomicExch(&ctl->bar_root[s.team].v, 0u);
        last = true;
      }
    }
    s.last = last;
  }
  __syncthreads();
  const unsigned next = s.epoch + 1;
  const int fpt = kFlags / a.teams;  // release flags per team
  if (s.last) {
    if (threadIdx.x < kWave) {
      if (decide_next) decide<W>(a, s);
      if (threadIdx.x == 0) st_dev(&ctl->tc[s.team].epoch, next);
      wait_vm();
      if ((int)threadIdx.x < fpt) st_dev(&ctl->flag[s.team * fpt + (int)threadIdx.x].v, next);
    }
  } else if (wait_others && threadIdx.x == 0) {
    const unsigned* f = &ctl->flag[s.team * fpt + s.team_rank % fpt].v;
    while (ld_dev(f) < next) __builtin_amdgcn_s_sleep(2);
  }
  __syncthreads();
  if (threadIdx.x == 0) s.epoch = next;
}

// Adds the wavefront's counts to the totals (all 64 lanes call it together)
// and clears them.
__device__ void flush_counters(const Args& a, Counters& c) {
  unsigned long long v[5] = {c.relax, c.improve, c.push_local, c.push_global, c.far};
#pragma unroll
  for (int i = 0; i < 5; ++i)
    for (int o = 32; o >= 1; o >>= 1) v[i] += __shfl_xor(v[i], o);
  if (lane_id() == 0) {
    Ctl* ctl = a.ctl;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (v[i]) atomicAdd(&ctl->st[kStRelax + i].v, v[i]);
    if (threadIdx.x == 0 && c.batches) atomicAdd(&ctl->st[kStBatches].v, (unsigned long long)c.batches);
  }
  c.relax = c.improve = c.push_local = c.push_global = c.far = 0;
  if (threadIdx.x == 0) c.batches = 0;
}

// ---------------------------------------------------------------- kernels

// Writes up to kTableChunk entries of the query table (sources, then
// targets) into the workspace; the values travel in the kernel arguments,
// so the host buffer need not outlive the call.
constexpr int kTableChunk = 240;
struct TableChunk {
  int offset, count;
  int vals[kTableChunk];
};
__global__ void k_put_table(int* table, TableChunk tc) {
  for (int i = threadIdx.x; i < tc.count; i += blockDim.x) table[tc.offset + i] = tc.vals[i];
}

__global__ __launch_bounds__(kBlock) void k_init(Args a, int inf_bits) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    a.dist[v] = inf_bits;
    if (a.aux) a.aux[v] = 0;
  }
  // zero the control block (grid-stride over its words)
  unsigned* words = reinterpret_cast<unsigned*>(a.ctl);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (long long)(sizeof(Ctl) / 4); i += stride)
    words[i] = 0;
}

// Sources: dist = 0, one (s, 0) entry each in far list 0, far_min = the
// smallest source bucket.  The first round is a far round: it processes the
// sources of the smallest bucket and files the others (A* estimates can put
// sources of different queries in different buckets).
template <class W>
__global__ __launch_bounds__(kBlock) void k_init_sources(Args a) {
  Ctl* c = a.ctl;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.nsrc; i += gridDim.x * blockDim.x) {
    const int s = a.srcs[i];
    a.dist[s] = 0;
    if (a.teams == 1) {
      // far list 0's first chunks are chunks 0, 1, ... of the pool (k_pool_init)
      st_entry(a.pool, (size_t)i, s, 0);
      atomicMin(&c->tq[0].far_min[0].v, W::bucket(a, W::key(a, s, 0)));
    } else {
      // the source's team files it in its far list 0 (every writer of a
      // chunk's first position in this launch is running, so the chunk
      // hand-over of store_at cannot wait on a thread that has not started)
      const int t = query_of(a, s) % a.teams;
      const unsigned pos = atomicAdd(&c->tq[t].far_tail[0].v, 1u);
      store_at(a, list_of(a, t, kInFar, 0), pos, s, 0);
      atomicMin(&c->tq[t].far_min[0].v, W::bucket(a, W::key(a, s, 0)));
    }
  }
}

// Light/heavy split of every row: a copy with the light edges (w < Delta)
// first and the heavy ones after, each group in its original order, and
// lsplit[v] = light edges of v; hmark is cleared.  Rows of up to
// kSplitSmall edges are split by one thread; longer rows are listed for
// k_split_big (one wavefront per row).
constexpr int kSplitSmall = 64;
__global__ __launch_bounds__(kBlock) void k_split_small(Args a, int* ecol, int* ew, int* lsplit, int* big) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long v = t0; v < a.n; v += stride) a.hmark[v] = 0u;
  for (long long v = t0; v < a.nbase; v += stride) {
    const long long r0 = a.row_ptr[v], r1 = a.row_ptr[v + 1];
    if (r1 - r0 > kSplitSmall) {
      big[atomicAdd(&a.ctl->big_rows.v, 1u)] = (int)v;
      continue;
    }
    int l = 0;
    for (long long e = r0; e < r1; ++e) l += SplitW::light(a, a.w[e]) ? 1 : 0;
    long long li = r0, hi = r0 + l;
    for (long long e = r0; e < r1; ++e) {
      const int c = a.col[e], w = a.w[e];
      const long long o = SplitW::light(a, w) ? li++ : hi++;
      ecol[o] = c;
      ew[o] = w;
    }
    lsplit[v] = l;
  }
}

__global__ __launch_bounds__(kBlock) void k_split_big(Args a, int* ecol, int* ew, int* lsplit, const int* big) {
  const unsigned nbig = a.ctl->big_rows.v;
  const unsigned lane = lane_id();
  const unsigned nwave = gridDim.x * (kBlock / kWave);
  for (unsigned i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < nbig; i += nwave) {
    const int v = big[i];
    const long long r0 = a.row_ptr[v], r1 = a.row_ptr[v + 1];
    long long l = 0;
    for (long long e0 = r0; e0 < r1; e0 += kWave) {
      const long long e = e0 + lane;
      l += __popcll(__ballot(e < r1 && SplitW::light(a, a.w[e])));
    }
    long long li = r0, hi = r0 + l;
    for (long long e0 = r0; e0 < r1; e0 += kWave) {
      const long long e = e0 + lane;
      const bool in = e < r1;
      int c = 0, w = 0;
      if (in) {
        c = a.col[e];
        w = a.w[e];
      }
      const bool lt = in && SplitW::light(a, w);
      const unsigned long long ml = __ballot(lt), mh = __ballot(in && !lt);
      if (in) {
        const long long o = lt ? li + __popcll(ml & lanemask_lt()) : hi + __popcll(mh & lanemask_lt());
        ecol[o] = c;
        ew[o] = w;
      }
      li += __popcll(ml);
      hi += __popcll(mh);
    }
    if (lane == 0) lsplit[v] = (int)l;
  }
}

__global__ __launch_bounds__(kBlock) void k_zero_ctl(Ctl* ctl) {
  unsigned* words = reinterpret_cast<unsigned*>(ctl);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (long long)(sizeof(Ctl) / 4);
       i += (long long)gridDim.x * blockDim.x)
    words[i] = 0;
}

// k-core: the priority vector starts at every vertex's degree and every
// vertex is filed in far list 0 (generation 0) with that priority; the
// first round is a far round at the smallest degree.
__global__ __launch_bounds__(kBlock) void k_init_core(Args a) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned lo = kNoBucket;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int d = (int)(a.row_ptr[v + 1] - a.row_ptr[v]);
    a.dist[v] = d;
    a.mark[v] = 0;
    if (a.aux) a.aux[v] = 0;
    st_entry(a.pool, (size_t)v, (int)v, d);  // far list 0: pool chunks 0, 1, ...
    lo = (unsigned)d < lo ? (unsigned)d : lo;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned y = __shfl_xor(lo, o);
    lo = y < lo ? y : lo;
  }
  if (lane_id() == 0 && lo != kNoBucket) atomicMin(&a.ctl->tq[0].far_min[0].v, lo);
}

// The queue pool at the start of a call: every chunk table entry empty but
// team 0's far list 0's first `pre` (chunks 0 .. pre-1, where a single
// team's sources or, for k-core, all vertices are filed; pre is 0 when more
// teams run), each team's other chunks on its stack.  Runs after the
// control block is zeroed.
__global__ __launch_bounds__(kBlock) void k_pool_init(Args a, unsigned pre) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  const unsigned long long ntab = (unsigned long long)a.teams * (a.K + 4) * a.tchunks;
  const int far0 = a.K + 2;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < ntab; i += stride) {
    const unsigned j = (unsigned)(i % a.tchunks);
    a.ctab[i] = (int)(i / a.tchunks) == far0 && j < pre ? (int)j : kNoChunk;
  }
  // team t's stack, at positions lo .. hi-1, lists its chunks lo .. hi-1
  // (team 0's after the first pre)
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.pool_chunks;
       i += stride) {
    int t = (int)((i * (unsigned long long)a.teams) / a.pool_chunks);
    while (t + 1 < a.teams && team_lo(a.pool_chunks, a.teams, t + 1) <= i) ++t;
    while (t > 0 && team_lo(a.pool_chunks, a.teams, t) > i) --t;
    const unsigned lo = team_lo(a.pool_chunks, a.teams, t);
    const unsigned skip = t == 0 ? pre : 0u;
    const unsigned size = team_lo(a.pool_chunks, a.teams, t + 1) - lo;
    const unsigned j = (unsigned)i - lo;
    if (j + skip < size) a.fstack[i] = (int)(lo + skip + j);
  }
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)a.teams) {
    const int t = (int)threadIdx.x;
    const unsigned size = team_lo(a.pool_chunks, a.teams, t + 1) - team_lo(a.pool_chunks, a.teams, t);
    const unsigned skip = t == 0 ? pre : 0u;
    a.ctl->free_top[t].v = size - skip;
    a.ctl->pool_peak[t].v = skip;
  }
}

__global__ void k_init_ctl(Args a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctl* c = a.ctl;
  unsigned most = 0;
  if (a.teams == 1) c->tq[0].far_tail[0].v = (unsigned)a.nsrc;  // (more teams: counted by k_init_sources)
  for (int t = 0; t < a.teams; ++t) {
    TeamQ& q = c->tq[t];
    q.in_count.v = q.far_tail[0].v;
    most = q.far_tail[0].v > most ? q.far_tail[0].v : most;
    q.far_min[1].v = kNoBucket;
  }
  for (int t = 0; t < a.teams; ++t) {
    const unsigned b = c->tq[t].far_min[0].v;
    Control& tc = c->tc[t];
    tc.cur = b;
    tc.in_kind = kInFar;
    tc.in_index = 0;
    tc.far_in = 0;
    tc.win_hi = sat_add(b, (unsigned)a.K);
    tc.buckets = 1;
  }
  c->live.v = (unsigned)a.teams;
  c->teams.v = (unsigned)a.teams;
  c->need.v = most;
  c->blk_out.v = (unsigned)a.nwg;  // vertex blocks: one input-scan token per workgroup
}

// Pull instantiations: the direction of the first round.
__global__ void k_init_pull(Args a) {
  if (threadIdx.x == 0 && blockIdx.x == 0) a.ctl->tc[0].pull = pull_round(a, a.ctl->tq[0].in_count.v);
}

// Pull instantiations: the slices of every row longer than kLongRow, as
// (vertex, slice index) pairs; the count goes to the control block.  The
// list never exceeds slice_cap(m) entries (a longer one would mean a
// malformed graph and ends the call with OG_ERR_INTERNAL).
__global__ __launch_bounds__(kBlock) void k_pull_slices(Args a, int2* slices) {
  const unsigned long long cap = slice_cap(a.m);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long vb = (long long)blockIdx.x * blockDim.x + threadIdx.x; vb < a.nbase; vb += stride) {
    const long long deg = a.row_ptr[vb + 1] - a.row_ptr[vb];
    if (deg <= kLongRow) continue;
    const unsigned long long k = (unsigned long long)((deg + kSlice - 1) / kSlice);
    const unsigned long long base = atomicAdd(&a.ctl->slices.v, (unsigned)k);
    if (base + k > cap) {
      set_status(a.ctl, OG_ERR_INTERNAL);
      continue;
    }
    for (unsigned long long j = 0; j < k; ++j) slices[base + j] = make_int2((int)vb, (int)j);
  }
}

__global__ void k_far_min_init(Ctl* c) {
  if (threadIdx.x < kMaxTeams && blockIdx.x == 0) c->tq[threadIdx.x].far_min[0].v = kNoBucket;
}

// OG_FLAG_VALIDATE: the CSR structure (row_ptr[0] = 0, non-decreasing,
// row_ptr[n] = m; every column index in [0, n)) and, when weights are given,
// their sign (a float32 weight's sign bit reads as a negative int32).
__global__ __launch_bounds__(kBlock) void k_validate(const long long* row_ptr, int n, const int* col, const int* w,
                                                      long long m, Ctl* ctl) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad_w = false, bad_g = false;
  for (long long e = t0; e < m; e += stride) {
    bad_g |= (unsigned)col[e] >= (unsigned)n;
    if (w) bad_w |= w[e] < 0;
  }
  for (long long v = t0; v <= n; v += stride) {
    const long long r = row_ptr[v];
    bad_g |= v == 0 ? r != 0 : r < row_ptr[v - 1];
    if (v == n) bad_g |= r != m;
  }
  if (__ballot(bad_g) && lane_id() == 0) atomicExch(reinterpret_cast<int*>(&ctl->status.v), OG_ERR_INVALID_ARG);
  if (__ballot(bad_w) && lane_id() == 0) set_status(ctl, OG_ERR_NEGATIVE_WEIGHT);
}

// OG_FLAG_VALIDATE with a pull direction, after k_validate has passed: the
// graph must be symmetric (each edge (u, v, w) has a reverse (v, u, w)),
// since a pull round reads a vertex's row as its in-edges.  The multiset of
// edges equals the multiset of reversed edges exactly when the sums of a
// 64-bit hash over both agree (up to hash collisions); the hash is the
// SplitMix64 finaliser of the packed triple.  One thread per row.
__device__ __forceinline__ unsigned long long edge_hash(unsigned u, unsigned v, unsigned w) {
  unsigned long long x = ((unsigned long long)u << 32 | v) ^ ((unsigned long long)w * 0x9E3779B97F4A7C15ull);
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ __launch_bounds__(kBlock) void k_validate_sym(const long long* row_ptr, int n, const int* col, const int* w,
                                                          Ctl* ctl) {
  unsigned long long acc = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
    for (long long e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      const unsigned v = (unsigned)col[e], wt = w ? (unsigned)w[e] : 0u;
      acc += edge_hash((unsigned)u, v, wt) - edge_hash(v, (unsigned)u, wt);
    }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane_id() == 0 && acc) atomicAdd(&ctl->sym.v, acc);
}
__global__ void k_validate_sym_verdict(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && ctl->sym.v != 0) set_status(ctl, OG_ERR_INVALID_ARG);
}

// Persistent engine: one cooperative launch; rounds separated by a
// device-wide barrier whose last arriver takes the bucket decision.  A lazy
// round has a second barrier between recording the changes and filing them.
template <class W>
__global__ __launch_bounds__(kBlock) void k_persistent(Args a) {
  __shared__ Smem s;
  Counters c;
  if constexpr (W::kBin) {
    if (threadIdx.x == 0) s.flat_any = 0;
  }
  if (threadIdx.x == 0) {
    init_team(a, s);
    load_control<W>(a, s);
  }
  __syncthreads();
  while (!s.done) {
    if (W::kPull && s.pull) {
      run_mark<W>(a, s, c);
      round_barrier<W>(a, s, c, true, false);
      run_pull<W>(a, s, c);
    } else if constexpr (W::kBin) {
      run_round_binned<W>(a, s, c);
    } else {
      run_round<W>(a, s, c);
    }
    if (a.lazy) {
      round_barrier<W>(a, s, c, true, false);
      run_flush<W>(a, s, c);
    }
    round_barrier<W>(a, s, c, true, true);
    if (threadIdx.x == 0) load_control<W>(a, s);
    __syncthreads();
  }
  flush_counters(a, c);
}

// Host-driven engine: one launch per round (two for a lazy round: phase 0
// records, phase 1 files; three with a pull instantiation: phase 0 pushes or
// marks the frontier, phase 1 pulls or does nothing, phase 2 files); the
// last workgroup to finish the round takes the bucket decision for the next
// launch.
template <class W>
__global__ __launch_bounds__(kBlock) void k_round(Args a, int phase) {
  __shared__ Smem s;
  Counters c;
  if constexpr (W::kBin) {
    if (threadIdx.x == 0) s.flat_any = 0;
  }
  if (threadIdx.x == 0) {
    init_team(a, s);
    load_control<W>(a, s);
  }
  __syncthreads();
  if (s.done) return;
  if constexpr (W::kPull) {
    if (phase == 0) {
      if (s.pull) run_mark<W>(a, s, c);
      else run_round<W>(a, s, c);
    } else if (phase == 1) {
      if (!s.pull) return;
      run_pull<W>(a, s, c);
    } else {
      run_flush<W>(a, s, c);
    }
    round_barrier<W>(a, s, c, false, phase == 2);
    flush_counters(a, c);
    return;
  }
  if (phase == 0) {
    if constexpr (W::kBin) run_round_binned<W>(a, s, c);
    else run_round<W>(a, s, c);
    round_barrier<W>(a, s, c, false, !a.lazy);
  } else {
    run_flush<W>(a, s, c);
    round_barrier<W>(a, s, c, false, true);
  }
  flush_counters(a, c);
}

__global__ __launch_bounds__(kBlock) void k_fill(int* p, long long n, int value) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) p[v] = value;
}

// ------------------------------------------------------------ vertex blocks
//
// Bucket fusion at the granularity of a vertex block (section 3.3: a worker
// keeps processing its share of the current bucket without a global
// synchronisation).  The vertices are grouped into compact blocks (at most
// kBcap vertices and kEcap internal edges each); a workgroup that takes a
// block loads its distances, its processed labels and its internal edges
// into LDS and drains the block's part of the current bucket there: each
// internal relaxation is an LDS atomic minimum, and an improved vertex of
// the current bucket goes back on the block's LDS worklist at once.  Only
// edges that leave the block touch dist in HBM.  An improvement across a
// block boundary in the current bucket marks the target block dirty and
// queues it in a device-wide ring of blocks, which idle workgroups serve
// within the same round; one in a later bucket is filed in the window or
// far list as usual.  A round ends when every work item of the round (one
// input-scan token per workgroup, plus every queued block) is finished.
//
// Per-vertex state across activations: brel[p] is the distance at which the
// vertex at position p last had its edges relaxed; the vertex is pending
// when dist < brel.  Only the owner of a block reads or writes its brel
// entries.  A block's state word holds kBlkDirty (queued, or changed while
// owned) and kBlkOwned; a block is queued only on the transition from 0 to
// dirty, so the ring holds each block at most once.
constexpr int kBcap = 4096;   // vertices per block
constexpr int kEcap = 12288;  // internal edges per block
constexpr int kBwords = kBcap / 32;
constexpr int kDefaultBlockSize = 2048;  // mean block size the clustering aims at
constexpr int kIedgeWmax = 65536;        // an internal edge carries a 16-bit weight
constexpr unsigned kBlkDirty = 1u, kBlkOwned = 2u;
// Waits on the block ring give up after this many polls (seconds of
// waiting, far beyond any round): the call then ends with OG_ERR_INTERNAL
// instead of hanging on a broken invariant.
constexpr unsigned kBlkSpinLimit = 1u << 23;

struct BlkSmem {
  int dist[kBcap];   // distances of the block's vertices
  int rel[kBcap];    // distance at which each vertex's edges were last relaxed
  int orig[kBcap];   // distances as loaded (the write-back sends what fell below them)
  int vert[kBcap];   // vertex id of each local index
  int xrow[kBcap + 1];   // leaving-edge offsets into xcol / xw / xblk
  unsigned edge[kEcap];  // internal edges: local target | weight << 16
  unsigned short row[kBcap + 2];  // internal-edge offsets (the +2 keeps the next array aligned)
  unsigned short wl[kBcap];  // worklist ring of local indices; after a drain, the list of
                             // relaxed vertices with leaving edges
  unsigned prc[kBwords];     // edges relaxed in this drain
  unsigned wl_head, wl_tail;
  int xn;
  int claim, again, ok, nv, p0, e0, ne;
  // control snapshot (the fields load_control, round_barrier and
  // wave_push_global use)
  unsigned cur, in_count, win_hi, round, epoch, far_stamp;
  int in_kind, in_index, done, spill_out, far_out;
  int team, team_rank, team_size;  // this workgroup's team, its index in it, the team's workgroups
  int hout;
  unsigned hgen;
  int pull;
  int last, exhausted, mode, nb;
  unsigned gbase;
};

// Ring slots carry the position they were filled for, so a ticket never
// takes another lap's entry: slot p % size holds (p << 32) | (block + 1)
// while queued and (p << 32) once taken.
__device__ __forceinline__ unsigned long long ld_slot(const unsigned long long* q) {
  return __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_slot(unsigned long long* q, unsigned long long x) {
  __hip_atomic_store(q, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Marks block b dirty; on the transition from clean it becomes a work item
// of the round and is queued.  The caller holds a work item itself, so the
// round cannot end in between; the count is raised before the block can be
// taken (and so finished and counted down).  The slot's previous entry (a
// lap earlier) has been taken unless its ticket holder is still reading it.
__device__ void blk_mark(const Args& a, int b) {
  const unsigned old = atomicOr(a.bstate + b, kBlkDirty);
  if (old & (kBlkDirty | kBlkOwned)) return;
  atomicAdd(&a.ctl->blk_out.v, 1u);
  const unsigned pos = atomicAdd(&a.ctl->blk_tail.v, 1u);
  wait_vm();
  unsigned long long* slot = a.ring + (pos & a.ring_mask);
  for (unsigned spin = 0; (unsigned)ld_slot(slot) != 0u; ++spin) {
    if (spin == kBlkSpinLimit) {
      set_status(a.ctl, OG_ERR_INTERNAL);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  st_slot(slot, ((unsigned long long)pos << 32) | (unsigned)(b + 1));
}

// Takes a queued block (thread 0 of a workgroup): draws the next ticket
// (ring position) and waits for the block pushed at that position; -1 once
// no work item of the round is left (that position is then never filled:
// every pushed block is counted until it is finished).  Positions start
// from 0 each round (reset by the bucket decision).
__device__ int blk_pop(const Args& a) {
  Ctl* c = a.ctl;
  const unsigned t = atomicAdd(&c->blk_head.v, 1u);
  unsigned long long* slot = a.ring + (t & a.ring_mask);
  int nap = 1;
  for (unsigned polls = 0;; ++polls) {
    if (polls == kBlkSpinLimit) {
      set_status(c, OG_ERR_INTERNAL);
      return -1;
    }
    const unsigned long long x = ld_slot(slot);
    if ((unsigned)(x >> 32) == t && (unsigned)x != 0u) {
      st_slot(slot, (unsigned long long)t << 32);
      return (int)((unsigned)x - 1u);
    }
    if (ld_dev(&c->blk_out.v) == 0u) return -1;
    for (int k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(4);
    nap = nap < 8 ? 2 * nap : 8;
  }
}

// Appends local index j of the lanes with push to the worklist (all 64
// lanes call it together; one LDS atomic per wavefront).
__device__ __forceinline__ void blk_wl_push(BlkSmem& s, bool push, int j) {
  const unsigned long long m = __ballot(push);
  if (m == 0) return;
  const int leader = __ffsll((long long)m) - 1;
  unsigned base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(&s.wl_tail, (unsigned)__popcll(m));
  base = __shfl(base, leader);
  if (push) s.wl[(base + (unsigned)__popcll(m & lanemask_lt())) & (unsigned)(kBcap - 1)] = (unsigned short)j;
}

__device__ __forceinline__ int blk_window_target(const Args& a, const BlkSmem& s, bool has, unsigned bk) {
  return has ? (bk < s.win_hi ? (int)(bk & (unsigned)(a.K - 1)) : a.K + 1) : 0;
}

// Internal edges a lane relaxes together in a drain step.
constexpr int kBlkIlp = 4;

// Drains the block's worklist in LDS.  A vertex is on the worklist exactly
// while it is pending in the current bucket (dist < rel and bucket(dist) <=
// current), so the ring never holds more than the block's vertices.  Each
// step takes up to kBlock entries, one per lane: the lane publishes rel =
// dist for its vertex before a barrier, then relaxes the vertex's internal
// edges with LDS atomic minima; an improvement queues its target when that
// makes the target pending (it was not, or only in a later bucket).
// Leaving edges wait for the end of the drain (blk_leave_and_write).  (A
// lane-level chase, one lane following a chain of improvements without
// barriers, relaxed 2.2-2.5 times as many edges on the road grid and was
// twice as slow.)
template <class W>
__device__ void blk_drain(const Args& a, BlkSmem& s, Counters& c, unsigned cur) {
  const int tid = threadIdx.x;
  unsigned n_relax = 0, n_improve = 0, n_push = 0;  // (32-bit: few registers in the loop)
  for (;;) {
    __syncthreads();  // the previous step's pushes are in place
    const unsigned h = s.wl_head, t = s.wl_tail;
    if (h == t) break;
    const unsigned nb = t - h < (unsigned)kBlock ? t - h : (unsigned)kBlock;
    int d = 0, k0 = 0, k1 = 0;
    if ((unsigned)tid < nb) {
      const int i = s.wl[(h + (unsigned)tid) & (unsigned)(kBcap - 1)];
      d = s.dist[i];
      if (d < s.rel[i]) {
        s.rel[i] = d;
        atomicOr(&s.prc[i >> 5], 1u << (i & 31));
        k0 = s.row[i];
        k1 = s.row[i + 1];
      }
    }
    __syncthreads();  // ring pointers read, the step's rel values published
    if (tid == 0) s.wl_head = h + nb;
    for (int k = k0; __ballot(k < k1) != 0; k += kBlkIlp) {
      int j[kBlkIlp], nd[kBlkIlp];
      bool go[kBlkIlp];
#pragma unroll
      for (int q = 0; q < kBlkIlp; ++q) {
        go[q] = k + q < k1;
        j[q] = 0;
        nd[q] = 0;
        if (go[q]) {
          const unsigned e = s.edge[k + q];
          j[q] = (int)(e & 0xffffu);
          n_relax++;
          go[q] = W::add(a, d, (int)(e >> 16), &nd[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < kBlkIlp; ++q)
        if (go[q]) go[q] = nd[q] < s.dist[j[q]];
      bool push[kBlkIlp];
#pragma unroll
      for (int q = 0; q < kBlkIlp; ++q) {
        push[q] = false;
        if (go[q]) {
          const int old = atomicMin(&s.dist[j[q]], nd[q]);
          if (nd[q] < old) {
            n_improve++;
            push[q] = W::bucket(a, (unsigned)nd[q]) <= cur &&
                      (old >= s.rel[j[q]] || W::bucket(a, (unsigned)old) > cur);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kBlkIlp; ++q) {
        if (push[q]) n_push++;
        blk_wl_push(s, push[q], j[q]);
      }
    }
  }
  c.relax += n_relax;
  c.improve += n_improve;
  c.push_local += n_push;
}

// After a drain: the leaving edges of the vertices it relaxed, each at the
// vertex's final distance, all in flight together; and the write-back of
// every distance the drain lowered (one device-scope atomic minimum per
// vertex, filed in its later bucket when that improves it) and of the
// relaxed labels.  An improvement across the boundary in the current bucket
// marks the target block.
template <class W>
__device__ void blk_leave_and_write(const Args& a, BlkSmem& s, Counters& c, unsigned cur) {
  constexpr int kPer = kBcap / kBlock;
  const int tid = threadIdx.x;
  const int nv = s.nv, p0 = s.p0;
  if (tid == 0) s.xn = 0;
  __syncthreads();  // (the drain ended on a barrier: the ring is free for the list)
  // write-back atomics first: their round trips overlap the leaving edges'
  int old[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int i = q * kBlock + tid;
    old[q] = -1;
    if (i < nv && s.dist[i] < s.orig[i]) old[q] = atomicMin(&a.dist[s.vert[i]], s.dist[i]);
  }
  for (int base = 0; base < nv; base += kBlock) {
    const int i = base + tid;
    bool lx = false;
    if (i < nv && ((s.prc[i >> 5] >> (i & 31)) & 1u)) {
      st_dev(reinterpret_cast<unsigned*>(a.brel) + p0 + i, (unsigned)s.rel[i]);
      lx = s.xrow[i + 1] > s.xrow[i];
    }
    const unsigned long long m = __ballot(lx);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      int pos = 0;
      if ((int)lane_id() == leader) pos = atomicAdd(&s.xn, __popcll(m));
      pos = __shfl(pos, leader);
      if (lx) s.wl[pos + __popcll(m & lanemask_lt())] = (unsigned short)i;
    }
  }
  __syncthreads();
  const int xn = s.xn;
  for (int base = 0; base < xn; base += kBlock) {
    int x0 = 0, x1 = 0, d = 0;
    if (base + tid < xn) {
      const int i = s.wl[base + tid];
      x0 = s.xrow[i];
      x1 = s.xrow[i + 1];
      d = s.rel[i];
    }
    for (int k = x0; __ballot(k < x1) != 0; ++k) {
      bool has = false;
      int u = 0, nd = 0;
      unsigned bk = 0;
      if (k < x1) {
        u = a.xcol[k];
        const int w = a.xw[k];
        c.relax++;
        if (W::add(a, d, w, &nd)) {
          const int o = atomicMin(&a.dist[u], nd);
          if (nd < o) {
            c.improve++;
            bk = W::bucket(a, (unsigned)nd);
            if (bk <= cur) blk_mark(a, a.xblk[k]);
            else has = true;
          }
        }
      }
      wave_push_global(a, s, c, has, blk_window_target(a, s, has, bk), u, nd, bk);
    }
  }
  // the write-back's results: an improvement into a later bucket is filed
  // there (one in the current bucket was relaxed in the drain)
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (q * kBlock >= nv) break;
    const int i = q * kBlock + tid;
    bool has = false;
    int v = 0, nd = 0;
    unsigned bk = 0;
    if (i < nv && old[q] >= 0) {
      nd = s.dist[i];
      if (nd < old[q]) {
        v = s.vert[i];
        bk = W::bucket(a, (unsigned)nd);
        has = bk > cur;
      }
    }
    wave_push_global(a, s, c, has, blk_window_target(a, s, has, bk), v, nd, bk);
  }
  wait_vm();  // the block's results are in HBM before it can be released
}

// One activation of block b (taken from the ring): load it, then drain,
// relax its leaving edges and write back until no other workgroup has
// changed it meanwhile.
template <class W>
__device__ void blk_process(const Args& a, BlkSmem& s, Counters& c, int b) {
  constexpr int kPer = kBcap / kBlock, kPerE = kEcap / kBlock;
  const int tid = threadIdx.x;
  const unsigned cur = s.cur;
  if (tid == 0) {
    int ok = (unsigned)b < (unsigned)a.nb;
    int4 mt = make_int4(0, 0, 0, 0);
    if (ok) {
      const unsigned st = atomicCAS(a.bstate + b, kBlkDirty, kBlkOwned);
      mt = a.bmeta[b];  // issued together with the claim
      ok = st == kBlkDirty && mt.y >= 1 && mt.y <= kBcap && mt.w >= 0 && mt.w <= kEcap;
    }
    if (!ok) set_status(a.ctl, OG_ERR_INTERNAL);
    s.ok = ok;
    s.p0 = mt.x;
    s.nv = mt.y;
    s.e0 = mt.z;
    s.ne = mt.w;
  }
  __syncthreads();
  if (!s.ok) return;
  const int nv = s.nv, p0 = s.p0, ne = s.ne, e0 = s.e0;
  {
    // the block's loads in groups of kLoadGroup per thread, each group's
    // loads in flight together
    constexpr int kLoadGroup = 4;
    for (int q0 = 0; q0 < kPer; q0 += kLoadGroup) {
      if (q0 * kBlock >= nv) break;
      int vv[kLoadGroup], rr[kLoadGroup], ro[kLoadGroup], xr[kLoadGroup];
#pragma unroll
      for (int q = 0; q < kLoadGroup; ++q) {
        const int i = (q0 + q) * kBlock + tid;
        vv[q] = rr[q] = ro[q] = xr[q] = 0;
        if (i < nv) {
          vv[q] = a.verts[p0 + i];
          rr[q] = (int)ld_dev(reinterpret_cast<const unsigned*>(a.brel) + p0 + i);
          ro[q] = a.irow[p0 + i];
          xr[q] = a.xrow[p0 + i];
        }
      }
#pragma unroll
      for (int q = 0; q < kLoadGroup; ++q) {
        const int i = (q0 + q) * kBlock + tid;
        if (i < nv) {
          s.vert[i] = vv[q];
          s.rel[i] = rr[q];
          s.row[i] = (unsigned short)(ro[q] - e0);
          s.xrow[i] = xr[q];
        }
      }
    }
    constexpr int kEdgeGroup = 8;
    for (int q0 = 0; q0 < kPerE; q0 += kEdgeGroup) {
      if (q0 * kBlock >= ne) break;
      unsigned ev[kEdgeGroup];
#pragma unroll
      for (int q = 0; q < kEdgeGroup; ++q) {
        const int k = (q0 + q) * kBlock + tid;
        ev[q] = k < ne ? a.iedge[e0 + k] : 0u;
      }
#pragma unroll
      for (int q = 0; q < kEdgeGroup; ++q) {
        const int k = (q0 + q) * kBlock + tid;
        if (k < ne) s.edge[k] = ev[q];
      }
    }
    if (tid == 0) {
      s.row[nv] = (unsigned short)ne;
      s.xrow[nv] = a.xrow[p0 + nv];
    }
  }
  for (;;) {
    for (int k = tid; k < kBwords; k += kBlock) s.prc[k] = 0u;
    __syncthreads();
    // the current distances: device-scope loads see every other
    // workgroup's atomic minimum that completed before it marked the block
    for (int q0 = 0; q0 < kPer; q0 += 8) {
      if (q0 * kBlock >= nv) break;
      int dd[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = (q0 + q) * kBlock + tid;
        dd[q] = i < nv ? (int)ld_dev(reinterpret_cast<const unsigned*>(a.dist) + s.vert[i]) : 0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = (q0 + q) * kBlock + tid;
        if (i < nv) {
          s.dist[i] = dd[q];
          s.orig[i] = dd[q];
        }
      }
    }
    if (tid == 0) s.wl_head = s.wl_tail = 0u;
    __syncthreads();
    // the block's pending vertices of the current bucket start the worklist
    for (int base = 0; base < nv; base += kBlock) {
      const int i = base + tid;
      bool push = false;
      if (i < nv) {
        const int d = s.dist[i];
        push = d < s.rel[i] && W::bucket(a, (unsigned)d) <= cur;
      }
      blk_wl_push(s, push, i);
    }
    blk_drain<W>(a, s, c, cur);
    blk_leave_and_write<W>(a, s, c, cur);
    __syncthreads();
    if (tid == 0) {
      int again = 0;
      if (atomicCAS(a.bstate + b, kBlkOwned, 0u) != kBlkOwned) {  // dirtied while owned
        atomicExch(a.bstate + b, kBlkOwned);
        again = 1;
      }
      s.again = again;
    }
    __syncthreads();
    if (!s.again) break;
  }
}

// One round of the block engine: scan the round input (one chunk at a time,
// as run_round) and mark the blocks of its live entries, give back the
// scan token, then serve queued blocks until the round's work is done.
template <class W>
__device__ void run_round_blocks(const Args& a, BlkSmem& s, Counters& c) {
  const int tid = threadIdx.x;
  const int in_list = list_of(a, s.team, s.in_kind, s.in_index);
  const unsigned count = s.in_count;
  const unsigned tsize = (unsigned)s.team_size;
  const bool fixed = count <= tsize * (unsigned)kBlock;
  const unsigned per = fixed ? (count + tsize - 1) / tsize : (unsigned)kBlock;
  const unsigned cur = s.cur;
  if (tid == 0) s.exhausted = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      s.mode = 0;
      if (!s.exhausted) {
        unsigned base;
        if (fixed) {
          base = (unsigned)s.team_rank * per;
          s.exhausted = 1;
        } else {
          base = atomicAdd(&a.ctl->tq[s.team].in_head.v, (unsigned)kBlock);
        }
        if (base < count) {
          s.mode = 2;
          const unsigned left = count - base;
          s.nb = (int)(left < per ? left : per);
          s.gbase = base;
        } else {
          s.exhausted = 1;
        }
      }
    }
    __syncthreads();
    if (s.mode == 0) break;
    int v = -1, d = 0;
    if (tid < s.nb) {
      const int2 e = load_at(a, in_list, s.gbase + (unsigned)tid);
      v = e.x;
      d = e.y;
      if (v >= 0 && v >= a.n) {
        set_status(a.ctl, OG_ERR_INTERNAL);
        v = -1;
      }
    }
    bool repush = false, live = false;
    unsigned rb = 0;
    if (v >= 0 && d <= a.dist[v]) {
      rb = W::bucket(a, W::key(a, v, d));
      if (rb > cur) repush = true;  // a far-list entry of a later bucket
      else live = true;
    }
    wave_push_global(a, s, c, repush, blk_window_target(a, s, repush, rb), v, d, rb);
    if (live) blk_mark(a, a.blk_of[v]);
  }
  if (tid == 0) atomicSub(&a.ctl->blk_out.v, 1u);  // the scan token (every wave's marks are complete)
  for (;;) {
    __syncthreads();
    if (tid == 0) s.claim = blk_pop(a);
    __syncthreads();
    const int b = s.claim;
    if (b < 0) break;
    blk_process<W>(a, s, c, b);
    __syncthreads();
    if (tid == 0) {
      wait_vm();
      atomicSub(&a.ctl->blk_out.v, 1u);
    }
    c.batches++;
    c.round_batches++;
  }
}

// Persistent block engine: rounds separated by the device-wide barrier
// whose last arriver takes the bucket decision (as k_persistent).
template <class W>
__global__ __launch_bounds__(kBlock) void k_blocks(Args a) {
  __shared__ BlkSmem s;
  Counters c;
  if (threadIdx.x == 0) {
    init_team(a, s);
    load_control<W>(a, s);
  }
  __syncthreads();
  while (!s.done) {
    run_round_blocks<W>(a, s, c);
    round_barrier<W>(a, s, c, true, true);
    if (threadIdx.x == 0) load_control<W>(a, s);
    __syncthreads();
  }
  flush_counters(a, c);
}

// ---- building the blocked copy
//
// Blocks are the cells of a graph Voronoi partition: seeds are sampled
// (rate 1 / block_size), every vertex takes the seed nearest to it in hops
// (ties to the smaller seed id, so the partition is unique), found by a
// level-synchronous multi-source BFS along out-edges.  A cell with more than
// kBcap vertices or kEcap internal edges is split by re-running the BFS over
// it from two seeds, its old one and its farthest vertex; vertices no seed
// reaches are sampled again at a higher rate.  A label packs (hops << 32 |
// seed).
constexpr unsigned long long kNoLab = ~0ull;

__device__ __forceinline__ unsigned long long cl_lab(unsigned hop, int v) {
  return ((unsigned long long)hop << 32) | (unsigned)v;
}
__device__ __forceinline__ int cl_seed(unsigned long long l) { return (int)(unsigned)(l & 0xffffffffull); }
// 32-bit integer hash (the finaliser of MurmurHash3)
__device__ __forceinline__ unsigned cl_hash(unsigned x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  return x ^ (x >> 16);
}
__device__ __forceinline__ bool cl_internal(int v, int u, int w, int bv, int bu) {
  return u != v && bu == bv && w >= 0 && w < kIedgeWmax;
}

// Which vertices this pass labels (fr = 1) and its seeds: unlabelled
// vertices are sampled at 1 / rate.  A vertex of an oversized cell is
// reset; the cell's seed and its farthest vertex stay seeds, and more are
// sampled in it, about twice as many as the pieces it must be cut into,
// doubled on every further pass (from pass 17 on every vertex is a seed,
// and a one-vertex cell is never oversized, so the passes end).
__global__ __launch_bounds__(kBlock) void k_cl_prep(int n, unsigned long long* lab, int* fr, const int* over,
                                                     const unsigned long long* far, const int* cnt, const int* ecnt,
                                                     unsigned rate, int target, int pass, unsigned salt) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    unsigned long long l = pass == 0 ? kNoLab : lab[v];
    int f = 0;
    if (l == kNoLab) {
      f = 1;
      l = cl_hash((unsigned)v ^ salt) % rate == 0u ? cl_lab(0, (int)v) : kNoLab;
    } else {
      const int sd = cl_seed(l);
      if (over[sd]) {
        f = 1;
        const long long c = cnt[sd], pieces_v = (c + target - 1) / target,
                        pieces_e = ((long long)ecnt[sd] + kEcap / 2 - 1) / (kEcap / 2);
        long long dens = (pieces_v > pieces_e ? pieces_v : pieces_e) * 2;
        dens <<= (pass < 16 ? pass : 16);
        const unsigned r = c / dens > 1 ? (unsigned)(c / dens) : 1u;
        l = (v == sd || v == cl_seed(far[sd]) || cl_hash((unsigned)v ^ salt) % r == 0u) ? cl_lab(0, (int)v) : kNoLab;
      }
    }
    lab[v] = l;
    fr[v] = f;
  }
}

// One BFS level over the vertices being labelled: a vertex at `level` hops
// offers (level + 1, its seed) to its free out-neighbours.
__global__ __launch_bounds__(kBlock) void k_cl_bfs(int n, const long long* row_ptr, const int* col,
                                                    unsigned long long* lab, const int* fr, unsigned level,
                                                    unsigned* changed) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool any = false;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    if (!fr[v]) continue;
    const unsigned long long l = lab[v];
    if (l == kNoLab || (unsigned)(l >> 32) != level) continue;
    const unsigned long long cand = cl_lab(level + 1u, cl_seed(l));
    for (long long e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int u = col[e];
      if (u == v || !fr[u] || cand >= lab[u]) continue;
      if (atomicMin(&lab[u], cand) > cand) any = true;
    }
  }
  if (__ballot(any) != 0 && lane_id() == 0) atomicAdd(changed, 1u);
}

// Cell sizes, internal edge counts and each cell's farthest vertex.
__global__ __launch_bounds__(kBlock) void k_cl_count(int n, const long long* row_ptr, const int* col, const int* w,
                                                      const unsigned long long* lab, int* cnt, int* ecnt,
                                                      unsigned long long* far) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const unsigned long long l = lab[v];
    if (l == kNoLab) continue;
    const int sd = cl_seed(l);
    atomicAdd(&cnt[sd], 1);
    int k = 0;
    for (long long e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int u = col[e];
      const unsigned long long lu = lab[u];
      if (lu != kNoLab && cl_internal((int)v, u, w[e], sd, cl_seed(lu))) ++k;
    }
    if (k) atomicAdd(&ecnt[sd], k);
    atomicMax(&far[sd], ((l >> 32) << 32) | (unsigned long long)v);
  }
}

// Oversized cells (flagged by seed) and the vertices still unlabelled.
__global__ __launch_bounds__(kBlock) void k_cl_over(int n, const unsigned long long* lab, const int* cnt,
                                                     const int* ecnt, int* over, unsigned* flags) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool o_any = false, u_any = false;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const bool o = cnt[v] > kBcap || ecnt[v] > kEcap;
    over[v] = o ? 1 : 0;
    o_any |= o;
    u_any |= lab[v] == kNoLab;
  }
  if (__ballot(o_any) != 0 && lane_id() == 0) atomicAdd(&flags[0], 1u);
  if (__ballot(u_any) != 0 && lane_id() == 0) atomicAdd(&flags[1], 1u);
}

// seed flags (a seed is the only vertex at hop 0 of its own cell)
__global__ __launch_bounds__(kBlock) void k_cl_isseed(int n, const unsigned long long* lab, int* flag) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride)
    flag[v] = v < n && lab[v] == cl_lab(0, (int)v) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_cl_assign(int n, const unsigned long long* lab, const int* bid,
                                                       int* blk_of, int* bsize) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int b = bid[cl_seed(lab[v])];
    blk_of[v] = b;
    atomicAdd(&bsize[b], 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_cl_scatter(int n, const int* blk_of, const int* bstart, int* fill,
                                                        int* verts) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int b = blk_of[v];
    verts[bstart[b] + atomicAdd(&fill[b], 1)] = (int)v;
  }
}

// Each block's vertices in increasing id order (bitonic sort in LDS, one
// workgroup per block), so that the blocked order does not depend on the
// order of the scatter's atomics.
__global__ __launch_bounds__(kBlock) void k_cl_sort(int nb, const int* bstart, int* verts) {
  __shared__ int key[kBcap];
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int p0 = bstart[b], nv = bstart[b + 1] - p0;
    if (nv > kBcap) continue;  // never built (the engine reports such a block as internal)
    int np = 1;
    while (np < nv) np <<= 1;
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += kBlock) key[i] = i < nv ? verts[p0 + i] : INT_MAX;
    for (int k = 2; k <= np; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        __syncthreads();
        for (int i = threadIdx.x; i < np; i += kBlock) {
          const int l = i ^ j;
          if (l > i) {
            const int x = key[i], y = key[l];
            if (((i & k) == 0) == (x > y)) {
              key[i] = y;
              key[l] = x;
            }
          }
        }
      }
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += kBlock) verts[p0 + i] = key[i];
  }
}

// Per block: first position, vertices, first internal edge, internal edges.
__global__ __launch_bounds__(kBlock) void k_cl_meta(int nb, const int* bstart, const int* irow, int4* bmeta) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += stride) {
    const int p0 = bstart[b], p1 = bstart[b + 1];
    bmeta[b] = make_int4(p0, p1 - p0, irow[p0], irow[p1] - irow[p0]);
  }
}

__global__ __launch_bounds__(kBlock) void k_cl_pos(int n, const int* verts, int* pos) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) pos[verts[p]] = (int)p;
}

// Internal and leaving edges of the vertex at each position.
__global__ __launch_bounds__(kBlock) void k_cl_ecount(int n, const long long* row_ptr, const int* col, const int* w,
                                                       const int* verts, const int* blk_of, int* icnt, int* xcnt) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p <= n; p += stride) {
    int ki = 0, kx = 0;
    if (p < n) {
      const int v = verts[p], b = blk_of[v];
      for (long long e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        const int u = col[e];
        if (cl_internal(v, u, w[e], b, blk_of[u])) ++ki;
        else ++kx;
      }
    }
    icnt[p] = ki;
    xcnt[p] = kx;
  }
}

__global__ __launch_bounds__(kBlock) void k_cl_efill(int n, const long long* row_ptr, const int* col, const int* w,
                                                      const int* verts, const int* blk_of, const int* pos,
                                                      const int* bstart, const int* irow, const int* xrow,
                                                      unsigned* iedge, int* xcol, int* xw, int* xblk) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int v = verts[p], b = blk_of[v];
    int ki = irow[p], kx = xrow[p];
    for (long long e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int u = col[e], wt = w[e], bu = blk_of[u];
      if (cl_internal(v, u, wt, b, bu)) {
        iedge[ki++] = (unsigned)(pos[u] - bstart[b]) | ((unsigned)wt << 16);
      } else {
        xcol[kx] = u;
        xw[kx] = wt;
        xblk[kx] = bu;
        ++kx;
      }
    }
  }
}

// Exclusive prefix sum of n ints in tiles of kScanTile: per-tile scans with
// their totals, a scan of the totals by one workgroup, then the tile
// offsets added.
constexpr int kScanPer = 8;
constexpr int kScanTile = kBlock * kScanPer;

__device__ int blk_scan_excl(int x, int* wsum, int* total) {
  const int lane = (int)lane_id(), wid = threadIdx.x / kWave;
  int v = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) wsum[wid] = v;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const int t = wsum[i];
    pre += i < wid ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return pre + v - x;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int* in, int* out, long long n, int* tile_sum) {
  __shared__ int wsum[kWaves];
  const long long t0 = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanPer;
  int x[kScanPer];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    x[k] = t0 + k < n ? in[t0 + k] : 0;
    sum += x[k];
  }
  int total;
  int run = blk_scan_excl(sum, wsum, &total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (t0 + k < n) out[t0 + k] = run;
    run += x[k];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(int* tile_sum, int ntiles) {
  __shared__ int wsum[kWaves];
  int carry = 0;
  for (int base = 0; base < ntiles; base += kBlock) {
    const int i = base + (int)threadIdx.x;
    const int x = i < ntiles ? tile_sum[i] : 0;
    int total;
    const int e = blk_scan_excl(x, wsum, &total);
    if (i < ntiles) tile_sum[i] = carry + e;
    carry += total;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int* out, long long n, const int* tile_sum) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] += tile_sum[i / kScanTile];
}

// Parity summary of the final distances for the predecessor pass: bit
// v % 64 of word v / 64 is the lowest bit of dist[v]'s bit pattern (one bit
// per vertex, 32 times smaller than dist).
__global__ __launch_bounds__(kBlock) void k_pred_summary(Args a, unsigned long long* sum) {
  const long long nv = a.n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long base = (long long)blockIdx.x * blockDim.x; base < nv; base += stride) {
    const long long v = base + threadIdx.x;
    const unsigned long long word = __ballot(v < nv && (a.dist[v] & 1));
    if (lane_id() == 0 && v < nv) sum[v >> 6] = word;
  }
}

// Whether the summary allows dist[u] to equal the would-be distance c: an
// edge whose c has the other parity is not tight, and its random dist read
// is saved.
__device__ __forceinline__ bool par_ok(const unsigned long long* sum, long long u, unsigned c) {
  return ((unsigned)(sum[u >> 6] >> (u & 63)) & 1u) == (c & 1u);
}

// Canonical predecessors: for every edge (u,v) of every query copy with
// dist[u] finite and dist[u] + w == dist[v], pred[v] = min(pred[v], u) (base
// vertex ids).  One wavefront per chunk of 64 consecutive source vertices of
// one copy: a wavefront scan numbers the chunk's edges, which the lanes then
// take 64 at a time, each finding its source lane by a binary search over
// the lanes' offsets; the edge loads of consecutive lanes are contiguous
// within a row.  When longs is given, a row longer than kPredLong edges is
// left out and listed instead as slices of kPredSlice edges (at most lcap
// entries) for k_pred_long.  With the parity summary (kPar), edges that
// cannot be tight by parity skip their dist read.  Also counts reached vertices and
// edges.  pred == nullptr: counts only.
template <class W, bool kPar>
__global__ __launch_bounds__(kBlock) void k_pred_edges(Args a, int* pred, int2* longs, unsigned long long lcap,
                                                       const unsigned long long* sum) {
  const int lane = (int)lane_id();
  const long long nwave = (long long)gridDim.x * (kBlock / kWave);
  const long long per_copy = ((long long)a.nbase + kWave - 1) / kWave;
  const long long chunks = per_copy * a.reps;
  unsigned long long rv = 0, re = 0;
  for (long long ch = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; ch < chunks; ch += nwave) {
    const long long q = ch / per_copy;
    const long long voff = q * a.nbase;
    const long long v0 = (ch - q * per_copy) * kWave;
    const long long v = v0 + lane;
    const long long e0 = a.row_ptr[v0];
    long long r0 = e0, r1 = e0;
    if (v < a.nbase) {
      r0 = a.row_ptr[v];
      r1 = a.row_ptr[v + 1];
    }
    const int dv = v < a.nbase ? a.dist[voff + v] : W::kInfBits;
    const int deg = (int)(r1 - r0);
    if (v < a.nbase && dv != W::kInfBits) {
      rv++;
      re += (unsigned long long)deg;
    }
    if (!pred) continue;
    const bool live = dv != W::kInfBits && deg > 0;
    const bool is_long = live && longs && deg > kPredLong;
    if (is_long) {  // its edges go to k_pred_long
      const unsigned nsl = (unsigned)((deg + kPredSlice - 1) / kPredSlice);
      const unsigned long long at = atomicAdd(&a.ctl->pred_slices.v, (unsigned long long)nsl);
      if (at + nsl <= lcap) {
        for (unsigned k = 0; k < nsl; ++k) longs[at + k] = make_int2((int)(voff + v), (int)k);
      } else {
        set_status(a.ctl, OG_ERR_INTERNAL);
      }
    }
    const int eff = live && !is_long ? deg : 0;
    int inc = eff;  // inclusive scan of eff over the wavefront
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int t = __shfl_up(inc, o);
      if (lane >= o) inc += t;
    }
    const int total = __shfl(inc, kWave - 1);
    const int off = inc - eff;
    const int rel = (int)(r0 - e0);
    // kPredIlp groups of 64 edges per step, their loads in flight together
    for (int k0 = 0; k0 < total; k0 += kPredIlp * kWave) {
      int cj[kPredIlp], du[kPredIlp], wt[kPredIlp], dd[kPredIlp], src[kPredIlp];
      bool ok[kPredIlp];
#pragma unroll
      for (int j = 0; j < kPredIlp; ++j) {  // edge loads of every group
        const int k = k0 + j * kWave + lane;
        int lo = 0;  // the last lane whose offset is <= k: it owns edge k
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
          const int o2 = __shfl(off, lo + step);
          if (o2 <= k) lo += step;
        }
        du[j] = __shfl(dv, lo);
        const int rj = __shfl(rel, lo);
        const int oj = __shfl(off, lo);
        src[j] = lo;
        ok[j] = k < total;
        cj[j] = 0;
        wt[j] = 0;
        if (ok[j]) {
          const long long e = e0 + rj + (k - oj);
          cj[j] = a.col[e];
          wt[j] = a.w[e];
        }
      }
#pragma unroll
      for (int j = 0; j < kPredIlp; ++j) {
        if constexpr (kPar) ok[j] = ok[j] && par_ok(sum, voff + cj[j], W::cand(du[j], wt[j]));
        dd[j] = ok[j] ? a.dist[voff + cj[j]] : 0;
      }
#pragma unroll
      for (int j = 0; j < kPredIlp; ++j)
        if (ok[j] && W::tight(du[j], wt[j], dd[j])) atomicMin(&pred[voff + cj[j]], (int)(v0 + src[j]));
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    rv += __shfl_xor(rv, o);
    re += __shfl_xor(re, o);
  }
  if (lane == 0) {
    if (rv) atomicAdd(&a.ctl->st[kStReachedV].v, rv);
    if (re) atomicAdd(&a.ctl->st[kStReachedE].v, re);
  }
}

// The long rows listed by k_pred_edges: one wavefront per slice of
// kPredSlice edges, the same test per edge.
template <class W, bool kPar>
__global__ __launch_bounds__(kBlock) void k_pred_long(Args a, int* pred, const int2* longs, unsigned long long lcap,
                                                      const unsigned long long* sum) {
  // more than lcap slices only for a malformed graph: the call then ends
  // with OG_ERR_INTERNAL and the list is not read
  const unsigned long long count =
      __hip_atomic_load(&a.ctl->pred_slices.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (count > lcap) return;
  const int lane = (int)lane_id();
  const long long nwave = (long long)gridDim.x * (kBlock / kWave);
  for (long long i = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < (long long)count;
       i += nwave) {
    const int2 ent = longs[i];
    const int vb = a.reps == 1 ? ent.x : (int)((unsigned)ent.x % (unsigned)a.nbase);
    const long long voff = (long long)ent.x - vb;
    const long long r1 = a.row_ptr[vb + 1];
    const long long s0 = a.row_ptr[vb] + (long long)ent.y * kPredSlice;
    const long long s1 = s0 + kPredSlice < r1 ? s0 + kPredSlice : r1;
    const int du = a.dist[ent.x];
    for (long long eb = s0; eb < s1; eb += kPredIlp * kWave) {
      int cj[kPredIlp], wt[kPredIlp], dd[kPredIlp];
      bool ok[kPredIlp];
#pragma unroll
      for (int j = 0; j < kPredIlp; ++j) {
        const long long e = eb + j * kWave + lane;
        ok[j] = e < s1;
        cj[j] = 0;
        wt[j] = 0;
        if (ok[j]) {
          cj[j] = a.col[e];
          wt[j] = a.w[e];
        }
      }
#pragma unroll
      for (int j = 0; j < kPredIlp; ++j) {
        if constexpr (kPar) ok[j] = ok[j] && par_ok(sum, voff + cj[j], W::cand(du, wt[j]));
        dd[j] = ok[j] ? a.dist[voff + cj[j]] : 0;
      }
#pragma unroll
      for (int j = 0; j < kPredIlp; ++j)
        if (ok[j] && W::tight(du, wt[j], dd[j])) atomicMin(&pred[voff + cj[j]], vb);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_pred_fix(int* pred, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    if (pred[v] == kInf) pred[v] = -1;
}

__global__ __launch_bounds__(kBlock) void k_pred_sources(Args a, int* pred) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.nsrc; i += gridDim.x * blockDim.x) {
    const int s = a.srcs[i];
    pred[s] = a.reps == 1 ? s : (int)((unsigned)s % (unsigned)a.nbase);
  }
}

// Tree edge of every vertex from its (canonical) predecessor: the index of
// the edge pred[v] -> v, found by binary search in pred[v]'s row (rows are
// sorted by destination).  -1 for the source and unreachable vertices.
__global__ __launch_bounds__(kBlock) void k_pred_edge_ids(Args a, const int* pred, int* pred_edge) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int p = pred[v];
    int e = -1;
    if (p >= 0 && p != (int)v) {
      long long lo = a.row_ptr[p], hi = a.row_ptr[p + 1] - 1;
      while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (a.col[mid] < (int)v) lo = mid + 1;
        else hi = mid;
      }
      if (lo <= hi && a.col[lo] == (int)v) e = (int)lo;
    }
    pred_edge[v] = e;
  }
}

// Backward pass of the differentiable search (reverse-topological subtree
// sums over the shortest-path tree): grad_w[e] for the tree edge e into v
// is the sum of grad_dist over v's subtree; non-tree edges get 0.  The
// workspace holds acc (float64 running sums), kids (tree children, fixed
// once counted) and pending (children not yet folded in).
__global__ __launch_bounds__(kBlock) void k_bw_init(const float* grad_dist, int n, float* grad_w, long long m,
                                                     double* acc, int* kids, int* pending) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long v = t0; v < n; v += stride) {
    acc[v] = (double)grad_dist[v];
    kids[v] = 0;
    pending[v] = 0;
  }
  for (long long e = t0; e < m; e += stride) grad_w[e] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_bw_count(const int* pred, const int* pred_edge, int n, int* kids,
                                                      int* pending) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    if (pred_edge[v] >= 0) {
      atomicAdd(&kids[pred[v]], 1);
      atomicAdd(&pending[pred[v]], 1);
    }
}

// Every leaf (kids == 0, never changed by this kernel) climbs towards the
// root, adding its subtree sum into its parent; the child that folds in
// last (its decrement of the parent's pending count reaches zero) carries
// on from the parent, whose sum is then complete.  Each addition finishes
// before the decrement that announces it (wait for completion), so the last
// child reads the full sum.
__global__ __launch_bounds__(kBlock) void k_bw_climb(const int* pred, const int* pred_edge, int n, float* grad_w,
                                                      double* acc, const int* kids, int* pending) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    if (pred_edge[v] < 0 || kids[v] != 0) continue;  // not a leaf of the tree
    int x = (int)v;
    double val = acc[x];
    for (;;) {
      const int e = pred_edge[x];
      if (e < 0) break;
      grad_w[e] = (float)val;
      const int p = pred[x];
      (void)atomicAdd(&acc[p], val);
      wait_vm();
      if (atomicSub(&pending[p], 1) != 1) break;
      x = p;
      val = __hip_atomic_load(&acc[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ------------------------------------------------------------------ host

struct DeviceInfo {
  int cus = 0;
  int occ_int = 0;    // co-resident k_persistent<IntW> workgroups per CU
  int occ_float = 0;  // co-resident k_persistent<FloatW> workgroups per CU
  int occ_core = 0;   // co-resident k_persistent<CoreW> workgroups per CU
  int occ_split = 0;  // co-resident k_persistent<SplitW> workgroups per CU
  int occ_pull = 0;   // co-resident k_persistent<PullW> workgroups per CU
  int occ_core_pull = 0;  // co-resident k_persistent<CorePullW> workgroups per CU
  int occ_bin = 0;    // co-resident k_persistent<BinW> workgroups per CU
  int occ_bin_float = 0;  // co-resident k_persistent<BinFloatW> workgroups per CU
  int occ_blocks = 0;  // co-resident k_blocks<BlockW> workgroups per CU
  int coop = 0;
  bool valid = false;
};

std::mutex g_info_mu;
DeviceInfo g_info[64];

bool device_info(int dev, DeviceInfo* out) {
  if (dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(g_info_mu);
  DeviceInfo& di = g_info[dev];
  if (!di.valid) {
    if (hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&di.coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_int, k_persistent<IntW>, kBlock, 0) != hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_float, k_persistent<FloatW>, kBlock, 0) != hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_core, k_persistent<CoreW>, kBlock, 0) != hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_split, k_persistent<SplitW>, kBlock, 0) != hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_pull, k_persistent<PullW>, kBlock, 0) != hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_core_pull, k_persistent<CorePullW>, kBlock, 0) !=
        hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_bin, k_persistent<BinW>, kBlock, 0) != hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_bin_float, k_persistent<BinFloatW>, kBlock, 0) !=
        hipSuccess)
      return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&di.occ_blocks, k_blocks<BlockW>, kBlock, 0) != hipSuccess)
      return false;
    di.valid = true;
  }
  *out = di;
  return true;
}

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Split copies of the rows held by workspaces (light/heavy split): the
// workspace, the graph's arrays and sizes, Delta and where the copy lies.
// A split call records what it built; every other call on a workspace
// forgets it, since its layout may cover the copy.  With OG_FLAG_KEEP_SPLIT
// a split call whose record matches reuses the copy instead of rebuilding.
struct SplitKey {
  const void* ws;
  const void* row_ptr;
  const void* col;
  const void* w;
  long long n, m;
  unsigned delta;  // the split's Delta, or the blocked copy's target block size
  const void* copy;
  int kind;           // 0: light/heavy split copy, 1: blocked copy
  long long nb = 0;   // blocked copy: its block count (not part of the match)
  bool operator==(const SplitKey& o) const {
    return ws == o.ws && row_ptr == o.row_ptr && col == o.col && w == o.w && n == o.n && m == o.m &&
           delta == o.delta && copy == o.copy && kind == o.kind;
  }
};
std::mutex g_split_mu;
std::vector<SplitKey> g_split_keys;

void forget_split(const void* ws) {
  std::lock_guard<std::mutex> lk(g_split_mu);
  g_split_keys.erase(std::remove_if(g_split_keys.begin(), g_split_keys.end(),
                                    [&](const SplitKey& k) { return k.ws == ws; }),
                     g_split_keys.end());
}

bool split_kept(const SplitKey& key, long long* nb = nullptr) {
  std::lock_guard<std::mutex> lk(g_split_mu);
  const auto it = std::find(g_split_keys.begin(), g_split_keys.end(), key);
  if (it == g_split_keys.end()) return false;
  if (nb) *nb = it->nb;
  return true;
}

void record_split(const SplitKey& key) {
  std::lock_guard<std::mutex> lk(g_split_mu);
  g_split_keys.erase(std::remove_if(g_split_keys.begin(), g_split_keys.end(),
                                    [&](const SplitKey& k) { return k.ws == key.ws; }),
                     g_split_keys.end());
  if (g_split_keys.size() >= 64) g_split_keys.erase(g_split_keys.begin());
  g_split_keys.push_back(key);
}

// Per-thread HIP events for OG_FLAG_TIMING (created on first use, destroyed
// by og_release).
struct Timers {
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool ok = false;
  bool init() {
    if (ok) return true;
    for (auto& e : ev)
      if (!e && hipEventCreate(&e) != hipSuccess) return false;
    ok = true;
    return true;
  }
  bool release() {
    bool good = true;
    for (auto& e : ev) {
      if (e && hipEventDestroy(e) != hipSuccess) good = false;
      e = nullptr;
    }
    ok = false;
    return good;
  }
};
thread_local Timers t_timers;

og_schedule resolved(const og_schedule* s) {
  og_schedule r = *s;
  if (r.update != OG_EAGER_NO_FUSION && r.update != OG_LAZY_UPDATE) r.update = OG_EAGER_WITH_FUSION;
  if (r.fusion_threshold <= 0) r.fusion_threshold = kDefaultThreshold;
  if (r.fusion_threshold > kLq) r.fusion_threshold = kLq;
  if (r.window_buckets <= 0) r.window_buckets = kDefaultK;
  if (r.bin_thread == 0) r.bin_thread = kBinLane;
  if (r.bin_thread > kBinLane) r.bin_thread = kBinLane;
  if (r.bin_wave == 0) r.bin_wave = kDefaultBinWave;
  if (r.block_size <= 0) r.block_size = kDefaultBlockSize;
  if (r.block_size > kBcap) r.block_size = kBcap;
  r.window_buckets = pow2_at_least(r.window_buckets < 2 ? 2 : r.window_buckets);
  return r;
}

// A call's shape: reps copies of the graph, nsrc sources, targets or not;
// core: a k-core decomposition (every vertex starts filed, no sources).
struct Shape {
  int reps;
  int nsrc;
  bool targets;
  bool core = false;
};

long long queue_cap(const og_graph* g, const og_schedule* r, const Shape& sh) {
  const long long per = sh.core ? 2LL * g->n + g->m / 8 : (long long)g->n + g->m / 8;
  long long cap = r->queue_capacity > 0 ? r->queue_capacity : (long long)sh.reps * per + (sh.core ? 0 : sh.nsrc);
  if (cap < 1024) cap = 1024;
  if (cap > 0x7fffffffLL) cap = 0x7fffffffLL;
  if (cap < sh.nsrc) cap = sh.nsrc;  // the sources start in a far list
  return cap;
}

size_t table_bytes(const Shape& sh) {
  if (sh.core) return 0;
  const size_t b = sizeof(int) * ((size_t)sh.nsrc + (sh.targets ? (size_t)sh.reps : 0));
  return (b + 255) & ~(size_t)255;
}

// Teams a call may split its workgroups into (its workspace holds their
// lists): a batched launch of the eager push engine, schedule.teams (0 =
// one per query up to 8, one per XCD: each team runs rounds of its own, the
// fastest on the road grid), at most one per query; any other call one.
// The launch runs min(that, workgroups).
int team_cap(const og_schedule* r, const Shape& sh) {
  if (sh.core || sh.reps < 2 || r->update == OG_LAZY_UPDATE) return 1;
  if (r->flags & (OG_FLAG_LIGHT_HEAVY | OG_FLAG_DENSE_PULL | OG_FLAG_HYBRID_DIRECTION | OG_FLAG_VERTEX_BLOCKS))
    return 1;
  int t = r->teams > 0 ? r->teams : kMaxTeams;
  if (t > kMaxTeams) t = kMaxTeams;
  if (t > sh.reps) t = sh.reps;
  return t;
}

// The global lists' pool, from byte offset off: the chunk tables (one per
// list of each team, tchunks entries each), the free stack and the chunks.
// When the call runs one team, far list 0 starts with chunks 0 .. pre-1,
// which hold the sources (k-core: every vertex); with more, each source
// takes its chunk through the usual hand-over.  Pool size: schedule.queue_pool entries rounded up to whole
// chunks, by default twice one list's capacity plus one chunk per list (the
// partly filled last chunks), never more than every list full at once, and
// never fewer than the sources' chunks plus one, nor than one chunk per team.
struct PoolLayout {
  unsigned tchunks, chunks, pre;
  size_t ctab, fstack, pool, end;
};

PoolLayout pool_layout(const og_schedule* r, const Shape& sh, long long cap, int teams, size_t off) {
  PoolLayout L;
  const long long ck = (long long)kChunk;
  const long long lists = (long long)teams * (r->window_buckets + 4);  // per team: K window slots, 2 spill, 2 far
  L.tchunks = (unsigned)((cap + ck - 1) / ck);
  L.pre = (unsigned)(((long long)sh.nsrc + ck - 1) / ck);  // far list 0's first chunks when one team runs
  long long ch = r->queue_pool > 0 ? (r->queue_pool + ck - 1) / ck : (2 * cap + ck - 1) / ck + lists;
  if (ch > lists * (long long)L.tchunks) ch = lists * (long long)L.tchunks;
  if (ch < (long long)L.pre + 1) ch = (long long)L.pre + 1;
  if (ch < teams) ch = teams;  // a chunk for every team's share
  L.chunks = (unsigned)ch;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  L.ctab = take(sizeof(int) * (size_t)lists * L.tchunks);
  L.fstack = take(sizeof(int) * (size_t)L.chunks);
  L.pool = take(sizeof(int2) * (size_t)L.chunks * kChunk);
  L.end = off;
  return L;
}

bool split_on(const og_schedule* r, const Shape& sh) { return !sh.core && (r->flags & OG_FLAG_LIGHT_HEAVY); }
bool blocks_on(const og_schedule* r, const Shape& sh) { return !sh.core && (r->flags & OG_FLAG_VERTEX_BLOCKS); }

// Workspace regions of the vertex-block engine, from byte offset off: the
// blocked copy (kept across calls with OG_FLAG_KEEP_BLOCKS), the per-query
// state, and the temporaries of building the copy.
struct BlkLayout {
  size_t bstart, bmeta, verts, blk_of, irow, xrow, iedge, xcol, xw, xblk;  // blocked copy
  size_t brel, bstate, ring;                                         // per query
  size_t lab, fr, cnt, ecnt, far, over, flag, bsize, fill, pos, icnt, xcnt, tiles, flags;  // build
  size_t end;
  unsigned long long ring_cap;
};

BlkLayout blk_layout(long long n, long long m, size_t off) {
  BlkLayout L;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t N = (size_t)n, M = (size_t)m;
  L.bstart = take(4 * (N + 1));
  L.bmeta = take(16 * N);
  L.verts = take(4 * N);
  L.blk_of = take(4 * N);
  L.irow = take(4 * (N + 1));
  L.xrow = take(4 * (N + 1));
  L.iedge = take(4 * M);
  L.xcol = take(4 * M);
  L.xw = take(4 * M);
  L.xblk = take(4 * M);
  L.brel = take(4 * N);
  L.bstate = take(4 * N);
  L.ring_cap = 1;
  while (L.ring_cap < N + 1) L.ring_cap <<= 1;  // more slots than blocks
  L.ring = take(8 * (size_t)L.ring_cap);
  L.lab = take(8 * N);
  L.fr = take(4 * N);
  L.cnt = take(4 * N);
  L.ecnt = take(4 * N);
  L.far = take(8 * N);
  L.over = take(4 * N);
  L.flag = take(4 * (N + 1));
  L.bsize = take(4 * (N + 1));
  L.fill = take(4 * N);
  L.pos = take(4 * N);
  L.icnt = take(4 * (N + 1));
  L.xcnt = take(4 * (N + 1));
  L.tiles = take(4 * ((N + 1) / kScanTile + 2));
  L.flags = take(256);
  L.end = off;
  return L;
}

int pull_mode(const og_schedule* r) {
  return (r->flags & OG_FLAG_DENSE_PULL) ? kPullAlways : (r->flags & OG_FLAG_HYBRID_DIRECTION) ? kPullHybrid : kPullNever;
}

// Per-vertex int arrays after the queues: lazy change flags / counts and
// the change buffer (lazy), peel marks (k-core); each 256-byte aligned.
size_t vec_bytes(long long n) { return ((size_t)n * sizeof(int) + 255) & ~(size_t)255; }

size_t ws_bytes_for(const og_graph* g, const og_schedule* r, const Shape& sh) {
  const long long cap = queue_cap(g, r, sh);
  size_t b = pool_layout(r, sh, cap, team_cap(r, sh), kCtlBytes + table_bytes(sh)).end;
  const long long nv = (long long)sh.reps * g->n;
  if (r->update == OG_LAZY_UPDATE) b += 2 * vec_bytes(nv);
  if (sh.core) b += vec_bytes(nv);
  // light/heavy split: col and w copies, light counts, long-row list, bucket
  // stamps and two heavy lists of (v, slice) entries
  if (split_on(r, sh))
    b += 2 * vec_bytes(g->m) + 2 * vec_bytes(g->n) + vec_bytes(nv) + 4 * vec_bytes(heavy_cap(nv, g->m, sh.reps));
  // pull direction: frontier marks ((stamp, distance) pairs; k-core: a
  // bitmap) and the long rows' slices
  if (pull_mode(r) != kPullNever)
    b += (sh.core ? vec_bytes((nv + 31) / 32) : vec_bytes(2 * nv)) + vec_bytes(2 * (long long)slice_cap(g->m));
  if (blocks_on(r, sh)) b = blk_layout(g->n, g->m, b).end;
  return b;
}

bool schedule_ok(const og_schedule* s) {
  if (!s) return false;
  if (s->delta < 1) return false;
  if (s->update != OG_EAGER_NO_FUSION && s->update != OG_EAGER_WITH_FUSION && s->update != OG_LAZY_UPDATE)
    return false;
  if (s->fusion_threshold < 0 || s->window_buckets < 0 || s->window_buckets > kKmax) return false;
  if (s->window_buckets == 1) return false;
  if (s->engine != OG_ENGINE_PERSISTENT && s->engine != OG_ENGINE_HOST_ROUNDS && s->engine != OG_ENGINE_GRAPH_ROUNDS)
    return false;
  if (s->max_rounds < 0 || s->workgroups < 0 || s->queue_capacity < 0 || s->queue_pool < 0 || s->teams < 0)
    return false;
  if (s->flags & ~(OG_FLAG_VALIDATE | OG_FLAG_ASYNC | OG_FLAG_TIMING | OG_FLAG_LIGHT_HEAVY | OG_FLAG_DENSE_PULL |
                   OG_FLAG_HYBRID_DIRECTION | OG_FLAG_DEGREE_BINS | OG_FLAG_KEEP_SPLIT | OG_FLAG_VERTEX_BLOCKS |
                   OG_FLAG_KEEP_BLOCKS))
    return false;
  if (s->bin_thread < 0 || s->bin_wave < 0 || s->block_size < 0) return false;
  // the vertex-block engine: its own instantiation, always fused, persistent
  if ((s->flags & OG_FLAG_VERTEX_BLOCKS) &&
      ((s->flags & (OG_FLAG_LIGHT_HEAVY | OG_FLAG_DEGREE_BINS | OG_FLAG_DENSE_PULL | OG_FLAG_HYBRID_DIRECTION)) ||
       s->update != OG_EAGER_WITH_FUSION || s->engine != OG_ENGINE_PERSISTENT))
    return false;
  // degree bins are their own instantiation: not with the split or a pull direction
  if ((s->flags & OG_FLAG_DEGREE_BINS) &&
      (s->flags & (OG_FLAG_LIGHT_HEAVY | OG_FLAG_DENSE_PULL | OG_FLAG_HYBRID_DIRECTION)))
    return false;
  if ((s->flags & OG_FLAG_LIGHT_HEAVY) && s->update == OG_LAZY_UPDATE) return false;
  // a direction other than push: lazy updates only, one direction flag
  if ((s->flags & OG_FLAG_DENSE_PULL) && (s->flags & OG_FLAG_HYBRID_DIRECTION)) return false;
  if ((s->flags & (OG_FLAG_DENSE_PULL | OG_FLAG_HYBRID_DIRECTION)) && s->update != OG_LAZY_UPDATE) return false;
  return true;
}

bool graph_ok(const og_graph* g, bool weighted = true) {
  if (!g || g->n < 1 || g->m < 0 || g->m > 0x7fffffffLL || !g->row_ptr) return false;
  if (g->m > 0 && (!g->col || (weighted && !g->w))) return false;
  return true;
}

bool shape_ok(const og_graph* g, const Shape& sh) {
  if (sh.reps < 1 || sh.reps > kMaxQueries || sh.nsrc < 1 || sh.nsrc > 0x7fffffff / 2) return false;
  return (long long)sh.reps * g->n < 0x7fffffffLL;
}

void fill_stats(const Ctl& h, og_stats* st, int nwg) {
  if (!st) return;
  st->status = (og_status)h.status.v;
  st->workgroups = nwg;
  // teams run rounds of their own: the rounds, barriers and critical path of
  // the team that took the most, the buckets of all teams, and the pool a
  // split into equal team shares needs
  const int T = h.teams.v >= 1 && h.teams.v <= (unsigned)kMaxTeams ? (int)h.teams.v : 1;
  int64_t rounds = 0, buckets = 0, barriers = 0, chain = 0, peak = 0;
  for (int t = 0; t < T; ++t) {
    rounds = std::max<int64_t>(rounds, h.tc[t].round);
    buckets += h.tc[t].buckets;
    barriers = std::max<int64_t>(barriers, h.tc[t].epoch);
    chain = std::max<int64_t>(chain, (int64_t)h.chain[t].v);
    peak = std::max<int64_t>(peak, h.pool_peak[t].v);
  }
  st->rounds = rounds;
  st->buckets = buckets;
  st->relaxations = (int64_t)h.st[kStRelax].v;
  st->improvements = (int64_t)h.st[kStImprove].v;
  st->pushes_local = (int64_t)h.st[kStPushLocal].v;
  st->pushes_global = (int64_t)h.st[kStPushGlobal].v;
  st->far_pushes = (int64_t)h.st[kStFar].v;
  st->reached_vertices = (int64_t)h.st[kStReachedV].v;
  st->reached_edges = (int64_t)h.st[kStReachedE].v;
  st->queue_needed = (int64_t)h.need.v;
  st->pool_needed = peak * T * kChunk;
  st->batches = (int64_t)h.st[kStBatches].v;
  st->chain = chain;
  st->barriers = barriers;
}

// Executable hipGraph of `group` host-driven rounds (two kernels per lazy
// round) chained in stream order.  Kept per host thread and reused while the
// kernel, grid, device and arguments are unchanged (repeated queries on one
// graph and workspace share them: the per-query sources live in the
// workspace).  Destroyed by og_release; never at exit, when the runtime may
// be gone already.
struct RoundGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* func = nullptr;
  int nwg = 0, nodes = 0, dev = -1;
  Args args;
  bool release() {
    bool good = true;
    if (exec && hipGraphExecDestroy(exec) != hipSuccess) good = false;
    if (graph && hipGraphDestroy(graph) != hipSuccess) good = false;
    exec = nullptr;
    graph = nullptr;
    func = nullptr;
    return good;
  }
};
thread_local RoundGraph t_round_graph;

template <class W>
hipGraphExec_t round_graph(const Args& a, int nwg, int group, int dev) {
  RoundGraph& rg = t_round_graph;
  const void* f = (const void*)k_round<W>;
  const int phases = W::kPull ? 3 : (a.lazy ? 2 : 1);  // launches per round
  const int nodes = group * phases;
  if (rg.exec && rg.func == f && rg.nwg == nwg && rg.nodes == nodes && rg.dev == dev &&
      std::memcmp(&rg.args, &a, sizeof(Args)) == 0)
    return rg.exec;
  if (rg.exec) (void)hipGraphExecDestroy(rg.exec);
  if (rg.graph) (void)hipGraphDestroy(rg.graph);
  rg.exec = nullptr;
  rg.graph = nullptr;
  hipGraph_t g = nullptr;
  if (hipGraphCreate(&g, 0) != hipSuccess) return nullptr;
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < nodes; ++i) {
    Args ac = a;
    int phase = i % phases;
    void* kargs[] = {&ac, &phase};
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(f);
    p.gridDim = dim3(nwg);
    p.blockDim = dim3(kBlock);
    p.sharedMemBytes = 0;
    p.kernelParams = kargs;
    p.extra = nullptr;
    hipGraphNode_t node = nullptr;
    if (hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return nullptr;
    }
    prev = node;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return nullptr;
  }
  rg.graph = g;
  rg.exec = ex;
  rg.func = f;
  rg.nwg = nwg;
  rg.nodes = nodes;
  rg.dev = dev;
  rg.args = a;
  return ex;
}

// Exclusive prefix sum of cnt ints (in place allowed).
void scan_excl(const int* in, int* out, long long cnt, int* tiles, int grid, hipStream_t st) {
  const long long nt = (cnt + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kBlock), 0, st, in, out, cnt, tiles);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, st, tiles, (int)nt);
  hipLaunchKernelGGL(k_scan_add, dim3(grid), dim3(kBlock), 0, st, out, cnt, (const int*)tiles);
}

bool read_back(void* host, const void* dev, size_t bytes, hipStream_t st) {
  return hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st) == hipSuccess &&
         hipStreamSynchronize(st) == hipSuccess;
}

// Builds the blocked copy of g in the workspace (layout L at base): the
// clustering passes, the block numbering, each block's vertices in id
// order, and the internal / leaving edge lists.  Waits on the stream
// between passes.  *nb_out receives the block count.
og_status build_blocks(const og_graph* g, int target, char* base, const BlkLayout& L, int grid, hipStream_t st,
                       int* nb_out) {
  const int n = g->n;
  const long long* rp = (const long long*)g->row_ptr;
  const int* col = g->col;
  const int* w = g->w;
  auto at = [&](size_t off) { return (void*)(base + off); };
  unsigned long long* lab = (unsigned long long*)at(L.lab);
  unsigned long long* far = (unsigned long long*)at(L.far);
  int* fr = (int*)at(L.fr);
  int* cnt = (int*)at(L.cnt);
  int* ecnt = (int*)at(L.ecnt);
  int* over = (int*)at(L.over);
  unsigned* flags = (unsigned*)at(L.flags);
  int* tiles = (int*)at(L.tiles);
  unsigned rate = (unsigned)(target > 0 ? target : 1);
  constexpr int kLevels = 4;  // BFS levels launched between two checks
  for (int pass = 0;; ++pass) {
    if (pass >= 64) return OG_ERR_INTERNAL;
    hipLaunchKernelGGL(k_cl_prep, dim3(grid), dim3(kBlock), 0, st, n, lab, fr, (const int*)over,
                       (const unsigned long long*)far, (const int*)cnt, (const int*)ecnt, rate, target, pass,
                       0x9e3779b9u * (unsigned)(pass + 1));
    for (long long level = 0;; level += kLevels) {
      if (level > (long long)n + kLevels) return OG_ERR_INTERNAL;
      hipLaunchKernelGGL(k_fill, dim3(1), dim3(kWave), 0, st, (int*)flags, (long long)kLevels, 0);
      for (int k = 0; k < kLevels; ++k)
        hipLaunchKernelGGL(k_cl_bfs, dim3(grid), dim3(kBlock), 0, st, n, rp, col, lab, (const int*)fr,
                           (unsigned)(level + k), flags + k);
      unsigned hf[kLevels];
      if (hipGetLastError() != hipSuccess || !read_back(hf, flags, sizeof(hf), st)) return OG_ERR_HIP;
      if (hf[kLevels - 1] == 0) break;  // the frontier after the group's last level is empty
    }
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, cnt, (long long)n, 0);
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, ecnt, (long long)n, 0);
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, (int*)far, 2LL * n, 0);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kWave), 0, st, (int*)flags, 2LL, 0);
    hipLaunchKernelGGL(k_cl_count, dim3(grid), dim3(kBlock), 0, st, n, rp, col, w, (const unsigned long long*)lab,
                       cnt, ecnt, far);
    hipLaunchKernelGGL(k_cl_over, dim3(grid), dim3(kBlock), 0, st, n, (const unsigned long long*)lab,
                       (const int*)cnt, (const int*)ecnt, over, flags);
    unsigned hf[2];
    if (hipGetLastError() != hipSuccess || !read_back(hf, flags, sizeof(hf), st)) return OG_ERR_HIP;
    if (hf[0] == 0 && hf[1] == 0) break;  // no oversized cell, every vertex labelled
    rate = rate > 8 ? rate / 8 : 1;
  }
  int* flag = (int*)at(L.flag);
  int* bsize = (int*)at(L.bsize);
  int* bstart = (int*)at(L.bstart);
  int* verts = (int*)at(L.verts);
  int* blk_of = (int*)at(L.blk_of);
  int* fill = (int*)at(L.fill);
  int* pos = (int*)at(L.pos);
  int* icnt = (int*)at(L.icnt);
  int* xcnt = (int*)at(L.xcnt);
  int* irow = (int*)at(L.irow);
  int* xrow = (int*)at(L.xrow);
  // block ids: seeds in increasing id order
  hipLaunchKernelGGL(k_cl_isseed, dim3(grid), dim3(kBlock), 0, st, n, (const unsigned long long*)lab, flag);
  scan_excl(flag, flag, (long long)n + 1, tiles, grid, st);
  int nb = 0;
  if (hipGetLastError() != hipSuccess || !read_back(&nb, flag + n, sizeof(int), st)) return OG_ERR_HIP;
  if (nb < 1 || nb > n) return OG_ERR_INTERNAL;
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, bsize, (long long)nb + 1, 0);
  hipLaunchKernelGGL(k_cl_assign, dim3(grid), dim3(kBlock), 0, st, n, (const unsigned long long*)lab,
                     (const int*)flag, blk_of, bsize);
  scan_excl(bsize, bstart, (long long)nb + 1, tiles, grid, st);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, fill, (long long)nb, 0);
  hipLaunchKernelGGL(k_cl_scatter, dim3(grid), dim3(kBlock), 0, st, n, (const int*)blk_of, (const int*)bstart, fill,
                     verts);
  hipLaunchKernelGGL(k_cl_sort, dim3(nb < 65536 ? nb : 65536), dim3(kBlock), 0, st, nb, (const int*)bstart, verts);
  hipLaunchKernelGGL(k_cl_pos, dim3(grid), dim3(kBlock), 0, st, n, (const int*)verts, pos);
  hipLaunchKernelGGL(k_cl_ecount, dim3(grid), dim3(kBlock), 0, st, n, rp, col, w, (const int*)verts,
                     (const int*)blk_of, icnt, xcnt);
  scan_excl(icnt, irow, (long long)n + 1, tiles, grid, st);
  scan_excl(xcnt, xrow, (long long)n + 1, tiles, grid, st);
  hipLaunchKernelGGL(k_cl_efill, dim3(grid), dim3(kBlock), 0, st, n, rp, col, w, (const int*)verts,
                     (const int*)blk_of, (const int*)pos, (const int*)bstart, (const int*)irow, (const int*)xrow,
                     (unsigned*)at(L.iedge), (int*)at(L.xcol), (int*)at(L.xw), (int*)at(L.xblk));
  hipLaunchKernelGGL(k_cl_meta, dim3(grid), dim3(kBlock), 0, st, nb, (const int*)bstart, (const int*)irow,
                     (int4*)at(L.bmeta));
  int ends[2] = {0, 0};
  if (hipGetLastError() != hipSuccess || !read_back(&ends[0], irow + n, sizeof(int), st) ||
      !read_back(&ends[1], xrow + n, sizeof(int), st))
    return OG_ERR_HIP;
  if ((long long)ends[0] + ends[1] != g->m) return OG_ERR_INTERNAL;
  *nb_out = nb;
  return OG_OK;
}

// Common driver.  vsrcs: nsrc virtual source ids; vtgts: reps virtual
// target ids or empty.  The caller has validated every argument.
template <class W>
og_status run(const og_graph* g, const Shape& sh, const std::vector<int>& vsrcs, const std::vector<int>& vtgts,
              const int32_t* h, const og_schedule* sched, int32_t* dist, int32_t* pred, int32_t* pred_edge, void* ws,
              size_t ws_size, og_stats* stats, void* stream_v, bool force_delta1) {
  auto fail = [&](og_status st) {
    if (stats) stats->status = st;
    return st;
  };
  og_schedule r = resolved(sched);
  if (force_delta1) r.delta = 1;
  if (ws_size < ws_bytes_for(g, &r, sh)) return fail(OG_ERR_WORKSPACE);
  // the block engine shares the int32 engine's initialisation and
  // predecessor kernels
  using PW = typename std::conditional<W::kBlocks, IntW, W>::type;

  hipStream_t stream = (hipStream_t)stream_v;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(OG_ERR_HIP);
  DeviceInfo di;
  if (!device_info(dev, &di)) return fail(OG_ERR_HIP);
  const bool persistent = r.engine == OG_ENGINE_PERSISTENT;
  if (persistent && !di.coop) return fail(OG_ERR_HIP);
  const int occ = std::is_same<W, FloatW>::value      ? di.occ_float
                  : std::is_same<W, CoreW>::value     ? di.occ_core
                  : std::is_same<W, SplitW>::value    ? di.occ_split
                  : std::is_same<W, PullW>::value     ? di.occ_pull
                  : std::is_same<W, CorePullW>::value ? di.occ_core_pull
                  : std::is_same<W, BinW>::value      ? di.occ_bin
                  : std::is_same<W, BinFloatW>::value ? di.occ_bin_float
                  : std::is_same<W, BlockW>::value    ? di.occ_blocks
                                                      : di.occ_int;
  int maxwg = di.cus * (occ > 0 ? occ : 1);
  int nwg = r.workgroups > 0 ? r.workgroups : maxwg;
  if (persistent && nwg > maxwg) nwg = maxwg;
  if (nwg > kMaxWg) nwg = kMaxWg;
  if (nwg < 1) nwg = 1;

  const long long cap = queue_cap(g, &r, sh);
  int *split_col = nullptr, *split_w = nullptr, *split_l = nullptr, *split_big = nullptr;
  int2* pull_slices = nullptr;
  BlkLayout bl{};
  char* base = (char*)ws;
  int* table = (int*)(base + kCtlBytes);
  Args a;
  std::memset(&a, 0, sizeof(a));  // padding too: cached round graphs compare arguments bytewise
  a.row_ptr = (const long long*)g->row_ptr;
  a.col = g->col;
  a.w = g->w;
  a.dist = dist;
  a.h = h;
  a.nbase = g->n;
  a.reps = sh.reps;
  a.n = sh.reps * g->n;
  a.srcs = table;
  a.nsrc = sh.nsrc;
  a.tgts = sh.targets ? table + sh.nsrc : nullptr;
  a.delta = (unsigned)r.delta;
  a.shift = -1;
  if ((r.delta & (r.delta - 1)) == 0) {
    int s = 0;
    while ((1 << s) < r.delta) s++;
    a.shift = s;
  }
  a.K = r.window_buckets;
  a.cap = (unsigned)cap;
  a.fused = r.update == OG_EAGER_WITH_FUSION;
  a.threshold = (unsigned)r.fusion_threshold;
  a.bin_thread = r.bin_thread;
  a.bin_wave = r.bin_wave;
  a.max_rounds = (unsigned)r.max_rounds;
  a.nwg = nwg;
  a.ctl = (Ctl*)base;
  const int tmax = team_cap(&r, sh);
  const PoolLayout pl = pool_layout(&r, sh, cap, tmax, kCtlBytes + table_bytes(sh));
  a.teams = tmax < nwg ? tmax : nwg;
  a.ctab = (int*)(base + pl.ctab);
  a.fstack = (int*)(base + pl.fstack);
  a.pool = (int2*)(base + pl.pool);
  a.pool_chunks = pl.chunks;
  a.tchunks = pl.tchunks;
  {
    size_t off = pl.end;
    a.lazy = r.update == OG_LAZY_UPDATE;
    a.aux = nullptr;
    a.buf = nullptr;
    a.buf_cap = 0;
    a.mark = nullptr;
    if (a.lazy) {
      a.aux = (int*)(base + off);
      off += vec_bytes(a.n);
      a.buf = (int*)(base + off);
      off += vec_bytes(a.n);
      a.buf_cap = (unsigned)a.n;
    }
    if (sh.core) {
      a.mark = (int*)(base + off);
      off += vec_bytes(a.n);
    }
    a.m = g->m;
    if constexpr (W::kSplit) {
      split_col = (int*)(base + off);
      off += vec_bytes(g->m);
      split_w = (int*)(base + off);
      off += vec_bytes(g->m);
      split_l = (int*)(base + off);
      off += vec_bytes(g->n);
      split_big = (int*)(base + off);
      off += vec_bytes(g->n);
      a.hmark = (unsigned*)(base + off);
      off += vec_bytes(a.n);
      a.heavy = (int2*)(base + off);
      a.hcap = (unsigned)heavy_cap(a.n, g->m, a.reps);
      a.ecol = split_col;
      a.ew = split_w;
      a.lsplit = split_l;
    }
    if constexpr (W::kPull) {
      a.pull = pull_mode(&r);
      if constexpr (W::kCore) {
        a.fbits = (unsigned*)(base + off);
        off += vec_bytes(((long long)a.n + 31) / 32);
      } else {
        a.front = (int2*)(base + off);
        off += vec_bytes(2 * (long long)a.n);
      }
      pull_slices = (int2*)(base + off);
      a.slices = pull_slices;
      off += vec_bytes(2 * (long long)slice_cap(g->m));
    }
    if constexpr (W::kBlocks) {
      bl = blk_layout(g->n, g->m, off);
      a.bstart = (const int*)(base + bl.bstart);
      a.bmeta = (const int4*)(base + bl.bmeta);
      a.verts = (const int*)(base + bl.verts);
      a.blk_of = (const int*)(base + bl.blk_of);
      a.irow = (const int*)(base + bl.irow);
      a.xrow = (const int*)(base + bl.xrow);
      a.iedge = (const unsigned*)(base + bl.iedge);
      a.xcol = (const int*)(base + bl.xcol);
      a.xw = (const int*)(base + bl.xw);
      a.xblk = (const int*)(base + bl.xblk);
      a.brel = (int*)(base + bl.brel);
      a.bstate = (unsigned*)(base + bl.bstate);
      a.ring = (unsigned long long*)(base + bl.ring);
      a.ring_mask = (unsigned)(bl.ring_cap - 1);
    }
  }

  // Before anything is launched: this call's layout may cover a split copy
  // held in the workspace, unless it is the same copy, kept on request.
  SplitKey split_key{};
  bool keep_split = false;
  long long kept_nb = 0;
  if constexpr (W::kSplit) {
    split_key = SplitKey{ws, g->row_ptr, g->col, g->w, (long long)g->n, g->m, a.delta, split_col, 0};
    keep_split = (r.flags & OG_FLAG_KEEP_SPLIT) && split_kept(split_key);
  }
  if constexpr (W::kBlocks) {
    split_key = SplitKey{ws, g->row_ptr, g->col, g->w, (long long)g->n, g->m, (unsigned)r.block_size,
                         base + bl.bstart, 1};
    keep_split = (r.flags & OG_FLAG_KEEP_BLOCKS) && split_kept(split_key, &kept_nb);
  }
  if (!keep_split) forget_split(ws);

  const bool timing = (r.flags & OG_FLAG_TIMING) && !(r.flags & OG_FLAG_ASYNC) && t_timers.init();
  float prep_ms = 0.f;
  if (timing) (void)hipEventRecord(t_timers.ev[0], stream);
  // query table: sources then targets, carried in kernel arguments
  {
    std::vector<int> all(vsrcs);
    all.insert(all.end(), vtgts.begin(), vtgts.end());
    for (size_t off = 0; off < all.size(); off += kTableChunk) {
      TableChunk tc;
      tc.offset = (int)off;
      tc.count = (int)std::min<size_t>(kTableChunk, all.size() - off);
      std::memcpy(tc.vals, all.data() + off, sizeof(int) * (size_t)tc.count);
      hipLaunchKernelGGL(k_put_table, dim3(1), dim3(kBlock), 0, stream, table, tc);
    }
  }
  const int fill_grid = di.cus * 8;
  const int src_grid = (sh.nsrc + kBlock - 1) / kBlock;
  const unsigned pre = a.teams == 1 ? pl.pre : 0u;  // more teams: sources take chunks as they are filed
  const int pool_grid = (int)std::min<long long>(
      fill_grid,
      ((long long)std::max<size_t>((size_t)a.teams * (a.K + 4) * pl.tchunks, pl.chunks) + kBlock - 1) / kBlock);
  if constexpr (W::kCore) {
    hipLaunchKernelGGL(k_zero_ctl, dim3(16), dim3(kBlock), 0, stream, a.ctl);
    hipLaunchKernelGGL(k_far_min_init, dim3(1), dim3(kWave), 0, stream, a.ctl);
    hipLaunchKernelGGL(k_pool_init, dim3(pool_grid), dim3(kBlock), 0, stream, a, pre);
    hipLaunchKernelGGL(k_init_core, dim3(fill_grid), dim3(kBlock), 0, stream, a);
  } else {
    hipLaunchKernelGGL(k_init, dim3(fill_grid), dim3(kBlock), 0, stream, a, (int)W::kInfBits);
    hipLaunchKernelGGL(k_far_min_init, dim3(1), dim3(kWave), 0, stream, a.ctl);
    hipLaunchKernelGGL(k_pool_init, dim3(pool_grid), dim3(kBlock), 0, stream, a, pre);
    hipLaunchKernelGGL(k_init_sources<PW>, dim3(src_grid), dim3(kBlock), 0, stream, a);
  }
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(kWave), 0, stream, a);
  if constexpr (W::kPull) {
    if constexpr (W::kCore)
      hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kBlock), 0, stream, (int*)a.fbits, ((long long)a.n + 31) / 32, 0);
    else
      hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kBlock), 0, stream, (int*)a.front, 2 * (long long)a.n, 0);
    hipLaunchKernelGGL(k_init_pull, dim3(1), dim3(kWave), 0, stream, a);
  }
  if (hipGetLastError() != hipSuccess) return fail(OG_ERR_HIP);
  if (r.flags & OG_FLAG_VALIDATE) {
    // checked before anything reads the graph's structure; a bad graph
    // returns here with nothing else launched
    hipLaunchKernelGGL(k_validate, dim3(fill_grid), dim3(kBlock), 0, stream, (const long long*)g->row_ptr, g->n,
                       g->col, W::kCore ? nullptr : g->w, (long long)g->m, a.ctl);
    unsigned hs[32];  // the status line
    if (hipMemcpyAsync(hs, &a.ctl->status, sizeof(hs), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return fail(OG_ERR_HIP);
    if (hs[0] != 0) return fail((og_status)(int)hs[0]);
    if constexpr (W::kPull) {
      // the rows are well formed: check that the graph is symmetric
      hipLaunchKernelGGL(k_validate_sym, dim3(fill_grid), dim3(kBlock), 0, stream, (const long long*)g->row_ptr,
                         g->n, g->col, W::kCore ? nullptr : g->w, a.ctl);
      hipLaunchKernelGGL(k_validate_sym_verdict, dim3(1), dim3(kWave), 0, stream, a.ctl);
      if (hipMemcpyAsync(hs, &a.ctl->status, sizeof(hs), hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess)
        return fail(OG_ERR_HIP);
      if (hs[0] != 0) return fail((og_status)(int)hs[0]);
    }
  }
  if constexpr (W::kPull)  // reads the rows: after their validation
    hipLaunchKernelGGL(k_pull_slices, dim3(fill_grid), dim3(kBlock), 0, stream, a, pull_slices);
  if constexpr (W::kSplit) {
    if (keep_split) {
      // the copy is in place: only the per-call heavy-list stamps are cleared
      hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kBlock), 0, stream, (int*)a.hmark, (long long)a.n, 0);
    } else {
      hipLaunchKernelGGL(k_split_small, dim3(fill_grid), dim3(kBlock), 0, stream, a, split_col, split_w, split_l,
                         split_big);
      hipLaunchKernelGGL(k_split_big, dim3(fill_grid), dim3(kBlock), 0, stream, a, split_col, split_w, split_l,
                         split_big);
      record_split(split_key);
    }
  }
  if constexpr (W::kBlocks) {
    // the blocked copy (built here unless kept), then the per-query block
    // state: no vertex relaxed yet, every block clean, an empty ring
    if (!keep_split) {
      if (timing) (void)hipEventRecord(t_timers.ev[4], stream);
      int nbb = 0;
      const og_status bs = build_blocks(g, r.block_size, base, bl, fill_grid, stream, &nbb);
      if (bs != OG_OK) return fail(bs);
      if (timing) {
        (void)hipEventRecord(t_timers.ev[5], stream);
        if (hipEventSynchronize(t_timers.ev[5]) != hipSuccess ||
            hipEventElapsedTime(&prep_ms, t_timers.ev[4], t_timers.ev[5]) != hipSuccess)
          prep_ms = 0.f;
      }
      kept_nb = nbb;
      split_key.nb = nbb;
      record_split(split_key);
    }
    a.nb = (int)kept_nb;
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kBlock), 0, stream, a.brel, (long long)g->n, kInf);
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kBlock), 0, stream, (int*)a.bstate, kept_nb, 0);
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kBlock), 0, stream, (int*)a.ring, 2 * (long long)bl.ring_cap, 0);
  }
  if (timing) (void)hipEventRecord(t_timers.ev[1], stream);

  if (persistent) {
    void* kargs[] = {&a};
    const void* kern;
    if constexpr (W::kBlocks) kern = (const void*)k_blocks<W>;
    else kern = (const void*)k_persistent<W>;
    if (hipLaunchCooperativeKernel(kern, dim3(nwg), dim3(kBlock), kargs, 0, stream) != hipSuccess)
      return fail(OG_ERR_HIP);
  } else if constexpr (!W::kBlocks) {
    // Launch rounds in groups and poll the done flag between groups; a
    // launch after completion returns at once.  OG_ENGINE_GRAPH_ROUNDS
    // replays one executable hipGraph holding the group's launches.
    const int group = 32;
    const int phases = W::kPull ? 3 : (a.lazy ? 2 : 1);  // launches per round
    int done = 0;
    long long launched = 0;
    const long long cap_launches = r.max_rounds > 0 ? (long long)r.max_rounds + group : (1LL << 40);
    hipGraphExec_t exec = nullptr;
    if (r.engine == OG_ENGINE_GRAPH_ROUNDS) {
      exec = round_graph<W>(a, nwg, group, dev);
      if (!exec) return fail(OG_ERR_HIP);
    }
    while (!done && launched < cap_launches) {
      if (exec) {
        if (hipGraphLaunch(exec, stream) != hipSuccess) return fail(OG_ERR_HIP);
      } else {
        for (int i = 0; i < group; ++i)
          for (int ph = 0; ph < phases; ++ph) hipLaunchKernelGGL(k_round<W>, dim3(nwg), dim3(kBlock), 0, stream, a, ph);
      }
      launched += group;
      Word hd[2];  // the status line and the live-teams line
      static_assert(offsetof(Ctl, live) == offsetof(Ctl, status) + sizeof(Word), "status and live adjacent");
      if (hipMemcpyAsync(hd, &a.ctl->status, sizeof(hd), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return fail(OG_ERR_HIP);
      if (hipStreamSynchronize(stream) != hipSuccess) return fail(OG_ERR_HIP);
      done = hd[1].v == 0 || hd[0].v;
    }
  }
  if (timing) (void)hipEventRecord(t_timers.ev[2], stream);
  if constexpr (W::kCore) {
    if (stats)
      hipLaunchKernelGGL((k_pred_edges<IntW, false>), dim3(fill_grid), dim3(kBlock), 0, stream, a, (int*)nullptr,
                         (int2*)nullptr, 0ull, (const unsigned long long*)nullptr);
  } else if (pred) {
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kBlock), 0, stream, pred, (long long)a.n, kInf);
    // the long rows' slice list and the parity summary go where the queues
    // were (unused once the engine is done), when they are large enough;
    // otherwise every row stays in its chunk and every edge reads dist
    const unsigned long long lcap = pred_slice_cap(g->m, a.reps);
    int2* longs = nullptr;
    unsigned long long* sum = nullptr;
    const unsigned long long sw = ((unsigned long long)a.n + 63) / 64;  // summary words
    if ((size_t)a.pool_chunks * kChunk >= lcap + sw) {
      longs = a.pool;
      hipLaunchKernelGGL(k_fill, dim3(1), dim3(kWave), 0, stream, (int*)&a.ctl->pred_slices.v, 2ll, 0);
      // The parity filter pays where a vertex's neighbours are scattered and
      // their dist reads miss the cache, which mean degree >= kPredParDeg
      // stands for (power-law graphs; a road grid's neighbours are local and
      // the extra read only adds latency there).
      if (g->m >= (long long)kPredParDeg * a.nbase) {
        sum = reinterpret_cast<unsigned long long*>(a.pool + lcap);
        hipLaunchKernelGGL(k_pred_summary, dim3(fill_grid), dim3(kBlock), 0, stream, a, sum);
      }
    }
    if (sum) {
      hipLaunchKernelGGL((k_pred_edges<PW, true>), dim3(fill_grid), dim3(kBlock), 0, stream, a, pred, longs, lcap,
                         (const unsigned long long*)sum);
      hipLaunchKernelGGL((k_pred_long<PW, true>), dim3(fill_grid), dim3(kBlock), 0, stream, a, pred, longs, lcap,
                         (const unsigned long long*)sum);
    } else {
      hipLaunchKernelGGL((k_pred_edges<PW, false>), dim3(fill_grid), dim3(kBlock), 0, stream, a, pred, longs, lcap,
                         (const unsigned long long*)nullptr);
      if (longs)
        hipLaunchKernelGGL((k_pred_long<PW, false>), dim3(fill_grid), dim3(kBlock), 0, stream, a, pred, longs, lcap,
                           (const unsigned long long*)nullptr);
    }
    hipLaunchKernelGGL(k_pred_fix, dim3(fill_grid), dim3(kBlock), 0, stream, pred, (long long)a.n);
    hipLaunchKernelGGL(k_pred_sources, dim3(src_grid), dim3(kBlock), 0, stream, a, pred);
    if (pred_edge) hipLaunchKernelGGL(k_pred_edge_ids, dim3(fill_grid), dim3(kBlock), 0, stream, a, pred, pred_edge);
  } else if (stats) {
    hipLaunchKernelGGL((k_pred_edges<PW, false>), dim3(fill_grid), dim3(kBlock), 0, stream, a, (int*)nullptr,
                       (int2*)nullptr, 0ull, (const unsigned long long*)nullptr);
  }
  if (timing) (void)hipEventRecord(t_timers.ev[3], stream);
  if (hipGetLastError() != hipSuccess) return fail(OG_ERR_HIP);
  if (r.flags & OG_FLAG_ASYNC) {
    if (stats) stats->workgroups = nwg;
    return OG_OK;
  }
  static thread_local Ctl hc;
  if (hipMemcpyAsync(&hc, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return fail(OG_ERR_HIP);
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(OG_ERR_HIP);
  fill_stats(hc, stats, nwg);
  if (stats && W::kBlocks) {
    stats->blocks = kept_nb;
    stats->prep_ms = prep_ms;
  }
  if (timing && stats) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t_timers.ev[0], t_timers.ev[1]) == hipSuccess) stats->init_ms = ms;
    if (hipEventElapsedTime(&ms, t_timers.ev[1], t_timers.ev[2]) == hipSuccess) stats->engine_ms = ms;
    if (hipEventElapsedTime(&ms, t_timers.ev[2], t_timers.ev[3]) == hipSuccess) stats->pred_ms = ms;
  }
  return (og_status)hc.status.v;
}

// The engine instantiation for a schedule and the call's weight type.
template <class W>
og_status dispatch(const og_graph* g, const Shape& sh, const std::vector<int>& vs, const std::vector<int>& vt,
                   const int32_t* h, const og_schedule* s, int32_t* dist, int32_t* pred, int32_t* pred_edge,
                   void* ws, size_t ws_bytes, og_stats* stats, void* stream, bool force_delta1) {
  auto fail = [&](og_status st) {
    if (stats) stats->status = st;
    return st;
  };
  if (s->flags & OG_FLAG_VERTEX_BLOCKS) {
    // one query at a time, no A* estimate (the blocks drain buckets of plain
    // distances)
    if constexpr (std::is_same<W, IntW>::value) {
      if (sh.reps == 1 && !h)
        return run<BlockW>(g, sh, vs, vt, h, s, dist, pred, pred_edge, ws, ws_bytes, stats, stream, force_delta1);
    }
    return fail(OG_ERR_INVALID_ARG);
  }
  if (s->flags & OG_FLAG_LIGHT_HEAVY) {
    if constexpr (std::is_same<W, IntW>::value)
      return run<SplitW>(g, sh, vs, vt, h, s, dist, pred, pred_edge, ws, ws_bytes, stats, stream, force_delta1);
    return fail(OG_ERR_INVALID_ARG);  // int32 weights only
  }
  if (s->flags & (OG_FLAG_DENSE_PULL | OG_FLAG_HYBRID_DIRECTION)) {
    if constexpr (std::is_same<W, IntW>::value)
      return run<PullW>(g, sh, vs, vt, h, s, dist, pred, pred_edge, ws, ws_bytes, stats, stream, force_delta1);
    return fail(OG_ERR_INVALID_ARG);  // int32 weights only
  }
  if (s->flags & OG_FLAG_DEGREE_BINS) {
    if constexpr (std::is_same<W, IntW>::value)
      return run<BinW>(g, sh, vs, vt, h, s, dist, pred, pred_edge, ws, ws_bytes, stats, stream, force_delta1);
    else
      return run<BinFloatW>(g, sh, vs, vt, h, s, dist, pred, pred_edge, ws, ws_bytes, stats, stream, force_delta1);
  }
  return run<W>(g, sh, vs, vt, h, s, dist, pred, pred_edge, ws, ws_bytes, stats, stream, force_delta1);
}

// Queries one launch can hold on a graph of n vertices: virtual vertex ids
// q * n + v are int32, and the target table of a launch has kMaxQueries
// entries.
int wave_queries(long long n) {
  const long long q = (0x7fffffffLL - 1) / n;
  return (int)(q < kMaxQueries ? q : kMaxQueries);
}

// Adds one wave's counters to a batch's (times and counts summed, the
// largest queue fill, the first error).
void add_stats(og_stats* to, const og_stats& w) {
  if (to->status == OG_OK) to->status = w.status;
  to->workgroups = w.workgroups;
  to->rounds += w.rounds;
  to->buckets += w.buckets;
  to->relaxations += w.relaxations;
  to->improvements += w.improvements;
  to->pushes_local += w.pushes_local;
  to->pushes_global += w.pushes_global;
  to->far_pushes += w.far_pushes;
  to->reached_vertices += w.reached_vertices;
  to->reached_edges += w.reached_edges;
  to->queue_needed = w.queue_needed > to->queue_needed ? w.queue_needed : to->queue_needed;
  to->pool_needed = w.pool_needed > to->pool_needed ? w.pool_needed : to->pool_needed;
  to->init_ms += w.init_ms;
  to->engine_ms += w.engine_ms;
  to->pred_ms += w.pred_ms;
  to->batches += w.batches;
  to->chain += w.chain;
  to->barriers += w.barriers;
  to->blocks = w.blocks;
  to->prep_ms += w.prep_ms;
}

// Argument checks shared by every entry point (nothing is launched on
// failure).  srcs / dsts are host arrays of base vertex ids.  A batch of
// more queries than one launch holds (wave_queries) runs as consecutive
// launches ("waves") of up to that many queries on the same workspace, each
// on its own slice of dist, pred and h; the counters are summed.
template <class W = IntW>
og_status checked_run(const og_graph* g, const int32_t* srcs, int32_t nsrc, const int32_t* dsts, int32_t reps,
                      bool multi, const int32_t* h, bool need_h, const og_schedule* s, int32_t* dist, int32_t* pred,
                      void* ws, size_t ws_bytes, og_stats* stats, void* stream, bool force_delta1,
                      int32_t* pred_edge = nullptr) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  auto fail = [&](og_status st) {
    if (stats) stats->status = st;
    return st;
  };
  if (!graph_ok(g) || !schedule_ok(s) || !dist || !ws || !srcs) return fail(OG_ERR_INVALID_ARG);
  if (((uintptr_t)ws & 255) != 0) return fail(OG_ERR_INVALID_ARG);
  if (need_h && !h) return fail(OG_ERR_INVALID_ARG);
  if (pred_edge && !pred) return fail(OG_ERR_INVALID_ARG);
  if (reps < 1 || reps > kMaxBatch || nsrc < 1) return fail(OG_ERR_INVALID_ARG);
  for (int i = 0; i < nsrc; ++i)
    if (srcs[i] < 0 || srcs[i] >= g->n) return fail(OG_ERR_INVALID_ARG);
  if (dsts)
    for (int q = 0; q < reps; ++q)
      if (dsts[q] < 0 || dsts[q] >= g->n) return fail(OG_ERR_INVALID_ARG);
  const int per = multi ? 1 : wave_queries(g->n);
  if (multi || reps <= per) {
    const Shape sh{reps, nsrc, dsts != nullptr};
    if (!shape_ok(g, sh)) return fail(OG_ERR_INVALID_ARG);
    std::vector<int> vs((size_t)nsrc), vt;
    for (int i = 0; i < nsrc; ++i) vs[i] = multi ? srcs[i] : i * g->n + srcs[i];
    if (dsts) {
      vt.resize((size_t)reps);
      for (int q = 0; q < reps; ++q) vt[q] = q * g->n + dsts[q];
    }
    return dispatch<W>(g, sh, vs, vt, h, s, dist, pred, pred_edge, ws, ws_bytes, stats, stream, force_delta1);
  }
  if (per < 1 || (s->flags & (OG_FLAG_VERTEX_BLOCKS | OG_FLAG_ASYNC))) return fail(OG_ERR_INVALID_ARG);
  og_stats total;
  std::memset(&total, 0, sizeof(total));
  og_status st = OG_OK;
  for (int q0 = 0; q0 < reps && st == OG_OK; q0 += per) {
    const int nq = reps - q0 < per ? reps - q0 : per;
    const Shape sh{nq, nq, dsts != nullptr};
    std::vector<int> vs((size_t)nq), vt;
    for (int i = 0; i < nq; ++i) vs[i] = i * g->n + srcs[q0 + i];
    if (dsts) {
      vt.resize((size_t)nq);
      for (int q = 0; q < nq; ++q) vt[q] = q * g->n + dsts[q0 + q];
    }
    const size_t off = (size_t)q0 * (size_t)g->n;
    og_stats ws_st;
    std::memset(&ws_st, 0, sizeof(ws_st));
    st = dispatch<W>(g, sh, vs, vt, h ? h + off : nullptr, s, dist + off, pred ? pred + off : nullptr, nullptr, ws,
                     ws_bytes, &ws_st, stream, force_delta1);
    add_stats(&total, ws_st);
    if (total.status == OG_OK) total.status = st;
  }
  if (stats) *stats = total;
  return st;
}

}  // namespace og

extern "C" {

int32_t og_version(void) { return (1 << 16) | 1; }

const char* og_status_string(og_status s) {
  switch (s) {
    case OG_OK: return "ok";
    case OG_ERR_INVALID_ARG: return "invalid argument";
    case OG_ERR_NEGATIVE_WEIGHT: return "negative edge weight";
    case OG_ERR_OVERFLOW: return "path length overflows int32";
    case OG_ERR_WORKSPACE: return "workspace too small or a queue overflowed";
    case OG_ERR_HIP: return "HIP runtime error";
    case OG_ERR_ROUND_LIMIT: return "round limit reached";
    case OG_ERR_INTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

og_status og_default_schedule(og_schedule* s) {
  if (!s) return OG_ERR_INVALID_ARG;
  std::memset(s, 0, sizeof(*s));
  s->delta = 1;
  s->update = OG_EAGER_WITH_FUSION;
  s->fusion_threshold = og::kDefaultThreshold;
  s->window_buckets = og::kDefaultK;
  s->engine = OG_ENGINE_PERSISTENT;
  s->bin_thread = og::kBinLane;
  s->bin_wave = og::kDefaultBinWave;
  s->block_size = og::kDefaultBlockSize;
  return OG_OK;
}

static size_t ws_bytes_shape(const og_graph* g, const og_schedule* s, const og::Shape& sh) {
  if (!og::graph_ok(g) || !og::schedule_ok(s) || !og::shape_ok(g, sh)) return 0;
  og_schedule r = og::resolved(s);
  return og::ws_bytes_for(g, &r, sh);
}

size_t og_workspace_bytes(const og_graph* g, const og_schedule* s) {
  return ws_bytes_shape(g, s, og::Shape{1, 1, true});
}

size_t og_workspace_bytes_batch(const og_graph* g, const og_schedule* s, int32_t nq) {
  if (!og::graph_ok(g) || nq < 1 || nq > og::kMaxBatch) return 0;
  const int per = og::wave_queries(g->n);
  const int q = nq < per ? nq : per;  // a larger batch runs in waves of `per` queries
  return ws_bytes_shape(g, s, og::Shape{q, q, true});
}

size_t og_workspace_bytes_multi(const og_graph* g, const og_schedule* s, int32_t nsrc) {
  return ws_bytes_shape(g, s, og::Shape{1, nsrc, false});
}

og_status og_sssp(const og_graph* g, int32_t src, const og_schedule* s, int32_t* dist, int32_t* pred,
                  void* ws, size_t ws_bytes, og_stats* stats, void* stream) {
  return og::checked_run(g, &src, 1, nullptr, 1, false, nullptr, false, s, dist, pred, ws, ws_bytes, stats, stream,
                         false);
}

og_status og_wbfs(const og_graph* g, int32_t src, const og_schedule* s, int32_t* dist, int32_t* pred,
                  void* ws, size_t ws_bytes, og_stats* stats, void* stream) {
  return og::checked_run(g, &src, 1, nullptr, 1, false, nullptr, false, s, dist, pred, ws, ws_bytes, stats, stream,
                         true);
}

og_status og_ppsp(const og_graph* g, int32_t src, int32_t dst, const og_schedule* s, int32_t* dist,
                  int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats, void* stream) {
  return og::checked_run(g, &src, 1, &dst, 1, false, nullptr, false, s, dist, pred, ws, ws_bytes, stats, stream,
                         false);
}

og_status og_astar(const og_graph* g, int32_t src, int32_t dst, const int32_t* h, const og_schedule* s,
                   int32_t* dist, int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats, void* stream) {
  return og::checked_run(g, &src, 1, &dst, 1, false, h, true, s, dist, pred, ws, ws_bytes, stats, stream, false);
}

og_status og_sssp_batch(const og_graph* g, const int32_t* srcs, int32_t nq, const og_schedule* s, int32_t* dist,
                        int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats, void* stream) {
  return og::checked_run(g, srcs, nq, nullptr, nq, false, nullptr, false, s, dist, pred, ws, ws_bytes, stats,
                         stream, false);
}

og_status og_ppsp_batch(const og_graph* g, const int32_t* srcs, const int32_t* dsts, int32_t nq,
                        const og_schedule* s, int32_t* dist, int32_t* pred, void* ws, size_t ws_bytes,
                        og_stats* stats, void* stream) {
  if (!dsts) {
    if (stats) std::memset(stats, 0, sizeof(*stats)), stats->status = OG_ERR_INVALID_ARG;
    return OG_ERR_INVALID_ARG;
  }
  return og::checked_run(g, srcs, nq, dsts, nq, false, nullptr, false, s, dist, pred, ws, ws_bytes, stats, stream,
                         false);
}

og_status og_astar_batch(const og_graph* g, const int32_t* srcs, const int32_t* dsts, int32_t nq, const int32_t* h,
                         const og_schedule* s, int32_t* dist, int32_t* pred, void* ws, size_t ws_bytes,
                         og_stats* stats, void* stream) {
  if (!dsts) {
    if (stats) std::memset(stats, 0, sizeof(*stats)), stats->status = OG_ERR_INVALID_ARG;
    return OG_ERR_INVALID_ARG;
  }
  return og::checked_run(g, srcs, nq, dsts, nq, false, h, true, s, dist, pred, ws, ws_bytes, stats, stream, false);
}

og_status og_sssp_multi(const og_graph* g, const int32_t* srcs, int32_t nsrc, const og_schedule* s, int32_t* dist,
                        int32_t* pred, void* ws, size_t ws_bytes, og_stats* stats, void* stream) {
  return og::checked_run(g, srcs, nsrc, nullptr, 1, true, nullptr, false, s, dist, pred, ws, ws_bytes, stats, stream,
                         false);
}

static_assert(sizeof(og_graph) == sizeof(og_graph_f32), "graph views share one layout");

size_t og_workspace_bytes_f32(const og_graph_f32* g, const og_schedule* s) {
  return ws_bytes_shape(reinterpret_cast<const og_graph*>(g), s, og::Shape{1, 1, false});
}

og_status og_sssp_f32(const og_graph_f32* g, int32_t src, const og_schedule* s, float* dist, int32_t* pred,
                      int32_t* pred_edge, void* ws, size_t ws_bytes, og_stats* stats, void* stream) {
  return og::checked_run<og::FloatW>(reinterpret_cast<const og_graph*>(g), &src, 1, nullptr, 1, false, nullptr, false,
                                     s, reinterpret_cast<int32_t*>(dist), pred, ws, ws_bytes, stats, stream, false,
                                     pred_edge);
}

size_t og_backward_workspace_bytes(int32_t n) {
  if (n < 1) return 0;
  const size_t b = sizeof(double) * (size_t)n + 2 * sizeof(int) * (size_t)n;
  return (b + 255) & ~(size_t)255;
}

og_status og_sssp_backward_f32(const og_graph_f32* g, const int32_t* pred, const int32_t* pred_edge,
                               const float* grad_dist, float* grad_w, void* ws, size_t ws_bytes, void* stream) {
  if (!og::graph_ok(reinterpret_cast<const og_graph*>(g)) || !pred || !pred_edge || !grad_dist || !grad_w || !ws)
    return OG_ERR_INVALID_ARG;
  if (((uintptr_t)ws & 255) != 0) return OG_ERR_INVALID_ARG;
  if (ws_bytes < og_backward_workspace_bytes(g->n)) return OG_ERR_WORKSPACE;
  int dev = 0;
  og::DeviceInfo di;
  if (hipGetDevice(&dev) != hipSuccess || !og::device_info(dev, &di)) return OG_ERR_HIP;
  hipStream_t st = (hipStream_t)stream;
  og::forget_split(ws);  // the workspace may have held a split copy
  double* acc = (double*)ws;
  int* kids = (int*)((char*)ws + sizeof(double) * (size_t)g->n);
  int* pending = kids + g->n;
  const int grid = di.cus * 8;
  hipLaunchKernelGGL(og::k_bw_init, dim3(grid), dim3(og::kBlock), 0, st, grad_dist, g->n, grad_w, (long long)g->m,
                     acc, kids, pending);
  hipLaunchKernelGGL(og::k_bw_count, dim3(grid), dim3(og::kBlock), 0, st, pred, pred_edge, g->n, kids, pending);
  // A wavefront runs until its longest climb ends, so a thread that takes
  // several leaves in turn adds their climbs up: on a deep tree (a road
  // grid's, thousands of levels) every vertex gets a thread of its own.  On
  // a power-law graph (mean degree >= kPredParDeg) the tree is shallow and
  // the hubs' many children contend for the hubs' sums, which the smaller
  // grid-stride launch spreads out.
  const int climb_grid = g->m >= (long long)og::kPredParDeg * g->n
                             ? grid
                             : (int)(((long long)g->n + og::kBlock - 1) / og::kBlock);
  hipLaunchKernelGGL(og::k_bw_climb, dim3(climb_grid), dim3(og::kBlock), 0, st, pred, pred_edge, g->n, grad_w, acc,
                     kids, pending);
  if (hipGetLastError() != hipSuccess) return OG_ERR_HIP;
  return OG_OK;
}

size_t og_workspace_bytes_kcore(const og_graph* g, const og_schedule* s) {
  if (!s) return 0;
  og_schedule r = og::resolved(s);
  r.delta = 1;
  r.flags &= ~(OG_FLAG_LIGHT_HEAVY | OG_FLAG_DEGREE_BINS | OG_FLAG_VERTEX_BLOCKS | OG_FLAG_KEEP_BLOCKS);
  if (!og::graph_ok(g, false) || !og::schedule_ok(&r)) return 0;
  return og::ws_bytes_for(g, &r, og::Shape{1, g->n, false, true});
}

og_status og_kcore(const og_graph* g, const og_schedule* s, int32_t* core, void* ws, size_t ws_bytes,
                   og_stats* stats, void* stream) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  auto fail = [&](og_status st) {
    if (stats) stats->status = st;
    return st;
  };
  if (!s) return fail(OG_ERR_INVALID_ARG);
  og_schedule r = *s;
  r.delta = 1;  // one bucket per degree value: peeling needs the strict order
  r.flags &= ~(OG_FLAG_LIGHT_HEAVY | OG_FLAG_DEGREE_BINS | OG_FLAG_VERTEX_BLOCKS | OG_FLAG_KEEP_BLOCKS);
  if (!og::graph_ok(g, false) || !og::schedule_ok(&r) || !core || !ws) return fail(OG_ERR_INVALID_ARG);
  if (((uintptr_t)ws & 255) != 0) return fail(OG_ERR_INVALID_ARG);
  const og::Shape sh{1, g->n, false, true};
  if (!og::shape_ok(g, sh)) return fail(OG_ERR_INVALID_ARG);
  if (r.flags & (OG_FLAG_DENSE_PULL | OG_FLAG_HYBRID_DIRECTION))
    return og::run<og::CorePullW>(g, sh, {}, {}, nullptr, &r, core, nullptr, nullptr, ws, ws_bytes, stats, stream,
                                  false);
  return og::run<og::CoreW>(g, sh, {}, {}, nullptr, &r, core, nullptr, nullptr, ws, ws_bytes, stats, stream, false);
}

}  // extern "C"

namespace og {

// Workspace of og_sssp_noalloc: one copy per device, allocated with the code
// object when the library is loaded on that device and held until the
// process ends.  Host code never uses this name as an address: the device
// address comes from hipGetSymbolAddress, per device.
constexpr size_t kScratchBytes = OG_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64];

// The device address of the current device's copy of scratch, looked up on
// the first call on that device.
og_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return OG_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OG_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return OG_OK;
}

}  // namespace og

extern "C" {

og_status og_sssp_noalloc(const og_graph* g, int32_t src, const og_schedule* s, int32_t* dist, int32_t* pred,
                          og_stats* stats, void* stream) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  auto fail = [&](og_status st) {
    if (stats) stats->status = st;
    return st;
  };
  // timing events and the replayed round graph are HIP objects created on
  // first use: not available here
  if (!s || (s->flags & OG_FLAG_TIMING) || s->engine == OG_ENGINE_GRAPH_ROUNDS) return fail(OG_ERR_INVALID_ARG);
  const size_t need = og_workspace_bytes(g, s);
  if (need == 0) return fail(OG_ERR_INVALID_ARG);
  if (need > og::kScratchBytes) return fail(OG_ERR_WORKSPACE);
  void* ws = nullptr;
  const og_status st = og::scratch_address(&ws);
  if (st != OG_OK) return fail(st);
  return og_sssp(g, src, s, dist, pred, ws, og::kScratchBytes, stats, stream);
}

og_status og_release(void) {
  // outstanding work on the calling thread's streams may still use the
  // round graph: wait for the device first
  bool good = hipDeviceSynchronize() == hipSuccess;
  good = og::t_round_graph.release() && good;
  good = og::t_timers.release() && good;
  return good ? OG_OK : OG_ERR_HIP;
}

og_status og_read_stats(const void* ws, og_stats* stats, void* stream) {
  if (!ws || !stats) return OG_ERR_INVALID_ARG;
  static thread_local og::Ctl hc;
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(&hc, ws, sizeof(og::Ctl), hipMemcpyDeviceToHost, st) != hipSuccess) return OG_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return OG_ERR_HIP;
  const int wg = stats->workgroups;
  og::fill_stats(hc, stats, wg);
  return (og_status)hc.status.v;
}

}  // extern "C"
