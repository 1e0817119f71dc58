// Internal data layout shared by the graph preparation, the solver engine and
// the C ABI. Device structures are plain structs of pointers and scalars that
// live in device memory; the host fills them once and launches with pointers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sssp {

constexpr uint32_t kInf = 0xFFFFFFFFu;   // +infinity: the single sentinel for dist and thresholds
constexpr int kWave = 64;                // CDNA wavefront
constexpr int kBlock = 256;              // threads per workgroup (4 waves)
constexpr int kRatioNum = 4096;          // RATIO_NUM, Section 4.1
constexpr uint32_t kRingMax = 65536;     // the longest exact selection-threshold window (max weight)
constexpr int kLdsRing = 1024;           // settle: distance bins privatised in LDS
constexpr int kStNum = 1024;             // ST_NUM, Section 4.1: selection-threshold grid per max weight
constexpr uint32_t kGridRing = 4096;     // grid bins kept (>= 2 ST_NUM + 2)
constexpr uint32_t kNoBin = 0xFFFFFFFFu; // a distance too large for the grid
constexpr int kLdsHist = 1024;           // settle: degree ranks privatised in LDS
constexpr int kHeavyChunk = 256;         // edges per heavy chunk
constexpr int kDefaultHeavy = 64;        // ranges longer than this are split (also the least split allowed)
constexpr int kHeavyPerBatch = 16;       // heavy chunks per workgroup batch
constexpr int kDefaultFuse = 256;        // rounds a workgroup may chain on a small frontier

// Tile shapes of the engine: each is its own instantiation of the engine
// kernel (a launch picks one; none changes a distance or the schedule).
template <int kIt, int kEd, int kSe, int kOcc>
struct TileShape {
  static constexpr int kItems = kIt;                     // round batches: items per thread
  static constexpr int kBatch = kBlock * kIt;            // items per round batch
  static constexpr int kEdges = kEd;                     // edges a thread relaxes per pass
  static constexpr int kSettle = kSe;                    // settle batches: items per thread
  static constexpr int kSettleBatch = kBlock * kSe;      // items per settle batch
  static constexpr int kStage = kBatch + kBlock * kEd + 256;  // LDS staging of list appends
  static constexpr int kMinBlocks = kOcc;                // workgroups per CU budgeted for
};
using ShapeStd = TileShape<2, 2, 4, 5>;     // 512-item round batches
using ShapeWide = TileShape<4, 2, 4, 3>;    // 1024-item round batches: longer single-workgroup rounds
using ShapeNarrow = TileShape<1, 2, 4, 5>;  // 256-item round batches: more batches per frontier
using ShapeSettle8 = TileShape<2, 2, 8, 5>; // 2048-item settle batches
enum ShapeId : int { SHAPE_STD = 0, SHAPE_WIDE = 1, SHAPE_NARROW = 2, SHAPE_SETTLE8 = 3, kNumShapes = 4 };
constexpr int round_batch_of(int shape) {
  return shape == SHAPE_WIDE ? ShapeWide::kBatch : shape == SHAPE_NARROW ? ShapeNarrow::kBatch
                                                                           : ShapeStd::kBatch;
}
constexpr int settle_batch_of(int shape) {
  return shape == SHAPE_SETTLE8 ? ShapeSettle8::kSettleBatch : ShapeStd::kSettleBatch;
}

// ------------------------------------------------------------------ graph --
// An unsettled-list (pull-list) entry: the vertex, the smallest weight of its
// row and the row's bounds, so that the pull reads no per-vertex array before
// deciding and searching.
struct alignas(16) UEntry {
  int32_t id;
  uint32_t wmin;
  int32_t rs, re;
};

struct DevGraph {
  int32_t n;
  int32_t nnz;
  uint32_t max_w;        // maxW(G, 1)
  uint32_t high_d0;      // highD(0)
  int32_t num_deg;       // distinct degrees >= 1 (D)
  int32_t n_nonisolated;
  int32_t max_deg;
  uint32_t rwi_width;        // weight width of the row-index buckets: ceil((maxW + 1) / 16)
  const int32_t* rowptr;     // n + 1
  const uint64_t* adj;       // nnz entries, (weight << 32) | column, each row ascending
  const uint32_t* wmin;      // n: smallest weight of the row (kInf for degree 0)
  const uint64_t* dinfo;     // n: (index of deg(v) among the distinct degrees, -1 for 0) << 32 | deg(v)
  const int32_t* deg_vals;   // D ascending distinct degrees
  const uint32_t* deg_cnt0;  // D: vertices with that degree
  const uint32_t* hub_bits;  // ceil(n/32) words: deg(v) >= highD(0)
  // n_nonisolated entries grouped by the weight bucket of their smallest
  // weight (bucket b holds weights in [b, b + 1) * ubucket_width, the last
  // bucket everything above), ascending, and by id within a bucket: the
  // vertices able to pull at all (smallest weight < ub - st) lie in a prefix
  // of whole buckets, and each bucket keeps the rows' memory order
  const UEntry* nonisolated;
  // kUBuckets + 1 entries: ufirst[j] is the first position of `nonisolated`
  // in bucket j or later (ufirst[kUBuckets] = the count)
  const int32_t* ufirst;
  // ceil((maxW + 1) / kUBucketDiv); binary32 weights: the bit pattern of
  // maxW / kUBucketDiv (bucket 0 holds the rows whose lightest edge is lighter)
  uint32_t ubucket_width;
  // 1: weights (and so distances) are IEEE binary32 bit patterns of finite
  // non-negative values. Such bit patterns order like the values, so every
  // comparison stays an unsigned one; only sums are taken in fp32.
  uint32_t float_w;
  uint32_t min_pos_w;        // smallest positive weight (UINT32_MAX if none)
  int32_t heavy_rows;        // vertices whose degree exceeds kDefaultHeavy (sizes the heavy-chunk lists)
  const uint32_t* rtow;      // 4096
  // per row, 16 int32: entry b - 1 (b = 1..15) is the first position of the
  // row whose weight is >= b * rwi_width (entry 15 unused). Written for rows
  // longer than kRowIndexMin only.
  const int32_t* rwi;
  // Internal vertex order: every array above is indexed by internal ids. With
  // a hub-first order (relabelled > 0 vertices moved to the front) these map
  // the caller's ids to internal ones and back; null when the order is the
  // caller's.
  const int32_t* new_of_old;
  const int32_t* old_of_new;
  int32_t relabelled;
  int32_t pad_g3;
};
// hub-first order: the least degree of a front vertex, and at most this many
// front vertices (their 8-byte state words fill 4 MiB, an XCD's L2)
constexpr int kHubMinDegree = 64;
constexpr int kHubPrefixMax = 1 << 19;
constexpr int kRowIndexMin = 8;
// Two pull-list buckets: smallest weight below 1/16 of the weight range (the
// first pull of a step sequence usually needs only these), and the rest. More
// buckets would interleave several id-ordered runs in one pull and lose the
// memory order that the pull's row and distance reads rely on.
constexpr int kUBuckets = 2;
constexpr int kUBucketDiv = 16;

// ------------------------------------------------------- solver instance --
enum Phase : uint32_t { PH_ROUND = 0, PH_SETTLE = 1, PH_DONE = 2 };

enum SegKind : int32_t {
  SEG_W = 0,   // settled list range: deferred pushes of settled vertices in [lb0, st]
  SEG_P = 1,   // pending list: first-step leftovers whose tentative dist fell into the band
  SEG_U = 2,   // pull over the unsettled list
  SEG_Q = 3,   // frontier queue
  SEG_H = 4,   // heavy chunks split off the previous tick
  SEG_ST = 5,  // settle: touched list
  SEG_SP = 6,  // settle: pending list compaction
};

struct StepRec {
  uint32_t lb, ub;
  int32_t seg_begin, seg_end;  // settled-list positions of this step's vertices
};

struct HeavyItem {
  int32_t u;
  uint32_t d;       // dist[u] when split (push) / unused (pull)
  int32_t lo;
  int32_t hi_kind;  // hi | (kind << 31): kind 1 = pull chunk
};

struct TraceRec {
  uint32_t lb, ub, st, rounds;
  uint32_t pulled, L;
  uint64_t S;
  uint32_t h, gap, st_next, pad;
};

struct Counters {
  unsigned long long expansions, band_expansions, push_scanned, pull_vertices, pull_scanned,
      relax_success, queue_entries, rounds, pulls, steps, ticks, fused_rounds, pull_unsettled;
};

struct alignas(128) HotI32 {
  int32_t v;
  int32_t pad[31];
};
struct alignas(128) HotU32 {
  uint32_t v;
  uint32_t pad[31];
};
struct alignas(128) HotU64 {
  unsigned long long v;
  unsigned long long pad[15];
};

constexpr int kMaxSegPerInst = 5;  // segments one instance may have in a tick

// A solver instance: fixed pointers and parameters of the solve, the control
// words (one contiguous base, so that the epilogue can take them into
// registers with a burst of wide loads and write them back the same way), the
// work counters, and the words that device atomics update.
struct InstFixed {
  const DevGraph* g;
  // a copy of *g: the batches read the graph's arrays and sizes with the
  // instance's own words, with no dependent load of the graph record
  DevGraph gc;
  uint32_t* dist;          // the caller's output, written once the solve ends
  int32_t* parent;         // the caller's tree output (Section 2.1's predecessors), or null
  // with a tree: per vertex (distance << 32) | the vertex whose relaxation set
  // that distance. A relaxation that lowers a distance is the only one that
  // sets that value, so the 64-bit atomicMin keeps the last one's source.
  uint64_t* best;
  // per vertex: (tentative distance << 32) | round id of its last decrease
  // (0: never decreased). One 64-bit atomicMin both lowers the distance and
  // returns the round of the previous decrease, which de-duplicates the next
  // frontier (once per round) and the step's touched list (once per step).
  uint64_t* state;
  int32_t* q[2];
  int32_t* touched;
  int32_t* settled;
  int32_t* plist[2];
  UEntry* ulist[2];        // unsettled (pull) lists
  HeavyItem* heavy[2];
  uint64_t* ring_mass;
  uint32_t* ring_cnt;
  uint32_t* hist_cnt;
  StepRec* steprec;
  TraceRec* trace;
  Counters* cslot;         // per-wave work counters: [maxw]
  int32_t maxw;            // waves the counter array can hold
  int32_t pad2;
  int32_t heavy_cap;
  uint32_t ring_mask;
  uint32_t steprec_mask;
  int32_t trace_cap;
  int32_t source;
  int32_t target;          // point-to-point query: stop once this vertex is settled; -1: none
  // source and target as internal ids (set by the per-solve initialisation)
  int32_t src_in, tgt_in;
  // which round-batch instantiation runs this instance: bit 0 a tree is
  // recorded (best != null), bit 1 the graph has binary32 weights
  uint32_t mode;
  // computeST's candidates for integer weights: 0 the exact window of
  // distinct settled distances while max weight <= kStNum, the ST_NUM grid
  // above; 1 the grid always; -1 the window while max weight <= kRingMax
  int32_t st_grid;
  int32_t n;
  uint32_t alpha;
  uint32_t traversal_opt;
  double beta;
  int32_t heavy_split;
  int32_t fuse_cap;        // rounds one workgroup may chain without a grid barrier (0: off)
};

// control words: written by the epilogue and by the heuristic
struct InstCtl {
  uint32_t phase;
  uint32_t tick_kind;      // PH_ROUND or PH_SETTLE: what the scheduled tick does
  uint32_t init_round;     // current round is a step's first (W / P / U segments)
  uint32_t pull_on;        // st < lb for this step
  uint32_t lb, ub, st, lb0;
  uint32_t first;          // first step (ub follows the nearest hub)
  uint32_t gap_cur;        // gap(lb) of the current step
  uint32_t M;
  uint32_t rid;            // round id of the current round
  uint32_t step_rid0;      // round-id marker of the current step (its rounds use > step_rid0)
  uint32_t step;
  uint32_t rounds_in_step;
  int32_t qsel, psel, usel, hsel;
  int32_t nF, wBegin, wEnd, nP, nU, nT, nH;
  // The pull list of a step is the compacted list of earlier pulls (nU
  // entries) followed by the part [u_done, u_end) of the sorted non-isolated
  // list that no earlier pull has read (u_end: first entry too heavy to pull
  // in this step).
  int32_t u_done, u_end;
  int32_t settled_mark;
  int32_t nsteprec;
  int32_t trace_len;
  int32_t settle_items;    // batches of the settle tick
  uint32_t high_d0, gap0;
  uint32_t pad1;
};

// an instance's segments of the next tick (written by its transition)
struct SegSpec {
  int32_t cnt[kMaxSegPerInst], kind[kMaxSegPerInst], pb[kMaxSegPerInst];
  int32_t pad;
};

struct Inst : InstFixed, InstCtl {
  SegSpec spec;
  Counters c;
  // ---- hot words: updated by device atomics from every CU, each on its own
  // 128-byte line so that they never share a line with the fields above ----
  HotI32 q_next_cnt, touched_cnt, p_next_cnt, u_next_cnt, settled_cnt, h_next_cnt, settle_done;
  HotU32 ub_next, max_settled, flags;
  HotU64 S;  // sumD(lb): degree mass of the unsettled set
};

// flags
constexpr uint32_t FLAG_MAYBE_OVERFLOW = 1u;  // an edge was cut by the +inf clamp
constexpr uint32_t FLAG_CAPACITY = 2u;        // an internal list overflowed (bug guard)
constexpr uint32_t FLAG_MASS = 4u;            // degree-mass bookkeeping mismatch (bug guard)
constexpr uint32_t FLAG_TIMEOUT = 8u;         // a grid barrier wait gave up
constexpr uint32_t FLAG_OVERFLOW = 16u;       // confirmed: a distance does not fit below kInf
constexpr uint32_t FLAG_TICKS = 32u;          // the tick limit stopped the engine
constexpr uint32_t FLAG_TREE = 64u;           // a tree entry disagrees with its distance (bug guard)

// ------------------------------------------------------------- tick table --

constexpr int kMaxXcd = 8;  // XCDs (each with its own L2) on an MI355X
constexpr int kTickLogWords = 8;  // words per tick of the debug tick log

// One segment of a tick's table: a run of batches of one kind of work of one
// instance. A batch needs only this record to start (one 16-byte load).
struct alignas(16) SegRec {
  int32_t first;  // the segment's first batch in the tick
  int32_t inst;   // instance
  int32_t count;  // items
  int32_t word;   // kind | instance mode (bit 0 tree, bit 1 binary32) << 4 | items per batch << 8
};
__host__ __device__ constexpr int32_t seg_word(int kind, uint32_t mode, int per_batch) {
  return kind | (int32_t)((mode & 3u) << 4) | (per_batch << 8);
}

struct Globals {
  // grid barrier: arrival counter and release generation on lines of their own
  HotU32 bar_count;
  HotU32 bar_gen;
  // per-XCD arrival counters, release words and workgroup counts. A release
  // word holds the XCD's release generation (low half) and the quota word of
  // the tick that release starts (high half): one load gives a waiting
  // workgroup both.
  HotU32 xcd_count[kMaxXcd];
  HotU64 xcd_gen[kMaxXcd];
  HotU32 xcd_members[kMaxXcd];
  unsigned int all_done;
  unsigned int error;
  // the next tick's quota word (workgroups per XCD that take part in it, the
  // rest wait aside; small- and stop-tick bits), set by the epilogue for the
  // XCD leaders to publish
  unsigned int quota_next;
  // current tick layout
  int32_t nseg;
  int32_t total_batches;
  int32_t ninst;
  int32_t max_ticks_hit;
  // items per round batch and per settle batch of the launch's tile shape
  int32_t round_batch, settle_batch;
  unsigned long long ticks;
  unsigned long long tick_limit;  // safety stop for a schedule that fails to end
  // optional: per tick kTickLogWords words {last arrival, batches, kind bits, release, earliest
  // batch start, latest batch end, heuristic start, heuristic end}
  unsigned long long* tick_log;
  unsigned long long tick_log_cap;
  unsigned long long t_start;     // wall clock when the engine started
  // the tick's segments, nseg + 1 records (the last one's first batch is the
  // tick's batch count)
  SegRec* seg;
  Inst* insts;
  // instances the set-up kernels act on: sel_list[0 .. n_sel), or all when n_sel < 0
  const int32_t* sel_list;
  int32_t n_sel;
  int32_t pad_sel;
};

// Every pointer in these structures points to global memory. Device code
// reads them through pointers of the global address space: loads through a
// generic pointer are flat instructions, which count against both the vector
// and the LDS wait counters, so every LDS access would also wait for the
// outstanding global loads.
#define SSSP_GBL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ SSSP_GBL T* gbl(T* p) {
  return (SSSP_GBL T*)p;
}
// whole-struct store into global memory (the implicit assignment operator
// only takes generic objects)
template <typename T>
__device__ __forceinline__ void gstore(SSSP_GBL T* p, const T& v) {
  *(T*)p = v;
}
// the HIP atomics on global-address-space pointers (the casts back to generic
// pointers are folded: the instructions stay global atomics), beside HIP's own
using ::atomicAdd;
using ::atomicSub;
using ::atomicMin;
using ::atomicMax;
using ::atomicOr;
__device__ __forceinline__ int atomicAdd(SSSP_GBL int* p, int v) { return ::atomicAdd((int*)p, v); }
__device__ __forceinline__ unsigned int atomicAdd(SSSP_GBL unsigned int* p, unsigned int v) {
  return ::atomicAdd((unsigned int*)p, v);
}
__device__ __forceinline__ unsigned long long atomicAdd(SSSP_GBL unsigned long long* p, unsigned long long v) {
  return ::atomicAdd((unsigned long long*)p, v);
}
__device__ __forceinline__ unsigned long atomicAdd(SSSP_GBL unsigned long* p, unsigned long v) {
  return ::atomicAdd((unsigned long*)p, v);
}
__device__ __forceinline__ unsigned int atomicSub(SSSP_GBL unsigned int* p, unsigned int v) {
  return ::atomicSub((unsigned int*)p, v);
}
__device__ __forceinline__ unsigned int atomicMin(SSSP_GBL unsigned int* p, unsigned int v) {
  return ::atomicMin((unsigned int*)p, v);
}
__device__ __forceinline__ unsigned long long atomicMin(SSSP_GBL unsigned long long* p, unsigned long long v) {
  return ::atomicMin((unsigned long long*)p, v);
}
__device__ __forceinline__ unsigned int atomicMax(SSSP_GBL unsigned int* p, unsigned int v) {
  return ::atomicMax((unsigned int*)p, v);
}
__device__ __forceinline__ unsigned int atomicOr(SSSP_GBL unsigned int* p, unsigned int v) {
  return ::atomicOr((unsigned int*)p, v);
}
// whole-struct load from global memory
template <typename T>
__device__ __forceinline__ T gload(const SSSP_GBL T* p) {
  return *(const T*)p;
}
using GInst = SSSP_GBL Inst;
using GGlobals = SSSP_GBL Globals;
using GDevGraph = SSSP_GBL const DevGraph;

// host launch wrappers (engine.hip)
hipError_t launch_init(Globals* dG, long long max_n, hipStream_t stream);
// workgroups per CU of the engine kernel of a tile shape
int engine_blocks_per_cu(int shape);
hipError_t launch_engine(Globals* dG, int grid, bool persistent, int max_ticks, hipStream_t stream,
                         int shape);
hipError_t launch_overflow_check(Globals* dG, long long max_n, hipStream_t stream);
// distances of the selected instances from their state into the outputs
hipError_t launch_finish(Globals* dG, long long max_n, hipStream_t stream);
// per-instance phase and flags (2 words each) into status[0 .. 2 * ninst)
hipError_t launch_status(Globals* dG, int ninst, uint32_t* status, hipStream_t stream);
// the set-up + engine + overflow-check sequence of one solve as graph nodes
// after `dep` (may be null); the engine node is cooperative
hipError_t add_solve_nodes(hipGraph_t graph, hipGraphNode_t dep, Globals* dG, long long max_n, int grid,
                           int shape, hipGraphNode_t* last);

}  // namespace sssp
