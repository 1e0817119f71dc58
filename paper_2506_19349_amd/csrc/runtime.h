// Host runtime shared by the C ABI sources: status reporting, solver
// workspaces (per-instance device buffers, the instance table, pinned
// staging), solver options, and the enqueue sequence of a solve.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sssp.h"
#include "engine.h"
#include "prep.h"

struct sssp_graph {
  sssp::GraphHost gh;
};

namespace sssp {

// Record a failure for sssp_last_error / sssp_last_error_message (thread-local).
sssp_status fail(sssp_status s, const std::string& m);
sssp_status ok();

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) return fail(SSSP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

uint32_t pow2_at_least(uint64_t x);

// ------------------------------------------------------------ workspaces --

// Device buffers of one solve instance, reused across solves while they fit.
struct SlotBuf {
  int32_t n_cap = 0, list_cap = 0, maxw = 0, heavy_cap = 0, hist_cap = 0, trace_cap = 0;
  uint32_t ring_cap = 0, steprec_cap = 0;
  uint64_t* state = nullptr;
  int32_t* q[2] = {nullptr, nullptr};
  int32_t* touched = nullptr;
  int32_t* settled = nullptr;
  int32_t* plist[2] = {nullptr, nullptr};
  UEntry* ulist[2] = {nullptr, nullptr};
  HeavyItem* heavy[2] = {nullptr, nullptr};
  uint64_t* ring_mass = nullptr;
  uint32_t* ring_cnt = nullptr;
  uint32_t* hist = nullptr;
  StepRec* steprec = nullptr;
  TraceRec* trace = nullptr;
  Counters* cslot = nullptr;
  // the tree's (distance, source) words: only for solves that ask for a tree
  uint64_t* best = nullptr;
  int32_t best_cap = 0;
  std::vector<void*> allocs;
  void release() {
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    n_cap = list_cap = maxw = heavy_cap = hist_cap = trace_cap = 0;
    ring_cap = steprec_cap = 0;
    best = nullptr;
    best_cap = 0;
  }
};

struct Needs {
  int32_t n, list, maxw, heavy, hist, trace;
  uint32_t ring, steprec;
};

Needs needs_for(const DevGraph& g, int maxw);
bool slot_fits(const SlotBuf& s, const Needs& nd);
hipError_t ensure_slot(SlotBuf& s, const Needs& nd);
// the tree's words for n vertices in slot s
hipError_t ensure_best(SlotBuf& s, int32_t n);
// device bytes a slot of these sizes holds
size_t needs_bytes(const Needs& nd);

// Everything one launch sequence needs: the instance table, the tick-table
// arrays, the slots, pinned staging and timing events.
struct Workspace {
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<SlotBuf> slots;
  int inst_cap = 0;
  Globals* dG = nullptr;
  Inst* dInst = nullptr;
  int32_t* seg = nullptr;  // the tick table: (kMaxSegPerInst * inst_cap + 1) 16-byte SegRec records
  std::vector<void*> allocs;
  // pinned staging ring
  static constexpr int kStages = 4;
  void* stage[kStages] = {nullptr, nullptr, nullptr, nullptr};
  size_t stage_cap[kStages] = {0, 0, 0, 0};
  hipEvent_t stage_ev[kStages] = {nullptr, nullptr, nullptr, nullptr};
  bool stage_used[kStages] = {false, false, false, false};
  int next_stage = 0;
  unsigned int* pinned_flag = nullptr;
  int grid = 0;
  int cus = 0;
  int occ = 0;                  // the most workgroups per CU of any tile shape (sizes per-wave slots)
  int occ_s[kNumShapes] = {};   // workgroups per CU of each tile shape's engine kernel
  // last solve
  int last_k = 0;
  bool persistent_failed = false;
  // optional per-tick log of the engine (debug)
  unsigned long long* d_tick_log = nullptr;
  int tick_log_cap = 0;
  // engine-kernel timing ring (HIP events around each engine launch)
  static constexpr int kTimes = 256;
  hipEvent_t tev[2][kTimes] = {};
  long long t_rec = 0, t_read = 0;
};

hipError_t ws_ensure_insts(Workspace& w, int k);
// Set up a workspace for the current device (events, pinned flag, grid size).
bool ws_setup(Workspace& w, hipStream_t stream, std::string* err);
// Release everything a workspace holds (the stream is not destroyed).
void ws_release(Workspace& w);
// The per-(device, stream) workspace of the plain solves.
Workspace* get_ws(hipStream_t stream, std::string* err);
void* ws_stage(Workspace& w, size_t bytes, int* idx);

struct Opts {
  uint32_t alpha = 3;
  double beta = 0.9;
  uint32_t topt = 1;
  bool host_driven = false;
  int blocks_per_cu = 0;
  int heavy = kDefaultHeavy;
  int fuse = kDefaultFuse;
  int shape = -1;  // tile shape (engine kernel instantiation); -1: by the graphs (resolve_shape)
  int st_grid = 0;  // computeST's candidates for integer weights (Inst::st_grid)
  unsigned long long tick_limit = 1ull << 22;
};

bool parse_opts(const sssp_options* o, Opts* r, std::string* err);
// The tile shape of a launch over these graphs: the one asked for, else the
// standard shape when a graph has skewed degrees (a hub-first order) and the
// narrow shape (256-item round batches, more of them per frontier) when none
// has.
int resolve_shape(const Opts& o, const sssp_graph* const* gs, int k);
// Persistent grid size for k instances of total_n vertices: the tuned or
// requested workgroups per CU, fewer for small graphs.
int engine_grid(const Workspace& w, const Opts& o, long long total_n);

// parent: the caller's tree output, or null (then the slot needs no tree words)
void fill_inst(Inst& I, const SlotBuf& s, const sssp_graph* g, int32_t source, uint32_t* dist,
               const Opts& o, int32_t* parent = nullptr);
// parents: null, or k tree outputs (entries may be null); targets: null, or k
// point-to-point targets (-1: none)
sssp_status run_instances(const sssp_graph* const* gs, const int32_t* sources, int k,
                          uint32_t* const* dists, const Opts& o, hipStream_t stream,
                          int32_t* const* parents = nullptr, const int32_t* targets = nullptr);
sssp_status run_instances_ws(Workspace& w, const sssp_graph* const* gs, const int32_t* sources, int k,
                             uint32_t* const* dists, const Opts& o, hipStream_t stream,
                             int32_t* const* parents = nullptr, const int32_t* targets = nullptr);
bool check_graph(const sssp_graph* g, std::string* err);
sssp_status collect_counters(Workspace& w, int i0, int k, sssp_counters* out);
sssp_status ws_take_times(Workspace& w, std::vector<float>* us);

}  // namespace sssp
