// C ABI of the SSSP engine: argument checking, graph objects, per-stream
// solver workspaces and the launch sequence of a solve. Batched plans,
// the autotuner (plan.cpp) and the query server (server.cpp) build on the
// runtime declared in runtime.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "runtime.h"
#include "sizing.h"

namespace sssp {

thread_local sssp_status t_status = SSSP_OK;
thread_local std::string t_msg;

sssp_status fail(sssp_status s, const std::string& m) {
  t_status = s;
  t_msg = m;
  return s;
}

sssp_status ok() {
  t_status = SSSP_OK;
  t_msg.clear();
  return SSSP_OK;
}


uint32_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return (uint32_t)p;
}

// ------------------------------------------------------------ workspaces --



Needs needs_for(const DevGraph& g, int maxw) {
  Needs r;
  r.n = g.n;
  r.maxw = maxw;
  r.list = g.n;
  const int64_t hc = heavy_list_capacity(g.nnz, g.heavy_rows, kHeavyChunk);
  r.heavy = (int32_t)std::min<int64_t>(hc, INT32_MAX);
  r.hist = std::max(g.num_deg, 1);
  r.trace = 1 << 16;
  if (g.float_w) {
    // binary32 weights: the selection-threshold grid (kStNum bins per maxW)
    r.ring = kGridRing;
    r.steprec = 1u << 17;
  } else if (g.max_w <= kRingMax) {
    // per distance of the exact window (a solve may ask for it while max
    // weight <= kRingMax), and at least the grid's bins
    r.ring = pow2_at_least(std::max<uint64_t>(kGridRing, 2ull * g.max_w + 2));
    r.steprec = pow2_at_least(std::max<uint64_t>(64, 2ull * g.max_w + 64));
  } else {
    r.ring = kGridRing;  // the selection-threshold grid
    r.steprec = 1u << 17;
  }
  return r;
}

template <typename T>
hipError_t dev_alloc(T** p, size_t count, std::vector<void*>& list) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) {
    list.push_back(v);
    *p = static_cast<T*>(v);
  }
  return e;
}

size_t needs_bytes(const Needs& m) {
  size_t b = 0;
  b += sizeof(uint64_t) * (size_t)m.n;             // state
  b += sizeof(int32_t) * (size_t)m.list * 3;       // q[2], touched
  b += sizeof(UEntry) * (size_t)m.list * 2;        // ulist[2]
  b += sizeof(int32_t) * (size_t)m.n * 3;          // settled, plist[2]
  b += sizeof(Counters) * (size_t)m.maxw;
  b += sizeof(HeavyItem) * (size_t)m.heavy * 2;
  b += (sizeof(uint64_t) + sizeof(uint32_t)) * (size_t)m.ring;
  b += sizeof(uint32_t) * (size_t)m.hist;
  b += sizeof(StepRec) * (size_t)m.steprec;
  b += sizeof(TraceRec) * (size_t)m.trace;
  return b;
}

hipError_t ensure_best(SlotBuf& s, int32_t n) {
  if (s.best_cap >= n) return hipSuccess;
  uint64_t* p = nullptr;
  hipError_t e = dev_alloc(&p, (size_t)n, s.allocs);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  s.best = p;  // an older, smaller array stays in allocs until the slot is released
  s.best_cap = n;
  return hipSuccess;
}

bool slot_fits(const SlotBuf& s, const Needs& nd) {
  return s.n_cap >= nd.n && s.list_cap >= nd.list && s.maxw >= nd.maxw && s.heavy_cap >= nd.heavy &&
         s.hist_cap >= nd.hist && s.trace_cap >= nd.trace && s.ring_cap >= nd.ring &&
         s.steprec_cap >= nd.steprec;
}

hipError_t ensure_slot(SlotBuf& s, const Needs& nd) {
  if (slot_fits(s, nd)) return hipSuccess;
  Needs m;
  m.n = std::max(s.n_cap, nd.n);
  m.list = std::max(s.list_cap, nd.list);
  m.maxw = std::max(s.maxw, nd.maxw);
  m.heavy = std::max(s.heavy_cap, nd.heavy);
  m.hist = std::max(s.hist_cap, nd.hist);
  m.trace = std::max(s.trace_cap, nd.trace);
  m.ring = std::max(s.ring_cap, nd.ring);
  m.steprec = std::max(s.steprec_cap, nd.steprec);
  s.release();
  hipError_t e = hipSuccess;
  auto A = [&](auto** p, size_t c) {
    if (e == hipSuccess) e = dev_alloc(p, c, s.allocs);
  };
  A(&s.state, m.n);
  A(&s.q[0], m.list);
  A(&s.q[1], m.list);
  A(&s.touched, m.list);
  A(&s.settled, m.n);
  A(&s.plist[0], m.n);
  A(&s.plist[1], m.n);
  A(&s.ulist[0], m.list);
  A(&s.ulist[1], m.list);
  A(&s.cslot, (size_t)m.maxw);
  A(&s.heavy[0], m.heavy);
  A(&s.heavy[1], m.heavy);
  A(&s.ring_mass, m.ring);
  A(&s.ring_cnt, m.ring);
  A(&s.hist, m.hist);
  A(&s.steprec, m.steprec);
  A(&s.trace, m.trace);
  if (e != hipSuccess) {
    s.release();
    (void)hipGetLastError();
    return e;
  }
  s.n_cap = m.n;
  s.list_cap = m.list;
  s.maxw = m.maxw;
  s.heavy_cap = m.heavy;
  s.hist_cap = m.hist;
  s.trace_cap = m.trace;
  s.ring_cap = m.ring;
  s.steprec_cap = m.steprec;
  return hipSuccess;
}


std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

hipError_t ws_ensure_insts(Workspace& w, int k) {
  if (w.inst_cap >= k) return hipSuccess;
  if (w.stream) (void)hipStreamSynchronize(w.stream);
  else (void)hipDeviceSynchronize();
  for (void* p : w.allocs) (void)hipFree(p);
  w.allocs.clear();
  int cap = std::max(k, 1);
  hipError_t e = dev_alloc(&w.dG, 1, w.allocs);
  if (e == hipSuccess) e = dev_alloc(&w.dInst, (size_t)cap, w.allocs);
  // the tick table: one 16-byte record per segment, plus the end record
  if (e == hipSuccess)
    e = dev_alloc(&w.seg, (sizeof(SegRec) / sizeof(int32_t)) * (size_t)(kMaxSegPerInst * cap + 1), w.allocs);
  if (e != hipSuccess) {
    w.inst_cap = 0;
    return e;
  }
  w.inst_cap = cap;
  if ((int)w.slots.size() < cap) w.slots.resize((size_t)cap);
  return hipSuccess;
}

bool ws_setup(Workspace& w, hipStream_t stream, std::string* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = "hipGetDevice failed";
    return false;
  }
  w.stream = stream;
  w.device = dev;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    *err = "hipGetDeviceProperties failed";
    return false;
  }
  w.cus = prop.multiProcessorCount;
  w.occ = 1;
  for (int sh = 0; sh < kNumShapes; ++sh) {
    w.occ_s[sh] = engine_blocks_per_cu(sh);
    w.occ = std::max(w.occ, w.occ_s[sh]);
  }
  w.grid = w.cus * w.occ_s[SHAPE_STD];
  for (int i = 0; i < Workspace::kStages; ++i) {
    if (hipEventCreateWithFlags(&w.stage_ev[i], hipEventDisableTiming) != hipSuccess) {
      *err = "hipEventCreate failed";
      return false;
    }
  }
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < Workspace::kTimes; ++i)
      if (hipEventCreate(&w.tev[a][i]) != hipSuccess) {
        *err = "hipEventCreate failed";
        return false;
      }
  if (hipHostMalloc((void**)&w.pinned_flag, sizeof(unsigned int) * 4, hipHostMallocDefault) != hipSuccess) {
    *err = "hipHostMalloc failed";
    return false;
  }
  return true;
}

void ws_release(Workspace& w) {
  for (SlotBuf& s : w.slots) s.release();
  w.slots.clear();
  for (void* p : w.allocs) (void)hipFree(p);
  w.allocs.clear();
  w.inst_cap = 0;
  for (int i = 0; i < Workspace::kStages; ++i) {
    if (w.stage[i]) (void)hipHostFree(w.stage[i]);
    w.stage[i] = nullptr;
    w.stage_cap[i] = 0;
    if (w.stage_ev[i]) (void)hipEventDestroy(w.stage_ev[i]);
    w.stage_ev[i] = nullptr;
  }
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < Workspace::kTimes; ++i) {
      if (w.tev[a][i]) (void)hipEventDestroy(w.tev[a][i]);
      w.tev[a][i] = nullptr;
    }
  if (w.pinned_flag) (void)hipHostFree(w.pinned_flag);
  w.pinned_flag = nullptr;
  if (w.d_tick_log) (void)hipFree(w.d_tick_log);
  w.d_tick_log = nullptr;
}

Workspace* get_ws(hipStream_t stream, std::string* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = "hipGetDevice failed";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto key = std::make_pair(dev, stream);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second;
  Workspace* w = new Workspace;
  if (!ws_setup(*w, stream, err)) {
    ws_release(*w);
    delete w;
    return nullptr;
  }
  g_ws[key] = w;
  return w;
}

// A pinned staging buffer of at least `bytes`, free of pending copies.
void* ws_stage(Workspace& w, size_t bytes, int* idx) {
  int i = w.next_stage;
  w.next_stage = (i + 1) % Workspace::kStages;
  if (w.stage_used[i]) (void)hipEventSynchronize(w.stage_ev[i]);
  w.stage_used[i] = false;
  if (w.stage_cap[i] < bytes) {
    if (w.stage[i]) (void)hipHostFree(w.stage[i]);
    w.stage[i] = nullptr;
    w.stage_cap[i] = 0;
    if (hipHostMalloc(&w.stage[i], bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    w.stage_cap[i] = bytes;
  }
  *idx = i;
  return w.stage[i];
}


bool parse_opts(const sssp_options* o, Opts* r, std::string* err) {
  if (!o) return true;
  if (o->alpha < 0) { *err = "alpha must be >= 0"; return false; }
  if (o->alpha > 0) r->alpha = (uint32_t)o->alpha;
  if (o->beta != 0.0) {
    if (!(o->beta > 0.0 && o->beta < 1.0)) { *err = "beta must be in (0, 1)"; return false; }
    r->beta = o->beta;
  }
  if (o->traversal_opt < 0) r->topt = 0;
  r->host_driven = o->host_driven != 0;
  if (o->blocks_per_cu < 0) { *err = "blocks_per_cu must be >= 0"; return false; }
  r->blocks_per_cu = o->blocks_per_cu;
  if (o->heavy_split < 0) { *err = "heavy_split must be >= 0"; return false; }
  // the heavy-chunk lists are sized for the least split (sizing.h)
  if (o->heavy_split > 0) r->heavy = std::max(o->heavy_split, kDefaultHeavy);
  if (o->fuse_rounds < 0) r->fuse = 0;
  else if (o->fuse_rounds > 0) r->fuse = o->fuse_rounds;
  if (o->tile_shape < 0 || o->tile_shape > kNumShapes) {
    *err = "tile_shape must be in 0.." + std::to_string(kNumShapes);
    return false;
  }
  if (o->tile_shape > 0) r->shape = o->tile_shape - 1;
  r->st_grid = o->st_grid > 0 ? 1 : (o->st_grid < 0 ? -1 : 0);
  return true;
}

// Host image of one solve instance (its control words are set on the device).
void fill_inst(Inst& I, const SlotBuf& s, const sssp_graph* g, int32_t source, uint32_t* dist,
               const Opts& o, int32_t* parent) {
  std::memset(&I, 0, sizeof(Inst));
  I.g = g->gh.d;
  I.gc = g->gh.h;
  I.dist = dist;
  I.parent = parent;
  I.best = parent ? s.best : nullptr;
  I.mode = (I.best ? 1u : 0u) | (g->gh.h.float_w ? 2u : 0u);
  I.state = s.state;
  I.q[0] = s.q[0];
  I.q[1] = s.q[1];
  I.touched = s.touched;
  I.settled = s.settled;
  I.plist[0] = s.plist[0];
  I.plist[1] = s.plist[1];
  I.ulist[0] = s.ulist[0];
  I.ulist[1] = s.ulist[1];
  I.heavy[0] = s.heavy[0];
  I.heavy[1] = s.heavy[1];
  I.ring_mass = s.ring_mass;
  I.ring_cnt = s.ring_cnt;
  I.hist_cnt = s.hist;
  I.steprec = s.steprec;
  I.trace = s.trace;
  I.cslot = s.cslot;
  I.maxw = s.maxw;
  I.heavy_cap = s.heavy_cap;
  Needs nd = needs_for(g->gh.h, s.maxw);
  I.ring_mask = nd.ring - 1;
  I.steprec_mask = nd.steprec - 1;
  I.trace_cap = s.trace_cap;
  I.source = source;
  I.target = -1;
  I.n = g->gh.h.n;
  I.alpha = o.alpha;
  I.traversal_opt = o.topt;
  I.st_grid = o.st_grid;
  I.beta = o.beta;
  I.heavy_split = o.heavy;
  I.fuse_cap = o.fuse;
  I.phase = PH_DONE;
}

sssp_status run_instances(const sssp_graph* const* gs, const int32_t* sources, int k,
                          uint32_t* const* dists, const Opts& o, hipStream_t stream,
                          int32_t* const* parents, const int32_t* targets) {
  std::string err;
  Workspace* wp = get_ws(stream, &err);
  if (!wp) return fail(SSSP_E_DEVICE, err);
  return run_instances_ws(*wp, gs, sources, k, dists, o, stream, parents, targets);
}

// Enqueue k instances on workspace w; every argument has been checked.
// The default tile shape. Skewed degrees (graphs given a hub-first order) over
// many vertices take the standard shape, whose larger round batches suit the
// hubs' long rows (R-MAT scale 24: narrow +5.5 %). Everything else takes the
// narrow shape, which spreads small frontiers over more workgroups (R-MAT
// scales 12-22: -11 % to -0.6 %; grids and G(n, m): -3 to -9 %).
constexpr long long kStdShapeMinVertices = 1ll << 23;  // over all instances of the launch

int resolve_shape(const Opts& o, const sssp_graph* const* gs, int k) {
  if (o.shape >= 0) return o.shape;
  bool skewed = false;
  long long total = 0;
  for (int i = 0; i < k; ++i) {
    skewed = skewed || gs[i]->gh.h.relabelled > 0;
    total += gs[i]->gh.h.n;
  }
  return skewed && total >= kStdShapeMinVertices ? SHAPE_STD : SHAPE_NARROW;
}

sssp_status run_instances_ws(Workspace& w, const sssp_graph* const* gs, const int32_t* sources, int k,
                             uint32_t* const* dists, const Opts& o_in, hipStream_t stream,
                             int32_t* const* parents, const int32_t* targets) {
  Opts o = o_in;
  o.shape = resolve_shape(o_in, gs, k);
  HIP_TRY(ws_ensure_insts(w, k));
  long long max_n = 0;
  for (int i = 0; i < k; ++i) {
    const DevGraph& g = gs[i]->gh.h;
    max_n = std::max<long long>(max_n, g.n);
    Needs nd = needs_for(g, w.cus * w.occ * (kBlock / kWave));
    SlotBuf& s = w.slots[(size_t)i];
    if (!slot_fits(s, nd)) {
      (void)hipStreamSynchronize(stream);
      hipError_t e = ensure_slot(s, nd);
      if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(SSSP_E_NOMEM, "workspace allocation failed");
      HIP_TRY(e);
    }
    if (parents && parents[i] && s.best_cap < g.n) {
      (void)hipStreamSynchronize(stream);
      hipError_t e = ensure_best(s, g.n);
      if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(SSSP_E_NOMEM, "workspace allocation failed");
      HIP_TRY(e);
    }
  }
  const size_t bytes = sizeof(Globals) + sizeof(Inst) * (size_t)k;
  int si = 0;
  void* st = ws_stage(w, bytes, &si);
  if (!st) return fail(SSSP_E_NOMEM, "pinned staging allocation failed");
  Globals* hG = static_cast<Globals*>(st);
  Inst* hI = reinterpret_cast<Inst*>(static_cast<char*>(st) + sizeof(Globals));
  std::memset(st, 0, bytes);
  hG->ninst = k;
  hG->tick_limit = o.tick_limit;
  hG->tick_log = w.d_tick_log;
  hG->tick_log_cap = (unsigned long long)w.tick_log_cap;
  hG->seg = reinterpret_cast<SegRec*>(w.seg);
  hG->insts = w.dInst;
  hG->sel_list = nullptr;
  hG->n_sel = -1;
  hG->round_batch = round_batch_of(o.shape);
  hG->settle_batch = settle_batch_of(o.shape);
  for (int i = 0; i < k; ++i) {
    fill_inst(hI[i], w.slots[(size_t)i], gs[i], sources[i], dists[i], o, parents ? parents[i] : nullptr);
    if (targets) hI[i].target = targets[i];
  }
  HIP_TRY(hipMemcpyAsync(w.dG, hG, sizeof(Globals), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(w.dInst, hI, sizeof(Inst) * (size_t)k, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(w.stage_ev[si], stream));
  w.stage_used[si] = true;
  HIP_TRY(launch_init(w.dG, max_n, stream));
  const int tslot = (int)(w.t_rec % Workspace::kTimes);
  HIP_TRY(hipEventRecord(w.tev[0][tslot], stream));
  bool host_driven = o.host_driven || w.persistent_failed;
  if (!host_driven) {
    long long total_n = 0;
    for (int i = 0; i < k; ++i) total_n += gs[i]->gh.h.n;
    hipError_t e = launch_engine(w.dG, engine_grid(w, o, total_n), true, 0, stream, o.shape);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      w.persistent_failed = true;
      host_driven = true;
    }
  }
  if (host_driven) {
    // one tick per launch; the host polls the completion flag
    const int grid = w.cus * std::max(1, std::min(w.occ_s[o.shape], 8));
    for (long long t = 0;; ++t) {
      HIP_TRY(launch_engine(w.dG, grid, false, 0, stream, o.shape));
      HIP_TRY(hipMemcpyAsync(w.pinned_flag, &w.dG->all_done, sizeof(unsigned int) * 2,
                             hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      if (w.pinned_flag[0] || w.pinned_flag[1]) break;
      if (t > (long long)o.tick_limit + 4) return fail(SSSP_E_DEVICE, "tick limit exceeded");
    }
  }
  HIP_TRY(hipEventRecord(w.tev[1][tslot], stream));
  w.t_rec += 1;
  HIP_TRY(launch_overflow_check(w.dG, max_n, stream));
  HIP_TRY(launch_finish(w.dG, max_n, stream));
  w.last_k = k;
  return ok();
}

int engine_grid(const Workspace& w, const Opts& o, long long total_n) {
  const int occ = w.occ_s[o.shape];
  const int bpc = o.blocks_per_cu > 0 ? std::min(o.blocks_per_cu, occ) : occ;
  const int full = w.cus * bpc;
  if (o.blocks_per_cu > 0) return full;  // an explicit choice is honoured
  // no tick has more batches than the vertices fill: small graphs take a
  // smaller grid (cheaper barriers), a multiple of the XCD count
  const int rb = round_batch_of(o.shape);
  long long need = (total_n + rb - 1) / rb;
  need = ((need + kMaxXcd - 1) / kMaxXcd) * kMaxXcd;
  if (need < kMaxXcd) need = kMaxXcd;
  return (int)std::min<long long>(full, need);
}

bool check_graph(const sssp_graph* g, std::string* err) {
  if (!g) { *err = "graph is NULL"; return false; }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->gh.device) {
    *err = "the graph lives on another device than the current one";
    return false;
  }
  return true;
}

// Counters of instances [i0, i0 + k) of the workspace's last launch (the
// stream has been synchronised), summed; maps the engine's flags to a status.
sssp_status collect_counters(Workspace& w, int i0, int k, sssp_counters* out) {
  std::memset(out, 0, sizeof(*out));
  std::vector<Inst> hi((size_t)k);
  HIP_TRY(hipMemcpy(hi.data(), w.dInst + i0, sizeof(Inst) * (size_t)k, hipMemcpyDeviceToHost));
  Globals hg;
  HIP_TRY(hipMemcpy(&hg, w.dG, sizeof(Globals), hipMemcpyDeviceToHost));
  uint32_t flags = 0;
  for (Inst& I : hi) {
    if (!I.cslot) continue;
    std::vector<Counters> cs((size_t)I.maxw);
    HIP_TRY(hipMemcpy(cs.data(), I.cslot, sizeof(Counters) * (size_t)I.maxw, hipMemcpyDeviceToHost));
    for (const Counters& c : cs) {
      I.c.expansions += c.expansions;
      I.c.band_expansions += c.band_expansions;
      I.c.push_scanned += c.push_scanned;
      I.c.pull_vertices += c.pull_vertices;
      I.c.pull_scanned += c.pull_scanned;
      I.c.relax_success += c.relax_success;
      I.c.queue_entries += c.queue_entries;
    }
  }
  for (const Inst& I : hi) {
    out->expansions += I.c.expansions;
    out->band_expansions += I.c.band_expansions;
    out->push_scanned += I.c.push_scanned;
    out->pull_vertices += I.c.pull_vertices;
    out->pull_scanned += I.c.pull_scanned;
    out->relax_success += I.c.relax_success;
    out->queue_entries += I.c.queue_entries;
    out->rounds += I.c.rounds;
    out->pulls += I.c.pulls;
    out->steps += I.c.steps;
    out->ticks += I.c.ticks;
    out->fused_rounds += I.c.fused_rounds;
    out->pull_unsettled += I.c.pull_unsettled;
    flags |= I.flags.v;
  }
  out->high_d0 = hi[0].high_d0;
  out->gap0 = hi[0].gap0;
  flags |= hg.error;
  out->flags = flags;
  if (flags & FLAG_OVERFLOW) return fail(SSSP_E_DIST_OVERFLOW, "a distance does not fit below UINT32_MAX");
  if (flags & (FLAG_CAPACITY | FLAG_MASS | FLAG_TIMEOUT | FLAG_TICKS | FLAG_TREE))
    return fail(SSSP_E_DEVICE, "internal engine condition, flags = " + std::to_string(flags));
  return ok();
}

// Engine durations recorded on the workspace since the last call (microseconds).
sssp_status ws_take_times(Workspace& w, std::vector<float>* us) {
  long long from = std::max(w.t_read, w.t_rec - Workspace::kTimes);
  for (long long i = from; i < w.t_rec; ++i) {
    int sl = (int)(i % Workspace::kTimes);
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, w.tev[0][sl], w.tev[1][sl]));
    us->push_back(ms * 1000.f);
  }
  w.t_read = w.t_rec;
  return ok();
}

}  // namespace sssp

using namespace sssp;

// ================================================================== C ABI

extern "C" {

sssp_graph* sssp_graph_create_ex(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                                 const uint32_t* weight, int32_t flags) {
  if (n < 1 || rowptr == nullptr) {
    fail(SSSP_E_INVAL, "n must be >= 1 and rowptr non-NULL");
    return nullptr;
  }
  sssp_graph* g = new (std::nothrow) sssp_graph;
  if (!g) {
    fail(SSSP_E_NOMEM, "host allocation failed");
    return nullptr;
  }
  std::string msg;
  int rc = prep_graph(n, rowptr, colidx, weight, flags, &g->gh, &msg);
  if (rc != 0) {
    free_graph(&g->gh);
    delete g;
    (void)hipGetLastError();
    fail((sssp_status)rc, msg);
    return nullptr;
  }
  ok();
  return g;
}

sssp_graph* sssp_graph_create(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                              const uint32_t* weight) {
  return sssp_graph_create_ex(n, rowptr, colidx, weight, 0);
}

sssp_status sssp_graph_destroy(sssp_graph* g) {
  if (!g) return ok();
  (void)hipDeviceSynchronize();
  free_graph(&g->gh);
  delete g;
  return ok();
}

sssp_status sssp_graph_info_get(const sssp_graph* g, sssp_graph_info* out) {
  if (!g || !out) return fail(SSSP_E_INVAL, "NULL argument");
  const DevGraph& h = g->gh.h;
  std::memset(out, 0, sizeof(*out));
  out->n = h.n;
  out->nnz = h.nnz;
  out->nonisolated = g->gh.nonisolated;
  out->max_degree = g->gh.max_degree;
  out->distinct_degrees = g->gh.distinct_degrees;
  out->max_weight = h.max_w;
  out->high_d0 = h.high_d0;
  out->hub_first = (uint32_t)h.relabelled;
  out->device_bytes = g->gh.bytes;
  return ok();
}

sssp_status sssp_graph_sorted_rows(const sssp_graph* g, int32_t* col_out, uint32_t* w_out) {
  std::string err;
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  const DevGraph& h = g->gh.h;
  if (h.nnz > 0 && (!col_out || !w_out)) return fail(SSSP_E_INVAL, "NULL output");
  std::vector<uint64_t> tmp((size_t)h.nnz);
  if (h.nnz > 0) HIP_TRY(hipMemcpy(tmp.data(), h.adj, sizeof(uint64_t) * (size_t)h.nnz, hipMemcpyDeviceToHost));
  if (!h.new_of_old) {
    for (size_t e = 0; e < tmp.size(); ++e) {
      col_out[e] = (int32_t)(uint32_t)(tmp[e] & 0xffffffffull);
      w_out[e] = (uint32_t)(tmp[e] >> 32);
    }
    return ok();
  }
  // hub-first internal order: rows and columns back to the caller's ids, each
  // row re-sorted by (weight, caller's column)
  const size_t n = (size_t)h.n;
  std::vector<int32_t> rp(n + 1), ren(n), back(n);
  HIP_TRY(hipMemcpy(rp.data(), h.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ren.data(), h.new_of_old, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(back.data(), h.old_of_new, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  size_t pos = 0;
  std::vector<uint64_t> row;
  for (size_t u = 0; u < n; ++u) {
    const int32_t r = ren[u];
    row.clear();
    for (int32_t e = rp[(size_t)r]; e < rp[(size_t)r + 1]; ++e) {
      const uint64_t k = tmp[(size_t)e];
      row.push_back((k & 0xffffffff00000000ull) | (uint32_t)back[(size_t)(uint32_t)(k & 0xffffffffull)]);
    }
    std::sort(row.begin(), row.end());
    for (uint64_t k : row) {
      col_out[pos] = (int32_t)(uint32_t)(k & 0xffffffffull);
      w_out[pos] = (uint32_t)(k >> 32);
      ++pos;
    }
  }
  return ok();
}

sssp_status sssp_graph_rtow(const sssp_graph* g, uint32_t* rtow_out) {
  std::string err;
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  if (!rtow_out) return fail(SSSP_E_INVAL, "NULL output");
  HIP_TRY(hipMemcpy(rtow_out, g->gh.h.rtow, sizeof(uint32_t) * kRatioNum, hipMemcpyDeviceToHost));
  return ok();
}

sssp_status sssp_solve_ex(const sssp_graph* g, int32_t source, uint32_t* dist_out,
                          const sssp_options* opt, hipStream_t stream) {
  std::string err;
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  if (source < 0 || source >= g->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
  if (!dist_out) return fail(SSSP_E_INVAL, "dist_out is NULL");
  Opts o;
  if (!parse_opts(opt, &o, &err)) return fail(SSSP_E_INVAL, err);
  const sssp_graph* gs[1] = {g};
  int32_t src[1] = {source};
  uint32_t* d[1] = {dist_out};
  return run_instances(gs, src, 1, d, o, stream);
}

sssp_status sssp_solve_tree(const sssp_graph* g, int32_t source, uint32_t* dist_out, int32_t* parent_out,
                            const sssp_options* opt, hipStream_t stream) {
  std::string err;
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  if (source < 0 || source >= g->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
  if (!dist_out || !parent_out) return fail(SSSP_E_INVAL, "dist_out and parent_out are required");
  Opts o;
  if (!parse_opts(opt, &o, &err)) return fail(SSSP_E_INVAL, err);
  const sssp_graph* gs[1] = {g};
  int32_t src[1] = {source};
  uint32_t* d[1] = {dist_out};
  int32_t* par[1] = {parent_out};
  return run_instances(gs, src, 1, d, o, stream, par);
}

sssp_status sssp_solve_p2p(const sssp_graph* g, int32_t source, int32_t target, uint32_t* dist_out,
                           const sssp_options* opt, hipStream_t stream) {
  std::string err;
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  if (source < 0 || source >= g->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
  if (target < 0 || target >= g->gh.h.n) return fail(SSSP_E_INVAL, "target out of range");
  if (!dist_out) return fail(SSSP_E_INVAL, "dist_out is NULL");
  Opts o;
  if (!parse_opts(opt, &o, &err)) return fail(SSSP_E_INVAL, err);
  const sssp_graph* gs[1] = {g};
  int32_t src[1] = {source};
  uint32_t* d[1] = {dist_out};
  int32_t tgt[1] = {target};
  return run_instances(gs, src, 1, d, o, stream, nullptr, tgt);
}

sssp_status sssp_solve(const sssp_graph* g, int32_t source, uint32_t* dist_out, hipStream_t stream) {
  return sssp_solve_ex(g, source, dist_out, nullptr, stream);
}

sssp_status sssp_solve_batch(const sssp_graph* g, const int32_t* sources, int32_t k, uint32_t* dist_out,
                             hipStream_t stream) {
  std::string err;
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  if (k < 1 || !sources || !dist_out) return fail(SSSP_E_INVAL, "k >= 1, sources and dist_out required");
  for (int i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
  std::vector<const sssp_graph*> gs((size_t)k, g);
  std::vector<uint32_t*> d((size_t)k);
  for (int i = 0; i < k; ++i) d[(size_t)i] = dist_out + (size_t)i * (size_t)g->gh.h.n;
  Opts o;
  return run_instances(gs.data(), sources, k, d.data(), o, stream);
}

sssp_status sssp_solve_multi(const sssp_graph* const* gs, const int32_t* sources, int32_t k,
                             uint32_t* const* dist_outs, const sssp_options* opt, hipStream_t stream) {
  std::string err;
  if (k < 1 || !gs || !sources || !dist_outs) return fail(SSSP_E_INVAL, "k >= 1 and arrays required");
  for (int i = 0; i < k; ++i) {
    if (!check_graph(gs[i], &err)) return fail(SSSP_E_INVAL, err);
    if (sources[i] < 0 || sources[i] >= gs[i]->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
    if (!dist_outs[i]) return fail(SSSP_E_INVAL, "dist_outs entry is NULL");
  }
  Opts o;
  if (!parse_opts(opt, &o, &err)) return fail(SSSP_E_INVAL, err);
  return run_instances(gs, sources, k, dist_outs, o, stream);
}

sssp_status sssp_solve_multi_ex(const sssp_graph* const* gs, const int32_t* sources, const int32_t* targets,
                                int32_t k, uint32_t* const* dist_outs, int32_t* const* parent_outs,
                                const sssp_options* opt, hipStream_t stream) {
  std::string err;
  if (k < 1 || !gs || !sources || !dist_outs) return fail(SSSP_E_INVAL, "k >= 1 and arrays required");
  for (int i = 0; i < k; ++i) {
    if (!check_graph(gs[i], &err)) return fail(SSSP_E_INVAL, err);
    if (sources[i] < 0 || sources[i] >= gs[i]->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
    if (targets && (targets[i] < -1 || targets[i] >= gs[i]->gh.h.n))
      return fail(SSSP_E_INVAL, "target out of range (-1: none)");
    if (!dist_outs[i]) return fail(SSSP_E_INVAL, "dist_outs entry is NULL");
  }
  Opts o;
  if (!parse_opts(opt, &o, &err)) return fail(SSSP_E_INVAL, err);
  return run_instances(gs, sources, k, dist_outs, o, stream, parent_outs, targets);
}

sssp_status sssp_get_counters(hipStream_t stream, sssp_counters* out) {
  if (!out) return fail(SSSP_E_INVAL, "NULL output");
  std::string err;
  Workspace* w = get_ws(stream, &err);
  if (!w) return fail(SSSP_E_DEVICE, err);
  std::memset(out, 0, sizeof(*out));
  if (w->last_k == 0) return fail(SSSP_E_INVAL, "no solve on this stream");
  HIP_TRY(hipStreamSynchronize(stream));
  return collect_counters(*w, 0, w->last_k, out);
}

sssp_status sssp_get_schedule(hipStream_t stream, sssp_step* out, int32_t cap, int32_t* len) {
  if (!len || (cap > 0 && !out)) return fail(SSSP_E_INVAL, "NULL output");
  std::string err;
  Workspace* w = get_ws(stream, &err);
  if (!w) return fail(SSSP_E_DEVICE, err);
  if (w->last_k == 0) return fail(SSSP_E_INVAL, "no solve on this stream");
  HIP_TRY(hipStreamSynchronize(stream));
  Inst I;
  HIP_TRY(hipMemcpy(&I, w->dInst, sizeof(Inst), hipMemcpyDeviceToHost));
  *len = I.trace_len;
  int m = std::min(std::min(cap, I.trace_len), I.trace_cap);
  if (m > 0) {
    std::vector<TraceRec> t((size_t)m);
    HIP_TRY(hipMemcpy(t.data(), I.trace, sizeof(TraceRec) * (size_t)m, hipMemcpyDeviceToHost));
    for (int i = 0; i < m; ++i) {
      sssp_step& s = out[i];
      std::memset(&s, 0, sizeof(s));
      s.lb = t[(size_t)i].lb;
      s.ub = t[(size_t)i].ub;
      s.st = t[(size_t)i].st;
      s.rounds = t[(size_t)i].rounds;
      s.pulled = t[(size_t)i].pulled;
      s.L = t[(size_t)i].L;
      s.S = t[(size_t)i].S;
      s.h = t[(size_t)i].h;
      s.gap = t[(size_t)i].gap;
      s.st_next = t[(size_t)i].st_next;
    }
  }
  return ok();
}

sssp_status sssp_engine_times(hipStream_t stream, float* us_out, int32_t cap, int32_t* n_out) {
  if (!n_out || (cap > 0 && !us_out)) return fail(SSSP_E_INVAL, "NULL output");
  std::string err;
  Workspace* w = get_ws(stream, &err);
  if (!w) return fail(SSSP_E_DEVICE, err);
  HIP_TRY(hipStreamSynchronize(stream));
  long long from = std::max(w->t_read, w->t_rec - Workspace::kTimes);
  int m = 0;
  for (long long i = from; i < w->t_rec && m < cap; ++i, ++m) {
    int sl = (int)(i % Workspace::kTimes);
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, w->tev[0][sl], w->tev[1][sl]));
    us_out[m] = ms * 1000.f;
  }
  *n_out = m;
  w->t_read = w->t_rec;
  return ok();
}

sssp_status sssp_debug_tick_log(hipStream_t stream, int32_t cap) {
  if (cap < 0) return fail(SSSP_E_INVAL, "cap must be >= 0");
  std::string err;
  Workspace* w = get_ws(stream, &err);
  if (!w) return fail(SSSP_E_DEVICE, err);
  HIP_TRY(hipStreamSynchronize(stream));
  if (w->d_tick_log) HIP_TRY(hipFree(w->d_tick_log));
  w->d_tick_log = nullptr;
  w->tick_log_cap = 0;
  if (cap > 0) {
    HIP_TRY(hipMalloc(&w->d_tick_log, sizeof(unsigned long long) * kTickLogWords * (size_t)cap));
    w->tick_log_cap = cap;
  }
  return ok();
}

sssp_status sssp_debug_get_tick_log(hipStream_t stream, uint64_t* out, int32_t cap, int32_t* len,
                                    uint64_t* t_start) {
  if (!len || !t_start || (cap > 0 && !out)) return fail(SSSP_E_INVAL, "NULL output");
  std::string err;
  Workspace* w = get_ws(stream, &err);
  if (!w) return fail(SSSP_E_DEVICE, err);
  if (!w->d_tick_log || w->last_k == 0) return fail(SSSP_E_INVAL, "tick log not enabled or no solve");
  HIP_TRY(hipStreamSynchronize(stream));
  Globals hg;
  HIP_TRY(hipMemcpy(&hg, w->dG, sizeof(Globals), hipMemcpyDeviceToHost));
  int m = (int)std::min<unsigned long long>(hg.ticks, (unsigned long long)w->tick_log_cap);
  *len = (int32_t)hg.ticks;
  *t_start = hg.t_start;
  m = std::min(m, cap);
  if (m > 0) HIP_TRY(hipMemcpy(out, w->d_tick_log, sizeof(uint64_t) * kTickLogWords * (size_t)m, hipMemcpyDeviceToHost));
  return ok();
}

sssp_status sssp_release_workspaces(void) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  sssp_status st = SSSP_OK;
  for (auto& kv : g_ws) {
    Workspace* w = kv.second;
    // the stream may already be gone: wait for the whole device instead
    if (hipSetDevice(kv.first.first) != hipSuccess || hipDeviceSynchronize() != hipSuccess) st = SSSP_E_DEVICE;
    ws_release(*w);
    delete w;
  }
  g_ws.clear();
  if (have_cur) (void)hipSetDevice(cur);
  if (st != SSSP_OK) return fail(st, "a device did not finish its work before release");
  return ok();
}

sssp_status sssp_last_error(void) { return t_status; }

const char* sssp_last_error_message(void) { return t_msg.c_str(); }

const char* sssp_status_str(sssp_status s) {
  switch (s) {
    case SSSP_OK: return "ok";
    case SSSP_E_INVAL: return "invalid argument";
    case SSSP_E_NOT_SYMMETRIC: return "graph is not symmetric";
    case SSSP_E_RANGE: return "size beyond limits";
    case SSSP_E_DIST_OVERFLOW: return "distance overflow";
    case SSSP_E_NOMEM: return "out of memory";
    case SSSP_E_DEVICE: return "device error";
    case SSSP_E_BUSY: return "busy";
  }
  return "unknown status";
}

const char* sssp_version(void) { return "paper_2506_19349_amd 0.1 (gfx950)"; }

}  // extern "C"
