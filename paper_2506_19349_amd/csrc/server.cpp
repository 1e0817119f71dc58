// Query server: continuous batching of single-source queries over graphs
// resident on one GPU.
//
// A pump thread owns a table of solver slots (one engine instance each) and
// runs the engine in bounded launches of `ticks_per_launch` device-wide ticks.
// Between two launches it retires the queries whose instance has finished and
// admits queued ones into free slots, as far as the memory budget allows; the
// admitted instances join the next launch while the others continue from
// their saved state. A query's result does not depend on what runs beside it:
// every instance keeps its own distances, lists and statistics, and the
// engine's schedule for it is a function of its own settled set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace sssp;

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState : int32_t { RS_DONE = 0, RS_QUEUED = 1, RS_RUNNING = 2 };

struct Request {
  int32_t graph = 0, source = 0;
  int32_t target = -1;          // point-to-point target, -1 for a full solve
  uint32_t* dist = nullptr;
  int32_t* parent = nullptr;    // shortest-path tree output, or NULL
  int32_t state = RS_QUEUED;
  int32_t status = SSSP_OK;
  int32_t slot = -1;
  double t_submit = 0, t_admit = -1, t_done = -1;
  uint32_t launches = 0;
};

}  // namespace

struct sssp_server {
  int device = 0;
  hipStream_t stream = nullptr;
  Workspace w;
  Opts o;
  int max_batch = 0, ticks_per_launch = 0, max_pending = 0;
  uint64_t budget = 0;
  std::vector<const sssp_graph*> graphs;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;
  std::unordered_map<int64_t, Request> reqs;
  // slot table: written by the pump thread only (under the lock), so the
  // pump reads it without locking
  std::vector<int64_t> slot_req;    // ticket in the slot, -1 when free
  std::vector<size_t> slot_bytes;   // device bytes of the slot's buffers
  std::vector<const sssp_graph*> slot_graph;
  std::vector<int32_t> slot_source;
  std::vector<int32_t> slot_target;
  std::vector<uint32_t*> slot_dist;
  std::vector<int32_t*> slot_parent;
  std::vector<uint64_t> slot_out;   // bytes of the running query's outputs
  uint64_t allocated = 0, peak_allocated = 0, out_active = 0, peak_in_use = 0;
  int active = 0, peak_active = 0;
  int64_t next_ticket = 1;
  bool stop = false;
  sssp_status dead = SSSP_OK;
  std::string dead_msg;
  uint64_t submitted = 0, admitted = 0, completed = 0, launches = 0;
  double busy_us = 0;

  int32_t* d_sel = nullptr;
  uint32_t* d_status = nullptr;
  char* h_pinned = nullptr;  // staging: Globals, max_batch Inst, selection list, its length
  Globals* hG = nullptr;
  Inst* hI = nullptr;
  int32_t* h_sel = nullptr;
  int32_t* h_nsel = nullptr;
  uint32_t* h_status = nullptr;
  hipEvent_t ev = nullptr;
  Clock::time_point t0;
  std::thread pump;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
  }
};

namespace {

int maxw_of(const Workspace& w) { return w.cus * w.occ * (kBlock / kWave); }

// Move queued requests into free slots while slots and the budget allow.
// Called with the lock held; the engine is not running.
void admit(sssp_server* S, std::vector<int>* fresh) {
  Workspace& w = S->w;
  while (!S->queue.empty()) {
    const int64_t t = S->queue.front();
    Request& r = S->reqs[t];
    const DevGraph& g = S->graphs[(size_t)r.graph]->gh.h;
    const Needs nd = needs_for(g, maxw_of(w));
    // the caller's outputs count against the budget while the query runs
    const uint64_t out_b = (r.parent ? 2 : 1) * sizeof(uint32_t) * (uint64_t)g.n;
    int pick = -1;
    size_t pick_bytes = 0;
    for (int i = 0; i < S->max_batch; ++i) {
      if (S->slot_req[(size_t)i] >= 0 || !slot_fits(w.slots[(size_t)i], nd)) continue;
      if (pick < 0 || S->slot_bytes[(size_t)i] < pick_bytes) {
        pick = i;
        pick_bytes = S->slot_bytes[(size_t)i];
      }
    }
    if (pick >= 0) {
      if (S->allocated + S->out_active + out_b > S->budget) {
        // release idle buffers of the other free slots, else wait for completions
        for (int i = 0; i < S->max_batch; ++i) {
          if (i == pick || S->slot_req[(size_t)i] >= 0 || S->slot_bytes[(size_t)i] == 0) continue;
          w.slots[(size_t)i].release();
          S->allocated -= S->slot_bytes[(size_t)i];
          S->slot_bytes[(size_t)i] = 0;
        }
        if (S->allocated + S->out_active + out_b > S->budget) break;
      }
    } else {
      // grow the free slot with the largest buffers (least to add)
      for (int i = 0; i < S->max_batch; ++i) {
        if (S->slot_req[(size_t)i] >= 0) continue;
        if (pick < 0 || S->slot_bytes[(size_t)i] > pick_bytes) {
          pick = i;
          pick_bytes = S->slot_bytes[(size_t)i];
        }
      }
      if (pick < 0) break;  // no free slot
      const SlotBuf& cur = w.slots[(size_t)pick];
      Needs m = nd;
      m.n = std::max(m.n, cur.n_cap);
      m.list = std::max(m.list, cur.list_cap);
      m.maxw = std::max(m.maxw, cur.maxw);
      m.heavy = std::max(m.heavy, cur.heavy_cap);
      m.hist = std::max(m.hist, cur.hist_cap);
      m.trace = std::max(m.trace, cur.trace_cap);
      m.ring = std::max(m.ring, cur.ring_cap);
      m.steprec = std::max(m.steprec, cur.steprec_cap);
      const size_t want = needs_bytes(m);
      if (S->allocated - pick_bytes + want + S->out_active + out_b > S->budget) {
        // release idle buffers of the other free slots
        for (int i = 0; i < S->max_batch; ++i) {
          if (i == pick || S->slot_req[(size_t)i] >= 0 || S->slot_bytes[(size_t)i] == 0) continue;
          w.slots[(size_t)i].release();
          S->allocated -= S->slot_bytes[(size_t)i];
          S->slot_bytes[(size_t)i] = 0;
        }
        if (S->allocated - pick_bytes + want + S->out_active + out_b > S->budget) break;
      }
      hipError_t e = ensure_slot(w.slots[(size_t)pick], m);
      S->allocated -= pick_bytes;
      S->slot_bytes[(size_t)pick] = 0;
      if (e != hipSuccess) {
        (void)hipGetLastError();
        r.state = RS_DONE;
        r.status = SSSP_E_NOMEM;
        r.t_done = S->now_us();
        S->queue.pop_front();
        S->completed += 1;
        continue;
      }
      S->slot_bytes[(size_t)pick] = want;
      S->allocated += want;
      S->peak_allocated = std::max(S->peak_allocated, S->allocated);
    }
    if (r.parent && w.slots[(size_t)pick].best_cap < g.n) {
      // a tree query also needs the slot's (distance, source) words
      const uint64_t extra = sizeof(uint64_t) * (uint64_t)g.n;
      if (S->allocated + extra + S->out_active + out_b > S->budget) {
        for (int i = 0; i < S->max_batch; ++i) {
          if (i == pick || S->slot_req[(size_t)i] >= 0 || S->slot_bytes[(size_t)i] == 0) continue;
          w.slots[(size_t)i].release();
          S->allocated -= S->slot_bytes[(size_t)i];
          S->slot_bytes[(size_t)i] = 0;
        }
        if (S->allocated + extra + S->out_active + out_b > S->budget) break;
      }
      if (ensure_best(w.slots[(size_t)pick], g.n) != hipSuccess) {
        (void)hipGetLastError();
        r.state = RS_DONE;
        r.status = SSSP_E_NOMEM;
        r.t_done = S->now_us();
        S->queue.pop_front();
        S->completed += 1;
        continue;
      }
      S->slot_bytes[(size_t)pick] += extra;
      S->allocated += extra;
      S->peak_allocated = std::max(S->peak_allocated, S->allocated);
    }
    S->slot_req[(size_t)pick] = t;
    S->slot_graph[(size_t)pick] = S->graphs[(size_t)r.graph];
    S->slot_source[(size_t)pick] = r.source;
    S->slot_target[(size_t)pick] = r.target;
    S->slot_dist[(size_t)pick] = r.dist;
    S->slot_parent[(size_t)pick] = r.parent;
    S->slot_out[(size_t)pick] = out_b;
    r.slot = pick;
    r.state = RS_RUNNING;
    r.t_admit = S->now_us();
    S->out_active += out_b;
    S->peak_in_use = std::max<uint64_t>(S->peak_in_use, S->allocated + S->out_active);
    S->queue.pop_front();
    fresh->push_back(pick);
    S->active += 1;
    S->admitted += 1;
    S->peak_active = std::max(S->peak_active, S->active);
  }
}

// One launch: set up the new instances, run the engine for a bounded number
// of ticks, and read every instance's phase and flags back.
sssp_status cycle(sssp_server* S, const std::vector<int>& fresh, std::vector<int>* finished) {
  Workspace& w = S->w;
  const hipStream_t st = S->stream;
  long long max_n = 1;
  for (size_t j = 0; j < fresh.size(); ++j) {
    const int i = fresh[j];
    const sssp_graph* g = S->slot_graph[(size_t)i];
    fill_inst(S->hI[i], w.slots[(size_t)i], g, S->slot_source[(size_t)i], S->slot_dist[(size_t)i], S->o,
              S->slot_parent[(size_t)i]);
    S->hI[i].target = S->slot_target[(size_t)i];
    max_n = std::max<long long>(max_n, g->gh.h.n);
    HIP_TRY(hipMemcpyAsync(w.dInst + i, S->hI + i, sizeof(Inst), hipMemcpyHostToDevice, st));
    S->h_sel[j] = i;
  }
  *S->h_nsel = (int32_t)fresh.size();
  if (!fresh.empty())
    HIP_TRY(hipMemcpyAsync(S->d_sel, S->h_sel, sizeof(int32_t) * fresh.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(&w.dG->n_sel, S->h_nsel, sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_init(w.dG, fresh.empty() ? 1 : max_n, st));
  const int occ = w.occ_s[S->o.shape];
  const int bpc = S->o.blocks_per_cu > 0 ? std::min(S->o.blocks_per_cu, occ) : occ;
  HIP_TRY(hipEventRecord(w.tev[0][0], st));
  HIP_TRY(launch_engine(w.dG, w.cus * bpc, true, S->ticks_per_launch, st, S->o.shape));
  HIP_TRY(hipEventRecord(w.tev[1][0], st));
  HIP_TRY(launch_status(w.dG, S->max_batch, S->d_status, st));
  HIP_TRY(hipMemcpyAsync(S->h_status, S->d_status, sizeof(uint32_t) * 2 * (size_t)S->max_batch,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(S->ev, st));
  HIP_TRY(hipEventSynchronize(S->ev));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, w.tev[0][0], w.tev[1][0]) == hipSuccess) S->busy_us += ms * 1000.0;
  S->launches += 1;
  // finished instances whose relaxations were cut by the +inf clamp: confirm
  std::vector<int> check;
  for (int i = 0; i < S->max_batch; ++i) {
    if (S->slot_req[(size_t)i] < 0 || S->h_status[2 * i] != PH_DONE) continue;
    finished->push_back(i);
    if (S->h_status[2 * i + 1] & FLAG_MAYBE_OVERFLOW) check.push_back(i);
  }
  if (!check.empty()) {
    long long cn = 1;
    for (size_t j = 0; j < check.size(); ++j) {
      S->h_sel[j] = check[j];
      cn = std::max<long long>(cn, S->slot_graph[(size_t)check[j]]->gh.h.n);
    }
    *S->h_nsel = (int32_t)check.size();
    HIP_TRY(hipMemcpyAsync(S->d_sel, S->h_sel, sizeof(int32_t) * check.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(&w.dG->n_sel, S->h_nsel, sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_overflow_check(w.dG, cn, st));
    HIP_TRY(launch_status(w.dG, S->max_batch, S->d_status, st));
    HIP_TRY(hipMemcpyAsync(S->h_status, S->d_status, sizeof(uint32_t) * 2 * (size_t)S->max_batch,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(S->ev, st));
    HIP_TRY(hipEventSynchronize(S->ev));
  }
  if (!finished->empty()) {
    // the finished queries' distances into their outputs
    long long fn = 1;
    for (size_t j = 0; j < finished->size(); ++j) {
      S->h_sel[j] = (*finished)[j];
      fn = std::max<long long>(fn, S->slot_graph[(size_t)(*finished)[j]]->gh.h.n);
    }
    *S->h_nsel = (int32_t)finished->size();
    HIP_TRY(hipMemcpyAsync(S->d_sel, S->h_sel, sizeof(int32_t) * finished->size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(&w.dG->n_sel, S->h_nsel, sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_finish(w.dG, fn, st));
    HIP_TRY(hipEventRecord(S->ev, st));
    HIP_TRY(hipEventSynchronize(S->ev));
  }
  return ok();
}

void pump_main(sssp_server* S) {
  (void)hipSetDevice(S->device);
  std::vector<int> fresh, finished;
  for (;;) {
    fresh.clear();
    finished.clear();
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || S->active > 0; });
      if (S->queue.empty() && S->active == 0) break;  // stop requested and nothing left
      if (S->dead == SSSP_OK) admit(S, &fresh);
      if (S->active == 0) {
        // nothing could be admitted and nothing runs: the queue waits for
        // memory that no running query will free -- fail the head
        if (!S->queue.empty()) {
          Request& r = S->reqs[S->queue.front()];
          r.state = RS_DONE;
          r.status = S->dead != SSSP_OK ? S->dead : SSSP_E_NOMEM;
          r.t_done = S->now_us();
          S->queue.pop_front();
          S->completed += 1;
          S->cv_done.notify_all();
        }
        continue;
      }
    }
    sssp_status st = cycle(S, fresh, &finished);
    std::string msg = st == SSSP_OK ? std::string() : std::string(sssp_last_error_message());
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const double t = S->now_us();
      if (st != SSSP_OK) {
        // a device failure ends every query in flight and refuses new ones
        S->dead = st;
        S->dead_msg = msg;
        finished.clear();
        for (int i = 0; i < S->max_batch; ++i)
          if (S->slot_req[(size_t)i] >= 0) finished.push_back(i);
      }
      for (int i = 0; i < S->max_batch; ++i)
        if (S->slot_req[(size_t)i] >= 0) S->reqs[S->slot_req[(size_t)i]].launches += 1;
      for (int i : finished) {
        Request& r = S->reqs[S->slot_req[(size_t)i]];
        uint32_t flags = S->h_status[2 * i + 1];
        if (st != SSSP_OK) r.status = st;
        else if (flags & FLAG_OVERFLOW) r.status = SSSP_E_DIST_OVERFLOW;
        else if (flags & (FLAG_CAPACITY | FLAG_MASS | FLAG_TIMEOUT | FLAG_TICKS | FLAG_TREE)) r.status = SSSP_E_DEVICE;
        else r.status = SSSP_OK;
        r.state = RS_DONE;
        r.t_done = t;
        S->slot_req[(size_t)i] = -1;
        S->out_active -= S->slot_out[(size_t)i];
        S->active -= 1;
        S->completed += 1;
      }
    }
    S->cv_done.notify_all();
  }
  S->cv_done.notify_all();
}

void server_free(sssp_server* S) {
  if (!S) return;
  if (S->ev) (void)hipEventDestroy(S->ev);
  if (S->d_sel) (void)hipFree(S->d_sel);
  if (S->d_status) (void)hipFree(S->d_status);
  if (S->h_pinned) (void)hipHostFree(S->h_pinned);
  ws_release(S->w);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

sssp_status server_setup(sssp_server* S) {
  HIP_TRY(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
  std::string err;
  if (!ws_setup(S->w, S->stream, &err)) return fail(SSSP_E_DEVICE, err);
  Workspace& w = S->w;
  HIP_TRY(ws_ensure_insts(w, S->max_batch));
  S->slot_req.assign((size_t)S->max_batch, -1);
  S->slot_bytes.assign((size_t)S->max_batch, 0);
  S->slot_graph.assign((size_t)S->max_batch, nullptr);
  S->slot_source.assign((size_t)S->max_batch, 0);
  S->slot_target.assign((size_t)S->max_batch, -1);
  S->slot_dist.assign((size_t)S->max_batch, nullptr);
  S->slot_parent.assign((size_t)S->max_batch, nullptr);
  S->slot_out.assign((size_t)S->max_batch, 0);
  HIP_TRY(hipMalloc(&S->d_sel, sizeof(int32_t) * (size_t)S->max_batch));
  HIP_TRY(hipMalloc(&S->d_status, sizeof(uint32_t) * 2 * (size_t)S->max_batch));
  const size_t bytes = sizeof(Globals) + sizeof(Inst) * (size_t)S->max_batch +
                       sizeof(int32_t) * ((size_t)S->max_batch + 1) + sizeof(uint32_t) * 2 * (size_t)S->max_batch;
  HIP_TRY(hipHostMalloc((void**)&S->h_pinned, bytes, hipHostMallocDefault));
  std::memset(S->h_pinned, 0, bytes);
  char* p = S->h_pinned;
  S->hG = reinterpret_cast<Globals*>(p);
  p += sizeof(Globals);
  S->hI = reinterpret_cast<Inst*>(p);
  p += sizeof(Inst) * (size_t)S->max_batch;
  S->h_sel = reinterpret_cast<int32_t*>(p);
  p += sizeof(int32_t) * (size_t)S->max_batch;
  S->h_nsel = reinterpret_cast<int32_t*>(p);
  p += sizeof(int32_t);
  S->h_status = reinterpret_cast<uint32_t*>(p);
  HIP_TRY(hipEventCreateWithFlags(&S->ev, hipEventDisableTiming));
  // the instance table starts with every slot idle
  Globals* hG = S->hG;
  hG->ninst = S->max_batch;
  hG->tick_limit = S->o.tick_limit;
  hG->seg = reinterpret_cast<SegRec*>(w.seg);
  hG->insts = w.dInst;
  hG->sel_list = S->d_sel;
  hG->n_sel = 0;
  // graphs come and go, so the shape is fixed here: the narrow one (on the
  // R-MAT scale 20/22/23 + 2048^2 grid mix: +1.3 % queries/s at saturation and
  // p99 -8 % against the standard shape; most ticks of a mix are small)
  if (S->o.shape < 0) S->o.shape = SHAPE_NARROW;
  hG->round_batch = round_batch_of(S->o.shape);
  hG->settle_batch = settle_batch_of(S->o.shape);
  for (int i = 0; i < S->max_batch; ++i) S->hI[i].phase = PH_DONE;
  HIP_TRY(hipMemcpyAsync(w.dG, hG, sizeof(Globals), hipMemcpyHostToDevice, S->stream));
  HIP_TRY(hipMemcpyAsync(w.dInst, S->hI, sizeof(Inst) * (size_t)S->max_batch, hipMemcpyHostToDevice,
                         S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  return ok();
}

}  // namespace

extern "C" {

sssp_server* sssp_server_create(const sssp_server_config* cfg, const sssp_options* opt) {
  if (!cfg) {
    fail(SSSP_E_INVAL, "config required");
    return nullptr;
  }
  if (cfg->max_batch < 0 || cfg->ticks_per_launch < 0 || cfg->max_pending < 0) {
    fail(SSSP_E_INVAL, "negative sizes");
    return nullptr;
  }
  std::string err;
  Opts o;
  if (!parse_opts(opt, &o, &err)) {
    fail(SSSP_E_INVAL, err);
    return nullptr;
  }
  if (o.host_driven) {
    fail(SSSP_E_INVAL, "the server runs the persistent engine: host_driven is not supported");
    return nullptr;
  }
  sssp_server* S = new (std::nothrow) sssp_server;
  if (!S) {
    fail(SSSP_E_NOMEM, "host allocation failed");
    return nullptr;
  }
  (void)hipGetDevice(&S->device);
  S->o = o;
  S->budget = cfg->budget_bytes;
  S->max_batch = cfg->max_batch > 0 ? cfg->max_batch : 64;
  S->ticks_per_launch = cfg->ticks_per_launch > 0 ? cfg->ticks_per_launch : 64;
  S->max_pending = cfg->max_pending > 0 ? cfg->max_pending : 1 << 16;
  S->t0 = Clock::now();
  sssp_status st = server_setup(S);
  if (st != SSSP_OK) {
    std::string m = sssp_last_error_message();
    server_free(S);
    (void)hipGetLastError();
    fail(st, m);
    return nullptr;
  }
  S->pump = std::thread(pump_main, S);
  ok();
  return S;
}

int32_t sssp_server_add_graph(sssp_server* S, const sssp_graph* g) {
  std::string err;
  if (!S) return fail(SSSP_E_INVAL, "server is NULL");
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  if (g->gh.device != S->device) return fail(SSSP_E_INVAL, "graph and server are on different devices");
  std::lock_guard<std::mutex> lk(S->mu);
  S->graphs.push_back(g);
  ok();
  return (int32_t)S->graphs.size() - 1;
}

int64_t sssp_server_query_bytes(sssp_server* S, int32_t graph_id) {
  if (!S) return fail(SSSP_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  if (graph_id < 0 || graph_id >= (int32_t)S->graphs.size()) return fail(SSSP_E_INVAL, "unknown graph id");
  const DevGraph& g = S->graphs[(size_t)graph_id]->gh.h;
  ok();
  return (int64_t)(needs_bytes(needs_for(g, maxw_of(S->w))) + sizeof(uint32_t) * (uint64_t)g.n);
}

sssp_status sssp_server_submit(sssp_server* S, int32_t graph_id, int32_t source, uint32_t* dist_out,
                               int64_t* ticket) {
  return sssp_server_submit_ex(S, graph_id, source, -1, dist_out, nullptr, ticket);
}

sssp_status sssp_server_submit_ex(sssp_server* S, int32_t graph_id, int32_t source, int32_t target,
                                  uint32_t* dist_out, int32_t* parent_out, int64_t* ticket) {
  if (!S || !dist_out || !ticket) return fail(SSSP_E_INVAL, "server, dist_out and ticket required");
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->dead != SSSP_OK) return fail(S->dead, "server stopped after a device failure: " + S->dead_msg);
  if (S->stop) return fail(SSSP_E_INVAL, "server is shutting down");
  if (graph_id < 0 || graph_id >= (int32_t)S->graphs.size()) return fail(SSSP_E_INVAL, "unknown graph id");
  const DevGraph& g = S->graphs[(size_t)graph_id]->gh.h;
  if (source < 0 || source >= g.n) return fail(SSSP_E_INVAL, "source out of range");
  if (target < -1 || target >= g.n) return fail(SSSP_E_INVAL, "target out of range (-1: none)");
  // workspace, the distance output and, for a tree, its output and 8-byte words
  const uint64_t need = needs_bytes(needs_for(g, maxw_of(S->w))) +
                        (parent_out ? 16 : 4) * (uint64_t)g.n;
  if (need > S->budget) return fail(SSSP_E_RANGE, "the query needs more device memory than the server's budget");
  if ((int)S->queue.size() >= S->max_pending) return fail(SSSP_E_BUSY, "admission queue is full");
  Request r;
  r.graph = graph_id;
  r.source = source;
  r.target = target;
  r.dist = dist_out;
  r.parent = parent_out;
  r.t_submit = S->now_us();
  const int64_t t = S->next_ticket++;
  S->reqs[t] = r;
  S->queue.push_back(t);
  S->submitted += 1;
  *ticket = t;
  lk.unlock();
  S->cv_work.notify_one();
  return ok();
}

sssp_status sssp_server_poll(sssp_server* S, int64_t ticket, int32_t* done) {
  if (!S || !done) return fail(SSSP_E_INVAL, "server and done required");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(SSSP_E_INVAL, "unknown ticket");
  *done = it->second.state == RS_DONE ? 1 : 0;
  return ok();
}

sssp_status sssp_server_wait(sssp_server* S, int64_t ticket) {
  if (!S) return fail(SSSP_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(SSSP_E_INVAL, "unknown ticket");
  S->cv_done.wait(lk, [&] { return S->reqs[ticket].state == RS_DONE; });
  const sssp_status st = (sssp_status)S->reqs[ticket].status;
  if (st != SSSP_OK) return fail(st, "query failed");
  return ok();
}

sssp_status sssp_server_request_info(sssp_server* S, int64_t ticket, sssp_request_info* out) {
  if (!S || !out) return fail(SSSP_E_INVAL, "server and output required");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(SSSP_E_INVAL, "unknown ticket");
  const Request& r = it->second;
  std::memset(out, 0, sizeof(*out));
  out->state = r.state;
  out->status = r.status;
  out->graph_id = r.graph;
  out->source = r.source;
  out->slot = r.slot;
  out->launches = r.launches;
  out->submit_us = r.t_submit;
  out->admit_us = r.t_admit;
  out->done_us = r.t_done;
  return ok();
}

sssp_status sssp_server_release(sssp_server* S, int64_t ticket) {
  if (!S) return fail(SSSP_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(SSSP_E_INVAL, "unknown ticket");
  if (it->second.state != RS_DONE) return fail(SSSP_E_BUSY, "query still in flight");
  S->reqs.erase(it);
  return ok();
}

sssp_status sssp_server_get_stats(sssp_server* S, sssp_server_stats* out) {
  if (!S || !out) return fail(SSSP_E_INVAL, "server and output required");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = S->submitted;
  out->admitted = S->admitted;
  out->completed = S->completed;
  out->launches = S->launches;
  out->engine_us = S->busy_us;
  out->now_us = S->now_us();
  out->budget_bytes = S->budget;
  out->allocated_bytes = S->allocated;
  out->peak_allocated_bytes = S->peak_allocated;
  out->peak_in_use_bytes = S->peak_in_use;
  out->active = S->active;
  out->peak_active = S->peak_active;
  out->queued = (int32_t)S->queue.size();
  out->max_batch = S->max_batch;
  return ok();
}

sssp_status sssp_server_destroy(sssp_server* S) {
  if (!S) return ok();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->pump.joinable()) S->pump.join();
  server_free(S);
  return ok();
}

}  // extern "C"
