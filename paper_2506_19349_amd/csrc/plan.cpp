// Batched solves captured once as a HIP graph and replayed with new sources,
// and the autotuner that picks the engine's launch knobs for a workload.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "runtime.h"

using namespace sssp;

struct sssp_plan {
  Workspace w;
  int k = 0;
  int device = 0;
  std::vector<const sssp_graph*> gs;
  Opts o;
  void* pinned = nullptr;  // Globals + k Inst images, read by the graph's copy nodes at replay
  Globals* hG = nullptr;
  Inst* hI = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool pending = false;
  hipStream_t last_stream = nullptr;
};

namespace {

void plan_free(sssp_plan* p) {
  if (!p) return;
  if (p->pending && p->done) (void)hipEventSynchronize(p->done);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->done) (void)hipEventDestroy(p->done);
  if (p->pinned) (void)hipHostFree(p->pinned);
  ws_release(p->w);
  delete p;
}

sssp_status plan_build(sssp_plan* p, uint32_t* const* dist_outs, int32_t* const* parent_outs,
                       hipStream_t stream) {
  Workspace& w = p->w;
  std::string err;
  if (!ws_setup(w, stream, &err)) return fail(SSSP_E_DEVICE, err);
  const int k = p->k;
  p->o.shape = resolve_shape(p->o, p->gs.data(), k);
  HIP_TRY(ws_ensure_insts(w, k));
  long long max_n = 0;
  for (int i = 0; i < k; ++i) {
    const DevGraph& g = p->gs[(size_t)i]->gh.h;
    max_n = std::max<long long>(max_n, g.n);
    hipError_t e = ensure_slot(w.slots[(size_t)i], needs_for(g, w.cus * w.occ * (kBlock / kWave)));
    if (e == hipSuccess && parent_outs && parent_outs[i]) e = ensure_best(w.slots[(size_t)i], g.n);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      return fail(SSSP_E_NOMEM, "workspace allocation failed");
    HIP_TRY(e);
  }
  const size_t bytes = sizeof(Globals) + sizeof(Inst) * (size_t)k;
  HIP_TRY(hipHostMalloc(&p->pinned, bytes, hipHostMallocDefault));
  std::memset(p->pinned, 0, bytes);
  p->hG = static_cast<Globals*>(p->pinned);
  p->hI = reinterpret_cast<Inst*>(static_cast<char*>(p->pinned) + sizeof(Globals));
  Globals* hG = p->hG;
  hG->ninst = k;
  hG->tick_limit = p->o.tick_limit;
  hG->seg = reinterpret_cast<SegRec*>(w.seg);
  hG->insts = w.dInst;
  hG->sel_list = nullptr;
  hG->n_sel = -1;
  hG->round_batch = round_batch_of(p->o.shape);
  hG->settle_batch = settle_batch_of(p->o.shape);
  for (int i = 0; i < k; ++i)
    fill_inst(p->hI[i], w.slots[(size_t)i], p->gs[(size_t)i], 0, dist_outs[i], p->o,
              parent_outs ? parent_outs[i] : nullptr);

  long long total_n = 0;
  for (int i = 0; i < k; ++i) total_n += p->gs[(size_t)i]->gh.h.n;
  const int grid = engine_grid(w, p->o, total_n);
  HIP_TRY(hipGraphCreate(&p->graph, 0));
  hipGraphNode_t n_g, n_i, last;
  HIP_TRY(hipGraphAddMemcpyNode1D(&n_g, p->graph, nullptr, 0, w.dG, p->hG, sizeof(Globals),
                                  hipMemcpyHostToDevice));
  HIP_TRY(hipGraphAddMemcpyNode1D(&n_i, p->graph, &n_g, 1, w.dInst, p->hI, sizeof(Inst) * (size_t)k,
                                  hipMemcpyHostToDevice));
  HIP_TRY(add_solve_nodes(p->graph, n_i, w.dG, max_n, grid, p->o.shape, &last));
  HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  HIP_TRY(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
  w.last_k = k;
  return ok();
}

}  // namespace

extern "C" {

sssp_plan* sssp_plan_create(const sssp_graph* const* gs, int32_t k, uint32_t* const* dist_outs,
                            const sssp_options* opt, hipStream_t stream) {
  return sssp_plan_create_ex(gs, k, dist_outs, nullptr, opt, stream);
}

sssp_plan* sssp_plan_create_ex(const sssp_graph* const* gs, int32_t k, uint32_t* const* dist_outs,
                               int32_t* const* parent_outs, const sssp_options* opt, hipStream_t stream) {
  std::string err;
  if (k < 1 || !gs || !dist_outs) {
    fail(SSSP_E_INVAL, "k >= 1, graphs and dist_outs required");
    return nullptr;
  }
  for (int i = 0; i < k; ++i) {
    if (!check_graph(gs[i], &err)) {
      fail(SSSP_E_INVAL, err);
      return nullptr;
    }
    if (!dist_outs[i]) {
      fail(SSSP_E_INVAL, "dist_outs entry is NULL");
      return nullptr;
    }
  }
  Opts o;
  if (!parse_opts(opt, &o, &err)) {
    fail(SSSP_E_INVAL, err);
    return nullptr;
  }
  if (o.host_driven) {
    fail(SSSP_E_INVAL, "a plan replays one persistent launch: host_driven is not supported");
    return nullptr;
  }
  sssp_plan* p = new (std::nothrow) sssp_plan;
  if (!p) {
    fail(SSSP_E_NOMEM, "host allocation failed");
    return nullptr;
  }
  p->k = k;
  p->gs.assign(gs, gs + k);
  p->o = o;
  (void)hipGetDevice(&p->device);
  sssp_status st = plan_build(p, dist_outs, parent_outs, stream);
  if (st != SSSP_OK) {
    std::string m = sssp_last_error_message();
    plan_free(p);
    (void)hipGetLastError();
    fail(st, m);
    return nullptr;
  }
  ok();
  return p;
}

sssp_status sssp_plan_run(sssp_plan* p, const int32_t* sources, hipStream_t stream) {
  return sssp_plan_run_ex(p, sources, nullptr, stream);
}

sssp_status sssp_plan_run_ex(sssp_plan* p, const int32_t* sources, const int32_t* targets, hipStream_t stream) {
  if (!p || !sources) return fail(SSSP_E_INVAL, "plan and sources required");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(SSSP_E_INVAL, "the plan lives on another device than the current one");
  for (int i = 0; i < p->k; ++i) {
    const int32_t n = p->gs[(size_t)i]->gh.h.n;
    if (sources[i] < 0 || sources[i] >= n) return fail(SSSP_E_INVAL, "source out of range");
    if (targets && (targets[i] < -1 || targets[i] >= n)) return fail(SSSP_E_INVAL, "target out of range (-1: none)");
  }
  // the previous replay's copy nodes read the pinned images: wait for it
  if (p->pending) HIP_TRY(hipEventSynchronize(p->done));
  for (int i = 0; i < p->k; ++i) {
    p->hI[i].source = sources[i];
    p->hI[i].target = targets ? targets[i] : -1;
  }
  HIP_TRY(hipGraphLaunch(p->exec, stream));
  HIP_TRY(hipEventRecord(p->done, stream));
  p->pending = true;
  p->last_stream = stream;
  return ok();
}

sssp_status sssp_plan_counters(sssp_plan* p, sssp_counters* out) {
  if (!p || !out) return fail(SSSP_E_INVAL, "plan and output required");
  if (!p->pending) return fail(SSSP_E_INVAL, "the plan has not run");
  HIP_TRY(hipEventSynchronize(p->done));
  return collect_counters(p->w, 0, p->k, out);
}

sssp_status sssp_plan_destroy(sssp_plan* p) {
  plan_free(p);
  return ok();
}

// ------------------------------------------------------------- autotuner --

sssp_status sssp_autotune(const sssp_graph* const* gs, const int32_t* sources, int32_t k, int32_t batched,
                          int32_t tune_beta, sssp_options* inout, sssp_tune_report* report,
                          hipStream_t stream) {
  std::string err;
  if (k < 1 || !gs || !sources || !inout) return fail(SSSP_E_INVAL, "k >= 1, graphs, sources and options required");
  for (int i = 0; i < k; ++i) {
    if (!check_graph(gs[i], &err)) return fail(SSSP_E_INVAL, err);
    if (sources[i] < 0 || sources[i] >= gs[i]->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
  }
  Opts base;
  if (!parse_opts(inout, &base, &err)) return fail(SSSP_E_INVAL, err);
  base.host_driven = false;

  Workspace w;
  if (!ws_setup(w, stream, &err)) {
    ws_release(w);
    return fail(SSSP_E_DEVICE, err);
  }
  // distance buffers the trials write into (results are discarded)
  size_t total = 0, max_n = 0;
  for (int i = 0; i < k; ++i) {
    total += (size_t)gs[i]->gh.h.n;
    max_n = std::max(max_n, (size_t)gs[i]->gh.h.n);
  }
  uint32_t* scratch = nullptr;
  const size_t words = batched ? total : max_n;
  if (hipMalloc(&scratch, sizeof(uint32_t) * words) != hipSuccess) {
    ws_release(w);
    (void)hipGetLastError();
    return fail(SSSP_E_NOMEM, "autotune scratch allocation failed");
  }
  std::vector<uint32_t*> outs((size_t)k);
  size_t off = 0;
  for (int i = 0; i < k; ++i) {
    outs[(size_t)i] = batched ? scratch + off : scratch;
    off += (size_t)gs[i]->gh.h.n;
  }

  int evals = 0;
  // engine microseconds of the workload under options o: one untimed pass,
  // then the timed pass
  auto measure = [&](const Opts& o, double* us) -> sssp_status {
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<float> t;
      sssp_status st = ws_take_times(w, &t);
      if (st != SSSP_OK) return st;
      if (batched) {
        st = run_instances_ws(w, gs, sources, k, outs.data(), o, stream);
        if (st != SSSP_OK) return st;
      } else {
        for (int i = 0; i < k; ++i) {
          st = run_instances_ws(w, gs + i, sources + i, 1, outs.data() + i, o, stream);
          if (st != SSSP_OK) return st;
        }
      }
      HIP_TRY(hipStreamSynchronize(stream));
      sssp_counters c;
      st = collect_counters(w, 0, batched ? k : 1, &c);
      if (st != SSSP_OK) return st;
      t.clear();
      st = ws_take_times(w, &t);
      if (st != SSSP_OK) return st;
      double s = 0;
      for (float x : t) s += x;
      *us = s;
    }
    ++evals;
    return ok();
  };

  sssp_status st = SSSP_OK;
  Opts best = base;
  double best_us = 0, base_us = 0;
  st = measure(best, &best_us);
  base_us = best_us;
  // coordinate descent over the launch knobs; none of them changes a distance
  // knobs in turn: the tile shape (engine instantiation: items per round
  // batch 256 / 512 / 1024, settle batch 1024 / 2048), workgroups per CU (1,
  // 2, all the shape allows), the heavy-range split, bucket fusion on / off,
  // and beta within the range Section 4.3 finds insensitive
  for (int knob = 0; knob < 5 && st == SSSP_OK; ++knob) {
    std::vector<Opts> cands;
    if (knob == 0) {
      for (int sh = 0; sh < kNumShapes; ++sh) { Opts o = best; o.shape = sh; cands.push_back(o); }
    } else if (knob == 1) {
      const int occ = w.occ_s[resolve_shape(best, gs, k)];
      for (int b : {1, 2, 0}) {
        if (b > occ) continue;
        Opts o = best;
        o.blocks_per_cu = b;  // 0: the default grid rule (all the shape allows, fewer for small graphs)
        cands.push_back(o);
      }
    } else if (knob == 2) {
      for (int h : {kDefaultHeavy, 256, 1024, 4096}) { Opts o = best; o.heavy = h; cands.push_back(o); }
    } else if (knob == 3) {
      for (int f : {kDefaultFuse, 0}) { Opts o = best; o.fuse = f; cands.push_back(o); }
    } else if (tune_beta) {
      for (double b : {0.85, 0.9, 0.95}) { Opts o = best; o.beta = b; cands.push_back(o); }
    }
    for (const Opts& o : cands) {
      double us = 0;
      st = measure(o, &us);
      if (st != SSSP_OK) break;
      if (us < best_us) {
        best_us = us;
        best = o;
      }
    }
  }
  (void)hipStreamSynchronize(stream);
  (void)hipFree(scratch);
  ws_release(w);
  if (st != SSSP_OK) return st;
  inout->alpha = (int32_t)best.alpha;
  inout->beta = best.beta;
  inout->traversal_opt = best.topt ? 1 : -1;
  inout->host_driven = 0;
  inout->blocks_per_cu = best.blocks_per_cu;  // 0: the default grid rule
  inout->heavy_split = best.heavy;
  inout->fuse_rounds = best.fuse > 0 ? best.fuse : -1;
  inout->tile_shape = best.shape + 1;  // 0 when the default rule won
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->default_us = base_us;
    report->best_us = best_us;
    report->evaluations = evals;
  }
  return ok();
}

}  // extern "C"
