// A single-source solve that allocates nothing: every buffer of the solve
// beyond the caller's graph and output -- the instance and tick tables, the
// per-vertex state, the frontier, touched, settled, pending and pull lists,
// the heavy-chunk lists, the statistics ring and histogram, the step records
// and the work counters -- is carved out of one file-scope device array of
// fixed size. For callers that cannot call hipMalloc (code under stream
// capture, tight serving loops, harnesses that forbid allocation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "runtime.h"

namespace sssp {

// Bytes of the device array behind sssp_solve_noalloc (one per GPU, held until
// the process ends).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kNoAllocTrace = 256;  // schedule records kept (sssp_get_schedule does not see them)

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Everything the set-up kernel writes into the instance and the tick table:
// device addresses inside the scratch array and the solve's parameters.
struct NoAllocDesc {
  Globals* G;
  Inst* I;
  SegRec* seg;
  const DevGraph* g;
  uint32_t* dist;
  uint64_t* state;
  int32_t* q0;
  int32_t* q1;
  int32_t* touched;
  int32_t* settled;
  int32_t* p0;
  int32_t* p1;
  UEntry* u0;
  UEntry* u1;
  HeavyItem* h0;
  HeavyItem* h1;
  uint64_t* ring_mass;
  uint32_t* ring_cnt;
  uint32_t* hist;
  StepRec* steprec;
  TraceRec* trace;
  Counters* cslot;
  unsigned long long tick_limit;
  double beta;
  int32_t source, n, maxw, heavy_cap, trace_cap, heavy_split, fuse_cap, pad0;
  uint32_t ring_mask, steprec_mask, alpha, topt, mode, pad;
  int32_t round_batch, settle_batch;
};

// Lays the buffers of one solve out in the array from `base` on, each on a
// 256-byte boundary; with base = 0 it only measures.
struct Carve {
  unsigned char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

__global__ void __launch_bounds__(kBlock) k_noalloc_setup(NoAllocDesc d) {
  // the array keeps the previous call's contents: start from zero
  uint32_t* gz = reinterpret_cast<uint32_t*>(d.G);
  for (size_t i = threadIdx.x; i < sizeof(Globals) / 4; i += kBlock) gz[i] = 0;
  uint32_t* iz = reinterpret_cast<uint32_t*>(d.I);
  for (size_t i = threadIdx.x; i < sizeof(Inst) / 4; i += kBlock) iz[i] = 0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  Inst& I = *d.I;
  I.g = d.g;
  I.gc = *d.g;
  I.dist = d.dist;
  I.parent = nullptr;
  I.best = nullptr;
  I.mode = d.mode;
  I.state = d.state;
  I.q[0] = d.q0;
  I.q[1] = d.q1;
  I.touched = d.touched;
  I.settled = d.settled;
  I.plist[0] = d.p0;
  I.plist[1] = d.p1;
  I.ulist[0] = d.u0;
  I.ulist[1] = d.u1;
  I.heavy[0] = d.h0;
  I.heavy[1] = d.h1;
  I.ring_mass = d.ring_mass;
  I.ring_cnt = d.ring_cnt;
  I.hist_cnt = d.hist;
  I.steprec = d.steprec;
  I.trace = d.trace;
  I.cslot = d.cslot;
  I.maxw = d.maxw;
  I.heavy_cap = d.heavy_cap;
  I.ring_mask = d.ring_mask;
  I.steprec_mask = d.steprec_mask;
  I.trace_cap = d.trace_cap;
  I.source = d.source;
  I.target = -1;
  I.n = d.n;
  I.alpha = d.alpha;
  I.traversal_opt = d.topt;
  I.beta = d.beta;
  I.heavy_split = d.heavy_split;
  I.fuse_cap = d.fuse_cap;
  I.phase = PH_DONE;
  Globals& G = *d.G;
  G.ninst = 1;
  G.tick_limit = d.tick_limit;
  G.tick_log = nullptr;
  G.tick_log_cap = 0;
  G.seg = d.seg;
  G.insts = d.I;
  G.sel_list = nullptr;
  G.n_sel = -1;
  G.round_batch = d.round_batch;
  G.settle_batch = d.settle_batch;
}

struct DeviceScratch {
  bool ready = false;
  unsigned char* ptr = nullptr;  // the array's address on that device
  int cus = 0;
  int occ[kNumShapes] = {};      // workgroups per CU of each tile shape's engine kernel
};
constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
DeviceScratch g_na[kMaxDevices];

}  // namespace
}  // namespace sssp

using namespace sssp;

extern "C" sssp_status sssp_solve_noalloc(const sssp_graph* g, int32_t source, uint32_t* dist_out,
                                          hipStream_t stream) {
  std::string err;
  if (!check_graph(g, &err)) return fail(SSSP_E_INVAL, err);
  if (source < 0 || source >= g->gh.h.n) return fail(SSSP_E_INVAL, "source out of range");
  if (!dist_out) return fail(SSSP_E_INVAL, "dist_out is NULL");
  const int dev = g->gh.device;
  if (dev < 0 || dev >= kMaxDevices) return fail(SSSP_E_RANGE, "device index beyond the library's table");
  DeviceScratch ds;
  {
    std::lock_guard<std::mutex> lk(g_na_mu);
    DeviceScratch& e = g_na[dev];
    if (!e.ready) {
      // once per device, with that device current (the graph's, checked above):
      // the array's name is a host-side stand-in, its address comes from here
      void* p = nullptr;
      HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      hipDeviceProp_t prop;
      HIP_TRY(hipGetDeviceProperties(&prop, dev));
      e.ptr = static_cast<unsigned char*>(p);
      e.cus = prop.multiProcessorCount;
      for (int sh = 0; sh < kNumShapes; ++sh) e.occ[sh] = engine_blocks_per_cu(sh);
      e.ready = true;
    }
    ds = e;
  }
  const DevGraph& h = g->gh.h;
  Opts o;
  const sssp_graph* gg[1] = {g};
  const int shape = resolve_shape(o, gg, 1);  // the tile shape sssp_solve takes for this graph
  const int maxw = ds.cus * ds.occ[shape] * (kBlock / kWave);
  Needs nd = needs_for(h, maxw);
  nd.trace = kNoAllocTrace;
  Carve c{ds.ptr};
  NoAllocDesc d;
  std::memset(&d, 0, sizeof(d));
  d.G = c.take<Globals>(1);
  d.I = c.take<Inst>(1);
  d.seg = c.take<SegRec>((size_t)kMaxSegPerInst + 1);
  d.state = c.take<uint64_t>((size_t)nd.n);
  d.q0 = c.take<int32_t>((size_t)nd.list);
  d.q1 = c.take<int32_t>((size_t)nd.list);
  d.touched = c.take<int32_t>((size_t)nd.list);
  d.settled = c.take<int32_t>((size_t)nd.n);
  d.p0 = c.take<int32_t>((size_t)nd.n);
  d.p1 = c.take<int32_t>((size_t)nd.n);
  d.u0 = c.take<UEntry>((size_t)nd.list);
  d.u1 = c.take<UEntry>((size_t)nd.list);
  d.h0 = c.take<HeavyItem>((size_t)nd.heavy);
  d.h1 = c.take<HeavyItem>((size_t)nd.heavy);
  d.ring_mass = c.take<uint64_t>(nd.ring);
  d.ring_cnt = c.take<uint32_t>(nd.ring);
  d.hist = c.take<uint32_t>((size_t)nd.hist);
  d.steprec = c.take<StepRec>(nd.steprec);
  d.trace = c.take<TraceRec>((size_t)nd.trace);
  d.cslot = c.take<Counters>((size_t)maxw);
  if (c.off > kScratchBytes)
    return fail(SSSP_E_RANGE, "this graph needs " + std::to_string(c.off) + " bytes of solver scratch; "
                "sssp_solve_noalloc holds " + std::to_string(kScratchBytes));
  d.g = g->gh.d;
  d.dist = dist_out;
  d.tick_limit = o.tick_limit;
  d.beta = o.beta;
  d.source = source;
  d.n = h.n;
  d.maxw = maxw;
  d.heavy_cap = nd.heavy;
  d.trace_cap = nd.trace;
  d.heavy_split = o.heavy;
  d.fuse_cap = o.fuse;
  d.ring_mask = nd.ring - 1;
  d.steprec_mask = nd.steprec - 1;
  d.alpha = o.alpha;
  d.topt = o.topt;
  d.mode = h.float_w ? 2u : 0u;
  d.round_batch = round_batch_of(shape);
  d.settle_batch = settle_batch_of(shape);
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(kBlock), 0, stream, d);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_init(d.G, h.n, stream));
  // the persistent grid of sssp_solve: every CU's occupancy, fewer workgroups
  // for small graphs (a multiple of the XCD count)
  const int rb = round_batch_of(shape);
  long long need = ((long long)h.n + rb - 1) / rb;
  need = ((need + kMaxXcd - 1) / kMaxXcd) * kMaxXcd;
  need = std::max<long long>(need, kMaxXcd);
  const int grid = (int)std::min<long long>((long long)ds.cus * ds.occ[shape], need);
  HIP_TRY(launch_engine(d.G, grid, true, 0, stream, shape));
  HIP_TRY(launch_overflow_check(d.G, h.n, stream));
  HIP_TRY(launch_finish(d.G, h.n, stream));
  return ok();
}
