// Solver engine: the heuristic SSSP algorithm of Yu, Wang and Luo (Section 3.3,
// the Algorithm with Function 1 initFrontiers and Function 2 computeST) on one
// gfx950 GPU.
//
// Execution model. A solve (or a batch of independent solves, "instances") is
// a sequence of device-wide ticks. A tick is either a push round of one or
// more instances (Algorithm, the while loop) or a settle pass that closes a
// step (statistics for the next pair). Ticks are separated by a grid barrier;
// the last workgroup to arrive runs a short serial epilogue (phase
// transitions and the next tick's work layout) before releasing the others.
// The same tick body runs either inside one persistent cooperative launch or
// as one launch per tick.
//
// Work of a tick is a list of segments (instance, kind, item count); items are
// cut into fixed batches and batches are dealt round-robin to the tick's
// participating workgroups (a per-XCD quota: ticks with little work run on few
// workgroups, the others wait aside).
//
// Relaxations are asynchronous within a round (a 64-bit atomicMin on the
// vertex's (distance, round) word; every relaxation's result is a real path
// length, so any interleaving reaches the exact distances). The per-step
// schedule <lb, ub, st> depends only on the settled set and is therefore
// deterministic.
#include "engine.h"

#include <cstring>

namespace sssp {

// ------------------------------------------------------------ wave helpers --

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    uint32_t y = __shfl_xor(x, o, kWave);
    x = y < x ? y : x;
  }
  return x;
}

__device__ __forceinline__ int lower_bound_key(const SSSP_GBL uint64_t* __restrict__ adj, int lo, int hi,
                                               uint64_t key) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (adj[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// First index in [lo, re) whose key is >= key. The next kProbe entries (one
// or two cache lines) are read at once first; a binary search handles the rest.
constexpr int kProbe = 8;
__device__ __forceinline__ int range_end(const SSSP_GBL uint64_t* __restrict__ adj, int lo, int re, uint64_t key) {
  const int lim = min(re, lo + kProbe);
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < kProbe; ++i)
    if (lo + i < lim) cnt += adj[lo + i] < key ? 1 : 0;
  if (lo + cnt < lim || lim == re) return lo + cnt;
  return lower_bound_key(adj, lim, re, key);
}

__device__ __forceinline__ bool is_hub(GDevGraph& g, int v) {
  return (gbl(g.hub_bits)[v >> 5] >> (v & 31)) & 1u;
}

// --------------------------------------------------------- block helpers --

template <typename T>
__device__ T block_excl_scan(T x, T* sh /* kBlock/kWave + 1 */, T* total) {
  const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
  T incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) sh[wid] = incl;
  __syncthreads();
  if (tid == 0) {
    T run = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      T t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[kBlock / kWave] = run;
  }
  __syncthreads();
  T res = sh[wid] + incl - x;
  *total = sh[kBlock / kWave];
  __syncthreads();
  return res;
}

// The sum of a distance and a weight: integers, or binary32 values held as
// bit patterns (rounded to nearest, as the CPU reference rounds).
template <bool kFloat>
__device__ __forceinline__ uint32_t dadd(uint32_t a, uint32_t b) {
  if (kFloat) return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
  return a + b;
}

// ---------------------------------------------------------- the heuristic --
// Eq. (1)-(3) and Eq. (4)-(6) in IEEE double, operation order fixed, no fused
// multiply-add (the file is compiled with -ffp-contract=off).

__device__ uint32_t gap_of(unsigned long long S, uint32_t h, int32_t nnz, uint32_t M,
                           const SSSP_GBL uint32_t* rtow, uint32_t alpha, double beta) {
  uint32_t g;
  if (h <= alpha) {
    g = M;
  } else {
    unsigned long long other = (unsigned long long)nnz - S;
    unsigned long long mx = S > other ? S : other;
    double p = (double)mx / (double)nnz;          // Eq. (1)
    if (beta < p) p = beta;
    double ph = p * (double)h;
    double r = 1.0 - pow(1.0 - p, 1.0 / ph);      // Eq. (2)
    double xr = r * (double)(kRatioNum - 1);
    long long idx = (long long)ceil(xr);
    if (idx < 0) idx = 0;
    if (idx > kRatioNum - 1) idx = kRatioNum - 1;
    g = rtow[idx];                                // Eq. (3): maxW(G, ratio)
  }
  return g < 1u ? 1u : g;
}

__device__ __forceinline__ double profit_of(uint32_t x, uint32_t L, unsigned long long Y,
                                            unsigned long long S, unsigned long long Sx,
                                            uint32_t M, int32_t nnz) {
  // x is within [L - M, L), so lb_0 = x (Section 3.2 clamps)
  unsigned long long ub0 = (unsigned long long)L + M;
  if (Y < ub0) ub0 = Y;
  unsigned long long ub1 = (unsigned long long)x + M;
  if (Y < ub1) ub1 = Y;
  double pushed = (double)(ub0 - L) * (double)(Sx - S) / (double)M;  // Eq. (4)
  double pulled = (double)(ub1 - x) * (double)S / (double)M;        // Eq. (5)
  double lng = pulled * (double)(Sx - S) / (double)nnz;             // Eq. (6)
  return (pushed - lng) - pulled;
}

struct HeurLds {
  unsigned long long scan[kBlock / kWave + 1];
  unsigned long long key[kBlock];
  double pbest[kBlock];
  uint32_t xbest[kBlock];
};

// highD over a degree histogram (distinct degrees deg_vals[0..D) ascending,
// cnt[r] vertices each): the threshold h minimising |mass(deg < h) -
// mass(deg >= h)|, smallest on ties, 0 if no mass. Whole workgroup.
__device__ uint32_t block_high_d(const SSSP_GBL int32_t* deg_vals, const SSSP_GBL uint32_t* cnt, int32_t D,
                                 unsigned long long* mass_total, unsigned long long* count_total,
                                 HeurLds& L) {
  const int tid = threadIdx.x;
  const int chunk = (D + kBlock - 1) / kBlock;
  const int r0 = min(D, tid * chunk), r1 = min(D, r0 + chunk);
  unsigned long long local = 0, lcount = 0;
  for (int r = r0; r < r1; ++r) {
    local += (unsigned long long)deg_vals[r] * cnt[r];
    lcount += cnt[r];
  }
  (void)block_excl_scan<unsigned long long>(lcount, L.scan, count_total);
  unsigned long long total;
  unsigned long long low = block_excl_scan<unsigned long long>(local, L.scan, &total);
  // best (diff, r) packed: diff < 2^33, r < 2^31 -> key = diff << 31 | r
  unsigned long long best = ~0ull;
  for (int r = r0; r < r1; ++r) {
    uint32_t c = cnt[r];
    if (c) {
      long long dif = 2ll * (long long)low - (long long)total;
      if (dif < 0) dif = -dif;
      unsigned long long k = ((unsigned long long)dif << 31) | (unsigned long long)r;
      if (k < best) best = k;
      low += (unsigned long long)deg_vals[r] * c;
    }
  }
  L.key[tid] = best;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s && L.key[tid + s] < L.key[tid]) L.key[tid] = L.key[tid + s];
    __syncthreads();
  }
  unsigned long long b = L.key[0];
  __syncthreads();
  *mass_total = total;
  if (b == ~0ull) return 0;
  return (uint32_t)deg_vals[b & 0x7fffffffull];
}

// Function 2 (computeST) for the next pair <L, L + gap(L)>. Whole workgroup.
__device__ uint32_t block_compute_st(const GInst& I, uint32_t L, uint32_t gapL, int32_t nnz,
                                     HeurLds& lds) {
  const uint32_t M = I.M;
  const unsigned long long S = I.S.v;
  if (!I.traversal_opt || M > kRingMax) return L;
  if (2ull * S >= (unsigned long long)nnz || I.gap_cur == M) return L;
  if (gapL == M) return L > M ? L - M : 0u;
  const uint32_t wlo = L > M ? L - M : 0u;
  const uint32_t W = L - wlo;
  unsigned long long Y = (unsigned long long)L + gapL;
  if (Y > kInf) Y = kInf;
  const int tid = threadIdx.x;
  const uint32_t chunk = (W + kBlock - 1) / kBlock;
  // thread t owns x in [wlo + a, wlo + b), ascending
  const uint32_t a = min(W, (uint32_t)tid * chunk), b = min(W, a + chunk);
  unsigned long long local = 0;
  for (uint32_t k = a; k < b; ++k) local += gbl(I.ring_mass)[(wlo + k) & I.ring_mask];
  unsigned long long total;
  unsigned long long before = block_excl_scan<unsigned long long>(local, lds.scan, &total);
  // mass at or above the end of my chunk: total - before - local
  unsigned long long acc = total - before - local;
  double bp = 0.0;
  uint32_t bx = L;
  for (uint32_t k = b; k > a; --k) {
    uint32_t x = wlo + k - 1;
    uint32_t slot = x & I.ring_mask;
    acc += gbl(I.ring_mass)[slot];
    if (gbl(I.ring_cnt)[slot]) {
      double p = profit_of(x, L, Y, S, S + acc, M, nnz);
      // ascending order, first strict maximum: prefer larger p, then smaller x
      if (p > bp || (p == bp && p > 0.0 && x < bx)) {
        bp = p;
        bx = x;
      }
    }
  }
  lds.pbest[tid] = bp;
  lds.xbest[tid] = bx;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      double p2 = lds.pbest[tid + s];
      uint32_t x2 = lds.xbest[tid + s];
      if (p2 > lds.pbest[tid] || (p2 == lds.pbest[tid] && p2 > 0.0 && x2 < lds.xbest[tid])) {
        lds.pbest[tid] = p2;
        lds.xbest[tid] = x2;
      }
    }
    __syncthreads();
  }
  uint32_t res = lds.pbest[0] > 0.0 ? lds.xbest[0] : L;
  __syncthreads();
  return res;
}

// The selection-threshold grid (Section 4.1: ST_NUM candidates per span),
// used for binary32 distances and for integer weights too large for the
// exact window: bin(d) = floor(value(d) * kStNum / maxW), evaluated in double,
// so it never decreases as d grows; kNoBin past 2^31 bins, for +inf and for
// the sentinel. value() is the binary32 value of the bit pattern, or the
// integer itself.
// Which candidate set computeST scores (Section 4.1): the ST_NUM grid for
// binary32 weights and, by default, for integer weights above ST_NUM (where a
// grid bin is wider than one distance unit and the grid has fewer candidates
// than the exact window); below, each bin holds at most one integer distance
// and the exact window of distinct settled distances is scored instead.
// st_grid = 1 asks for the grid always, -1 for the window while it fits.
__device__ __forceinline__ bool use_st_grid(bool fw, uint32_t M, int32_t st_grid) {
  if (fw || M > kRingMax) return true;
  if (st_grid != 0) return st_grid > 0;
  return M > (uint32_t)kStNum;
}

__device__ __forceinline__ double dval(uint32_t d, bool fw) {
  return fw ? (double)__uint_as_float(d) : (double)d;
}

__device__ __forceinline__ uint32_t dinf(bool fw) { return fw ? 0x7f800000u : kInf; }

__device__ __forceinline__ double grid_inv(uint32_t M, bool fw) {
  return (double)kStNum / dval(M, fw);
}

__device__ __forceinline__ uint32_t gbin(uint32_t d, double inv, bool fw) {
  if (d >= dinf(fw)) return kNoBin;
  const double x = dval(d, fw) * inv;
  return x < 2147483648.0 ? (uint32_t)x : kNoBin;
}

// Eq. 4-6 with real-valued ends: x is a grid point at or above about L - M
// (the clamp lb_0 = max(x, L - M) changes no term there, since x + M and
// L - M + M both stay at or below L < Y).
__device__ __forceinline__ double profit_of_f(double x, double L, double Y, unsigned long long S,
                                              unsigned long long Sx, double M, int32_t nnz) {
  double ub0 = L + M;
  if (Y < ub0) ub0 = Y;
  double ub1 = x + M;
  if (Y < ub1) ub1 = Y;
  double pushed = (ub0 - L) * (double)(Sx - S) / M;   // Eq. (4)
  double pulled = (ub1 - x) * (double)S / M;          // Eq. (5)
  double lng = pulled * (double)(Sx - S) / (double)nnz;  // Eq. (6)
  return (pushed - lng) - pulled;
}

// Function 2 (computeST) over the grid. The candidates are the grid points
// (kStNum per maxW) whose bin holds a settled vertex and has no key below
// lb0 = L - M; each is scored by Eq. 4-6 at the
// grid point with the settled mass of its bin and the bins above it. The
// threshold returned for the winning bin is the smallest key (binary32 bit
// pattern, or integer) in it, so that dist >= st holds exactly for the
// vertices of that bin and above. Whole workgroup.
__device__ uint32_t block_compute_st_grid(const GInst& I, uint32_t L, uint32_t gapL, uint32_t lb0,
                                          uint32_t ubn, int32_t nnz, bool fw, HeurLds& lds) {
  const uint32_t M = I.M;
  const unsigned long long S = I.S.v;
  if (!I.traversal_opt || M == 0u || L >= dinf(fw)) return L;
  if (2ull * S >= (unsigned long long)nnz || I.gap_cur == M) return L;
  if (gapL == M) return lb0;
  const double inv = grid_inv(M, fw);
  const uint32_t kL = gbin(L, inv, fw);
  if (kL == kNoBin) return L;
  // the first bin whose smallest key is at least lb0
  const uint32_t klo = lb0 == 0u ? 0u : gbin(lb0 - 1u, inv, fw) + 1u;
  if (klo > kL) return L;
  const uint32_t W = kL - klo + 1u;
  const double Mf = dval(M, fw);
  const double Lf = dval(L, fw);
  const double Y = ubn >= dinf(fw) ? __builtin_huge_val() : dval(ubn, fw);
  const double delta = Mf / (double)kStNum;
  const int tid = threadIdx.x;
  const uint32_t chunk = (W + kBlock - 1) / kBlock;
  // thread t owns bins klo + [a, b), ascending
  const uint32_t a = min(W, (uint32_t)tid * chunk), b = min(W, a + chunk);
  unsigned long long local = 0;
  for (uint32_t k = a; k < b; ++k) local += gbl(I.ring_mass)[(klo + k) & I.ring_mask];
  unsigned long long total;
  unsigned long long before = block_excl_scan<unsigned long long>(local, lds.scan, &total);
  unsigned long long acc = total - before - local;
  double bp = 0.0;
  uint32_t bx = kNoBin;
  for (uint32_t k = b; k > a; --k) {
    const uint32_t x = klo + k - 1;
    const uint32_t slot = x & I.ring_mask;
    acc += gbl(I.ring_mass)[slot];
    if (gbl(I.ring_cnt)[slot]) {
      double p = profit_of_f((double)x * delta, Lf, Y, S, S + acc, Mf, nnz);
      if (p > bp || (p == bp && p > 0.0 && x < bx)) {
        bp = p;
        bx = x;
      }
    }
  }
  lds.pbest[tid] = bp;
  lds.xbest[tid] = bx;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      double p2 = lds.pbest[tid + s];
      uint32_t x2 = lds.xbest[tid + s];
      if (p2 > lds.pbest[tid] || (p2 == lds.pbest[tid] && p2 > 0.0 && x2 < lds.xbest[tid])) {
        lds.pbest[tid] = p2;
        lds.xbest[tid] = x2;
      }
    }
    __syncthreads();
  }
  uint32_t res = L;
  if (lds.pbest[0] > 0.0) {
    // smallest key in bin kb (bin(L) = kL >= kb, so within [0, L])
    const uint32_t kb = lds.xbest[0];
    uint32_t lo = 0u, hi = L;
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (gbin(mid, inv, fw) >= kb) hi = mid; else lo = mid + 1u;
    }
    res = lo;
  }
  __syncthreads();
  return res;
}

// The end-of-step heuristic for one instance: statistics at L = ub, gap(L),
// computeST, step bookkeeping, termination test, and the next step's setup.
// Runs on one workgroup, after every settle batch of the instance is done.
__device__ __noinline__ void run_heuristic(GInst& I, HeurLds& lds) {
  GDevGraph& g = I.gc;
  const int tid = threadIdx.x;
  const uint32_t L = I.ub;
  unsigned long long mass;
  unsigned long long unsettled;  // vertices of degree >= 1 with dist >= L
  uint32_t h = block_high_d(gbl(g.deg_vals), gbl(I.hist_cnt), g.num_deg, &mass, &unsettled, lds);
  const unsigned long long S = I.S.v;
  uint32_t gapL = gap_of(S, h, g.nnz, I.M, gbl(g.rtow), I.alpha, I.beta);
  const bool fw = g.float_w != 0;
  unsigned long long ubn;
  uint32_t lb0;
  if (fw) {
    // The next band ends at L + gap (Section 3.3), rounded. The gap is
    // positive (Section 3.1 keeps it in (0, maxW]): a zero weight quantile
    // takes the smallest positive weight, as the integer gap takes 1, and
    // where L + gap rounds back to L the band still ends above L (the next
    // threshold is greater than the current one, Section 3). Infinity and
    // beyond are the +inf sentinel.
    const uint32_t gf = gapL > g.min_pos_w || g.min_pos_w == kInf ? gapL : g.min_pos_w;
    uint32_t e = dadd<true>(L, gf);
    if (e <= L) e = L + 1u;
    ubn = e >= 0x7f800000u ? (unsigned long long)kInf : (unsigned long long)e;
    // lb0 = L - M, lowered by two units in the last place of L: a settled
    // distance d whose rounded d + M still reaches L lies above it
    const float ulp = __uint_as_float(L + 1u) - __uint_as_float(L);
    const float lo = (__uint_as_float(L) - __uint_as_float(I.M)) - 2.0f * ulp;
    lb0 = lo > 0.0f ? __float_as_uint(lo) : 0u;
  } else {
    ubn = (unsigned long long)L + gapL;
    if (ubn > kInf) ubn = kInf;
    lb0 = L > I.M ? L - I.M : 0u;
  }
  // binary32 weights, or integer weights beyond the exact window: computeST
  // scores the points of the ST_NUM grid
  const bool grid = use_st_grid(fw, I.M, I.st_grid);
  uint32_t stn = grid ? block_compute_st_grid(I, L, gapL, lb0, (uint32_t)ubn, g.nnz, fw, lds)
                      : block_compute_st(I, L, gapL, g.nnz, lds);
  if (tid == 0) {
    if (mass != S) I.flags.v |= FLAG_MASS;
    StepRec rec;
    rec.lb = I.lb;
    rec.ub = L;
    rec.seg_begin = I.settled_mark;
    rec.seg_end = min(I.settled_cnt.v, I.n);
    gstore(gbl(I.steprec) + ((uint32_t)I.nsteprec & I.steprec_mask), rec);
    I.nsteprec += 1;
    if (I.trace_len < I.trace_cap) {
      TraceRec t;
      t.lb = I.lb; t.ub = L; t.st = I.st; t.rounds = I.rounds_in_step;
      t.pulled = I.pull_on; t.L = L; t.S = S; t.h = h; t.gap = gapL; t.st_next = stn; t.pad = 0;
      gstore(gbl(I.trace) + I.trace_len, t);
    }
    I.trace_len += 1;
    I.c.steps += 1;
  }
  // a point-to-point query (Section 5 lists them among the method's uses)
  // ends once its target is settled: every distance below L is final now
  const bool beyond = fw ? dadd<true>(I.max_settled.v, I.M) < L
                        : (unsigned long long)I.max_settled.v + I.M < L;
  const bool done = (L == kInf) || (I.p_next_cnt.v == 0 && beyond) ||
                    (I.tgt_in >= 0 && (uint32_t)(gbl(I.state)[I.tgt_in] >> 32) < L);
  if (done) {
    if (tid == 0) I.phase = PH_DONE;
    __syncthreads();
    return;
  }
  // clear the ring slots of the next band [L, ubn) before its settle pass;
  // on the grid: the bins after bin(L) up to bin(ubn) (bin(L) may already
  // hold settled vertices below L)
  uint32_t width, key0;
  if (grid) {
    const double inv = grid_inv(I.M, fw);
    const uint32_t kl = gbin(L, inv, fw), ku = gbin((uint32_t)ubn, inv, fw);
    const bool ok = kl != kNoBin && ku != kNoBin;
    width = ok ? ku - kl : 0u;
    key0 = kl + 1u;
  } else {
    width = (uint32_t)(ubn - L);
    key0 = L;
  }
  const uint32_t clr = width > I.ring_mask + 1 ? I.ring_mask + 1 : width;
  for (uint32_t k = tid; k < clr; k += kBlock) {
    uint32_t slot = (key0 + k) & I.ring_mask;
    gbl(I.ring_mass)[slot] = 0;
    gbl(I.ring_cnt)[slot] = 0;
  }
  // The settled-list range holding every vertex settled with dist in [lb0,
  // st]: from the first step record with ub > lb0 to the last with lb <= st
  // (records are ordered by band). Both ends usually lie among the newest
  // records: the newest kBlock are tested at once, one per thread; a bisection
  // over the older ones runs only when an end lies beyond them.
  __shared__ int32_t s_r0, s_r1;
  const int32_t nrec = I.nsteprec;
  const int32_t avail = nrec < (int32_t)(I.steprec_mask + 1) ? nrec : (int32_t)(I.steprec_mask + 1);
  const int32_t first = nrec - avail;  // oldest record still held
  const int32_t w0 = max(first, nrec - kBlock);
  if (tid == 0) {
    s_r0 = nrec;
    s_r1 = w0 - 1;
  }
  __syncthreads();
  {
    const int32_t i = nrec - 1 - tid;
    if (i >= w0) {
      const StepRec rec = gload(gbl(I.steprec) + ((uint32_t)i & I.steprec_mask));
      if (rec.ub > lb0) atomicMin(&s_r0, i);
      if (rec.lb <= stn) atomicMax(&s_r1, i);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int32_t r0 = s_r0, r1 = s_r1;
    if (r0 == w0 && w0 > first) {
      // first record with ub > lb0 among the older ones (w0 has it)
      int32_t lo = first, hi = w0;
      while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (gbl(I.steprec)[(uint32_t)mid & I.steprec_mask].ub > lb0) hi = mid; else lo = mid + 1;
      }
      r0 = lo;
    }
    if (r1 < w0 && w0 > first) {
      // last record with lb <= st among the older ones (w0 lacks it)
      int32_t lo = first, hi = w0;
      while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (gbl(I.steprec)[(uint32_t)mid & I.steprec_mask].lb <= stn) lo = mid + 1; else hi = mid;
      }
      r1 = lo - 1;
    }
    int32_t wb = 0, we = 0;
    if (r0 <= r1 && r0 < nrec && r1 >= first) {
      wb = gbl(I.steprec)[(uint32_t)r0 & I.steprec_mask].seg_begin;
      we = gbl(I.steprec)[(uint32_t)r1 & I.steprec_mask].seg_end;
      if (r0 == first && first > 0) wb = 0;  // older records evicted: scan from the start
    }
    I.wBegin = wb;
    I.wEnd = we;
    I.lb = L;
    I.ub = (uint32_t)ubn;
    I.st = stn;
    I.lb0 = lb0;
    I.pull_on = stn < L ? 1u : 0u;
    if (I.pull_on) {
      // the entries able to pull (smallest weight < ub - st) not read by an
      // earlier pull: up to the first weight bucket starting at or above
      // ub - st
      const unsigned long long bw = g.ubucket_width;
      unsigned long long j;
      if (fw) {
        // two buckets: the second holds lightest weights >= bw, which pull
        // only if st + bw, rounded, is below ub
        static_assert(kUBuckets == 2, "binary32 pull-list end assumes two buckets");
        j = dadd<true>(stn, (uint32_t)bw) < (uint32_t)ubn ? (unsigned long long)kUBuckets : 1ull;
      } else {
        const unsigned long long reach = ubn - stn;
        j = (reach + bw - 1) / bw;
      }
      const int32_t e = gbl(g.ufirst)[j < (unsigned long long)kUBuckets ? j : kUBuckets];
      I.u_end = e > I.u_done ? e : I.u_done;
      I.c.pull_unsettled += unsettled;
    }
    I.gap_cur = gapL;
    I.first = 0;
    I.step += 1;
    I.rounds_in_step = 0;
    I.step_rid0 = I.rid + 1;
    I.rid = I.step_rid0 + 1;
    I.phase = PH_ROUND;
    if (I.pull_on) I.c.pulls += 1;
  }
  __syncthreads();
}

// ------------------------------------------------------------ tick: rounds --

// The phase bodies below are kept out of line: inlined together they need
// more than twice the registers of the largest one, which halves occupancy.

// Everything a batch needs from its instance, read once into registers: the
// control words only change between ticks, and reading them through the
// instance struct inside the loops would re-load them after every atomic.
struct View {
  const SSSP_GBL int32_t* rowptr;
  const SSSP_GBL uint64_t* adj;
  const SSSP_GBL uint32_t* wmin;
  const SSSP_GBL uint32_t* hub_bits;
  const SSSP_GBL int32_t* rwi;
  SSSP_GBL uint64_t* state;
  SSSP_GBL int32_t* q_next;
  SSSP_GBL int32_t* touched;
  SSSP_GBL uint64_t* best;  // null: no tree
  GInst* inst;
  uint32_t lb, ub, st, lb0, rid, step_rid0;
  int32_t n, heavy_split, maxw;
  uint32_t first;
  uint32_t rwi_width;
};

__device__ __forceinline__ View make_view(GInst& I) {
  View v;
  GDevGraph& g = I.gc;
  v.rowptr = gbl(g.rowptr);
  v.adj = gbl(g.adj);
  v.wmin = gbl(g.wmin);
  v.hub_bits = gbl(g.hub_bits);
  v.rwi = gbl(g.rwi);
  v.rwi_width = g.rwi_width;
  v.state = gbl(I.state);
  v.q_next = gbl(I.q[I.qsel ^ 1]);
  v.touched = gbl(I.touched);
  v.best = I.best ? gbl(I.best) : nullptr;
  v.inst = &I;
  v.lb = I.lb;
  v.ub = I.ub;
  v.st = I.st;
  v.lb0 = I.lb0;
  v.rid = I.rid;
  v.step_rid0 = I.step_rid0;
  v.n = I.n;
  v.heavy_split = I.heavy_split;
  v.maxw = I.maxw;
  v.first = I.first;
  return v;
}

// The tentative distance of v (the high half of its state word).
__device__ __forceinline__ uint32_t dist_of(const SSSP_GBL uint64_t* state, int v) {
  return ((const SSSP_GBL uint32_t*)state)[2 * v + 1];
}

// Lower v's distance to c in round rid. Returns the previous state word; the
// decrease happened iff c is below its distance.
__device__ __forceinline__ uint64_t relax_state(SSSP_GBL uint64_t* state, int v, uint32_t c, uint32_t rid) {
  return atomicMin(reinterpret_cast<SSSP_GBL unsigned long long*>(state + v),
                   ((unsigned long long)c << 32) | (unsigned long long)rid);
}

struct WaveAcc {
  unsigned long long expansions, band, pscan, pvert, pullscan, success, qent;
  uint32_t hubmin;
};

// The work counters of a workgroup, gathered in LDS for one instance at a
// time and written to that instance's slot for this workgroup (no other
// workgroup adds to it) when the workgroup turns to another instance or the
// kernel ends: the batches themselves issue no counter atomics to memory.
struct WgAcc {
  unsigned long long v[7];  // expansions, band, push, pull vertices, pull entries, successes, queue
  int inst;                 // instance the values belong to, -1: none
  int pad;
};
static_assert(offsetof(Counters, band_expansions) == 8 && offsetof(Counters, push_scanned) == 16 &&
                  offsetof(Counters, pull_vertices) == 24 && offsetof(Counters, pull_scanned) == 32 &&
                  offsetof(Counters, relax_success) == 40 && offsetof(Counters, queue_entries) == 48,
              "the gathered counters follow Counters' order");
__shared__ WgAcc g_wgacc;

// Thread 0: write the gathered counters to their instance's slot and start over.
__device__ void wgacc_flush(GGlobals& G) {
  const int i = g_wgacc.inst;
  if (i >= 0) {
    GInst& I = gbl(G.insts)[i];
    if ((int)blockIdx.x < I.maxw) {
      SSSP_GBL unsigned long long* c = &gbl(I.cslot)[blockIdx.x].expansions;
      // Counters keeps the same order as v[]
      for (int k = 0; k < 7; ++k)
        if (g_wgacc.v[k]) atomicAdd(c + k, g_wgacc.v[k]);  // no returned value: nothing waits
    }
  }
  for (int k = 0; k < 7; ++k) g_wgacc.v[k] = 0;
  g_wgacc.inst = -1;
}

// Thread 0, before a batch of instance i: the gathered counters must be i's.
__device__ __forceinline__ void wgacc_select(GGlobals& G, int i) {
  if (g_wgacc.inst != i) {
    wgacc_flush(G);
    g_wgacc.inst = i;
  }
}

// The wave's counters go to the workgroup's gathered ones; the step-1 hub
// bound is a shared atomic.
__device__ __forceinline__ void flush_acc(GInst& I, int maxw, WaveAcc& a) {
  (void)maxw;
  unsigned long long e = wave_sum(a.expansions), b = wave_sum(a.band), ps = wave_sum(a.pscan),
                     pv = wave_sum(a.pvert), pl = wave_sum(a.pullscan), su = wave_sum(a.success),
                     qe = wave_sum(a.qent);
  uint32_t hm = wave_min_u32(a.hubmin);
  if (lane_id() == 0) {
    if (e) atomicAdd(&g_wgacc.v[0], e);
    if (b) atomicAdd(&g_wgacc.v[1], b);
    if (ps) atomicAdd(&g_wgacc.v[2], ps);
    if (pv) atomicAdd(&g_wgacc.v[3], pv);
    if (pl) atomicAdd(&g_wgacc.v[4], pl);
    if (su) atomicAdd(&g_wgacc.v[5], su);
    if (qe) atomicAdd(&g_wgacc.v[6], qe);
    if (hm != kInf) atomicMin(&I.ub_next.v, hm);
  }
}

__device__ __forceinline__ bool hub_bit(const SSSP_GBL uint32_t* bits, int v) {
  return (bits[v >> 5] >> (v & 31)) & 1u;
}

// Appends of a workgroup batch are staged in LDS and written out with one
// device atomic per list and flush: thousands of waves claiming list slots
// on the same counter would otherwise queue behind each other.
template <int kCap>
struct StageLds {
  static constexpr int kSize = kCap;
  int32_t q[kCap];  // next frontier
  int32_t t[kCap];  // touched list (and the surviving pull list in phase 1)
  int32_t nq, nt;
  int32_t base_q, base_t;
};

// Convergent within a wave.
__device__ __forceinline__ void stage_append(int32_t* buf, int32_t* cnt, bool want, int32_t val) {
  uint64_t m = __ballot(want);
  if (m == 0) return;
  int base = 0;
  const int leader = __ffsll((unsigned long long)m) - 1;
  if (lane_id() == leader) base = atomicAdd(cnt, __popcll(m));
  base = __shfl(base, leader, kWave);
  if (want) buf[base + __popcll(m & lanemask_lt())] = val;
}

// Whole workgroup: copy the pull-list entries whose positions were staged in
// q to `dst`. Position p is entry p of `cur` for p < ncur, else entry p - ncur
// of `fresh`.
template <class St>
__device__ void stage_flush_entries(St& S, const SSSP_GBL UEntry* cur, int ncur,
                                    const SSSP_GBL UEntry* fresh, SSSP_GBL UEntry* dst,
                                    SSSP_GBL int32_t* cnt, int cap, SSSP_GBL uint32_t* flags) {
  __syncthreads();
  const int np = S.nq;
  if (threadIdx.x == 0) {
    S.base_q = np ? atomicAdd(cnt, np) : 0;
    if (S.base_q + np > cap) atomicOr(flags, FLAG_CAPACITY);
  }
  __syncthreads();
  const int b = S.base_q;
  for (int i = threadIdx.x; i < np; i += kBlock) {
    const int p = S.q[i];
    if (b + i < cap) gstore(dst + b + i, gload(p < ncur ? cur + p : fresh + (p - ncur)));
  }
  __syncthreads();
  if (threadIdx.x == 0) S.nq = 0;
  __syncthreads();
}

// Whole workgroup: copy the staged entries to their lists.
template <class St>
__device__ void stage_flush(St& S, SSSP_GBL int32_t* qlist, SSSP_GBL int32_t* qcnt, SSSP_GBL int32_t* tlist,
                            SSSP_GBL int32_t* tcnt,
                            int cap, SSSP_GBL uint32_t* flags) {
  __syncthreads();
  const int nq = S.nq, nt = S.nt;
  if (threadIdx.x == 0) {
    S.base_q = nq ? atomicAdd(qcnt, nq) : 0;
    S.base_t = nt ? atomicAdd(tcnt, nt) : 0;
    if (S.base_q + nq > cap || S.base_t + nt > cap) atomicOr(flags, FLAG_CAPACITY);
  }
  __syncthreads();
  const int bq = S.base_q, bt = S.base_t;
  for (int i = threadIdx.x; i < nq; i += kBlock)
    if (bq + i < cap) qlist[bq + i] = S.q[i];
  for (int i = threadIdx.x; i < nt; i += kBlock)
    if (bt + i < cap) tlist[bt + i] = S.t[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    S.nq = 0;
    S.nt = 0;
  }
  __syncthreads();
}

// A successful decrease of dist[t] to c by vertex src during round `rid`,
// whose previous decrease was in round `prev`: t joins the next frontier once per round
// (SAP) and the step's touched list once per step. Convergent within a wave.
template <bool kTree, class St>
__device__ __forceinline__ void on_success(const View& V, bool ok, int t, uint32_t c, uint32_t prev, int src,
                                           WaveAcc& acc, St& S) {
  bool wq = false, wt = false;
  if (ok) {
    wq = prev != V.rid;
    wt = prev < V.step_rid0;
    acc.success += 1;
    // the tree: src set dist[t] to c (a later, smaller c replaces it)
    if (kTree) atomicMin((SSSP_GBL unsigned long long*)(V.best + t), ((unsigned long long)c << 32) | (uint32_t)src);
    acc.qent += (wq ? 1 : 0) + (wt ? 1 : 0);
    if (V.first && hub_bit(V.hub_bits, t) && c < acc.hubmin) acc.hubmin = c;
  }
  stage_append(S.q, &S.nq, wq, t);
  stage_append(S.t, &S.nt, wt, t);
}

// Split a long range into heavy chunks for the next tick (grid-wide).
__device__ void emit_heavy(GInst& I, int u, uint32_t d, int lo, int hi, bool pull) {
  int nch = (hi - lo + kHeavyChunk - 1) / kHeavyChunk;
  int base = atomicAdd(&I.h_next_cnt.v, nch);
  auto out = gbl(I.heavy[I.hsel ^ 1]);
  const int cap = I.heavy_cap;
  for (int k = 0; k < nch; ++k) {
    int pos = base + k;
    if (pos >= cap) {
      atomicOr(&I.flags.v, FLAG_CAPACITY);
      break;
    }
    int a = lo + k * kHeavyChunk;
    int b = min(hi, a + kHeavyChunk);
    HeavyItem it;
    it.u = u;
    it.d = d;
    it.lo = a;
    it.hi_kind = b | (pull ? (int)0x80000000 : 0);
    gstore(out + pos, it);
  }
}

// One workgroup processes a batch of a round segment in two phases.
// Phase 1 streams the items (kItemsPerThread per thread, their loads issued
// together), applies the filters and the pending-list / pull-list
// bookkeeping, and compacts the items that have edges to relax into LDS.
// Phase 2 finds each compacted item's edge range -- the band filter
// [lb - d, ub - d) on the weight-sorted row, or the pull prefix w < ub - st --
// and relaxes all of the batch's edges with a workgroup-wide merge path.
template <class Sh>
struct RoundLds {
  int32_t u[Sh::kBatch];
  uint32_t d[Sh::kBatch];
  // pull items: best candidate for dist[u] found in this batch; with a tree
  // (candidate << 32) | the settled neighbour it comes from
  union {
    uint32_t pmin32[Sh::kBatch];
    unsigned long long pmin64[Sh::kBatch];
  };
  int32_t lo[Sh::kBatch];
  int32_t re[Sh::kBatch];  // row end when the row is known (pull-list items), else -1
  int32_t sz[Sh::kBatch];  // size, -1 = range still to find; then exclusive offsets
  uint8_t pull[Sh::kBatch];
  int32_t count;
  int32_t iscan[kBlock / kWave + 1];
  StageLds<Sh::kStage> stage;
};

template <class RL>
__device__ __forceinline__ void lds_push_item(RL& L, bool want, int u, uint32_t d, int lo,
                                              int sz, bool pull, int re = -1) {
  uint64_t m = __ballot(want);
  if (m == 0) return;
  int base = 0;
  const int leader = __ffsll((unsigned long long)m) - 1;
  if (lane_id() == leader) base = atomicAdd(&L.count, __popcll(m));
  base = __shfl(base, leader, kWave);
  if (want) {
    const int w = base + __popcll(m & lanemask_lt());
    L.u[w] = u;
    L.d[w] = d;
    L.lo[w] = lo;
    L.re[w] = re;
    L.sz[w] = sz;
    L.pull[w] = pull ? 1 : 0;
  }
}

// kTree: the instance also records a shortest-path tree (a separate
// instantiation, so that solves without one pay nothing for it).
// kFloat: binary32 weights; the band searches then test dist + w itself
// against the band ends, rounded as the relaxation rounds it.
template <bool kTree, bool kFloat, class Sh>
__device__ __noinline__ void block_round(GInst& I, int kind, int item0, int nitems, RoundLds<Sh>& L) {
  constexpr int kItemsPerThread = Sh::kItems;
  constexpr int kEdgesPerThread = Sh::kEdges;
  constexpr int kStageCap = Sh::kStage;
  const View V = make_view(I);
  const int tid = threadIdx.x;
  const uint32_t lb = V.lb, ub = V.ub, st = V.st;
  WaveAcc acc = {0, 0, 0, 0, 0, 0, 0, kInf};
  auto& S = L.stage;
  if (tid == 0) {
    L.count = 0;
    S.nq = 0;
    S.nt = 0;
  }
  __syncthreads();

  // ---------------------------------------------------------- phase 1
  if (kind == SEG_H) {
    // heavy chunks: the range is known
    const int it = item0 + tid;
    bool want = false;
    int u = 0, lo = 0, sz = 0;
    uint32_t d = 0;
    bool pull = false;
    if (tid < kHeavyPerBatch && it < nitems) {
      HeavyItem h = gload(gbl(I.heavy[I.hsel]) + it);
      u = h.u;
      lo = h.lo;
      sz = (h.hi_kind & 0x7fffffff) - lo;
      pull = (h.hi_kind & (int)0x80000000) != 0;
      const uint32_t du = dist_of(V.state, u);
      if (pull) {
        d = du;
        want = du > lb;
      } else {
        d = h.d;
        want = (du == d);  // a newer, smaller dist[u] has its own expansion
      }
    }
    lds_push_item(L, want, u, d, lo, sz, pull);
  } else if (kind == SEG_U) {
    // unsettled-list entries carry the row's smallest weight and bounds: an
    // entry whose lightest edge cannot reach below ub from a settled vertex
    // (>= st) is kept without reading its distance. The list is the compacted
    // list of earlier pulls followed by the sorted entries no pull has read yet.
    const int usel = I.usel;
    const int ncur = I.nU;
    const SSSP_GBL UEntry* ucur = gbl(I.ulist[usel]);
    const SSSP_GBL UEntry* fresh = gbl(I.gc.nonisolated) + I.u_done;
    auto unext = gbl(I.ulist[usel ^ 1]);
    const uint32_t reach = ub - st;  // integer weights
    UEntry ee[kItemsPerThread];
    bool valid[kItemsPerThread];
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      const int it = item0 + k * kBlock + tid;
      valid[k] = it < nitems;
      if (valid[k]) ee[k] = gload(it < ncur ? ucur + it : fresh + (it - ncur));
    }
    uint32_t dd[kItemsPerThread];
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      const bool cand = valid[k] && (kFloat ? dadd<true>(st, ee[k].wmin) < ub : ee[k].wmin < reach);
      dd[k] = cand ? dist_of(V.state, ee[k].id) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      const int it = item0 + k * kBlock + tid;
      const bool cand = valid[k] && (kFloat ? dadd<true>(st, ee[k].wmin) < ub : ee[k].wmin < reach);
      const bool keep = valid[k] && (!cand || dd[k] >= lb);
      const bool active = cand && dd[k] > lb;
      acc.pvert += valid[k] ? 1 : 0;
      stage_append(S.q, &S.nq, keep, it);
      lds_push_item(L, active, valid[k] ? ee[k].id : 0, dd[k], valid[k] ? ee[k].rs : 0, -1, true,
                    valid[k] ? ee[k].re : -1);
    }
    // the surviving pull list goes out now; the stage is free for phase 2
    stage_flush_entries(S, ucur, ncur, fresh, unext, &I.u_next_cnt.v, V.n, &I.flags.v);
  } else {
    int uu[kItemsPerThread];
    const SSSP_GBL int32_t* src = (kind == SEG_W) ? gbl(I.settled) + I.wBegin
                         : (kind == SEG_P) ? gbl(I.plist[I.psel]) : gbl(I.q[I.qsel]);
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      const int it = item0 + k * kBlock + tid;
      uu[k] = it < nitems ? src[it] : -1;
    }
    // the distance and the row bounds of each item in one round trip (the
    // bounds are needed by almost every item that passes the filter)
    uint32_t dd[kItemsPerThread];
    int rsk[kItemsPerThread], rek[kItemsPerThread];
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      dd[k] = uu[k] >= 0 ? dist_of(V.state, uu[k]) : kInf;
      rsk[k] = uu[k] >= 0 ? V.rowptr[uu[k]] : 0;
      rek[k] = uu[k] >= 0 ? V.rowptr[uu[k] + 1] : 0;
    }
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      const int u = uu[k];
      const uint32_t d = dd[k];
      bool ok;
      if (kind == SEG_W) ok = u >= 0 && d >= V.lb0 && d <= st;
      else ok = u >= 0 && d >= lb && d < ub;
      if (kind == SEG_P) {
        // band members of the pending list join this step's touched list
        bool wt = false;
        if (ok) {
          // raise the round id (low half of the state word) to the step's marker
          uint32_t so = atomicMax(&((SSSP_GBL uint32_t*)V.state)[2 * u], V.step_rid0);
          wt = so < V.step_rid0;
          acc.qent += wt ? 1 : 0;
        }
        stage_append(S.t, &S.nt, wt, u);
      }
      lds_push_item(L, ok, u, d, rsk[k], -1, false, rek[k]);
    }
  }
  __syncthreads();
  const int m = L.count;
  for (int w = tid; w < m; w += kBlock) {
    if (kTree) L.pmin64[w] = ~0ull;
    else L.pmin32[w] = kInf;
  }

  // ---------------------------------------------------------- phase 2a: ranges
  // An item's range is [first weight >= lo key, first weight >= hi key) of
  // its weight-sorted row (lo key lb - d for a push, 0 for a pull; hi key
  // ub - d for a push, ub - st for a pull). The row index narrows each of the
  // two searches to one weight bucket (about deg/16 entries); the bounds of
  // those buckets are loaded together with the row bounds. Then a thread's
  // eight searches (two per item) bisect in lockstep, so the loads of one step
  // are in flight together.
  {
    constexpr int K2 = 2 * kItemsPerThread;
    int wi[kItemsPerThread], rs[kItemsPerThread], re[kItemsPerThread];
    int pb[K2][2];  // bucket bounds (positions) of each search
    uint32_t key[K2];
    // binary32 weights: search x looks for the first w with base + w >= bnd
    // (push: base d, bnd lb / ub; pull: base st, bnd ub), the row index unused
    uint32_t fbase[K2], fbnd[K2];
    bool need[kItemsPerThread], leaf[kItemsPerThread];
    const uint32_t W = V.rwi_width;
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      wi[k] = tid + k * kBlock;
      need[k] = wi[k] < m && L.sz[wi[k]] < 0;  // heavy chunks come with their range
      rs[k] = re[k] = 0;
      key[2 * k] = key[2 * k + 1] = 0;
      pb[2 * k][0] = pb[2 * k][1] = pb[2 * k + 1][0] = pb[2 * k + 1][1] = 0;
      if (!need[k]) continue;
      const int u = L.u[wi[k]];
      const uint32_t d = L.d[wi[k]];
      const bool pull = L.pull[wi[k]] != 0;
      key[2 * k] = pull ? 0u : (lb > d ? lb - d : 0u);
      key[2 * k + 1] = pull ? ub - st : ub - d;
      if (kFloat) {
        key[2 * k] = (pull || lb <= d) ? 0u : 1u;  // 0: the range starts at the row start
        fbase[2 * k] = d;
        fbnd[2 * k] = lb;
        fbase[2 * k + 1] = pull ? st : d;
        fbnd[2 * k + 1] = ub;
      }
      // row bounds: carried by pull-list items, else loaded
      const int kre = L.re[wi[k]];
      const bool known = kre >= 0;
      rs[k] = known ? L.lo[wi[k]] : V.rowptr[u];
      re[k] = known ? kre : V.rowptr[u + 1];
      // the bucket bounds are loaded with the row bounds (a known short row
      // needs none)
      const bool idx = !kFloat && (!known || kre - L.lo[wi[k]] > kRowIndexMin);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // bucket b (clamped to 16: past the last boundary) spans
        // [P[b], P[b + 1]], P[b] at rwi[16 u + b - 1] for b in 1..15 (P[0] and
        // P[16] are the row ends; -1 marks "use the row end")
        const uint32_t b = min(key[2 * k + h] / W, 16u);
        const SSSP_GBL int32_t* P = V.rwi + 16ll * u;
        pb[2 * k + h][0] = (idx && b >= 1u && b <= 15u) ? P[b - 1u] : -1;
        pb[2 * k + h][1] = (idx && b <= 14u) ? P[b] : -1;
      }
    }
    int a[K2], c[K2];
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      leaf[k] = false;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a[2 * k + h] = c[2 * k + h] = rs[k];
        if (!need[k]) continue;
        const uint32_t kk = key[2 * k + h];
        const uint32_t b = min(kk / W, 16u);
        if (kFloat || re[k] - rs[k] <= kRowIndexMin) {
          a[2 * k + h] = rs[k];
          c[2 * k + h] = re[k];
        } else {
          a[2 * k + h] = b == 0u ? rs[k] : (b >= 16u ? re[k] : pb[2 * k + h][0]);
          c[2 * k + h] = b >= 15u ? re[k] : pb[2 * k + h][1];
        }
        if (h == 0 && kk == 0) c[2 * k] = a[2 * k] = rs[k];  // starts at the row start
      }
      if (need[k] && !L.pull[wi[k]]) {
        leaf[k] = (re[k] - rs[k] == 1 && L.d[wi[k]] > 0);  // leaf pruning (Algorithm)
        if (leaf[k]) a[2 * k] = c[2 * k] = a[2 * k + 1] = c[2 * k + 1] = rs[k];
      }
    }
    const SSSP_GBL uint32_t* wts = (const SSSP_GBL uint32_t*)V.adj;  // weight: high half of an entry
    // rows of at most kRowIndexMin entries: one probe of the whole row answers
    // both searches
#pragma unroll
    for (int k0 = 0; k0 < kItemsPerThread; k0 += 2) {  // two items at a time (registers)
      uint32_t pw[2][kRowIndexMin];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int k = k0 + j;
        if (k >= kItemsPerThread) break;  // an odd count: the last pair is single
        const bool small = need[k] && re[k] - rs[k] <= kRowIndexMin;
#pragma unroll
        for (int i = 0; i < kRowIndexMin; ++i)
          pw[j][i] = (small && rs[k] + i < re[k]) ? wts[2ll * (rs[k] + i) + 1] : 0xffffffffu;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int k = k0 + j;
        if (k >= kItemsPerThread) break;
        if (!(need[k] && re[k] - rs[k] <= kRowIndexMin) || leaf[k]) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (a[2 * k + h] >= c[2 * k + h]) continue;  // already decided (row start)
          int cnt = 0;
#pragma unroll
          for (int i = 0; i < kRowIndexMin; ++i) {
            if (kFloat) cnt += (pw[j][i] != 0xffffffffu && dadd<true>(fbase[2 * k + h], pw[j][i]) < fbnd[2 * k + h]) ? 1 : 0;
            else cnt += pw[j][i] < key[2 * k + h] ? 1 : 0;
          }
          a[2 * k + h] = c[2 * k + h] = rs[k] + cnt;
        }
      }
    }
    for (;;) {
      int mid[K2];
      uint32_t val[K2];
      bool any = false;
#pragma unroll
      for (int x = 0; x < K2; ++x) {
        if (a[x] < c[x]) {
          mid[x] = (a[x] + c[x]) >> 1;
          val[x] = wts[2ll * mid[x] + 1];
          any = true;
        }
      }
      if (!any) break;
#pragma unroll
      for (int x = 0; x < K2; ++x) {
        if (a[x] < c[x]) {
          const bool below = kFloat ? dadd<true>(fbase[x], val[x]) < fbnd[x] : val[x] < key[x];
          if (below) a[x] = mid[x] + 1; else c[x] = mid[x];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      if (!need[k]) continue;
      const int w = wi[k];
      const bool pull = L.pull[w] != 0;
      const uint32_t d = L.d[w];
      const int lo = a[2 * k];
      const int hi = leaf[k] ? lo : max(lo, a[2 * k + 1]);
      if (pull) {
        acc.pullscan += (unsigned long long)(hi - lo);
      } else if (!leaf[k]) {
        if (ub == kInf && hi < re[k]) atomicOr(&I.flags.v, FLAG_MAYBE_OVERFLOW);
        acc.expansions += 1;
        acc.band += (d >= lb) ? 1 : 0;
        acc.pscan += (unsigned long long)(hi - lo);
      }
      int size = hi - lo;
      if (size > V.heavy_split) {
        emit_heavy(I, L.u[w], d, lo, hi, pull);
        size = 0;
      }
      L.lo[w] = lo;
      L.sz[w] = size;
    }
  }
  __syncthreads();

  // sizes -> exclusive offsets (each thread owns kItemsPerThread consecutive entries)
  int loc[kItemsPerThread];
  int run = 0;
#pragma unroll
  for (int k = 0; k < kItemsPerThread; ++k) {
    const int w = tid * kItemsPerThread + k;
    loc[k] = w < m ? L.sz[w] : 0;
    run += loc[k];
  }
  int total;
  int off = block_excl_scan<int>(run, L.iscan, &total);
#pragma unroll
  for (int k = 0; k < kItemsPerThread; ++k) {
    const int w = tid * kItemsPerThread + k;
    if (w < m) L.sz[w] = off;
    off += loc[k];
  }
  __syncthreads();

  // ---------------------------------------------------------- phase 2b: edges
  // Each thread takes kEdgesPerThread edges per pass; their row loads, then
  // their neighbour-distance loads, then their atomics are in flight together.
  const bool any_pull = (kind == SEG_U) || (kind == SEG_H);
  SSSP_GBL int32_t* qnext = V.q_next;
  constexpr int kPass = kEdgesPerThread * kBlock;
  for (int base = 0; base < total; base += kPass) {
    __syncthreads();
    if (S.nq > kStageCap - kPass || S.nt > kStageCap - kPass)
      stage_flush(S, qnext, &I.q_next_cnt.v, V.touched, &I.touched_cnt.v, V.n, &I.flags.v);
    int jj[kEdgesPerThread];
    uint64_t ent[kEdgesPerThread];
#pragma unroll
    for (int x = 0; x < kEdgesPerThread; ++x) {
      const int e = base + x * kBlock + tid;
      jj[x] = -1;
      ent[x] = 0;
      if (e < total) {
        int lo_j = 0, hi_j = m;  // largest j with offset[j] <= e
        while (hi_j - lo_j > 1) {
          const int mid = (lo_j + hi_j) >> 1;
          if (L.sz[mid] <= e) lo_j = mid; else hi_j = mid;
        }
        jj[x] = lo_j;
        ent[x] = V.adj[L.lo[lo_j] + (e - L.sz[lo_j])];
      }
    }
    uint32_t dv[kEdgesPerThread];
#pragma unroll
    for (int x = 0; x < kEdgesPerThread; ++x)
      dv[x] = jj[x] >= 0 ? dist_of(V.state, (int)(uint32_t)(ent[x] & 0xffffffffull)) : 0u;
    bool ok[kEdgesPerThread];
    int t[kEdgesPerThread], from[kEdgesPerThread];
    uint32_t c[kEdgesPerThread], prev[kEdgesPerThread];
#pragma unroll
    for (int x = 0; x < kEdgesPerThread; ++x) {
      ok[x] = false;
      t[x] = 0;
      from[x] = 0;
      c[x] = 0;
      prev[x] = 0;
      if (jj[x] < 0) continue;
      const int j = jj[x];
      const int v = (int)(uint32_t)(ent[x] & 0xffffffffull);
      const uint32_t w = (uint32_t)(ent[x] >> 32);
      const uint32_t dj = L.d[j];
      if (!(any_pull && L.pull[j])) {
        c[x] = dadd<kFloat>(dj, w);  // in [lb, ub) by the range
        t[x] = v;
        from[x] = L.u[j];
        if (c[x] < dv[x]) {
          const uint64_t old = relax_state(V.state, v, c[x], V.rid);
          ok[x] = c[x] < (uint32_t)(old >> 32);
          prev[x] = (uint32_t)old;
        }
      } else {
        // pull: the best candidate of u over this batch's edges, in LDS
        if (dv[x] >= st && dv[x] < lb) {
          unsigned long long cc = kFloat ? (unsigned long long)dadd<true>(dv[x], w)
                                         : (unsigned long long)dv[x] + w;
          if (cc < ub && cc < dj) {
            if (kTree) atomicMin(&L.pmin64[j], (cc << 32) | (uint32_t)v);
            else atomicMin(&L.pmin32[j], (uint32_t)cc);
          }
        }
      }
    }
#pragma unroll
    for (int x = 0; x < kEdgesPerThread; ++x) on_success<kTree>(V, ok[x], t[x], c[x], prev[x], from[x], acc, S);
  }
  if (any_pull) {
    // one device atomic per pulled vertex
    for (int base = 0; base < m; base += kPass) {
      __syncthreads();
      if (S.nq > kStageCap - kPass || S.nt > kStageCap - kPass)
        stage_flush(S, qnext, &I.q_next_cnt.v, V.touched, &I.touched_cnt.v, V.n, &I.flags.v);
      bool ok[kEdgesPerThread];
      int t[kEdgesPerThread], from[kEdgesPerThread];
      uint32_t c[kEdgesPerThread], prev[kEdgesPerThread];
#pragma unroll
      for (int x = 0; x < kEdgesPerThread; ++x) {
        const int w = base + x * kBlock + tid;
        ok[x] = false;
        t[x] = 0;
        from[x] = 0;
        c[x] = 0;
        prev[x] = 0;
        if (w < m && L.pull[w]) {
          if (kTree) {
            const unsigned long long pm = L.pmin64[w];
            c[x] = (uint32_t)(pm >> 32);
            from[x] = (int)(uint32_t)pm;
          } else {
            c[x] = L.pmin32[w];
          }
          if (c[x] < L.d[w]) {
            t[x] = L.u[w];
            const uint64_t old = relax_state(V.state, t[x], c[x], V.rid);
            ok[x] = c[x] < (uint32_t)(old >> 32);
            prev[x] = (uint32_t)old;
          }
        }
      }
#pragma unroll
      for (int x = 0; x < kEdgesPerThread; ++x) on_success<kTree>(V, ok[x], t[x], c[x], prev[x], from[x], acc, S);
    }
  }
  stage_flush(S, qnext, &I.q_next_cnt.v, V.touched, &I.touched_cnt.v, V.n, &I.flags.v);
  flush_acc(I, V.maxw, acc);
}

// ------------------------------------------------------------ tick: settle --

struct SettleLds {
  uint32_t mass[kLdsRing];
  uint32_t cnt[kLdsRing];
  uint32_t hist[kLdsHist];
  unsigned long long sdec[kBlock / kWave];
  uint32_t maxd[kBlock / kWave];
  int iscan[kBlock / kWave + 1];
  int base[2];
};

template <class Sh>
union BlockLds {
  SettleLds s;
  HeurLds h;
  RoundLds<Sh> r;
};

// One workgroup settles up to kSettleBatch items (kSettlePer per thread): the
// step's touched vertices (with dist < ub they are final; in the first step
// the rest stay pending) and the pending list's compaction. Degree mass moves from the unsettled histogram
// to the per-distance ring; settled vertices are appended to the settled list.
template <class Sh>
__device__ __noinline__ void block_settle(GInst& I, int kind, int item0, int nitems, SettleLds& L) {
  constexpr int kSettlePer = Sh::kSettle;
  GDevGraph& g = I.gc;
  const int tid = threadIdx.x;
  const uint32_t lb = I.lb, ub = I.ub, M = I.M;
  // the ring feeds computeST: per distance, or per bin of the ST_NUM grid
  // (binary32 weights, or integer weights beyond the exact window; bins
  // klb..kub hold this step's settled vertices)
  const bool fw = g.float_w != 0;
  const bool grid = use_st_grid(fw, M, I.st_grid);
  const double inv = grid ? grid_inv(M, fw) : 0.0;
  const uint32_t klb = grid ? gbin(lb, inv, fw) : lb;
  const uint32_t kub = grid ? gbin(ub, inv, fw) : ub;
  const bool frec = grid && klb != kNoBin && kub != kNoBin;
  const uint32_t band = grid ? (frec ? kub - klb + 1u : 0u) : ub - lb;
  const uint32_t nb = band < (uint32_t)kLdsRing ? band : (uint32_t)kLdsRing;
  const int nh = g.num_deg < kLdsHist ? g.num_deg : kLdsHist;
  auto dinfo = gbl(g.dinfo);
  auto state = gbl(I.state);
  auto ring_mass = gbl(I.ring_mass);
  auto ring_cnt = gbl(I.ring_cnt);
  auto hist_cnt = gbl(I.hist_cnt);
  const uint32_t ring_mask = I.ring_mask;
  auto touched = gbl(I.touched);
  auto pcur = gbl(I.plist[I.psel]);
  auto pnext = gbl(I.plist[I.psel ^ 1]);
  auto settled = gbl(I.settled);
  const int n = I.n;
  const int maxw = I.maxw;
  for (uint32_t k = tid; k < nb; k += kBlock) { L.mass[k] = 0; L.cnt[k] = 0; }
  for (int k = tid; k < nh; k += kBlock) L.hist[k] = 0;
  __syncthreads();
  // kSettlePer items per thread, their loads in flight together
  int vv[kSettlePer];
  uint32_t dd[kSettlePer];
  uint64_t di[kSettlePer];
#pragma unroll
  for (int k = 0; k < kSettlePer; ++k) {
    const int it = item0 + k * kBlock + tid;
    vv[k] = it < nitems ? (kind == SEG_ST ? touched[it] : pcur[it]) : -1;
  }
#pragma unroll
  for (int k = 0; k < kSettlePer; ++k) {
    dd[k] = kInf;
    di[k] = 0;
    if (vv[k] >= 0) {
      dd[k] = dist_of(state, vv[k]);
      di[k] = dinfo[vv[k]];
    }
  }
  unsigned long long sdec = 0;
  uint32_t maxd = 0;
  int ns = 0, np = 0;
#pragma unroll
  for (int k = 0; k < kSettlePer; ++k) {
    const int v = vv[k];
    const uint32_t d = dd[k];
    const bool settle = (kind == SEG_ST) && v >= 0 && d < ub;
    const bool pend = v >= 0 && d >= ub;
    ns += settle ? 1 : 0;
    np += pend ? 1 : 0;
    if (!settle) continue;
    const int deg = (int)(uint32_t)di[k];
    // only the window [ub - M, ub) is read by the next computeST; the first
    // step's band may be wider, and older values would alias ring slots
    // (grid: only the last ring-size bins up to bin(ub) are kept)
    uint32_t key = d;
    bool rec = (unsigned long long)d + M >= ub;
    if (grid) {
      key = frec ? gbin(d, inv, fw) : 0u;
      rec = frec && (unsigned long long)key + ring_mask + 1ull > kub;
    }
    if (rec) {
      const uint32_t off = key - klb;
      if (off < nb) {
        atomicAdd(&L.mass[off], (uint32_t)deg);
        atomicAdd(&L.cnt[off], 1u);
      } else {
        atomicAdd(&ring_mass[key & ring_mask], (unsigned long long)deg);
        atomicAdd(&ring_cnt[key & ring_mask], 1u);
      }
    }
    const int r = (int)(di[k] >> 32);
    if (r >= 0) {
      if (r < nh) atomicAdd(&L.hist[r], 1u); else atomicSub(&hist_cnt[r], 1u);
    }
    sdec += (unsigned long long)deg;
    maxd = d > maxd ? d : maxd;
  }
  // one atomic per workgroup and list
  int tot_s, tot_p;
  int off_s = block_excl_scan<int>(ns, L.iscan, &tot_s);
  int off_p = block_excl_scan<int>(np, L.iscan, &tot_p);
  if (tid == 0) {
    L.base[0] = tot_s ? atomicAdd(&I.settled_cnt.v, tot_s) : 0;
    L.base[1] = tot_p ? atomicAdd(&I.p_next_cnt.v, tot_p) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSettlePer; ++k) {
    const int v = vv[k];
    if (v < 0) continue;
    if (kind == SEG_ST && dd[k] < ub) {
      const int p = L.base[0] + off_s++;
      if (p < n) settled[p] = v; else atomicOr(&I.flags.v, FLAG_CAPACITY);
    } else if (dd[k] >= ub) {
      const int q = L.base[1] + off_p++;
      if (q < n) pnext[q] = v; else atomicOr(&I.flags.v, FLAG_CAPACITY);
    }
  }
  unsigned long long ws = wave_sum(sdec);
  uint32_t wm = maxd;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    uint32_t y = __shfl_xor(wm, o, kWave);
    wm = y > wm ? y : wm;
  }
  unsigned long long qe = wave_sum((unsigned long long)(ns + np));
  if (lane_id() == 0) {
    L.sdec[tid / kWave] = ws;
    L.maxd[tid / kWave] = wm;
    if (qe) atomicAdd(&g_wgacc.v[6], qe);
  }
  __syncthreads();
  for (uint32_t k = tid; k < nb; k += kBlock) {
    uint32_t c = L.cnt[k];
    if (c) {
      uint32_t slot = (klb + k) & ring_mask;
      atomicAdd(&ring_mass[slot], (unsigned long long)L.mass[k]);
      atomicAdd(&ring_cnt[slot], c);
    }
  }
  for (int k = tid; k < nh; k += kBlock) {
    uint32_t c = L.hist[k];
    if (c) atomicSub(&hist_cnt[k], c);
  }
  if (tid == 0) {
    unsigned long long s = 0;
    uint32_t m = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      s += L.sdec[w];
      m = L.maxd[w] > m ? L.maxd[w] : m;
    }
    if (s) atomicAdd(&I.S.v, (unsigned long long)(0ull - s));
    if (m) atomicMax(&I.max_settled.v, m);
  }
  __syncthreads();
}

// ------------------------------------------------------------- scheduling --

// The record of the segment holding batch b: the last one whose first batch
// is <= b. With few segments each thread loads one record (a single round of
// loads); with many, a bisection. Whole workgroup.
__device__ SegRec find_segment(const GGlobals& G, int b) {
  const int nseg = G.nseg;  // the table has nseg + 1 records
  const SSSP_GBL SegRec* seg = gbl(G.seg);
  if (nseg <= kBlock) {
    __shared__ SegRec s_rec;
    const int t = threadIdx.x;
    SegRec r = {0, 0, 0, 0};
    if (t < nseg) r = gload(seg + t);
    // first batches do not decrease: the count of segments starting at or
    // before b is the index of b's segment plus one, and the thread of that
    // index hands its record over
    const int idx = __syncthreads_count(t < nseg && r.first <= b) - 1;
    if (t == idx) s_rec = r;
    __syncthreads();
    return s_rec;
  }
  int lo = 0, hi = nseg;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (seg[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  return gload(seg + lo);
}

// Bucket fusion (Section 4.1: up to FUSED = 256 rounds on a local frontier
// between two synchronisations). Here: while an instance's next frontier fits
// one batch and produced no heavy chunks, the workgroup that ran the round
// applies the round transition itself and runs the next round at once -- no
// grid barrier, no other workgroup involved. The band is fixed meanwhile, so
// any grouping of rounds reaches the same settled set. When the frontier
// empties or grows past one batch, the epilogue takes over with its usual
// transition of the last round.
template <bool kTree, bool kFloat, class Sh>
__device__ __noinline__ void fused_rounds(GInst& I, RoundLds<Sh>& L) {
  __shared__ int s_go, s_nq;
  const int cap = I.fuse_cap;
  for (int r = 0; r < cap; ++r) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      // the round's list appends and distance updates came from this
      // workgroup's waves and sit in this XCD's L2; the acquire drops stale
      // lines from this CU's cache before the next round reads them
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int nq = __hip_atomic_load(&I.q_next_cnt.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int nh = __hip_atomic_load(&I.h_next_cnt.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool go = nh == 0 && nq > 0 && nq <= Sh::kBatch;
      if (go) {
        const uint32_t ubn = __hip_atomic_load(&I.ub_next.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (I.first && ubn < I.ub) I.ub = ubn;
        I.c.rounds += 1;
        I.c.fused_rounds += 1;
        I.rounds_in_step += 1;
        __hip_atomic_store(&I.q_next_cnt.v, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        I.qsel ^= 1;
        I.hsel ^= 1;
        I.nF = nq;
        I.nH = 0;
        I.rid += 1;
      }
      s_go = go ? 1 : 0;
      s_nq = nq;
    }
    __syncthreads();
    if (!s_go) break;
    block_round<kTree, kFloat, Sh>(I, SEG_Q, 0, s_nq, L);
  }
}

// Debug tick log: words 4..7 of a tick's entry (earliest batch start, latest
// batch end, heuristic start and end) are opened before the tick runs.
__device__ void tick_log_open(GGlobals& G, unsigned long long t) {
  auto e = gbl(G.tick_log) + kTickLogWords * t;
  e[4] = ~0ull;
  e[5] = 0;
  e[6] = 0;
  e[7] = 0;
}

__device__ __forceinline__ SSSP_GBL unsigned long long* tick_log_entry(GGlobals& G) {
  if (!G.tick_log) return nullptr;
  const unsigned long long t = G.ticks;
  return t < G.tick_log_cap ? gbl(G.tick_log) + kTickLogWords * t : nullptr;
}

// One tick's batches, taken round-robin by the P participating workgroups
// (this one is number pid).
template <class Sh>
__device__ void run_tick(GGlobals& G, BlockLds<Sh>& lds, int pid, int P) {
  __shared__ int s_last;
  const int total_batches = G.total_batches;
  SSSP_GBL unsigned long long* tl = tick_log_entry(G);
  if (tl && threadIdx.x == 0 && pid < total_batches) atomicMin((unsigned long long*)(tl + 4), wall_clock64());
  for (int b = pid; b < total_batches; b += P) {
    const SegRec sr = find_segment(G, b);
    const int ii = sr.inst;
    GInst& I = gbl(G.insts)[ii];
    __syncthreads();  // the previous batch's counter additions are in
    if (threadIdx.x == 0) wgacc_select(G, ii);  // block_settle / block_round sync before adding
    const int kind = sr.word & 15;
    const int pb = sr.word >> 8;
    const int item0 = (b - sr.first) * pb;
    const int cnt = sr.count;
    if (kind == SEG_ST || kind == SEG_SP) {
      block_settle<Sh>(I, kind, item0, cnt, lds.s);
      // the heuristic only reads words updated by device atomics: waiting for
      // this batch's atomics to complete is enough before counting it done
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) {
        int done = atomicAdd(&I.settle_done.v, 1) + 1;
        s_last = (done == I.settle_items);
      }
      __syncthreads();
      if (s_last) {
        if (threadIdx.x == 0) {
          __threadfence();
          if (tl) tl[6] = wall_clock64();
        }
        __syncthreads();
        run_heuristic(I, lds.h);
        if (tl && threadIdx.x == 0) tl[7] = wall_clock64();
        // its plain stores (next step's control words, ring clears) must be
        // out of this XCD's L2 before other XCDs use them: done at the barrier
      }
      __syncthreads();
    } else {
      const uint32_t mode = (uint32_t)(sr.word >> 4) & 3u;
      const bool tree = (mode & 1u) != 0;
      const bool fw = (mode & 2u) != 0;
      if (fw) {
        if (tree) block_round<true, true, Sh>(I, kind, item0, cnt, lds.r);
        else block_round<false, true, Sh>(I, kind, item0, cnt, lds.r);
      } else {
        if (tree) block_round<true, false, Sh>(I, kind, item0, cnt, lds.r);
        else block_round<false, false, Sh>(I, kind, item0, cnt, lds.r);
      }
      // a frontier that fits one batch, with no heavy chunks, belongs to this
      // workgroup alone for the whole tick: chain its next rounds here
      if (kind == SEG_Q && cnt <= pb && I.nH == 0 && I.fuse_cap > 0) {
        if (fw) {
          if (tree) fused_rounds<true, true, Sh>(I, lds.r);
          else fused_rounds<false, true, Sh>(I, lds.r);
        } else {
          if (tree) fused_rounds<true, false, Sh>(I, lds.r);
          else fused_rounds<false, false, Sh>(I, lds.r);
        }
      }
    }
  }
  if (tl && threadIdx.x == 0 && pid < total_batches) atomicMax((unsigned long long*)(tl + 5), wall_clock64());
}

// Words updated by device atomics during a tick that the transition reads.
struct HotIn {
  int32_t u_next, q_next, h_next, touched, settled, p_next;
  uint32_t ub_next;
};

// Phase transition of one instance after a tick, on a register copy X of its
// control words (the caller loads and stores them in bulk); its segments of
// the next tick go to Sp. Resets the hot words it consumed in I.
// Serial per instance; called by one thread per instance.
__device__ void transition(InstCtl& X, SegSpec& Sp, const HotIn& h, int32_t n, int32_t heavy_cap,
                           int32_t rb, int32_t sb, unsigned long long& rounds, GInst& I) {
#pragma unroll
  for (int s = 0; s < kMaxSegPerInst; ++s) {
    Sp.cnt[s] = 0;
    Sp.kind[s] = SEG_Q;
    Sp.pb[s] = kBlock;
  }
  if (X.phase == PH_DONE) return;
  if (X.tick_kind == PH_ROUND) {
    if (X.init_round && X.pull_on) {
      X.usel ^= 1;
      X.nU = min(h.u_next, n);
      I.u_next_cnt.v = 0;
      X.u_done = X.u_end;
    }
    X.init_round = 0;
    if (X.first && h.ub_next < X.ub) X.ub = h.ub_next;
    rounds += 1;
    X.rounds_in_step += 1;
    const int nq = min(h.q_next, n), nh = min(h.h_next, heavy_cap);
    I.q_next_cnt.v = 0;
    I.h_next_cnt.v = 0;
    if (nq > 0 || nh > 0) {
      X.qsel ^= 1;
      X.hsel ^= 1;
      X.nF = nq;
      X.nH = nh;
      X.rid += 1;
      Sp.cnt[0] = nq; Sp.kind[0] = SEG_Q; Sp.pb[0] = rb;
      Sp.cnt[1] = nh; Sp.kind[1] = SEG_H; Sp.pb[1] = kHeavyPerBatch;
      return;
    }
    if (X.first && X.ub == kInf) {
      X.phase = PH_DONE;
      return;
    }
    X.tick_kind = PH_SETTLE;
    X.phase = PH_SETTLE;
    X.nT = min(h.touched, n);
    X.settled_mark = min(h.settled, n);
    I.settle_done.v = 0;
    int bt = (X.nT + sb - 1) / sb;
    if (bt < 1) bt = 1;
    int bp = (X.nP + sb - 1) / sb;
    X.settle_items = bt + bp;
    // a settle tick always has at least one batch so that the heuristic runs:
    // -1 marks one empty batch
    Sp.cnt[0] = X.nT == 0 ? -1 : X.nT; Sp.kind[0] = SEG_ST; Sp.pb[0] = sb;
    Sp.cnt[1] = X.nP; Sp.kind[1] = SEG_SP; Sp.pb[1] = sb;
    return;
  }
  // a settle tick ran; the heuristic has set phase to ROUND or DONE
  X.psel ^= 1;
  X.nP = min(h.p_next, n);
  I.p_next_cnt.v = 0;
  I.touched_cnt.v = 0;
  if (X.phase == PH_DONE) return;
  X.tick_kind = PH_ROUND;
  X.init_round = 1;
  X.nF = 0;
  Sp.cnt[0] = X.wEnd - X.wBegin; Sp.kind[0] = SEG_W; Sp.pb[0] = rb;
  Sp.cnt[1] = X.nP; Sp.kind[1] = SEG_P; Sp.pb[1] = rb;
  Sp.cnt[2] = X.pull_on ? X.nU + (X.u_end - X.u_done) : 0; Sp.kind[2] = SEG_U;
  Sp.pb[2] = rb;
}

// Build the tick table. With do_transition, every instance first takes its
// phase transition (and, with count, an active instance counts the tick that
// just ended), which records its segments of the next tick in the instance;
// otherwise the recorded segments are laid out as they are (a new launch
// continuing earlier instances, or the first tick of new ones). One
// workgroup; each thread handles a contiguous run of instances, and every
// word an instance's transition needs is loaded before any of them is used.
__device__ void build_table(GGlobals& G, bool do_transition, bool count) {
  const int tid = threadIdx.x;
  const int k = G.ninst;
  __shared__ unsigned long long sh[kBlock / kWave + 1];
  __shared__ int s_active;
  if (tid == 0) s_active = 0;
  __syncthreads();
  const int per = (k + kBlock - 1) / kBlock;
  const int i0 = min(k, tid * per), i1 = min(k, i0 + per);
  SSSP_GBL Inst* insts = gbl(G.insts);
  SSSP_GBL SegRec* seg = gbl(G.seg);
  int local_batches = 0, local_segs = 0;
  int nb_last[kMaxSegPerInst], cnt_last[kMaxSegPerInst], word_last[kMaxSegPerInst];
#pragma unroll
  for (int s = 0; s < kMaxSegPerInst; ++s) nb_last[s] = cnt_last[s] = word_last[s] = 0;
  for (int i = i0; i < i1; ++i) {
    GInst& I = insts[i];
    SSSP_GBL InstCtl* ctl = (SSSP_GBL InstCtl*)&I;
    InstCtl X = gload((const SSSP_GBL InstCtl*)ctl);
    SegSpec Sp;
    if (do_transition) {
      const HotIn h = {I.u_next_cnt.v, I.q_next_cnt.v, I.h_next_cnt.v, I.touched_cnt.v,
                       I.settled_cnt.v, I.p_next_cnt.v, I.ub_next.v};
      const int32_t n = I.n, heavy_cap = I.heavy_cap;
      unsigned long long rounds = I.c.rounds, ticks = I.c.ticks;
      if (count && X.phase != PH_DONE) ticks += 1;
      transition(X, Sp, h, n, heavy_cap, G.round_batch, G.settle_batch, rounds, I);
      gstore(ctl, X);
      gstore(&I.spec, Sp);
      I.c.rounds = rounds;
      I.c.ticks = ticks;
    } else {
      Sp = gload((const SSSP_GBL SegSpec*)&I.spec);
    }
    if (X.phase != PH_DONE) atomicAdd(&s_active, 1);
    const uint32_t mode = I.mode;
#pragma unroll
    for (int s = 0; s < kMaxSegPerInst; ++s) {
      int c = X.phase == PH_DONE ? 0 : Sp.cnt[s];
      const int pb = Sp.pb[s] > 0 ? Sp.pb[s] : kBlock;
      int nb;
      if (c < 0) { nb = 1; c = 0; }
      else nb = (c + pb - 1) / pb;
      cnt_last[s] = c;
      word_last[s] = seg_word(Sp.kind[s], mode, pb);
      if (per > 1) {
        // the first batch is known after the scan: the count for now
        const SegRec r = {nb, i, c, word_last[s]};
        gstore(seg + i * kMaxSegPerInst + s, r);
      }
      nb_last[s] = nb;
      local_batches += nb;
      local_segs += nb > 0 ? 1 : 0;
    }
  }
  // With at most kBlock instances the table lists only segments that have
  // batches (inactive instances and empty lists take no record), so that a
  // launch of many instances, most of them idle or with one or two kinds of
  // work, keeps a table short enough for the one-load segment search. One scan
  // gives both offsets: batches in the low half (a tick has fewer than 2^31),
  // records in the high half.
  const unsigned long long mine =
      per == 1 ? ((unsigned long long)local_segs << 32) | (unsigned long long)local_batches
               : (unsigned long long)local_batches;
  unsigned long long total;
  const unsigned long long before = block_excl_scan<unsigned long long>(mine, sh, &total);
  int run = per == 1 ? (int)(uint32_t)before : (int)before;
  if (per == 1) {
    if (i0 < i1) {
      int pos = (int)(before >> 32);
#pragma unroll
      for (int s = 0; s < kMaxSegPerInst; ++s) {
        if (nb_last[s] == 0) continue;
        const SegRec r = {run, i0, cnt_last[s], word_last[s]};
        gstore(seg + pos, r);
        ++pos;
        run += nb_last[s];
      }
    }
  } else {
    for (int i = i0; i < i1; ++i) {
      for (int s = 0; s < kMaxSegPerInst; ++s) {
        SSSP_GBL int32_t* first = &seg[i * kMaxSegPerInst + s].first;
        const int nb = *first;
        *first = run;
        run += nb;
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    const int nseg = per == 1 ? (int)(total >> 32) : k * kMaxSegPerInst;
    const int batches = per == 1 ? (int)(uint32_t)total : (int)total;
    G.nseg = nseg;
    const SegRec end = {batches, 0, 0, 0};
    gstore(seg + nseg, end);
    G.total_batches = batches;
    G.all_done = (s_active == 0) ? 1u : 0u;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- kernels --

// ----------------------------------------------------------- grid barrier --
// Workgroups are spread over the chip's XCDs (read from the XCC_ID hardware
// register); each XCD has its own L2. Between ticks, data written by one XCD
// must reach the others: the L2 of the writer is written back and the L2 of
// the reader invalidated. Doing that from every workgroup serialises hundreds
// of whole-cache operations per XCD per tick, so the barrier is two-level:
// the last workgroup of an XCD to arrive writes back and invalidates that
// XCD's L2 once, and arrives at the grid-wide counter; the last of those runs
// the epilogue; on release every XCD leader invalidates its L2 and then
// releases its own workgroups.

__device__ __forceinline__ uint32_t xcd_of_this_wg() {
  uint32_t r;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(r));
  return r & (uint32_t)(kMaxXcd - 1);
}

// A workgroup released by its XCD leader must drop stale cached lines. The
// leader's own fence already wrote this XCD's L2 back and the workgroup's
// stores reached that L2 before it arrived, so an agent-scope acquire (no
// write-back) completes the release/acquire chain. (A workgroup-scope
// invalidate is not enough: measured, stale data was read.)
__device__ __forceinline__ void acquire_after_release() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Wait until *word differs from old. kSleep (units of 64 cycles) paces the
// polling: every poll is a coherent load of the same line, and hundreds of
// workgroups polling one line slow down the memory channel behind it, the
// release write included.
template <int kSleep>
__device__ bool spin_until_changed(SSSP_GBL unsigned int* word, unsigned int old, SSSP_GBL unsigned int* err) {
  unsigned long long spins = 0;
  while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == old) {
    __builtin_amdgcn_s_sleep(kSleep);
    if (++spins > (1ull << 27)) {
      atomicOr(err, FLAG_TIMEOUT);
      return false;
    }
  }
  return true;
}

// Workgroups per XCD for the next tick: one batch each as far as there are
// batches, at least one per XCD. The others sit the tick out, so a tick with
// little work synchronises few workgroups (the barrier's cost grows with the
// number of workgroups that write back and invalidate caches).
//
// A tick of at most kLocalBatches batches runs on one XCD (the first
// populated one): every batch goes to its workgroups, and each other XCD sends
// one workgroup to the barrier with no work. A run of small ticks (the rounds
// and settle passes of a high-diameter graph) then reads what the previous
// tick wrote from that XCD's own L2. Such a tick's word is the quota of the
// working XCD with kLocalTick set.
constexpr int kLocalBatches = 64;
constexpr unsigned int kLocalTick = 0x80000000u;
// A quota word with kStopTick set ends the launch: the solves are done or an
// error was raised (the next tick would have nothing to do).
constexpr unsigned int kStopTick = 0x40000000u;
__device__ __forceinline__ unsigned int quota_for(int total_batches, unsigned int nxcd,
                                                  unsigned int min_members, unsigned int members0) {
  const unsigned int nx = nxcd ? nxcd : 1u;
  if (nx > 1u && total_batches <= kLocalBatches && (unsigned int)total_batches <= members0) {
    const unsigned int q = total_batches < 1 ? 1u : (unsigned int)total_batches;
    return q | kLocalTick;
  }
  unsigned int q = ((unsigned int)total_batches + nx - 1) / nx;
  if (q < 1u) q = 1u;
  if (q > min_members) q = min_members;
  return q;
}


// The serial part between two ticks (one workgroup): tick log, phase
// transitions and the next tick's work layout.
__device__ __forceinline__ void epilogue(GGlobals& G, unsigned int gen, unsigned int nxcd,
                                     unsigned int min_members, unsigned int members0) {
  if (threadIdx.x == 0) {
    if (gbl(G.tick_log) && G.ticks < G.tick_log_cap) {
      auto e = gbl(G.tick_log) + kTickLogWords * G.ticks;
      e[0] = wall_clock64();
      e[1] = (unsigned long long)G.total_batches;
      const GInst& I0 = gbl(G.insts)[0];
      e[2] = (unsigned long long)I0.tick_kind | ((unsigned long long)I0.init_round << 8) |
             ((unsigned long long)I0.pull_on << 9) | ((unsigned long long)I0.step << 16);
    }
  }
  __syncthreads();
  build_table(G, true, true);
  if (threadIdx.x == 0) {
    // the next tick's quota word (published with the release; the stop bit
    // is added below once the tick count is known)
    G.quota_next = quota_for(G.total_batches, nxcd, min_members, members0);
    if (gbl(G.tick_log) && G.ticks < G.tick_log_cap) gbl(G.tick_log)[kTickLogWords * G.ticks + 3] = wall_clock64();
    G.ticks += 1;
    if (gbl(G.tick_log) && G.ticks < G.tick_log_cap) tick_log_open(G, G.ticks);
    if (G.ticks >= G.tick_limit) {
      G.error |= FLAG_TICKS;
      G.all_done = 1u;
    }
    if (G.all_done || __hip_atomic_load(&G.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      G.quota_next |= kStopTick;
  }
  __syncthreads();
}

struct BarrierState {
  unsigned int gen;    // grid-wide release generation seen last
  unsigned int xgen;   // this XCD's release generation seen last
  uint32_t xcd;
  uint32_t members;    // workgroups on this XCD
  uint32_t nxcd;       // XCDs with at least one workgroup
  uint32_t rank;       // this workgroup's rank among its XCD's workgroups
  uint32_t xidx;       // this XCD's index among the populated XCDs
  uint32_t q0;         // quota word of the launch's first tick
  uint32_t min_members;  // workgroups on the least populated XCD
  uint32_t members0;   // workgroups on the first populated XCD (where small ticks run)
};

// Flat barrier with full fences by every workgroup: the whole barrier of the
// one-launch-per-tick mode (where the kernel boundary does the waiting).
__device__ bool barrier_flat(GGlobals& G, unsigned int& gen, bool wait, bool run_epilogue) {
  __shared__ int s_last;
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned int arrived = atomicAdd(&G.bar_count.v, 1u);
    s_last = (arrived == gridDim.x - 1);
    s_ok = 1;
  }
  __syncthreads();
  if (s_last) {
    if (threadIdx.x == 0) __threadfence();
    __syncthreads();
    if (run_epilogue) epilogue(G, gen, 1u, 1u, 1u);
    if (threadIdx.x == 0) {
      __hip_atomic_store(&G.bar_count.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      atomicAdd(&G.bar_gen.v, 1u);
    }
  } else if (wait) {
    if (threadIdx.x == 0) {
      s_ok = spin_until_changed<1>(&G.bar_gen.v, gen, &G.error) ? 1 : 0;
      __threadfence();
    }
  }
  __syncthreads();
  gen += 1;
  return s_ok != 0;
}

// The release word of an XCD: generation in the low half, the quota word of
// the tick it starts in the high half.
__device__ __forceinline__ unsigned long long release_word(unsigned int gen, unsigned int quota) {
  return ((unsigned long long)quota << 32) | gen;
}

// A workgroup outside the current tick waits for its XCD's release of the
// tick: one line per XCD, polled with long sleeps (it is not on the tick's
// critical path, and hundreds of parked workgroups polling one line would slow
// the channel behind it). Returns the release word that ended the wait (its
// generation tells how many ticks have passed), 0 if an error stopped the
// engine or the wait gave up. (The end of the engine is released like any
// tick, with the stop bit in its quota word.)
__device__ unsigned long long park_until_released(GGlobals& G, unsigned int xcd, unsigned int xgen) {
  unsigned long long spins = 0;
  unsigned long long w;
  while ((unsigned int)(w = __hip_atomic_load(&G.xcd_gen[xcd].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ==
         xgen) {
    __builtin_amdgcn_s_sleep(16);
    ++spins;
    if ((spins & 63u) == 0 && __hip_atomic_load(&G.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 0ull;
    if (spins > (1ull << 23)) {
      atomicOr(&G.error, FLAG_TIMEOUT);
      return 0ull;
    }
  }
  return w;
}

// A member of the tick waits for its XCD leader's release: returns the
// release word, 0 if the wait gave up.
__device__ unsigned long long spin_until_released(GGlobals& G, unsigned int xcd, unsigned int xgen) {
  unsigned long long spins = 0;
  unsigned long long w;
  while ((unsigned int)(w = __hip_atomic_load(&G.xcd_gen[xcd].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ==
         xgen) {
    __builtin_amdgcn_s_sleep(4);
    if (++spins > (1ull << 27)) {
      atomicOr(&G.error, FLAG_TIMEOUT);
      return 0ull;
    }
  }
  return w;
}

// Two-level barrier of the persistent engine among the tick's participants
// (quota per XCD); the grid-wide last arriver runs the epilogue. The next
// tick's quota word comes back in *next (from the epilogue, through each XCD
// leader's release word). Returns false if a wait gave up.
__device__ bool barrier_tick(GGlobals& G, BarrierState& B, unsigned int quota, unsigned int* next) {
  __shared__ int s_role;  // 0 wait for the XCD leader, 1 XCD leader, 2 epilogue
  __shared__ int s_ok;
  __shared__ unsigned int s_next;
  // every wave's stores and atomics of this tick are complete before arriving
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    s_ok = 1;
    unsigned int a = atomicAdd(&G.xcd_count[B.xcd].v, 1u);
    if (a == quota - 1) {
      __hip_atomic_store(&G.xcd_count[B.xcd].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();  // this XCD's writes leave its L2
      unsigned int b = atomicAdd(&G.bar_count.v, 1u);
      if (b == B.nxcd - 1) {
        __hip_atomic_store(&G.bar_count.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();  // see every XCD's written-back data
        s_role = 2;
      } else {
        s_ok = spin_until_changed<2>(&G.bar_gen.v, B.gen, &G.error) ? 1 : 0;
        __threadfence();  // drop stale lines from this XCD's L2
        s_role = 1;
      }
    } else {
      s_role = 0;
    }
  }
  __syncthreads();
  const int role = s_role;
  if (role == 2) {
    epilogue(G, B.gen, B.nxcd, B.min_members, B.members0);
    if (threadIdx.x == 0) {
      const unsigned int qn = G.quota_next;
      __threadfence();
      atomicAdd(&G.bar_gen.v, 1u);
      __hip_atomic_store(&G.xcd_gen[B.xcd].v, release_word(B.xgen + 1u, qn), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      s_next = qn;
    }
  } else if (role == 1) {
    if (threadIdx.x == 0) {
      // after the leader's fence the epilogue's word is current; a leader
      // whose wait gave up releases its XCD into a stop
      const unsigned int qn =
          s_ok ? __hip_atomic_load(&G.quota_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kStopTick;
      __hip_atomic_store(&G.xcd_gen[B.xcd].v, release_word(B.xgen + 1u, qn), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      s_next = qn;
    }
  } else {
    if (threadIdx.x == 0) {
      const unsigned long long w = spin_until_released(G, B.xcd, B.xgen);
      s_ok = w != 0ull ? 1 : 0;
      s_next = (unsigned int)(w >> 32);
      acquire_after_release();
    }
  }
  __syncthreads();
  B.gen += 1;
  B.xgen += 1;
  *next = s_next;
  return s_ok != 0;
}

// Registration of a persistent launch (thread 0 of each workgroup, after it
// took its rank on its XCD): the last workgroup of the grid to arrive reads
// the final member counts and releases every populated XCD with the launch's
// layout in the high half of the release word: the populated-XCD mask (bits
// 0-7), the fewest workgroups on one XCD (bits 8-19) and the workgroups of the
// first populated XCD (bits 20-31); at most 8 workgroups of 256 threads fit a
// CU, so a count stays below 4096. The others wait on their own XCD's line.
// Nothing but the counts is exchanged (the launch's data was written by
// earlier kernels), so no cache is written back or invalidated. Returns the
// layout, 0 if the wait gave up.
__device__ uint32_t register_launch(GGlobals& G, uint32_t xcd, unsigned int xgen) {
  // the rank's atomic is complete before this workgroup counts as arrived
  __builtin_amdgcn_s_waitcnt(0);
  const unsigned int a = atomicAdd(&G.bar_count.v, 1u);
  if (a != gridDim.x - 1u) return (uint32_t)(spin_until_released(G, xcd, xgen) >> 32);
  uint32_t mask = 0, mn = 0xffffffffu, m0 = 0;
  for (int x = 0; x < kMaxXcd; ++x) {
    const uint32_t m = __hip_atomic_load(&G.xcd_members[x].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (m == 0) continue;
    if (mask == 0) m0 = m;
    mask |= 1u << x;
    mn = m < mn ? m : mn;
  }
  const uint32_t lay = mask | (mn << 8) | (m0 << 20);
  __hip_atomic_store(&G.bar_count.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int x = 0; x < kMaxXcd; ++x) {
    if (!(mask >> x & 1u)) continue;
    const unsigned int g = (uint32_t)x == xcd ? xgen
        : (unsigned int)__hip_atomic_load(&G.xcd_gen[x].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&G.xcd_gen[x].v, release_word(g + 1u, lay), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return lay;
}

template <class Sh>
__global__ void __launch_bounds__(kBlock, Sh::kMinBlocks) k_engine(Globals* Gp, int persistent, int max_ticks) {
  __shared__ BlockLds<Sh> lds;
  __shared__ BarrierState s_b;
  GGlobals& G = *gbl(Gp);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 7; ++k) g_wgacc.v[k] = 0;
    g_wgacc.inst = -1;
    s_b.gen = __hip_atomic_load(&G.bar_gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (blockIdx.x == 0 && G.ticks == 0) G.t_start = wall_clock64();
  }
  __syncthreads();
  if (!persistent) {
    // one tick; the kernel boundary is the barrier
    if (__hip_atomic_load(&G.all_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    run_tick<Sh>(G, lds, blockIdx.x, gridDim.x);
    __syncthreads();
    if (threadIdx.x == 0) wgacc_flush(G);
    unsigned int gen = s_b.gen;
    barrier_flat(G, gen, false, true);
    return;
  }
  // register this workgroup with its XCD (and take a rank there); the last
  // of the grid to register releases every XCD with the final layout
  if (threadIdx.x == 0) {
    s_b.xcd = xcd_of_this_wg();
    s_b.xgen = (unsigned int)__hip_atomic_load(&G.xcd_gen[s_b.xcd].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_b.rank = atomicAdd(&G.xcd_members[s_b.xcd].v, 1u);
    const uint32_t lay = register_launch(G, s_b.xcd, s_b.xgen);
    s_b.nxcd = 0;  // no layout: the wait gave up
    if (lay != 0u) {
      const uint32_t mask = lay & 0xffu;
      const uint32_t mn = (lay >> 8) & 0xfffu, m0 = lay >> 20;
      s_b.nxcd = (uint32_t)__builtin_popcount(mask);
      s_b.xidx = (uint32_t)__builtin_popcount(mask & ((1u << s_b.xcd) - 1u));
      s_b.xgen += 1u;
      // every workgroup computes the same values, the first tick's quota
      // included (from the table the set-up kernel built); the epilogue
      // publishes the later ones
      s_b.q0 = quota_for(G.total_batches, s_b.nxcd, mn, m0);
      s_b.min_members = mn;
      s_b.members0 = m0;
    }
  }
  __syncthreads();
  if (s_b.nxcd == 0u) return;
  __syncthreads();
  BarrierState B = s_b;
  bool stale = false;  // parked since the last acquire
  // the quota word of the coming tick: computed for the first, then handed
  // over by each release (no shared word is read between ticks)
  unsigned int qw = B.q0;
  if (__hip_atomic_load(&G.all_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
      __hip_atomic_load(&G.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    qw |= kStopTick;
  for (int t = 0;;) {
    if (qw & kStopTick) break;
    const bool local = (qw & kLocalTick) != 0;
    const unsigned int qx = qw & ~kLocalTick;
    // this XCD's participants: a small tick's batches all go to the first XCD
    const unsigned int q = local ? (B.xidx == 0 ? qx : 1u) : qx;
    if (B.rank < q) {
      if (stale) {
        // back from waiting aside: drop cached lines before reading the tick's data
        if (threadIdx.x == 0) acquire_after_release();
        __syncthreads();
        stale = false;
      }
      if (local) run_tick<Sh>(G, lds, B.xidx == 0 ? (int)B.rank : 0x7fffffff, (int)qx);
      else run_tick<Sh>(G, lds, (int)(B.rank * B.nxcd + B.xidx), (int)(q * B.nxcd));
      if (!barrier_tick(G, B, q, &qw)) break;
      t += 1;
    } else {
      // not needed in this tick: wait for its release
      __shared__ unsigned long long s_rel;
      if (threadIdx.x == 0) s_rel = park_until_released(G, B.xcd, B.xgen);
      __syncthreads();
      const unsigned long long w = s_rel;
      if (w == 0ull) break;  // error or timeout
      const unsigned int d = (unsigned int)w - B.xgen;
      qw = (unsigned int)(w >> 32);
      t += (int)d;
      B.xgen += d;
      B.gen += d;
      stale = true;
    }
    if (max_ticks > 0 && t >= max_ticks) {
      if (threadIdx.x == 0 && blockIdx.x == 0) G.max_ticks_hit = 1;
      break;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) wgacc_flush(G);
}

// Per-solve state reset: state words, histogram, ring, counters. Grid-stride
// over every selected instance.
__global__ void k_init_arrays(Globals* Gp) {
  GGlobals& G = *gbl(Gp);
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int nsel = G.n_sel < 0 ? G.ninst : G.n_sel;
  for (int j = 0; j < nsel; ++j) {
    GInst& I = gbl(G.insts)[G.n_sel < 0 ? j : gbl(G.sel_list)[j]];
    GDevGraph& g = I.gc;
    auto state = gbl(I.state);
    for (long long v = tid; v < I.n; v += stride) state[v] = (unsigned long long)kInf << 32;
    if (I.best)
      for (long long v = tid; v < I.n; v += stride) gbl(I.best)[v] = ~0ull;
    for (long long x = tid; x < I.maxw; x += stride) {
      Counters z = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      gstore(gbl(I.cslot) + x, z);
    }
    for (long long r = tid; r < g.num_deg; r += stride) gbl(I.hist_cnt)[r] = gbl(g.deg_cnt0)[r];
    for (long long r = tid; r <= (long long)I.ring_mask; r += stride) {
      gbl(I.ring_mass)[r] = 0;
      gbl(I.ring_cnt)[r] = 0;
    }
  }
}

// Per-solve control reset and the first tick's table. One workgroup.
__global__ void __launch_bounds__(kBlock) k_init_ctl(Globals* Gp) {
  GGlobals& G = *gbl(Gp);
  const int nsel = G.n_sel < 0 ? G.ninst : G.n_sel;
  for (int j = 0; j < nsel; ++j) {
    GInst& I = gbl(G.insts)[G.n_sel < 0 ? j : gbl(G.sel_list)[j]];
    GDevGraph& g = I.gc;
    if (threadIdx.x == 0) {
      // the caller's ids to internal ones
      const SSSP_GBL int32_t* ren = g.new_of_old ? gbl(g.new_of_old) : nullptr;
      const int s = ren ? ren[I.source] : I.source;
      I.src_in = s;
      I.tgt_in = I.target < 0 ? -1 : (ren ? ren[I.target] : I.target);
      const int deg_s = gbl(g.rowptr)[s + 1] - gbl(g.rowptr)[s];
      I.M = g.max_w;
      I.lb = 0; I.ub = kInf; I.st = 0; I.lb0 = 0;
      I.first = 1;
      I.step = 0;
      I.rounds_in_step = 0;
      I.qsel = 0; I.psel = 0; I.usel = 0; I.hsel = 0;
      I.nP = 0; I.nU = 0; I.nT = 0; I.nH = 0;
      I.u_done = 0; I.u_end = 0;
      I.wBegin = 0; I.wEnd = 0;
      I.q_next_cnt.v = 0; I.touched_cnt.v = 0; I.p_next_cnt.v = 0; I.u_next_cnt.v = 0;
      I.settled_cnt.v = 0; I.h_next_cnt.v = 0;
      I.settled_mark = 0;
      I.nsteprec = 0;
      I.trace_len = 0;
      I.max_settled.v = 0;
      I.S.v = (unsigned long long)g.nnz;
      I.settle_items = 0; I.settle_done.v = 0;
      I.flags.v = 0;
      I.pull_on = 0;
      I.init_round = 0;
      I.tick_kind = PH_ROUND;
      I.high_d0 = g.high_d0;
      Counters z = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      gstore(&I.c, z);
      // round ids restart with every solve (the state words are reset)
      I.step_rid0 = 1;
      gbl(I.state)[s] = (unsigned long long)I.step_rid0;  // distance 0, touched in step 1
      if (I.best) gbl(I.best)[s] = (unsigned long long)(uint32_t)s;  // the root is its own parent
      I.rid = I.step_rid0 + 1;
      gbl(I.touched)[0] = s;
      I.touched_cnt.v = 1;
      gbl(I.q[0])[0] = s;
      I.nF = 1;
      I.ub_next.v = is_hub(g, s) ? 0u : kInf;
      I.phase = deg_s > 0 ? PH_ROUND : PH_DONE;
      // first tick: the source alone
      for (int sg = 0; sg < kMaxSegPerInst; ++sg) {
        I.spec.cnt[sg] = 0;
        I.spec.kind[sg] = SEG_Q;
        I.spec.pb[sg] = G.round_batch;
      }
      I.spec.cnt[0] = I.nF;
    }
    __syncthreads();
    // gap(0) from whole-graph statistics: sumD(0) = nnz, highD(0)
    uint32_t g0 = gap_of((unsigned long long)g.nnz, g.high_d0, g.nnz, g.max_w, gbl(g.rtow), I.alpha, I.beta);
    if (threadIdx.x == 0) {
      I.gap0 = g0;
      I.gap_cur = g0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    G.bar_count.v = 0;
    for (int x = 0; x < kMaxXcd; ++x) {
      G.xcd_count[x].v = 0;
      G.xcd_members[x].v = 0;
    }
    G.error = 0;
    G.max_ticks_hit = 0;
    G.ticks = 0;
    if (gbl(G.tick_log) && G.tick_log_cap > 0) tick_log_open(G, 0);
  }
  __syncthreads();
  build_table(G, false, false);
}

// Overflow confirmation (only when a range was cut by the +inf clamp): a
// vertex with a finite neighbour but no distance is reachable with a length
// the uint32 range cannot hold.
__global__ void k_overflow_check(Globals* Gp) {
  GGlobals& G = *gbl(Gp);
  const int nsel = G.n_sel < 0 ? G.ninst : G.n_sel;
  for (int j = 0; j < nsel; ++j) {
    GInst& I = gbl(G.insts)[G.n_sel < 0 ? j : gbl(G.sel_list)[j]];
    if (!(I.flags.v & FLAG_MAYBE_OVERFLOW)) continue;
    GDevGraph& g = I.gc;
    bool found = false;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < g.n && !found;
         v += (long long)gridDim.x * blockDim.x) {
      if (dist_of(gbl(I.state), (int)v) != kInf) continue;
      for (int e = gbl(g.rowptr)[v]; e < gbl(g.rowptr)[v + 1]; ++e) {
        int u = (int)(uint32_t)(gbl(g.adj)[e] & 0xffffffffull);
        if (dist_of(gbl(I.state), u) != kInf) {
          found = true;
          break;
        }
      }
    }
    if (found) atomicOr(&I.flags.v, FLAG_OVERFLOW);
  }
}

// The distances of the selected instances into their outputs.
__global__ void k_finish(Globals* Gp) {
  GGlobals& G = *gbl(Gp);
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int nsel = G.n_sel < 0 ? G.ninst : G.n_sel;
  for (int j = 0; j < nsel; ++j) {
    GInst& I = gbl(G.insts)[G.n_sel < 0 ? j : gbl(G.sel_list)[j]];
    GDevGraph& g = I.gc;
    auto state = gbl(I.state);
    auto dist = gbl(I.dist);
    // outputs are indexed by the caller's ids: v is the caller's, ren[v] internal
    const SSSP_GBL int32_t* ren = g.new_of_old ? gbl(g.new_of_old) : nullptr;
    const SSSP_GBL int32_t* back = g.old_of_new ? gbl(g.old_of_new) : nullptr;
    for (long long v = tid; v < I.n; v += stride) dist[v] = (uint32_t)(state[ren ? ren[v] : v] >> 32);
    if (I.parent && I.best) {
      auto parent = gbl(I.parent);
      auto best = gbl(I.best);
      for (long long v = tid; v < I.n; v += stride) {
        const long long vi = ren ? ren[v] : v;
        const uint32_t d = (uint32_t)(state[vi] >> 32);
        const unsigned long long b = best[vi];
        const int32_t p = (int32_t)(uint32_t)b;
        parent[v] = d == kInf ? -1 : (back ? back[p] : p);
        if (d != kInf && (uint32_t)(b >> 32) != d) atomicOr(&I.flags.v, FLAG_TREE);
      }
    }
  }
}

// Phase and flags of every instance, for a host that polls completions.
__global__ void k_status(Globals* Gp, uint32_t* status) {
  GGlobals& G = *gbl(Gp);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < G.ninst; i += gridDim.x * blockDim.x) {
    const GInst& I = gbl(G.insts)[i];
    status[2 * i] = I.phase;
    status[2 * i + 1] = I.flags.v | G.error;
  }
}

// highD over a degree histogram, exported for the graph preparation.
__global__ void __launch_bounds__(kBlock) k_high_d(const int32_t* deg_vals, const uint32_t* cnt,
                                                   int32_t D, uint32_t* out_h,
                                                   unsigned long long* out_mass) {
  __shared__ HeurLds lds;
  unsigned long long mass, count;
  uint32_t h = block_high_d(gbl(deg_vals), gbl(cnt), D, &mass, &count, lds);
  if (threadIdx.x == 0) {
    *out_h = h;
    *out_mass = mass;
  }
}


// ================================================================ host side

hipError_t launch_high_d(const int32_t* deg_vals, const uint32_t* cnt, int32_t D, uint32_t* out_h,
                         unsigned long long* out_mass, hipStream_t stream) {
  k_high_d<<<1, kBlock, 0, stream>>>(deg_vals, cnt, D, out_h, out_mass);
  return hipGetLastError();
}

hipError_t launch_init(Globals* dG, long long max_n, hipStream_t stream) {
  long long blocks = (max_n + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  k_init_arrays<<<(int)blocks, kBlock, 0, stream>>>(dG);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_init_ctl<<<1, kBlock, 0, stream>>>(dG);
  return hipGetLastError();
}

// The engine kernel of a tile shape.
const void* engine_fn(int shape) {
  switch (shape) {
    case SHAPE_WIDE: return reinterpret_cast<const void*>(k_engine<ShapeWide>);
    case SHAPE_NARROW: return reinterpret_cast<const void*>(k_engine<ShapeNarrow>);
    case SHAPE_SETTLE8: return reinterpret_cast<const void*>(k_engine<ShapeSettle8>);
    default: return reinterpret_cast<const void*>(k_engine<ShapeStd>);
  }
}

int engine_blocks_per_cu(int shape) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, engine_fn(shape), kBlock, 0) != hipSuccess)
    return 1;
  return nb < 1 ? 1 : nb;
}

hipError_t launch_engine(Globals* dG, int grid, bool persistent, int max_ticks, hipStream_t stream,
                         int shape) {
  int pers = persistent ? 1 : 0;
  int mt = persistent ? max_ticks : 0;
  void* args[] = {(void*)&dG, (void*)&pers, (void*)&mt};
  if (!persistent)
    return hipLaunchKernel(engine_fn(shape), dim3(grid), dim3(kBlock), args, 0, stream);
  return hipLaunchCooperativeKernel(engine_fn(shape), dim3(grid), dim3(kBlock), args, 0, stream);
}

hipError_t launch_status(Globals* dG, int ninst, uint32_t* status, hipStream_t stream) {
  int blocks = (ninst + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  k_status<<<blocks, kBlock, 0, stream>>>(dG, status);
  return hipGetLastError();
}

hipError_t add_solve_nodes(hipGraph_t graph, hipGraphNode_t dep, Globals* dG, long long max_n, int grid,
                           int shape, hipGraphNode_t* last) {
  long long ib = (max_n + kBlock - 1) / kBlock;
  ib = ib < 1 ? 1 : (ib > 16384 ? 16384 : ib);
  long long ob = (max_n + kBlock - 1) / kBlock;
  ob = ob < 1 ? 1 : (ob > 4096 ? 4096 : ob);
  int pers = 1, max_ticks = 0;
  void* a_g[] = {(void*)&dG};
  void* a_e[] = {(void*)&dG, (void*)&pers, (void*)&max_ticks};
  hipKernelNodeParams p;
  std::memset(&p, 0, sizeof(p));
  p.blockDim = dim3(kBlock);
  hipGraphNode_t n_arr, n_ctl, n_eng, n_ovf;
  size_t nd = dep ? 1 : 0;
  p.func = reinterpret_cast<void*>(k_init_arrays);
  p.gridDim = dim3((unsigned)ib);
  p.kernelParams = a_g;
  hipError_t e = hipGraphAddKernelNode(&n_arr, graph, dep ? &dep : nullptr, nd, &p);
  if (e != hipSuccess) return e;
  p.func = reinterpret_cast<void*>(k_init_ctl);
  p.gridDim = dim3(1);
  e = hipGraphAddKernelNode(&n_ctl, graph, &n_arr, 1, &p);
  if (e != hipSuccess) return e;
  p.func = const_cast<void*>(engine_fn(shape));
  p.gridDim = dim3((unsigned)grid);
  p.kernelParams = a_e;
  e = hipGraphAddKernelNode(&n_eng, graph, &n_ctl, 1, &p);
  if (e != hipSuccess) return e;
  hipKernelNodeAttrValue v;
  std::memset(&v, 0, sizeof(v));
  v.cooperative = 1;
  e = hipGraphKernelNodeSetAttribute(n_eng, hipKernelNodeAttributeCooperative, &v);
  if (e != hipSuccess) return e;
  p.func = reinterpret_cast<void*>(k_overflow_check);
  p.gridDim = dim3((unsigned)ob);
  p.kernelParams = a_g;
  e = hipGraphAddKernelNode(&n_ovf, graph, &n_eng, 1, &p);
  if (e != hipSuccess) return e;
  hipGraphNode_t n_fin;
  long long fb = (max_n + kBlock - 1) / kBlock;
  fb = fb < 1 ? 1 : (fb > 8192 ? 8192 : fb);
  p.func = reinterpret_cast<void*>(k_finish);
  p.gridDim = dim3((unsigned)fb);
  e = hipGraphAddKernelNode(&n_fin, graph, &n_ovf, 1, &p);
  if (e != hipSuccess) return e;
  *last = n_fin;
  return hipSuccess;
}

hipError_t launch_finish(Globals* dG, long long max_n, hipStream_t stream) {
  long long blocks = (max_n + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  k_finish<<<(int)blocks, kBlock, 0, stream>>>(dG);
  return hipGetLastError();
}

hipError_t launch_overflow_check(Globals* dG, long long max_n, hipStream_t stream) {
  long long blocks = (max_n + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  k_overflow_check<<<(int)blocks, kBlock, 0, stream>>>(dG);
  return hipGetLastError();
}

}  // namespace sssp
