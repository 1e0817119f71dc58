// Graph preparation on the GPU: the paper's preprocessing (Section 4.1: every
// vertex's incident edges sorted in weight order; the weight distribution
// quantised into RtoW[RATIO_NUM]) plus the inputs of the statistics pass
// (Section 3: degrees for sumD and highD, highD(0) for the first step's hub
// bound, Section 3.3).
//
// Row layout: one 64-bit key per CSR entry, (weight << 32) | column, each row
// ascending -- the band filter of a push is then two binary searches.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"
#include "prep.h"

namespace sssp {

// ----------------------------------------------------------- validation --

__global__ void k_validate(const int32_t* rowptr, const int32_t* col, const uint32_t* w, int32_t n,
                           int32_t nnz, unsigned int* err, unsigned int* maxw, int* maxdeg,
                           unsigned int* minpos) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long v = t0; v < n; v += stride) {
    int a = rowptr[v], b = rowptr[v + 1];
    if (b < a) atomicOr(err, 1u);
    else atomicMax(maxdeg, b - a);
  }
  uint32_t mw = 0, mp = 0xffffffffu;
  bool bad = false;
  for (long long e = t0; e < nnz; e += stride) {
    int c = col[e];
    if (c < 0 || c >= n) bad = true;
    uint32_t x = w[e];
    mw = x > mw ? x : mw;
    if (x > 0u && x < mp) mp = x;
  }
  if (bad) atomicOr(err, 2u);
  if (mw) atomicMax(maxw, mw);
  if (mp != 0xffffffffu) atomicMin(minpos, mp);
}

__global__ void k_pack(const int32_t* col, const uint32_t* w, int32_t nnz, uint64_t* adj) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
       e += (long long)gridDim.x * blockDim.x)
    adj[e] = ((uint64_t)w[e] << 32) | (uint32_t)col[e];
}

// Relabelled packing: row u of the input becomes row new_of_old[u]; its
// columns are renamed the same way. One wave per input row.
__global__ void k_pack_relabel(const int32_t* rp_in, const int32_t* col, const uint32_t* w,
                               const int32_t* new_of_old, const int32_t* rowptr, int32_t n, uint64_t* adj) {
  const int lane = __lane_id();
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) / kWave;
  for (long long u = wave; u < n; u += nwaves) {
    const int a = rp_in[u], b = rp_in[u + 1];
    const long long dst = rowptr[new_of_old[u]];
    for (int e = a + lane; e < b; e += kWave)
      adj[dst + (e - a)] = ((uint64_t)w[e] << 32) | (uint32_t)new_of_old[col[e]];
  }
}

// ------------------------------------------------------- segmented sort --

// rows by length: 2..64 -> small, 65..kMedMax -> medium, longer -> large
constexpr int kMedMax = 4096;

// one atomic per wave and list (every lane of the wave calls it)
__device__ __forceinline__ int wave_slot(int32_t* counter, bool want) {
  uint64_t m = __ballot(want);
  if (m == 0) return -1;
  int leader = __ffsll((unsigned long long)m) - 1;
  int base = 0;
  if (__lane_id() == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader, kWave);
  return want ? base + __popcll(m & ((1ull << __lane_id()) - 1ull)) : -1;
}

__global__ void k_classify(const int32_t* rowptr, int32_t n, int32_t* small, int32_t* nsmall,
                           int32_t* medium, int32_t* nmed, int32_t* large, int32_t* nlarge) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long n_round = ((long long)n + stride - 1) / stride * stride;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n_round; v += stride) {
    int len = v < n ? rowptr[v + 1] - rowptr[v] : 0;
    int p0 = wave_slot(nsmall, len >= 2 && len <= 64);
    int p1 = wave_slot(nmed, len > 64 && len <= kMedMax);
    int p2 = wave_slot(nlarge, len > kMedMax);
    if (p0 >= 0) small[p0] = (int32_t)v;
    if (p1 >= 0) medium[p1] = (int32_t)v;
    if (p2 >= 0) large[p2] = (int32_t)v;
  }
}

// One wave per row of 2..64 keys: bitonic sort across lanes.
__global__ void k_sort_small(uint64_t* adj, const int32_t* rowptr, const int32_t* rows, int32_t nrows) {
  const int lane = __lane_id();
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = (gridDim.x * blockDim.x) / kWave;
  for (int r = wave; r < nrows; r += nwaves) {
    int v = rows[r];
    int a = rowptr[v], len = rowptr[v + 1] - a;
    uint64_t x = lane < len ? adj[a + lane] : ~0ull;
    for (int k = 2; k <= kWave; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        uint64_t y = __shfl_xor(x, j, kWave);
        bool up = ((lane & k) == 0);
        bool lower = ((lane & j) == 0);
        // lower lane keeps min when ascending
        uint64_t mn = x < y ? x : y, mx = x < y ? y : x;
        x = (lower == up) ? mn : mx;
      }
    }
    if (lane < len) adj[a + lane] = x;
  }
}

// One workgroup per segment of up to kMedMax keys: bitonic sort in LDS.
// Segments are given as (offset, length) pairs.
__global__ void __launch_bounds__(kBlock) k_sort_medium(uint64_t* adj, const int64_t* seg_off,
                                                        const int32_t* seg_len, int32_t nseg) {
  __shared__ uint64_t sh[kMedMax];
  for (int s = blockIdx.x; s < nseg; s += gridDim.x) {
    const int64_t a = seg_off[s];
    const int len = seg_len[s];
    int p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (int i = threadIdx.x; i < p2; i += kBlock) sh[i] = i < len ? adj[a + i] : ~0ull;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < p2; i += kBlock) {
          int ixj = i ^ j;
          if (ixj > i) {
            uint64_t x = sh[i], y = sh[ixj];
            bool up = (i & k) == 0;
            if ((x > y) == up) {
              sh[i] = y;
              sh[ixj] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < len; i += kBlock) adj[a + i] = sh[i];
    __syncthreads();
  }
}

// One merge pass over the large rows: runs of `width` keys merged pairwise
// from src into dst. A tile is 2048 outputs of one pair (width >= 4096 so a
// tile never straddles pairs); each thread merges 8 consecutive outputs found
// by a merge-path search (ties taken from the left run: stable).
constexpr int kMergePer = 8;
constexpr int kMergeTile = kBlock * kMergePer;

__global__ void __launch_bounds__(kBlock) k_merge_pass(const uint64_t* src, uint64_t* dst,
                                                       const int64_t* tile_row_off,
                                                       const int32_t* tile_row_len,
                                                       const int32_t* tile_out0, int32_t ntiles,
                                                       int32_t width) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t off = tile_row_off[t];
    const int len = tile_row_len[t];
    const int o0 = tile_out0[t];
    const long long pair0 = ((long long)o0 / (2ll * width)) * (2ll * width);
    const int a0 = (int)pair0;
    const int alen = max(0, min(width, len - a0));
    const int blen = max(0, min(width, len - a0 - width));
    const uint64_t* A = src + off + a0;
    const uint64_t* B = A + alen;
    const int diag = (o0 - a0) + threadIdx.x * kMergePer;
    const int total = alen + blen;
    if (diag < total) {
      int lo = max(0, diag - blen), hi = min(diag, alen);
      while (lo < hi) {
        int i = (lo + hi) >> 1;
        // take A[i] before B[diag-1-i]?  A[i] <= B[diag-1-i] means i is too small
        if (A[i] <= B[diag - 1 - i]) lo = i + 1; else hi = i;
      }
      int i = lo, j = diag - lo;
      uint64_t* out = dst + off + a0 + diag;
      for (int k = 0; k < kMergePer && diag + k < total; ++k) {
        bool takeA = (j >= blen) || (i < alen && A[i] <= B[j]);
        out[k] = takeA ? A[i++] : B[j++];
      }
    }
  }
}

__global__ void k_copy_segments(const uint64_t* src, uint64_t* dst, const int64_t* tile_row_off,
                                const int32_t* tile_row_len, const int32_t* tile_out0, int32_t ntiles) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t off = tile_row_off[t];
    const int len = tile_row_len[t];
    const int o0 = tile_out0[t];
    for (int k = threadIdx.x; k < kMergeTile && o0 + k < len; k += blockDim.x)
      dst[off + o0 + k] = src[off + o0 + k];
  }
}

// --------------------------------------------------------- symmetry check --
// (u, v, w) must occur in row v as (v, u, w) equally often. Each run of equal
// keys in row u is counted once against row v.
__device__ __forceinline__ bool sym_entry_ok(const int32_t* rowptr, const uint64_t* adj, int u, int a,
                                             int b, int e) {
  const uint64_t k = adj[e];
  if (e > a && adj[e - 1] == k) return true;
  int cu = 1;
  while (e + cu < b && adj[e + cu] == k) ++cu;
  const int v = (int)(uint32_t)(k & 0xffffffffull);
  const uint64_t kv = (k & 0xffffffff00000000ull) | (uint32_t)u;
  int lo = rowptr[v], hi = rowptr[v + 1];
  const int end = hi;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (adj[mid] < kv) lo = mid + 1; else hi = mid;
  }
  int cv = 0;
  while (lo + cv < end && adj[lo + cv] == kv) ++cv;
  return cv == cu;
}

// rows of at most 64 entries: one thread per row
__global__ void k_symcheck_short(const int32_t* rowptr, const uint64_t* adj, int32_t n, unsigned int* err) {
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (long long)gridDim.x * blockDim.x) {
    const int a = rowptr[u], b = rowptr[u + 1];
    if (b - a > 64) continue;
    for (int e = a; e < b; ++e)
      if (!sym_entry_ok(rowptr, adj, (int)u, a, b, e)) {
        atomicOr(err, 4u);
        return;
      }
  }
}

// listed longer rows: one workgroup per row
__global__ void k_symcheck_rows(const int32_t* rowptr, const uint64_t* adj, const int32_t* rows,
                                int32_t nrows, unsigned int* err) {
  for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int u = rows[r];
    const int a = rowptr[u], b = rowptr[u + 1];
    bool bad = false;
    for (int e = a + threadIdx.x; e < b; e += blockDim.x)
      if (!sym_entry_ok(rowptr, adj, u, a, b, e)) bad = true;
    if (bad) atomicOr(err, 4u);
  }
}

// ------------------------------------------------------- degree statistics --

constexpr int kDegDirect = 1 << 20;  // degrees below this are counted in an array
constexpr int kDegLds = 2048;

__global__ void __launch_bounds__(kBlock) k_deg_count(const int32_t* rowptr, int32_t n, uint32_t* cnt,
                                                      int32_t* big, int32_t* nbig) {
  __shared__ uint32_t sh[kDegLds];
  for (int i = threadIdx.x; i < kDegLds; i += kBlock) sh[i] = 0;
  __syncthreads();
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x) {
    int d = rowptr[v + 1] - rowptr[v];
    if (d < kDegLds) atomicAdd(&sh[d], 1u);
    else if (d < kDegDirect) atomicAdd(&cnt[d], 1u);
    else big[atomicAdd(nbig, 1)] = d;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDegLds; i += kBlock)
    if (sh[i]) atomicAdd(&cnt[i], sh[i]);
}

__global__ void k_deg_rank(const int32_t* rowptr, int32_t n, const int32_t* rank_small,
                           const int32_t* deg_vals, int32_t D, uint64_t* dinfo, uint32_t* wmin,
                           const uint64_t* adj) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x) {
    int a = rowptr[v];
    int d = rowptr[v + 1] - a;
    int r = -1;
    if (d >= 1 && d < kDegDirect) {
      r = rank_small[d];
    } else if (d >= kDegDirect) {
      int lo = 0, hi = D;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (deg_vals[mid] < d) lo = mid + 1; else hi = mid;
      }
      r = lo;
    }
    dinfo[v] = ((uint64_t)(uint32_t)r << 32) | (uint64_t)(uint32_t)d;
    wmin[v] = d > 0 ? (uint32_t)(adj[a] >> 32) : kInf;
  }
}

// Row index: per row, the first position of each weight bucket boundary, so
// that a weight range search starts inside a bucket of about deg/16 entries.
__global__ void k_row_index(const int32_t* rowptr, const uint64_t* adj, int32_t n, uint32_t width,
                            int32_t* rwi) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x) {
    const int rs = rowptr[v], re = rowptr[v + 1];
    if (re - rs <= kRowIndexMin) continue;
    int lo = rs;
    for (int b = 1; b < 16; ++b) {
      const unsigned long long t = (unsigned long long)b * width;
      int pos = re;
      if (t <= 0xffffffffull) {
        const uint64_t key = t << 32;
        int a = lo, c = re;  // positions only grow with b
        while (a < c) {
          const int mid = (a + c) >> 1;
          if (adj[mid] < key) a = mid + 1; else c = mid;
        }
        pos = a;
      }
      rwi[v * 16 + (b - 1)] = pos;
      lo = pos;
    }
    rwi[v * 16 + 15] = re;
  }
}

__global__ void k_hub_bits(const int32_t* rowptr, int32_t n, uint32_t hd, uint32_t* bits) {
  const int nw = (n + 31) / 32;
  const int thr = hd < 1u ? 1 : (int)hd;
  for (long long wd = (long long)blockIdx.x * blockDim.x + threadIdx.x; wd < nw;
       wd += (long long)gridDim.x * blockDim.x) {
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      long long v = wd * 32 + b;
      if (v < n && rowptr[v + 1] - rowptr[v] >= thr) word |= 1u << b;
    }
    bits[wd] = word;
  }
}

// Ordered compaction of the vertices with degree >= 1 into pull-list entries
// (id, smallest weight, row bounds): per-block counts, then per-block writes
// at the scanned offsets.
constexpr int kCompactPer = kBlock * 8;

__global__ void __launch_bounds__(kBlock) k_noniso_count(const int32_t* rowptr, int32_t n, int32_t* bcnt) {
  __shared__ int s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kCompactPer;
  int c = 0;
  for (int k = threadIdx.x; k < kCompactPer; k += kBlock) {
    long long v = base + k;
    if (v < n && rowptr[v + 1] > rowptr[v]) ++c;
  }
  atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) bcnt[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_noniso_write(const int32_t* rowptr, const uint32_t* wmin,
                                                         int32_t n, const int32_t* boff, UEntry* out) {
  __shared__ int wsum[kBlock / kWave];
  __shared__ int run;
  if (threadIdx.x == 0) run = boff[blockIdx.x];
  __syncthreads();
  const long long base = (long long)blockIdx.x * kCompactPer;
  for (int k0 = 0; k0 < kCompactPer; k0 += kBlock) {
    long long v = base + k0 + threadIdx.x;
    bool f = v < n && rowptr[v + 1] > rowptr[v];
    uint64_t m = __ballot(f);
    int lane = __lane_id(), wid = threadIdx.x / kWave;
    int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(m);
    __syncthreads();
    int woff = 0;
    for (int w2 = 0; w2 < wid; ++w2) woff += wsum[w2];
    if (f) {
      UEntry e;
      e.id = (int32_t)v;
      e.wmin = wmin[v];
      e.rs = rowptr[v];
      e.re = rowptr[v + 1];
      out[run + woff + pre] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int w2 = 0; w2 < kBlock / kWave; ++w2) t += wsum[w2];
      run += t;
    }
    __syncthreads();
  }
}

// The pull list's order: by the weight bucket of the smallest weight, then by
// id. A step's pull only concerns vertices whose lightest edge is below
// ub - st: a prefix of whole buckets, found in ufirst. Within a bucket the
// ascending ids keep the memory order of the rows and distances the pull
// reads (and of the frontier it produces).
__device__ __forceinline__ uint32_t ubucket(uint32_t wmin, uint32_t width) {
  return min(wmin / width, (uint32_t)(kUBuckets - 1));
}

__global__ void k_ukeys(const UEntry* e, int32_t cnt, uint32_t width, uint64_t* keys) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x)
    keys[i] = ((uint64_t)ubucket(e[i].wmin, width) << 32) | (uint32_t)e[i].id;
}

__global__ void k_uentries(const uint64_t* keys, int32_t cnt, const int32_t* rowptr, const uint32_t* wmin,
                           UEntry* out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    UEntry e;
    e.id = (int32_t)(uint32_t)(k & 0xffffffffull);
    e.wmin = wmin[e.id];
    e.rs = rowptr[e.id];
    e.re = rowptr[e.id + 1];
    out[i] = e;
  }
}

// ufirst[j] = first position in bucket j or later; the host fills every entry
// with cnt first (buckets past the last one present).
__global__ void k_ufirst(const uint64_t* keys, int32_t cnt, int32_t* ufirst) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(keys[i] >> 32);
    const int bp = i == 0 ? -1 : (int)(keys[i - 1] >> 32);
    for (int j = bp + 1; j <= b; ++j) ufirst[j] = (int32_t)i;
  }
}

// ----------------------------------------------------- weight quantiles --
// RtoW by radix selection over the packed keys' weights: three digit passes
// (bits 31..21, 20..10, 9..0). Each pass histograms the next digit of every
// weight whose higher bits match one of the active prefixes (sorted, one per
// quantile still undecided).

__global__ void __launch_bounds__(kBlock) k_wdigit_hist(const uint64_t* adj, int32_t nnz, int shift_hi,
                                                        int shift_lo, int digit_bits,
                                                        const uint32_t* prefixes, int32_t nprefix,
                                                        uint32_t* hist /* nprefix << digit_bits */) {
  // LDS-privatised when every bin fits (up to 8K bins)
  __shared__ uint32_t sh[8192];
  __shared__ uint32_t sp[4096];
  const int nbins = nprefix << digit_bits;
  const bool priv = nbins <= 8192;
  for (int i = threadIdx.x; i < nprefix && i < 4096; i += kBlock) sp[i] = prefixes[i];
  if (priv)
    for (int i = threadIdx.x; i < nbins; i += kBlock) sh[i] = 0;
  __syncthreads();
  const uint32_t dmask = (1u << digit_bits) - 1u;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
       e += (long long)gridDim.x * blockDim.x) {
    uint32_t w = (uint32_t)(adj[e] >> 32);
    uint32_t pre = shift_hi >= 32 ? 0u : (w >> shift_hi);
    int lo = 0, hi = nprefix;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (sp[mid] < pre) lo = mid + 1; else hi = mid;
    }
    if (lo < nprefix && sp[lo] == pre) {
      uint32_t dg = (w >> shift_lo) & dmask;
      int bin = (lo << digit_bits) | (int)dg;
      if (priv) atomicAdd(&sh[bin], 1u); else atomicAdd(&hist[bin], 1u);
    }
  }
  if (priv) {
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += kBlock)
      if (sh[i]) atomicAdd(&hist[i], sh[i]);
  }
}


// ================================================================ host side

namespace {

struct Alloc {
  GraphHost* g;
  bool ok = true;
  template <typename T>
  T* get(size_t count) {
    void* p = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    g->allocs.push_back(p);
    g->bytes += bytes;
    return static_cast<T*>(p);
  }
};

// scratch device buffer freed at scope exit
struct Scratch {
  std::vector<void*> ptrs;
  bool ok = true;
  template <typename T>
  T* get(size_t count) {
    void* p = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

int grid_for(long long work, int per_block = kBlock, int cap = 8192) {
  long long b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

#define PREP_CHECK(expr)                                      \
  do {                                                        \
    hipError_t _e = (expr);                                   \
    if (_e != hipSuccess) {                                   \
      *msg = std::string(#expr) + ": " + hipGetErrorString(_e); \
      return -6;                                              \
    }                                                         \
  } while (0)

}  // namespace

// The vertices moved to the front of the internal order: degree at least
// max(kHubMinDegree, 4 x the mean degree), at most kHubPrefixMax of them (the
// highest degrees), by descending degree, ties by id. Empty when no vertex
// qualifies (uniform-degree graphs such as grids and G(n, m) keep their order).
std::vector<int32_t> hub_prefix(const std::vector<int32_t>& rp, int32_t n, int32_t nnz) {
  std::vector<int32_t> out;
  if (n < 2 || nnz == 0) return out;
  const long long thr = std::max<long long>(kHubMinDegree, 4ll * nnz / n);
  for (int32_t u = 0; u < n; ++u)
    if (rp[(size_t)u + 1] - rp[(size_t)u] >= thr) out.push_back(u);
  std::sort(out.begin(), out.end(), [&](int32_t a, int32_t b) {
    const int32_t da = rp[(size_t)a + 1] - rp[(size_t)a], db = rp[(size_t)b + 1] - rp[(size_t)b];
    return da != db ? da > db : a < b;
  });
  if (out.size() > (size_t)kHubPrefixMax) out.resize((size_t)kHubPrefixMax);
  return out;
}

void free_graph(GraphHost* g) {
  for (void* p : g->allocs) (void)hipFree(p);
  g->allocs.clear();
  g->d = nullptr;
}

int prep_graph(int32_t n, const int32_t* rowptr_in, const int32_t* col_in, const uint32_t* w_in,
               int flags, GraphHost* out, std::string* msg) {
  if (n < 1 || rowptr_in == nullptr) {
    *msg = "n must be >= 1 and rowptr non-NULL";
    return -1;
  }
  PREP_CHECK(hipGetDevice(&out->device));
  // host copy of rowptr (needed to plan the sort of long rows)
  std::vector<int32_t> rp((size_t)n + 1);
  const bool rp_dev = is_device_ptr(rowptr_in);
  PREP_CHECK(hipMemcpy(rp.data(), rowptr_in, sizeof(int32_t) * ((size_t)n + 1),
                       rp_dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
  if (rp[0] != 0 || rp[(size_t)n] < 0) {
    *msg = "rowptr[0] must be 0 and rowptr[n] >= 0";
    return -1;
  }
  const int32_t nnz = rp[(size_t)n];
  if (nnz > 0 && (col_in == nullptr || w_in == nullptr)) {
    *msg = "colidx and weight must be non-NULL when nnz > 0";
    return -1;
  }
  Alloc A{out};
  Scratch T;
  int32_t* rowptr = A.get<int32_t>((size_t)n + 1);
  uint64_t* adj = A.get<uint64_t>((size_t)nnz);
  uint32_t* wmin = A.get<uint32_t>((size_t)n);
  uint64_t* dinfo = A.get<uint64_t>((size_t)n);
  uint32_t* hub = A.get<uint32_t>(((size_t)n + 31) / 32);
  uint32_t* rtow = A.get<uint32_t>(kRatioNum);
  int32_t* rwi = A.get<int32_t>((size_t)n * 16);
  if (!A.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  PREP_CHECK(hipMemcpy(rowptr, rp.data(), sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
  unsigned int* d_flags = T.get<unsigned int>(4);
  int* d_int = T.get<int>(8);
  if (!T.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  PREP_CHECK(hipMemset(d_flags, 0, sizeof(unsigned int) * 4));
  PREP_CHECK(hipMemset(d_int, 0, sizeof(int) * 8));
  uint32_t maxw = 0;
  uint32_t minpos = 0xffffffffu;  // smallest positive weight
  int maxdeg = 0;
  int32_t* new_of_old = nullptr;  // set when the vertices are renumbered hub-first
  int32_t* old_of_new = nullptr;
  int32_t relabelled = 0;
  if (nnz > 0) {
    int32_t* col = T.get<int32_t>((size_t)nnz);
    uint32_t* w = T.get<uint32_t>((size_t)nnz);
    if (!T.ok) {
      *msg = "device allocation failed";
      return -5;
    }
    PREP_CHECK(hipMemcpy(col, col_in, sizeof(int32_t) * (size_t)nnz, hipMemcpyDefault));
    PREP_CHECK(hipMemcpy(w, w_in, sizeof(uint32_t) * (size_t)nnz, hipMemcpyDefault));
    const unsigned int none = 0xffffffffu;
    PREP_CHECK(hipMemcpy(d_flags + 2, &none, sizeof(none), hipMemcpyHostToDevice));
    k_validate<<<grid_for(std::max<long long>(n, nnz)), kBlock>>>(rowptr, col, w, n, nnz, d_flags,
                                                                  d_flags + 1, d_int, d_flags + 2);
    PREP_CHECK(hipGetLastError());
    unsigned int hf[3];
    PREP_CHECK(hipMemcpy(hf, d_flags, sizeof(hf), hipMemcpyDeviceToHost));
    minpos = hf[2];
    PREP_CHECK(hipMemcpy(&maxdeg, d_int, sizeof(int), hipMemcpyDeviceToHost));
    if (hf[0] & 1u) {
      *msg = "rowptr is not non-decreasing";
      return -1;
    }
    if (hf[0] & 2u) {
      *msg = "colidx out of range";
      return -1;
    }
    maxw = hf[1];
    // binary32 weights: the largest bit pattern is below +inf exactly when
    // every weight is finite and non-negative (the sign bit set is above it)
    if ((flags & 2) && maxw >= 0x7f800000u) {
      *msg = "binary32 weights must be finite and non-negative";
      return -1;
    }
    // Hub-first vertex order (internal ids): on a skewed graph the rows of at
    // least 4x the mean degree (the vertices most relaxations land on) are
    // moved to the front, by descending degree, so that their distance words
    // share cache lines; the other vertices keep their order. Callers see
    // their own ids: sources and targets are renamed on the way in, distances
    // and parents on the way out.
    std::vector<int32_t> prefix = hub_prefix(rp, n, nnz);
    if (!prefix.empty()) {
      const int32_t H = (int32_t)prefix.size();
      std::vector<int32_t> n_of_o((size_t)n), o_of_n((size_t)n);
      std::vector<char> in_prefix((size_t)n, 0);
      for (int32_t i = 0; i < H; ++i) {
        n_of_o[(size_t)prefix[(size_t)i]] = i;
        in_prefix[(size_t)prefix[(size_t)i]] = 1;
      }
      int32_t next = H;
      for (int32_t u = 0; u < n; ++u)
        if (!in_prefix[(size_t)u]) n_of_o[(size_t)u] = next++;
      for (int32_t u = 0; u < n; ++u) o_of_n[(size_t)n_of_o[(size_t)u]] = u;
      std::vector<int32_t> rp_new((size_t)n + 1);
      rp_new[0] = 0;
      for (int32_t r = 0; r < n; ++r) {
        const int32_t u = o_of_n[(size_t)r];
        rp_new[(size_t)r + 1] = rp_new[(size_t)r] + (rp[(size_t)u + 1] - rp[(size_t)u]);
      }
      int32_t* d_rp_in = T.get<int32_t>((size_t)n + 1);
      new_of_old = A.get<int32_t>((size_t)n);
      old_of_new = A.get<int32_t>((size_t)n);
      if (!T.ok || !A.ok) {
        *msg = "device allocation failed";
        return -5;
      }
      PREP_CHECK(hipMemcpy(d_rp_in, rp.data(), sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
      PREP_CHECK(hipMemcpy(new_of_old, n_of_o.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
      PREP_CHECK(hipMemcpy(old_of_new, o_of_n.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
      PREP_CHECK(hipMemcpy(rowptr, rp_new.data(), sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
      k_pack_relabel<<<grid_for((long long)n * kWave), kBlock>>>(d_rp_in, col, w, new_of_old, rowptr, n, adj);
      PREP_CHECK(hipGetLastError());
      rp.swap(rp_new);
      relabelled = H;
    } else {
      k_pack<<<grid_for(nnz), kBlock>>>(col, w, nnz, adj);
      PREP_CHECK(hipGetLastError());
    }
  } else {
    for (int32_t v = 0; v < n; ++v)
      if (rp[(size_t)v + 1] < rp[(size_t)v]) {
        *msg = "rowptr is not non-decreasing";
        return -1;
      }
  }

  // ---- per-row sort by (weight, column)
  if (nnz > 0) {
    int32_t* small = T.get<int32_t>((size_t)n);
    int32_t* medium = T.get<int32_t>((size_t)n);
    int32_t* large = T.get<int32_t>((size_t)n);
    if (!T.ok) {
      *msg = "device allocation failed";
      return -5;
    }
    PREP_CHECK(hipMemset(d_int, 0, sizeof(int) * 8));
    k_classify<<<grid_for(n), kBlock>>>(rowptr, n, small, d_int, medium, d_int + 1, large, d_int + 2);
    PREP_CHECK(hipGetLastError());
    int cnts[3];
    PREP_CHECK(hipMemcpy(cnts, d_int, sizeof(cnts), hipMemcpyDeviceToHost));
    if (cnts[0] > 0) {
      k_sort_small<<<grid_for((long long)cnts[0] * kWave), kBlock>>>(adj, rowptr, small, cnts[0]);
      PREP_CHECK(hipGetLastError());
    }
    // medium rows and the 4096-key chunks of large rows share one sort
    std::vector<int32_t> lrows((size_t)cnts[2]);
    if (cnts[2] > 0)
      PREP_CHECK(hipMemcpy(lrows.data(), large, sizeof(int32_t) * (size_t)cnts[2], hipMemcpyDeviceToHost));
    std::vector<int32_t> mrows((size_t)cnts[1]);
    if (cnts[1] > 0)
      PREP_CHECK(hipMemcpy(mrows.data(), medium, sizeof(int32_t) * (size_t)cnts[1], hipMemcpyDeviceToHost));
    std::vector<int64_t> soff;
    std::vector<int32_t> slen;
    soff.reserve(mrows.size());
    for (int32_t v : mrows) {
      soff.push_back(rp[(size_t)v]);
      slen.push_back(rp[(size_t)v + 1] - rp[(size_t)v]);
    }
    int maxlarge = 0;
    for (int32_t v : lrows) {
      int64_t a = rp[(size_t)v];
      int len = rp[(size_t)v + 1] - rp[(size_t)v];
      maxlarge = std::max(maxlarge, len);
      for (int c = 0; c < len; c += kMedMax) {
        soff.push_back(a + c);
        slen.push_back(std::min(kMedMax, len - c));
      }
    }
    if (!soff.empty()) {
      int64_t* d_off = T.get<int64_t>(soff.size());
      int32_t* d_len = T.get<int32_t>(slen.size());
      if (!T.ok) {
        *msg = "device allocation failed";
        return -5;
      }
      PREP_CHECK(hipMemcpy(d_off, soff.data(), sizeof(int64_t) * soff.size(), hipMemcpyHostToDevice));
      PREP_CHECK(hipMemcpy(d_len, slen.data(), sizeof(int32_t) * slen.size(), hipMemcpyHostToDevice));
      k_sort_medium<<<grid_for((long long)soff.size(), 1, 65536), kBlock>>>(adj, d_off, d_len,
                                                                            (int32_t)soff.size());
      PREP_CHECK(hipGetLastError());
    }
    if (!lrows.empty()) {
      // merge passes over the large rows, ping-pong adj <-> tmp
      std::vector<int64_t> toff;
      std::vector<int32_t> tlen, to0;
      for (int32_t v : lrows) {
        int len = rp[(size_t)v + 1] - rp[(size_t)v];
        for (int o = 0; o < len; o += kMergeTile) {
          toff.push_back(rp[(size_t)v]);
          tlen.push_back(len);
          to0.push_back(o);
        }
      }
      uint64_t* tmp = T.get<uint64_t>((size_t)nnz);
      int64_t* d_toff = T.get<int64_t>(toff.size());
      int32_t* d_tlen = T.get<int32_t>(tlen.size());
      int32_t* d_to0 = T.get<int32_t>(to0.size());
      if (!T.ok) {
        *msg = "device allocation failed";
        return -5;
      }
      PREP_CHECK(hipMemcpy(d_toff, toff.data(), sizeof(int64_t) * toff.size(), hipMemcpyHostToDevice));
      PREP_CHECK(hipMemcpy(d_tlen, tlen.data(), sizeof(int32_t) * tlen.size(), hipMemcpyHostToDevice));
      PREP_CHECK(hipMemcpy(d_to0, to0.data(), sizeof(int32_t) * to0.size(), hipMemcpyHostToDevice));
      const int nt = (int)toff.size();
      uint64_t* src = adj;
      uint64_t* dst = tmp;
      for (long long width = kMedMax; width < maxlarge; width *= 2) {
        k_merge_pass<<<grid_for(nt, 1, 65536), kBlock>>>(src, dst, d_toff, d_tlen, d_to0, nt, (int32_t)width);
        PREP_CHECK(hipGetLastError());
        std::swap(src, dst);
      }
      if (src != adj) {
        k_copy_segments<<<grid_for(nt, 1, 65536), kBlock>>>(src, adj, d_toff, d_tlen, d_to0, nt);
        PREP_CHECK(hipGetLastError());
      }
    }
    PREP_CHECK(hipDeviceSynchronize());
    // ---- symmetry
    if (!(flags & 1)) {
      PREP_CHECK(hipMemset(d_flags, 0, sizeof(unsigned int)));
      k_symcheck_short<<<grid_for(n), kBlock>>>(rowptr, adj, n, d_flags);
      PREP_CHECK(hipGetLastError());
      if (cnts[1] > 0) {
        k_symcheck_rows<<<grid_for(cnts[1], 1, 65536), kBlock>>>(rowptr, adj, medium, cnts[1], d_flags);
        PREP_CHECK(hipGetLastError());
      }
      if (cnts[2] > 0) {
        k_symcheck_rows<<<grid_for(cnts[2], 1, 65536), kBlock>>>(rowptr, adj, large, cnts[2], d_flags);
        PREP_CHECK(hipGetLastError());
      }
      unsigned int hf;
      PREP_CHECK(hipMemcpy(&hf, d_flags, sizeof(hf), hipMemcpyDeviceToHost));
      if (hf & 4u) {
        *msg = "the CSR is not symmetric: some (u, v, w) lacks its (v, u, w)";
        return -2;
      }
    }
  }

  // ---- degree statistics
  uint32_t* cnt = T.get<uint32_t>(kDegDirect);
  int32_t* big = T.get<int32_t>(std::max<size_t>(1, (size_t)nnz / kDegDirect + 1));
  if (!T.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  PREP_CHECK(hipMemset(cnt, 0, sizeof(uint32_t) * kDegDirect));
  PREP_CHECK(hipMemset(d_int, 0, sizeof(int) * 8));
  k_deg_count<<<grid_for(n), kBlock>>>(rowptr, n, cnt, big, d_int);
  PREP_CHECK(hipGetLastError());
  std::vector<uint32_t> hcnt(kDegDirect);
  PREP_CHECK(hipMemcpy(hcnt.data(), cnt, sizeof(uint32_t) * kDegDirect, hipMemcpyDeviceToHost));
  int nbig = 0;
  PREP_CHECK(hipMemcpy(&nbig, d_int, sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int32_t> hbig((size_t)nbig);
  if (nbig > 0) PREP_CHECK(hipMemcpy(hbig.data(), big, sizeof(int32_t) * (size_t)nbig, hipMemcpyDeviceToHost));
  std::sort(hbig.begin(), hbig.end());
  std::vector<int32_t> deg_vals;
  std::vector<uint32_t> deg_cnt;
  std::vector<int32_t> rank_small(kDegDirect, -1);
  for (int d = 1; d < kDegDirect; ++d)
    if (hcnt[(size_t)d]) {
      rank_small[(size_t)d] = (int32_t)deg_vals.size();
      deg_vals.push_back(d);
      deg_cnt.push_back(hcnt[(size_t)d]);
    }
  for (size_t i = 0; i < hbig.size(); ++i) {
    if (i > 0 && hbig[i] == hbig[i - 1]) {
      deg_cnt.back() += 1;
    } else {
      deg_vals.push_back(hbig[i]);
      deg_cnt.push_back(1);
    }
  }
  const int32_t D = (int32_t)deg_vals.size();
  int32_t* d_deg_vals = A.get<int32_t>(std::max<int32_t>(D, 1));
  uint32_t* d_deg_cnt = A.get<uint32_t>(std::max<int32_t>(D, 1));
  int32_t* d_rank_small = T.get<int32_t>(kDegDirect);
  if (!A.ok || !T.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  if (D > 0) {
    PREP_CHECK(hipMemcpy(d_deg_vals, deg_vals.data(), sizeof(int32_t) * (size_t)D, hipMemcpyHostToDevice));
    PREP_CHECK(hipMemcpy(d_deg_cnt, deg_cnt.data(), sizeof(uint32_t) * (size_t)D, hipMemcpyHostToDevice));
  }
  PREP_CHECK(hipMemcpy(d_rank_small, rank_small.data(), sizeof(int32_t) * kDegDirect, hipMemcpyHostToDevice));
  k_deg_rank<<<grid_for(n), kBlock>>>(rowptr, n, d_rank_small, d_deg_vals, D, dinfo, wmin, adj);
  PREP_CHECK(hipGetLastError());
  uint32_t* d_h = T.get<uint32_t>(1);
  unsigned long long* d_mass = T.get<unsigned long long>(1);
  if (!T.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  PREP_CHECK(launch_high_d(d_deg_vals, d_deg_cnt, D, d_h, d_mass, 0));
  uint32_t high_d0 = 0;
  unsigned long long mass0 = 0;
  PREP_CHECK(hipMemcpy(&high_d0, d_h, sizeof(uint32_t), hipMemcpyDeviceToHost));
  PREP_CHECK(hipMemcpy(&mass0, d_mass, sizeof(unsigned long long), hipMemcpyDeviceToHost));
  if (mass0 != (unsigned long long)nnz) {
    *msg = "internal: degree mass mismatch";
    return -6;
  }
  k_hub_bits<<<grid_for((n + 31) / 32), kBlock>>>(rowptr, n, high_d0, hub);
  PREP_CHECK(hipGetLastError());
  const uint32_t rwi_width = (uint32_t)(((unsigned long long)maxw + 16ull) / 16ull);
  k_row_index<<<grid_for(n), kBlock>>>(rowptr, adj, n, rwi_width, rwi);
  PREP_CHECK(hipGetLastError());
  // non-isolated vertices in ascending order
  const int nb = (int)(((long long)n + kCompactPer - 1) / kCompactPer);
  int32_t* bcnt = T.get<int32_t>((size_t)nb);
  if (!T.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  k_noniso_count<<<nb, kBlock>>>(rowptr, n, bcnt);
  PREP_CHECK(hipGetLastError());
  std::vector<int32_t> hb((size_t)nb);
  PREP_CHECK(hipMemcpy(hb.data(), bcnt, sizeof(int32_t) * (size_t)nb, hipMemcpyDeviceToHost));
  int32_t run = 0;
  for (int i = 0; i < nb; ++i) {
    int32_t c = hb[(size_t)i];
    hb[(size_t)i] = run;
    run += c;
  }
  const int32_t nonisolated = run;
  UEntry* noniso = A.get<UEntry>(std::max<int32_t>(nonisolated, 1));
  if (!A.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  PREP_CHECK(hipMemcpy(bcnt, hb.data(), sizeof(int32_t) * (size_t)nb, hipMemcpyHostToDevice));
  k_noniso_write<<<nb, kBlock>>>(rowptr, wmin, n, bcnt, noniso);
  PREP_CHECK(hipGetLastError());
  // ...then ordered by (weight bucket of the smallest weight, id): 4096-key
  // chunks sorted in LDS, then merge passes over the whole list
  uint32_t ub_width = (uint32_t)(((unsigned long long)maxw + kUBucketDiv) / kUBucketDiv);
  if (flags & 2) {
    // binary32: bucket 0 = lightest edge below maxW / kUBucketDiv in value
    float f;
    std::memcpy(&f, &maxw, sizeof f);
    f /= (float)kUBucketDiv;
    std::memcpy(&ub_width, &f, sizeof f);
    if (ub_width == 0) ub_width = 1;
  }
  int32_t* ufirst = A.get<int32_t>(kUBuckets + 1);
  if (!A.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  {
    std::vector<int32_t> hf((size_t)kUBuckets + 1, nonisolated);
    PREP_CHECK(hipMemcpy(ufirst, hf.data(), sizeof(int32_t) * hf.size(), hipMemcpyHostToDevice));
  }
  if (nonisolated > 0) {
    uint64_t* keys = T.get<uint64_t>((size_t)nonisolated);
    uint64_t* ktmp = T.get<uint64_t>((size_t)nonisolated);
    std::vector<int64_t> coff, toff;
    std::vector<int32_t> clen, tlen, to0;
    for (int32_t c = 0; c < nonisolated; c += kMedMax) {
      coff.push_back(c);
      clen.push_back(std::min(kMedMax, nonisolated - c));
    }
    for (int32_t o = 0; o < nonisolated; o += kMergeTile) {
      toff.push_back(0);
      tlen.push_back(nonisolated);
      to0.push_back(o);
    }
    int64_t* d_coff = T.get<int64_t>(coff.size());
    int32_t* d_clen = T.get<int32_t>(clen.size());
    int64_t* d_toff = T.get<int64_t>(toff.size());
    int32_t* d_tlen = T.get<int32_t>(tlen.size());
    int32_t* d_to0 = T.get<int32_t>(to0.size());
    if (!T.ok) {
      *msg = "device allocation failed";
      return -5;
    }
    PREP_CHECK(hipMemcpy(d_coff, coff.data(), sizeof(int64_t) * coff.size(), hipMemcpyHostToDevice));
    PREP_CHECK(hipMemcpy(d_clen, clen.data(), sizeof(int32_t) * clen.size(), hipMemcpyHostToDevice));
    PREP_CHECK(hipMemcpy(d_toff, toff.data(), sizeof(int64_t) * toff.size(), hipMemcpyHostToDevice));
    PREP_CHECK(hipMemcpy(d_tlen, tlen.data(), sizeof(int32_t) * tlen.size(), hipMemcpyHostToDevice));
    PREP_CHECK(hipMemcpy(d_to0, to0.data(), sizeof(int32_t) * to0.size(), hipMemcpyHostToDevice));
    k_ukeys<<<grid_for(nonisolated), kBlock>>>(noniso, nonisolated, ub_width, keys);
    PREP_CHECK(hipGetLastError());
    k_sort_medium<<<grid_for((long long)coff.size(), 1, 65536), kBlock>>>(keys, d_coff, d_clen,
                                                                          (int32_t)coff.size());
    PREP_CHECK(hipGetLastError());
    uint64_t* src = keys;
    uint64_t* dst = ktmp;
    const int nt = (int)toff.size();
    for (long long width = kMedMax; width < nonisolated; width *= 2) {
      k_merge_pass<<<grid_for(nt, 1, 65536), kBlock>>>(src, dst, d_toff, d_tlen, d_to0, nt, (int32_t)width);
      PREP_CHECK(hipGetLastError());
      std::swap(src, dst);
    }
    k_uentries<<<grid_for(nonisolated), kBlock>>>(src, nonisolated, rowptr, wmin, noniso);
    PREP_CHECK(hipGetLastError());
    k_ufirst<<<grid_for(nonisolated), kBlock>>>(src, nonisolated, ufirst);
    PREP_CHECK(hipGetLastError());
    PREP_CHECK(hipDeviceSynchronize());
  }

  // ---- RtoW[x] = maxW(G, x / 4095): the ceil(x * nnz / 4095)-th smallest weight
  std::vector<uint32_t> hr(kRatioNum, 0);
  if (nnz > 0) {
    std::vector<uint64_t> rank(kRatioNum);
    for (int x = 0; x < kRatioNum; ++x) {
      uint64_t need = ((uint64_t)x * (uint64_t)nnz + (kRatioNum - 2)) / (kRatioNum - 1);
      rank[(size_t)x] = need > 0 ? need - 1 : 0;
    }
    std::vector<uint32_t> prefix(kRatioNum, 0);  // decided high bits per quantile
    const int shifts_hi[3] = {32, 21, 10};
    const int shifts_lo[3] = {21, 10, 0};
    const int bits[3] = {11, 11, 10};
    uint32_t* d_pref = T.get<uint32_t>(kRatioNum);
    uint32_t* d_hist = T.get<uint32_t>((size_t)kRatioNum << 11);
    if (!T.ok) {
      *msg = "device allocation failed";
      return -5;
    }
    for (int pass = 0; pass < 3; ++pass) {
      std::vector<uint32_t> act(prefix.begin(), prefix.end());
      std::sort(act.begin(), act.end());
      act.erase(std::unique(act.begin(), act.end()), act.end());
      const int np = (int)act.size();
      const size_t nbins = (size_t)np << bits[pass];
      PREP_CHECK(hipMemcpy(d_pref, act.data(), sizeof(uint32_t) * (size_t)np, hipMemcpyHostToDevice));
      PREP_CHECK(hipMemset(d_hist, 0, sizeof(uint32_t) * nbins));
      k_wdigit_hist<<<grid_for(nnz, kBlock, 4096), kBlock>>>(adj, nnz, shifts_hi[pass], shifts_lo[pass],
                                                             bits[pass], d_pref, np, d_hist);
      PREP_CHECK(hipGetLastError());
      std::vector<uint32_t> hh(nbins);
      PREP_CHECK(hipMemcpy(hh.data(), d_hist, sizeof(uint32_t) * nbins, hipMemcpyDeviceToHost));
      for (int x = 0; x < kRatioNum; ++x) {
        size_t slot = (size_t)(std::lower_bound(act.begin(), act.end(), prefix[(size_t)x]) - act.begin());
        const uint32_t* h = hh.data() + (slot << bits[pass]);
        uint64_t r = rank[(size_t)x];
        uint32_t dg = 0;
        for (;; ++dg) {
          if (r < h[dg]) break;
          r -= h[dg];
        }
        rank[(size_t)x] = r;
        prefix[(size_t)x] = (prefix[(size_t)x] << bits[pass]) | dg;
      }
    }
    for (int x = 0; x < kRatioNum; ++x) hr[(size_t)x] = prefix[(size_t)x];
  }
  PREP_CHECK(hipMemcpy(rtow, hr.data(), sizeof(uint32_t) * kRatioNum, hipMemcpyHostToDevice));

  DevGraph& h = out->h;
  h.n = n;
  h.nnz = nnz;
  h.max_w = maxw;
  h.high_d0 = high_d0;
  h.num_deg = D;
  h.n_nonisolated = nonisolated;
  h.max_deg = maxdeg;
  h.rowptr = rowptr;
  h.adj = adj;
  h.wmin = wmin;
  h.dinfo = dinfo;
  h.deg_vals = d_deg_vals;
  h.deg_cnt0 = d_deg_cnt;
  h.hub_bits = hub;
  h.nonisolated = noniso;
  h.ufirst = ufirst;
  h.ubucket_width = ub_width;
  h.float_w = (flags & 2) ? 1u : 0u;
  h.min_pos_w = minpos;
  {
    int64_t hr = 0;
    for (int32_t i = 0; i < D; ++i)
      if (deg_vals[(size_t)i] > kDefaultHeavy) hr += deg_cnt[(size_t)i];
    h.heavy_rows = (int32_t)hr;
  }
  h.rtow = rtow;
  h.rwi = rwi;
  h.rwi_width = rwi_width;
  h.new_of_old = new_of_old;
  h.old_of_new = old_of_new;
  h.relabelled = relabelled;
  out->d = A.get<DevGraph>(1);
  if (!A.ok) {
    *msg = "device allocation failed";
    return -5;
  }
  PREP_CHECK(hipMemcpy(out->d, &h, sizeof(DevGraph), hipMemcpyHostToDevice));
  PREP_CHECK(hipDeviceSynchronize());
  out->nonisolated = nonisolated;
  out->distinct_degrees = D;
  out->max_degree = maxdeg;
  return 0;
}

}  // namespace sssp
