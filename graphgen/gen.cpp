// Seeded synthetic graph generators and edge-list -> CSR cleaning.
//
// This file produces inputs only. It holds none of the shortest-path method's
// arithmetic: no distances, no statistics, no schedule. Both the oracle and the
// GPU library consume what it writes (the oracle the raw undirected edge list,
// the GPU library the cleaned symmetric CSR).
//
// Random numbers come from one counter-based generator: the SplitMix64 output
// function (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) applied to key + (counter+1) * golden-gamma.
// Every draw is addressed by (seed, stream, counter), so any slice of an edge
// list can be regenerated on its own and the output does not depend on the
// number of threads.
//
// Generators (the paper's workloads, Section 4.2, stood in for by synthetic
// graphs of the same shape):
//   R-MAT      recursive quadrant descent with probabilities (a, b, c, d),
//              then a seeded random relabelling of the vertices
//   G(n, m)    m endpoint pairs drawn uniformly (an Erdos-Renyi multigraph)
//   grid       rows x cols 4-neighbour lattice, each edge kept with p_keep,
//              plus a (r,c)-(r+1,c+1) diagonal kept with p_diag
// Weights are 1 + floor(u * W) for a 53-bit uniform u, i.e. uniform on 1..W.
//
// Cleaning (edges_to_csr): self-loops are dropped, each undirected edge is
// stored in both rows, rows are sorted by column, and parallel edges are
// merged keeping the minimum weight (multigraph semantics).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed * kGamma + mix64(stream + 0x632BE59BD9B4E019ULL));
}

inline uint64_t draw(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * kGamma); }

// uniform integer in [0, bound) by 64x64 -> high 64 multiply (Lemire)
inline uint64_t below(uint64_t r, uint64_t bound) {
  return (uint64_t)(((__uint128_t)r * (__uint128_t)bound) >> 64);
}

inline uint32_t weight_from(uint64_t r, uint32_t wmax) {
  double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
  uint64_t w = 1 + (uint64_t)(u * (double)wmax);
  if (w > wmax) w = wmax;
  return (uint32_t)w;
}

enum : uint64_t { kStreamEdge = 1, kStreamPerm = 2, kStreamWeight = 3, kStreamSource = 4 };

}  // namespace

extern "C" {

// Fisher-Yates permutation of 0..n-1 drawn from (seed, kStreamPerm).
void gg_permutation(int64_t n, uint64_t seed, int32_t* perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  uint64_t key = stream_key(seed, kStreamPerm);
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)below(draw(key, (uint64_t)i), (uint64_t)(i + 1));
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

// R-MAT edge list: m = edge_factor << scale undirected edges. Quadrant per
// level from one 32-bit uniform: [0,a) -> (0,0), [a,a+b) -> (0,1),
// [a+b,a+b+c) -> (1,0), else (1,1); most significant bit first. Vertex ids
// are then relabelled by a seeded permutation when relabel != 0.
int gg_rmat(int32_t scale, int64_t edge_factor, double a, double b, double c, uint32_t wmax,
            uint64_t seed, int32_t relabel, int32_t* src, int32_t* dst, uint32_t* w) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || wmax < 1) return -1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edge_factor << scale;
  const double two32 = 4294967296.0;
  const uint64_t ta = (uint64_t)(a * two32);
  const uint64_t tab = (uint64_t)((a + b) * two32);
  const uint64_t tabc = (uint64_t)((a + b + c) * two32);
  const uint64_t ekey = stream_key(seed, kStreamEdge);
  const uint64_t wkey = stream_key(seed, kStreamWeight);
  std::vector<int32_t> perm;
  if (relabel) {
    perm.resize((size_t)n);
    gg_permutation(n, seed, perm.data());
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t s = 0, d = 0;
    uint64_t r = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
      uint64_t u;
      if ((lvl & 1) == 0) {
        r = draw(ekey, (uint64_t)i * 16 + (uint64_t)(lvl >> 1));
        u = r >> 32;
      } else {
        u = r & 0xffffffffULL;
      }
      uint32_t sb, db;
      if (u < ta) { sb = 0; db = 0; }
      else if (u < tab) { sb = 0; db = 1; }
      else if (u < tabc) { sb = 1; db = 0; }
      else { sb = 1; db = 1; }
      s = (s << 1) | sb;
      d = (d << 1) | db;
    }
    if (relabel) {
      s = (uint32_t)perm[s];
      d = (uint32_t)perm[d];
    }
    src[i] = (int32_t)s;
    dst[i] = (int32_t)d;
    w[i] = weight_from(draw(wkey, (uint64_t)i), wmax);
  }
  return 0;
}

// Degrees of the R-MAT multigraph (self-loops dropped, parallel edges
// counted) without storing the edge list: deg[v] for v < 2^scale.
int gg_rmat_degrees(int32_t scale, int64_t edge_factor, double a, double b, double c,
                    uint64_t seed, int32_t relabel, int64_t* deg) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return -1;
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edge_factor << scale;
  const double two32 = 4294967296.0;
  const uint64_t ta = (uint64_t)(a * two32);
  const uint64_t tab = (uint64_t)((a + b) * two32);
  const uint64_t tabc = (uint64_t)((a + b + c) * two32);
  const uint64_t ekey = stream_key(seed, kStreamEdge);
  std::vector<int32_t> perm;
  if (relabel) {
    perm.resize((size_t)n);
    gg_permutation(n, seed, perm.data());
  }
  std::memset(deg, 0, sizeof(int64_t) * (size_t)n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t s = 0, d = 0;
    uint64_t r = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
      uint64_t u;
      if ((lvl & 1) == 0) {
        r = draw(ekey, (uint64_t)i * 16 + (uint64_t)(lvl >> 1));
        u = r >> 32;
      } else {
        u = r & 0xffffffffULL;
      }
      uint32_t sb, db;
      if (u < ta) { sb = 0; db = 0; }
      else if (u < tab) { sb = 0; db = 1; }
      else if (u < tabc) { sb = 1; db = 0; }
      else { sb = 1; db = 1; }
      s = (s << 1) | sb;
      d = (d << 1) | db;
    }
    if (s == d) continue;
    if (relabel) {
      s = (uint32_t)perm[s];
      d = (uint32_t)perm[d];
    }
    __atomic_fetch_add(&deg[s], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&deg[d], 1, __ATOMIC_RELAXED);
  }
  return 0;
}

// G(n, m): m endpoint pairs, each endpoint uniform on [0, n).
// Weights of a variant graph (the paper's integer-power variants, Eq. 7):
// x uniform on (0, 1] from the weight stream of `seed` (edge i uses counter
// i, as the generators do), then the integer nearest to 1 + x * (2^power - 2),
// halves rounded up, so that the 2^power - 1 integers 1 .. 2^power - 1 occur.
// power = 1 gives unit weights.
int gg_weights_power(int64_t m, uint64_t seed, int32_t power, uint32_t* w) {
  if (m < 0 || power < 1 || power > 31) return -1;
  const uint64_t wkey = stream_key(seed, kStreamWeight);
  const double span = (double)((1ULL << power) - 2);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const uint64_t r = draw(wkey, (uint64_t)i);
    const double x = (double)((r >> 11) + 1) * (1.0 / 9007199254740992.0);  // (0, 1]
    w[i] = (uint32_t)(1.0 + x * span + 0.5);
  }
  return 0;
}

// Real weights as IEEE binary32 bit patterns, from the same weight stream:
// mode 0 the gr26 graphs' weights, x uniform on (0, 1]; mode 1 the float-pivot
// variants (Eq. 8), converge(x, pivot) = pivot - pivot (1 - 2x)^2 for x <= 1/2,
// pivot + (1 - pivot)(1 - 2x)^2 above, computed in double and rounded to the
// nearest binary32.
int gg_weights_f32(int64_t m, uint64_t seed, int32_t mode, double pivot, uint32_t* w) {
  if (m < 0 || mode < 0 || mode > 1 || !(pivot > 0.0 && pivot < 1.0)) return -1;
  const uint64_t wkey = stream_key(seed, kStreamWeight);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const uint64_t r = draw(wkey, (uint64_t)i);
    const double x = (double)((r >> 11) + 1) * (1.0 / 9007199254740992.0);  // (0, 1]
    double y = x;
    if (mode == 1) {
      const double t = (1.0 - 2.0 * x) * (1.0 - 2.0 * x);
      y = x <= 0.5 ? pivot - pivot * t : pivot + (1.0 - pivot) * t;
    }
    const float f = (float)y;
    uint32_t b;
    memcpy(&b, &f, sizeof b);
    w[i] = b;
  }
  return 0;
}

int gg_gnm(int64_t n, int64_t m, uint32_t wmax, uint64_t seed, int32_t* src, int32_t* dst,
           uint32_t* w) {
  if (n < 1 || n > INT32_MAX || m < 0 || wmax < 1) return -1;
  const uint64_t ekey = stream_key(seed, kStreamEdge);
  const uint64_t wkey = stream_key(seed, kStreamWeight);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    src[i] = (int32_t)below(draw(ekey, (uint64_t)i * 2), (uint64_t)n);
    dst[i] = (int32_t)below(draw(ekey, (uint64_t)i * 2 + 1), (uint64_t)n);
    w[i] = weight_from(draw(wkey, (uint64_t)i), wmax);
  }
  return 0;
}

// Grid: for cell (r, c) three edge slots 3*(r*cols+c)+k: k=0 right neighbour,
// k=1 down neighbour (each kept with p_keep), k=2 the (r+1, c+1) diagonal
// (kept with p_diag). Writes the kept edges in slot order; returns the count
// (or -1). Pass src == NULL to only count.
int64_t gg_grid(int32_t rows, int32_t cols, double p_keep, double p_diag, uint32_t wmax,
                uint64_t seed, int32_t* src, int32_t* dst, uint32_t* w) {
  if (rows < 1 || cols < 1 || (int64_t)rows * cols > INT32_MAX || wmax < 1) return -1;
  const uint64_t ekey = stream_key(seed, kStreamEdge);
  const uint64_t wkey = stream_key(seed, kStreamWeight);
  const double two53 = 9007199254740992.0;
  const uint64_t tk = (uint64_t)(p_keep * two53);
  const uint64_t td = (uint64_t)(p_diag * two53);
  const int64_t cells = (int64_t)rows * cols;
  // pass 1: per-row counts so that the output order is deterministic
  std::vector<int64_t> row_cnt((size_t)rows + 1, 0);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    int64_t cnt = 0;
    for (int64_t c = 0; c < cols; ++c) {
      int64_t cell = r * cols + c;
      for (int k = 0; k < 3; ++k) {
        bool valid = (k == 0) ? (c + 1 < cols) : (k == 1) ? (r + 1 < rows) : (r + 1 < rows && c + 1 < cols);
        if (!valid) continue;
        uint64_t u = draw(ekey, (uint64_t)(cell * 3 + k)) >> 11;
        if (u < (k == 2 ? td : tk)) ++cnt;
      }
    }
    row_cnt[(size_t)r + 1] = cnt;
  }
  for (int64_t r = 0; r < rows; ++r) row_cnt[(size_t)r + 1] += row_cnt[(size_t)r];
  const int64_t total = row_cnt[(size_t)rows];
  if (src == nullptr) return total;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    int64_t pos = row_cnt[(size_t)r];
    for (int64_t c = 0; c < cols; ++c) {
      int64_t cell = r * cols + c;
      for (int k = 0; k < 3; ++k) {
        bool valid = (k == 0) ? (c + 1 < cols) : (k == 1) ? (r + 1 < rows) : (r + 1 < rows && c + 1 < cols);
        if (!valid) continue;
        uint64_t slot = (uint64_t)(cell * 3 + k);
        uint64_t u = draw(ekey, slot) >> 11;
        if (u >= (k == 2 ? td : tk)) continue;
        int64_t other = (k == 0) ? cell + 1 : (k == 1) ? cell + cols : cell + cols + 1;
        src[pos] = (int32_t)cell;
        dst[pos] = (int32_t)other;
        w[pos] = weight_from(draw(wkey, slot), wmax);
        ++pos;
      }
    }
  }
  (void)cells;
  return total;
}

// Undirected edge list -> symmetric CSR. Self-loops dropped; both directions
// stored; rows sorted by column; parallel edges merged to the minimum weight.
// gg_csr_build does the work and returns an opaque handle (NULL on error,
// *nnz_out = -2 if nnz exceeds INT32_MAX); gg_csr_copy writes rowptr[n+1],
// col[nnz], w[nnz]; gg_csr_free releases the handle.
struct gg_csr {
  int64_t n;
  std::vector<int64_t> ptr;
  std::vector<uint64_t> ent;  // (col << 32) | weight
};

void* gg_csr_build(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   const uint32_t* w, int64_t* nnz_out) {
  *nnz_out = -1;
  if (n < 1 || n > INT32_MAX || m < 0) return nullptr;
  std::vector<int64_t> deg((size_t)n, 0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = src[i], d = dst[i];
    if (s == d || s < 0 || d < 0 || s >= n || d >= n) continue;
    __atomic_fetch_add(&deg[(size_t)s], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&deg[(size_t)d], 1, __ATOMIC_RELAXED);
  }
  std::vector<int64_t> ptr((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) ptr[(size_t)v + 1] = ptr[(size_t)v] + deg[(size_t)v];
  const int64_t total = ptr[(size_t)n];
  std::vector<uint64_t> ent((size_t)total);
  std::vector<int64_t> cur(ptr.begin(), ptr.end() - 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = src[i], d = dst[i];
    if (s == d || s < 0 || d < 0 || s >= n || d >= n) continue;
    int64_t ps = __atomic_fetch_add(&cur[(size_t)s], 1, __ATOMIC_RELAXED);
    int64_t pd = __atomic_fetch_add(&cur[(size_t)d], 1, __ATOMIC_RELAXED);
    ent[(size_t)ps] = ((uint64_t)(uint32_t)d << 32) | w[i];
    ent[(size_t)pd] = ((uint64_t)(uint32_t)s << 32) | w[i];
  }
  // sort rows by (col, w) and keep the first entry of each column run
  std::vector<int64_t> kept((size_t)n + 1, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    uint64_t* b = ent.data() + ptr[(size_t)v];
    uint64_t* e = ent.data() + ptr[(size_t)v + 1];
    std::sort(b, e);
    int64_t k = 0;
    for (uint64_t* p = b; p < e; ++p) {
      if (k > 0 && (b[k - 1] >> 32) == (*p >> 32)) continue;
      b[k++] = *p;
    }
    kept[(size_t)v + 1] = k;
  }
  for (int64_t v = 0; v < n; ++v) kept[(size_t)v + 1] += kept[(size_t)v];
  const int64_t nnz = kept[(size_t)n];
  if (nnz > INT32_MAX) {
    *nnz_out = -2;
    return nullptr;
  }
  // compact in place (rows only move left)
  for (int64_t v = 0; v < n; ++v) {
    int64_t from = ptr[(size_t)v], to = kept[(size_t)v];
    int64_t len = kept[(size_t)v + 1] - to;
    if (from != to) std::memmove(ent.data() + to, ent.data() + from, (size_t)len * sizeof(uint64_t));
  }
  ent.resize((size_t)nnz);
  gg_csr* h = new gg_csr;
  h->n = n;
  h->ptr.swap(kept);
  h->ent.swap(ent);
  *nnz_out = nnz;
  return h;
}

void gg_csr_copy(void* handle, int32_t* rowptr, int32_t* col, uint32_t* wout) {
  gg_csr* h = static_cast<gg_csr*>(handle);
  for (int64_t v = 0; v <= h->n; ++v) rowptr[v] = (int32_t)h->ptr[(size_t)v];
  const int64_t nnz = h->ptr[(size_t)h->n];
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nnz; ++e) {
    uint64_t x = h->ent[(size_t)e];
    col[e] = (int32_t)(x >> 32);
    wout[e] = (uint32_t)(x & 0xffffffffULL);
  }
}

void gg_csr_free(void* handle) { delete static_cast<gg_csr*>(handle); }

// k distinct sources drawn uniformly among vertices of degree >= 1.
// Returns the number written (< k only if fewer such vertices exist).
int32_t gg_pick_sources(int64_t n, const int32_t* rowptr, int32_t k, uint64_t seed,
                        int32_t* out) {
  std::vector<int32_t> cand;
  for (int64_t v = 0; v < n; ++v)
    if (rowptr[v + 1] > rowptr[v]) cand.push_back((int32_t)v);
  if (cand.empty() || k <= 0) return 0;
  uint64_t key = stream_key(seed, kStreamSource);
  int32_t got = 0;
  uint64_t ctr = 0;
  std::vector<int32_t> chosen;
  while (got < k && (size_t)got < cand.size()) {
    int32_t v = cand[(size_t)below(draw(key, ctr++), cand.size())];
    if (std::find(chosen.begin(), chosen.end(), v) != chosen.end()) continue;
    chosen.push_back(v);
    out[got++] = v;
  }
  return got;
}

int gg_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
