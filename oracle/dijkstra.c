/*
 * ORACLE -- test infrastructure only. Nothing in the product path may call,
 * link or load this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.
 *
 * Single-source shortest paths by its plain definition: dist[v] is the minimum
 * over all s->v paths of the summed edge weights, dist[s] = 0, and a vertex
 * with no path keeps +infinity (the paper's problem statement, Section 2).
 * Computed with the textbook binary-heap Dijkstra (the exact sequential method
 * the paper contrasts with, Section 2.2), lazy deletion, 64-bit accumulation.
 *
 * The input is the RAW undirected edge list (u, v, w): every edge is usable in
 * both directions, self-loops and parallel edges are kept as given. The
 * adjacency is built here from that list; nothing is shared with the GPU path.
 *
 * Output: uint32 distances, UINT32_MAX for unreachable vertices. A reachable
 * vertex whose true distance does not fit below UINT32_MAX makes the call
 * return ORACLE_OVERFLOW (its slot holds UINT32_MAX).
 *
 * Real weights (the gr26 graphs and their Eq. 8 variants): with weights
 * given as IEEE binary32 bit patterns, the same Dijkstra with binary32
 * distances: d[v] = min over u of fl(d[u] + w), each addition a single
 * binary32 round-to-nearest. fl(a + w) never decreases as a grows, so this is
 * the smallest over all paths of the path's weights summed in order in
 * binary32, which is what any complete relaxation order converges to.
 *
 * Optionally the predecessor array of the same problem statement (Section
 * 2.1): the textbook Dijkstra keeps, for every vertex, the vertex whose edge
 * last lowered its tentative distance; at the end that edge is tight and the
 * predecessors form a tree rooted at s (parent[s] = s, -1 when unreachable).
 *
 * Also here: an invariant checker over a CSR (dist[s] = 0; no edge can
 * improve a distance; every finite vertex other than s has a tight incoming
 * edge; every finite vertex is reached from s over tight edges; infinite
 * vertices only have infinite neighbours), used as the any-size property check,
 * and a checker of a candidate predecessor array against a distance vector.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_BAD_ARGS -1
#define ORACLE_NOMEM -2
#define ORACLE_OVERFLOW 1

#define INF32 0xFFFFFFFFu

typedef struct {
  int64_t n;
  int64_t *off; /* n + 1 */
  int32_t *nbr; /* 2m */
  uint32_t *wt; /* 2m */
} oracle_adj;

/* Build the undirected adjacency of a raw edge list (both directions). */
void *oracle_adj_build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                       const uint32_t *w) {
  if (n < 1 || m < 0) return NULL;
  for (int64_t i = 0; i < m; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return NULL;
  oracle_adj *a = (oracle_adj *)calloc(1, sizeof(oracle_adj));
  if (!a) return NULL;
  a->n = n;
  a->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  a->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  a->wt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(2 * m + 1));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!a->off || !a->nbr || !a->wt || !cur) {
    free(a->off); free(a->nbr); free(a->wt); free(a); free(cur);
    return NULL;
  }
  for (int64_t i = 0; i < m; ++i) {
    a->off[src[i] + 1]++;
    a->off[dst[i] + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) a->off[v + 1] += a->off[v];
  memcpy(cur, a->off, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; ++i) {
    int64_t p = cur[src[i]]++;
    a->nbr[p] = dst[i];
    a->wt[p] = w[i];
    p = cur[dst[i]]++;
    a->nbr[p] = src[i];
    a->wt[p] = w[i];
  }
  free(cur);
  return a;
}

void oracle_adj_free(void *h) {
  oracle_adj *a = (oracle_adj *)h;
  if (!a) return;
  free(a->off);
  free(a->nbr);
  free(a->wt);
  free(a);
}

typedef struct {
  uint64_t d;
  int32_t v;
} heap_item;

typedef struct {
  heap_item *a;
  int64_t size, cap;
} heap;

static int heap_push(heap *h, uint64_t d, int32_t v) {
  if (h->size == h->cap) {
    int64_t nc = h->cap ? h->cap * 2 : 1024;
    heap_item *na = (heap_item *)realloc(h->a, sizeof(heap_item) * (size_t)nc);
    if (!na) return -1;
    h->a = na;
    h->cap = nc;
  }
  int64_t i = h->size++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->a[p].d <= d) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i].d = d;
  h->a[i].v = v;
  return 0;
}

static heap_item heap_pop(heap *h) {
  heap_item top = h->a[0];
  heap_item last = h->a[--h->size];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->size) break;
    if (c + 1 < h->size && h->a[c + 1].d < h->a[c].d) ++c;
    if (h->a[c].d >= last.d) break;
    h->a[i] = h->a[c];
    i = c;
  }
  if (h->size > 0) h->a[i] = last;
  return top;
}

/* Dijkstra from s on a built adjacency. Returns ORACLE_OK / ORACLE_OVERFLOW /
 * an error code. dist_out has n entries. */
/* parent_out may be NULL (distances only). */
static int adj_dijkstra(const oracle_adj *a, int32_t s, uint32_t *dist_out, int32_t *parent_out) {
  if (!a || s < 0 || s >= a->n) return ORACLE_BAD_ARGS;
  const int64_t n = a->n;
  uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
  heap h = {NULL, 0, 0};
  if (!d || !done) {
    free(d); free(done);
    return ORACLE_NOMEM;
  }
  for (int64_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
  if (parent_out)
    for (int64_t v = 0; v < n; ++v) parent_out[v] = -1;
  d[s] = 0;
  if (parent_out) parent_out[s] = s;
  int rc = ORACLE_OK;
  if (heap_push(&h, 0, s)) rc = ORACLE_NOMEM;
  while (rc == ORACLE_OK && h.size > 0) {
    heap_item it = heap_pop(&h);
    int32_t u = it.v;
    if (done[u] || it.d != d[u]) continue; /* stale entry */
    done[u] = 1;
    for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
      int32_t v = a->nbr[e];
      uint64_t nd = d[u] + (uint64_t)a->wt[e];
      if (nd < d[v]) {
        d[v] = nd;
        if (parent_out) parent_out[v] = u;
        if (heap_push(&h, nd, v)) {
          rc = ORACLE_NOMEM;
          break;
        }
      }
    }
  }
  if (rc == ORACLE_OK) {
    for (int64_t v = 0; v < n; ++v) {
      if (d[v] == UINT64_MAX) {
        dist_out[v] = INF32;
      } else if (d[v] >= (uint64_t)INF32) {
        dist_out[v] = INF32;
        rc = ORACLE_OVERFLOW;
      } else {
        dist_out[v] = (uint32_t)d[v];
      }
    }
  }
  free(h.a);
  free(d);
  free(done);
  return rc;
}

int oracle_adj_dijkstra(const void *hv, int32_t s, uint32_t *dist_out) {
  return adj_dijkstra((const oracle_adj *)hv, s, dist_out, NULL);
}

/* Distances and the predecessor array (parent_out: n entries). */
int oracle_adj_dijkstra_tree(const void *hv, int32_t s, uint32_t *dist_out, int32_t *parent_out) {
  if (!parent_out) return ORACLE_BAD_ARGS;
  return adj_dijkstra((const oracle_adj *)hv, s, dist_out, parent_out);
}

static float f32_of(uint32_t b) {
  float f;
  memcpy(&f, &b, sizeof f);
  return f;
}

static uint32_t bits_of(float f) {
  uint32_t b;
  memcpy(&b, &f, sizeof b);
  return b;
}

/* Binary32 weights and distances (bit patterns in and out; INF32 for
 * unreachable vertices). Non-negative binary32 bit patterns order like their
 * values, so the heap keys on them. */
int oracle_adj_dijkstra_f32(const void *hv, int32_t s, uint32_t *dist_out) {
  const oracle_adj *a = (const oracle_adj *)hv;
  if (!a || s < 0 || s >= a->n) return ORACLE_BAD_ARGS;
  const int64_t n = a->n;
  uint32_t *d = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
  heap h = {NULL, 0, 0};
  if (!d || !done) {
    free(d); free(done);
    return ORACLE_NOMEM;
  }
  for (int64_t v = 0; v < n; ++v) d[v] = INF32;
  d[s] = bits_of(0.0f);
  int rc = ORACLE_OK;
  if (heap_push(&h, d[s], s)) rc = ORACLE_NOMEM;
  while (rc == ORACLE_OK && h.size > 0) {
    heap_item it = heap_pop(&h);
    int32_t u = it.v;
    if (done[u] || it.d != d[u]) continue; /* stale entry */
    done[u] = 1;
    const float du = f32_of(d[u]);
    for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
      int32_t v = a->nbr[e];
      const uint32_t c = bits_of(du + f32_of(a->wt[e]));
      if (c < d[v]) {
        d[v] = c;
        if (heap_push(&h, c, v)) {
          rc = ORACLE_NOMEM;
          break;
        }
      }
    }
  }
  if (rc == ORACLE_OK) memcpy(dist_out, d, sizeof(uint32_t) * (size_t)n);
  free(h.a);
  free(d);
  free(done);
  return rc;
}

/* One-shot: build the adjacency from the raw edge list, solve, free. */
int oracle_dijkstra(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    const uint32_t *w, int32_t s, uint32_t *dist_out) {
  void *a = oracle_adj_build(n, m, src, dst, w);
  if (!a) return ORACLE_BAD_ARGS;
  int rc = oracle_adj_dijkstra(a, s, dist_out);
  oracle_adj_free(a);
  return rc;
}

/* k sources over a shared adjacency on `threads` POSIX threads, one Dijkstra
 * per query. Row i of dist_out (n entries) belongs to sources[i]. Returns the
 * first nonzero per-query status, else 0. */
typedef struct {
  const oracle_adj *a;
  const int32_t *sources;
  uint32_t *out;
  int32_t k;
  volatile int32_t next;
  volatile int rc;
  pthread_mutex_t mu;
} many_ctx;

static void *many_worker(void *p) {
  many_ctx *c = (many_ctx *)p;
  for (;;) {
    pthread_mutex_lock(&c->mu);
    int32_t i = c->next++;
    pthread_mutex_unlock(&c->mu);
    if (i >= c->k) break;
    int r = oracle_adj_dijkstra(c->a, c->sources[i], c->out + (size_t)i * (size_t)c->a->n);
    if (r != ORACLE_OK) {
      pthread_mutex_lock(&c->mu);
      if (c->rc == ORACLE_OK) c->rc = r;
      pthread_mutex_unlock(&c->mu);
    }
  }
  return NULL;
}

int oracle_adj_dijkstra_many(const void *hv, int32_t k, const int32_t *sources, uint32_t *dist_out,
                             int32_t threads) {
  const oracle_adj *a = (const oracle_adj *)hv;
  if (!a || k < 0 || threads < 1) return ORACLE_BAD_ARGS;
  many_ctx c;
  c.a = a;
  c.sources = sources;
  c.out = dist_out;
  c.k = k;
  c.next = 0;
  c.rc = ORACLE_OK;
  pthread_mutex_init(&c.mu, NULL);
  pthread_t *tids = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
  int started = 0;
  for (int t = 0; t < threads; ++t)
    if (pthread_create(&tids[t], NULL, many_worker, &c) == 0) ++started;
  if (started == 0) many_worker(&c);
  for (int t = 0; t < started; ++t) pthread_join(tids[t], NULL);
  free(tids);
  pthread_mutex_destroy(&c.mu);
  return c.rc;
}

/* Invariant checker on a CSR (rowptr[n+1], col[nnz], w[nnz]) for a candidate
 * distance vector. counts[0..4] receive the number of violations of:
 *   0  dist[s] != 0
 *   1  an edge (u,v,w) with dist[u] finite and dist[u] + w < dist[v]
 *   2  a finite vertex v != s with no tight incoming edge (dist[u]+w == dist[v])
 *   3  a finite vertex not reached from s along tight edges
 *   4  an infinite vertex adjacent to a finite one (subsumed by 1; kept apart)
 * Returns the total. With every weight >= 1, zero violations of 0..2 pin the
 * vector to the exact distances; check 3 closes the zero-weight loophole. */
int64_t oracle_check_sssp(int64_t n, const int32_t *rowptr, const int32_t *col, const uint32_t *w,
                          int32_t s, const uint32_t *dist, int64_t *counts) {
  for (int i = 0; i < 5; ++i) counts[i] = 0;
  if (n < 1 || s < 0 || s >= n) return -1;
  if (dist[s] != 0) counts[0]++;
  unsigned char *tight_in = (unsigned char *)calloc((size_t)n, 1);
  unsigned char *seen = (unsigned char *)calloc((size_t)n, 1);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!tight_in || !seen || !queue) {
    free(tight_in); free(seen); free(queue);
    return -2;
  }
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      int32_t v = col[e];
      if (dist[u] == INF32) {
        if (dist[v] != INF32) counts[4]++;
        continue;
      }
      uint64_t c = (uint64_t)dist[u] + (uint64_t)w[e];
      if (c < (uint64_t)dist[v]) counts[1]++;
      if (c == (uint64_t)dist[v]) tight_in[v] = 1;
    }
  }
  for (int64_t v = 0; v < n; ++v)
    if (v != s && dist[v] != INF32 && !tight_in[v]) counts[2]++;
  /* BFS over tight edges from s */
  int64_t head = 0, tail = 0;
  if (dist[s] == 0) {
    seen[s] = 1;
    queue[tail++] = s;
  }
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      int32_t v = col[e];
      if (!seen[v] && dist[v] != INF32 && (uint64_t)dist[u] + w[e] == (uint64_t)dist[v]) {
        seen[v] = 1;
        queue[tail++] = v;
      }
    }
  }
  for (int64_t v = 0; v < n; ++v)
    if (dist[v] != INF32 && !seen[v]) counts[3]++;
  free(tight_in);
  free(seen);
  free(queue);
  return counts[0] + counts[1] + counts[2] + counts[3] + counts[4];
}

/* Checker of a candidate predecessor array on a CSR (rowptr[n+1], col[nnz],
 * w[nnz]; undirected: row v lists the edges at v) against a distance vector
 * (taken as given: check it with oracle_check_sssp). counts[0..3] receive the
 * number of violations of:
 *   0  parent[s] != s
 *   1  an unreachable vertex (dist = +inf) with parent != -1, or a reachable
 *      vertex other than s whose parent is not a vertex id
 *   2  a reachable vertex v != s with no edge (parent[v], v, w) in its row
 *      such that dist[parent[v]] + w == dist[v] (the parent edge is not tight)
 *   3  a reachable vertex from which following parents does not end at s
 *      (a cycle, or a chain through an invalid or unreachable vertex)
 * Returns the total, -1 for bad arguments, -2 when out of memory. */
int64_t oracle_check_tree(int64_t n, const int32_t *rowptr, const int32_t *col, const uint32_t *w,
                          int32_t s, const uint32_t *dist, const int32_t *parent, int64_t *counts) {
  for (int i = 0; i < 4; ++i) counts[i] = 0;
  if (n < 1 || s < 0 || s >= n) return -1;
  if (parent[s] != s) counts[0]++;
  for (int64_t v = 0; v < n; ++v) {
    if (dist[v] == INF32) {
      if (parent[v] != -1) counts[1]++;
      continue;
    }
    if (v == s) continue;
    const int32_t p = parent[v];
    if (p < 0 || p >= n) {
      counts[1]++;
      continue;
    }
    int tight = 0;
    if (dist[p] != INF32)
      for (int64_t e = rowptr[v]; e < rowptr[v + 1] && !tight; ++e)
        if (col[e] == p && (uint64_t)dist[p] + w[e] == (uint64_t)dist[v]) tight = 1;
    if (!tight) counts[2]++;
  }
  /* chains: 0 unvisited, 1 on the current walk, 2 ends at s, 3 does not */
  unsigned char *color = (unsigned char *)calloc((size_t)n, 1);
  int32_t *path = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!color || !path) {
    free(color); free(path);
    return -2;
  }
  color[s] = parent[s] == s ? 2 : 3;
  for (int64_t v0 = 0; v0 < n; ++v0) {
    if (dist[v0] == INF32 || color[v0]) continue;
    int64_t len = 0;
    int64_t v = v0;
    unsigned char end;
    for (;;) {
      if (v < 0 || v >= n || dist[v] == INF32) { end = 3; break; }
      if (color[v] == 2 || color[v] == 3) { end = color[v]; break; }
      if (color[v] == 1) { end = 3; break; } /* a cycle */
      color[v] = 1;
      path[len++] = (int32_t)v;
      v = parent[v];
    }
    for (int64_t i = 0; i < len; ++i) {
      color[path[i]] = end;
      if (end == 3) counts[3]++;
    }
  }
  free(color);
  free(path);
  return counts[0] + counts[1] + counts[2] + counts[3];
}
