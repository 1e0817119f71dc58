/*
 * sssp.h -- C ABI of an MI355X (gfx950) engine for single-source shortest
 * paths on undirected graphs with non-negative integer (or, on request,
 * binary32) weights, following Yu, Wang and Luo, "A Heuristic Algorithm for
 * Shortest Path Search" (arXiv 2506.19349).
 *
 * What is computed (the paper's problem statement, Section 2): for a source s,
 * dist[v] is the length of the shortest s-v path, dist[s] = 0, and a vertex
 * with no path to s keeps +infinity, written as UINT32_MAX. The engine reaches
 * exactly these values; its heuristics (dynamic stepping, Section 3.1, and
 * traversal optimisation, Section 3.2, driving the Algorithm of Section 3.3)
 * only decide which relaxations run together. The predecessor array of
 * Section 2 comes with the tree entry points (sssp_solve_tree and the _ex
 * forms of the batched, replayed and served solves).
 *
 * Conventions for every call:
 *  - Graphs are symmetric CSR: rowptr[n+1] (int32, rowptr[0] = 0,
 *    non-decreasing, rowptr[n] = nnz <= INT32_MAX), colidx[nnz] (int32 in
 *    [0, n)), weight[nnz] (uint32). Each undirected edge appears in both rows
 *    with the same weight (as a multiset of (u, v, w) triples). Parallel edges
 *    and self-loops are allowed and mean what they mean in a multigraph.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary (or pinned) host memory.
 *  - Argument errors are detected on the host before anything is enqueued;
 *    such a call writes nothing.
 *  - Calls that take a stream enqueue their GPU work on it and return without
 *    waiting (unless stated). Results are valid once the stream is
 *    synchronised. A NULL stream is the null stream.
 *  - Status codes are negative on failure; sssp_last_error() and
 *    sssp_last_error_message() describe the most recent failure of the
 *    calling thread.
 */
#ifndef SSSP_H
#define SSSP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SSSP_OK = 0,
  SSSP_E_INVAL = -1,         /* bad argument (NULL pointer, n < 1, source out of range, bad CSR) */
  SSSP_E_NOT_SYMMETRIC = -2, /* CSR is not symmetric as a multiset of (u, v, w) */
  SSSP_E_RANGE = -3,         /* n, nnz or a size beyond the library's limits */
  SSSP_E_DIST_OVERFLOW = -4, /* a reachable vertex's distance does not fit below UINT32_MAX */
  SSSP_E_NOMEM = -5,         /* device or host allocation failed */
  SSSP_E_DEVICE = -6,        /* a HIP call or a kernel failed */
  SSSP_E_BUSY = -7           /* serving: no room to admit the request now */
} sssp_status;

typedef struct sssp_graph sssp_graph; /* opaque, library-owned, read-only after create */

/* Solver options. Zero-initialise and set what you need; zero fields take the
 * defaults given here (the paper's constants, Section 4.1). None of them
 * changes a distance. */
typedef struct {
  int32_t traversal_opt; /* 0: default (on); 1: on; -1: off (st = lb in every step) */
  int32_t alpha;         /* highD threshold of Eq. (3); 0 -> 3 */
  double beta;           /* Eq. (1) trade-off in (0, 1); 0 -> 0.9 */
  int32_t host_driven;   /* 1: one kernel launch per tick with a host sync (debug); 0: persistent */
  int32_t blocks_per_cu; /* persistent grid size; 0 -> tuned / default */
  int32_t heavy_split;   /* ranges longer than this are split across the grid; 0 -> default */
  int32_t fuse_rounds;   /* bucket fusion (Section 4.1's FUSED): rounds one workgroup may chain
                            without a grid-wide synchronisation while the frontier fits one
                            batch; 0 -> 256, -1 -> off */
  int32_t tile_shape;    /* engine tile shape (one kernel instantiation each): 1: 512-item round
                            batches, 1024-item settle batches; 2: 1024-item round batches (longer
                            rounds within one workgroup, 3 workgroups per CU); 3: 256-item round
                            batches; 4: 2048-item settle batches. 0 -> default: 1 when a graph of
                            the solve has skewed degrees (sssp_graph_info.hub_first > 0), else 3;
                            the query server uses 1 */
  int32_t st_grid;       /* computeST's candidates for integer weights (Section 4.1): 0 -> the exact window of
                            distinct settled distances while maxW <= 1024 (= ST_NUM: a grid bin is then at
                            most one unit wide) and the ST_NUM grid of 1024 bins per maxW above; 1 -> the grid
                            always; -1 -> the window while maxW <= 65536. Binary32 weights and integer
                            weights above 65536 always use the grid. Changes the schedule, never a
                            distance */
  int32_t reserved[6];
} sssp_options;

/* Work counters of one solve (the paper's Section 4 measures). */
typedef struct {
  uint64_t expansions;      /* vertex expansions (paths extended), band and deferred */
  uint64_t band_expansions; /* expansions of vertices at or above lb (nFrontier's count) */
  uint64_t push_scanned;    /* CSR entries scanned by push (edges relaxed) */
  uint64_t pull_vertices;   /* unsettled-list entries scanned by the pull */
  uint64_t pull_scanned;    /* CSR entries scanned by the pull (requests) */
  uint64_t relax_success;   /* successful distance decreases */
  uint64_t queue_entries;   /* frontier / touched / settled list entries written */
  uint64_t rounds;          /* push rounds (synchronisations of the round loop) */
  uint64_t pulls;           /* pull phases */
  uint64_t steps;           /* scheduling-threshold pairs <lb, ub> */
  uint64_t ticks;           /* device-wide phases executed (rounds + settle passes) */
  uint64_t fused_rounds;    /* rounds run back to back by one workgroup (bucket fusion) */
  uint64_t pull_unsettled;  /* unsettled vertices of degree >= 1 (dist >= lb) at each pull, summed:
                               the vertices Function 1's pull examines */
  uint32_t high_d0;         /* highD(0) */
  uint32_t gap0;            /* gap(0) */
  uint32_t flags;           /* nonzero: internal condition (see sssp_status_str of status) */
  uint32_t reserved;
} sssp_counters;

/* One step of the schedule (Section 3.3): the band, the selection threshold,
 * and the statistics taken at the step's end for the next pair. */
typedef struct {
  uint32_t lb, ub, st; /* this step's pair and selection threshold */
  uint32_t rounds;     /* push rounds in this step */
  uint32_t pulled;     /* 1 if the pull ran (st < lb) */
  uint32_t L;          /* next lb (= this step's final ub) */
  uint64_t S;          /* sumD(L) */
  uint32_t h;          /* highD(L) */
  uint32_t gap;        /* gap(L), Eq. (3) */
  uint32_t st_next;    /* computeST for <L, L + gap(L)> (Function 2) */
  uint32_t reserved;
} sssp_step;

typedef struct {
  int32_t n;
  int32_t nnz;
  int32_t nonisolated;  /* vertices of degree >= 1 */
  int32_t max_degree;
  int32_t distinct_degrees;
  uint32_t max_weight;  /* maxW(G, 1) */
  uint32_t high_d0;     /* highD(0) over the whole vertex set */
  uint32_t hub_first;   /* vertices the preparation moved to the front of its internal order
                           (rows of at least 4x the mean degree, at most 2^19; 0: the caller's
                           order is kept). Ids in and out of every call stay the caller's. */
  uint64_t device_bytes; /* device memory held by the graph */
} sssp_graph_info;

/* ---- graphs ------------------------------------------------------------- */

/* Build the device graph of the Section 2 problem (an undirected graph
 * G = <V, E, w> with non-negative weights): validate the CSR, check symmetry,
 * sort each row by (weight, column), and precompute the statistics inputs --
 * degrees, the degree histogram and highD(0), the weight quantiles RtoW[4096]
 * (Section 4.1: RtoW[x] = maxW(G, x/4095)). This is the paper's preprocessing
 * (Section 4.1, Section 4.6). n >= 1 vertices; rowptr/colidx/weight (layout
 * above) may be host or device pointers; they are copied, and the caller
 * keeps ownership. Synchronous. Returns NULL on error (see sssp_last_error:
 * SSSP_E_INVAL for n < 1, NULL arrays or an invalid CSR, SSSP_E_NOT_SYMMETRIC,
 * SSSP_E_RANGE, SSSP_E_NOMEM, SSSP_E_DEVICE). The graph lives on the device
 * current at creation; sssp_graph_destroy frees it. */
sssp_graph* sssp_graph_create(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                              const uint32_t* weight);

#define SSSP_CREATE_SKIP_SYMMETRY_CHECK 1
/* Real weights (the paper's gr26 graphs and their Eq. 8 variants): `weight`
 * holds IEEE binary32 bit patterns of finite non-negative values (-0.0, inf
 * and NaN are rejected). Distances are then binary32 bit patterns too: each
 * is the smallest, over all paths, of the path's weights summed in order in
 * binary32 (round to nearest), the value the textbook Dijkstra computes in
 * binary32; UINT32_MAX still marks unreachable vertices. computeST (Eq. 4-6)
 * then scores the points of a grid of 1024 bins per largest weight (ST_NUM,
 * Section 4.1), as it does for integer weights above 1024 (sssp_options.st_grid). */
#define SSSP_CREATE_FLOAT_WEIGHTS 2
/* As sssp_graph_create, with flags (SSSP_CREATE_*). Skipping the symmetry
 * check leaves correctness to the caller: the pull (Section 3.2) relies on it. */
sssp_graph* sssp_graph_create_ex(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                                 const uint32_t* weight, int32_t flags);

/* Free the graph. No solve on it may be in flight. NULL is accepted. */
sssp_status sssp_graph_destroy(sssp_graph* g);

/* Sizes and statistics of a graph (host struct). */
sssp_status sssp_graph_info_get(const sssp_graph* g, sssp_graph_info* out);

/* Copy the preprocessed rows to host arrays of nnz entries: columns and
 * weights of each row in ascending (weight, column) order. Synchronous. */
sssp_status sssp_graph_sorted_rows(const sssp_graph* g, int32_t* col_out, uint32_t* w_out);

/* Copy RtoW[4096] (uint32, host). Synchronous. */
sssp_status sssp_graph_rtow(const sssp_graph* g, uint32_t* rtow_out);

/* ---- solves ------------------------------------------------------------- */

/* The single-source problem of Section 2 (its problem statement: the length
 * of a shortest path from the source to every vertex, +infinity for vertices
 * the source does not reach), solved by the Algorithm of Section 3.3.
 * source: a vertex in [0, n). dist_out: caller-owned device memory of n uint32,
 * written in `stream` order; dist_out[source] = 0, unreachable vertices get
 * UINT32_MAX. The graph stays read-only, so solves on different streams may
 * run at once; each stream has its own workspace, allocated on first use.
 * Errors: SSSP_E_INVAL (NULL graph or dist_out, a source out of range, a graph
 * of another device), returned before anything is enqueued; SSSP_E_NOMEM,
 * SSSP_E_DEVICE. Asynchronous: a reachable vertex whose distance is >=
 * UINT32_MAX (the distances are then incomplete) is reported by
 * sssp_get_counters returning SSSP_E_DIST_OVERFLOW. */
sssp_status sssp_solve(const sssp_graph* g, int32_t source, uint32_t* dist_out,
                       hipStream_t stream);

/* As sssp_solve with options (NULL = defaults). */
sssp_status sssp_solve_ex(const sssp_graph* g, int32_t source, uint32_t* dist_out,
                          const sssp_options* opt, hipStream_t stream);

/* Distances and a shortest-path tree from `source` (Section 2.1's output:
 * dist and the predecessor of every vertex). dist_out as sssp_solve;
 * parent_out (device, n int32): parent_out[source] = source, parent_out[v] =
 * the vertex before v on a shortest source-v path, -1 for unreachable
 * vertices. Every parent edge is tight, dist[parent[v]] + w = dist[v], and
 * following parents from a reachable vertex ends at the source (also with
 * zero weights: a parent always reached its distance before its child). Where
 * several shortest paths exist, which one is reported may vary between runs.
 * Both buffers are caller-owned; enqueued on `stream`; options as
 * sssp_solve_ex (NULL = defaults). The solve keeps 8 more bytes per vertex of
 * device workspace while a tree is requested. */
sssp_status sssp_solve_tree(const sssp_graph* g, int32_t source, uint32_t* dist_out,
                            int32_t* parent_out, const sssp_options* opt, hipStream_t stream);

/* Point-to-point query (Section 5 names it among the method's uses): the
 * solve stops at the end of the first step after which `target` is settled.
 * dist_out (device, n uint32, caller-owned) then holds the exact distance of
 * target, and of every vertex whose distance is not above the target's (all
 * of them lie below the band's lower end when the solve stops); the other
 * entries are upper bounds of their distances (UINT32_MAX where no path has
 * been found yet), all of them above the target's distance. An unreachable target runs the whole solve and reads
 * UINT32_MAX. Options as sssp_solve_ex (NULL = defaults); enqueued on
 * `stream`; sssp_get_counters and sssp_get_schedule describe the steps run. */
sssp_status sssp_solve_p2p(const sssp_graph* g, int32_t source, int32_t target, uint32_t* dist_out,
                           const sssp_options* opt, hipStream_t stream);

/* k sources on one graph in one persistent launch: the paper's trial
 * protocol (Section 4: 64 sources per graph, drawn among the vertices of
 * degree >= 1, run one after another there) as one batch of k independent
 * solves of the Section 2 problem. sources: host array of k vertex ids (k >=
 * 1; repeats allowed); dist_out: caller-owned device memory of k * n uint32,
 * row i (n entries from dist_out + i * n) for sources[i], written in `stream`
 * order as sssp_solve writes one row. The batch keeps one solver workspace per
 * source on the stream. Errors as sssp_solve, plus k < 1 or NULL sources. */
sssp_status sssp_solve_batch(const sssp_graph* g, const int32_t* sources, int32_t k,
                             uint32_t* dist_out, hipStream_t stream);

/* k independent (graph, source) pairs in one persistent launch (the Section 2
 * problem for each pair; Section 4's trial protocol over many graphs); graphs
 * may differ in size. gs, sources, dist_outs: host arrays of k entries;
 * dist_outs[i] is caller-owned device memory of gs[i]'s n uint32, written in
 * `stream` order. Errors as sssp_solve for any pair, plus k < 1 or NULL
 * arrays, all before anything is enqueued. */
sssp_status sssp_solve_multi(const sssp_graph* const* gs, const int32_t* sources, int32_t k,
                             uint32_t* const* dist_outs, const sssp_options* opt,
                             hipStream_t stream);

/* As sssp_solve_multi, each pair optionally a point-to-point query and
 * optionally with its shortest-path tree (the outputs of sssp_solve_p2p and
 * sssp_solve_tree, Sections 2.1 and 5). targets: NULL, or a host array of k
 * entries, -1 for a full solve, else the target vertex of pair i (that
 * solve stops once its target is settled; the entries of the vertices whose
 * distance is not above the target's are exact, the others upper bounds). parent_outs: NULL,
 * or a host array of k entries, each NULL or device memory of gs[i]'s n
 * int32 (parent[s] = s, -1 where the distance is UINT32_MAX; the parent
 * edge of every other vertex is tight for its returned distance). Argument
 * errors as for sssp_solve_multi, plus a target outside [-1, n). */
sssp_status sssp_solve_multi_ex(const sssp_graph* const* gs, const int32_t* sources,
                                const int32_t* targets, int32_t k, uint32_t* const* dist_outs,
                                int32_t* const* parent_outs, const sssp_options* opt,
                                hipStream_t stream);

/* Counters of the last solve enqueued on `stream` (for a batch: summed over
 * its instances). Synchronises the stream. */
sssp_status sssp_get_counters(hipStream_t stream, sssp_counters* out);

/* Schedule of the last single-source solve on `stream`: up to cap steps into
 * out (host); *len receives the number of steps taken. Synchronises. */
sssp_status sssp_get_schedule(hipStream_t stream, sssp_step* out, int32_t cap, int32_t* len);

/* Durations (microseconds, host array) of the engine kernel of the solves
 * enqueued on `stream` since the previous call (at most the 256 most recent),
 * oldest first, measured with HIP events recorded around the engine launch
 * on that stream. *n receives the count. Synchronises the stream. */
sssp_status sssp_engine_times(hipStream_t stream, float* us_out, int32_t cap, int32_t* n);

/* ---- batched plans (persistent launch captured in a HIP graph) ----------- */

typedef struct sssp_plan sssp_plan; /* opaque */

/* Capture the whole launch sequence of a k-instance solve -- instance set-up,
 * the persistent engine (a cooperative graph node) and the overflow check --
 * in a HIP graph, for k (graph, dist_out) pairs fixed here (graphs may repeat
 * for several sources on one graph, or differ for a batch of small graphs).
 * dist_outs[i]: device memory of gs[i]'s n uint32, written at every run.
 * The plan owns its own workspace (device buffers sized for these graphs). A
 * plan serves one run at a time and is used on the device it was created on.
 * The graphs must outlive the plan. Returns NULL on error. */
sssp_plan* sssp_plan_create(const sssp_graph* const* gs, int32_t k, uint32_t* const* dist_outs,
                            const sssp_options* opt, hipStream_t stream);

/* Replay the plan for k new sources (host array; sources[i] is a vertex of
 * gs[i]) on `stream`. Waits for the plan's previous run to finish first (its
 * instance images are re-staged). Asynchronous otherwise. */
sssp_status sssp_plan_run(sssp_plan* p, const int32_t* sources, hipStream_t stream);

/* As sssp_plan_create, with a shortest-path tree per instance: parent_outs
 * NULL, or k entries, each NULL or device memory of gs[i]'s n int32 written
 * at every run (as in sssp_solve_multi_ex). */
sssp_plan* sssp_plan_create_ex(const sssp_graph* const* gs, int32_t k, uint32_t* const* dist_outs,
                               int32_t* const* parent_outs, const sssp_options* opt, hipStream_t stream);

/* As sssp_plan_run, each instance optionally a point-to-point query:
 * targets NULL, or k entries, -1 for a full solve (as in
 * sssp_solve_multi_ex). */
sssp_status sssp_plan_run_ex(sssp_plan* p, const int32_t* sources, const int32_t* targets,
                             hipStream_t stream);

/* Counters of the plan's last run, summed over its instances (waits for it). */
sssp_status sssp_plan_counters(sssp_plan* p, sssp_counters* out);

/* Free the plan (waits for its last run). NULL is accepted. */
sssp_status sssp_plan_destroy(sssp_plan* p);

/* ---- autotuner ----------------------------------------------------------- */

typedef struct {
  double default_us;    /* engine time of the workload under the options passed in */
  double best_us;       /* engine time under the options returned */
  int32_t evaluations;  /* option sets timed */
  int32_t reserved[7];
} sssp_tune_report;

/* Time the workload -- k (graph, source) pairs, solved one at a time
 * (batched = 0) or as one k-instance launch (batched = 1) -- under candidate
 * launch knobs and return the fastest in *inout. The knobs, in this order:
 * the tile shape (tile_shape 1..4: round batches of 512, 1024 or 256 items,
 * settle batches of 1024 or 2048), workgroups per CU (1, 2, or all the
 * shape's kernel allows), the heavy-row split threshold (64, 256, 1024, 4096:
 * ranges above it are spread over the grid in 256-entry chunks), bucket
 * fusion on/off, and, when tune_beta is nonzero, beta of Eq. (1) in {0.85,
 * 0.9, 0.95} (Section 4.3 finds the method insensitive there; 0.9 is the
 * paper's value). Knobs are tuned one at a time from the values passed in
 * (coordinate descent), each candidate measured by HIP events around the
 * engine launch after one untimed pass. No knob changes a distance; beta
 * changes the schedule. Synchronous; allocates scratch distance buffers for
 * the trials. report may be NULL. */
sssp_status sssp_autotune(const sssp_graph* const* gs, const int32_t* sources, int32_t k, int32_t batched,
                          int32_t tune_beta, sssp_options* inout, sssp_tune_report* report,
                          hipStream_t stream);

/* ---- query server (continuous batching over resident graphs) ------------ */

typedef struct sssp_server sssp_server; /* opaque */

typedef struct {
  uint64_t budget_bytes;    /* device memory the server may hold for queries in flight: solver
                               workspaces it allocates plus the n * 4 bytes of each admitted
                               query's output (graphs are resident already and not counted) */
  int32_t max_batch;        /* solver slots, i.e. queries in flight at once; 0 -> 64 */
  int32_t ticks_per_launch; /* device-wide ticks per engine launch between admissions; 0 -> 64 */
  int32_t max_pending;      /* queued (not yet admitted) queries; 0 -> 65536 */
  int32_t reserved[5];
} sssp_server_config;

typedef struct {
  int32_t state;    /* 0 done, 1 queued, 2 running */
  int32_t status;   /* final status once done (SSSP_OK, SSSP_E_DIST_OVERFLOW, ...) */
  int32_t graph_id, source, slot;
  uint32_t launches;  /* engine launches the query was part of */
  double submit_us, admit_us, done_us;  /* server clock (microseconds since create); -1: not yet */
} sssp_request_info;

typedef struct {
  uint64_t submitted, admitted, completed, launches;
  double engine_us;   /* total engine-kernel time (HIP events) */
  double now_us;      /* server clock */
  uint64_t budget_bytes, allocated_bytes, peak_allocated_bytes, peak_in_use_bytes;
  int32_t active, peak_active, queued, max_batch;
} sssp_server_stats;

/* Start a server on the current device, with its own stream and a pump
 * thread. Queries are single-source solves (options as for sssp_solve_ex,
 * NULL = defaults) on graphs registered with sssp_server_add_graph. The pump
 * runs the persistent engine in launches of ticks_per_launch ticks; between
 * launches it retires finished queries and admits queued ones (in arrival
 * order) into free slots while the budget allows, so queries that arrive
 * while others run join the next launch and share the device with them.
 * Returns NULL on error. */
sssp_server* sssp_server_create(const sssp_server_config* cfg, const sssp_options* opt);

/* Register a resident graph (created on the same device; it must outlive the
 * server). Returns its id (>= 0) or a negative status. */
int32_t sssp_server_add_graph(sssp_server* s, const sssp_graph* g);

/* Device bytes one query on graph `graph_id` is charged against the budget
 * when it runs alone in a fresh slot (workspace + output), or a negative
 * status. */
int64_t sssp_server_query_bytes(sssp_server* s, int32_t graph_id);

/* Queue a query: distances from `source` on graph `graph_id` into dist_out
 * (device, n uint32, caller-owned; it must stay allocated until the query is
 * done). *ticket identifies the query. SSSP_E_RANGE if the query alone
 * exceeds the budget; SSSP_E_BUSY if the queue is full. Thread-safe. */
sssp_status sssp_server_submit(sssp_server* s, int32_t graph_id, int32_t source, uint32_t* dist_out,
                               int64_t* ticket);

/* As sssp_server_submit, optionally a point-to-point query (target >= 0;
 * -1 for a full solve) and optionally with its shortest-path tree into
 * parent_out (device, n int32, caller-owned, or NULL); outputs as in
 * sssp_solve_multi_ex. A tree query counts 12 more bytes per vertex against
 * the budget (its output and the solve's tree words). */
sssp_status sssp_server_submit_ex(sssp_server* s, int32_t graph_id, int32_t source, int32_t target,
                                  uint32_t* dist_out, int32_t* parent_out, int64_t* ticket);

/* *done = 1 once the query is finished (its distances are then complete in
 * device memory and visible to any stream). */
sssp_status sssp_server_poll(sssp_server* s, int64_t ticket, int32_t* done);

/* Block until the query is finished; returns its final status. */
sssp_status sssp_server_wait(sssp_server* s, int64_t ticket);

/* Timing and placement of one query (its record is kept until released). */
sssp_status sssp_server_request_info(sssp_server* s, int64_t ticket, sssp_request_info* out);

/* Forget a finished query's record. */
sssp_status sssp_server_release(sssp_server* s, int64_t ticket);

sssp_status sssp_server_get_stats(sssp_server* s, sssp_server_stats* out);

/* Finish every submitted query, stop the pump and free the server. */
sssp_status sssp_server_destroy(sssp_server* s);

/* ---- debugging ---------------------------------------------------------- */

/* Enable (cap > 0) or disable (cap = 0) a per-tick log of the engine for the
 * solves that follow on `stream`: for each device-wide tick, eight uint64 on
 * the 100 MHz wall clock unless stated -- [0] when the tick's last workgroup
 * arrived at the barrier, [1] the tick's work batches, [2] bits of instance
 * 0's state (tick kind | init round << 8 | pull << 9 | step << 16), [3] when
 * the next tick was released, [4] when the tick's first batch started, [5]
 * when its last workgroup finished its batches, [6] and [7] when the step's
 * heuristic started and ended (0 if none ran in the tick). Synchronises the
 * stream. */
sssp_status sssp_debug_tick_log(hipStream_t stream, int32_t cap);

/* Copy the tick log of the last solve on `stream` (cap entries of eight uint64
 * into out); *len receives the tick count, *t_start the engine's start time. */
sssp_status sssp_debug_get_tick_log(hipStream_t stream, uint64_t* out, int32_t cap, int32_t* len,
                                    uint64_t* t_start);

/* ---- a solve that allocates nothing -------------------------------------- */

/* For callers that cannot allocate device or host memory during the call
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): sssp_solve's result, computed by the same kernels, with every
 * solver buffer carved out of one device array of SSSP_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends. The
 * caller passes the graph (created beforehand), the source and dist_out
 * (device, n uint32, caller-owned), as for sssp_solve; the call makes no
 * allocation of any kind. Returns SSSP_E_RANGE, before anything is enqueued,
 * for a graph whose solver buffers do not fit the array (64 bytes per vertex,
 * 1/4 byte per CSR entry and 64 bytes per row longer than 64 entries, plus
 * about 0.6 MB; the 16,384-vertex R-MAT graph of edge factor 16 needs about
 * 2 MB, a graph of a million vertices does not fit), and the
 * other argument errors of sssp_solve. Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (on different streams, or from
 * different threads without ordering) race and give wrong results; calls
 * ordered on one stream are safe. No counters, schedule or engine timing are
 * recorded for sssp_get_counters / sssp_get_schedule / sssp_engine_times; a
 * distance overflow leaves the affected entries at UINT32_MAX unreported. */
#define SSSP_NOALLOC_SCRATCH_BYTES (64u << 20)
sssp_status sssp_solve_noalloc(const sssp_graph* g, int32_t source, uint32_t* dist_out,
                               hipStream_t stream);

/* ---- teardown ----------------------------------------------------------- */

/* Free what the library holds on its own behalf: the per-stream solver
 * workspaces of the plain, tree, point-to-point and batched solves (device
 * buffers, pinned staging buffers, HIP events) on every device. Graphs, plans
 * and servers belong to the caller and are not touched. Waits for each device
 * that held a workspace to finish its work first. A later solve sets its
 * workspace up again. For a process about to exit, so that no HIP object of
 * the library outlives the runtime's own teardown (the Python package calls it
 * from an exit hook after closing its graphs, plans and servers); no solve may
 * be enqueued concurrently. */
sssp_status sssp_release_workspaces(void);

/* ---- the device's random-access rates ----------------------------------- */

/* The rates at which the current device serves the random accesses the solve
 * engine is made of: the reference for the engine's roofline. The method
 * (Section 3: relaxations, the pull's reads, the settle's statistics) moves a
 * few bytes per access at positions no cache predicts, so its ceiling is the
 * rate of independent random accesses, not HBM bandwidth. */
typedef struct {
  double rows64_per_s;         /* 64-byte rows gathered at random from a 4 GiB table */
  double words8_small_per_s;   /* 8-byte words read at random from a 128 MiB array (the size of a
                                  2^24-vertex graph's per-vertex state, which the 256 MB last-level
                                  cache holds) */
  double words8_large_per_s;   /* 8-byte words read at random from a 4 GiB array */
  double atomics8_small_per_s; /* 64-bit atomicMin at random words of the 128 MiB array */
  int64_t accesses;            /* accesses per timed launch (2^24) */
  int32_t reserved[6];
} sssp_random_rates;

/* Measure the rates on the current device (16 workgroups of 256 threads per
 * CU; positions from a counter-based hash; each rate the best of 3 timed
 * launches after an untimed one, timed with HIP events on `stream`).
 * Synchronous. Allocates and frees about 8.4 GB of device memory; returns
 * SSSP_E_NOMEM when it does not fit. */
sssp_status sssp_device_random_rates(sssp_random_rates* out, hipStream_t stream);

/* ---- errors ------------------------------------------------------------- */

sssp_status sssp_last_error(void);
const char* sssp_last_error_message(void);
const char* sssp_status_str(sssp_status s);
/* Library version string. */
const char* sssp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SSSP_H */
