/*
 * dg.h -- C boundary of libdg, a snapshot-query dynamic graph for MI355X.
 *
 * The graph is a shared object in the sense of the paper's concurrent-graph
 * vocabulary (preamble: linearizable shared graph with vertex-list /
 * edge-list, non-blocking).  Its operations are the ADT calls the paper names
 * PutV / RemoveV / GetV / PutE / RemoveE / GetE, and the snapshot queries it
 * names BFS, SSSP and BC.  Updates arrive in batches; the ops of a batch are
 * linearized in index order, and each non-empty batch publishes one new
 * snapshot epoch.  A query reads exactly the graph as of one epoch.
 *
 * Conventions for every call:
 *   - Return value: DG_OK (0) or a negative dg_status.  No C++ exception
 *     crosses this boundary.  On error, dg_last_error() describes it.
 *   - "device" pointers are HIP device memory of the GPU the graph was
 *     created on; "host or device" pointers are classified with
 *     hipPointerGetAttributes.  The caller owns every buffer it passes in;
 *     the library owns the graph store and all internal scratch.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device outputs
 *     are written asynchronously on that stream; host outputs are complete
 *     when the call returns.
 *   - A dg_graph is driven by one caller thread at a time.  Concurrency
 *     between updates and queries goes through dg_query_batch (many queries
 *     in one launch) and the dg_server_* serving loop.
 */
#ifndef DG_H
#define DG_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_graph dg_graph;
typedef uint32_t dg_epoch;      /* 0 = empty graph; epoch k = after k batches */
typedef int32_t dg_status;

#define DG_EPOCH_LATEST 0xFFFFFFFFu

enum {
  DG_OK = 0,
  DG_E_INVALID_ARG = -1,
  DG_E_OUT_OF_MEMORY = -2,
  DG_E_VERTEX_RANGE = -3,   /* an id >= v_capacity in the batch: whole batch rejected */
  DG_E_WEIGHT_RANGE = -4,   /* an AddEdge weight outside [1, w_max]: batch rejected */
  DG_E_EPOCH_RETIRED = -5,  /* epoch older than the retained window, or not yet published */
  DG_E_SOURCE_ABSENT = -6,  /* a query source is not a live vertex at that epoch */
  DG_E_OVERFLOW = -7,       /* a BC shortest-path count exceeded int64 */
  DG_E_HIP = -8,            /* a HIP runtime error; text in dg_last_error */
  DG_E_BUSY = -9,           /* serving loop: no admission capacity right now */
  DG_E_UNIMPLEMENTED = -10
};

/* Operation record, 16 bytes: the six ADT calls.  For vertex ops only `u` is
 * read (the vertex); `w` is read only by AddEdge. */
typedef struct { uint32_t type, u, v; int32_t w; } dg_op;
enum { DG_ADD_VERTEX = 0, DG_REMOVE_VERTEX = 1, DG_CONTAINS_VERTEX = 2,
       DG_ADD_EDGE = 3, DG_REMOVE_EDGE = 4, DG_CONTAINS_EDGE = 5 };
/* Per-op result byte: 0 = false/absent/no change, 1 = true/done,
 * 2 = an endpoint of an edge op is not a live vertex at that point. */

#define DG_UNDIRECTED 1u

typedef struct {
  uint32_t v_capacity;         /* vertex ids are [0, v_capacity) */
  uint32_t flags;              /* DG_UNDIRECTED: key of (u,v) is {min,max}, both arcs stored */
  int32_t w_max;               /* AddEdge weights in [1, w_max]; (v_capacity-1)*w_max < 2^31 */
  uint32_t max_resident_epochs;/* epochs kept queryable besides pinned ones (>= 1) */
  uint64_t edge_capacity;      /* expected peak number of stored arcs (sizing hint) */
  uint64_t mem_budget;         /* bytes of device memory the store may use; 0 = no limit */
} dg_config;

/* Create an empty graph (epoch 0) on the current HIP device. */
dg_status dg_create(const dg_config* cfg, dg_graph** out);
dg_status dg_destroy(dg_graph* g);
/* Text of the last error on g (or of the last failed dg_create if g is NULL). */
const char* dg_last_error(const dg_graph* g);
dg_epoch dg_latest_epoch(const dg_graph* g);

/*
 * Apply ops[0..n) as one batch (ADT ops named in the paper's preamble,
 * linearized in index order; a Contains is answered at its position).
 * ops: host or device array of n dg_op.  results: host or device array of n
 * bytes, or NULL.  On success *new_epoch = the published epoch (unchanged
 * for n == 0).  The whole batch is validated before any op applies: on
 * DG_E_VERTEX_RANGE / DG_E_WEIGHT_RANGE / DG_E_INVALID_ARG (unknown type)
 * nothing changes.  The call returns after the epoch is published.
 */
dg_status dg_apply_batch(dg_graph* g, const dg_op* ops, uint64_t n, uint8_t* results,
                         dg_epoch* new_epoch, void* stream);

/* Single-op forms: a batch of one op.  *res receives the result byte. */
dg_status dg_add_vertex(dg_graph* g, uint32_t v, uint8_t* res, dg_epoch* ep);
dg_status dg_remove_vertex(dg_graph* g, uint32_t v, uint8_t* res, dg_epoch* ep);
dg_status dg_contains_vertex(dg_graph* g, uint32_t v, uint8_t* res, dg_epoch* ep);
dg_status dg_add_edge(dg_graph* g, uint32_t u, uint32_t v, int32_t w, uint8_t* res, dg_epoch* ep);
dg_status dg_remove_edge(dg_graph* g, uint32_t u, uint32_t v, uint8_t* res, dg_epoch* ep);
dg_status dg_contains_edge(dg_graph* g, uint32_t u, uint32_t v, uint8_t* res, dg_epoch* ep);

/*
 * Snapshots.  The last max_resident_epochs epochs are queryable; acquiring
 * an epoch pins it (reference count) so it stays queryable until released.
 * want = DG_EPOCH_LATEST pins the latest epoch.  Old versions are reclaimed
 * only below the oldest queryable epoch.
 */
dg_status dg_snapshot_acquire(dg_graph* g, dg_epoch want, dg_epoch* pinned);
dg_status dg_snapshot_release(dg_graph* g, dg_epoch e);
/* Reclaim versions invisible to every queryable epoch and repack the slabs
 * (stream-ordered; waits for work queued on `stream`). */
dg_status dg_compact(dg_graph* g, void* stream);

/*
 * Snapshot queries on epoch e (DG_EPOCH_LATEST allowed).
 * dist: device array of v_capacity int32.
 *   dg_bfs:  dist[v] = fewest arcs on a path src -> v visible at e, -1 if none.
 *   dg_sssp: dist[v] = least total weight of such a path, -1 if none.
 * bc: device array of v_capacity double; srcs: host array of k distinct live
 *   vertices.  bc[v] = sum over s in srcs (in order), s != v, of the Brandes
 *   dependency delta_s(v) on the unweighted snapshot (int64 path counts,
 *   FP64 dependencies; no normalisation).  DG_E_OVERFLOW if a path count
 *   exceeds int64.
 * The call validates the epoch and sources on the host, enqueues the work on
 * `stream` and returns; dg_bc returns after the overflow flag is read.
 */
dg_status dg_bfs(dg_graph* g, dg_epoch e, uint32_t src, int32_t* dist, void* stream);
dg_status dg_sssp(dg_graph* g, dg_epoch e, uint32_t src, int32_t* dist, void* stream);
dg_status dg_bc(dg_graph* g, dg_epoch e, const uint32_t* srcs, uint32_t k, double* bc, void* stream);

/*
 * dg_bfs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and result as dg_bfs; dist must be device memory.  Every
 * scratch buffer of the search (frontier queues and their chunk maps,
 * bitmaps, counters) is carved from one fixed device area of
 * DG_NOALLOC_SCRATCH_BYTES per GPU, held from the library's first use on
 * that GPU until the process ends; the call makes no device or pinned-host
 * allocation, and waits for its stream between levels instead of polling
 * pinned memory.  A graph whose search needs more than the area
 * (about 48 B per vertex of capacity plus 2.5 B per bucket of the slab
 * pools; R-MAT scale 20 fits) is rejected with DG_E_OUT_OF_MEMORY and a
 * message giving both sizes, before any work is enqueued.  All calls on one
 * GPU share its area: calls that overlap on one GPU (from two threads, or on
 * two streams with work in flight) race and must not be issued.
 */
#define DG_NOALLOC_SCRATCH_BYTES (96ull << 20)
dg_status dg_bfs_noalloc(dg_graph* g, dg_epoch e, uint32_t src, int32_t* dist, void* stream);

/*
 * Strongly connected components of the snapshot at epoch e (the GetSCC query
 * named in the preamble of arXiv 2109.09527; textbook semantics): u and v
 * share a component iff each reaches the other.  comp: device array of
 * v_capacity int32, comp[v] = the smallest id in v's component for a vertex
 * live at e, -1 otherwise (an undirected graph's components are its connected
 * components).  n_components (host, optional): the number of components.
 * The call returns after the last round's counts are read back.
 */
dg_status dg_scc(dg_graph* g, dg_epoch e, int32_t* comp, uint32_t* n_components, void* stream);

/*
 * Diameter of the snapshot at epoch e (the GD query named in the preamble of
 * arXiv 2109.09527; textbook semantics): the largest number of arcs on a
 * shortest path from u to v, over ordered pairs of vertices live at e with v
 * reachable from u; 0 when no arc is visible.  Exact (a BFS from every live
 * vertex, 256 at a time, bit-parallel).  diameter: host.  The call returns
 * when the value is known.
 */
dg_status dg_diameter(dg_graph* g, dg_epoch e, uint32_t* diameter, void* stream);

/*
 * Maximum s-t flow of the snapshot at epoch e (the GetNF query named in the
 * preamble of arXiv 2109.09527; textbook semantics): arc weights are
 * capacities, an undirected edge carrying its weight in each direction.
 * flow (host) receives the value.  DG_E_VERTEX_RANGE / DG_E_SOURCE_ABSENT when
 * s or t is out of range or not live at e, DG_E_INVALID_ARG when s == t.
 * The call returns when the value is known.
 */
dg_status dg_maxflow(dg_graph* g, dg_epoch e, uint32_t s, uint32_t t, int64_t* flow, void* stream);

/*
 * DFS collect from s on the snapshot at epoch e (the GetDFS query named in
 * the preamble of arXiv 2109.09527; textbook semantics): a depth-first search
 * over the arcs visible at e, each vertex taking its out-neighbours (for an
 * undirected graph, its neighbours) in ascending id order.
 * disc: device array of v_capacity int32, disc[v] = v's position in the
 *   discovery order (s is 0), -1 where v is not reached.
 * parent (device, optional): v_capacity int32, the vertex whose arc
 *   discovered v; -1 for s and for vertices not reached.
 * n_reached (host, optional): the number of vertices reached.
 * DG_E_VERTEX_RANGE / DG_E_SOURCE_ABSENT when s is out of range or not live
 * at e; DG_E_INVALID_ARG when disc or parent is not device memory.  The visit
 * order is sequential by nature, so the walk runs on one wave.  The call
 * returns when the walk has ended; the arrays are then complete.
 */
dg_status dg_dfs(dg_graph* g, dg_epoch e, uint32_t s, int32_t* disc, int32_t* parent, uint32_t* n_reached,
                 void* stream);

/*
 * Snapshot PageRank on epoch e: Eq. (1) of arXiv 2109.09527, iterated as its
 * synchronous Barrier baseline (Alg. 1), in FP64.  With n the live vertices
 * at e and q(v) the visible out-degree, every live vertex starts at 1/n, and
 * an iteration sets pr(u) = (1 - damping)/n + damping * sum over visible arcs
 * (v, u) of pr(v)/q(v), all from the previous iteration's values.  The loop
 * stops after the first iteration whose largest |change| over the live
 * vertices is at most `threshold` (the paper uses damping 0.85 and threshold
 * 1e-16), or after max_iters iterations.  Vertices without out-arcs pass
 * nothing on (no redistribution).
 * pr: device array of v_capacity doubles, written for every id (0 where the
 *   vertex is not live at e, and everywhere when no iteration runs).
 * iterations, last_change (host, optional): iterations run and the largest
 *   change of the last one; last_change > threshold means max_iters stopped it.
 * DG_E_INVALID_ARG for damping outside [0, 1), a negative or NaN threshold,
 * or pr not in device memory.  The call returns after the last iteration's
 * change is read back; pr is then complete in stream order.
 */
dg_status dg_pagerank(dg_graph* g, dg_epoch e, double damping, double threshold, uint32_t max_iters, double* pr,
                      uint32_t* iterations, double* last_change, void* stream);

/*
 * The No-Sync PageRank of the same paper (Alg. 3, thread-level convergence):
 * the same Eq. (1) with no barrier between iterations.  Workgroups own
 * disjoint vertex ranges, update their ranks in place from whatever values
 * the others last stored, and each keeps sweeping while the largest change
 * any workgroup last published exceeds `threshold`, or until it has swept
 * max_iters times.  The result differs from run to run; at the stop it lies
 * within the convergence tolerance of the synchronous result.
 * sweeps (host, optional): the most sweeps any workgroup ran.
 * last_change (host, optional): the largest published change at the end.
 * Arguments and errors as for dg_pagerank.
 */
dg_status dg_pagerank_nosync(dg_graph* g, dg_epoch e, double damping, double threshold, uint32_t max_iters,
                             double* pr, uint32_t* sweeps, double* last_change, void* stream);

/*
 * Either form with the loop perforation of the paper's Alg. 5: a live vertex
 * whose change in an iteration (or sweep) is nonzero and below freeze_below
 * keeps its value and is not recomputed afterwards (the paper uses 1e-21
 * with threshold 1e-16).  freeze_below = 0 freezes nothing: the calls above.
 * nosync = 0 runs dg_pagerank's form, 1 dg_pagerank_nosync's.  DG_E_INVALID_ARG
 * also for a negative or NaN freeze_below, or opts NULL.
 */
typedef struct {
  double damping;
  double threshold;
  double freeze_below;
  uint32_t max_iters;
  int nosync;
} dg_pagerank_opts;
dg_status dg_pagerank_ex(dg_graph* g, dg_epoch e, const dg_pagerank_opts* opts, double* pr, uint32_t* iterations,
                         double* last_change, void* stream);

/*
 * Many queries in one persistent launch.  Each query names its kind, epoch
 * and source(s) and a caller-owned device output (int32[v_capacity] for BFS
 * and SSSP, double[v_capacity] for BC).  per_query (host, nq entries)
 * receives each query's status.  Outputs equal the single-query calls.
 */
enum { DG_Q_BFS = 0, DG_Q_SSSP = 1, DG_Q_BC = 2 };
typedef struct {
  uint32_t kind;
  uint32_t src;            /* BFS / SSSP source */
  dg_epoch epoch;
  uint32_t k;              /* BC: number of sources */
  const uint32_t* srcs;    /* BC: host array of k sources */
  void* out;               /* device output */
} dg_query;
dg_status dg_query_batch(dg_graph* g, const dg_query* q, uint32_t nq, dg_status* per_query,
                         void* stream);

/* Traversal tuning.  dg_autotune times candidate values on the latest epoch
 * and keeps the fastest; dg_get_tuning reports the values in use.  None of
 * them changes a result. */
typedef struct {
  uint32_t chunk_buckets;  /* buckets of a frontier work chunk handed to one wave: 16, 32 or 64 */
  uint32_t sssp_delta;     /* delta-stepping bucket width */
  uint32_t alpha, beta;    /* direction-switch thresholds of the BFS */
  uint32_t batch_groups;   /* workgroups per query team in the persistent launch; 0 = automatic */
  uint32_t batch_delta;    /* delta-stepping bucket width inside the persistent launch */
  uint32_t batch_gang;     /* SSSP queries advanced in lockstep by one persistent launch, 1..128; 0 = automatic */
} dg_tuning;
dg_status dg_get_tuning(const dg_graph* g, dg_tuning* t);
dg_status dg_set_tuning(dg_graph* g, const dg_tuning* t);
dg_status dg_autotune(dg_graph* g, uint32_t seed, dg_tuning* chosen, void* stream);

/*
 * Kernel timing.  While enabled, each launch of a kernel family is bracketed
 * by HIP events on the stream it runs on, and the visible arcs each launch
 * examined are counted on the device.  dg_profile_read waits for the
 * recorded events and reports, per family: launches, summed duration and
 * summed arcs.  Names are static strings owned by the library.  The entry
 * "pool_growth" counts reallocations of the slab pools instead (host clock,
 * including the wait for running engine launches to finish), and
 * "batch_sssp_scan" counts the batched engine's multi-source SSSP searches
 * with the arcs they scanned (each scan serves every query of its group;
 * "batch_sssp" counts their relaxations, one per arc and query).
 */
typedef struct {
  const char* name;
  uint64_t launches;
  double total_ms;
  uint64_t arcs;
} dg_kernel_stat;
dg_status dg_profile_enable(dg_graph* g, int on);
dg_status dg_profile_read(dg_graph* g, dg_kernel_stat* out, uint32_t cap, uint32_t* n_out, int reset);

/* Counts on epoch e: live vertices and visible arcs. */
dg_status dg_stats(dg_graph* g, dg_epoch e, uint64_t* n_vertices, uint64_t* n_arcs, void* stream);
/* Visible out-degree of every vertex at epoch e (device uint32[v_capacity]). */
dg_status dg_out_degrees(dg_graph* g, dg_epoch e, uint32_t* deg, void* stream);

/*
 * Serving loop: requests are admitted in arrival order.  Update batches run
 * on an update stream (each publishes the next epoch).  BFS and SSSP queries
 * join a running multi-source search of their kind (an executor: 64 slots
 * for BFS, 32 for SSSP): before each of its passes, waiting queries take the
 * free slots, each bound to the latest epoch published at that moment (its
 * linearization point), and a slot frees up as soon as its query's search
 * is complete.  BC queries (and, with bfs_rounds or sssp_rounds, those
 * kinds too) run on query_lanes lanes, each a host thread with a stream and an
 * engine instance of its own: a free lane takes the queries at the head of
 * its queue (up to max_batch, within max_inflight queries admitted in all)
 * and runs them in one engine call, binding each to the latest epoch
 * published when it is admitted.  Queries that arrive while a lane is busy
 * go to the next lane to come free, so the executor's passes, the lanes'
 * launches and the update batches overlap on the device.  Admission
 * reserves device memory for a query's output from mem_budget; queries wait
 * while the budget is exhausted.
 * dg_server_submit_* copy their inputs and return a ticket immediately;
 * dg_server_poll reports whether a ticket finished, its status, bound epoch
 * and latency; dg_server_take copies a finished query's output to a host
 * buffer (int32[v] or double[v]) or an update's result bytes.
 */
typedef struct dg_server dg_server;
typedef struct {
  uint64_t mem_budget;     /* bytes for in-flight query outputs; 0 = 8 GiB */
  uint32_t max_inflight;   /* queries admitted and not yet finished, over all lanes; 0 = 1024 */
  uint32_t max_batch;      /* queries fused into one launch; 0 = 64 */
  uint32_t query_lanes;    /* engine launches in flight at once, 1..4; 0 = 1 */
  uint32_t log_ops;        /* 1 = keep every update's ops for dg_server_log (16 B per op until stop) */
  uint32_t bfs_rounds;     /* 1 = BFS queries run in the lanes' rounds; 0 = in the continuous BFS executor */
  uint32_t sssp_rounds;    /* 1 = SSSP queries run in the lanes' rounds; 0 = in the continuous SSSP executor */
} dg_server_config;
typedef struct {
  uint64_t completed, updates, queries, ops_applied;
  double p50_ms, p99_ms;             /* all requests, arrival -> completion */
  double p50_query_ms, p99_query_ms, p50_update_ms, p99_update_ms;
  double wall_s;                     /* first arrival -> last completion */
  uint64_t edges_traversed;          /* sum of TEPS numerators of finished queries */
  uint64_t joined_running;           /* queries admitted into an executor's search while others ran in it */
} dg_server_stats;
dg_status dg_server_start(dg_graph* g, const dg_server_config* cfg, dg_server** out);
dg_status dg_server_stop(dg_server* s);
dg_status dg_server_submit_update(dg_server* s, const dg_op* ops, uint64_t n, uint64_t* ticket);
dg_status dg_server_submit_query(dg_server* s, uint32_t kind, const uint32_t* srcs, uint32_t k,
                                 uint64_t* ticket);
/*
 * The server's log: one record per finished request, in linearization
 * order.  An update that published epoch e comes before every query bound
 * to e, and those queries follow it in ticket order; a rejected update
 * (status < 0, no epoch published) stands, in ticket order, among the
 * queries bound to the epoch that was latest when it was applied.
 * Replaying the updates in this order on an empty graph that first receives
 * the graph's state at the server's start reproduces every epoch, and each
 * query's result is the plain query's on its epoch.
 *   recs (host, optional): the records; ops (host, optional): the op records
 *   of every update, concatenated, which are kept only when the server was
 *   started with log_ops = 1 (otherwise an update's ops_off is UINT64_MAX);
 *   srcs (host, optional): every query's sources, concatenated.
 * Each array receives at most its capacity; *n_recs / *n_ops / *n_srcs
 * (optional) receive the full counts, so a call with null arrays sizes
 * them.  Records stay until dg_server_stop; dg_server_take does not remove
 * them.
 */
typedef struct {
  uint64_t ticket;
  int32_t kind;        /* -1 update batch, else DG_Q_BFS / DG_Q_SSSP / DG_Q_BC */
  dg_status status;    /* the request's call status */
  dg_epoch epoch;      /* update: the epoch it published (rejected: the latest then); query: its bound epoch */
  uint32_t n;          /* update: ops in the batch; query: sources */
  uint64_t off;        /* index of its first op in ops[] (updates) or source in srcs[] (queries) */
  double t_arrive_ms;  /* submission, ms after dg_server_start */
  double t_done_ms;    /* completion, same clock */
} dg_log_record;
dg_status dg_server_log(dg_server* s, dg_log_record* recs, uint64_t rec_cap, uint64_t* n_recs, dg_op* ops,
                        uint64_t ops_cap, uint64_t* n_ops, uint32_t* srcs, uint64_t srcs_cap, uint64_t* n_srcs);
/* done = 1 when finished; status/epoch/latency_ms valid then. */
dg_status dg_server_poll(dg_server* s, uint64_t ticket, int* done, dg_status* status,
                         dg_epoch* epoch, double* latency_ms);
dg_status dg_server_take(dg_server* s, uint64_t ticket, void* host_out, uint64_t bytes);
dg_status dg_server_drain(dg_server* s);
dg_status dg_server_get_stats(dg_server* s, dg_server_stats* st);

#ifdef __cplusplus
}
#endif
#endif
