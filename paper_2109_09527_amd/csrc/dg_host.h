// Host-side state of a graph and the entry points of each kernel family.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dg.h"
#include "dg_internal.h"

namespace dg {

// ------------------------------------------------------------ primitives
uint64_t scan_scratch_words(uint64_t n);
void exclusive_scan_u32(uint32_t* data, uint64_t n, uint32_t* scratch, hipStream_t s);
uint64_t sort_scratch_words(uint32_t n);
bool radix_sort_pairs(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint32_t n, int bits,
                      uint32_t* scratch, hipStream_t s);

// One turn of a host thread's wait for a word the device publishes into
// pinned memory: a pause instruction for the first few thousand turns
// (about the length of a short kernel), then a yield of the core, so that
// long waits do not hold a core that other host threads need.
inline void host_pause(uint32_t turn) {
  if (turn < 4096) __builtin_ia32_pause();
  else std::this_thread::yield();
}

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};
hipError_t ensure(DevBuf& b, size_t bytes);
void release(DevBuf& b);

struct HipError {
  hipError_t e;
  const char* what;
};
#define DG_CHECK(call)                                   \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) throw ::dg::HipError{_e, #call}; \
  } while (0)

// Device counters of one update batch (zeroed at batch start).
struct UpdCounters {
  uint32_t flags;
  uint32_t nv;                  // vertex ops in the batch
  uint32_t n_touch_f, n_touch_r;
  uint32_t n_clear, n_vchange;
  uint32_t n_grow;              // slabs that grow this batch
  uint32_t pad1;
  unsigned long long arcs_delta;  // visible arcs added minus tombstoned (two's complement)
  unsigned long long demand_f, demand_r;
  unsigned long long cursor0_f, cursor0_r;
};
constexpr uint32_t VCHANGE_INLINE = 4096;   // vertex changes copied with the counters

struct UpdateScratch {
  DevBuf keys0, keys1, vals0, vals1, sortw, vafter, vlastrem, recflags, recw;
  DevBuf ops, results, touch, plan, clear;
  DevBuf grow;                  // growing slabs: touch index, new offset, kept count
  DevBuf summary;               // UpdCounters followed by the vertex-change list
  void* host_summary = nullptr; // coherent pinned copy of the first part of summary, plus a sequence word
  uint32_t pub_seq = 0;         // sequence number of the last publication
  uint64_t cap = 0;
};

// Per-query scratch for the plain (one query per launch) path.
struct QueryScratch {
  DevBuf qa, qb;                // frontier items
  DevBuf cmap_a, cmap_b;        // their chunk maps
  DevBuf fa, fb;                // BC: vertex order; bottom-up BFS: tile items
  DevBuf bm0, bm1;              // frontier bitmaps
  DevBuf stamp, flag8;          // SSSP dedup state
  DevBuf sigma, delta, level;   // BC
  DevBuf bt;                    // BC: backward tile lists and sums
  DevBuf rlist, rstamp;         // SSSP: vertices of the current bucket
  DevBuf counters;
  void* host_counters = nullptr;
  void* host_pub = nullptr;     // coherent pinned block the device publishes counters into
  uint32_t pub_seq = 0;         // sequence number of the last publication
  // fixed: the buffers are carved from a device area that is neither grown
  // nor freed, and counters are published into dev_pub (device memory,
  // copied back) instead of host_pub
  bool fixed = false;
  void* dev_pub = nullptr;
  uint64_t items_cap = 0, chunks_cap = 0;
  uint32_t lch = 6;             // log2 of the chunk size in buckets
};

// Snapshot PageRank: the in-CSR of one call and its iteration state.
struct PrScratch {
  DevBuf live, dsnap, ntiles, tile_v, tcount, off, pfirst, piece_v, csr, q, contrib, part, ring, scan;
  DevBuf sort, key0, key1, val0, val1, rank, q_r, live_r, off_r, csr_r, pr_r;   // rank order
  DevBuf pb, vb, werr, sweeps;   // No-Sync: workgroup ranges, published changes, sweep counts
  DevBuf frozen;                  // loop perforation: vertices no longer recomputed (rank order)
  void* host = nullptr;   // pinned: liveness mask upload, totals and changes read back
};

// Strongly connected components: the two snapshot CSRs, their pieces and the
// colouring state.
struct SccScratch {
  DevBuf off_in, csr_in, off_out, csr_out, pf_in, pv_in, pf_out, pv_out, colour, mark, rem, flags, scan;
  void* host = nullptr;   // pinned: counters read back
};

// Diameter: the in-arc snapshot CSR, its pieces, and the bit-parallel BFS
// words (reached, frontier, next: 4 x 64 bits per vertex each).
struct DiamScratch {
  DevBuf off, csr, pf, pv, vis, fr, nx, src, flag, scan;
  void* host = nullptr;
};

// Maximum flow: the out-arc snapshot with capacities, the arcs by target,
// flows, and the BFS state of one augmenting search.
struct FlowScratch {
  DevBuf off, csr, cap, esrc, keys0, keys1, vals0, vals1, inoff, flow, parent, queue, sort, scan, ctl;
  void* host = nullptr;
  void* pub = nullptr;   // coherent pinned: polled control words and their sequence number
  uint32_t seq = 0;
};

struct DfsScratch {
  DevBuf off, csr, keys0, keys1, vals0, vals1, par, stk, sort, ctl;
  void* host = nullptr;
};

// Multi-source SSSP (msssp.hip): one group search's buffers, carved from
// one area, and the pinned block its counters are published into.
struct MsScratch {
  DevBuf area;
  void* host = nullptr;
  uint32_t seq = 0;
  uint32_t relax_grid = 0, split_grid = 0;   // resident workgroups of its kernels
};

// Multi-source BFS (msbfs.hip): one group search's buffers and its pinned
// counter block.
struct MfScratch {
  DevBuf area;
  void* host = nullptr;
  uint32_t seq = 0;
  uint32_t pass_grid = 0, final_grid = 0;   // resident workgroups of its kernels
};

// Multi-source BC (msbc.hip): one group search's buffers and its pinned
// counter block.
struct MbScratch {
  DevBuf area;
  void* host = nullptr;
  uint32_t seq = 0;
  uint32_t fwd_grid = 0, bwd_grid = 0, tiles_grid = 0;
};

// Per-kernel-family event timing (dg_profile_*).
enum KernelId {
  KID_UPDATE = 0,   // the whole update pipeline of one batch
  KID_BFS_TD,
  KID_BFS_BU,
  KID_SSSP_RELAX,
  KID_SSSP_SPLIT,
  KID_BC_FWD,
  KID_BC_BWD,
  KID_BATCH_BFS,    // one persistent multi-query launch, per query kind
  KID_BATCH_SSSP,
  KID_BATCH_BC,
  KID_PAGERANK,     // one PageRank iteration (pull and apply)
  KID_PAGERANK_NOSYNC,  // one No-Sync PageRank launch
  KID_SCC,          // one colouring or collecting pass of the SCC query
  KID_DIAMETER,     // one level of a bit-parallel BFS sweep (diameter)
  KID_MAXFLOW,      // one level of an augmenting-path search (maximum flow)
  KID_DFS,          // the one-wave depth-first walk
  KID_POOL_GROW,    // one reallocation of the bucket pools (host clock, waits included)
  KID_BATCH_SSSP_SCAN,  // multi-source SSSP searches: arcs scanned once for a whole group
  KID_SERVE_BFS,    // one expansion pass of the serving loop's BFS executor
  KID_SERVE_SSSP,   // one relaxation pass of the serving loop's SSSP executor
  KID_COUNT
};
// Kernel timing state.  Several host threads time kernels at once (the
// serving loop's update thread, lanes and executors), so every access to the
// event pool, the pending records and the totals holds mu (a leaf lock:
// nothing else is taken while it is held).
struct Prof {
  std::mutex mu;
  bool on = false;
  struct Rec {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  uint64_t launches[KID_COUNT] = {};
  double ms[KID_COUNT] = {};
  uint64_t arcs[KID_COUNT] = {};
};

struct Tuning {
  uint32_t chunk_buckets = 64;
  uint32_t sssp_delta = 64;
  uint32_t alpha = 14, beta = 24;
  uint32_t batch_groups = 0;   // workgroups per query team; 0 = automatic
  uint32_t batch_delta = 512;  // delta of the SSSP queries inside a batch launch
  uint32_t batch_gang = 0;     // SSSP queries per lockstep launch; 0 = automatic
};

}  // namespace dg

struct dg_graph {
  dg_config cfg{};
  int device = 0;
  uint32_t L = 1;               // key bits per vertex id
  dg::Store st{};
  dg::DevBuf fdesc, rdesc, fused, rused, fpool, rpool, fsum, rsum, cursor, alive, insf, insr;
  uint32_t epoch = 0;           // latest published epoch
  std::map<uint32_t, int> pins;
  // vertex liveness history: first toggle epoch per vertex (0 = never);
  // later toggles form a chain per vertex through vlog, newest first
  // (vlog[i] = {epoch, the vertex's previous entry}; vhead[v] = its newest,
  // VLOG_NONE for none), and vtoggled lists each vertex with a chain once.
  // Appending costs no allocation per change: a hash map of per-vertex
  // vectors had cost about 60 us per batch of 300 vertex changes.
  std::vector<uint32_t> vfirst;
  std::vector<uint32_t> vhead;
  std::vector<std::pair<uint32_t, uint32_t>> vlog;
  std::vector<uint32_t> vtoggled;
  uint64_t n_live = 0;
  std::vector<uint64_t> arcs_by_epoch{0};   // visible arcs at each epoch
  std::vector<uint64_t> live_by_epoch{0};   // live vertices at each epoch
  dg::UpdateScratch us;
  dg::QueryScratch qs;
  dg::PrScratch pr;
  dg::SccScratch scc;
  dg::DiamScratch diam;
  dg::FlowScratch flow;
  dg::DfsScratch dfs;
  dg::Tuning tune;
  dg::Prof prof;
  int concurrent_writers = 0;   // >0 while the serving loop may update under running queries
  uint32_t engine_share_pct = 100;  // share of resident workgroup slots a batch launch may fill
  std::atomic<uint64_t> engine_arcs{0};  // visible arcs examined by all batch launches
  hipEvent_t last_query = nullptr;  // end of the last plain query's work; updates wait for it
  std::string err;
  std::mutex mu;                // host state: epoch, pins, history, store descriptors
  // Engine launches copy the store descriptors (pool base addresses) under
  // mu and then run without it; a pool reallocation or compaction, which
  // frees the old pools, waits until none of them is running
  // (pool_readers), and new readers wait while one is pending.
  std::condition_variable pool_cv;
  int pool_readers = 0;
  int pool_writers = 0;
  // A search that spans many passes (the serving loop's BFS executor) keeps
  // slab descriptors in its frontier between passes: compaction, which
  // moves slabs, waits until no such search runs (search_holds), and
  // searches admit no new queries while a compaction waits.
  int search_holds = 0;
  std::atomic<int> compact_waiting{0};
  // Set by the serving loop while it applies an update batch: multi-pass
  // searches hold their next pass back for a while (yield_to_updates), so
  // the batch's short dependent kernels find free compute units.
  std::atomic<int> update_running{0};
  std::mutex upd_mu;            // one update batch (or compaction) at a time
};

namespace dg {
// graph-level helpers (api.cpp)
// With g->mu held in lk: wait until no pool reallocation is pending, then
// count the caller as a reader of the store descriptors it copies next.
void pool_read_begin(dg_graph* g, std::unique_lock<std::mutex>& lk);
// Ends a read begun by pool_read_begin (takes g->mu).
void pool_read_end(dg_graph* g);
// Waits (up to 4 ms) while the serving loop applies an update batch.
void yield_to_updates(dg_graph* g);
uint32_t gc_floor(const dg_graph* g);
constexpr uint32_t VLOG_NONE = 0xFFFFFFFFu;
bool alive_at(const dg_graph* g, uint32_t v, uint32_t e);
bool is_device_ptr(const void* p);
hipError_t grow_pools(dg_graph* g, uint64_t need_f, uint64_t need_r);

// Event bracket around one launch of a kernel family (no-op unless enabled).
struct ProfScope {
  dg_graph* g;
  int kid;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(dg_graph* g_, int kid_, hipStream_t s_);
  ~ProfScope();
};
void prof_arcs(dg_graph* g, int kid, uint64_t arcs);
// Counts one search of a family that is not timed by itself, with `arcs`.
void prof_scans(dg_graph* g, int kid, uint64_t arcs);

// update.hip: sizes the batch scratch (us.*) for n ops; callers that stage
// ops into us.ops do so after this, since growing it replaces the buffer.
hipError_t ensure_update_scratch(dg_graph* g, uint64_t n);
// update.hip: runs one batch; returns a dg_status.
dg_status apply_batch_dev(dg_graph* g, const dg_op* dops, uint64_t n, uint8_t* dres, hipStream_t s);

// query.hip
dg_status bfs_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* dist, hipStream_t s, QueryScratch& q);
dg_status sssp_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* dist, hipStream_t s, QueryScratch& q);
dg_status bc_dev(dg_graph* g, uint32_t e, const uint32_t* srcs, uint32_t k, double* bc, hipStream_t s,
                 QueryScratch& q);
dg_status stats_dev(dg_graph* g, uint32_t e, uint64_t* n_arcs, uint32_t* deg, hipStream_t s);
// Lays a BFS's buffers out from base into q (marked fixed) and returns the
// bytes they take; with q null only the size.
uint64_t bfs_fixed_layout(const dg_graph* g, char* base, QueryScratch* q);
// noalloc.hip: finds the device address of the fixed area on `device`
// (which must be current) once; noalloc_area returns it (null before set-up).
hipError_t noalloc_setup(int device);
void* noalloc_area(int device);
void free_query_scratch(QueryScratch& q);

// pagerank.hip
dg_status pagerank_dev(dg_graph* g, uint32_t e, double damping, double threshold, double freeze_below,
                       uint32_t max_iters, double* pr, uint32_t* iters, double* last_change, hipStream_t s,
                       bool nosync);
void free_pr_scratch(PrScratch& s);
// Snapshot helpers shared by the whole-graph queries (they use the PageRank
// build scratch): liveness at e as a device byte mask, and the visible arcs
// at e of the live vertices' slabs in `pool` as a CSR (off: V + 1 entries;
// csr: the other endpoint of each arc, in slab order); m = arcs.  With wts,
// also each arc's weight (forward pool only).
hipError_t snapshot_live(dg_graph* g, uint32_t e, DevBuf& live, hipStream_t s);
hipError_t snapshot_csr(dg_graph* g, uint32_t e, const Pool& pool, const uint64_t* desc, const uint8_t* live,
                        DevBuf& off, DevBuf& csr, uint32_t* m, hipStream_t s, DevBuf* wts = nullptr);
// scc.hip
dg_status scc_dev(dg_graph* g, uint32_t e, int32_t* comp, uint32_t* n_comp, uint32_t* rounds, hipStream_t s);
void free_scc_scratch(SccScratch& s);
// diameter.hip
dg_status diameter_dev(dg_graph* g, uint32_t e, uint32_t* diameter, hipStream_t s);
void free_diam_scratch(DiamScratch& s);
// flow.hip
dg_status maxflow_dev(dg_graph* g, uint32_t e, uint32_t src, uint32_t dst, int64_t* flow, hipStream_t s);
void free_flow_scratch(FlowScratch& s);
dg_status dfs_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* disc, int32_t* parent, uint32_t* n_reached,
                  hipStream_t s);
void free_dfs_scratch(DfsScratch& s);

// msbfs.hip: up to ms_bfs_width() BFS queries of one snapshot e (sources
// srcs, outputs outs[i], int32 hop distances, -1 unreached) as one
// multi-source BFS on stream s; adds the visible arcs examined to *arcs_out.
uint32_t ms_bfs_width();
dg_status ms_bfs_dev(dg_graph* g, const Store& st, uint32_t e, int fast, const uint32_t* srcs, uint32_t k,
                     void* const* outs, uint32_t chunk_buckets, MfScratch& mf, hipStream_t s, uint64_t* arcs_out);
void free_mf_scratch(MfScratch& mf);

// msssp.hip: up to ms_sssp_width() SSSP queries of one snapshot e (sources
// srcs[0..k), device outputs outs[0..k), host arrays) as one delta-stepping
// search over a shared frontier; adds the relaxations to *arcs_out.
uint32_t ms_sssp_width();
dg_status ms_sssp_dev(dg_graph* g, const Store& st, uint32_t e, int fast, const uint32_t* srcs, uint32_t k,
                      void* const* outs, int32_t delta, uint32_t chunk_buckets, MsScratch& ms, hipStream_t s,
                      uint64_t* arcs_out);
void free_ms_scratch(MsScratch& ms);
// msbc.hip: up to ms_bc_width() distinct sources srcs[0..k) (host) of one BC
// query on snapshot e as one search; adds their dependencies to the device
// array bc in source order (bc must hold the sums of earlier sources, or
// zeros); adds the arcs examined to *arcs_out.  DG_E_OVERFLOW when a path
// count exceeds int64.
uint32_t ms_bc_width();
dg_status ms_bc_dev(dg_graph* g, const Store& st, uint32_t e, int fast, const uint32_t* srcs, uint32_t k, double* bc,
                    uint32_t chunk_buckets, MbScratch& mb, hipStream_t s, uint64_t* arcs_out);
void free_mb_scratch(MbScratch& mb);

// batch.hip
// lane: engine instance (its own buffers); lanes may run at once on
// different streams, each within its share of the resident workgroups.
dg_status query_batch_dev(dg_graph* g, const dg_query* q, uint32_t nq, dg_status* per_query,
                          hipStream_t s, uint32_t lane);
void free_batch_state(dg_graph* g);

}  // namespace dg
