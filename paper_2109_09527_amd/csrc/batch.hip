// Batched queries: many BFS / SSSP / BC queries, on any mix of retained
// epochs, in one call.  Queries of one kind on one snapshot share adjacency
// scans: BFS groups of up to 64 (msbfs.hip), SSSP groups of up to 32
// (msssp.hip) and BC queries of 4 or more sources (msbc.hip) run as
// multi-source searches driven level by level from the host.  The rest runs
// in a persistent engine, one launch per query kind:
//
// BFS and BC run in teams.  The grid holds at most 90% of the workgroups
// that can be resident at once (from the occupancy API).  Workgroups join
// teams of S in the order they start running, so a team's members are
// resident together; a team becomes active only when all S members have
// joined, and members still waiting when the query queue runs dry leave
// without work (the forming / active / dead state is settled by one
// compare-and-swap, so every member takes the same decision).  An active
// team takes the next query from a device counter, runs it level by level
// with the steps of frontier.h over its own scratch, separating levels with
// a team barrier (arrival counter + generation word in global memory, a
// release fence before it and an acquire fence after it, so no workgroup
// reads stale lines of another's writes), and takes the next query when
// done.  Each query terminates on its own.
//
// SSSP runs in lockstep gangs (below): the whole grid is one team, and all
// queries of the gang advance one delta-stepping pass at a time over their
// combined frontiers, so the thin passes of many queries fill the GPU
// together.
//
// Every wait is bounded by a wall-clock limit: a workgroup that waits too
// long sets an abort flag that releases every other waiter, so the launch
// always drains.  Only one engine launch runs on a device at a time
// (workgroups spin on each other, so two engines could starve each other of
// resident workgroups).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>

#include "dg_host.h"
#include "frontier.h"

namespace dg {

// Arrival counters of a team barrier: members arrive at one of up to
// SYNC_FAN counters, whose last arrivals arrive at the team counter.
constexpr uint32_t SYNC_FAN = 32;

// One arrival counter and its release word, on a 128-byte line of its own.
struct alignas(128) SyncLine {
  uint32_t count;   // members of this group at the current barrier
  uint32_t gen;     // barriers released
  uint32_t pad[30];
};

struct TeamSync {
  uint32_t count;    // groups complete at the current barrier
  uint32_t q;        // the team's current query (engine teams)
  uint32_t joined;   // members that have started
  uint32_t state;    // 0 forming, 1 active, 2 dead
  uint32_t pad[28];
  SyncLine line[SYNC_FAN];
};

// A workgroup's place in its team's barrier.
struct BarrierPos {
  uint32_t gen;   // barriers passed
  uint32_t w;     // index of the workgroup in its team
};

struct Ctrl {
  uint32_t next;
  uint32_t abort;
  uint32_t arrive;   // start order of the workgroups
  uint32_t done;     // queries finished
  unsigned long long arcs;   // visible arcs examined by the launch
  uint32_t pad[10];
};

// Worker 0 adds a finished step's examined-arc count to the launch total.
__device__ inline void add_step_arcs(Ctrl* c, const QCounters* step, uint32_t w) {
  if (w == 0 && threadIdx.x == 0) {
    unsigned long long n = ld_relaxed(&step->arcs);
    if (n) atomicAdd(&c->arcs, n);
  }
}

// One engine job: a query (for BC, k sources in srcs).
struct QDesc {
  uint32_t kind, src, epoch, k;
  const uint32_t* srcs;   // device copy of BC sources
  void* out;
};

// Scratch of one team (device pointers into one allocation).
struct TeamScratch {
  Item* qa;
  Item* qb;
  uint32_t* cmap_a;       // chunk maps of qa / qb
  uint32_t* cmap_b;
  uint32_t qcap, ccap;    // their capacities
  uint32_t lch;           // log2 of the chunk size
  Item* qbig;
  uint32_t* bm0;          // three rotating frontier bitmaps
  uint32_t* bm1;
  uint32_t* bm2;
  QCounters* cnt;         // [0..2] rotating level counters, [3] BC totals
  uint32_t* fa;
  uint32_t* fb;
  uint32_t* stamp;
  uint32_t* infar;
  unsigned long long* sigma;
  double* delta;          // BC: (1 + dependency) / path count of each finished vertex
  int32_t* level;
  uint32_t* off;          // BC: start of each level in the discovery order
  uint32_t* rlist;        // SSSP bucket record list (aliases sigma)
  uint32_t* rstamp;       // SSSP bucket record stamps (aliases delta)
  TeamSync* sync;
};

// uni_scratch copies every field; a new field must be added there too.
static_assert(sizeof(TeamScratch) == 4 * 8 + 4 * 4 + 16 * 8, "TeamScratch layout changed: update uni_scratch");

struct BatchArgs {
  Store st;
  int fast;
  int32_t delta;
  int32_t w_max;
  uint32_t alpha, beta;
  const QDesc* q;
  const uint32_t* qidx;   // indices of this launch's queries (one kind)
  uint32_t nq;
  int32_t* status;        // per query
  const uint64_t* arcs;   // visible arcs per epoch
  const uint64_t* live;   // live vertices per epoch
  const TeamScratch* teams;
  uint32_t n_teams, team_size;
  Ctrl* ctrl;
  uint64_t spin_ticks;    // longest wait, in wall-clock ticks
};

// Wait, bounded, until *p differs from old; a timeout or another member's
// abort sets the launch's abort flag.
__device__ inline bool wait_change(const uint32_t* p, uint32_t old, Ctrl* ctrl, uint64_t spin_ticks) {
  const uint64_t t0 = wall_clock64();
  for (uint32_t k = 1; ld_relaxed(p) == old; k++) {
    __builtin_amdgcn_s_sleep(1);
    if (wall_clock64() - t0 > spin_ticks || ((k & 15) == 0 && ld_relaxed(&ctrl->abort))) {
      atomicExch(&ctrl->abort, 1u);
      return false;
    }
  }
  return true;
}

// Team barrier.  Each member writes its data back from its XCD's L2
// (agent-scope release by one wave, after the workgroup barrier) and
// arrives at counter w mod F; the last arrival of a counter arrives at the
// team counter, and the last of those releases every counter's waiters.
// After the release, one wave per workgroup invalidates its CU's L1 and its
// XCD's L2 (agent-scope acquire); the workgroup barrier after it orders the
// other waves behind that invalidation.  Fanning arrivals over F counters
// keeps each counter's chain of same-address atomics short.
// Returns false when a wait timed out or another member aborted.
__device__ inline bool team_barrier(TeamSync* ts, uint32_t S, BarrierPos& bp, Ctrl* ctrl, Shared& sh,
                                    uint64_t spin_ticks) {
  __syncthreads();
  const uint32_t my = bp.gen;
  bp.gen = my + 1;
  if (threadIdx.x < 64) {
    uint32_t ab = 0;
    if (S > 1) {
      const uint32_t F = S < SYNC_FAN ? S : SYNC_FAN;
      const uint32_t grp = bp.w % F, ng = S / F + (grp < S % F ? 1u : 0u);
      uint32_t last = 0;
      if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (atomicAdd(&ts->line[grp].count, 1u) == ng - 1) {
          atomicExch(&ts->line[grp].count, 0u);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (atomicAdd(&ts->count, 1u) == F - 1) {
            atomicExch(&ts->count, 0u);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            last = 1;
          }
        }
      }
      last = __shfl(last, 0);
      if (last) {
        for (uint32_t i = threadIdx.x; i < F; i += 64) st_relaxed(&ts->line[i].gen, my + 1);
      } else if (threadIdx.x == 0 && !wait_change(&ts->line[grp].gen, my, ctrl, spin_ticks)) {
        ab = 1;
      }
    }
    if (threadIdx.x == 0) sh.flag = ab | ld_relaxed(&ctrl->abort);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return sh.flag == 0;
}

// Rotating bitmap i (selected without indexing a register array).
__device__ inline uint32_t* bm_at(const TeamScratch& ts, uint32_t i) {
  uint64_t p0 = (uint64_t)ts.bm0, p1 = (uint64_t)ts.bm1, p2 = (uint64_t)ts.bm2;
  return (uint32_t*)(i == 0 ? p0 : (i == 1 ? p1 : p2));
}

template <class T>
__device__ inline void team_fill(T* p, uint64_t n, T v, uint32_t w, uint32_t S) {
  for (uint64_t i = (uint64_t)w * Q_THREADS + threadIdx.x; i < n; i += (uint64_t)S * Q_THREADS) p[i] = v;
}

__device__ inline QCounters read_cnt(const QCounters* c) {
  // every lane reads the same settled counters (after a team barrier)
  QCounters r;
  r.fq = uni(ld_relaxed(&c->fq));
  r.n_verts = uni(ld_relaxed(&c->n_verts));
  r.m_next = uni(ld_relaxed(&c->m_next));
  r.n_far = uni(ld_relaxed(&c->n_far));
  r.far_min = uni(ld_relaxed(&c->far_min));
  r.overflow = uni(ld_relaxed(&c->overflow));
  r.n_order = uni(ld_relaxed(&c->n_order));
  r.n_big = uni(ld_relaxed(&c->n_big));
  return r;
}

// A team's scratch and a query's descriptor are read by every lane from
// the same address; these copies make that uniformity visible, so the
// pointers live in scalar registers instead of occupying two vector
// registers each for the whole launch.
__device__ inline TeamScratch uni_scratch(const TeamScratch& x) {
  TeamScratch r;
  r.qa = uni(x.qa);
  r.qb = uni(x.qb);
  r.cmap_a = uni(x.cmap_a);
  r.cmap_b = uni(x.cmap_b);
  r.qcap = uni(x.qcap);
  r.ccap = uni(x.ccap);
  r.lch = uni(x.lch);
  r.qbig = uni(x.qbig);
  r.bm0 = uni(x.bm0);
  r.bm1 = uni(x.bm1);
  r.bm2 = uni(x.bm2);
  r.cnt = uni(x.cnt);
  r.fa = uni(x.fa);
  r.fb = uni(x.fb);
  r.stamp = uni(x.stamp);
  r.infar = uni(x.infar);
  r.sigma = uni(x.sigma);
  r.delta = uni(x.delta);
  r.level = uni(x.level);
  r.off = uni(x.off);
  r.rlist = uni(x.rlist);
  r.rstamp = uni(x.rstamp);
  r.sync = uni(x.sync);
  return r;
}

__device__ inline QDesc uni_desc(const QDesc& x) {
  QDesc r;
  r.kind = uni(x.kind);
  r.src = uni(x.src);
  r.epoch = uni(x.epoch);
  r.k = uni(x.k);
  r.srcs = uni(x.srcs);
  r.out = uni(x.out);
  return r;
}

__device__ inline Front team_front(const TeamScratch& ts, int which) {
  return Front{which ? ts.qb : ts.qa, which ? ts.cmap_b : ts.cmap_a, ts.qcap, ts.ccap, ts.lch};
}

// Worker 0 of the team writes the seed frontier of src into queue qa, its
// chunk map and counters slot 0 (the caller has set dist/level[src] and
// cleared the other slots).
__device__ inline void team_seed(const Store& st, uint32_t src, const TeamScratch& ts, QCounters* c0, uint32_t w) {
  if (w != 0) return;
  const uint64_t desc = st.fdesc[src];
  const uint32_t nb = desc ? 1u << (desc & 63) : 0;
  const uint32_t nc = (nb + (1u << ts.lch) - 1) >> ts.lch;
  for (uint32_t c = threadIdx.x; c < nc && c < ts.ccap; c += blockDim.x) ts.cmap_a[c] = 0;
  if (threadIdx.x != 0) return;
  if (nb) ts.qa[0] = Item{desc, src, 0};
  c0->fq = nb ? 1ull | ((unsigned long long)nb << 32) : 0ull;
  c0->n_verts = 1;
  c0->m_next = st.fused[src];
}

#define BARRIER()                                          \
  do {                                                     \
    if (!team_barrier(ts.sync, S, bp, a.ctrl, sh, a.spin_ticks)) return false; \
  } while (0)

// A frontier queue ran out of room: the query fails (every member reads the
// same counters after the barrier, so all leave together).
#define QUEUE_CHECK(cnt)                                                          \
  do {                                                                            \
    if (ld_relaxed(&(cnt)->overflow) & OVF_QUEUE) {                               \
      if (w == 0 && threadIdx.x == 0) *status = DG_E_OUT_OF_MEMORY;              \
      return true;                                                                \
    }                                                                             \
  } while (0)

__device__ __forceinline__ bool run_bfs(const BatchArgs& a, const QDesc& qd, const TeamScratch& ts, uint32_t w,
                                        uint32_t S, BarrierPos& bp, Shared& sh, int32_t* status) {
  const uint32_t V = a.st.V;
  const uint64_t bmw = (V + 31) / 32 + 1;
  int32_t* dist = static_cast<int32_t*>(qd.out);
  team_fill<int32_t>(dist, V, -1, w, S);
  team_fill<uint32_t>(ts.bm0, bmw, 0u, w, S);
  team_fill<uint32_t>(ts.bm1, bmw, 0u, w, S);
  if (w == 0 && threadIdx.x == 0)
    for (int i = 0; i < 3; i++) zero_counters(&ts.cnt[i]);
  BARRIER();
  if (w == 0 && threadIdx.x == 0) {
    dist[qd.src] = 0;
    ts.bm0[qd.src >> 5] |= 1u << (qd.src & 31);
  }
  team_seed(a.st, qd.src, ts, &ts.cnt[0], w);
  BARRIER();
  int64_t m_u = (int64_t)a.arcs[qd.epoch];
  const uint64_t n_live = a.live[qd.epoch] ? a.live[qd.epoch] : 1;
  bool bu = false;
  for (uint32_t level = 0;; level++) {
    QCounters c = read_cnt(&ts.cnt[level % 3]);
    if (c.n_verts == 0) break;
    if (!bu && (int64_t)c.m_next * (int64_t)a.alpha > m_u) bu = true;
    else if (bu && (uint64_t)c.n_verts * a.beta < n_live) bu = false;
    m_u -= (int64_t)c.m_next;
    QCounters* cout = &ts.cnt[(level + 1) % 3];
    uint32_t* bnext = bm_at(ts, (level + 1) % 3);
    team_fill<uint32_t>(bm_at(ts, (level + 2) % 3), bmw, 0u, w, S);
    if (w == 0 && threadIdx.x == 0) zero_counters(&ts.cnt[(level + 2) % 3]);
    LevelArgs la{a.st,   qd.epoch, a.fast, team_front(ts, level & 1), team_front(ts, (level + 1) & 1), ts.qbig,
                 bm_at(ts, level % 3), bnext, dist, (int32_t)level + 1, cout};
    if (bu) {
      bu_step(la, w, S, sh);
      BARRIER();
      bu_big_step(la, uni(ld_relaxed(&cout->n_big)), w, S, sh);
    } else {
      td_step(la, c.fq, w, S, sh);
    }
    BARRIER();
    add_step_arcs(a.ctrl, cout, w);
    QUEUE_CHECK(cout);
  }
  return true;
}

__device__ __forceinline__ bool run_bc(const BatchArgs& a, const QDesc& qd, const TeamScratch& ts, uint32_t w,
                                       uint32_t S, BarrierPos& bp, Shared& sh, int32_t* status) {
  const uint32_t V = a.st.V;
  double* bc = static_cast<double*>(qd.out);
  team_fill<double>(bc, V, 0.0, w, S);
  for (uint32_t si = 0; si < qd.k; si++) {
    const uint32_t src = qd.srcs[si];
    team_fill<int32_t>(ts.level, V, -1, w, S);
    team_fill<unsigned long long>(ts.sigma, V, 0ull, w, S);
    if (w == 0 && threadIdx.x == 0)
      for (int i = 0; i < 4; i++) zero_counters(&ts.cnt[i]);
    BARRIER();
    if (w == 0 && threadIdx.x == 0) {
      ts.level[src] = 0;
      ts.sigma[src] = 1ull;
      ts.fa[0] = src;
      ts.cnt[3].n_order = 1;
      ts.off[0] = 0;
      ts.off[1] = 1;
    }
    team_seed(a.st, src, ts, &ts.cnt[0], w);
    BARRIER();
    uint32_t nlev = 1;   // levels discovered so far (level 0 = src)
    for (uint32_t lvl = 0;; lvl++) {
      QCounters c = read_cnt(&ts.cnt[lvl % 3]);
      if (lvl > 0 && c.n_verts == 0) break;
      QCounters* cout = &ts.cnt[(lvl + 1) % 3];
      if (w == 0 && threadIdx.x == 0) zero_counters(&ts.cnt[(lvl + 2) % 3]);
      BcFwdArgs fa{a.st,     qd.epoch,  a.fast,   team_front(ts, lvl & 1), team_front(ts, (lvl + 1) & 1),
                   ts.fa,    ts.level,  ts.sigma, (int32_t)lvl + 1,        cout,
                   &ts.cnt[3]};
      bcfwd_step(fa, c.fq, w, S, sh);
      BARRIER();
      add_step_arcs(a.ctrl, cout, w);
      QUEUE_CHECK(cout);
      uint32_t found = uni(ld_relaxed(&cout->n_verts));
      if (found == 0) break;
      if (w == 0 && threadIdx.x == 0) ts.off[nlev + 1] = ts.off[nlev] + found;
      nlev++;
    }
    // the backward's tile lists live in the bottom-up chunk buffer, which
    // a BC job does not otherwise use; the counts start at zero
    const BwdTiles bt = bwd_tiles_at(reinterpret_cast<char*>(ts.qbig), a.st.fp.cap, 1);
    if (w == 0 && threadIdx.x == 0) {
      bt.head->verts[0] = bt.head->verts[1] = 0;
      bt.head->tiles[0] = bt.head->tiles[1] = 0;
      bt.head->ovf = 0;
    }
    BARRIER();
    if (ld_relaxed(&ts.cnt[3].overflow) & OVF_SIGMA) {
      if (w == 0 && threadIdx.x == 0) *status = DG_E_OVERFLOW;
      return true;
    }
    for (int L = (int)nlev - 1; L >= 0; L--) {
      uint32_t o0 = uni(ld_relaxed(&ts.off[L])), o1 = uni(ld_relaxed(&ts.off[L + 1]));
      bcbwd_step(a.st, qd.epoch, a.fast != 0, ts.fa + o0, o1 - o0, src, ts.level, L, ts.sigma, ts.delta, bc, bt, w,
                 S);
      BARRIER();
      const uint32_t nt = uni(ld_relaxed(&bt.head->tiles[L & 1]));
      if (nt) {
        bcbwd_tiles(a.st, qd.epoch, a.fast != 0, ts.level, L, ts.delta, bt, nt, w, S);
        BARRIER();
        bcbwd_combine(bt, uni(ld_relaxed(&bt.head->verts[L & 1])), src, ts.sigma, ts.delta, bc, w, S);
        BARRIER();
      }
    }
    if (ld_relaxed(&bt.head->ovf)) {
      if (w == 0 && threadIdx.x == 0) *status = DG_E_OUT_OF_MEMORY;
      return true;
    }
  }
  return true;
}

// One launch serves the queries of one kind, so each kind's kernel gets its
// own register allocation.
// Join a team in start order; returns false when the team never becomes
// active (queue exhausted first, or a wait timed out).
__device__ inline bool team_join(Ctrl* ctrl, uint32_t nq, uint64_t spin_ticks, TeamSync* sync, uint32_t S,
                                 uint32_t w, Shared& sh, BarrierPos& bp) {
  if (threadIdx.x == 0) {
    uint32_t go = 0;
    if (atomicAdd(&sync->joined, 1u) + 1 == S) {
      go = atomicCAS(&sync->state, 0u, 1u) == 0u;
    } else {
      const uint64_t t0 = wall_clock64();
      for (;;) {
        uint32_t stt = ld_relaxed(&sync->state);
        if (stt == 1u) { go = 1; break; }
        if (stt == 2u) break;
        if (ld_relaxed(&ctrl->next) >= nq || ld_relaxed(&ctrl->abort)) {
          uint32_t old = atomicCAS(&sync->state, 0u, 2u);
          if (old == 1u) { go = 1; break; }
          break;
        }
        if (wall_clock64() - t0 > spin_ticks) {
          // a team that cannot assemble dissolves; the host checks that
          // every query was still served
          uint32_t old = atomicCAS(&sync->state, 0u, 2u);
          go = old == 1u;
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
    }
    sh.flag = go;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  bp.gen = 0;
  bp.w = w;
  return sh.flag != 0;
}

// One launch serves the queries of one kind, so each kind's kernel gets its
// own register allocation.
template <int KIND>
__global__ __launch_bounds__(Q_THREADS, 4) void k_team(BatchArgs a) {
  __shared__ Shared sh;
  if (threadIdx.x == 0) sh.base = atomicAdd(&a.ctrl->arrive, 1u);
  __syncthreads();
  const uint32_t slot = uni(sh.base);
  const uint32_t S = a.team_size;
  const uint32_t t = slot / S, w = slot % S;
  if (t >= a.n_teams) return;
  const TeamScratch ts = uni_scratch(a.teams[t]);
  BarrierPos bp;
  if (!team_join(a.ctrl, a.nq, a.spin_ticks, ts.sync, S, w, sh, bp)) return;
  for (;;) {
    if (w == 0 && threadIdx.x == 0) ts.sync->q = atomicAdd(&a.ctrl->next, 1u);
    if (!team_barrier(ts.sync, S, bp, a.ctrl, sh, a.spin_ticks)) return;
    const uint32_t k = uni(ld_relaxed(&ts.sync->q));
    if (k >= a.nq) return;
    const uint32_t qi = uni(a.qidx[k]);
    const QDesc qd = uni_desc(a.q[qi]);
    bool ok = true;
    if (a.status[qi] == DG_OK) {
      if (KIND == DG_Q_BFS) ok = run_bfs(a, qd, ts, w, S, bp, sh, &a.status[qi]);
      else ok = run_bc(a, qd, ts, w, S, bp, sh, &a.status[qi]);
    }
    if (!ok || !team_barrier(ts.sync, S, bp, a.ctrl, sh, a.spin_ticks)) return;
    if (w == 0 && threadIdx.x == 0) atomicAdd(&a.ctrl->done, 1u);
  }
}


// ----------------------------------------------------- lockstep SSSP gang
//
// All SSSP queries of a gang advance together, one pass at a time, in one
// persistent launch whose workgroups form a single team.  A pass does, for
// every query still running, the next step of its delta-stepping (a relax
// pass over its near frontier, light / heavy / all arcs; the item expansion
// of a settled bucket's recorded vertices; or a split of its far set at a
// raised threshold).  The work units of all queries (frontier chunks, blocks
// of 64 list entries) form one index space, cut into equal contiguous
// ranges, one per wave; a grid barrier ends the pass.  Every workgroup then
// reads the counters of all queries and advances an identical copy of each
// query's state machine in its LDS, so no further synchronisation is needed
// to agree on the next pass.  Thin delta-stepping buckets of many queries
// thus fill the GPU together, and each query's per-pass cost is one barrier
// shared by the gang instead of one host round trip of its own.

constexpr uint32_t GANG_BLOCK = 64;   // units per round-robin block of a pass
constexpr uint32_t GANG_MAX = 128;   // queries per gang launch (LDS and registers sized for 5 waves per SIMD)

enum GKind : uint32_t { G_RELAX = 0, G_EXPAND = 1, G_HEAVY = 2, G_SPLIT = 3, G_DONE = 4 };

// Scratch and output of one query (device pointers, fixed for the launch).
struct GQuery {
  uint32_t epoch;
  int32_t* dist;
  Item* qa;
  Item* qb;
  uint32_t* cmap_a;
  uint32_t* cmap_b;
  uint32_t* stamp;
  uint32_t* infar;
  uint32_t* rlist;
  uint32_t* rstamp;
  QCounters* cnt;   // [0..2] rotating pass counters, [3].n_order bucket record count
};

// A query's delta-stepping state, kept identically by every workgroup.
struct GState {
  unsigned long long near;   // fq of the near frontier
  uint32_t kind, n_far, n_rec, it, phase, slot, qi;
  int32_t thr, far_min;
  uint32_t reset_rec;        // clear the bucket record count in the next plan
};

struct GangArgs {
  Store st;
  int fast;
  int32_t delta;
  int32_t w_max;
  uint32_t qcap, ccap, lch;
  const GQuery* q;
  int32_t* status;
  uint32_t nq;
  TeamSync* sync;
  Ctrl* ctrl;
  uint64_t spin_ticks;
};

__device__ inline Front gang_front(const GangArgs& a, const GQuery& q, uint32_t which) {
  return Front{which ? q.qb : q.qa, which ? q.cmap_b : q.cmap_a, a.qcap, a.ccap, a.lch};
}

__device__ inline uint32_t gang_units(const GangArgs& a, const GState& s) {
  switch (s.kind) {
    case G_RELAX:
    case G_HEAVY: return min(fq_chunks(s.near, a.lch), a.ccap);
    case G_EXPAND: return (min(s.n_rec, a.st.V) + 63) / 64;
    case G_SPLIT: return (a.st.V + 63) / 64;
    default: return 0;
  }
}

// Leave the bucket: split the far set (at a threshold one delta higher),
// or finish.
__device__ inline void gang_to_split(GState& s, int32_t delta) {
  if (s.n_far == 0) {
    s.kind = G_DONE;
    return;
  }
  s.kind = G_SPLIT;
  s.far_min = DIST_INF;
  s.thr = (int32_t)min((int64_t)DIST_INF, (int64_t)s.thr + delta);
}

// Advance query q's state after a pass, from the counters that pass wrote.
//
// Workgroups reach this point at different times, and workgroup 0 may
// already be planning the next pass while others still read these
// counters; so nothing read here is written by the next pass's plan or
// work: the pass counters rotate over three slots, and the bucket record
// count is cleared only in the plan of the pass after an expansion.
__device__ inline void gang_advance(const GangArgs& a, const GQuery& q, GState& s, int32_t* status) {
  s.reset_rec = 0;
  if (s.kind == G_DONE) return;
  const bool split_lh = a.delta < a.w_max;
  const uint32_t nx = (s.slot + 1) % 3;
  const QCounters* c = &q.cnt[nx];
  const unsigned long long fq = ld_relaxed(&c->fq);
  if (ld_relaxed(&c->overflow) & OVF_QUEUE) {
    *status = DG_E_OUT_OF_MEMORY;
    s.kind = G_DONE;
    return;
  }
  switch (s.kind) {
    case G_RELAX:
    case G_HEAVY: {
      const bool heavy = s.kind == G_HEAVY;
      s.near = fq;
      s.n_far += ld_relaxed(&c->n_far);
      s.qi ^= 1;
      s.it++;
      s.slot = nx;
      if (heavy) s.phase++;
      else if (split_lh) s.n_rec = ld_relaxed(&q.cnt[3].n_order);
      if (s.near) s.kind = G_RELAX;
      else if (!heavy && split_lh && s.n_rec) s.kind = G_EXPAND;
      else {
        if (!heavy && split_lh) s.phase++;
        gang_to_split(s, a.delta);
      }
      break;
    }
    case G_EXPAND:
      s.slot = nx;
      s.n_rec = 0;
      s.reset_rec = 1;
      if (fq) {
        s.near = fq;
        s.kind = G_HEAVY;
      } else {
        s.phase++;
        gang_to_split(s, a.delta);
      }
      break;
    case G_SPLIT: {
      s.slot = nx;
      s.n_far = ld_relaxed(&c->n_far);
      s.near = fq;
      s.far_min = ld_relaxed(&c->far_min);
      if (s.near) {
        s.it++;
        s.kind = G_RELAX;
      } else if (s.n_far) {
        // raise the threshold until some far entry falls below it
        s.thr = (int32_t)min((int64_t)DIST_INF, ((int64_t)s.far_min / a.delta + 1) * a.delta);
      } else {
        s.kind = G_DONE;
      }
      break;
    }
  }
}

// Units [j0, j1) of query qn's current step, by the calling wave.
__device__ inline GQuery uni_gquery(const GQuery& x) {
  GQuery r;
  r.epoch = uni(x.epoch);
  r.dist = uni(x.dist);
  r.qa = uni(x.qa);
  r.qb = uni(x.qb);
  r.cmap_a = uni(x.cmap_a);
  r.cmap_b = uni(x.cmap_b);
  r.stamp = uni(x.stamp);
  r.infar = uni(x.infar);
  r.rlist = uni(x.rlist);
  r.rstamp = uni(x.rstamp);
  r.cnt = uni(x.cnt);
  return r;
}
static_assert(sizeof(GQuery) == 8 + 10 * 8, "GQuery layout changed: update uni_gquery");

__device__ inline GState uni_state(const GState& x) {
  GState r;
  r.near = uni(x.near);
  r.kind = uni(x.kind);
  r.n_far = uni(x.n_far);
  r.n_rec = uni(x.n_rec);
  r.it = uni(x.it);
  r.phase = uni(x.phase);
  r.slot = uni(x.slot);
  r.qi = uni(x.qi);
  r.thr = uni(x.thr);
  r.far_min = uni(x.far_min);
  r.reset_rec = uni(x.reset_rec);
  return r;
}
static_assert(sizeof(GState) == 8 + 10 * 4, "GState layout changed: update uni_state");

// Returns the visible arcs the wave examined (counted into the launch
// total once per wave, at the end of the launch).
__device__ __forceinline__ unsigned long long gang_work(const GangArgs& a, uint32_t qn, const GState& s, uint32_t j0,
                                                        uint32_t j1, Shared& sh) {
  const GQuery q = uni_gquery(a.q[qn]);
  const uint32_t wave = threadIdx.x >> 6;
  const bool split_lh = a.delta < a.w_max;
  QCounters* cout = &q.cnt[(s.slot + 1) % 3];
  ItemQ qn_ = item_q(sh.ws[wave], 0, WSTAGE);
  LaneCounts lc;
  if (s.kind == G_RELAX || s.kind == G_HEAVY) {
    const int mode = s.kind == G_HEAVY ? 2 : (split_lh ? 1 : 0);
    RelaxArgs ra{a.st,    q.epoch,  a.fast,           gang_front(a, q, s.qi), gang_front(a, q, s.qi ^ 1),
                 q.dist,  q.stamp,  q.infar,          s.thr,                  s.it,
                 cout,    mode,     a.delta,          q.rlist,                &q.cnt[3].n_order,
                 q.rstamp, s.phase};
    const uint32_t nitems = front_items(ra.fin, s.near), nb = fq_buckets(s.near);
    for (uint32_t c = j0; c < j1; c++) relax_chunk(ra, c, nitems, nb, qn_, lc);
    flush_front(qn_, ra.fout, cout);
  } else if (s.kind == G_EXPAND) {
    const Front f = gang_front(a, q, s.qi);
    const uint32_t n_rec = min(s.n_rec, a.st.V);
    for (uint32_t b = j0; b < j1; b++) expand_block(a.st, q.rlist, n_rec, b * 64, f, cout, qn_);
    flush_front(qn_, f, cout);
  } else {
    SplitArgs sa{a.st, gang_front(a, q, s.qi), q.dist, q.stamp, q.infar, s.thr, s.it, cout};
    int32_t mn = DIST_INF;
    for (uint32_t b = j0; b < j1; b++) split_block(sa, b * 64, qn_, lc, mn);
    flush_front(qn_, sa.fout, cout);
    commit_far_min(mn, cout);
  }
  return lc.commit_wave(cout);
}

__global__ __launch_bounds__(Q_THREADS, 5) void k_gang_sssp(GangArgs a) {
  __shared__ Shared sh;
  __shared__ GState gs[GANG_MAX];
  __shared__ uint32_t pre[GANG_MAX + 1];
  if (threadIdx.x == 0) sh.base = atomicAdd(&a.ctrl->arrive, 1u);
  __syncthreads();
  const uint32_t w = uni(sh.base), S = gridDim.x;
  BarrierPos bp;
  if (!team_join(a.ctrl, 0xFFFFFFFFu, a.spin_ticks, a.sync, S, w, sh, bp)) return;
  const uint32_t nq = a.nq;
  for (uint32_t i = threadIdx.x; i < nq; i += Q_THREADS) {
    GState s{};
    s.near = ld_relaxed(&a.q[i].cnt[0].fq);
    s.kind = s.near ? G_RELAX : G_DONE;
    s.thr = a.delta;
    s.far_min = DIST_INF;
    s.it = 1;
    s.phase = 1;
    gs[i] = s;
  }
  const uint32_t wave = threadIdx.x >> 6, nw = S * Q_WAVES, gw = w * Q_WAVES + wave;
  unsigned long long wave_arcs = 0;
  for (;;) {
    // plan the pass: units per query and their prefix (nq <= Q_THREADS)
    __syncthreads();
    const uint32_t my = threadIdx.x < nq ? gang_units(a, gs[threadIdx.x]) : 0;
    uint32_t total;
    const uint32_t ex = block_excl_scan(my, &total, sh);
    if (threadIdx.x < nq) pre[threadIdx.x] = ex;
    if (threadIdx.x == 0) pre[nq] = total;
    if (w == 0 && threadIdx.x < nq) {
      // clear the counters the pass after this one will fill, and the
      // bucket record count once its expansion is done
      const GState& s = gs[threadIdx.x];
      if (s.kind != G_DONE) zero_counters(&a.q[threadIdx.x].cnt[(s.slot + 2) % 3]);
      if (s.reset_rec) st_relaxed(&a.q[threadIdx.x].cnt[3].n_order, 0u);
    }
    __syncthreads();
    total = uni(total);
    if (total == 0) break;
    // blocks of GANG_BLOCK units dealt round-robin to the waves: each wave
    // gets work of many queries, so queries in a costly phase (many
    // improvements and pushes) do not pile onto a few waves
    for (uint32_t b = gw; (uint64_t)b * GANG_BLOCK < total; b += nw) {
      uint32_t u = b * GANG_BLOCK;
      const uint32_t hi = min(total, u + GANG_BLOCK);
      while (u < hi) {
        uint32_t l = 0, h = nq;   // pre[l] <= u < pre[h]
        while (h - l > 1) {
          const uint32_t m = (l + h) >> 1;
          if (pre[m] <= u) l = m;
          else h = m;
        }
        const uint32_t qn = uni(l);
        const uint32_t p0 = uni(pre[qn]), end = min(hi, uni(pre[qn + 1]));
        wave_arcs += gang_work(a, qn, uni_state(gs[qn]), u - p0, end - p0, sh);
        u = end;
      }
    }
    if (!team_barrier(a.sync, S, bp, a.ctrl, sh, a.spin_ticks)) return;
    for (uint32_t i = threadIdx.x; i < nq; i += Q_THREADS) gang_advance(a, a.q[i], gs[i], &a.status[i]);
  }
  if (lane_id() == 0 && wave_arcs) atomicAdd(&a.ctrl->arcs, wave_arcs);
  if (w == 0 && threadIdx.x == 0) atomicAdd(&a.ctrl->done, nq);
}

// Per-query start state of a gang: grid (x: blocks over V, y: query).
__global__ void k_gang_init(const GQuery* gq, uint32_t V, int split_lh) {
  const GQuery q = gq[blockIdx.y];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < V; i += gridDim.x * blockDim.x) {
    q.dist[i] = DIST_INF;
    q.stamp[i] = 0u;
    q.infar[i] = 0u;
    if (split_lh) q.rstamp[i] = 0u;
  }
}

// Seed query blockIdx.x at its source: dist 0, the source's item and chunk
// map, counters slot 0 = the seed frontier, other slots cleared.  One wave
// per query, after k_gang_init.
__global__ void k_gang_seed(const GQuery* gq, const uint32_t* src, Store st, uint32_t ccap, uint32_t lch) {
  const GQuery q = gq[blockIdx.x];
  const uint32_t v = src[blockIdx.x];
  const uint64_t desc = st.fdesc[v];
  const uint32_t nb = desc ? 1u << (desc & 63) : 0;
  const uint32_t nc = (nb + (1u << lch) - 1) >> lch;
  for (uint32_t c = threadIdx.x; c < nc && c < ccap; c += blockDim.x) q.cmap_a[c] = 0;
  if (threadIdx.x != 0) return;
  if (nb) q.qa[0] = Item{desc, v, 0};
  q.dist[v] = 0;
  for (int i = 0; i < 4; i++) zero_counters(&q.cnt[i]);
  q.cnt[0].fq = nb ? 1ull | ((unsigned long long)nb << 32) : 0ull;
}

__global__ void k_gang_finish(const GQuery* gq, uint32_t V) {
  int32_t* d = gq[blockIdx.y].dist;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < V; i += gridDim.x * blockDim.x)
    if (d[i] == DIST_INF) d[i] = -1;
}

// out[v] = sum over t < k of part[t * V + v], added in t order.
__global__ void k_bc_sum(const double* part, uint32_t k, uint64_t V, double* out) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (uint64_t)gridDim.x * blockDim.x) {
    double r = 0.0;
    for (uint32_t t = 0; t < k; t++) r += part[(uint64_t)t * V + v];
    out[v] = r;
  }
}

// ------------------------------------------------------------ host side

struct BatchState {
  std::mutex mu;                 // one batch at a time per graph (shared buffers)
  uint64_t spin_ticks = 0;       // 2 s of the device wall clock
  DevBuf scratch, teams, qdesc, qidx, srcs, outs, status, arcs, live, ctrl;
  int grid_cap[3] = {0, 0, 0};   // resident workgroups of each kind's engine kernel
  DevBuf gang_scratch, gq, gsrc, gsync, gctrl, gstatus;
  int gang_cap = 0;              // resident workgroups of the gang kernel
  DevBuf bc_part;                // per-source dependency arrays of split BC queries
  uint32_t* hflag = nullptr;     // completion sequence number (coherent pinned memory)
  uint32_t seq = 0;
  void* hres = nullptr;          // pinned landing area of per-query statuses and control records
  size_t hres_bytes = 0;
  MfScratch mf;                  // multi-source BFS groups
  MsScratch ms;                  // multi-source SSSP groups
  MbScratch mb;                  // multi-source BC groups
};

// Completion of everything enqueued on s so far, seen by polling: a one-wave
// kernel stores a sequence number to coherent pinned memory (system scope)
// and the host spins on it, so the wait does not depend on how the runtime
// blocks inside a stream synchronisation.  Not seen within two seconds, the
// wait falls back to synchronising the stream, which reports any device
// error.
__global__ void k_batch_signal(uint32_t* flag, uint32_t seq) {
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

static hipError_t host_area(BatchState* bs, size_t bytes) {
  hipError_t e;
  if (!bs->hflag) {
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&bs->hflag), 64, hipHostMallocCoherent)) != hipSuccess) {
      bs->hflag = nullptr;
      return e;
    }
    *bs->hflag = 0;
    bs->seq = 0;
  }
  if (bs->hres_bytes < bytes) {
    if (bs->hres) (void)hipHostFree(bs->hres);
    bs->hres = nullptr;
    bs->hres_bytes = 0;
    if ((e = hipHostMalloc(&bs->hres, bytes, hipHostMallocDefault)) != hipSuccess) {
      bs->hres = nullptr;
      return e;
    }
    bs->hres_bytes = bytes;
  }
  return hipSuccess;
}

static hipError_t wait_polled(BatchState* bs, hipStream_t s) {
  const uint32_t seq = ++bs->seq;
  k_batch_signal<<<1, 64, 0, s>>>(bs->hflag, seq);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 1; __atomic_load_n(bs->hflag, __ATOMIC_ACQUIRE) != seq; spin++) {
    host_pause(spin);
    if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (__atomic_load_n(bs->hflag, __ATOMIC_ACQUIRE) != seq) return hipErrorUnknown;
      break;
    }
  }
  return hipSuccess;
}

static std::mutex g_engine_mu;   // one engine launch enqueued per process at a time
// Engine state per (graph, lane): each lane owns its buffers, so launches of
// different lanes can be in flight together on different streams.
static std::map<std::pair<const dg_graph*, uint32_t>, BatchState*> g_states;
static std::mutex g_states_mu;

static BatchState* state_of(dg_graph* g, uint32_t lane) {
  std::lock_guard<std::mutex> lk(g_states_mu);
  auto& p = g_states[{g, lane}];
  if (!p) p = new BatchState();
  return p;
}

void free_batch_state(dg_graph* g) {
  std::lock_guard<std::mutex> lk(g_states_mu);
  for (auto it = g_states.begin(); it != g_states.end();) {
    if (it->first.first != g) {
      ++it;
      continue;
    }
    BatchState* b = it->second;
    for (DevBuf* d : {&b->scratch, &b->teams, &b->qdesc, &b->qidx, &b->srcs, &b->outs, &b->status, &b->arcs,
                      &b->live, &b->ctrl, &b->gang_scratch, &b->gq, &b->gsrc, &b->gsync, &b->gctrl, &b->gstatus,
                      &b->bc_part})
      release(*d);
    if (b->hflag) (void)hipHostFree(b->hflag);
    if (b->hres) (void)hipHostFree(b->hres);
    free_mf_scratch(b->mf);
    free_ms_scratch(b->ms);
    free_mb_scratch(b->mb);
    delete b;
    it = g_states.erase(it);
  }
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Bytes of one team's scratch and, if base is set, the pointers into it.
static uint64_t team_layout(const Store& st, uint32_t chunk_buckets, char* base, TeamScratch* ts) {
  const uint64_t V = st.V;
  const uint64_t items = V + 1024;          // a frontier holds each vertex at most once
  const uint64_t chunks = st.fp.cap / CH_MIN + 2;
  const uint64_t big = V + std::max(st.fp.cap, st.rp.cap) / BU_CHUNK + 1024;
  const uint64_t bmw = (V + 31) / 32 + 1;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o;
    o += align256(bytes);
    return base ? base + at : nullptr;
  };
  char* p;
  p = take(items * sizeof(Item)); if (ts) ts->qa = reinterpret_cast<Item*>(p);
  p = take(items * sizeof(Item)); if (ts) ts->qb = reinterpret_cast<Item*>(p);
  p = take(chunks * 4); if (ts) ts->cmap_a = reinterpret_cast<uint32_t*>(p);
  p = take(chunks * 4); if (ts) ts->cmap_b = reinterpret_cast<uint32_t*>(p);
  if (ts) {
    ts->qcap = (uint32_t)std::min<uint64_t>(items, 0xFFFFFFFFu);
    ts->ccap = (uint32_t)std::min<uint64_t>(chunks, 0xFFFFFFFFu);
    ts->lch = 31 - __builtin_clz(chunk_buckets);
  }
  // a BC job keeps its backward tile lists here
  p = take(std::max<uint64_t>(big * sizeof(Item), bwd_tiles_bytes(st.fp.cap, 1))); if (ts) ts->qbig = reinterpret_cast<Item*>(p);
  p = take(bmw * 4); if (ts) ts->bm0 = reinterpret_cast<uint32_t*>(p);
  p = take(bmw * 4); if (ts) ts->bm1 = reinterpret_cast<uint32_t*>(p);
  p = take(bmw * 4); if (ts) ts->bm2 = reinterpret_cast<uint32_t*>(p);
  p = take(4 * sizeof(QCounters)); if (ts) ts->cnt = reinterpret_cast<QCounters*>(p);
  p = take(V * 4 + 64); if (ts) ts->fa = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (ts) ts->fb = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (ts) ts->stamp = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (ts) ts->infar = reinterpret_cast<uint32_t*>(p);
  p = take(V * 8 + 64); if (ts) ts->sigma = reinterpret_cast<unsigned long long*>(p);
  if (ts) ts->rlist = reinterpret_cast<uint32_t*>(p);
  p = take(V * 8 + 64); if (ts) ts->delta = reinterpret_cast<double*>(p);
  if (ts) ts->rstamp = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (ts) ts->level = reinterpret_cast<int32_t*>(p);
  p = take((V + 2) * 4 + 64); if (ts) ts->off = reinterpret_cast<uint32_t*>(p);
  p = take(sizeof(TeamSync)); if (ts) ts->sync = reinterpret_cast<TeamSync*>(p);
  return o;
}

bool alive_at(const dg_graph* g, uint32_t v, uint32_t e);

static dg_status bfail(dg_graph* g, dg_status st, const std::string& m) {
  g->err = m;
  return st;
}

static const void* kernel_of(int kind) {
  if (kind == DG_Q_BFS) return reinterpret_cast<const void*>(&k_team<DG_Q_BFS>);
  return reinterpret_cast<const void*>(&k_team<DG_Q_BC>);
}

// Bytes of one gang query's scratch and, if base is set, its pointers.
static uint64_t gang_layout(const Store& st, char* base, GQuery* q) {
  const uint64_t V = st.V;
  const uint64_t items = V + 1024;
  const uint64_t chunks = st.fp.cap / CH_MIN + 2;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o;
    o += align256(bytes);
    return base ? base + at : nullptr;
  };
  char* p;
  p = take(items * sizeof(Item)); if (q) q->qa = reinterpret_cast<Item*>(p);
  p = take(items * sizeof(Item)); if (q) q->qb = reinterpret_cast<Item*>(p);
  p = take(chunks * 4); if (q) q->cmap_a = reinterpret_cast<uint32_t*>(p);
  p = take(chunks * 4); if (q) q->cmap_b = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (q) q->stamp = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (q) q->infar = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (q) q->rlist = reinterpret_cast<uint32_t*>(p);
  p = take(V * 4 + 64); if (q) q->rstamp = reinterpret_cast<uint32_t*>(p);
  p = take(4 * sizeof(QCounters)); if (q) q->cnt = reinterpret_cast<QCounters*>(p);
  return o;
}

// The SSSP queries idx[] of a batch, in gangs of lockstep queries.
static dg_status run_sssp_gangs(dg_graph* g, BatchState* bs, const Store& st_, const Tuning& tune, int fast,
                                uint32_t share, const std::vector<QDesc>& qd, const std::vector<uint32_t>& idx,
                                std::vector<int32_t>& st, uint64_t budget, hipStream_t s) {
  hipError_t e;
  const uint32_t V = st_.V;
  const int32_t delta = (int32_t)std::max<uint32_t>(1, tune.batch_delta);
  const int split_lh = delta < g->cfg.w_max ? 1 : 0;
  const uint64_t per_q = gang_layout(st_, nullptr, nullptr);
  const uint32_t want = tune.batch_gang ? std::min<uint32_t>(tune.batch_gang, GANG_MAX) : GANG_MAX;
  const uint32_t gang = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>({(uint64_t)want, budget / per_q, (uint64_t)idx.size()}));
  if (!bs->gang_cap) {
    int per_cu = 0, cus = 0, dev = 0;
    hipGetDevice(&dev);
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_gang_sssp, Q_THREADS, 0)) !=
            hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return bfail(g, DG_E_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
    bs->gang_cap = std::max(1, per_cu * cus);
  }
  const uint32_t G = std::max<uint32_t>(1, (uint32_t)((uint64_t)bs->gang_cap * 9 / 10 * share / 100));
  const uint32_t lch = 31 - __builtin_clz(tune.chunk_buckets);
  if ((e = ensure(bs->gang_scratch, per_q * gang)) != hipSuccess ||
      (e = ensure(bs->gq, gang * sizeof(GQuery))) != hipSuccess || (e = ensure(bs->gsrc, gang * 4)) != hipSuccess ||
      (e = ensure(bs->gsync, sizeof(TeamSync))) != hipSuccess || (e = ensure(bs->gctrl, sizeof(Ctrl))) != hipSuccess ||
      (e = ensure(bs->gstatus, gang * 4)) != hipSuccess)
    return bfail(g, DG_E_OUT_OF_MEMORY, "gang scratch allocation");
  for (size_t g0 = 0; g0 < idx.size(); g0 += gang) {
    const uint32_t n = (uint32_t)std::min<size_t>(gang, idx.size() - g0);
    std::vector<GQuery> gq(n);
    std::vector<uint32_t> src(n);
    std::vector<int32_t> gst(n, DG_OK);
    for (uint32_t i = 0; i < n; i++) {
      const QDesc& d = qd[idx[g0 + i]];
      gang_layout(st_, bs->gang_scratch.as<char>() + per_q * i, &gq[i]);
      gq[i].epoch = d.epoch;
      gq[i].dist = static_cast<int32_t*>(d.out);
      src[i] = d.src;
    }
    Ctrl c0{};
    if ((e = hipMemcpyAsync(bs->gq.p, gq.data(), n * sizeof(GQuery), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(bs->gsrc.p, src.data(), n * 4, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(bs->gstatus.p, gst.data(), n * 4, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(bs->gctrl.p, &c0, sizeof(c0), hipMemcpyHostToDevice, s)) ||
        (e = hipMemsetAsync(bs->gsync.p, 0, sizeof(TeamSync), s)))
      return bfail(g, DG_E_HIP, std::string("gang upload: ") + hipGetErrorString(e));
    const dim3 fill_grid(std::max<uint32_t>(1, std::min<uint32_t>((V + 255) / 256, 1024)), n);
    k_gang_init<<<fill_grid, 256, 0, s>>>(bs->gq.as<GQuery>(), V, split_lh);
    k_gang_seed<<<n, 64, 0, s>>>(bs->gq.as<GQuery>(), bs->gsrc.as<uint32_t>(), st_,
                                 (uint32_t)std::min<uint64_t>(st_.fp.cap / CH_MIN + 2, 0xFFFFFFFFu), lch);
    GangArgs a{st_,
               fast,
               delta,
               (int32_t)g->cfg.w_max,
               (uint32_t)std::min<uint64_t>((uint64_t)V + 1024, 0xFFFFFFFFu),
               (uint32_t)std::min<uint64_t>(st_.fp.cap / CH_MIN + 2, 0xFFFFFFFFu),
               lch,
               bs->gq.as<GQuery>(),
               bs->gstatus.as<int32_t>(),
               n,
               bs->gsync.as<TeamSync>(),
               bs->gctrl.as<Ctrl>(),
               bs->spin_ticks};
    {
      ProfScope ps(g, KID_BATCH_SSSP, s);
      k_gang_sssp<<<G, Q_THREADS, 0, s>>>(a);
    }
    k_gang_finish<<<fill_grid, 256, 0, s>>>(bs->gq.as<GQuery>(), V);
    if ((e = hipGetLastError()) != hipSuccess)
      return bfail(g, DG_E_HIP, std::string("gang launch: ") + hipGetErrorString(e));
    Ctrl cres;
    const size_t st_bytes = align256(n * 4ull);
    if ((e = host_area(bs, st_bytes + sizeof(Ctrl))) != hipSuccess ||
        (e = hipMemcpyAsync(bs->hres, bs->gstatus.p, n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(static_cast<char*>(bs->hres) + st_bytes, bs->gctrl.p, sizeof(cres),
                            hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = wait_polled(bs, s)) != hipSuccess)
      return bfail(g, DG_E_HIP, std::string("gang: ") + hipGetErrorString(e));
    std::memcpy(gst.data(), bs->hres, n * 4);
    std::memcpy(&cres, static_cast<char*>(bs->hres) + st_bytes, sizeof(cres));
    if (cres.abort) return bfail(g, DG_E_HIP, "gang engine: a barrier timed out");
    if (cres.done != n) return bfail(g, DG_E_HIP, "gang engine: the gang could not assemble");
    prof_arcs(g, KID_BATCH_SSSP, cres.arcs);
    g->engine_arcs += cres.arcs;
    for (uint32_t i = 0; i < n; i++) st[idx[g0 + i]] = gst[i];
  }
  return DG_OK;
}

dg_status query_batch_dev(dg_graph* g, const dg_query* q, uint32_t nq, dg_status* per_query, hipStream_t s,
                          uint32_t lane) {
  if (nq == 0) return DG_OK;
  if (!q || !per_query) return bfail(g, DG_E_INVALID_ARG, "null query array or status array");
  BatchState* bs = state_of(g, lane);
  std::lock_guard<std::mutex> blk(bs->mu);
  hipError_t e;
  // host state is read (and the epochs in use pinned) under the graph
  // mutex; the launch itself runs without it, beside update batches
  Store st_;
  Tuning tune;
  uint32_t share = 100;
  std::vector<uint64_t> arcs, live;
  int fast = 1;
  std::vector<QDesc> qd(nq);
  std::vector<int32_t> st(nq, DG_OK);
  std::vector<uint32_t> all_srcs;
  std::vector<uint64_t> src_off(nq, 0);
  std::vector<uint32_t> by_kind[3];
  std::vector<uint32_t> pinned;
  // the copied descriptors hold the pools' base addresses: pool
  // reallocation waits until this call's last launch has finished
  struct PoolRead {
    dg_graph* g;
    bool on = false;
    ~PoolRead() {
      if (on) pool_read_end(g);
    }
  } pool_read{g};
  {
    std::unique_lock<std::mutex> lk(g->mu);
    pool_read_begin(g, lk);
    pool_read.on = true;
    st_ = g->st;
    tune = g->tune;
    arcs = g->arcs_by_epoch;
    live = g->live_by_epoch;
    fast = g->concurrent_writers ? 0 : 1;
    share = std::max<uint32_t>(1, std::min<uint32_t>(100, g->engine_share_pct));
    const uint32_t fl = gc_floor(g);
    for (uint32_t i = 0; i < nq; i++) {
      const dg_query& x = q[i];
      uint32_t ep = x.epoch == DG_EPOCH_LATEST ? g->epoch : x.epoch;
      qd[i] = QDesc{x.kind, x.src, ep, 0, nullptr, x.out};
      if (x.kind > DG_Q_BC || !x.out || !is_device_ptr(x.out)) { st[i] = DG_E_INVALID_ARG; continue; }
      if (ep > g->epoch || ep < fl) { st[i] = DG_E_EPOCH_RETIRED; continue; }
      if (x.kind == DG_Q_BC) {
        if (x.k && !x.srcs) { st[i] = DG_E_INVALID_ARG; continue; }
        std::vector<uint32_t> S(x.srcs, x.srcs + x.k);
        for (uint32_t v : S) {
          if (v >= g->cfg.v_capacity) { st[i] = DG_E_VERTEX_RANGE; break; }
          if (!alive_at(g, v, ep)) { st[i] = DG_E_SOURCE_ABSENT; break; }
        }
        std::vector<uint32_t> sorted = S;
        std::sort(sorted.begin(), sorted.end());
        if (st[i] == DG_OK && std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
          st[i] = DG_E_INVALID_ARG;
        src_off[i] = all_srcs.size();
        all_srcs.insert(all_srcs.end(), S.begin(), S.end());
        qd[i].k = x.k;
      } else {
        if (x.src >= g->cfg.v_capacity) st[i] = DG_E_VERTEX_RANGE;
        else if (!alive_at(g, x.src, ep)) st[i] = DG_E_SOURCE_ABSENT;
      }
      if (st[i] == DG_OK) {
        by_kind[x.kind].push_back(i);
        if (g->pins[ep]++ == 0) pinned.push_back(ep);
        else pinned.push_back(ep);
      }
    }
  }
  // unpin on every exit path
  struct Unpin {
    dg_graph* g;
    std::vector<uint32_t>& eps;
    ~Unpin() {
      std::lock_guard<std::mutex> lk(g->mu);
      for (uint32_t ep : eps) {
        auto it = g->pins.find(ep);
        if (it != g->pins.end() && --it->second == 0) g->pins.erase(it);
      }
    }
  } unpin{g, pinned};
  // BFS queries on one snapshot run in groups of up to ms_bfs_width() as
  // one multi-source BFS each (host-driven levels, a kernel boundary per
  // level); fewer than MS_MIN stay single and run in the engine's teams
  constexpr size_t MS_MIN = 4;
  std::vector<std::vector<uint32_t>> bgroups;
  {
    std::map<uint32_t, std::vector<uint32_t>> by_ep;
    for (uint32_t i : by_kind[DG_Q_BFS]) by_ep[qd[i].epoch].push_back(i);
    std::vector<uint32_t> single;
    const size_t W = ms_bfs_width();
    for (auto& kv : by_ep) {
      const std::vector<uint32_t>& v = kv.second;
      for (size_t o = 0; o < v.size(); o += W) {
        const size_t n = std::min<size_t>(W, v.size() - o);
        if (n < MS_MIN) single.insert(single.end(), v.begin() + o, v.begin() + o + n);
        else bgroups.emplace_back(v.begin() + o, v.begin() + o + n);
      }
    }
    by_kind[DG_Q_BFS] = single;
  }
  // SSSP queries on one snapshot run in groups of up to ms_sssp_width() as
  // one multi-source search each (a shared frontier, the group's distances
  // of a vertex in one line); fewer than MS_MIN stay single and run in the
  // lockstep gangs
  std::vector<std::vector<uint32_t>> sgroups;
  {
    std::map<uint32_t, std::vector<uint32_t>> by_ep;
    for (uint32_t i : by_kind[DG_Q_SSSP]) by_ep[qd[i].epoch].push_back(i);
    std::vector<uint32_t> single;
    const size_t W = ms_sssp_width();
    for (auto& kv : by_ep) {
      const std::vector<uint32_t>& v = kv.second;
      for (size_t o = 0; o < v.size(); o += W) {
        const size_t n = std::min<size_t>(W, v.size() - o);
        if (n < MS_MIN) single.insert(single.end(), v.begin() + o, v.begin() + o + n);
        else sgroups.emplace_back(v.begin() + o, v.begin() + o + n);
      }
    }
    by_kind[DG_Q_SSSP] = single;
  }
  // A BC query of at least MS_MIN sources runs as multi-source searches of
  // up to ms_bc_width() sources each (after the engine launch), adding its
  // sources' dependencies in order, bit for bit as the plain call does.
  std::vector<uint32_t> mbq;
  {
    std::vector<uint32_t> rest;
    for (uint32_t i : by_kind[DG_Q_BC]) (qd[i].k >= MS_MIN ? mbq : rest).push_back(i);
    by_kind[DG_Q_BC] = rest;
  }
  // A BC query of k > 1 sources runs as k one-source jobs, each writing its
  // own dependency array, when those fit the engine's memory budget; a
  // reduction then adds the k arrays in source order.  A single
  // team would have added the same per-source terms to zero in the same
  // order (x + 0 = x exactly where a source does not reach or is the
  // vertex), so the sum is the same bit for bit, and the sources run on
  // k teams at once.
  const uint64_t budget = g->cfg.mem_budget ? g->cfg.mem_budget / 4 : (16ull << 30);
  struct BcSplit {
    uint32_t q, j0, k;
    uint64_t off;   // first partial array, in doubles from the partials buffer
  };
  std::vector<BcSplit> splits;
  uint64_t part_words = 0;
  {
    const uint64_t V = st_.V;
    std::vector<uint32_t> jobs, whole;   // whole: multi-source queries left unsplit
    for (uint32_t i : by_kind[DG_Q_BC]) {
      const uint32_t k = qd[i].k;
      if (k < 2 || (part_words + (uint64_t)k * V) * 8 > budget) {
        (k < 2 ? jobs : whole).push_back(i);
        continue;
      }
      splits.push_back(BcSplit{i, (uint32_t)qd.size(), k, part_words});
      part_words += (uint64_t)k * V;
      for (uint32_t t = 0; t < k; t++) {
        jobs.push_back((uint32_t)qd.size());
        src_off.push_back(src_off[i] + t);
        qd.push_back(QDesc{DG_Q_BC, 0, qd[i].epoch, 1, nullptr, nullptr});
        st.push_back(DG_OK);
      }
    }
    // the longest jobs (unsplit multi-source queries) are taken first
    whole.insert(whole.end(), jobs.begin(), jobs.end());
    by_kind[DG_Q_BC] = whole;
  }
  const uint32_t nj = (uint32_t)qd.size();   // queries, group jobs and BC source jobs
  // resident workgroups per kind's kernel
  for (int k = 0; k < 3; k++) {
    if (bs->grid_cap[k] || by_kind[k].empty() || k == DG_Q_SSSP) continue;
    int per_cu = 0, cus = 0, dev = 0;
    hipGetDevice(&dev);
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_of(k), Q_THREADS, 0)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return bfail(g, DG_E_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
    bs->grid_cap[k] = std::max(1, per_cu * cus);
  }
  if (!bs->spin_ticks) {
    int khz = 0, dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    bs->spin_ticks = (uint64_t)khz * 1000ull * 2ull;
  }
  // teams: size from the tuning (0 = automatic), count bounded by memory
  const uint64_t per_team = team_layout(st_, tune.chunk_buckets, nullptr, nullptr);
  const uint32_t max_teams = (uint32_t)std::max<uint64_t>(1, budget / per_team);
  uint32_t S_of[3] = {1, 1, 1}, T_of[3] = {0, 0, 0}, most = 1;
  for (int k = 0; k < 3; k++) {
    uint32_t n = (uint32_t)by_kind[k].size();
    if (!n || k == DG_Q_SSSP) continue;   // SSSP runs in lockstep gangs
    // 90% of the resident capacity (times the share a server leaves to the engine)
    const uint32_t G = std::max<uint32_t>(1, (uint32_t)((uint64_t)bs->grid_cap[k] * 9 / 10 * share / 100));
    uint32_t S = tune.batch_groups;
    if (S == 0 || S > G) S = std::max<uint32_t>(1, G / std::min<uint32_t>(n, max_teams));
    S_of[k] = S;
    T_of[k] = std::max<uint32_t>(1, std::min<uint32_t>({G / S, n, max_teams}));
    most = std::max(most, T_of[k]);
  }
  size_t e_cnt = arcs.size();
  if ((e = ensure(bs->scratch, per_team * most)) != hipSuccess)
    return bfail(g, DG_E_OUT_OF_MEMORY, "batch scratch allocation");
  std::vector<TeamScratch> tsv(most);
  for (uint32_t t = 0; t < most; t++) team_layout(st_, tune.chunk_buckets, bs->scratch.as<char>() + per_team * t, &tsv[t]);
  if ((e = ensure(bs->teams, most * sizeof(TeamScratch))) != hipSuccess ||
      (e = ensure(bs->qdesc, nj * sizeof(QDesc))) != hipSuccess || (e = ensure(bs->qidx, nj * 4)) != hipSuccess ||
      (e = ensure(bs->srcs, std::max<size_t>(1, all_srcs.size()) * 4)) != hipSuccess ||
      (e = ensure(bs->status, nj * 4)) != hipSuccess || (e = ensure(bs->arcs, e_cnt * 8)) != hipSuccess ||
      (e = ensure(bs->live, e_cnt * 8)) != hipSuccess || (e = ensure(bs->ctrl, 3 * sizeof(Ctrl))) != hipSuccess ||
      (part_words && (e = ensure(bs->bc_part, part_words * 8)) != hipSuccess))
    return bfail(g, DG_E_OUT_OF_MEMORY, "batch descriptor allocation");
  for (uint32_t i = 0; i < nq; i++)
    if (qd[i].kind == DG_Q_BC) qd[i].srcs = bs->srcs.as<uint32_t>() + src_off[i];
  for (const BcSplit& sp : splits)
    for (uint32_t t = 0; t < sp.k; t++) {
      QDesc& d = qd[sp.j0 + t];
      d.srcs = bs->srcs.as<uint32_t>() + src_off[sp.j0 + t];
      d.out = bs->bc_part.as<double>() + sp.off + (uint64_t)t * st_.V;
    }
  std::vector<uint32_t> qidx;
  uint32_t koff[3] = {0, 0, 0};
  for (int k = 0; k < 3; k++) {
    koff[k] = (uint32_t)qidx.size();
    qidx.insert(qidx.end(), by_kind[k].begin(), by_kind[k].end());
  }
  Ctrl c0[3] = {};
  if ((e = hipMemcpyAsync(bs->teams.p, tsv.data(), most * sizeof(TeamScratch), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(bs->qdesc.p, qd.data(), nj * sizeof(QDesc), hipMemcpyHostToDevice, s)) ||
      (qidx.size() && (e = hipMemcpyAsync(bs->qidx.p, qidx.data(), qidx.size() * 4, hipMemcpyHostToDevice, s))) ||
      (all_srcs.size() &&
       (e = hipMemcpyAsync(bs->srcs.p, all_srcs.data(), all_srcs.size() * 4, hipMemcpyHostToDevice, s))) ||
      (e = hipMemcpyAsync(bs->status.p, st.data(), nj * 4, hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(bs->arcs.p, arcs.data(), e_cnt * 8, hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(bs->live.p, live.data(), e_cnt * 8, hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(bs->ctrl.p, c0, sizeof(c0), hipMemcpyHostToDevice, s)))
    return bfail(g, DG_E_HIP, std::string("batch upload: ") + hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> lk(g_engine_mu);
    for (int k = 0; k < 3; k++) {
      if (by_kind[k].empty() || k == DG_Q_SSSP) continue;
      for (uint32_t t = 0; t < T_of[k]; t++)
        if ((e = hipMemsetAsync(tsv[t].sync, 0, sizeof(TeamSync), s)) != hipSuccess)
          return bfail(g, DG_E_HIP, std::string("batch upload: ") + hipGetErrorString(e));
      BatchArgs a{st_,
                  fast,
                  (int32_t)std::max<uint32_t>(1, tune.batch_delta),
                  (int32_t)g->cfg.w_max,
                  tune.alpha,
                  tune.beta,
                  bs->qdesc.as<QDesc>(),
                  bs->qidx.as<uint32_t>() + koff[k],
                  (uint32_t)by_kind[k].size(),
                  bs->status.as<int32_t>(),
                  bs->arcs.as<uint64_t>(),
                  bs->live.as<uint64_t>(),
                  bs->teams.as<TeamScratch>(),
                  T_of[k],
                  S_of[k],
                  bs->ctrl.as<Ctrl>() + k,
                  bs->spin_ticks};
      ProfScope ps(g, KID_BATCH_BFS + k, s);
      if (k == DG_Q_BFS) k_team<DG_Q_BFS><<<T_of[k] * S_of[k], Q_THREADS, 0, s>>>(a);
      else k_team<DG_Q_BC><<<T_of[k] * S_of[k], Q_THREADS, 0, s>>>(a);
      if ((e = hipGetLastError()) != hipSuccess)
        return bfail(g, DG_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    Ctrl cres[3];
    const size_t st_bytes = align256(nj * 4ull);
    if ((e = host_area(bs, st_bytes + sizeof(cres))) != hipSuccess ||
        (e = hipMemcpyAsync(bs->hres, bs->status.p, nj * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(static_cast<char*>(bs->hres) + st_bytes, bs->ctrl.p, sizeof(cres), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = wait_polled(bs, s)) != hipSuccess)
      return bfail(g, DG_E_HIP, std::string("batch: ") + hipGetErrorString(e));
    std::memcpy(st.data(), bs->hres, nj * 4);
    std::memcpy(cres, static_cast<char*>(bs->hres) + st_bytes, sizeof(cres));
    for (uint32_t i : mbq) {
      const uint32_t* S = all_srcs.data() + src_off[i];
      double* out = static_cast<double*>(qd[i].out);
      if ((e = hipMemsetAsync(out, 0, st_.V * sizeof(double), s)) != hipSuccess)
        return bfail(g, DG_E_HIP, std::string("batch BC clear: ") + hipGetErrorString(e));
      uint64_t ga = 0;
      dg_status r = DG_OK;
      for (uint32_t o = 0; o < qd[i].k && r == DG_OK; o += ms_bc_width())
        r = ms_bc_dev(g, st_, qd[i].epoch, fast, S + o, std::min(ms_bc_width(), qd[i].k - o), out, tune.chunk_buckets,
                      bs->mb, s, &ga);
      if (r != DG_OK && r != DG_E_OVERFLOW) return r;
      st[i] = r;
      prof_arcs(g, KID_BATCH_BC, ga);
      g->engine_arcs += ga;
    }
    for (const std::vector<uint32_t>& grp : bgroups) {
      std::vector<uint32_t> srcs;
      std::vector<void*> outs;
      for (uint32_t i : grp) {
        srcs.push_back(qd[i].src);
        outs.push_back(qd[i].out);
      }
      uint64_t ga = 0;
      dg_status r = ms_bfs_dev(g, st_, qd[grp[0]].epoch, fast, srcs.data(), (uint32_t)grp.size(), outs.data(),
                               tune.chunk_buckets, bs->mf, s, &ga);
      if (r != DG_OK) return r;
      for (uint32_t i : grp) st[i] = DG_OK;
      prof_arcs(g, KID_BATCH_BFS, ga);
      g->engine_arcs += ga;
    }
    for (const std::vector<uint32_t>& grp : sgroups) {
      std::vector<uint32_t> srcs;
      std::vector<void*> outs;
      for (uint32_t i : grp) {
        srcs.push_back(qd[i].src);
        outs.push_back(qd[i].out);
      }
      uint64_t ga = 0;
      dg_status r = ms_sssp_dev(g, st_, qd[grp[0]].epoch, fast, srcs.data(), (uint32_t)grp.size(), outs.data(),
                                (int32_t)std::max<uint32_t>(1, tune.batch_delta), tune.chunk_buckets, bs->ms, s, &ga);
      if (r != DG_OK) return r;
      for (uint32_t i : grp) st[i] = DG_OK;
      prof_arcs(g, KID_BATCH_SSSP, ga);
      g->engine_arcs += ga;
    }
    if (!by_kind[DG_Q_SSSP].empty()) {
      dg_status r = run_sssp_gangs(g, bs, st_, tune, fast, share, qd, by_kind[DG_Q_SSSP], st, budget, s);
      if (r != DG_OK) return r;
    }
    for (int k = 0; k < 3; k++) {
      if (k == DG_Q_SSSP) continue;
      if (cres[k].abort) return bfail(g, DG_E_HIP, "batch engine: a team barrier timed out");
      if (cres[k].done != by_kind[k].size())
        return bfail(g, DG_E_HIP, "batch engine: queries left unserved (teams could not assemble)");
      if (!by_kind[k].empty()) {
        prof_arcs(g, KID_BATCH_BFS + k, cres[k].arcs);
        g->engine_arcs += cres[k].arcs;
      }
    }
  }
  if (!splits.empty()) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>((st_.V + 255) / 256, 4096);
    for (const BcSplit& sp : splits) {
      st[sp.q] = DG_OK;
      for (uint32_t t = 0; t < sp.k && st[sp.q] == DG_OK; t++) st[sp.q] = st[sp.j0 + t];
      if (st[sp.q] == DG_OK)
        k_bc_sum<<<std::max<uint32_t>(1, grid), 256, 0, s>>>(bs->bc_part.as<double>() + sp.off, sp.k, st_.V,
                                                             static_cast<double*>(qd[sp.q].out));
    }
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
      return bfail(g, DG_E_HIP, std::string("batch BC sum: ") + hipGetErrorString(e));
  }
  for (uint32_t i = 0; i < nq; i++) per_query[i] = st[i];
  return DG_OK;
}

}  // namespace dg

extern "C" dg_status dg_query_batch(dg_graph* g, const dg_query* q, uint32_t nq, dg_status* per_query, void* stream) {
  if (!g) return DG_E_INVALID_ARG;
  try {
    return dg::query_batch_dev(g, q, nq, per_query, static_cast<hipStream_t>(stream), 0);
  } catch (...) {
    g->err = "unexpected failure in dg_query_batch";
    return DG_E_HIP;
  }
}

// ------------------------------------------------------------ autotuner
// Coordinate descent over the frontier-tile shape and the traversal
// parameters at the latest epoch: each candidate is timed on the same
// seeded sample of sources (plain BFS for the tile size and the direction
// thresholds, plain SSSP for delta, one engine launch of mixed queries for
// the team size) and the fastest value is kept.  Every candidate computes
// the same results; only the time differs.

namespace dg {
uint32_t pick_u32(uint64_t& x) {   // splitmix64 step
  x += 0x9e3779b97f4a7c15ull;
  uint64_t z = x;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return (uint32_t)((z ^ (z >> 31)) >> 32);
}
}  // namespace dg

extern "C" dg_status dg_autotune(dg_graph* g, uint32_t seed, dg_tuning* chosen, void* stream) {
  using namespace dg;
  if (!g) return DG_E_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t V = g->cfg.v_capacity;
  const uint32_t e = dg_latest_epoch(g);
  DevBuf deg, d0, d1;
  if (ensure(deg, V * 4ull) != hipSuccess || ensure(d0, V * 4ull) != hipSuccess) return DG_E_OUT_OF_MEMORY;
  dg_status st = dg_out_degrees(g, e, deg.as<uint32_t>(), stream);
  if (st != DG_OK) return st;
  std::vector<uint32_t> hd(V);
  if (hipMemcpyAsync(hd.data(), deg.p, V * 4ull, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DG_E_HIP;
  std::vector<uint32_t> cand;
  for (uint32_t v = 0; v < V; v++)
    if (hd[v]) cand.push_back(v);
  if (cand.empty()) {
    release(deg);
    release(d0);
    return dg_get_tuning(g, chosen);
  }
  uint64_t rs = 0x243f6a8885a308d3ull ^ seed;
  std::vector<uint32_t> src(4);
  for (auto& x : src) x = cand[pick_u32(rs) % cand.size()];
  // the batched call's sample: 64 distinct sources, each a BFS and an SSSP
  // query, so the searches have the widths they have in real batches
  std::vector<uint32_t> bsrc;
  for (uint32_t t = 0; t < 4 * 64 && bsrc.size() < std::min<size_t>(64, cand.size()); t++) {
    const uint32_t x = cand[pick_u32(rs) % cand.size()];
    if (std::find(bsrc.begin(), bsrc.end(), x) == bsrc.end()) bsrc.push_back(x);
  }
  auto time_queries = [&](int kind) -> double {
    auto t0 = std::chrono::steady_clock::now();
    for (uint32_t x : src) {
      dg_status r = kind == 0 ? dg_bfs(g, e, x, d0.as<int32_t>(), stream) : dg_sssp(g, e, x, d0.as<int32_t>(), stream);
      if (r != DG_OK) return 1e30;
    }
    hipStreamSynchronize(s);
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  std::vector<DevBuf> outs(2 * bsrc.size());
  auto time_batch = [&]() -> double {
    std::vector<dg_query> qs;
    for (uint32_t i = 0; i < outs.size(); i++) {
      if (ensure(outs[i], V * 4ull) != hipSuccess) return 1e30;
      qs.push_back(dg_query{i % 2 ? (uint32_t)DG_Q_SSSP : (uint32_t)DG_Q_BFS, bsrc[i / 2], e, 0, nullptr,
                            outs[i].p});
    }
    std::vector<dg_status> qst(qs.size());
    auto t0 = std::chrono::steady_clock::now();
    if (dg_query_batch(g, qs.data(), (uint32_t)qs.size(), qst.data(), stream) != DG_OK) return 1e30;
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  dg_tuning best;
  dg_get_tuning(g, &best);
  auto try_field = [&](uint32_t dg_tuning::*field, std::initializer_list<uint32_t> vals, int what) {
    double best_t = 1e30;
    uint32_t best_v = best.*field;
    for (uint32_t v : vals) {
      dg_tuning t = best;
      t.*field = v;
      if (dg_set_tuning(g, &t) != DG_OK) continue;
      if (what == 2) time_batch();   // the first launch sizes its scratch
      double dt = what == 2 ? time_batch() : time_queries(what);
      dt = std::min(dt, what == 2 ? time_batch() : time_queries(what));
      if (dt < best_t) {
        best_t = dt;
        best_v = v;
      }
    }
    best.*field = best_v;
    dg_set_tuning(g, &best);
  };
  time_queries(0);   // warm-up
  try_field(&dg_tuning::chunk_buckets, {16, 32, 64}, 0);
  try_field(&dg_tuning::alpha, {4, 14, 40, 1000000}, 0);
  try_field(&dg_tuning::beta, {8, 24, 64}, 0);
  try_field(&dg_tuning::sssp_delta, {16, 32, 64, 128, 256, 512}, 1);
  try_field(&dg_tuning::batch_delta, {64, 128, 256, 512, 1024, 2048}, 2);
  try_field(&dg_tuning::batch_groups, {0, 4, 8, 16, 32}, 2);
  release(deg);
  release(d0);
  for (auto& o : outs) release(o);
  if (chosen) *chosen = best;
  return DG_OK;
}
