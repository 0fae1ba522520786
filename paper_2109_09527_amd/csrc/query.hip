// Snapshot queries on epoch e in the plain form: one query per call, the
// host driving its levels (one launch per BFS level / SSSP pass / BC level,
// counters read back between them).  The level steps themselves live in
// frontier.h and are shared with the persistent multi-query engine.
//
//   BFS   direction-optimising (Beamer, Asanovic & Patterson, SC 2012):
//         top-down over out-slabs with a CAS claim of dist, or bottom-up over
//         in-slabs of unvisited vertices with a frontier bitmap and early
//         exit; switch when the frontier's slot count exceeds the unexplored
//         count / alpha, back when the frontier falls below live vertices /
//         beta.  Hop distances are the same either way.
//   SSSP  delta-stepping in near/far form (Meyer & Sanders 2003; Davidson
//         et al., IPDPS 2014): label-correcting relaxations with atomicMin
//         below the threshold, far flags above it, threshold += delta when
//         the near queue drains (a dense split moves flagged vertices below
//         the new threshold into the near queue); light arcs are relaxed
//         until a bucket settles, heavy arcs once per settled bucket.
//         Exact for every delta.
//   BC    Brandes (2001): level-synchronous forward BFS with int64
//         shortest-path counts (atomic adds, overflow flagged), then
//         dependencies pulled from successors level by level in FP64 with a
//         fixed lane order (no float atomics); bc[v] += delta[v] for v != s,
//         sources in order.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dg_host.h"
#include "frontier.h"
#include <map>
#include <mutex>

namespace dg {

constexpr uint32_t BIG_GRID = 2048;

// ---------------------------------------------------- counter publication

// Layout of q.counters: four counter slots, the finished-workgroup counts
// of the running step (DONE_OFF: DONE_GROUPS group counts and the total,
// each on its own 64-byte line), then (from STRIPE_OFF) the N_STRIPES count
// stripes of each slot.
constexpr uint32_t DONE_GROUPS = 16;
constexpr uint32_t DONE_STRIDE = 16;   // words between two done counts
constexpr size_t DONE_OFF = 192;
constexpr size_t STRIPE_OFF = DONE_OFF + (DONE_GROUPS + 1) * DONE_STRIDE * 4;
constexpr size_t COUNTERS_BYTES = STRIPE_OFF + 4 * N_STRIPES * sizeof(CountStripe);
static_assert(4 * sizeof(QCounters) <= DONE_OFF, "counter slots overlap the done count");

// What the device publishes to the host after a step: one slot's counters
// with its stripes added in, the running bucket record count, and the
// sequence number that marks the publication complete.
struct HostCounters {
  QCounters c;
  uint32_t rc;
  uint32_t seq;
};

// One publication: the counters of `slot` go to h with sequence number seq.
// A step kernel given a PubArgs with h set publishes from its last
// workgroup to finish; h null: the step publishes nothing.
struct PubArgs {
  const QCounters* cnt;
  const CountStripe* st;   // the stripes of all four slots, slot-major
  uint32_t* done;          // the done counts, zero between steps
  HostCounters* h;
  int slot;
  uint32_t seq;
};

// One lane: writes the counters r and the running record count rc, then the
// sequence number with a system-scope release, which makes the two writes
// before it visible first.
__device__ inline void publish_write(const PubArgs& p, const QCounters& r, uint32_t rc) {
  p.h->c = r;
  p.h->rc = rc;
  __hip_atomic_store(&p.h->seq, p.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A counter word as the device-scope atomics left it (a plain load could
// hit a line this workgroup's cache still holds from earlier in the step).
template <class T>
__device__ inline T ld_coherent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave (lanes 0..63): sums the slot's stripes into its counters and
// writes the result to h, the sequence number last (system scope), so the
// host can wait by polling instead of synchronising the stream.
__device__ inline void publish_wave(const PubArgs& p) {
  const uint32_t lane = threadIdx.x;
  unsigned long long m = 0, arcs = 0;
  uint32_t verts = 0, far = 0, far_inv = 0;
  if (lane < N_STRIPES) {
    const CountStripe* x = p.st + (size_t)p.slot * N_STRIPES + lane;
    m = ld_coherent(&x->m);
    arcs = ld_coherent(&x->arcs);
    verts = ld_coherent(&x->verts);
    far = ld_coherent(&x->far);
    far_inv = ld_coherent(&x->far_inv);
  }
  m = wave_sum_u64(m);
  arcs = wave_sum_u64(arcs);
  verts = wave_sum_u32(verts);
  far = wave_sum_u32(far);
  far_inv = wave_max_u32(far_inv);
  if (lane != 0) return;
  const QCounters* c = p.cnt + p.slot;
  QCounters r;
  r.fq = ld_coherent(&c->fq);
  r.n_verts = ld_coherent(&c->n_verts) + verts;
  r.n_far = ld_coherent(&c->n_far) + far;
  r.m_next = ld_coherent(&c->m_next) + m;
  r.far_min = min(ld_coherent(&c->far_min), (int32_t)(DIST_INF - far_inv));
  r.overflow = ld_coherent(&c->overflow);
  r.n_order = ld_coherent(&c->n_order);
  r.n_big = ld_coherent(&c->n_big);
  r.arcs = ld_coherent(&c->arcs) + arcs;
  publish_write(p, r, ld_coherent(&p.cnt[3].n_order));
}

// End of a step kernel (workgroup-uniform call): every workgroup counts
// itself done once its waves' memory operations have completed, and the
// last one publishes.  The step's counters change only through device-scope
// atomics, which are performed at the device's coherent level, so waiting
// for completion (no cache write-back or invalidation, which an agent-scope
// fence would cost every workgroup) orders them before the count.  A
// workgroup counts itself in group b mod DONE_GROUPS; the one that
// completes its group counts the group in the total, and the one that
// completes the total is last (a grid of a thousand workgroups then puts
// at most a few dozen atomics on any one word).  No workgroup waits for
// another, and the last clears the counts for the next step.  A separate
// publishing launch per step had cost its own dispatch on every level's
// host round trip.
__device__ inline void publish_if_last(const PubArgs& p) {
  if (!p.h) return;
  __shared__ uint32_t last;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);   // vmcnt, expcnt and lgkmcnt all zero
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nwg = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
    const uint32_t grp = b % DONE_GROUPS;
    const uint32_t in_grp = (nwg - grp + DONE_GROUPS - 1) / DONE_GROUPS;   // workgroups of group grp
    bool l = false;
    if (__hip_atomic_fetch_add(&p.done[grp * DONE_STRIDE], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u ==
        in_grp) {
      const uint32_t groups = min(nwg, DONE_GROUPS);
      l = __hip_atomic_fetch_add(&p.done[DONE_GROUPS * DONE_STRIDE], 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) + 1u == groups;
    }
    last = l;
  }
  __syncthreads();
  if (!last || threadIdx.x >= 64) return;
  publish_wave(p);
  if (threadIdx.x <= DONE_GROUPS)
    __hip_atomic_store(&p.done[threadIdx.x * DONE_STRIDE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_publish(PubArgs p) { publish_wave(p); }

// --------------------------------------------------------------- fills

template <class T>
__global__ void k_fill(T* p, uint64_t n, T v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <class T>
static void fill(T* p, uint64_t n, T v, hipStream_t s) {
  if (!n) return;
  uint64_t b = std::min<uint64_t>((n + 255) / 256, 4096);
  k_fill<T><<<(uint32_t)b, 256, 0, s>>>(p, n, v);
}

// Up to four 32-bit fills in one launch (a query's start-up clears), so a
// search does not pay a launch per array before its seed.
struct Fills {
  uint32_t* p[4];
  uint64_t n[4];
  uint32_t v[4];
};
__global__ void k_fills(Fills f) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
#pragma unroll
  for (int k = 0; k < 4; k++)
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.n[k]; i += stride) f.p[k][i] = f.v[k];
}
static void fills(const Fills& f, hipStream_t s) {
  uint64_t n = 0;
  for (int k = 0; k < 4; k++) n = std::max(n, f.n[k]);
  if (!n) return;
  k_fills<<<(uint32_t)std::min<uint64_t>((n + 255) / 256, 4096), 256, 0, s>>>(f);
}

// Seed a query at src: dist/level d0, the item of src and its chunk map,
// bitmap bit; counters slot 0 describes the seed frontier, slot 1 is
// cleared.  One wave.
__global__ void k_seed(Store st, uint32_t src, int32_t* dist, int32_t d0, Front f, uint32_t* bm, QCounters* cnt,
                       uint32_t* order, PubArgs pub) {
  const uint64_t desc = st.fdesc[src];
  const uint32_t nb = desc ? 1u << (desc & 63) : 0;
  const uint32_t nc = (nb + (1u << f.lch) - 1) >> f.lch;
  for (uint32_t c = threadIdx.x; c < nc && c < f.ccap; c += blockDim.x) f.cmap[c] = 0;
  if (threadIdx.x != 0) return;
  if (nb) f.q[0] = Item{desc, src, 0};
  if (dist) dist[src] = d0;
  if (bm) bm[src >> 5] |= 1u << (src & 31);
  if (order) order[0] = src;
  QCounters c0{};
  c0.fq = nb ? 1ull | ((unsigned long long)nb << 32) : 0ull;
  c0.n_verts = 1;
  c0.m_next = st.fused[src];
  c0.n_order = 1;
  c0.far_min = DIST_INF;
  cnt[0] = c0;
  zero_counters(&cnt[1]);
  // the seed frontier's counts are c0 (slot 0's stripes are clear)
  if (pub.h) publish_write(pub, c0, cnt[3].n_order);
}

__device__ inline void reset_other(QCounters* c) {
  if (blockIdx.x == 0 && threadIdx.x == 0) zero_counters(c);
}

// Clears slot c and, when st is set, its count stripes.
__device__ inline void reset_other(QCounters* c, CountStripe* st) {
  reset_other(c);
  if (st && blockIdx.x == 0 && threadIdx.x < N_STRIPES) {
    CountStripe* x = st + threadIdx.x;
    x->m = 0;
    x->arcs = 0;
    x->verts = 0;
    x->far = 0;
    x->far_inv = 0;
  }
}

__global__ __launch_bounds__(Q_THREADS) void k_bfs_td(LevelArgs a, unsigned long long nfq, QCounters* reset,
                                                       CountStripe* reset_st, PubArgs pub) {
  __shared__ Shared sh;
  reset_other(reset, reset_st);
  td_step(a, nfq, blockIdx.x, gridDim.x, sh);
  publish_if_last(pub);
}

__global__ __launch_bounds__(Q_THREADS) void k_bfs_bu(LevelArgs a, QCounters* reset, CountStripe* reset_st) {
  __shared__ Shared sh;
  reset_other(reset, reset_st);
  bu_step(a, blockIdx.x, gridDim.x, sh);
}

__global__ __launch_bounds__(Q_THREADS) void k_bfs_bu_big(LevelArgs a, PubArgs pub) {
  __shared__ Shared sh;
  bu_big_step(a, a.cnt_out->n_big, blockIdx.x, gridDim.x, sh);
  publish_if_last(pub);
}

__global__ __launch_bounds__(Q_THREADS) void k_sssp_relax(RelaxArgs a, unsigned long long nfq, QCounters* reset,
                                                           CountStripe* reset_st, PubArgs pub) {
  __shared__ Shared sh;
  reset_other(reset, reset_st);
  relax_step(a, nfq, blockIdx.x, gridDim.x, sh);
  publish_if_last(pub);
}

__global__ __launch_bounds__(Q_THREADS) void k_sssp_expand(Store st, const uint32_t* list, uint32_t n, Front fout,
                                                            QCounters* cnt_out, QCounters* reset,
                                                            CountStripe* reset_st, PubArgs pub) {
  __shared__ Shared sh;
  reset_other(reset, reset_st);
  expand_step(st, list, n, fout, cnt_out, blockIdx.x, gridDim.x, sh);
  publish_if_last(pub);
}

__global__ __launch_bounds__(Q_THREADS) void k_sssp_split(SplitArgs a, QCounters* reset, CountStripe* reset_st,
                                                           PubArgs pub) {
  __shared__ Shared sh;
  reset_other(reset, reset_st);
  split_step(a, blockIdx.x, gridDim.x, sh);
  publish_if_last(pub);
}

__global__ __launch_bounds__(Q_THREADS) void k_bc_fwd(BcFwdArgs a, unsigned long long nfq, QCounters* reset) {
  __shared__ Shared sh;
  reset_other(reset);
  bcfwd_step(a, nfq, blockIdx.x, gridDim.x, sh);
}

__global__ __launch_bounds__(Q_THREADS) void k_bc_bwd(Store st, uint32_t e, int fast, const uint32_t* verts,
                                                      uint32_t nv, uint32_t src, const int32_t* level, int32_t L,
                                                      const unsigned long long* sigma, double* delta, double* bc,
                                                      BwdTiles bt) {
  bcbwd_step(st, e, fast != 0, verts, nv, src, level, L, sigma, delta, bc, bt, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(Q_THREADS) void k_bc_tiles(Store st, uint32_t e, int fast, const int32_t* level, int32_t L,
                                                        const double* coef, BwdTiles bt) {
  bcbwd_tiles(st, e, fast != 0, level, L, coef, bt, bt.head->tiles[L & 1], blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(Q_THREADS) void k_bc_combine(BwdTiles bt, int32_t L, uint32_t src,
                                                          const unsigned long long* sigma, double* coef, double* bc) {
  bcbwd_combine(bt, bt.head->verts[L & 1], src, sigma, coef, bc, blockIdx.x, gridDim.x);
}

__global__ void k_inf_to_minus1(int32_t* d, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (d[i] == DIST_INF) d[i] = -1;
}

// A frontier holds each vertex at most once, and its slabs are distinct
// slabs of the forward pool.
static uint64_t items_capacity(const dg_graph* g) { return (uint64_t)g->cfg.v_capacity + 1024; }
static uint64_t chunks_capacity(const dg_graph* g) { return g->st.fp.cap / CH_MIN + 2; }
static uint32_t log2_of(uint32_t x) { return 31 - __builtin_clz(x); }

static Front front_of(const QueryScratch& q, int which) {
  const DevBuf& items = which ? q.qb : q.qa;
  const DevBuf& cmap = which ? q.cmap_b : q.cmap_a;
  return Front{items.as<Item>(), cmap.as<uint32_t>(), (uint32_t)std::min<uint64_t>(q.items_cap, 0xFFFFFFFFu),
               (uint32_t)std::min<uint64_t>(q.chunks_cap, 0xFFFFFFFFu), q.lch};
}

// Bytes of each plain-query buffer for this graph (0 = not needed by the
// query kinds asked for).
struct QuerySizes {
  uint64_t items, chunks;
  uint64_t qa, qb, cmap_a, cmap_b, bm0, bm1, counters, fb, stamp, flag8, rlist, rstamp, fa, sigma, delta, level, bt;
};

static QuerySizes query_sizes(const dg_graph* g, bool sssp, bool bc) {
  QuerySizes z{};
  const uint64_t V = g->cfg.v_capacity;
  z.items = items_capacity(g);
  z.chunks = chunks_capacity(g);
  z.qa = z.qb = z.items * sizeof(Item);
  z.cmap_a = z.cmap_b = z.chunks * 4;
  z.bm0 = z.bm1 = ((V + 31) / 32 + 1) * 4;
  z.counters = COUNTERS_BYTES;
  // bottom-up chunk items of long in-slabs
  if (!sssp && !bc) z.fb = (V + std::max(g->st.fp.cap, g->st.rp.cap) / BU_CHUNK + 1024) * sizeof(Item);
  if (sssp) z.stamp = z.flag8 = z.rlist = z.rstamp = V * 4 + 64;
  if (bc) {
    z.fa = V * 4 + 64;
    z.sigma = z.delta = V * 8 + 64;
    z.level = V * 4 + 64;
    z.bt = bwd_tiles_bytes(g->st.fp.cap, 1);
  }
  return z;
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// A BFS's buffers laid out one after another from base (each 256-byte
// aligned), followed by the block its counters are published into;
// returns the bytes used.  With q null only the size is computed.
uint64_t bfs_fixed_layout(const dg_graph* g, char* base, QueryScratch* q) {
  const QuerySizes z = query_sizes(g, false, false);
  uint64_t off = 0;
  auto carve = [&](DevBuf* b, uint64_t bytes) {
    if (q) {
      b->p = base + off;
      b->bytes = bytes;
    }
    off += align256(bytes);
  };
  QueryScratch dummy;
  QueryScratch& t = q ? *q : dummy;
  carve(&t.qa, z.qa);
  carve(&t.qb, z.qb);
  carve(&t.cmap_a, z.cmap_a);
  carve(&t.cmap_b, z.cmap_b);
  carve(&t.bm0, z.bm0);
  carve(&t.bm1, z.bm1);
  carve(&t.counters, z.counters);
  carve(&t.fb, z.fb);
  DevBuf pub;
  carve(&pub, sizeof(HostCounters));
  if (q) {
    q->fixed = true;
    q->dev_pub = pub.p;
  }
  return off;
}

static hipError_t ensure_query_scratch(dg_graph* g, QueryScratch& q, bool sssp, bool bc) {
  const QuerySizes z = query_sizes(g, sssp, bc);
  q.items_cap = z.items;
  q.chunks_cap = z.chunks;
  q.lch = log2_of(g->tune.chunk_buckets);
  if (q.fixed) {
    // a fixed area is never grown: its layout was computed from the same sizes
    const std::pair<const DevBuf*, uint64_t> need[] = {
        {&q.qa, z.qa},       {&q.qb, z.qb},       {&q.cmap_a, z.cmap_a}, {&q.cmap_b, z.cmap_b},
        {&q.bm0, z.bm0},     {&q.bm1, z.bm1},     {&q.counters, z.counters}, {&q.fb, z.fb},
        {&q.stamp, z.stamp}, {&q.flag8, z.flag8}, {&q.rlist, z.rlist},   {&q.rstamp, z.rstamp},
        {&q.fa, z.fa},       {&q.sigma, z.sigma}, {&q.delta, z.delta},   {&q.level, z.level},
        {&q.bt, z.bt}};
    for (const auto& n : need)
      if (n.second && (!n.first->p || n.first->bytes < n.second)) return hipErrorInvalidValue;
    return q.dev_pub ? hipSuccess : hipErrorInvalidValue;
  }
  hipError_t e;
  const std::pair<DevBuf*, uint64_t> need[] = {
      {&q.qa, z.qa},       {&q.qb, z.qb},       {&q.cmap_a, z.cmap_a}, {&q.cmap_b, z.cmap_b},
      {&q.bm0, z.bm0},     {&q.bm1, z.bm1},     {&q.counters, z.counters}, {&q.fb, z.fb},
      {&q.stamp, z.stamp}, {&q.flag8, z.flag8}, {&q.rlist, z.rlist},   {&q.rstamp, z.rstamp},
      {&q.fa, z.fa},       {&q.sigma, z.sigma}, {&q.delta, z.delta},   {&q.level, z.level},
        {&q.bt, z.bt}};
  for (const auto& n : need)
    if (n.second && (e = ensure(*n.first, n.second)) != hipSuccess) return e;
  if (!q.host_pub) {
    if ((e = hipHostMalloc(&q.host_pub, sizeof(HostCounters), hipHostMallocCoherent)) != hipSuccess) return e;
    std::memset(q.host_pub, 0, sizeof(HostCounters));
    q.pub_seq = 0;
  }
  if (!q.host_counters) {
    if ((e = hipHostMalloc(&q.host_counters, COUNTERS_BYTES, hipHostMallocDefault)) != hipSuccess) return e;
  }
  return hipSuccess;
}

void free_query_scratch(QueryScratch& q) {
  release(q.qa); release(q.qb); release(q.cmap_a); release(q.cmap_b); release(q.fa); release(q.fb); release(q.bm0); release(q.bm1);
  release(q.stamp); release(q.flag8); release(q.sigma); release(q.delta); release(q.level);
  release(q.rlist); release(q.rstamp); release(q.bt);
  release(q.counters);
  if (q.host_counters) hipHostFree(q.host_counters);
  q.host_counters = nullptr;
  if (q.host_pub) hipHostFree(q.host_pub);
  q.host_pub = nullptr;
}

static CountStripe* stripes_of(QueryScratch& q, int slot) {
  return reinterpret_cast<CountStripe*>(q.counters.as<char>() + STRIPE_OFF) + (size_t)slot * N_STRIPES;
}

static uint32_t* done_of(QueryScratch& q) { return reinterpret_cast<uint32_t*>(q.counters.as<char>() + DONE_OFF); }

// Zero the step's done count and every slot's stripes (one fill).
static void clear_counts(QueryScratch& q, hipStream_t s) {
  fill<uint32_t>(done_of(q), (COUNTERS_BYTES - DONE_OFF) / 4, 0u, s);
}

// The next publication of slot's counters (with its stripes added in, plus
// the running bucket record count of slot 3): to pinned host memory, or,
// for a fixed area, which has no pinned block, to its device word.
static PubArgs pub_args(QueryScratch& q, int slot) {
  HostCounters* h = static_cast<HostCounters*>(q.fixed ? q.dev_pub : q.host_pub);
  return PubArgs{q.counters.as<QCounters>(), stripes_of(q, 0), done_of(q), h, slot, ++q.pub_seq};
}

// Wait for publication p: the host polls its sequence number (a stream
// synchronisation costs more than the step it follows when steps are
// short); one not seen within two seconds falls back to synchronising the
// stream, which reports any device error.  A fixed area's publication is
// copied back after the stream has drained.
static hipError_t await_counters(QueryScratch& q, const PubArgs& p, QCounters* out, uint32_t* rc, hipStream_t s) {
  hipError_t e;
  if (q.fixed) {
    HostCounters hc;
    if ((e = hipMemcpyAsync(&hc, p.h, sizeof(hc), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (hc.seq != p.seq) return hipErrorUnknown;
    *out = hc.c;
    *rc = hc.rc;
    return hipSuccess;
  }
  const HostCounters* h = p.h;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 1; __atomic_load_n(&h->seq, __ATOMIC_ACQUIRE) != p.seq; spin++) {
    host_pause(spin);
    if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (__atomic_load_n(&h->seq, __ATOMIC_ACQUIRE) != p.seq) return hipErrorUnknown;
      break;
    }
  }
  std::memcpy(out, &h->c, sizeof(QCounters));
  *rc = h->rc;
  return hipSuccess;
}

// The counters of a slot filled by steps that do not publish themselves:
// a one-wave kernel publishes them.
static hipError_t read_counters_rc(QueryScratch& q, int slot, QCounters* out, uint32_t* rc, hipStream_t s) {
  const PubArgs p = pub_args(q, slot);
  k_publish<<<1, 64, 0, s>>>(p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return await_counters(q, p, out, rc, s);
}

static hipError_t await_counters(QueryScratch& q, const PubArgs& p, QCounters* out, hipStream_t s) {
  uint32_t rc;
  return await_counters(q, p, out, &rc, s);
}

static hipError_t read_counters(QueryScratch& q, int slot, QCounters* out, hipStream_t s) {
  uint32_t rc;
  return read_counters_rc(q, slot, out, &rc, s);
}

static uint32_t grid_for(uint64_t units, uint32_t per_block, uint32_t cap = 16384) {
  uint64_t b = (units + per_block - 1) / per_block;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, cap));
}

// Workgroups of `kernel` resident on the current device at once.
static uint32_t resident(const void* kernel) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, uint32_t> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(dev, kernel);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, Q_THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  const uint32_t r = (uint32_t)std::max(1, per_cu * cus);
  cache[key] = r;
  return r;
}

// Grid of a frontier step: one wave per chunk, never more than fit at once.
static uint32_t chunks_grid(const void* kernel, unsigned long long fq, uint32_t lch) {
  return grid_for(fq_chunks(fq, lch), Q_WAVES, resident(kernel));
}

static dg_status queue_overflow(dg_graph* g) {
  g->err = "frontier queue capacity exceeded";
  return DG_E_OUT_OF_MEMORY;
}

// Grid of a step with one unit per lane, at most what fits at once.
static uint32_t lanes_grid(const void* kernel, uint64_t n) {
  return grid_for(n, Q_THREADS, resident(kernel));
}

static dg_status hip_fail(dg_graph* g, hipError_t e, const char* where) {
  g->err = std::string(where) + ": " + hipGetErrorString(e);
  return DG_E_HIP;
}

uint64_t arcs_at(const dg_graph* g, uint32_t e);
uint64_t live_at(const dg_graph* g, uint32_t e);

dg_status bfs_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* dist, hipStream_t s, QueryScratch& q) {
  const int fast = g->concurrent_writers ? 0 : 1;
  hipError_t he = ensure_query_scratch(g, q, false, false);
  if (he != hipSuccess) return hip_fail(g, he, "bfs scratch");
  const uint32_t V = g->cfg.v_capacity;
  const uint64_t bmw = (V + 31) / 32 + 1;
  Front fr[2] = {front_of(q, 0), front_of(q, 1)};
  Item* qbig = q.fb.as<Item>();
  uint32_t* bm[2] = {q.bm0.as<uint32_t>(), q.bm1.as<uint32_t>()};
  QCounters* cnt = q.counters.as<QCounters>();
  fills(Fills{{reinterpret_cast<uint32_t*>(dist), done_of(q), bm[0], nullptr},
               {V, (COUNTERS_BYTES - DONE_OFF) / 4, bmw, 0},
               {0xFFFFFFFFu, 0u, 0u, 0u}},
        s);
  PubArgs pub = pub_args(q, 0);
  k_seed<<<1, 64, 0, s>>>(g->st, src, dist, 0, fr[0], bm[0], cnt, nullptr, pub);
  QCounters hc;
  if ((he = await_counters(q, pub, &hc, s)) != hipSuccess) return hip_fail(g, he, "bfs seed");
  int64_t m_u = (int64_t)arcs_at(g, e);
  const uint64_t n_live = std::max<uint64_t>(1, live_at(g, e));
  bool bu = false;
  unsigned long long fq = hc.fq;
  uint32_t n_verts = hc.n_verts;
  uint64_t m_f = hc.m_next;
  int level = 0;
  while (n_verts > 0) {
    int cur = level & 1, nxt = cur ^ 1;
    // Beamer's switches, with one change: a bottom-up level scans every
    // vertex, so a frontier below the switch-back size stays top-down even
    // when few unexplored arcs remain (the last levels of a search had
    // flipped to bottom-up and back)
    const bool small = (uint64_t)n_verts * g->tune.beta < n_live;
    if (!bu && (int64_t)m_f * (int64_t)g->tune.alpha > m_u && !small) bu = true;
    else if (bu && small) bu = false;
    m_u -= (int64_t)m_f;
    fill<uint32_t>(bm[nxt], bmw, 0u, s);
    LevelArgs a{g->st, e, fast, fr[cur], fr[nxt], qbig, bm[cur], bm[nxt], dist, level + 1, cnt + nxt,
                stripes_of(q, nxt)};
    pub = pub_args(q, nxt);
    if (bu) {
      ProfScope ps(g, KID_BFS_BU, s);
      // half the resident workgroups: each workgroup's final counter commit
      // and queue reservations are atomics on shared words, and fewer
      // workgroups over more vertices each won at R-MAT 20 (level time with
      // half: 53 us; a quarter: 59; an eighth: 72)
      k_bfs_bu<<<grid_for(V, Q_THREADS, std::max<uint32_t>(1, resident((const void*)k_bfs_bu) / 2)), Q_THREADS, 0, s>>>(
          a, cnt + cur, stripes_of(q, cur));
      k_bfs_bu_big<<<std::min(BIG_GRID, resident((const void*)k_bfs_bu_big)), Q_THREADS, 0, s>>>(a, pub);
    } else {
      ProfScope ps(g, KID_BFS_TD, s);
      k_bfs_td<<<chunks_grid((const void*)k_bfs_td, fq, q.lch), Q_THREADS, 0, s>>>(a, fq, cnt + cur,
                                                                                    stripes_of(q, cur), pub);
    }
    if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "bfs level launch");
    if ((he = await_counters(q, pub, &hc, s)) != hipSuccess) return hip_fail(g, he, "bfs level");
    if (hc.overflow & OVF_QUEUE) return queue_overflow(g);
    prof_arcs(g, bu ? KID_BFS_BU : KID_BFS_TD, hc.arcs);
    fq = hc.fq;
    n_verts = hc.n_verts;
    m_f = hc.m_next;
    level++;
  }
  return DG_OK;
}

// ----------------------------------------------------------------- SSSP

dg_status sssp_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* dist, hipStream_t s, QueryScratch& q) {
  const int fast = g->concurrent_writers ? 0 : 1;
  hipError_t he = ensure_query_scratch(g, q, true, false);
  if (he != hipSuccess) return hip_fail(g, he, "sssp scratch");
  const uint32_t V = g->cfg.v_capacity;
  const int32_t delta = (int32_t)std::max<uint32_t>(1, g->tune.sssp_delta);
  // with delta >= w_max every arc is light and the heavy passes vanish
  const bool split_lh = delta < g->cfg.w_max;
  Front fr[2] = {front_of(q, 0), front_of(q, 1)};
  int qi = 0;   // queue holding the current near frontier
  uint32_t* stamp = q.stamp.as<uint32_t>();
  uint32_t* infar = q.flag8.as<uint32_t>();
  uint32_t* rlist = q.rlist.as<uint32_t>();
  uint32_t* rstamp = q.rstamp.as<uint32_t>();
  QCounters* cnt = q.counters.as<QCounters>();
  uint32_t* rcount = &cnt[3].n_order;
  fills(Fills{{reinterpret_cast<uint32_t*>(dist), done_of(q), stamp, infar},
               {V, (COUNTERS_BYTES - DONE_OFF) / 4, V, (V + 31) / 32 + 1},
               {(uint32_t)DIST_INF, 0u, 0u, 0u}},
        s);
  if (split_lh) {
    fill<uint32_t>(rstamp, V, 0u, s);
    fill<uint32_t>(rcount, 1, 0u, s);
  }
  PubArgs pub = pub_args(q, 0);
  k_seed<<<1, 64, 0, s>>>(g->st, src, dist, 0, fr[0], nullptr, cnt, nullptr, pub);
  QCounters hc;
  if ((he = await_counters(q, pub, &hc, s)) != hipSuccess) return hip_fail(g, he, "sssp seed");
  unsigned long long near = hc.fq;
  uint32_t n_far = 0;
  int32_t thr = delta;
  uint32_t it = 1;      // stamp of the queue being filled; the source's queue had stamp 0
  uint32_t phase = 1;   // bucket number (stamp of the recorded vertices)
  uint32_t n_rec = 0;   // vertices recorded in the current bucket
  int slot = 0;
  bool ovf = false;
  auto relax = [&](unsigned long long nfq, int mode) -> hipError_t {
    int nxt = slot ^ 1;
    // far entries found by this pass are appended after the current far list
    RelaxArgs a{g->st, e,     fast,  fr[qi], fr[qi ^ 1], dist,  stamp,  infar, thr,
                it,    cnt + nxt, mode, delta,  rlist,      rcount, rstamp, phase, stripes_of(q, nxt)};
    const PubArgs p = pub_args(q, nxt);
    {
      ProfScope ps(g, KID_SSSP_RELAX, s);
      k_sssp_relax<<<chunks_grid((const void*)k_sssp_relax, nfq, q.lch), Q_THREADS, 0, s>>>(a, nfq, cnt + slot,
                                                                                            stripes_of(q, slot), p);
    }
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    if ((r = await_counters(q, p, &hc, &n_rec, s)) != hipSuccess) return r;
    ovf |= (hc.overflow & OVF_QUEUE) != 0;
    prof_arcs(g, KID_SSSP_RELAX, hc.arcs);
    near = hc.fq;
    n_far += hc.n_far;
    qi ^= 1;
    it++;
    slot = nxt;
    return hipSuccess;
  };
  for (;;) {
    if (ovf) return queue_overflow(g);
    if (near) {
      if ((he = relax(near, split_lh ? 1 : 0)) != hipSuccess) return hip_fail(g, he, "sssp relax");
      continue;
    }
    if (split_lh) {
      // the bucket has settled: its recorded vertices relax their heavy arcs once
      if (n_rec) {
        const uint32_t n_r = n_rec;
        fill<uint32_t>(rcount, 1, 0u, s);
        n_rec = 0;
        int nxt = slot ^ 1;
        pub = pub_args(q, nxt);
        k_sssp_expand<<<lanes_grid((const void*)k_sssp_expand, n_r), Q_THREADS, 0, s>>>(
            g->st, rlist, n_r, fr[qi], cnt + nxt, cnt + slot, stripes_of(q, slot), pub);
        if ((he = hipGetLastError()) != hipSuccess || (he = await_counters(q, pub, &hc, s)) != hipSuccess)
          return hip_fail(g, he, "sssp expand");
        if (hc.overflow & OVF_QUEUE) return queue_overflow(g);
        slot = nxt;
        if (hc.fq && (he = relax(hc.fq, 2)) != hipSuccess) return hip_fail(g, he, "sssp heavy");
        n_rec = 0;
        if (ovf) return queue_overflow(g);
      }
      phase++;
      // heavy arcs leave the bucket (w > delta); should any land in it, keep going
      if (near) continue;
    }
    if (n_far == 0) break;
    int32_t far_min = DIST_INF;
    // advance the threshold until some far entry falls below it
    do {
      thr = far_min == DIST_INF ? thr + delta
                                : (int32_t)std::min<int64_t>(DIST_INF, ((int64_t)far_min / delta + 1) * delta);
      int nxt = slot ^ 1;
      SplitArgs a{g->st, fr[qi], dist, stamp, infar, thr, it, cnt + nxt, stripes_of(q, nxt)};
      pub = pub_args(q, nxt);
      {
        ProfScope ps(g, KID_SSSP_SPLIT, s);
        k_sssp_split<<<lanes_grid((const void*)k_sssp_split, V), Q_THREADS, 0, s>>>(a, cnt + slot,
                                                                                    stripes_of(q, slot), pub);
      }
      if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "sssp split launch");
      if ((he = await_counters(q, pub, &hc, s)) != hipSuccess) return hip_fail(g, he, "sssp split");
      if (hc.overflow & OVF_QUEUE) return queue_overflow(g);
      slot = nxt;
      n_far = hc.n_far;
      near = hc.fq;
      far_min = hc.far_min;
    } while (!near && n_far > 0);
    it++;
  }
  k_inf_to_minus1<<<grid_for(V, 256, 4096), 256, 0, s>>>(dist, V);
  if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "sssp finish");
  return DG_OK;
}

// ------------------------------------------------------------------- BC

dg_status bc_dev(dg_graph* g, uint32_t e, const uint32_t* srcs, uint32_t k, double* bc, hipStream_t s,
                 QueryScratch& q) {
  const int fast = g->concurrent_writers ? 0 : 1;
  hipError_t he = ensure_query_scratch(g, q, false, true);
  if (he != hipSuccess) return hip_fail(g, he, "bc scratch");
  const uint32_t V = g->cfg.v_capacity;
  Front fr[2] = {front_of(q, 0), front_of(q, 1)};
  uint32_t* order = q.fa.as<uint32_t>();
  int32_t* level = q.level.as<int32_t>();
  unsigned long long* sigma = q.sigma.as<unsigned long long>();
  double* delta = q.delta.as<double>();   // per vertex (1 + dependency) / path count, once finished
  QCounters* cnt = q.counters.as<QCounters>();
  // cnt[0..1] alternate per level; cnt[2] holds the running order total
  // and the overflow flag of the current source
  QCounters* tot = cnt + 2;
  const BwdTiles bt = bwd_tiles_at(q.bt.as<char>(), g->st.fp.cap, 1);
  fill<double>(bc, V, 0.0, s);
  clear_counts(q, s);
  fill<uint32_t>(reinterpret_cast<uint32_t*>(bt.head), sizeof(BwdHead) / 4, 0u, s);
  std::vector<uint32_t> off, nbig;
  for (uint32_t si = 0; si < k; si++) {
    uint32_t src = srcs[si];
    fill<int32_t>(level, V, -1, s);
    fill<unsigned long long>(sigma, V, 0ull, s);
    k_seed<<<1, 64, 0, s>>>(g->st, src, level, 0, fr[0], nullptr, cnt, order, PubArgs{});
    fill<unsigned long long>(reinterpret_cast<unsigned long long*>(tot), sizeof(QCounters) / 8, 0ull, s);
    fill<unsigned long long>(sigma + src, 1, 1ull, s);
    fill<uint32_t>(&tot->n_order, 1, 1u, s);
    QCounters hc;
    if ((he = read_counters(q, 0, &hc, s)) != hipSuccess) return hip_fail(g, he, "bc seed");
    off.assign(1, 0);
    off.push_back(1);
    nbig.assign(1, 1);   // the source's slab is not counted: assume it is long
    unsigned long long fq = hc.fq;
    int lvl = 0;
    while (true) {
      int cur = lvl & 1, nxt = cur ^ 1;
      BcFwdArgs a{g->st, e, fast, fr[cur], fr[nxt], order, level, sigma, lvl + 1, cnt + nxt, tot};
      if (fq) {
        ProfScope ps(g, KID_BC_FWD, s);
        k_bc_fwd<<<chunks_grid((const void*)k_bc_fwd, fq, q.lch), Q_THREADS, 0, s>>>(a, fq, cnt + cur);
      } else {
        fill<unsigned long long>(reinterpret_cast<unsigned long long*>(cnt + nxt), sizeof(QCounters) / 8, 0ull, s);
      }
      if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "bc fwd launch");
      if ((he = read_counters(q, nxt, &hc, s)) != hipSuccess) return hip_fail(g, he, "bc fwd");
      if (hc.overflow & OVF_QUEUE) return queue_overflow(g);
      prof_arcs(g, KID_BC_FWD, hc.arcs);
      if (hc.n_verts == 0) break;
      off.push_back(off.back() + hc.n_verts);
      nbig.push_back(hc.n_far);
      fq = hc.fq;
      lvl++;
    }
    {
      QCounters ht;
      (void)hipMemcpyAsync(q.host_counters, tot, sizeof(QCounters), hipMemcpyDeviceToHost, s);
      if ((he = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(g, he, "bc overflow");
      std::memcpy(&ht, q.host_counters, sizeof(QCounters));
      if (ht.overflow) {
        g->err = "shortest-path count exceeds int64";
        return DG_E_OVERFLOW;
      }
    }
    // both parities' tile counts start at zero
    fill<uint32_t>(reinterpret_cast<uint32_t*>(bt.head), 4, 0u, s);
    for (int L = (int)off.size() - 2; L >= 0; L--) {
      uint32_t nv = off[L + 1] - off[L];
      ProfScope ps(g, KID_BC_BWD, s);
      k_bc_bwd<<<grid_for(nv, Q_WAVES), Q_THREADS, 0, s>>>(g->st, e, fast, order + off[L], nv, src, level, L,
                                                           sigma, delta, bc, bt);
      // the forward's count of long slabs is exact only while no update can
      // move a slab in between
      if (nbig[L] || !fast) {
        k_bc_tiles<<<resident((const void*)k_bc_tiles), Q_THREADS, 0, s>>>(g->st, e, fast, level, L, delta, bt);
        k_bc_combine<<<grid_for(fast ? nbig[L] : 4096u * Q_THREADS, Q_THREADS), Q_THREADS, 0, s>>>(bt, L, src, sigma,
                                                                                                    delta, bc);
      }
    }
    if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "bc bwd launch");
  }
  {
    uint32_t ovf = 0;
    if ((he = hipMemcpyAsync(q.host_counters, &bt.head->ovf, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (he = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(g, he, "bc tiles");
    std::memcpy(&ovf, q.host_counters, 4);
    if (ovf) {
      g->err = "backward tile list capacity exceeded";
      return DG_E_OUT_OF_MEMORY;
    }
  }
  return DG_OK;
}

// ---------------------------------------------------------------- stats

// Visible slots of buckets [b0, b1) of a slab, summed over the wave.  With
// trusted summaries (fast), a bucket whose versions were all born by e
// decides most slots from its summary, and a slot's stamp is read only
// where the summary cannot tell.
__device__ inline uint32_t visible_in(const Slab& s, uint32_t b0, uint32_t b1, uint32_t e, bool fast) {
  const uint32_t lane = lane_id(), j = lane & 15;
  uint32_t c = 0;
  for (uint32_t b = b0 + (lane >> 4); b < b1; b += 4) {
    uint32_t* bp = bucket_ptr(s, b);
    const uint4 sm = fast ? *reinterpret_cast<const uint4*>(&s.sum[SUM_WORDS * b])
                          : make_uint4(0xFFFFFFFFu, 0xFFFFu, 0xFFFFFFFFu, 0u);
    if (bp[j] != EMPTY && visible_by_summary(sm, fast, j, e, slot_stamp(bp, j, FWD_WORDS))) c++;
  }
  return wave_sum_u32(c);
}

// One lane per vertex for slabs of at most DEG_OWN buckets (nearly all
// vertices), each bucket read as lines; the wave takes the longer slabs of
// its 64 vertices one after another, and lists those longer than one
// backward tile (BWD_TILE buckets), with their tiles, for k_degree_tiles
// (parity 0), so a hub does not hold one wave for its whole slab.  A wave
// per vertex had left most lanes idle on one-bucket slabs.
constexpr uint32_t DEG_OWN = 2;
__global__ __launch_bounds__(Q_THREADS) void k_degrees(Store st, uint32_t e, int fast, uint32_t* deg,
                                                       unsigned long long* total, BwdTiles bt) {
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  unsigned long long sum = 0;
  for (uint32_t base = gwave * 64; base < st.V; base += nwaves * 64) {   // wave-uniform
    const uint32_t v = base + lane;
    const bool act = v < st.V;
    const uint64_t desc = act ? st.fdesc[v] : 0;
    const Slab s = slab_of(st.fp, desc);
    const bool own = act && s.nb <= DEG_OWN;
    if (own) {
      uint32_t c = 0;
      for (uint32_t b = 0; b < s.nb; b++) {
        uint32_t* bp = bucket_ptr(s, b);
        uint32_t d[BSLOTS];
        load_dsts(bp, d);
        const uint4 sm = fast ? *reinterpret_cast<const uint4*>(&s.sum[SUM_WORDS * b])
                              : make_uint4(0xFFFFFFFFu, 0xFFFFu, 0xFFFFFFFFu, 0u);
#pragma unroll
        for (int j = 0; j < BSLOTS; j++)
          c += d[j] != EMPTY && visible_by_summary(sm, fast != 0, j, e, slot_stamp(bp, j, FWD_WORDS)) ? 1u : 0u;
      }
      if (deg) deg[v] = c;
      sum += c;
    }
    for (unsigned long long m = __ballot(act && !own); m; m &= m - 1) {
      const int l = __ffsll((long long)m) - 1;
      const uint32_t vv = __shfl(v, l, 64);
      const uint64_t dv = __shfl((unsigned long long)desc, l, 64);
      if (bwd_is_big(dv)) {
        if (deg && lane == 0) deg[vv] = 0;
        bwd_list(bt, 0, vv, dv);
        continue;
      }
      const Slab sv = slab_of(st.fp, dv);
      const uint32_t c = visible_in(sv, 0, sv.nb, e, fast != 0);
      if (lane == 0) {
        if (deg) deg[vv] = c;
        sum += c;
      }
    }
  }
  sum = wave_sum_u64(sum);
  if (lane == 0 && sum) atomicAdd(total, sum);
}

// One wave per listed tile: its count added to the vertex's degree.
__global__ __launch_bounds__(Q_THREADS) void k_degree_tiles(Store st, uint32_t e, int fast, uint32_t* deg,
                                                            unsigned long long* total, BwdTiles bt) {
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  const uint32_t nt = min(bt.head->tiles[0], bt.cap_tiles);
  unsigned long long sum = 0;
  for (uint32_t t = gwave; t < nt; t += nwaves) {
    const uint32_t i = bt.tmap[t];
    if (i >= bt.cap_verts) continue;
    const BigVert bv = bt.big[i];
    if (t < bv.base || t - bv.base >= bv.n) continue;
    const Slab s = slab_of(st.fp, bv.desc);
    const uint32_t b0 = (t - bv.base) << BWD_TILE_LOG;
    if (b0 >= s.nb) continue;
    const uint32_t c = visible_in(s, b0, min(s.nb, b0 + BWD_TILE), e, fast != 0);
    if (lane == 0 && c) {
      if (deg) atomicAdd(&deg[bv.v], c);
      sum += c;
    }
  }
  if (lane == 0 && sum) atomicAdd(total, sum);
}

dg_status stats_dev(dg_graph* g, uint32_t e, uint64_t* n_arcs, uint32_t* deg, hipStream_t s) {
  hipError_t he = ensure_query_scratch(g, g->qs, false, false);
  if (he != hipSuccess) return hip_fail(g, he, "stats scratch");
  if ((he = ensure(g->qs.bt, bwd_tiles_bytes(g->st.fp.cap, 1))) != hipSuccess) return hip_fail(g, he, "stats scratch");
  const BwdTiles bt = bwd_tiles_at(g->qs.bt.as<char>(), g->st.fp.cap, 1);
  unsigned long long* tot = reinterpret_cast<unsigned long long*>(g->qs.counters.as<QCounters>() + 3);
  fill<unsigned long long>(tot, 1, 0ull, s);
  fill<uint32_t>(reinterpret_cast<uint32_t*>(bt.head), sizeof(BwdHead) / 4, 0u, s);
  const int fast = g->concurrent_writers ? 0 : 1;
  k_degrees<<<grid_for(g->cfg.v_capacity, Q_THREADS, 8192), Q_THREADS, 0, s>>>(g->st, e, fast, deg, tot, bt);
  k_degree_tiles<<<resident((const void*)k_degree_tiles), Q_THREADS, 0, s>>>(g->st, e, fast, deg, tot, bt);
  if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "stats launch");
  if (n_arcs) {
    if ((he = hipMemcpyAsync(g->qs.host_counters, tot, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(g, he, "stats copy");
    if ((he = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(g, he, "stats sync");
    std::memcpy(n_arcs, g->qs.host_counters, 8);
  }
  return DG_OK;
}

}  // namespace dg
