// Snapshot queries on epoch e (plain form: one query, host-driven levels).
//
// Frontier work items are (slab descriptor, vertex, tile): a tile is up to
// T consecutive buckets of the vertex's forward slab, so a hub's adjacency
// spreads over many items and every item costs at most T bucket scans.  The
// descriptor is read once when the vertex is pushed and carried in the item,
// so all tiles of a vertex read the same slab even if a concurrent update
// regrows it (the old slab stays intact and holds every version visible at
// e).  A 16-lane group handles one item: lane j reads slot j of a bucket.
//
//   BFS   direction-optimising (Beamer, Asanovic & Patterson, SC 2012):
//         top-down over out-slabs with a CAS claim of dist, or bottom-up
//         over in-slabs of unvisited vertices with a frontier bitmap and
//         early exit; switch when the frontier's slot count exceeds the
//         unexplored count / alpha, back when the frontier falls below
//         live vertices / beta.  Hop distances are the same either way.
//   SSSP  delta-stepping in near/far form (Meyer & Sanders 2003; Davidson
//         et al., IPDPS 2014): label-correcting relaxations with atomicMin
//         below the threshold, far queue above it, threshold += delta when
//         the near queue drains.  Exact for every delta.
//   BC    Brandes (2001): level-synchronous forward BFS with int64
//         shortest-path counts (atomic adds, overflow flagged), then
//         dependencies pulled from successors level by level in FP64 with a
//         fixed lane order (no float atomics); bc[v] += delta[v] for v != s,
//         sources in order.
#include <algorithm>
#include <cstring>

#include "dg_host.h"

namespace dg {

constexpr int Q_THREADS = 256;
constexpr int Q_WAVES = Q_THREADS / 64;
constexpr int Q_ITEMS_PER_BLOCK = Q_WAVES * 4;   // four 16-lane groups per wave

struct Item {
  uint64_t desc;
  uint32_t v;
  uint32_t tile;
};

struct QCounters {
  uint32_t n_items;
  uint32_t n_verts;
  unsigned long long m_next;
  uint32_t n_far;
  int32_t far_min;
  uint32_t overflow;
  uint32_t n_order;
};

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

// ---------------------------------------------------------- item pushes

__device__ inline uint32_t tiles_of(uint64_t desc, uint32_t T) {
  if (desc == 0) return 0;
  uint32_t nb = 1u << (desc & 63);
  return (nb + T - 1) / T;
}

// Every lane of the wave calls this; lanes with push=false add nothing.
__device__ inline void push_items(bool push, uint32_t y, uint64_t desc, uint32_t T, Item* q, uint32_t* counter) {
  uint32_t k = push ? tiles_of(desc, T) : 0;
  uint32_t pos = wave_reserve(counter, k);
  for (uint32_t t = 0; t < k; t++) q[pos + t] = Item{desc, y, t};
}

__device__ inline void count_verts(bool found, uint32_t used, QCounters* c) {
  unsigned long long m = __ballot(found);
  unsigned long long tot = wave_sum_u64(found ? used : 0);
  if (lane_id() == 0 && m) {
    atomicAdd(&c->n_verts, (uint32_t)__popcll(m));
    atomicAdd(&c->m_next, tot);
  }
}

__device__ inline bool bm_test(const uint32_t* bm, uint32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }
__device__ inline void bm_set(uint32_t* bm, uint32_t v) { atomicOr(&bm[v >> 5], 1u << (v & 31)); }

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
  return v;
}

// Seed a query at src: dist/level 0, items of src, bitmap bit.
__global__ void k_seed(Store st, uint32_t src, int32_t* dist, int32_t d0, Item* q, uint32_t* bm, uint32_t T,
                       QCounters* cnt, uint32_t* order) {
  if (threadIdx.x != 0) return;
  uint64_t desc = st.fdesc[src];
  uint32_t k = tiles_of(desc, T);
  for (uint32_t t = 0; t < k; t++) q[t] = Item{desc, src, t};
  if (dist) dist[src] = d0;
  if (bm) bm[src >> 5] |= 1u << (src & 31);
  if (order) order[0] = src;
  QCounters c0{};
  c0.n_items = k;
  c0.n_verts = 1;
  c0.m_next = st.fused[src];
  c0.n_order = 1;
  c0.far_min = DIST_INF;
  cnt[0] = c0;
  QCounters z{};
  z.far_min = DIST_INF;
  cnt[1] = z;
}

// ------------------------------------------------------------------ BFS

struct LevelArgs {
  Store st;
  uint32_t e;
  const Item* qin;
  uint32_t nin;
  Item* qout;
  const uint32_t* bm_cur;
  uint32_t* bm_next;
  int32_t* dist;
  int32_t next_level;
  uint32_t T;
  QCounters* cnt_out;
  QCounters* cnt_reset;
};

__global__ __launch_bounds__(Q_THREADS) void k_bfs_td(LevelArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    QCounters z{};
    z.far_min = DIST_INF;
    *a.cnt_reset = z;
  }
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  for (uint32_t base = gwave * 4; base < a.nin; base += nwaves * 4) {
    uint32_t it = base + grp;
    bool act = it < a.nin;
    Item item = act ? a.qin[it] : Item{0, 0, 0};
    Slab s = slab_of(a.st.fp, item.desc);
    uint32_t b0 = item.tile * a.T;
    uint32_t nbk = act && s.nb > b0 ? min(a.T, s.nb - b0) : 0;
    uint32_t maxnb = wave_max_u32(nbk);
    for (uint32_t i = 0; i < maxnb; i++) {
      bool found = false;
      uint32_t y = 0;
      if (i < nbk) {
        uint32_t* bp = bucket_ptr(s, b0 + i);
        uint32_t d = bp[j];
        if (d != EMPTY && visible(*slot_stamp(bp, j, FWD_WORDS), a.e) && a.dist[d] < 0) {
          if (atomicCAS(&a.dist[d], -1, a.next_level) == -1) {
            found = true;
            y = d;
          }
        }
      }
      uint64_t ydesc = found ? a.st.fdesc[y] : 0;
      push_items(found, y, ydesc, a.T, a.qout, &a.cnt_out->n_items);
      if (found) bm_set(a.bm_next, y);
      count_verts(found, found ? a.st.fused[y] : 0, a.cnt_out);
    }
  }
}

// Bottom-up: each 16-lane group takes one unvisited vertex and scans its
// in-slab (the forward slab when undirected) for a parent in the frontier.
__global__ __launch_bounds__(Q_THREADS) void k_bfs_bu(LevelArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    QCounters z{};
    z.far_min = DIST_INF;
    *a.cnt_reset = z;
  }
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  const uint32_t V = a.st.V;
  const Pool& ip = a.st.undirected ? a.st.fp : a.st.rp;
  const uint64_t* idesc = a.st.undirected ? a.st.fdesc : a.st.rdesc;
  for (uint32_t base = gwave * 4; base < V; base += nwaves * 4) {
    uint32_t y = base + grp;
    bool act = y < V && a.dist[y] < 0;
    Slab s = slab_of(ip, act ? idesc[y] : 0);
    uint32_t nbk = act ? s.nb : 0;
    uint32_t maxnb = wave_max_u32(nbk);
    bool found = false;
    for (uint32_t i = 0; i < maxnb; i++) {
      bool hit = false;
      if (!found && i < nbk) {
        uint32_t* bp = bucket_ptr(s, i);
        uint32_t x = bp[j];
        hit = x != EMPTY && bm_test(a.bm_cur, x) && visible(*slot_stamp(bp, j, s.words), a.e);
      }
      if (group16_ballot(hit)) found = true;
      if (__ballot(!found && i + 1 < nbk) == 0) break;
    }
    bool lead = found && j == 0;
    if (lead) {
      a.dist[y] = a.next_level;
      bm_set(a.bm_next, y);
    }
    uint64_t ydesc = lead ? a.st.fdesc[y] : 0;
    push_items(lead, y, ydesc, a.T, a.qout, &a.cnt_out->n_items);
    count_verts(lead, lead ? a.st.fused[y] : 0, a.cnt_out);
  }
}

static hipError_t ensure_query_scratch(dg_graph* g, QueryScratch& q, bool sssp, bool bc) {
  hipError_t e;
  const uint64_t V = g->cfg.v_capacity;
  uint64_t items = V + g->st.fp.cap / std::max<uint32_t>(1, g->tune.tile_buckets) + 1024;
  if ((e = ensure(q.qa, items * sizeof(Item))) != hipSuccess) return e;
  if ((e = ensure(q.qb, items * sizeof(Item))) != hipSuccess) return e;
  q.items_cap = items;
  uint64_t bmw = (V + 31) / 32 + 1;
  if ((e = ensure(q.bm0, bmw * 4)) != hipSuccess) return e;
  if ((e = ensure(q.bm1, bmw * 4)) != hipSuccess) return e;
  if ((e = ensure(q.counters, 4 * sizeof(QCounters))) != hipSuccess) return e;
  if (!q.host_counters) {
    if ((e = hipHostMalloc(&q.host_counters, 4 * sizeof(QCounters), hipHostMallocDefault)) != hipSuccess) return e;
  }
  if (sssp) {
    if ((e = ensure(q.fa, V * 4 + 64)) != hipSuccess) return e;
    if ((e = ensure(q.fb, V * 4 + 64)) != hipSuccess) return e;
    if ((e = ensure(q.stamp, V * 4 + 64)) != hipSuccess) return e;
    if ((e = ensure(q.flag8, V * 4 + 64)) != hipSuccess) return e;
  }
  if (bc) {
    if ((e = ensure(q.fa, V * 4 + 64)) != hipSuccess) return e;
    if ((e = ensure(q.sigma, V * 8 + 64)) != hipSuccess) return e;
    if ((e = ensure(q.delta, V * 8 + 64)) != hipSuccess) return e;
    if ((e = ensure(q.level, V * 4 + 64)) != hipSuccess) return e;
  }
  return hipSuccess;
}

void free_query_scratch(QueryScratch& q) {
  release(q.qa); release(q.qb); release(q.fa); release(q.fb); release(q.bm0); release(q.bm1);
  release(q.stamp); release(q.flag8); release(q.sigma); release(q.delta); release(q.level);
  release(q.counters);
  if (q.host_counters) hipHostFree(q.host_counters);
  q.host_counters = nullptr;
}

static hipError_t read_counters(QueryScratch& q, int slot, QCounters* out, hipStream_t s) {
  QCounters* dc = q.counters.as<QCounters>() + slot;
  hipError_t e = hipMemcpyAsync(q.host_counters, dc, sizeof(QCounters), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  std::memcpy(out, q.host_counters, sizeof(QCounters));
  return hipSuccess;
}

static uint32_t grid_for(uint64_t units, uint32_t per_block, uint32_t cap = 16384) {
  uint64_t b = (units + per_block - 1) / per_block;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, cap));
}

static dg_status hip_fail(dg_graph* g, hipError_t e, const char* where) {
  g->err = std::string(where) + ": " + hipGetErrorString(e);
  return DG_E_HIP;
}

uint64_t arcs_at(const dg_graph* g, uint32_t e);
uint64_t live_at(const dg_graph* g, uint32_t e);

dg_status bfs_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* dist, hipStream_t s, QueryScratch& q) {
  hipError_t he = ensure_query_scratch(g, q, false, false);
  if (he != hipSuccess) return hip_fail(g, he, "bfs scratch");
  const uint32_t V = g->cfg.v_capacity, T = g->tune.tile_buckets;
  const uint64_t bmw = (V + 31) / 32 + 1;
  Item* qa = q.qa.as<Item>();
  Item* qb = q.qb.as<Item>();
  uint32_t* bm[2] = {q.bm0.as<uint32_t>(), q.bm1.as<uint32_t>()};
  QCounters* cnt = q.counters.as<QCounters>();
  fill<int32_t>(dist, V, -1, s);
  fill<uint32_t>(bm[0], bmw, 0u, s);
  k_seed<<<1, 64, 0, s>>>(g->st, src, dist, 0, qa, bm[0], T, cnt, nullptr);
  QCounters hc;
  if ((he = read_counters(q, 0, &hc, s)) != hipSuccess) return hip_fail(g, he, "bfs seed");
  int64_t m_u = (int64_t)arcs_at(g, e);
  const uint64_t n_live = std::max<uint64_t>(1, live_at(g, e));
  bool bu = false;
  uint32_t n_items = hc.n_items, n_verts = hc.n_verts;
  uint64_t m_f = hc.m_next;
  int level = 0;
  Item* qin = qa;
  Item* qout = qb;
  while (n_verts > 0) {
    int cur = level & 1, nxt = cur ^ 1;
    if (!bu && (int64_t)m_f * (int64_t)g->tune.alpha > m_u) bu = true;
    else if (bu && (uint64_t)n_verts * g->tune.beta < n_live) bu = false;
    m_u -= (int64_t)m_f;
    fill<uint32_t>(bm[nxt], bmw, 0u, s);
    LevelArgs a{g->st, e, qin, n_items, qout, bm[cur], bm[nxt], dist, level + 1, T, cnt + nxt, cnt + cur};
    if (bu) k_bfs_bu<<<grid_for(V, Q_ITEMS_PER_BLOCK), Q_THREADS, 0, s>>>(a);
    else k_bfs_td<<<grid_for(n_items, Q_ITEMS_PER_BLOCK), Q_THREADS, 0, s>>>(a);
    if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "bfs level launch");
    if ((he = read_counters(q, nxt, &hc, s)) != hipSuccess) return hip_fail(g, he, "bfs level");
    n_items = hc.n_items;
    n_verts = hc.n_verts;
    m_f = hc.m_next;
    std::swap(qin, qout);
    level++;
  }
  return DG_OK;
}

// ----------------------------------------------------------------- SSSP

struct RelaxArgs {
  Store st;
  uint32_t e;
  const Item* qin;
  uint32_t nin;
  Item* qout;
  uint32_t* far_out;
  int32_t* dist;
  uint32_t* stamp;     // iteration stamp of the last push into the near queue
  uint32_t* infar;
  int32_t thr;
  uint32_t it1;        // stamp value of the queue being filled
  uint32_t T;
  QCounters* cnt_out;
  QCounters* cnt_reset;
};

__global__ __launch_bounds__(Q_THREADS) void k_sssp_relax(RelaxArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    QCounters z{};
    z.far_min = DIST_INF;
    *a.cnt_reset = z;
  }
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  for (uint32_t base = gwave * 4; base < a.nin; base += nwaves * 4) {
    uint32_t it = base + grp;
    bool act = it < a.nin;
    Item item = act ? a.qin[it] : Item{0, 0, 0};
    Slab s = slab_of(a.st.fp, item.desc);
    uint32_t b0 = item.tile * a.T;
    uint32_t nbk = act && s.nb > b0 ? min(a.T, s.nb - b0) : 0;
    int32_t du = act ? __hip_atomic_load(&a.dist[item.v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    uint32_t maxnb = wave_max_u32(nbk);
    for (uint32_t i = 0; i < maxnb; i++) {
      bool to_near = false, to_far = false;
      uint32_t y = 0;
      if (i < nbk) {
        uint32_t* bp = bucket_ptr(s, b0 + i);
        uint32_t d = bp[j];
        if (d != EMPTY && visible(*slot_stamp(bp, j, FWD_WORDS), a.e)) {
          int32_t nd = du + (int32_t)bp[16 + j];
          if (nd < a.dist[d]) {
            int32_t old = atomicMin(&a.dist[d], nd);
            if (nd < old) {
              y = d;
              if (nd < a.thr) to_near = atomicExch(&a.stamp[d], a.it1) != a.it1;
              else to_far = atomicExch(&a.infar[d], 1u) == 0u;
            }
          }
        }
      }
      uint64_t ydesc = to_near ? a.st.fdesc[y] : 0;
      push_items(to_near, y, ydesc, a.T, a.qout, &a.cnt_out->n_items);
      uint32_t fpos = wave_reserve(&a.cnt_out->n_far, to_far ? 1u : 0u);
      if (to_far) a.far_out[fpos] = y;
      count_verts(to_near, 0, a.cnt_out);
    }
  }
}

struct SplitArgs {
  Store st;
  const uint32_t* far_in;
  uint32_t nin;
  uint32_t* far_out;
  Item* qout;
  int32_t* dist;
  uint32_t* stamp;
  uint32_t* infar;
  int32_t thr;
  uint32_t it1;
  uint32_t T;
  QCounters* cnt_out;
  QCounters* cnt_reset;
};

// Move far entries below the new threshold into the near queue; keep the
// rest and report their minimum distance.
__global__ __launch_bounds__(Q_THREADS) void k_sssp_split(SplitArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    QCounters z{};
    z.far_min = DIST_INF;
    *a.cnt_reset = z;
  }
  for (uint32_t base = blockIdx.x * Q_THREADS; base < a.nin; base += gridDim.x * Q_THREADS) {
    uint32_t i = base + threadIdx.x;
    bool act = i < a.nin;
    uint32_t v = act ? a.far_in[i] : 0;
    int32_t dv = act ? a.dist[v] : DIST_INF;
    bool near = act && dv < a.thr;
    bool keep = act && !near;
    if (near) {
      a.infar[v] = 0u;
      near = atomicExch(&a.stamp[v], a.it1) != a.it1;
    }
    uint64_t vdesc = near ? a.st.fdesc[v] : 0;
    push_items(near, v, vdesc, a.T, a.qout, &a.cnt_out->n_items);
    uint32_t fpos = wave_reserve(&a.cnt_out->n_far, keep ? 1u : 0u);
    if (keep) a.far_out[fpos] = v;
    int32_t m = keep ? dv : DIST_INF;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = min(m, (int32_t)__shfl_xor(m, o, 64));
    if (lane_id() == 0 && m < DIST_INF) atomicMin(&a.cnt_out->far_min, m);
    count_verts(near, 0, a.cnt_out);
  }
}

__global__ void k_inf_to_minus1(int32_t* d, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (d[i] == DIST_INF) d[i] = -1;
}

dg_status sssp_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* dist, hipStream_t s, QueryScratch& q) {
  hipError_t he = ensure_query_scratch(g, q, true, false);
  if (he != hipSuccess) return hip_fail(g, he, "sssp scratch");
  const uint32_t V = g->cfg.v_capacity, T = g->tune.tile_buckets;
  const int32_t delta = (int32_t)std::max<uint32_t>(1, g->tune.sssp_delta);
  Item* qin = q.qa.as<Item>();
  Item* qout = q.qb.as<Item>();
  uint32_t* fin = q.fa.as<uint32_t>();
  uint32_t* fout = q.fb.as<uint32_t>();
  uint32_t* stamp = q.stamp.as<uint32_t>();
  uint32_t* infar = q.flag8.as<uint32_t>();
  QCounters* cnt = q.counters.as<QCounters>();
  fill<int32_t>(dist, V, DIST_INF, s);
  fill<uint32_t>(stamp, V, 0u, s);
  fill<uint32_t>(infar, V, 0u, s);
  k_seed<<<1, 64, 0, s>>>(g->st, src, dist, 0, qin, nullptr, T, cnt, nullptr);
  QCounters hc;
  if ((he = read_counters(q, 0, &hc, s)) != hipSuccess) return hip_fail(g, he, "sssp seed");
  uint32_t n_near = hc.n_items, n_far = 0;
  int32_t thr = delta;
  uint32_t it = 1;   // stamp of the queue being filled; source queue had stamp 0
  int slot = 0;
  for (;;) {
    int nxt = slot ^ 1;
    if (n_near > 0) {
      RelaxArgs a{g->st, e, qin, n_near, qout, fout, dist, stamp, infar, thr, it, T, cnt + nxt, cnt + slot};
      // far entries pushed by this pass land after the current far list
      a.far_out = fin + n_far;
      k_sssp_relax<<<grid_for(n_near, Q_ITEMS_PER_BLOCK), Q_THREADS, 0, s>>>(a);
      if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "sssp relax launch");
      if ((he = read_counters(q, nxt, &hc, s)) != hipSuccess) return hip_fail(g, he, "sssp relax");
      n_near = hc.n_items;
      n_far += hc.n_far;
      std::swap(qin, qout);
      it++;
      slot = nxt;
      continue;
    }
    if (n_far == 0) break;
    int32_t far_min = DIST_INF;
    // advance the threshold until some far entry falls below it
    do {
      thr = far_min == DIST_INF ? thr + delta
                                : (int32_t)std::min<int64_t>(DIST_INF, ((int64_t)far_min / delta + 1) * delta);
      nxt = slot ^ 1;
      SplitArgs a{g->st, fin, n_far, fout, qin, dist, stamp, infar, thr, it, T, cnt + nxt, cnt + slot};
      k_sssp_split<<<grid_for(n_far, Q_THREADS), Q_THREADS, 0, s>>>(a);
      if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "sssp split launch");
      if ((he = read_counters(q, nxt, &hc, s)) != hipSuccess) return hip_fail(g, he, "sssp split");
      slot = nxt;
      std::swap(fin, fout);
      n_far = hc.n_far;
      n_near = hc.n_items;
      far_min = hc.far_min;
    } while (n_near == 0 && n_far > 0);
    it++;
  }
  k_inf_to_minus1<<<grid_for(V, 256, 4096), 256, 0, s>>>(dist, V);
  if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "sssp finish");
  return DG_OK;
}

// ------------------------------------------------------------------- BC

struct BcFwdArgs {
  Store st;
  uint32_t e;
  const Item* qin;
  uint32_t nin;
  Item* qout;
  uint32_t* order;      // vertices in discovery order
  int32_t* level;
  unsigned long long* sigma;
  int32_t next_level;
  uint32_t T;
  QCounters* cnt_out;
  QCounters* cnt_reset;
  QCounters* cnt_total; // n_order running total and the overflow flag
};

__global__ __launch_bounds__(Q_THREADS) void k_bc_fwd(BcFwdArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    QCounters z{};
    z.far_min = DIST_INF;
    *a.cnt_reset = z;
  }
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  uint32_t ovf = 0;
  for (uint32_t base = gwave * 4; base < a.nin; base += nwaves * 4) {
    uint32_t it = base + grp;
    bool act = it < a.nin;
    Item item = act ? a.qin[it] : Item{0, 0, 0};
    Slab s = slab_of(a.st.fp, item.desc);
    uint32_t b0 = item.tile * a.T;
    uint32_t nbk = act && s.nb > b0 ? min(a.T, s.nb - b0) : 0;
    unsigned long long su = act ? a.sigma[item.v] : 0;
    uint32_t maxnb = wave_max_u32(nbk);
    for (uint32_t i = 0; i < maxnb; i++) {
      bool found = false;
      uint32_t y = 0;
      if (i < nbk) {
        uint32_t* bp = bucket_ptr(s, b0 + i);
        uint32_t d = bp[j];
        if (d != EMPTY && visible(*slot_stamp(bp, j, FWD_WORDS), a.e)) {
          int32_t lv = a.level[d];
          if (lv < 0) {
            lv = atomicCAS(&a.level[d], -1, a.next_level);
            if (lv == -1) {
              found = true;
              y = d;
              lv = a.next_level;
            }
          }
          if (lv == a.next_level) {
            unsigned long long old = atomicAdd(&a.sigma[d], su);
            if (old + su > 0x7FFFFFFFFFFFFFFFull || old + su < old) ovf = 1;
          }
        }
      }
      uint64_t ydesc = found ? a.st.fdesc[y] : 0;
      push_items(found, y, ydesc, a.T, a.qout, &a.cnt_out->n_items);
      uint32_t opos = wave_reserve(&a.cnt_total->n_order, found ? 1u : 0u);
      if (found) a.order[opos] = y;
      count_verts(found, 0, a.cnt_out);
    }
  }
  if (ovf) atomicOr(&a.cnt_total->overflow, 1u);
}

// One wave per vertex of level L: delta[v] = sum over visible arcs v->w
// with level[w] = L+1 of sigma[v]/sigma[w] * (1 + delta[w]); lane l reads
// slot l%16 of bucket l/16 of each group of four buckets; the 64 partial
// sums combine by a fixed butterfly, so the result is deterministic.
__global__ __launch_bounds__(Q_THREADS) void k_bc_bwd(Store st, uint32_t e, const uint32_t* verts, uint32_t nv,
                                                      uint32_t src, const int32_t* level, int32_t L,
                                                      const unsigned long long* sigma, double* delta,
                                                      double* bc) {
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  for (uint32_t k = gwave; k < nv; k += nwaves) {
    uint32_t v = verts[k];
    Slab s = slab_of(st.fp, st.fdesc[v]);
    double sv = (double)sigma[v];
    double acc = 0.0;
    for (uint32_t b = lane >> 4; b < s.nb; b += 4) {
      uint32_t* bp = bucket_ptr(s, b);
      uint32_t j = lane & 15;
      uint32_t w = bp[j];
      if (w != EMPTY && visible(*slot_stamp(bp, j, FWD_WORDS), e) && level[w] == L + 1)
        acc += sv / (double)sigma[w] * (1.0 + delta[w]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) {
      delta[v] = acc;
      if (v != src) bc[v] += acc;
    }
  }
}

dg_status bc_dev(dg_graph* g, uint32_t e, const uint32_t* srcs, uint32_t k, double* bc, hipStream_t s,
                 QueryScratch& q) {
  hipError_t he = ensure_query_scratch(g, q, false, true);
  if (he != hipSuccess) return hip_fail(g, he, "bc scratch");
  const uint32_t V = g->cfg.v_capacity, T = g->tune.tile_buckets;
  Item* qa = q.qa.as<Item>();
  Item* qb = q.qb.as<Item>();
  uint32_t* order = q.fa.as<uint32_t>();
  int32_t* level = q.level.as<int32_t>();
  unsigned long long* sigma = q.sigma.as<unsigned long long>();
  double* delta = q.delta.as<double>();
  QCounters* cnt = q.counters.as<QCounters>();
  // cnt[0..1] alternate per level; cnt[2] holds the running order total
  // and the overflow flag of the current source
  QCounters* tot = cnt + 2;
  fill<double>(bc, V, 0.0, s);
  std::vector<uint32_t> off;
  for (uint32_t si = 0; si < k; si++) {
    uint32_t src = srcs[si];
    fill<int32_t>(level, V, -1, s);
    fill<unsigned long long>(sigma, V, 0ull, s);
    k_seed<<<1, 64, 0, s>>>(g->st, src, level, 0, qa, nullptr, T, cnt, order);
    fill<unsigned long long>(reinterpret_cast<unsigned long long*>(tot), sizeof(QCounters) / 8, 0ull, s);
    fill<unsigned long long>(sigma + src, 1, 1ull, s);
    fill<uint32_t>(&tot->n_order, 1, 1u, s);
    QCounters hc;
    if ((he = read_counters(q, 0, &hc, s)) != hipSuccess) return hip_fail(g, he, "bc seed");
    off.assign(1, 0);
    off.push_back(1);
    uint32_t n_items = hc.n_items;
    Item* qin = qa;
    Item* qout = qb;
    int lvl = 0;
    while (true) {
      int cur = lvl & 1, nxt = cur ^ 1;
      BcFwdArgs a{g->st, e, qin, n_items, qout, order, level, sigma, lvl + 1, T, cnt + nxt, cnt + cur, tot};
      if (n_items) k_bc_fwd<<<grid_for(n_items, Q_ITEMS_PER_BLOCK), Q_THREADS, 0, s>>>(a);
      else fill<unsigned long long>(reinterpret_cast<unsigned long long*>(cnt + nxt), sizeof(QCounters) / 8, 0ull, s);
      if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "bc fwd launch");
      if ((he = read_counters(q, nxt, &hc, s)) != hipSuccess) return hip_fail(g, he, "bc fwd");
      if (hc.n_verts == 0) break;
      off.push_back(off.back() + hc.n_verts);
      n_items = hc.n_items;
      std::swap(qin, qout);
      lvl++;
    }
    // overflow flag of the whole forward pass
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
    for (int L = (int)off.size() - 2; L >= 0; L--) {
      uint32_t nv = off[L + 1] - off[L];
      k_bc_bwd<<<grid_for(nv, Q_WAVES), Q_THREADS, 0, s>>>(g->st, e, order + off[L], nv, src, level, L, sigma,
                                                           delta, bc);
    }
    if ((he = hipGetLastError()) != hipSuccess) return hip_fail(g, he, "bc bwd launch");
  }
  return DG_OK;
}

// ---------------------------------------------------------------- stats

__global__ __launch_bounds__(Q_THREADS) void k_degrees(Store st, uint32_t e, uint32_t* deg,
                                                       unsigned long long* total) {
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * Q_WAVES;
  unsigned long long sum = 0;
  for (uint32_t v = gwave; v < st.V; v += nwaves) {
    Slab s = slab_of(st.fp, st.fdesc[v]);
    uint32_t c = 0;
    for (uint32_t b = lane >> 4; b < s.nb; b += 4) {
      uint32_t* bp = bucket_ptr(s, b);
      uint32_t j = lane & 15;
      if (bp[j] != EMPTY && visible(*slot_stamp(bp, j, FWD_WORDS), e)) c++;
    }
    c = wave_sum_u32(c);
    if (lane == 0) {
      if (deg) deg[v] = c;
      sum += c;
    }
  }
  if (lane == 0 && sum) atomicAdd(total, sum);
}

dg_status stats_dev(dg_graph* g, uint32_t e, uint64_t* n_arcs, uint32_t* deg, hipStream_t s) {
  hipError_t he = ensure_query_scratch(g, g->qs, false, false);
  if (he != hipSuccess) return hip_fail(g, he, "stats scratch");
  unsigned long long* tot = reinterpret_cast<unsigned long long*>(g->qs.counters.as<QCounters>());
  fill<unsigned long long>(tot, 1, 0ull, s);
  k_degrees<<<grid_for(g->cfg.v_capacity, Q_WAVES, 8192), Q_THREADS, 0, s>>>(g->st, e, deg, tot);
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
