// Level steps of the snapshot queries, shared by the one-query kernels
// (query.hip) and the persistent multi-query engine (batch.hip).
//
// A step is executed by `nworkers` workgroups numbered `worker`; each
// workgroup loops over its share of the step's units in workgroup-uniform
// strides and may use the LDS block `Shared`.
//
// Frontier work items are (slab descriptor, vertex, tile): a tile is up to
// T consecutive buckets of the vertex's forward slab, so a hub's adjacency
// spreads over many items and every item costs at most T bucket scans.  The
// descriptor is read once when the vertex is pushed and carried in the item,
// so all tiles of a vertex read the same slab even if a concurrent update
// regrows it (the old slab stays intact and holds every version visible at
// e).  A 16-lane group handles one item: lane j reads slot j of a bucket,
// four buckets in flight at a time.  Pushes are staged in LDS and flushed
// with one global atomic per workgroup pass; counters live in registers
// and are added once per wave.
#pragma once
#include "dg_internal.h"

namespace dg {

constexpr int Q_THREADS = 256;
constexpr int Q_WAVES = Q_THREADS / 64;
constexpr int Q_ITEMS_PER_BLOCK = Q_WAVES * 4;   // four 16-lane groups per wave
constexpr int STAGE = 2048;                      // staged pushes per workgroup pass
constexpr int STAGE_BIG = 256;
constexpr uint32_t BU_CHUNK = 8;                 // buckets per bottom-up chunk item

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
  unsigned long long arcs;   // visible arcs examined
  uint32_t n_big;            // bottom-up chunk items
  uint32_t pad;
};

__device__ inline void zero_counters(QCounters* c) {
  QCounters z{};
  z.far_min = DIST_INF;
  *c = z;
}

// Which buckets of a slab an item covers: tiles of `chunk` buckets starting
// at bucket `first`.
struct TileShape {
  uint32_t first, chunk;
  __device__ uint32_t tiles(uint64_t desc) const {
    if (desc == 0) return 0;
    uint32_t nb = 1u << (desc & 63);
    return nb > first ? (nb - first + chunk - 1) / chunk : 0;
  }
};

// ------------------------------------------------------- LDS staging

template <int N>
struct ItemStageT {
  uint32_t cnt;
  uint32_t v[N];
  uint64_t d[N];
};
template <int N>
struct U32StageT {
  uint32_t cnt;
  uint32_t v[N];
};

struct Shared {
  ItemStageT<STAGE> a;              // next-frontier items
  union {
    ItemStageT<STAGE_BIG> b;        // bottom-up chunk items
    U32StageT<STAGE> u;             // far queue / discovery order
  };
  uint32_t wsum[Q_WAVES];
  uint32_t base;
  uint32_t flag;
};

__device__ inline uint32_t wave_rank(unsigned long long m) {
  return (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
}

// Wave-uniform call: lanes with push append (v, desc).  Positions past the
// stage capacity go straight to the global queue.
template <int N>
__device__ inline void stage_item(ItemStageT<N>& sb, bool push, uint32_t v, uint64_t desc, Item* gq,
                                  uint32_t* gcnt, TileShape ts) {
  unsigned long long m = __ballot(push);
  if (m == 0) return;
  int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(&sb.cnt, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  uint32_t pos = base + wave_rank(m);
  if (push) {
    if (pos < (uint32_t)N) {
      sb.v[pos] = v;
      sb.d[pos] = desc;
    } else {
      uint32_t k = ts.tiles(desc);
      uint32_t p = atomicAdd(gcnt, k);
      for (uint32_t t = 0; t < k; t++) gq[p + t] = Item{desc, v, t};
    }
  }
}

template <int N>
__device__ inline void stage_u32(U32StageT<N>& sb, bool push, uint32_t v, uint32_t* gq, uint32_t* gcnt) {
  unsigned long long m = __ballot(push);
  if (m == 0) return;
  int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(&sb.cnt, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  uint32_t pos = base + wave_rank(m);
  if (push) {
    if (pos < (uint32_t)N) sb.v[pos] = v;
    else gq[atomicAdd(gcnt, 1u)] = v;
  }
}

__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* total, uint32_t* wsum) {
  uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < Q_WAVES; w++) {
    uint32_t s = wsum[w];
    if ((uint32_t)w < wave) off += s;
    tot += s;
  }
  *total = tot;
  return off + incl - x;
}

// Workgroup-wide: write the staged vertices' tiles to the global queue.
template <int N>
__device__ inline void flush_items(ItemStageT<N>& sb, Item* gq, uint32_t* gcnt, TileShape ts, Shared& sh) {
  constexpr int PER = (N + Q_THREADS - 1) / Q_THREADS;
  __syncthreads();
  uint32_t n = min(sb.cnt, (uint32_t)N);
  if (n == 0) return;   // workgroup-uniform
  uint32_t tl[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    uint32_t e = threadIdx.x * PER + k;
    tl[k] = e < n ? ts.tiles(sb.d[e]) : 0;
    sum += tl[k];
  }
  uint32_t total;
  uint32_t off = block_excl_scan(sum, &total, sh.wsum);
  if (threadIdx.x == 0) {
    sh.base = total ? atomicAdd(gcnt, total) : 0;
    sb.cnt = 0;
  }
  __syncthreads();
  uint32_t p = sh.base + off;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    uint32_t e = threadIdx.x * PER + k;
    if (e < n) {
      uint64_t d = sb.d[e];
      uint32_t v = sb.v[e];
      for (uint32_t t = 0; t < tl[k]; t++) gq[p + t] = Item{d, v, t};
    }
    p += tl[k];
  }
  __syncthreads();
}

template <int N>
__device__ inline void flush_u32(U32StageT<N>& sb, uint32_t* gq, uint32_t* gcnt, Shared& sh) {
  __syncthreads();
  uint32_t n = min(sb.cnt, (uint32_t)N);
  if (n == 0) return;
  if (threadIdx.x == 0) {
    sh.base = atomicAdd(gcnt, n);
    sb.cnt = 0;
  }
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < n; e += Q_THREADS) gq[sh.base + e] = sb.v[e];
  __syncthreads();
}

__device__ inline void stages_init(Shared& sh) {
  if (threadIdx.x == 0) {
    sh.a.cnt = 0;
    sh.b.cnt = 0;
    sh.u.cnt = 0;
  }
  __syncthreads();
}

// Register counters, added once per wave.
struct LaneCounts {
  uint32_t verts = 0;
  unsigned long long m = 0;
  uint32_t arcs = 0;
  __device__ void commit(QCounters* c) {
    uint32_t v = wave_sum_u32(verts);
    unsigned long long mm = wave_sum_u64(m);
    unsigned long long a = wave_sum_u64(arcs);
    if (lane_id() == 0) {
      if (v) atomicAdd(&c->n_verts, v);
      if (mm) atomicAdd(&c->m_next, mm);
      if (a) atomicAdd(&c->arcs, a);
    }
  }
};

__device__ inline bool bm_test(const uint32_t* bm, uint32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }
__device__ inline void bm_set(uint32_t* bm, uint32_t v) { atomicOr(&bm[v >> 5], 1u << (v & 31)); }

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
  return v;
}

// The group's item: slab, first bucket and bucket count (0 when inactive).
struct ItemView {
  Slab s;
  uint32_t b0, nbk, v;
};

__device__ inline ItemView view_item(const Pool& p, const Item* q, uint32_t idx, uint32_t n, TileShape ts) {
  ItemView iv;
  bool act = idx < n;
  Item it = act ? q[idx] : Item{0, 0, 0};
  iv.s = slab_of(p, it.desc);
  iv.b0 = ts.first + it.tile * ts.chunk;
  iv.nbk = act && iv.s.nb > iv.b0 ? min(ts.chunk, iv.s.nb - iv.b0) : 0;
  iv.v = it.v;
  return iv;
}

// Slot j of four consecutive buckets of an item (EMPTY past its end), with
// visibility at e resolved from the bucket summaries and, where needed,
// the stamps.
struct Slots4 {
  uint32_t d[4];
  int32_t w[4];
  bool vis[4];
};

template <bool WITH_W>
__device__ inline Slots4 load4(const ItemView& iv, uint32_t i, uint32_t j, uint32_t e, bool fast) {
  Slots4 r;
  uint2 sm[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    r.d[k] = EMPTY;
    r.w[k] = 0;
    sm[k] = make_uint2(0xFFFFFFFFu, 0xFFFFu);
    if (i + k < iv.nbk) {
      uint32_t b = iv.b0 + i + k;
      uint32_t* bp = bucket_ptr(iv.s, b);
      r.d[k] = bp[j];
      if (WITH_W) r.w[k] = (int32_t)bp[16 + j];
      if (fast) sm[k] = *reinterpret_cast<const uint2*>(&iv.s.sum[2 * b]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    bool v = false;
    if (r.d[k] != EMPTY) {
      if (fast && sm[k].x <= e && !((sm[k].y >> j) & 1u)) v = true;
      else v = visible(*slot_stamp(bucket_ptr(iv.s, iv.b0 + i + k), j, iv.s.words), e);
    }
    r.vis[k] = v;
  }
  return r;
}

// ------------------------------------------------------------------ BFS

struct LevelArgs {
  Store st;
  uint32_t e;
  int fast;
  const Item* qin;
  Item* qout;
  Item* qbig;
  const uint32_t* bm_cur;
  uint32_t* bm_next;
  int32_t* dist;
  int32_t next_level;
  uint32_t T;
  QCounters* cnt_out;
};

__device__ __forceinline__ void td_step(const LevelArgs& a, uint32_t nin, uint32_t worker, uint32_t nworkers, Shared& sh) {
  const TileShape ts{0, a.T};
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15, wave = threadIdx.x >> 6;
  LaneCounts lc;
  for (uint32_t base = worker * Q_ITEMS_PER_BLOCK; base < nin; base += nworkers * Q_ITEMS_PER_BLOCK) {
    ItemView iv = view_item(a.st.fp, a.qin, base + wave * 4 + grp, nin, ts);
    uint32_t maxnb = wave_max_u32(iv.nbk);
    for (uint32_t i = 0; i < maxnb; i += 4) {
      Slots4 s4 = load4<false>(iv, i, j, a.e, a.fast);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        bool found = false;
        uint32_t d = s4.d[k];
        if (s4.vis[k]) {
          lc.arcs++;
          if (a.dist[d] < 0 && atomicCAS(&a.dist[d], -1, a.next_level) == -1) found = true;
        }
        uint64_t yd = 0;
        if (found) {
          yd = a.st.fdesc[d];
          bm_set(a.bm_next, d);
          lc.verts++;
          lc.m += a.st.fused[d];
        }
        stage_item(sh.a, found, d, yd, a.qout, &a.cnt_out->n_items, ts);
      }
    }
    flush_items(sh.a, a.qout, &a.cnt_out->n_items, ts, sh);
  }
  lc.commit(a.cnt_out);
}

// Bottom-up, one unvisited vertex per lane: a one-bucket in-slab (the
// forward slab when undirected) is scanned by the lane itself, stopping at
// the first empty slot or at a parent in the frontier; longer in-slabs
// become chunk items of BU_CHUNK buckets for bu_big_step.
__device__ __forceinline__ void bu_step(const LevelArgs& a, uint32_t worker, uint32_t nworkers, Shared& sh) {
  const TileShape ts{0, a.T}, tbig{0, BU_CHUNK};
  const uint32_t V = a.st.V;
  const Pool& ip = a.st.undirected ? a.st.fp : a.st.rp;
  const uint64_t* idesc = a.st.undirected ? a.st.fdesc : a.st.rdesc;
  LaneCounts lc;
  for (uint32_t base = worker * Q_THREADS; base < V; base += nworkers * Q_THREADS) {
    uint32_t y = base + threadIdx.x;
    bool act = y < V && a.dist[y] < 0;
    uint64_t ydesc_in = act ? idesc[y] : 0;
    Slab s = slab_of(ip, ydesc_in);
    bool found = false;
    if (act && s.nb == 1) {
      const uint4* src4 = reinterpret_cast<const uint4*>(s.base);
      uint2 sm = a.fast ? *reinterpret_cast<const uint2*>(s.sum) : make_uint2(0xFFFFFFFFu, 0xFFFFu);
      bool fastb = a.fast && sm.x <= a.e;
      bool more = true;   // no empty slot seen yet (used slots are a prefix)
      // four slots per 16-byte load; each slot is tested in turn until a
      // parent is found or an empty slot ends the bucket
      auto slot = [&](uint32_t x, int j) {
        if (!more || found) return;
        if (x == EMPTY) {
          more = false;
          return;
        }
        bool vis = (fastb && !((sm.y >> j) & 1u)) || visible(*slot_stamp(s.base, j, s.words), a.e);
        if (vis) {
          lc.arcs++;
          found = bm_test(a.bm_cur, x);
        }
      };
#pragma unroll
      for (int q = 0; q < 4; q++) {
        uint4 v = src4[q];
        slot(v.x, 4 * q);
        slot(v.y, 4 * q + 1);
        slot(v.z, 4 * q + 2);
        slot(v.w, 4 * q + 3);
      }
    }
    uint64_t yd = 0;
    if (found) {
      a.dist[y] = a.next_level;
      bm_set(a.bm_next, y);
      yd = a.st.fdesc[y];
      lc.verts++;
      lc.m += a.st.fused[y];
    }
    stage_item(sh.a, found, y, yd, a.qout, &a.cnt_out->n_items, ts);
    stage_item(sh.b, act && s.nb > 1, y, ydesc_in, a.qbig, &a.cnt_out->n_big, tbig);
    flush_items(sh.a, a.qout, &a.cnt_out->n_items, ts, sh);
    flush_items(sh.b, a.qbig, &a.cnt_out->n_big, tbig, sh);
  }
  lc.commit(a.cnt_out);
}

// Chunk items of multi-bucket in-slabs: 16 lanes per chunk; a chunk whose
// vertex already has a parent is skipped, and the first finder claims it.
__device__ __forceinline__ void bu_big_step(const LevelArgs& a, uint32_t nbig, uint32_t worker, uint32_t nworkers,
                                   Shared& sh) {
  const TileShape ts{0, a.T}, tbig{0, BU_CHUNK};
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15, wave = threadIdx.x >> 6;
  const Pool& ip = a.st.undirected ? a.st.fp : a.st.rp;
  LaneCounts lc;
  for (uint32_t base = worker * Q_ITEMS_PER_BLOCK; base < nbig; base += nworkers * Q_ITEMS_PER_BLOCK) {
    ItemView iv = view_item(ip, a.qbig, base + wave * 4 + grp, nbig, tbig);
    uint32_t y = iv.v;
    if (iv.nbk && a.dist[y] >= 0) iv.nbk = 0;
    uint32_t maxnb = wave_max_u32(iv.nbk);
    bool found = false;
    for (uint32_t i = 0; i < maxnb; i += 4) {
      Slots4 s4 = load4<false>(iv, i, j, a.e, a.fast);
      bool hit = false;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if (s4.vis[k]) {
          lc.arcs++;
          hit |= bm_test(a.bm_cur, s4.d[k]);
        }
      }
      if (group16_ballot(hit)) found = true;
      if (__ballot(!found && i + 4 < iv.nbk) == 0) break;
    }
    bool win = found && j == 0 && atomicCAS(&a.dist[y], -1, a.next_level) == -1;
    uint64_t yd = 0;
    if (win) {
      bm_set(a.bm_next, y);
      yd = a.st.fdesc[y];
      lc.verts++;
      lc.m += a.st.fused[y];
    }
    stage_item(sh.a, win, y, yd, a.qout, &a.cnt_out->n_items, ts);
    flush_items(sh.a, a.qout, &a.cnt_out->n_items, ts, sh);
  }
  lc.commit(a.cnt_out);
}

// ----------------------------------------------------------------- SSSP

struct RelaxArgs {
  Store st;
  uint32_t e;
  int fast;
  const Item* qin;
  Item* qout;
  uint32_t* far_out;
  int32_t* dist;
  uint32_t* stamp;     // iteration stamp of the last push into the near queue
  uint32_t* infar;
  int32_t thr;
  uint32_t it1;        // stamp value of the queue being filled
  uint32_t T;
  QCounters* cnt_out;
  // light/heavy split (Meyer & Sanders): mode 0 relaxes every arc; mode 1
  // only arcs with w <= light and records each processed vertex once per
  // bucket (rstamp == phase) in rlist; mode 2 only arcs with w > light
  int mode;
  int32_t light;
  uint32_t* rlist;
  uint32_t* rcount;
  uint32_t* rstamp;
  uint32_t phase;
};

__device__ __forceinline__ void relax_step(const RelaxArgs& a, uint32_t nin, uint32_t worker, uint32_t nworkers,
                                  Shared& sh) {
  const TileShape ts{0, a.T};
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15, wave = threadIdx.x >> 6;
  LaneCounts lc;
  for (uint32_t base = worker * Q_ITEMS_PER_BLOCK; base < nin; base += nworkers * Q_ITEMS_PER_BLOCK) {
    ItemView iv = view_item(a.st.fp, a.qin, base + wave * 4 + grp, nin, ts);
    int32_t du = iv.nbk ? __hip_atomic_load(&a.dist[iv.v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    if (a.mode == 1) {
      // the first tile's item records its vertex for the bucket's heavy pass
      bool rec = iv.nbk && iv.b0 == 0 && j == 0 && atomicExch(&a.rstamp[iv.v], a.phase) != a.phase;
      uint32_t pos = wave_reserve(a.rcount, rec ? 1u : 0u);
      if (rec) a.rlist[pos] = iv.v;
    }
    uint32_t maxnb = wave_max_u32(iv.nbk);
    for (uint32_t i = 0; i < maxnb; i += 4) {
      Slots4 s4 = load4<true>(iv, i, j, a.e, a.fast);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        bool to_near = false, to_far = false;
        uint32_t d = s4.d[k];
        bool take = a.mode == 0 || ((a.mode == 1) == (s4.w[k] <= a.light));
        if (s4.vis[k] && take) {
          lc.arcs++;
          int32_t nd = du + s4.w[k];
          if (nd < a.dist[d]) {
            int32_t old = atomicMin(&a.dist[d], nd);
            if (nd < old) {
              if (nd < a.thr) to_near = atomicExch(&a.stamp[d], a.it1) != a.it1;
              else to_far = atomicExch(&a.infar[d], 1u) == 0u;
            }
          }
        }
        uint64_t yd = to_near ? a.st.fdesc[d] : 0;
        lc.verts += to_near ? 1 : 0;
        stage_item(sh.a, to_near, d, yd, a.qout, &a.cnt_out->n_items, ts);
        stage_u32(sh.u, to_far, d, a.far_out, &a.cnt_out->n_far);
      }
    }
    flush_items(sh.a, a.qout, &a.cnt_out->n_items, ts, sh);
    flush_u32(sh.u, a.far_out, &a.cnt_out->n_far, sh);
  }
  lc.commit(a.cnt_out);
}

// Items of every vertex in list[0..n): the recorded vertices of a settled
// bucket, for its heavy-arc pass.
__device__ __forceinline__ void expand_step(const Store& st, const uint32_t* list, uint32_t n, Item* qout,
                                            QCounters* cnt_out, uint32_t T, uint32_t worker, uint32_t nworkers,
                                            Shared& sh) {
  const TileShape ts{0, T};
  for (uint32_t base = worker * Q_THREADS; base < n; base += nworkers * Q_THREADS) {
    uint32_t i = base + threadIdx.x;
    bool act = i < n;
    uint32_t v = act ? list[i] : 0;
    uint64_t vd = act ? st.fdesc[v] : 0;
    stage_item(sh.a, act && vd != 0, v, vd, qout, &cnt_out->n_items, ts);
    flush_items(sh.a, qout, &cnt_out->n_items, ts, sh);
  }
}

struct SplitArgs {
  Store st;
  const uint32_t* far_in;
  uint32_t* far_out;
  Item* qout;
  int32_t* dist;
  uint32_t* stamp;
  uint32_t* infar;
  int32_t thr;
  uint32_t it1;
  uint32_t T;
  QCounters* cnt_out;
};

// Move far entries below the threshold into the near queue; keep the rest
// and report their minimum distance.
__device__ __forceinline__ void split_step(const SplitArgs& a, uint32_t nin, uint32_t worker, uint32_t nworkers,
                                  Shared& sh) {
  const TileShape ts{0, a.T};
  LaneCounts lc;
  int32_t mn = DIST_INF;
  for (uint32_t base = worker * Q_THREADS; base < nin; base += nworkers * Q_THREADS) {
    uint32_t i = base + threadIdx.x;
    bool act = i < nin;
    uint32_t v = act ? a.far_in[i] : 0;
    int32_t dv = act ? a.dist[v] : DIST_INF;
    bool near = act && dv < a.thr;
    bool keep = act && !near;
    if (near) {
      a.infar[v] = 0u;
      near = atomicExch(&a.stamp[v], a.it1) != a.it1;
    }
    if (keep) mn = min(mn, dv);
    uint64_t vd = near ? a.st.fdesc[v] : 0;
    lc.verts += near ? 1 : 0;
    stage_item(sh.a, near, v, vd, a.qout, &a.cnt_out->n_items, ts);
    stage_u32(sh.u, keep, v, a.far_out, &a.cnt_out->n_far);
    flush_items(sh.a, a.qout, &a.cnt_out->n_items, ts, sh);
    flush_u32(sh.u, a.far_out, &a.cnt_out->n_far, sh);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mn = min(mn, (int32_t)__shfl_xor(mn, o, 64));
  if (lane_id() == 0 && mn < DIST_INF) atomicMin(&a.cnt_out->far_min, mn);
  lc.commit(a.cnt_out);
}

// ------------------------------------------------------------------- BC

struct BcFwdArgs {
  Store st;
  uint32_t e;
  int fast;
  const Item* qin;
  Item* qout;
  uint32_t* order;      // vertices in discovery order
  int32_t* level;
  unsigned long long* sigma;
  int32_t next_level;
  uint32_t T;
  QCounters* cnt_out;
  QCounters* cnt_total; // discovery-order length and the overflow flag
};

__device__ __forceinline__ void bcfwd_step(const BcFwdArgs& a, uint32_t nin, uint32_t worker, uint32_t nworkers,
                                  Shared& sh) {
  const TileShape ts{0, a.T};
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15, wave = threadIdx.x >> 6;
  LaneCounts lc;
  uint32_t ovf = 0;
  for (uint32_t base = worker * Q_ITEMS_PER_BLOCK; base < nin; base += nworkers * Q_ITEMS_PER_BLOCK) {
    ItemView iv = view_item(a.st.fp, a.qin, base + wave * 4 + grp, nin, ts);
    unsigned long long su = iv.nbk ? a.sigma[iv.v] : 0;
    uint32_t maxnb = wave_max_u32(iv.nbk);
    for (uint32_t i = 0; i < maxnb; i += 4) {
      Slots4 s4 = load4<false>(iv, i, j, a.e, a.fast);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        bool found = false;
        uint32_t d = s4.d[k];
        if (s4.vis[k]) {
          lc.arcs++;
          int32_t lv = a.level[d];
          if (lv < 0) {
            lv = atomicCAS(&a.level[d], -1, a.next_level);
            if (lv == -1) {
              found = true;
              lv = a.next_level;
            }
          }
          if (lv == a.next_level) {
            unsigned long long old = atomicAdd(&a.sigma[d], su);
            if (old + su > 0x7FFFFFFFFFFFFFFFull) ovf = 1;
          }
        }
        uint64_t yd = found ? a.st.fdesc[d] : 0;
        lc.verts += found ? 1 : 0;
        stage_item(sh.a, found, d, yd, a.qout, &a.cnt_out->n_items, ts);
        stage_u32(sh.u, found, d, a.order, &a.cnt_total->n_order);
      }
    }
    flush_items(sh.a, a.qout, &a.cnt_out->n_items, ts, sh);
    flush_u32(sh.u, a.order, &a.cnt_total->n_order, sh);
  }
  if (ovf) atomicOr(&a.cnt_total->overflow, 1u);
  lc.commit(a.cnt_out);
}

// One wave per vertex of level L: delta[v] = sum over visible arcs v->w
// with level[w] = L+1 of sigma[v]/sigma[w] * (1 + delta[w]); lane l reads
// slot l%16 of bucket l/16 of each group of four buckets; the 64 partial
// sums combine by a fixed butterfly, so the result is deterministic for a
// given slab layout.
__device__ __forceinline__ void bcbwd_step(const Store& st, uint32_t e, bool fast, const uint32_t* verts, uint32_t nv,
                                  uint32_t src, const int32_t* level, int32_t L, const unsigned long long* sigma,
                                  double* delta, double* bc, uint32_t worker, uint32_t nworkers) {
  const uint32_t lane = lane_id();
  const uint32_t gwave = worker * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = nworkers * Q_WAVES;
  for (uint32_t k = gwave; k < nv; k += nwaves) {
    uint32_t v = verts[k];
    Slab s = slab_of(st.fp, st.fdesc[v]);
    double sv = (double)sigma[v];
    double acc = 0.0;
    const uint32_t j = lane & 15;
    for (uint32_t b = lane >> 4; b < s.nb; b += 4) {
      uint32_t* bp = bucket_ptr(s, b);
      uint32_t w = bp[j];
      if (w != EMPTY && slot_visible(s, bp, b, j, e, fast) && level[w] == L + 1)
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

}  // namespace dg
