// Level steps of the snapshot queries, shared by the one-query kernels
// (query.hip) and the persistent multi-query engine (batch.hip).
//
// A step is executed by `nworkers` workgroups numbered `worker`; inside a
// step every wave works on its own, and the only workgroup barrier is the
// one that sums the step's counters at its end.
//
// Frontier queues (Front) hold one item per pushed vertex: its forward-slab
// descriptor, read once at push time and carried in the item so that a
// concurrent regrowth cannot change the slab under a query (the old slab
// stays intact and holds every version visible at e), and its flat start.
// The slabs of the queue's items are laid end to end in one flat bucket
// sequence, item by item in queue order; a flush reserves its items and
// their buckets with one 64-bit atomic, so item order and flat order agree.
// The flat sequence is cut into chunks of 16, 32 or 64 buckets (a tuning
// value), and cmap[c] names the item holding the first bucket of chunk c.
// A consuming step hands out
// whole chunks to waves, so every wave gets the same number of buckets no
// matter how degrees are distributed: a hub's slab spreads over many waves,
// and runs of one-bucket vertices fill a wave's lanes.  Within a chunk, a
// 16-lane group handles one (item, bucket) pair at a time, lane j reading
// slot j, with four pairs in flight per group.
//
// Pushes are staged in the wave's own LDS arrays with a wave-uniform count
// and appended to the global queue with one atomic per flush; a wave
// flushes when its stage could overflow on the next round and at the end
// of the step.
#pragma once
#include "dg_internal.h"

namespace dg {

constexpr int Q_THREADS = 256;
constexpr int Q_WAVES = Q_THREADS / 64;
constexpr uint32_t CH_MAX = 64;                   // largest chunk (a chunk holds at most CH_MAX items)
constexpr uint32_t CH_MIN = 16;
constexpr int WSTAGE = 256;                       // staged pushes per wave
constexpr uint32_t BU_CHUNK = 8;                  // buckets per bottom-up chunk item

struct Item {
  uint64_t desc;
  uint32_t v;
  uint32_t aux;   // frontier queue: flat start; bottom-up chunk queue: chunk index
};

// A frontier queue and its chunk map, with their capacities; chunks hold
// 1 << lch buckets (16, 32 or 64).
struct Front {
  Item* q;
  uint32_t* cmap;
  uint32_t qcap, ccap;
  uint32_t lch;
};

enum : uint32_t { OVF_SIGMA = 1, OVF_QUEUE = 2 };

struct QCounters {
  unsigned long long fq;     // frontier items (low half) | flat buckets (high half)
  uint32_t n_verts;
  uint32_t n_far;
  unsigned long long m_next;
  int32_t far_min;
  uint32_t overflow;         // OVF_* bits
  uint32_t n_order;
  uint32_t n_big;            // bottom-up chunk items
  unsigned long long arcs;   // visible arcs examined
};

__host__ __device__ inline uint32_t fq_items(unsigned long long fq) { return (uint32_t)fq; }
__host__ __device__ inline uint32_t fq_buckets(unsigned long long fq) { return (uint32_t)(fq >> 32); }
__host__ __device__ inline uint32_t fq_chunks(unsigned long long fq, uint32_t lch) {
  return (uint32_t)(((uint64_t)fq_buckets(fq) + (1u << lch) - 1) >> lch);
}

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

// ------------------------------------------------------ wave helpers

__device__ inline uint32_t wave_rank(unsigned long long m) {
  return (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
}

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

__device__ inline unsigned long long wave_incl_scan64(unsigned long long x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
  return v;
}

// LDS written by some lanes of a wave is read by others after this.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------- wave-private staging

struct WaveStage {
  uint32_t v[WSTAGE];
  uint64_t d[WSTAGE];
  uint32_t u[WSTAGE];
  uint32_t s[WSTAGE];   // flat starts of a flush's items (chunk map)
};

struct Shared {
  WaveStage ws[Q_WAVES];
  unsigned long long part[Q_WAVES][4];   // per-wave counter sums
  uint32_t wsum[Q_WAVES];
  uint32_t base;
  uint32_t flag;
};

// Workgroup-wide exclusive prefix sum of one value per thread (takes a
// barrier); *total receives the sum over the workgroup.
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* total, Shared& sh) {
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t incl = wave_incl_scan(x);
  if (lane == 63) sh.wsum[wave] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < Q_WAVES; w++) {
    const uint32_t v = sh.wsum[w];
    if ((uint32_t)w < wave) off += v;
    tot += v;
  }
  *total = tot;
  return off + incl - x;
}

// A wave's item stage: LDS arrays plus a wave-uniform count.
struct ItemQ {
  uint32_t* v;
  uint64_t* d;
  uint32_t* s;
  uint32_t cap;
  uint32_t n;
};
struct U32Q {
  uint32_t* v;
  uint32_t cap;
  uint32_t n;
};

__device__ inline ItemQ item_q(WaveStage& s, uint32_t off, uint32_t cap) {
  return ItemQ{s.v + off, s.d + off, s.s + off, cap, 0};
}
__device__ inline U32Q u32_q(WaveStage& s) { return U32Q{s.u, WSTAGE, 0}; }

// Wave-uniform call: lanes with push append (v, desc).
__device__ inline void push_item(ItemQ& q, bool push, uint32_t v, uint64_t desc) {
  unsigned long long m = __ballot(push);
  uint32_t pos = q.n + wave_rank(m);
  if (push) {
    q.v[pos] = v;
    q.d[pos] = desc;
  }
  q.n += (uint32_t)__popcll(m);
}

__device__ inline void push_u32(U32Q& q, bool push, uint32_t v) {
  unsigned long long m = __ballot(push);
  uint32_t pos = q.n + wave_rank(m);
  if (push) q.v[pos] = v;
  q.n += (uint32_t)__popcll(m);
}

// Tile queue (bottom-up chunk items): write the staged vertices' tiles
// (one atomic).
// Staged entries' tile counts and first tiles (in q.s), and the wave total.
__device__ inline uint32_t tiles_stage_scan(ItemQ& q, TileShape ts) {
  constexpr int PER = WSTAGE / 64;
  const uint32_t lane = lane_id();
  uint32_t tl[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    uint32_t e = lane * PER + k;
    tl[k] = e < q.n ? ts.tiles(q.d[e]) : 0;
    sum += tl[k];
  }
  uint32_t incl = wave_incl_scan(sum);
  uint32_t p = incl - sum;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    uint32_t e = lane * PER + k;
    if (e < q.n) q.s[e] = p;
    p += tl[k];
  }
  wave_lds_sync();
  return __shfl(incl, 63, 64);
}

// The wave writes its tiles at gb together, consecutive lanes consecutive
// tiles, so a hub's many tiles do not fall to one lane.
__device__ inline void tiles_stage_write(ItemQ& q, Item* gq, uint32_t gb, uint32_t total) {
  for (uint32_t i = lane_id(); i < total; i += 64) {
    uint32_t lo = 0, hi = q.n;   // last entry whose first tile is <= i
    while (hi - lo > 1) {
      const uint32_t m = (lo + hi) >> 1;
      if (q.s[m] <= i) lo = m;
      else hi = m;
    }
    gq[gb + i] = Item{q.d[lo], q.v[lo], i - q.s[lo]};
  }
  q.n = 0;
  wave_lds_sync();
}

__device__ inline void flush_tiles(ItemQ& q, Item* gq, uint32_t* gcnt, TileShape ts) {
  if (q.n == 0) return;   // wave-uniform
  wave_lds_sync();
  const uint32_t total = tiles_stage_scan(q, ts);
  uint32_t gb = 0;
  if (lane_id() == 0 && total) gb = atomicAdd(gcnt, total);
  gb = __shfl(gb, 0, 64);
  tiles_stage_write(q, gq, gb, total);
}

// Final tile flush for all waves of the workgroup (workgroup-uniform, two
// barriers): one reservation per workgroup.
__device__ inline void flush_tiles_wg(ItemQ& q, Item* gq, uint32_t* gcnt, TileShape ts, Shared& sh) {
  const uint32_t wave = threadIdx.x >> 6;
  wave_lds_sync();
  const uint32_t total = tiles_stage_scan(q, ts);
  if (lane_id() == 0) sh.part[wave][0] = total;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < Q_WAVES; w++) t += sh.part[w][0];
    sh.part[0][1] = t ? atomicAdd(gcnt, (uint32_t)t) : 0u;
  }
  __syncthreads();
  uint32_t gb = (uint32_t)sh.part[0][1];
#pragma unroll
  for (int w = 0; w < Q_WAVES; w++)
    if ((uint32_t)w < wave) gb += (uint32_t)sh.part[w][0];
  __syncthreads();
  tiles_stage_write(q, gq, gb, total);
}

__device__ inline void flush_u32_q(U32Q& q, uint32_t* gq, uint32_t* gcnt) {
  if (q.n == 0) return;
  wave_lds_sync();
  const uint32_t lane = lane_id();
  uint32_t gb = 0;
  if (lane == 0) gb = atomicAdd(gcnt, q.n);
  gb = __shfl(gb, 0, 64);
  for (uint32_t e = lane; e < q.n; e += 64) gq[gb + e] = q.v[e];
  q.n = 0;
  wave_lds_sync();
}

// Frontier queue: append the staged vertices that have buckets as items,
// reserving items and flat buckets with one atomic, and point every chunk
// that starts inside the reserved flat range at its item.
// Staged items' reservation unit: items (low half) | buckets (high half),
// as a wave-inclusive scan (lane 63 holds the wave total).
__device__ inline unsigned long long front_stage_scan(const ItemQ& q, uint32_t* nb, unsigned long long* x_out) {
  constexpr int PER = WSTAGE / 64;
  const uint32_t lane = lane_id();
  uint32_t ni = 0, nbs = 0;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    uint32_t e = lane * PER + k;
    uint64_t d = e < q.n ? q.d[e] : 0;
    nb[k] = d ? 1u << (d & 63) : 0;
    ni += nb[k] ? 1 : 0;
    nbs += nb[k];
  }
  const unsigned long long x = (unsigned long long)ni | ((unsigned long long)nbs << 32);
  *x_out = x;
  return wave_incl_scan64(x);
}

// Write the wave's staged items at base (items | buckets, already
// reserved) and point every chunk that starts in their buckets at its item.
__device__ inline void front_stage_write(ItemQ& q, const Front& f, QCounters* cnt, unsigned long long base,
                                         unsigned long long total, unsigned long long incl, unsigned long long x,
                                         const uint32_t* nb) {
  constexpr int PER = WSTAGE / 64;
  const uint32_t lane = lane_id();
  const unsigned long long ex = incl - x;
  const uint32_t ib = fq_items(base), bb = fq_buckets(base);
  uint32_t io = fq_items(ex), bo = fq_buckets(ex);
  bool ovf = false;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    if (nb[k]) {
      const uint32_t e = lane * PER + k;
      const uint32_t p = ib + io;
      if (p < f.qcap) f.q[p] = Item{q.d[e], q.v[e], bb + bo};
      else ovf = true;
      q.s[io] = bo;
      io++;
      bo += nb[k];
    }
  }
  wave_lds_sync();
  const uint32_t NI = fq_items(total), B = fq_buckets(total);
  const uint32_t ch = 1u << f.lch;
  const uint32_t c0 = (uint32_t)(((uint64_t)bb + ch - 1) >> f.lch), c1 = (uint32_t)(((uint64_t)bb + B + ch - 1) >> f.lch);
  for (uint32_t c = c0 + lane; c < c1; c += 64) {
    const uint32_t rel = (c << f.lch) - bb;
    uint32_t lo = 0, hi = NI;   // q.s[lo] <= rel < q.s[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (q.s[mid] <= rel) lo = mid;
      else hi = mid;
    }
    if (c < f.ccap) f.cmap[c] = ib + lo;
    else ovf = true;
  }
  if (__ballot(ovf) && lane == 0) atomicOr(&cnt->overflow, OVF_QUEUE);
  q.n = 0;
  wave_lds_sync();
}

__device__ inline void flush_front(ItemQ& q, const Front& f, QCounters* cnt) {
  constexpr int PER = WSTAGE / 64;
  if (q.n == 0) return;   // wave-uniform
  wave_lds_sync();
  uint32_t nb[PER];
  unsigned long long x;
  const unsigned long long incl = front_stage_scan(q, nb, &x);
  const unsigned long long total = __shfl(incl, 63, 64);
  unsigned long long base = 0;
  if (lane_id() == 0 && total) base = atomicAdd(&cnt->fq, total);
  base = __shfl(base, 0, 64);
  front_stage_write(q, f, cnt, base, total, incl, x, nb);
}

// The final flush of a step, for all waves of the workgroup at once
// (workgroup-uniform call, two barriers): one reservation per workgroup
// instead of one per wave, since every reservation is an atomic on the
// same counter word.
__device__ inline void flush_front_wg(ItemQ& q, const Front& f, QCounters* cnt, Shared& sh) {
  constexpr int PER = WSTAGE / 64;
  const uint32_t wave = threadIdx.x >> 6;
  wave_lds_sync();
  uint32_t nb[PER];
  unsigned long long x;
  const unsigned long long incl = front_stage_scan(q, nb, &x);
  const unsigned long long total = __shfl(incl, 63, 64);
  if (lane_id() == 0) sh.part[wave][0] = total;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < Q_WAVES; w++) t += sh.part[w][0];
    sh.part[0][1] = t ? atomicAdd(&cnt->fq, t) : 0ull;
  }
  __syncthreads();
  // waves' items and buckets follow one another in wave order
  unsigned long long base = sh.part[0][1];
#pragma unroll
  for (int w = 0; w < Q_WAVES; w++)
    if ((uint32_t)w < wave) base += sh.part[w][0];
  __syncthreads();
  if (total) front_stage_write(q, f, cnt, base, total, incl, x, nb);
  else q.n = 0;
}

// Keep room for `next` more pushes.
__device__ inline void room_front(ItemQ& q, uint32_t next, const Front& f, QCounters* cnt) {
  if (q.n + next > q.cap) flush_front(q, f, cnt);
}
__device__ inline void room_tiles(ItemQ& q, uint32_t next, Item* gq, uint32_t* gcnt, TileShape ts) {
  if (q.n + next > q.cap) flush_tiles(q, gq, gcnt, ts);
}
__device__ inline void room_u32(U32Q& q, uint32_t next, uint32_t* gq, uint32_t* gcnt) {
  if (q.n + next > q.cap) flush_u32_q(q, gq, gcnt);
}

// Additive counts of one step, spread over N_STRIPES lines: a workgroup
// adds to stripe blockIdx.x mod N_STRIPES instead of the step's counter
// words, so the workgroups of a large grid do not queue on the same
// addresses; the reader sums the stripes into the counters.
constexpr uint32_t N_STRIPES = 16;
struct alignas(128) CountStripe {
  unsigned long long m, arcs;
  uint32_t verts, far;
  uint32_t far_inv;   // DIST_INF - least far distance (0: none), raised by atomicMax
  uint32_t pad[25];
};

// Register counters, summed per workgroup and added with one atomic per
// counter (workgroup-uniform call: it takes a barrier).
struct LaneCounts {
  uint32_t verts = 0;
  unsigned long long m = 0;
  uint32_t arcs = 0;
  uint32_t far = 0;   // SSSP: vertices flagged far
  // to the counters c, or to a stripe when st is set
  __device__ void commit(QCounters* c, Shared& sh, CountStripe* st) {
    if (!st) {
      commit(c, sh);
      return;
    }
    uint32_t v = wave_sum_u32(verts);
    unsigned long long mm = wave_sum_u64(m);
    unsigned long long a = wave_sum_u64(arcs);
    uint32_t f = wave_sum_u32(far);
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0) {
      sh.part[wave][0] = v;
      sh.part[wave][1] = mm;
      sh.part[wave][2] = a;
      sh.part[wave][3] = f;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      CountStripe* x = st + blockIdx.x % N_STRIPES;
      unsigned long long t = 0;
#pragma unroll
      for (int w = 0; w < Q_WAVES; w++) t += sh.part[w][threadIdx.x];
      if (t) {
        if (threadIdx.x == 0) atomicAdd(&x->verts, (uint32_t)t);
        else if (threadIdx.x == 1) atomicAdd(&x->m, t);
        else if (threadIdx.x == 2) atomicAdd(&x->arcs, t);
        else atomicAdd(&x->far, (uint32_t)t);
      }
    }
    __syncthreads();
  }
  __device__ void commit(QCounters* c, Shared& sh) {
    uint32_t v = wave_sum_u32(verts);
    unsigned long long mm = wave_sum_u64(m);
    unsigned long long a = wave_sum_u64(arcs);
    uint32_t f = wave_sum_u32(far);
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0) {
      sh.part[wave][0] = v;
      sh.part[wave][1] = mm;
      sh.part[wave][2] = a;
      sh.part[wave][3] = f;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      unsigned long long t = 0;
#pragma unroll
      for (int w = 0; w < Q_WAVES; w++) t += sh.part[w][threadIdx.x];
      if (t) {
        if (threadIdx.x == 0) atomicAdd(&c->n_verts, (uint32_t)t);
        else if (threadIdx.x == 1) atomicAdd(&c->m_next, t);
        else if (threadIdx.x == 2) atomicAdd(&c->arcs, t);
        else atomicAdd(&c->n_far, (uint32_t)t);
      }
    }
    __syncthreads();
  }
  // Wave-uniform call: add this wave's counts with atomics of lane 0;
  // returns the wave's arc count.
  __device__ unsigned long long commit_wave(QCounters* c) {
    uint32_t v = wave_sum_u32(verts);
    unsigned long long mm = wave_sum_u64(m);
    unsigned long long a = wave_sum_u64(arcs);
    uint32_t f = wave_sum_u32(far);
    if (lane_id() == 0) {
      if (v) atomicAdd(&c->n_verts, v);
      if (mm) atomicAdd(&c->m_next, mm);
      if (a) atomicAdd(&c->arcs, a);
      if (f) atomicAdd(&c->n_far, f);
    }
    verts = 0;
    m = 0;
    arcs = 0;
    far = 0;
    return a;
  }
};

__device__ inline bool bm_test(const uint32_t* bm, uint32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }
__device__ inline void bm_set(uint32_t* bm, uint32_t v) { atomicOr(&bm[v >> 5], 1u << (v & 31)); }

// ------------------------------------------------------------- chunks

// The items touching chunk c of a frontier: lane l holds item cmap[c] + l
// (start = 0xFFFFFFFF past the queue's end).  At most 64 items touch a
// chunk of at most 64 buckets, each item holding at least one bucket.
struct ChunkView {
  uint64_t desc;
  uint32_t v, start;
  uint32_t lo, hi;   // flat range of the chunk
};

// Chunks and items a step may read: a producer that ran out of room has
// flagged OVF_QUEUE, and the query fails; the clamps keep every read inside
// the queue until then.
__device__ inline uint32_t front_chunks(const Front& f, unsigned long long fq) { return min(fq_chunks(fq, f.lch), f.ccap); }
__device__ inline uint32_t front_items(const Front& f, unsigned long long fq) { return min(fq_items(fq), f.qcap); }

__device__ inline ChunkView chunk_view(const Front& f, uint32_t c, uint32_t nitems, uint32_t nbuckets) {
  ChunkView cv;
  const uint32_t i0 = f.cmap[c];
  const uint32_t idx = i0 + lane_id();
  Item it = idx < nitems ? f.q[idx] : Item{0, 0, 0xFFFFFFFFu};
  cv.desc = it.desc;
  cv.v = it.v;
  cv.start = it.aux;
  cv.lo = c << f.lch;
  cv.hi = min(cv.lo + (1u << f.lch), nbuckets);
  return cv;
}

// Does this lane's item start inside the chunk (each item is counted by
// exactly one chunk this way)?
__device__ inline bool starts_here(const ChunkView& cv) { return cv.start >= cv.lo && cv.start < cv.hi; }
// Does this lane's item hold any bucket of the chunk?
__device__ inline bool touches(const ChunkView& cv) { return cv.start < cv.hi; }

// Slot j of the flat positions f0 + 4 grp + k (k < 4) of a chunk (EMPTY
// past its end), with visibility at e resolved from the bucket summaries
// and, where needed, the stamps; item[k] is the lane holding the owner.
struct Pairs4 {
  uint32_t d[4];
  int32_t w[4];
  bool vis[4];
  uint32_t item[4];
};

template <bool WITH_W>
__device__ inline Pairs4 load_pairs(const Pool& p, const ChunkView& cv, uint32_t f0, uint32_t grp, uint32_t j,
                                    uint32_t e, bool fast) {
  Pairs4 r;
  uint4 sm[4];
  uint32_t* bp[4];
  // owner of f0: the last lane whose item starts at or before it (starts
  // increase with the lane); owners of f0 + 1 .. f0 + 15 follow it
  const unsigned long long m0 = __ballot(cv.start <= f0);
  const uint32_t L0 = (uint32_t)__popcll(m0) - 1;
  uint32_t nxt[15];
#pragma unroll
  for (int m = 1; m < 16; m++)
    nxt[m - 1] = L0 + m < 64 ? (uint32_t)__builtin_amdgcn_readlane((int)cv.start, (int)(L0 + m)) : 0xFFFFFFFFu;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t f = f0 + grp * 4 + k;
    uint32_t own = L0;
#pragma unroll
    for (int m = 0; m < 15; m++) own += nxt[m] <= f ? 1u : 0u;
    const uint64_t desc = __shfl(cv.desc, (int)own, 64);
    const uint32_t st = __shfl(cv.start, (int)own, 64);
    r.item[k] = own;
    r.d[k] = EMPTY;
    r.w[k] = 0;
    sm[k] = make_uint4(0xFFFFFFFFu, 0xFFFFu, 0xFFFFFFFFu, 0u);
    bp[k] = p.base;
    if (f < cv.hi) {
      Slab s = slab_of(p, desc);
      const uint32_t b = f - st;
      bp[k] = bucket_ptr(s, b);
      r.d[k] = bp[k][j];
      if (WITH_W) r.w[k] = (int32_t)bp[k][16 + j];
      if (fast) sm[k] = *reinterpret_cast<const uint4*>(&s.sum[SUM_WORDS * b]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    bool v = false;
    if (r.d[k] != EMPTY) {
      v = visible_by_summary(sm[k], fast, j, e, slot_stamp(bp[k], j, p.words));
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
  Front fin;              // current frontier (top-down)
  Front fout;             // next frontier
  Item* qbig;             // bottom-up chunk items of long in-slabs
  const uint32_t* bm_cur;
  uint32_t* bm_next;
  int32_t* dist;
  int32_t next_level;
  QCounters* cnt_out;
  CountStripe* stripes;   // additive counts of cnt_out spread (null: into cnt_out)
};

// Top-down over the chunks of the current frontier (nfq: its fq counter).
__device__ __forceinline__ void td_step(const LevelArgs& a, unsigned long long nfq, uint32_t worker, uint32_t nworkers,
                                        Shared& sh) {
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15, wave = threadIdx.x >> 6;
  const uint32_t gw = worker * Q_WAVES + wave, nw = nworkers * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  LaneCounts lc;
  for (uint32_t c = gw; c < nc; c += nw) {
    const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
    for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
      Pairs4 s4 = load_pairs<false>(a.st.fp, cv, f0, grp, j, a.e, a.fast);
      // each stage issues its loads or atomics for all four arcs before any
      // result is used, so their round trips overlap
      int32_t cur[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        cur[k] = s4.vis[k] ? a.dist[s4.d[k]] : 0;
        lc.arcs += s4.vis[k] ? 1 : 0;
      }
      int32_t prev[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        prev[k] = 0;
        if (s4.vis[k] && cur[k] < 0) prev[k] = atomicCAS(&a.dist[s4.d[k]], -1, a.next_level);
      }
      bool found[4];
      uint64_t yd[4];
      uint32_t used[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        found[k] = s4.vis[k] && cur[k] < 0 && prev[k] == -1;
        yd[k] = 0;
        used[k] = 0;
        if (found[k]) {
          yd[k] = a.st.fdesc[s4.d[k]];
          used[k] = a.st.fused[s4.d[k]];
          bm_set(a.bm_next, s4.d[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; k++) {
        lc.verts += found[k] ? 1 : 0;
        lc.m += used[k];
        room_front(qn, 64, a.fout, a.cnt_out);
        push_item(qn, found[k], s4.d[k], yd[k]);
      }
    }
  }
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  lc.commit(a.cnt_out, sh, a.stripes);
}

// Bottom-up, one unvisited vertex per lane: a one-bucket in-slab (the
// forward slab when undirected) is scanned by the lane itself, stopping at
// the first empty slot or at a parent in the frontier; longer in-slabs
// become chunk items of BU_CHUNK buckets for bu_big_step.
__device__ __forceinline__ void bu_step(const LevelArgs& a, uint32_t worker, uint32_t nworkers, Shared& sh) {
  const TileShape tbig{0, BU_CHUNK};
  const uint32_t V = a.st.V;
  const Pool& ip = a.st.undirected ? a.st.fp : a.st.rp;
  const uint64_t* idesc = a.st.undirected ? a.st.fdesc : a.st.rdesc;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = worker * Q_WAVES + wave, nw = nworkers * Q_WAVES;
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE / 2);
  ItemQ qb = item_q(sh.ws[wave], WSTAGE / 2, WSTAGE / 2);
  LaneCounts lc;
  for (uint32_t base = gw * 64; base < V; base += nw * 64) {
    uint32_t y = base + lane_id();
    bool act = y < V && a.dist[y] < 0;
    uint64_t ydesc_in = act ? idesc[y] : 0;
    Slab s = slab_of(ip, ydesc_in);
    bool found = false;
    if (act && s.nb == 1) {
      const uint4 sm = a.fast ? *reinterpret_cast<const uint4*>(s.sum)
                              : make_uint4(0xFFFFFFFFu, 0xFFFFu, 0xFFFFFFFFu, 0u);
      uint32_t x[BSLOTS];
      load_dsts(s.base, x);
      const int used = first_empty(x);   // used slots are a prefix
      // the frontier bits of eight slots are fetched together, and a second
      // eight only when the first hold no parent; arcs examined are counted
      // in slot order up to the first parent, as a scan that stops there
#pragma unroll
      for (int h = 0; h < BSLOTS; h += 8) {
        if (h >= used || found) break;
        bool vis[8];
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
          const int j = h + i;
          vis[i] = j < used && visible_by_summary(sm, a.fast, j, a.e, slot_stamp(s.base, j, s.words));
          w[i] = vis[i] ? a.bm_cur[x[j] >> 5] : 0u;
        }
        int first = 8;
#pragma unroll
        for (int i = 7; i >= 0; i--)
          if (vis[i] && ((w[i] >> (x[h + i] & 31)) & 1u)) first = i;
#pragma unroll
        for (int i = 0; i < 8; i++) lc.arcs += vis[i] && i <= first ? 1 : 0;
        found = first < 8;
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
    room_front(qn, 64, a.fout, a.cnt_out);
    push_item(qn, found, y, yd);
    room_tiles(qb, 64, a.qbig, &a.cnt_out->n_big, tbig);
    push_item(qb, act && s.nb > 1, y, ydesc_in);
  }
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  flush_tiles_wg(qb, a.qbig, &a.cnt_out->n_big, tbig, sh);
  lc.commit(a.cnt_out, sh, a.stripes);
}

// View of one chunk item for a 16-lane group.
struct ItemView {
  Slab s;
  uint32_t b0, nbk, v;
};

__device__ inline ItemView view_item(const Pool& p, const Item* q, uint32_t idx, uint32_t n, TileShape ts) {
  ItemView iv;
  bool act = idx < n;
  Item it = act ? q[idx] : Item{0, 0, 0};
  iv.s = slab_of(p, it.desc);
  iv.b0 = ts.first + it.aux * ts.chunk;
  iv.nbk = act && iv.s.nb > iv.b0 ? min(ts.chunk, iv.s.nb - iv.b0) : 0;
  iv.v = it.v;
  return iv;
}

// Chunk items of multi-bucket in-slabs: 16 lanes per chunk; a chunk whose
// vertex already has a parent is skipped, and the first finder claims it.
__device__ __forceinline__ void bu_big_step(const LevelArgs& a, uint32_t nbig, uint32_t worker, uint32_t nworkers,
                                   Shared& sh) {
  const TileShape tbig{0, BU_CHUNK};
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15, wave = threadIdx.x >> 6;
  const uint32_t gw = worker * Q_WAVES + wave, nw = nworkers * Q_WAVES;
  const Pool& ip = a.st.undirected ? a.st.fp : a.st.rp;
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  LaneCounts lc;
  for (uint32_t base = gw * 4; base < nbig; base += nw * 4) {
    ItemView iv = view_item(ip, a.qbig, base + grp, nbig, tbig);
    uint32_t y = iv.v;
    if (iv.nbk && a.dist[y] >= 0) iv.nbk = 0;
    uint32_t maxnb = wave_max_u32(iv.nbk);
    bool found = false;
    for (uint32_t i = 0; i < maxnb; i += 4) {
      bool hit = false;
      uint32_t d[4];
      uint32_t* bp[4];
      uint4 sm[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        d[k] = EMPTY;
        bp[k] = iv.s.base;
        sm[k] = make_uint4(0xFFFFFFFFu, 0xFFFFu, 0xFFFFFFFFu, 0u);
        if (!found && i + k < iv.nbk) {
          const uint32_t b = iv.b0 + i + k;
          bp[k] = bucket_ptr(iv.s, b);
          d[k] = bp[k][j];
          if (a.fast) sm[k] = *reinterpret_cast<const uint4*>(&iv.s.sum[SUM_WORDS * b]);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if (d[k] == EMPTY) continue;
        bool vis = visible_by_summary(sm[k], a.fast, j, a.e, slot_stamp(bp[k], j, iv.s.words));
        if (vis) {
          lc.arcs++;
          hit |= bm_test(a.bm_cur, d[k]);
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
    room_front(qn, 4, a.fout, a.cnt_out);
    push_item(qn, win, y, yd);
  }
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  lc.commit(a.cnt_out, sh, a.stripes);
}

// ----------------------------------------------------------------- SSSP

// The far set of delta-stepping is the bitmap infar, one bit per vertex (no
// list): a relax that improves a vertex to a distance at or above the
// threshold sets its bit, and a split scans the bitmap densely, reading the
// distances of flagged vertices only and moving those below the new
// threshold into the near frontier.  A split then costs one streaming pass
// over V / 8 bytes, whatever the number of far vertices, instead of a
// random read per far entry; a flag word per vertex had cost 4 bytes per
// vertex in every split and a line per flag test in the relax.
__device__ inline uint32_t far_bit(uint32_t v) { return 1u << (v & 31); }
struct RelaxArgs {
  Store st;
  uint32_t e;
  int fast;
  Front fin;
  Front fout;
  int32_t* dist;
  uint32_t* stamp;     // iteration stamp of the last push into the near queue
  uint32_t* infar;     // far bitmap (new flags are counted in cnt_out->n_far)
  int32_t thr;
  uint32_t it1;        // stamp value of the queue being filled
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
  CountStripe* stripes;   // additive counts of cnt_out spread (null: into cnt_out)
};

// One chunk of the near frontier (all lanes of the wave).
__device__ __forceinline__ void relax_chunk(const RelaxArgs& a, uint32_t c, uint32_t nitems, uint32_t nb, ItemQ& qn,
                                            LaneCounts& lc) {
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
  const int32_t du_l =
      touches(cv) ? __hip_atomic_load(&a.dist[cv.v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  if (a.mode == 1) {
    // the chunk holding a vertex's first bucket records it for the
    // bucket's heavy pass
    bool rec = starts_here(cv) && atomicExch(&a.rstamp[cv.v], a.phase) != a.phase;
    uint32_t pos = wave_reserve(a.rcount, rec ? 1u : 0u);
    if (rec) a.rlist[pos] = cv.v;
  }
  for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
    Pairs4 s4 = load_pairs<true>(a.st.fp, cv, f0, grp, j, a.e, a.fast);
    // Each stage below issues its loads or atomics for all four arcs before
    // any result is used, so their round trips overlap.  The targets'
    // distances are read first; distances only fall, so an early read is
    // an upper bound and the atomicMin decides.
    bool take[4];
    int32_t nd[4], cur[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      take[k] = s4.vis[k] && (a.mode == 0 || ((a.mode == 1) == (s4.w[k] <= a.light)));
      cur[k] = take[k] ? a.dist[s4.d[k]] : 0;
      nd[k] = __shfl(du_l, (int)s4.item[k], 64) + s4.w[k];
      lc.arcs += take[k] ? 1 : 0;
    }
    // The atomicMin's result is not waited for: an arc whose tentative
    // distance beats the read value counts as an improvement even when a
    // racing arc lowered the target further in between.  That arc pushes or
    // flags the target too, so the push below at worst repeats one the
    // target needs anyway (the stamp keeps one queue entry per pass) or
    // raises a far flag that a later split finds already below its
    // threshold.  Distances only fall, so every result stays exact.
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (take[k] && nd[k] < cur[k]) atomicMin(&a.dist[s4.d[k]], nd[k]);
    // an improvement below the threshold claims the target's place in the
    // next near frontier (once per pass); one at or above it raises the
    // target's far flag
    uint32_t prev[4], fl[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      prev[k] = 0u;
      fl[k] = 0u;
      if (take[k] && nd[k] < cur[k]) {
        if (nd[k] < a.thr) {
          prev[k] = atomicExch(&a.stamp[s4.d[k]], a.it1);
          fl[k] = a.infar[s4.d[k] >> 5] & far_bit(s4.d[k]);
        } else {
          prev[k] = atomicOr(&a.infar[s4.d[k] >> 5], far_bit(s4.d[k])) & far_bit(s4.d[k]);
        }
      }
    }
    bool to_near[4];
    uint64_t yd[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const bool imp = take[k] && nd[k] < cur[k];
      to_near[k] = imp && nd[k] < a.thr && prev[k] != a.it1;
      // settled in this bucket: no later split needs to move it again
      if (imp && nd[k] < a.thr && fl[k]) atomicAnd(&a.infar[s4.d[k] >> 5], ~far_bit(s4.d[k]));
      if (imp && nd[k] >= a.thr && prev[k] == 0u) lc.far++;
      yd[k] = to_near[k] ? a.st.fdesc[s4.d[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      lc.verts += to_near[k] ? 1 : 0;
      room_front(qn, 64, a.fout, a.cnt_out);
      push_item(qn, to_near[k], s4.d[k], yd[k]);
    }
  }
}

__device__ __forceinline__ void relax_step(const RelaxArgs& a, unsigned long long nfq, uint32_t worker,
                                           uint32_t nworkers, Shared& sh) {
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = worker * Q_WAVES + wave, nw = nworkers * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  LaneCounts lc;
  for (uint32_t c = gw; c < nc; c += nw) relax_chunk(a, c, nitems, nb, qn, lc);
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  lc.commit(a.cnt_out, sh, a.stripes);
}

// Items of every vertex in list[0..n): the recorded vertices of a settled
// bucket, for its heavy-arc pass.  One block of 64 entries per call.
__device__ __forceinline__ void expand_block(const Store& st, const uint32_t* list, uint32_t n, uint32_t base,
                                             const Front& fout, QCounters* cnt_out, ItemQ& qn) {
  uint32_t i = base + lane_id();
  bool act = i < n;
  uint32_t v = act ? list[i] : 0;
  uint64_t vd = act ? st.fdesc[v] : 0;
  room_front(qn, 64, fout, cnt_out);
  push_item(qn, act && vd != 0, v, vd);
}

__device__ __forceinline__ void expand_step(const Store& st, const uint32_t* list, uint32_t n, const Front& fout,
                                            QCounters* cnt_out, uint32_t worker, uint32_t nworkers, Shared& sh) {
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = worker * Q_WAVES + wave, nw = nworkers * Q_WAVES;
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  for (uint32_t base = gw * 64; base < n; base += nw * 64) expand_block(st, list, n, base, fout, cnt_out, qn);
  flush_front(qn, fout, cnt_out);
}

struct SplitArgs {
  Store st;
  Front fout;
  int32_t* dist;
  uint32_t* stamp;
  uint32_t* infar;
  int32_t thr;
  uint32_t it1;
  QCounters* cnt_out;   // near items; n_far = far vertices left; far_min
  CountStripe* stripes;   // additive counts of cnt_out spread (null: into cnt_out)
};

// Vertices [base, base + 64): flagged ones below the threshold move into the
// near queue; the rest stay flagged, counted, with their minimum distance.
__device__ __forceinline__ void split_block(const SplitArgs& a, uint32_t base, ItemQ& qn, LaneCounts& lc,
                                            int32_t& mn) {
  // base is a multiple of 64: lanes 0-31 and 32-63 share one flag word
  // each, and no other wave touches either (no relax runs beside a split)
  const uint32_t v = base + lane_id();
  const uint32_t w = v < a.st.V ? a.infar[v >> 5] : 0u;
  const bool flagged = (w & far_bit(v)) != 0u;
  const int32_t dv = flagged ? a.dist[v] : DIST_INF;
  bool near = flagged && dv < a.thr;
  const unsigned long long moved = __ballot(near);
  if ((lane_id() & 31) == 0 && v < a.st.V) {
    const uint32_t m = (uint32_t)(moved >> (lane_id() & 32));
    if (m) a.infar[v >> 5] = w & ~m;
  }
  if (near) {
    near = atomicExch(&a.stamp[v], a.it1) != a.it1;
  } else if (flagged) {
    mn = min(mn, dv);
    lc.far++;
  }
  uint64_t vd = near ? a.st.fdesc[v] : 0;
  lc.verts += near ? 1 : 0;
  room_front(qn, 64, a.fout, a.cnt_out);
  push_item(qn, near, v, vd);
}

// The far minimum reaches the counters once per wave.
__device__ inline void commit_far_min(int32_t mn, QCounters* c) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mn = min(mn, (int32_t)__shfl_xor(mn, o, 64));
  if (lane_id() == 0 && mn < DIST_INF) atomicMin(&c->far_min, mn);
}

// The far minimum of a workgroup (workgroup-uniform call, one barrier)
// reaches its count stripe with one atomic: a split's waves had each put an
// atomicMin on the one far_min word, about ten thousand at R-MAT 20.
__device__ inline void commit_far_min_striped(int32_t mn, CountStripe* st) {
  __shared__ int32_t wmin[Q_WAVES];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mn = min(mn, (int32_t)__shfl_xor(mn, o, 64));
  if (lane_id() == 0) wmin[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t m = DIST_INF;
#pragma unroll
    for (int w = 0; w < Q_WAVES; w++) m = min(m, wmin[w]);
    if (m < DIST_INF) atomicMax(&st[blockIdx.x % N_STRIPES].far_inv, (uint32_t)(DIST_INF - m));
  }
}

__device__ __forceinline__ void split_step(const SplitArgs& a, uint32_t worker, uint32_t nworkers, Shared& sh) {
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = worker * Q_WAVES + wave, nw = nworkers * Q_WAVES;
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  LaneCounts lc;
  int32_t mn = DIST_INF;
  for (uint32_t base = gw * 64; base < a.st.V; base += nw * 64) split_block(a, base, qn, lc, mn);
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  if (a.stripes) commit_far_min_striped(mn, a.stripes);
  else commit_far_min(mn, a.cnt_out);
  lc.commit(a.cnt_out, sh, a.stripes);
}

// ------------------------------------------------------------------- BC

// The BC backward sums a slab of more than BWD_TILE buckets as tiles (see
// bcbwd_step below); the forward counts such vertices per level.
constexpr uint32_t BWD_TILE = 32;        // buckets per tile (slabs hold 2^k buckets)
constexpr uint32_t BWD_TILE_LOG = 5;
__host__ __device__ inline bool bwd_is_big(uint64_t desc) { return desc != 0 && (desc & 63) > BWD_TILE_LOG; }

struct BcFwdArgs {
  Store st;
  uint32_t e;
  int fast;
  Front fin;
  Front fout;
  uint32_t* order;      // vertices in discovery order
  int32_t* level;
  unsigned long long* sigma;
  int32_t next_level;
  QCounters* cnt_out;
  QCounters* cnt_total; // discovery-order length and the overflow flag
};

__device__ __forceinline__ void bcfwd_step(const BcFwdArgs& a, unsigned long long nfq, uint32_t worker,
                                           uint32_t nworkers, Shared& sh) {
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15, wave = threadIdx.x >> 6;
  const uint32_t gw = worker * Q_WAVES + wave, nw = nworkers * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  U32Q qo = u32_q(sh.ws[wave]);
  LaneCounts lc;
  uint32_t ovf = 0;
  for (uint32_t c = gw; c < nc; c += nw) {
    const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
    const unsigned long long su_l = touches(cv) ? a.sigma[cv.v] : 0;
    for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
      Pairs4 s4 = load_pairs<false>(a.st.fp, cv, f0, grp, j, a.e, a.fast);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const unsigned long long su = __shfl(su_l, (int)s4.item[k], 64);
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
        lc.far += bwd_is_big(yd) ? 1 : 0;   // slabs the backward splits into tiles
        room_front(qn, 64, a.fout, a.cnt_out);
        push_item(qn, found, d, yd);
        room_u32(qo, 64, a.order, &a.cnt_total->n_order);
        push_u32(qo, found, d);
      }
    }
  }
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  flush_u32_q(qo, a.order, &a.cnt_total->n_order);
  if (ovf) atomicOr(&a.cnt_total->overflow, OVF_SIGMA);
  lc.commit(a.cnt_out, sh);
}

// ------------------------------------------------- multi-source BFS
//
// Up to 64 BFS queries on one snapshot share every adjacency scan: vertex v
// keeps a 64-bit mask of the queries that have reached it (vis), of those
// whose frontier it is in at the current level (fr), and of those that reach
// it in the current level (nxt).  Expanding a frontier vertex u ORs
// fr[u] & ~vis[v] into nxt[v] for each visible arc (u, v); the first
// contribution to nxt[v] lists v as touched and queues its slab for the
// next level.  Finalising a touched v then moves the new bits into vis and
// fr and writes the level into the distance array of each new query.

struct MsArgs {
  Store st;
  uint32_t e;
  int fast;
  Front fin;                      // vertices with a nonzero frontier mask
  Front fout;                     // touched vertices that have an out-slab
  const unsigned long long* fr;
  // per vertex one 16-byte record {visited mask, next-level mask}, so an
  // arc's target costs one line
  unsigned long long* vn;
  uint32_t* touched;              // all touched vertices (count in cnt_out->n_far)
  QCounters* cnt_out;
};

__device__ __forceinline__ void msbfs_chunk(const MsArgs& a, uint32_t c, uint32_t nitems, uint32_t nb, ItemQ& qn,
                                            U32Q& qt, LaneCounts& lc) {
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
  const unsigned long long f_l = touches(cv) ? a.fr[cv.v] : 0ull;
  for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
    Pairs4 s4 = load_pairs<false>(a.st.fp, cv, f0, grp, j, a.e, a.fast);
    // each stage issues its loads or atomics for all four arcs before any
    // result is used, so their round trips overlap
    unsigned long long want[4], have[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const unsigned long long fm = __shfl(f_l, (int)s4.item[k], 64);   // all lanes take part
      want[k] = 0ull;
      have[k] = 0ull;
      if (s4.vis[k]) {
        // next-level masks only gain bits within a level, so a stale copy
        // is a subset and at most costs an atomicOr that adds nothing
        const ulonglong2 r = *reinterpret_cast<const ulonglong2*>(&a.vn[2 * (uint64_t)s4.d[k]]);
        want[k] = fm & ~r.x;
        have[k] = r.y;
      }
      lc.arcs += s4.vis[k] ? 1 : 0;
    }
    unsigned long long before[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      before[k] = 1ull;
      if (want[k] & ~have[k]) before[k] = atomicOr(&a.vn[2 * (uint64_t)s4.d[k] + 1], want[k]);
    }
    bool first[4];
    uint64_t yd[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      first[k] = before[k] == 0ull;
      yd[k] = first[k] ? a.st.fdesc[s4.d[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      room_front(qn, 64, a.fout, a.cnt_out);
      push_item(qn, first[k], s4.d[k], yd[k]);
      room_u32(qt, 64, a.touched, &a.cnt_out->n_far);
      push_u32(qt, first[k], s4.d[k]);
    }
  }
}

// ------------------------------------------------- BC backward tiles
//
// The dependency of v at level L (Brandes' backward recurrence):
//   delta[v] = sum over visible arcs v->w with level[w] = L+1 of
//              sigma[v]/sigma[w] * (1 + delta[w])
//            = sigma[v] * (sum of coef[w]),  coef[w] = (1 + delta[w]) / sigma[w].
// A finished vertex stores coef (one division per vertex, not per arc), so
// a pull reads one value per arc.  The sum's order is fixed by the slab
// layout alone: the slab is cut
// into tiles of BWD_TILE buckets; in tile t, lane l adds the matching slots
// l % 16 of buckets t BWD_TILE + l / 16 + 4i in increasing i, the 64 lane
// sums combine by a fixed butterfly, and the tile sums add in tile order.
// A slab of at most BWD_TILE buckets is one tile, summed by the wave that
// takes the vertex; a longer one (a hub) is listed for a tile pass, one
// wave per tile, and a combine pass adds its tile sums.  The plain, team
// and multi-source searches all follow this order, so their dependencies
// agree bit for bit.

// Vertex v owns tiles [base, base + n) of the slab desc it was listed with
// (tiles read that slab even if an update has since moved v's arcs to a
// larger one: slabs are never reused while a search can hold them).
struct BigVert {
  uint64_t desc;
  uint32_t v, base, n, pad;
};
// Counts of the listed vertices and their tiles, by level parity (a level
// fills one parity while its pass zeroes the other's), and an overflow flag.
struct BwdHead {
  uint32_t verts[2], tiles[2];
  uint32_t ovf, pad[3];
};
struct BwdTiles {
  BwdHead* head;
  BigVert* big;
  uint32_t* tmap;     // tile -> index into big
  double* part;       // tile sums (per tile: `per` doubles)
  uint32_t cap_verts, cap_tiles;
};


// Capacities from the pool's bucket count: a listed slab holds at least
// 2 BWD_TILE buckets, and the slabs of one level are distinct, so one
// level lists at most cap / BWD_TILE tiles and cap / (2 BWD_TILE) vertices.
__host__ __device__ inline uint64_t bwd_cap_tiles(uint64_t pool_buckets) { return pool_buckets / BWD_TILE + 1; }
__host__ __device__ inline uint64_t bwd_cap_verts(uint64_t pool_buckets) { return pool_buckets / (2 * BWD_TILE) + 1; }
__host__ __device__ inline uint64_t bwd_al(uint64_t x) { return (x + 255) & ~255ull; }
__host__ __device__ inline uint64_t bwd_tiles_bytes(uint64_t pool_buckets, uint32_t per) {
  return bwd_al(sizeof(BwdHead)) + bwd_al(bwd_cap_verts(pool_buckets) * sizeof(BigVert)) +
         bwd_al(bwd_cap_tiles(pool_buckets) * 4) + bwd_al(bwd_cap_tiles(pool_buckets) * 8 * (uint64_t)per);
}
__host__ __device__ inline BwdTiles bwd_tiles_at(char* p, uint64_t pool_buckets, uint32_t per) {
  BwdTiles t;
  const uint64_t cv = bwd_cap_verts(pool_buckets), ct = bwd_cap_tiles(pool_buckets);
  t.head = reinterpret_cast<BwdHead*>(p);
  p += bwd_al(sizeof(BwdHead));
  t.big = reinterpret_cast<BigVert*>(p);
  p += bwd_al(cv * sizeof(BigVert));
  t.tmap = reinterpret_cast<uint32_t*>(p);
  p += bwd_al(ct * 4);
  t.part = reinterpret_cast<double*>(p);
  t.cap_verts = (uint32_t)(cv < 0xFFFFFFFFull ? cv : 0xFFFFFFFFull);
  t.cap_tiles = (uint32_t)(ct < 0xFFFFFFFFull ? ct : 0xFFFFFFFFull);
  return t;
}

// Wave-uniform: list vertex v (slab desc of more than BWD_TILE buckets) for
// the tile pass of its level (parity par); a full list raises the overflow
// flag.
__device__ inline void bwd_list(const BwdTiles& t, uint32_t par, uint32_t v, uint64_t desc) {
  const uint32_t n = (1u << (desc & 63)) >> BWD_TILE_LOG;
  uint32_t idx = 0, base = 0;
  if (lane_id() == 0) {
    idx = atomicAdd(&t.head->verts[par], 1u);
    base = atomicAdd(&t.head->tiles[par], n);
  }
  idx = uni(idx);
  base = uni(base);
  if (idx >= t.cap_verts || base >= t.cap_tiles || n > t.cap_tiles - base) {
    if (lane_id() == 0) atomicOr(&t.head->ovf, 1u);
    return;
  }
  if (lane_id() == 0) t.big[idx] = BigVert{desc, v, base, n, 0};
  for (uint32_t i = lane_id(); i < n; i += 64) t.tmap[base + i] = idx;
}

// The wave's sum of coef[w] over tile [b0, b1) of v's slab (combined over
// lanes).
__device__ __forceinline__ double bwd_tile_sum(const Slab& s, uint32_t b0, uint32_t b1, uint32_t e, bool fast,
                                               const int32_t* level, int32_t L, const double* coef) {
  const uint32_t lane = lane_id(), j = lane & 15;
  double acc = 0.0;
  for (uint32_t b = b0 + (lane >> 4); b < b1; b += 4) {
    uint32_t* bp = bucket_ptr(s, b);
    uint32_t w = bp[j];
    if (w != EMPTY && slot_visible(s, bp, b, j, e, fast) && level[w] == L + 1) acc += coef[w];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  return acc;
}

// v's dependency from its sum of coefficients: added to bc (v not the
// source), and v's own coefficient stored for the level above.  Every
// operation rounds on its own (no fused multiply-add), as in the
// multi-source form, which stores the dependency before adding it.
__device__ inline void bwd_finish(uint32_t v, double sum, uint32_t src, const unsigned long long* sigma, double* coef,
                                  double* bc) {
#pragma clang fp contract(off)
  const double sv = (double)sigma[v];
  const double d = sv * sum;
  if (v != src) bc[v] += d;
  coef[v] = (1.0 + d) / sv;
}

// One wave per vertex of level L's list verts[0..nv): slabs of one tile
// are summed here; longer slabs are listed for bcbwd_tiles.  Worker 0
// zeroes the other parity's counts for the next level.
__device__ __forceinline__ void bcbwd_step(const Store& st, uint32_t e, bool fast, const uint32_t* verts, uint32_t nv,
                                           uint32_t src, const int32_t* level, int32_t L,
                                           const unsigned long long* sigma, double* coef, double* bc,
                                           const BwdTiles& bt, uint32_t worker, uint32_t nworkers) {
  const uint32_t lane = lane_id();
  const uint32_t par = (uint32_t)L & 1u;
  if (worker == 0 && threadIdx.x == 0) {
    bt.head->verts[par ^ 1] = 0;
    bt.head->tiles[par ^ 1] = 0;
  }
  const uint32_t gwave = worker * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = nworkers * Q_WAVES;
  for (uint32_t k = gwave; k < nv; k += nwaves) {
    const uint32_t v = verts[k];
    const uint64_t desc = st.fdesc[v];
    const Slab s = slab_of(st.fp, desc);
    if (bwd_is_big(desc)) {
      bwd_list(bt, par, v, desc);
      continue;
    }
    const double acc = bwd_tile_sum(s, 0, s.nb, e, fast, level, L, coef);
    if (lane == 0) bwd_finish(v, acc, src, sigma, coef, bc);
  }
}

// One wave per listed tile of level L: its sum into part[tile].
__device__ __forceinline__ void bcbwd_tiles(const Store& st, uint32_t e, bool fast, const int32_t* level, int32_t L,
                                            const double* coef, const BwdTiles& bt, uint32_t nt, uint32_t worker,
                                            uint32_t nworkers) {
  const uint32_t gwave = worker * Q_WAVES + (threadIdx.x >> 6);
  const uint32_t nwaves = nworkers * Q_WAVES;
  nt = min(nt, bt.cap_tiles);
  for (uint32_t t = gwave; t < nt; t += nwaves) {
    const uint32_t i = bt.tmap[t];
    if (i >= bt.cap_verts) continue;
    const BigVert bv = bt.big[i];
    if (t < bv.base || t - bv.base >= bv.n) continue;
    const Slab s = slab_of(st.fp, bv.desc);
    const uint32_t b0 = (t - bv.base) << BWD_TILE_LOG;
    if (b0 >= s.nb) continue;
    const double acc = bwd_tile_sum(s, b0, min(s.nb, b0 + BWD_TILE), e, fast, level, L, coef);
    if (lane_id() == 0) bt.part[t] = acc;
  }
}

// One lane per listed vertex of level L: its tile sums added in tile order.
__device__ __forceinline__ void bcbwd_combine(const BwdTiles& bt, uint32_t nbig, uint32_t src,
                                              const unsigned long long* sigma, double* coef, double* bc,
                                              uint32_t worker, uint32_t nworkers) {
  nbig = min(nbig, bt.cap_verts);
  for (uint32_t i = worker * Q_THREADS + threadIdx.x; i < nbig; i += nworkers * Q_THREADS) {
    const BigVert bv = bt.big[i];
    if (bv.n == 0 || bv.base >= bt.cap_tiles || bv.n > bt.cap_tiles - bv.base) continue;
    double acc = bt.part[bv.base];
    for (uint32_t t = 1; t < bv.n; t++) acc += bt.part[bv.base + t];
    bwd_finish(bv.v, acc, src, sigma, coef, bc);
  }
}

}  // namespace dg
