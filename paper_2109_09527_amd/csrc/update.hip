// Batched update: one batch of ADT ops (AddVertex / RemoveVertex /
// ContainsVertex / AddEdge / RemoveEdge / ContainsEdge) applied as if
// linearized in index order, published as one new epoch E' = e + 1.
//
//   k_upd_init        zero the batch counters, snapshot the pool cursors
//   k_prep            validate every op; sort key = [edge:1][a:L][b:L]
//                     (vertex op: a = vertex, b = 0; edge op: (u,v), or
//                     {min,max} when undirected); value = op index
//   radix sort        stable, so each key's ops stay in index order
//   k_resolve_vertex  one thread per vertex-key segment walks its ops in
//                     order: result of each op, liveness after it, index of
//                     the last successful RemoveVertex so far
//   k_resolve_edge    one thread per edge-key segment: state at e from one
//                     probe of the store, then each op in order, with the
//                     endpoints' liveness at that index from a binary search
//                     of the vertex timelines and the edge cleared whenever a
//                     successful RemoveVertex of an endpoint lies between two
//                     state points; net effect per key = tombstone the
//                     current version and/or insert a new one
//   k_grow_*          slabs that would pass 75% load get a new slab at <=50%
//                     load; versions dead at or below the oldest queryable
//                     epoch are dropped while rehashing.  plan lists the
//                     growing slabs; alloc reserves their new slabs; init
//                     and move spread each slab's words and slots over
//                     several workgroups (hubs included); publish swaps
//                     the descriptors
//   k_clear           successful RemoveVertex of a vertex live at e:
//                     tombstone every current arc at it and its mirror
//   k_commit_edge     per key: tombstone (death = E') and/or insert
//                     (birth = E'), mirrored into the reverse slab
//   k_commit_vertex   liveness of vertices whose state changed
// Every kernel after k_prep returns at once when the batch was rejected;
// the commit kernels also when the growth step ran out of pool space, so
// a rejected batch leaves the store untouched.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dg_host.h"

namespace dg {

constexpr int UPD_THREADS = 256;

__global__ void k_upd_init(UpdCounters* c, const unsigned long long* cursor) {
  if (threadIdx.x == 0) {
    UpdCounters z{};
    z.cursor0_f = cursor[0];
    z.cursor0_r = cursor[1];
    *c = z;
  }
}

__global__ __launch_bounds__(UPD_THREADS) void k_prep(const dg_op* ops, uint32_t n, uint32_t V, int und,
                                                       int32_t wmax, uint32_t L, uint64_t* keys,
                                                       uint32_t* vals, UpdCounters* c) {
  uint32_t i = blockIdx.x * UPD_THREADS + threadIdx.x;
  uint32_t flags = 0;
  bool isv = false;
  if (i < n) {
    dg_op op = ops[i];
    bool edge = op.type >= DG_ADD_EDGE;
    if (op.type > DG_CONTAINS_EDGE) flags |= F_BAD_TYPE;
    if (op.u >= V || (edge && op.v >= V)) flags |= F_BAD_VERTEX;
    if (op.type == DG_ADD_EDGE && (op.w < 1 || op.w > wmax)) flags |= F_BAD_WEIGHT;
    uint64_t a = op.u, b = edge ? op.v : 0;
    if (edge && und && a > b) {
      uint64_t t = a;
      a = b;
      b = t;
    }
    uint64_t mask = (1ull << L) - 1;
    keys[i] = ((uint64_t)(edge ? 1 : 0) << (2 * L)) | ((a & mask) << L) | (b & mask);
    vals[i] = i;
    isv = !edge;
  }
  unsigned long long m = __ballot(isv);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) flags |= __shfl_xor(flags, o, 64);
  if (lane_id() == 0) {
    if (m) atomicAdd(&c->nv, (uint32_t)__popcll(m));
    if (flags) atomicOr(&c->flags, flags);
  }
}

struct VState {
  uint8_t alive;
  uint32_t lastrem;   // index of the last successful RemoveVertex, or NONE
};

// Filter of the vertices that have ops in the batch: one bit per hash of a
// vertex in LDS, so an edge op on a vertex without vertex ops (nearly all of
// them) takes its liveness from the store instead of a binary search of the
// vertex ops, whose ten or more dependent loads dominated edge resolution.
constexpr uint32_t VF_WORDS = 2048;          // 64 Kbit
constexpr uint32_t VF_MAX_VERTS = 16384;     // larger vertex parts search every time
__device__ inline uint32_t vf_hash(uint32_t x) { return (x * 0x9E3779B1u) >> 16; }
__device__ inline bool vf_maybe(const uint32_t* vf, uint32_t x) {
  if (!vf) return true;
  const uint32_t h = vf_hash(x);
  return (vf[h >> 5] >> (h & 31)) & 1u;
}

// State of vertex x just before op index i: the last vertex op on x with a
// smaller index (sorted part [0, nv) is ordered by (vertex, index)).
// alive_x: x's liveness at e (st.alive[x], loaded by the caller).
__device__ inline VState vstate(const uint64_t* keys, const uint32_t* vals, uint32_t nv, uint32_t L, uint32_t x,
                                uint32_t i, uint8_t alive_x, const uint8_t* vafter, const uint32_t* vlastrem,
                                const uint32_t* vf) {
  if (!vf_maybe(vf, x)) return VState{alive_x, NONE};
  uint32_t lo = 0, hi = nv;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    uint32_t vx = (uint32_t)(keys[mid] >> L);
    if (vx < x || (vx == x && vals[mid] < i)) lo = mid + 1;
    else hi = mid;
  }
  if (lo > 0 && (uint32_t)(keys[lo - 1] >> L) == x) return VState{vafter[lo - 1], vlastrem[lo - 1]};
  return VState{alive_x, NONE};
}

__global__ __launch_bounds__(UPD_THREADS) void k_resolve_vertex(const uint64_t* keys, const uint32_t* vals,
                                                                 const dg_op* ops, uint32_t n, uint32_t L,
                                                                 const uint8_t* alive, uint8_t* results,
                                                                 uint8_t* vafter, uint32_t* vlastrem,
                                                                 uint32_t* clear_list, uint32_t* vchange,
                                                                 UpdCounters* c) {
  if (c->flags) return;
  uint32_t nv = c->nv;
  uint32_t k = blockIdx.x * UPD_THREADS + threadIdx.x;
  if (k >= nv) return;
  uint32_t x = (uint32_t)(keys[k] >> L);
  if (k > 0 && (uint32_t)(keys[k - 1] >> L) == x) return;
  uint8_t init = alive[x], state = init;
  uint32_t lastrem = NONE;
  for (uint32_t j = k; j < nv && (uint32_t)(keys[j] >> L) == x; j++) {
    uint32_t i = vals[j];
    uint32_t t = ops[i].type;
    uint8_t r;
    if (t == DG_ADD_VERTEX) {
      r = state ? 0 : 1;
      state = 1;
    } else if (t == DG_REMOVE_VERTEX) {
      r = state;
      if (state) lastrem = i;
      state = 0;
    } else {
      r = state;
    }
    results[i] = r;
    vafter[j] = state;
    vlastrem[j] = lastrem;
  }
  if (init && lastrem != NONE) clear_list[atomicAdd(&c->n_clear, 1u)] = x;
  if (state != init) vchange[atomicAdd(&c->n_vchange, 1u)] = x | ((uint32_t)state << 31);
}

// Append x to list for every lane with `want`, with one atomicAdd per wave
// on the list's count.  Any subset of the wave's lanes may be active.
__device__ inline void wave_append(uint32_t* list, uint32_t* count, bool want, uint32_t x) {
  const unsigned long long m = __ballot(want);
  if (!m) return;
  const int lead = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == lead) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = __shfl(base, lead, 64);
  if (want) list[base + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull))] = x;
}

// One edge-key segment starting at k: each op's result in index order, and
// the net effect on the store recorded for the commit (recflags: 1 =
// tombstone the version present at e, 2 = insert a new one; recw: its
// weight).  Returns whether the key inserts.
__device__ __forceinline__ bool resolve_key(const uint64_t* keys, const uint32_t* vals, const dg_op* ops, uint32_t n,
                                            uint32_t nv, uint32_t L, const Store& st, uint8_t* results,
                                            const uint8_t* vafter, const uint32_t* vlastrem, const uint32_t* vf,
                                            uint32_t k, uint64_t key, uint8_t* recflags, int32_t* recw,
                                            uint32_t* a_out, uint32_t* b_out) {
  const uint64_t mask = (1ull << L) - 1;
  const uint32_t a = (uint32_t)((key >> L) & mask), b = (uint32_t)(key & mask);
  *a_out = a;
  *b_out = b;
  // loads that do not depend on the store probe go out first
  const dg_op op0 = ops[vals[k]];
  const uint8_t alive_a = st.alive[a], alive_b = st.alive[b];
  Slab sa = slab_of(st.fp, st.fdesc[a]);
  SlotRef ref = find_current(sa, b);
  bool present0 = ref.bp != nullptr;
  int32_t w0 = present0 ? (int32_t)*slot_w(ref.bp, ref.j) : 0;
  bool present = present0;
  int32_t w = w0;
  int64_t last_pt = -1;
  for (uint32_t j = k; j < n && keys[j] == key; j++) {
    uint32_t i = vals[j];
    dg_op op = j == k ? op0 : ops[i];
    VState sa_ = vstate(keys, vals, nv, L, a, i, alive_a, vafter, vlastrem, vf);
    VState sb_ = vstate(keys, vals, nv, L, b, i, alive_b, vafter, vlastrem, vf);
    int64_t tc = -1;
    if (sa_.lastrem != NONE) tc = sa_.lastrem;
    if (sb_.lastrem != NONE && (int64_t)sb_.lastrem > tc) tc = sb_.lastrem;
    if (tc > last_pt) present = false;   // an endpoint was removed since the last state point
    uint8_t r;
    if (!sa_.alive || !sb_.alive) {
      r = 2;
    } else if (op.type == DG_ADD_EDGE) {
      if (present) r = 0;
      else {
        present = true;
        w = op.w;
        r = 1;
      }
    } else if (op.type == DG_REMOVE_EDGE) {
      r = present ? 1 : 0;
      present = false;
    } else {
      r = present ? 1 : 0;
    }
    results[i] = r;
    last_pt = i;
  }
  VState ea = vstate(keys, vals, nv, L, a, n, alive_a, vafter, vlastrem, vf);
  VState eb = vstate(keys, vals, nv, L, b, n, alive_b, vafter, vlastrem, vf);
  int64_t tce = -1;
  if (ea.lastrem != NONE) tce = ea.lastrem;
  if (eb.lastrem != NONE && (int64_t)eb.lastrem > tce) tce = eb.lastrem;
  if (tce > last_pt) present = false;
  // an endpoint live at e and removed in this batch: its clear tombstones
  // the version present at e
  bool cleared = present0 && tce >= 0;
  bool tomb = present0 && !cleared && (!present || w != w0);
  bool ins = present && (!present0 || cleared || w != w0);
  recflags[k] = (uint8_t)((tomb ? 1 : 0) | (ins ? 2 : 0));
  recw[k] = w;
  return ins;
}

// Wave-uniform call: adds each inserting lane's insert to cnt[x] and tells
// the lane that made the count leave zero.  Keys are sorted by source, so a
// vertex's inserts often sit on consecutive lanes; such a run adds its
// length with one atomic from its first lane (a hub's inserts had queued
// one atomic per key on one word).
__device__ inline bool count_inserts(uint32_t* cnt, bool ins, uint32_t x) {
  const uint32_t lane = lane_id();
  const uint32_t xp = __shfl_up(x, 1, 64);
  const bool insp = __shfl_up(ins ? 1 : 0, 1, 64) != 0;
  const bool cont = ins && lane > 0 && insp && xp == x;
  const unsigned long long mc = __ballot(cont);
  if (!ins || cont) return false;
  const unsigned long long after = lane == 63 ? 0ull : mc >> (lane + 1);
  const uint32_t len = 1u + (uint32_t)__builtin_ctzll(~after);
  return atomicAdd(&cnt[x], len) == 0;
}

__global__ __launch_bounds__(UPD_THREADS) void k_resolve_edge(
    const uint64_t* keys, const uint32_t* vals, const dg_op* ops, uint32_t n, uint32_t L, Store st,
    uint8_t* results, const uint8_t* vafter, const uint32_t* vlastrem, uint8_t* recflags, int32_t* recw,
    uint32_t* touch_f, uint32_t* touch_r, uint32_t* insf, uint32_t* insr, UpdCounters* c) {
  if (c->flags) return;
  const uint32_t nv = c->nv;
  if (nv + blockIdx.x * UPD_THREADS >= n) return;   // workgroup-uniform
  __shared__ uint32_t vf_lds[VF_WORDS];
  const uint32_t* vf = nullptr;
  if (nv <= VF_MAX_VERTS) {
    for (uint32_t w = threadIdx.x; w < VF_WORDS; w += UPD_THREADS) vf_lds[w] = 0u;
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < nv; j += UPD_THREADS) {
      const uint32_t h = vf_hash((uint32_t)(keys[j] >> L));
      atomicOr(&vf_lds[h >> 5], 1u << (h & 31));
    }
    __syncthreads();
    vf = vf_lds;
  }
  const uint32_t k = nv + blockIdx.x * UPD_THREADS + threadIdx.x;
  bool ins = false;
  uint32_t a = 0, b = 0;
  if (k < n) {
    const uint64_t key = keys[k];
    if (k > nv && keys[k - 1] == key) recflags[k] = 0;
    else ins = resolve_key(keys, vals, ops, n, nv, L, st, results, vafter, vlastrem, vf, k, key, recflags, recw, &a, &b);
  }
  // count the insert at each endpoint; the first insert at a vertex lists
  // it as touched (one list reservation per wave, not per lane)
  const bool fa = count_inserts(insf, ins, a);
  wave_append(touch_f, &c->n_touch_f, fa, a);
  if (!st.undirected) {
    const bool fb = count_inserts(insr, ins, b);
    wave_append(touch_r, &c->n_touch_r, fb, b);
  } else {
    const bool fb = count_inserts(insf, ins && a != b, b);
    wave_append(touch_f, &c->n_touch_f, fb, b);
  }
}

// One lane per touched vertex: decide whether its slab must grow.
// plan[k] = log2(new buckets) + 1, or 0 when the slab keeps its size.  The
// versions a growing slab keeps are counted by its own lane when the slab
// is small, else by its whole wave, one such slab after another; a wave
// per touched vertex had left 63 lanes idle on nearly every vertex.
__global__ __launch_bounds__(UPD_THREADS) void k_grow_plan(Store st, const uint32_t* touch_f,
                                                            const uint32_t* touch_r, uint32_t* plan,
                                                            uint32_t* plan_ins, uint32_t* glist, uint32_t* insf,
                                                            uint32_t* insr, uint32_t floor_e,
                                                            UpdCounters* c) {
  if (c->flags) return;
  const uint32_t nf = c->n_touch_f, nt = nf + c->n_touch_r;
  const uint32_t lane = lane_id();
  const uint32_t gw = (blockIdx.x * UPD_THREADS + threadIdx.x) >> 6, nw = (gridDim.x * UPD_THREADS) >> 6;
  for (uint32_t base = gw * 64; base < nt; base += nw * 64) {   // wave-uniform
    const uint32_t k = base + lane;
    const bool act = k < nt, fwd = k < nf;
    uint32_t ins = 0;
    Slab sl{nullptr, nullptr, 0, 0};
    bool grow = false;
    if (act) {
      const uint32_t x = fwd ? touch_f[k] : touch_r[k - nf];
      uint32_t* insa = fwd ? insf : insr;
      uint32_t* useda = fwd ? st.fused : st.rused;
      ins = insa[x];
      const uint32_t used = useda[x];
      sl = slab_of(fwd ? st.fp : st.rp, fwd ? st.fdesc[x] : st.rdesc[x]);
      grow = (uint64_t)used + ins > 12ull * sl.nb;
      insa[x] = 0;
      if (!grow) {
        useda[x] = used + ins;
        plan[k] = 0;
      }
    }
    // a slab of at most SMALL_GROW buckets is counted by its own lane
    constexpr uint32_t SMALL_GROW = 2;
    uint32_t kept_own = 0;
    if (grow && sl.nb <= SMALL_GROW) {
      for (uint32_t bk = 0; bk < sl.nb; bk++) {
        uint32_t* bp = bucket_ptr(sl, bk);
        uint32_t d[BSLOTS];
        load_dsts(bp, d);
#pragma unroll
        for (int j = 0; j < BSLOTS; j++)
          kept_own += d[j] != EMPTY && *slot_death(bp, j, sl.words) > floor_e ? 1u : 0u;
      }
    }
    for (unsigned long long gm = __ballot(grow && sl.nb > SMALL_GROW); gm; gm &= gm - 1) {
      const int l = __ffsll((long long)gm) - 1;
      uint32_t* sb = reinterpret_cast<uint32_t*>(__shfl(reinterpret_cast<unsigned long long>(sl.base), l, 64));
      const uint32_t snb = __shfl(sl.nb, l, 64), sw = __shfl(sl.words, l, 64);
      uint32_t kept = 0;
      for (uint32_t t = lane; t < snb * BSLOTS; t += 64) {
        uint32_t* bp = sb + (uint64_t)(t / BSLOTS) * sw;
        const uint32_t j = t % BSLOTS;
        if (*slot_dst(bp, j) != EMPTY && *slot_death(bp, j, sw) > floor_e) kept++;
      }
      kept = wave_sum_u32(kept);
      if ((int)lane == l) kept_own = kept;
    }
    if (grow) {
      const uint64_t target = (uint64_t)kept_own + ins;
      uint32_t lg = 0;
      while ((8ull << lg) < target) lg++;
      plan[k] = lg + 1;
      plan_ins[k] = ins;
      atomicAdd(fwd ? &c->demand_f : &c->demand_r, 1ull << lg);
      glist[atomicAdd(&c->n_grow, 1u)] = k;
    }
  }
}

// Growing slab i of the batch: its touch-list entry and pool.
struct GrowRef {
  uint32_t k, x, lg;
  bool fwd;
};
__device__ inline GrowRef grow_ref(uint32_t i, const uint32_t* glist, const uint32_t* plan, const uint32_t* touch_f,
                                   const uint32_t* touch_r, uint32_t nf) {
  GrowRef r;
  r.k = glist[i];
  r.fwd = r.k < nf;
  r.x = r.fwd ? touch_f[r.k] : touch_r[r.k - nf];
  r.lg = plan[r.k] - 1;
  return r;
}

__device__ inline unsigned long long wave_incl_sum64(unsigned long long x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

// Reserve each growing slab's new space (or flag the batch out of memory):
// a wave takes its slabs' space with one atomic per pool cursor.
__global__ __launch_bounds__(UPD_THREADS) void k_grow_alloc(Store st, const uint32_t* glist, const uint32_t* plan,
                                                             unsigned long long* goff, uint32_t* gkept,
                                                             UpdCounters* c) {
  if (c->flags) return;
  if (c->cursor0_f + c->demand_f > st.fp.cap || (!st.undirected && c->cursor0_r + c->demand_r > st.rp.cap)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&c->flags, (uint32_t)F_OOM);
    return;
  }
  const uint32_t ng = c->n_grow, nf = c->n_touch_f;
  const uint32_t lane = lane_id();
  const uint32_t gw = (blockIdx.x * UPD_THREADS + threadIdx.x) >> 6, nw = (gridDim.x * UPD_THREADS) >> 6;
  for (uint32_t base = gw * 64; base < ng; base += nw * 64) {   // wave-uniform
    const uint32_t i = base + lane;
    const bool act = i < ng;
    const uint32_t k = act ? glist[i] : 0u;
    const bool fwd = act && k < nf;
    const unsigned long long sz = act ? 1ull << (plan[k] - 1) : 0ull;
    const unsigned long long szf = fwd ? sz : 0ull, szr = fwd ? 0ull : sz;
    const unsigned long long xf = wave_incl_sum64(szf), xr = wave_incl_sum64(szr);
    const unsigned long long tf = __shfl(xf, 63, 64), tr = __shfl(xr, 63, 64);
    unsigned long long bf = 0, br = 0;
    if (lane == 0) {
      if (tf) bf = atomicAdd(&st.cursor[0], tf);
      if (tr) br = atomicAdd(&st.cursor[1], tr);
    }
    bf = __shfl(bf, 0, 64);
    br = __shfl(br, 0, 64);
    if (act) {
      goff[i] = fwd ? bf + xf - szf : br + xr - szr;
      gkept[i] = 0;
    }
  }
}

// Empty the new slabs: workgroups (x, y) share slab x's words.
__global__ __launch_bounds__(UPD_THREADS) void k_grow_init(Store st, const uint32_t* glist, const uint32_t* plan,
                                                            const unsigned long long* goff, UpdCounters* c) {
  if (c->flags) return;
  const uint32_t ng = c->n_grow, nf = c->n_touch_f;
  const uint32_t t0 = blockIdx.y * UPD_THREADS + threadIdx.x, tstep = gridDim.y * UPD_THREADS;
  for (uint32_t i = blockIdx.x; i < ng; i += gridDim.x) {
    const uint32_t k = glist[i];
    const Pool& p = k < nf ? st.fp : st.rp;
    const uint32_t nb2 = 1u << (plan[k] - 1);
    Slab ns = slab_at(p, goff[i], nb2);
    for (uint64_t t = t0; t < (uint64_t)nb2 * p.words; t += tstep) ns.base[t] = 0xFFFFFFFFu;
    clear_summaries(ns.sum, nb2, t0, tstep);
  }
}

// Rehash the versions that stay (death above the floor) into the new slabs:
// workgroups (x, y) share slab x's old slots.
__global__ __launch_bounds__(UPD_THREADS) void k_grow_move(Store st, const uint32_t* touch_f, const uint32_t* touch_r,
                                                            const uint32_t* glist, const uint32_t* plan,
                                                            const unsigned long long* goff, uint32_t* gkept,
                                                            uint32_t floor_e, UpdCounters* c) {
  if (c->flags) return;
  const uint32_t ng = c->n_grow, nf = c->n_touch_f;
  const uint32_t t0 = blockIdx.y * UPD_THREADS + threadIdx.x, tstep = gridDim.y * UPD_THREADS;
  for (uint32_t i = blockIdx.x; i < ng; i += gridDim.x) {
    const GrowRef g = grow_ref(i, glist, plan, touch_f, touch_r, nf);
    const Pool& p = g.fwd ? st.fp : st.rp;
    Slab ns = slab_at(p, goff[i], 1u << g.lg);
    Slab os = slab_of(p, (g.fwd ? st.fdesc : st.rdesc)[g.x]);
    uint32_t kept = 0;
    for (uint32_t t = t0; t < os.nb * BSLOTS; t += tstep) {
      uint32_t* bp = bucket_ptr(os, t / BSLOTS);
      uint32_t j = t % BSLOTS;
      uint32_t d = *slot_dst(bp, j);
      if (d == EMPTY) continue;
      uint64_t stamp = *slot_stamp(bp, j, os.words);
      if ((uint32_t)(stamp >> 32) <= floor_e) continue;
      SlotRef r = claim_slot(ns, d, (uint32_t)stamp);
      if (g.fwd) *slot_w(r.bp, r.j) = *slot_w(bp, j);
      *slot_stamp(r.bp, r.j, ns.words) = stamp;
      if ((uint32_t)(stamp >> 32) != INF_EPOCH) mark_tomb(ns, r.b, r.j, (uint32_t)(stamp >> 32));
      kept++;
    }
    kept = wave_sum_u32(kept);
    if (lane_id() == 0 && kept) atomicAdd(&gkept[i], kept);
  }
}

// Point each grown vertex at its new slab.
__global__ __launch_bounds__(UPD_THREADS) void k_grow_publish(Store st, const uint32_t* touch_f,
                                                               const uint32_t* touch_r, const uint32_t* glist,
                                                               const uint32_t* plan, const uint32_t* plan_ins,
                                                               const unsigned long long* goff, const uint32_t* gkept,
                                                               UpdCounters* c) {
  if (c->flags) return;
  const uint32_t ng = c->n_grow, nf = c->n_touch_f;
  for (uint32_t i = blockIdx.x * UPD_THREADS + threadIdx.x; i < ng; i += gridDim.x * UPD_THREADS) {
    const GrowRef g = grow_ref(i, glist, plan, touch_f, touch_r, nf);
    (g.fwd ? st.fdesc : st.rdesc)[g.x] = make_desc(goff[i], g.lg);
    (g.fwd ? st.fused : st.rused)[g.x] = gkept[i] + plan_ins[g.k];
  }
}

// Tombstone the current version of `key` (death INF -> E).  Returns true
// for the one thread whose compare-and-swap made the transition.
__device__ inline bool tombstone_in(const Pool& p, uint64_t desc, uint32_t key, uint32_t E) {
  Slab s = slab_of(p, desc);
  SlotRef r = find_current(s, key);
  if (!r.bp) return false;
  if (atomicCAS(slot_death(r.bp, r.j, s.words), INF_EPOCH, E) != INF_EPOCH) return false;
  mark_tomb(s, r.b, r.j, E);
  return true;
}

// One workgroup per cleared vertex.  arcs_delta counts forward-pool slots
// whose version this batch tombstoned (each exactly once, via the CAS).
__global__ __launch_bounds__(UPD_THREADS) void k_clear(Store st, const uint32_t* clear_list, uint32_t E,
                                                        UpdCounters* c) {
  if (c->flags) return;
  const uint32_t ncl = c->n_clear;
  // workgroups (x, y) share vertex x's slots: y strides over them, so a
  // hub's arcs are spread over gridDim.y workgroups
  const uint32_t t0 = blockIdx.y * UPD_THREADS + threadIdx.x, tstep = gridDim.y * UPD_THREADS;
  for (uint32_t k = blockIdx.x; k < ncl; k += gridDim.x) {
    uint32_t x = clear_list[k];
    int dropped = 0;
    Slab fs = slab_of(st.fp, st.fdesc[x]);
    for (uint32_t t = t0; t < fs.nb * BSLOTS; t += tstep) {
      uint32_t* bp = bucket_ptr(fs, t / BSLOTS);
      uint32_t j = t % BSLOTS;
      uint32_t d = ld_relaxed(slot_dst(bp, j));
      if (d == EMPTY) continue;
      if (atomicCAS(slot_death(bp, j, fs.words), INF_EPOCH, E) != INF_EPOCH) continue;
      mark_tomb(fs, t / BSLOTS, j, E);
      dropped++;
      if (!st.undirected) tombstone_in(st.rp, st.rdesc[d], x, E);
      else if (d != x && tombstone_in(st.fp, st.fdesc[d], x, E)) dropped++;
    }
    if (!st.undirected) {
      Slab rs = slab_of(st.rp, st.rdesc[x]);
      for (uint32_t t = t0; t < rs.nb * BSLOTS; t += tstep) {
        uint32_t* bp = bucket_ptr(rs, t / BSLOTS);
        uint32_t j = t % BSLOTS;
        uint32_t sv = ld_relaxed(slot_dst(bp, j));
        if (sv == EMPTY) continue;
        if (atomicCAS(slot_death(bp, j, rs.words), INF_EPOCH, E) != INF_EPOCH) continue;
        mark_tomb(rs, t / BSLOTS, j, E);
        if (tombstone_in(st.fp, st.fdesc[sv], x, E)) dropped++;
      }
    }
    uint32_t tot = wave_sum_u32((uint32_t)dropped);
    if (lane_id() == 0 && tot) atomicAdd(&c->arcs_delta, (unsigned long long)(-(long long)tot));
  }
}

__device__ inline void insert_in(const Pool& p, uint64_t desc, uint32_t key, int32_t w, bool has_w, uint32_t E) {
  Slab s = slab_of(p, desc);
  SlotRef r = claim_slot(s, key, E);
  if (!r.bp) return;   // unreachable: growth guarantees a free slot
  if (has_w) *slot_w(r.bp, r.j) = (uint32_t)w;
  *slot_stamp(r.bp, r.j, s.words) = (uint64_t)E | ((uint64_t)INF_EPOCH << 32);
}

__global__ __launch_bounds__(UPD_THREADS) void k_commit_edge(const uint64_t* keys, uint32_t n, uint32_t L,
                                                              Store st, const uint8_t* recflags,
                                                              const int32_t* recw, uint32_t E,
                                                              UpdCounters* c) {
  if (c->flags) return;
  uint32_t k = c->nv + blockIdx.x * UPD_THREADS + threadIdx.x;
  uint8_t f = k < n ? recflags[k] : 0;
  int delta = 0;
  if (f) {
    const uint64_t mask = (1ull << L) - 1;
    uint64_t key = keys[k];
    uint32_t a = (uint32_t)((key >> L) & mask), b = (uint32_t)(key & mask);
    if (f & 1) {
      if (tombstone_in(st.fp, st.fdesc[a], b, E)) delta--;
      if (!st.undirected) tombstone_in(st.rp, st.rdesc[b], a, E);
      else if (a != b && tombstone_in(st.fp, st.fdesc[b], a, E)) delta--;
    }
    if (f & 2) {
      int32_t w = recw[k];
      insert_in(st.fp, st.fdesc[a], b, w, true, E);
      delta++;
      if (!st.undirected) insert_in(st.rp, st.rdesc[b], a, 0, false, E);
      else if (a != b) {
        insert_in(st.fp, st.fdesc[b], a, w, true, E);
        delta++;
      }
    }
  }
  // wave-aggregated count of arcs added minus arcs tombstoned
  int tot = 0;
  {
    int v = delta;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    tot = v;
  }
  if (lane_id() == 0 && tot) atomicAdd(&c->arcs_delta, (unsigned long long)(long long)tot);
}

__global__ __launch_bounds__(UPD_THREADS) void k_commit_vertex(Store st, const uint32_t* vchange, UpdCounters* c) {
  if (c->flags) return;
  uint32_t nvc = c->n_vchange;
  for (uint32_t k = blockIdx.x * UPD_THREADS + threadIdx.x; k < nvc; k += gridDim.x * UPD_THREADS) {
    uint32_t x = vchange[k];
    st.alive[x & 0x7FFFFFFFu] = (uint8_t)(x >> 31);
  }
}

static inline uint32_t blocks_for(uint64_t n, uint32_t per, uint32_t cap = 1u << 20) {
  uint64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (uint32_t)b;
}

hipError_t ensure_update_scratch(dg_graph* g, uint64_t n) {
  UpdateScratch& u = g->us;
  if (n <= u.cap && u.host_summary) return hipSuccess;
  uint64_t c = std::max<uint64_t>(n, 1024);
  hipError_t e;
#define ENS(buf, bytes) \
  if ((e = ensure(u.buf, (bytes))) != hipSuccess) return e;
  ENS(keys0, c * 8) ENS(keys1, c * 8) ENS(vals0, c * 4) ENS(vals1, c * 4)
  ENS(sortw, sort_scratch_words((uint32_t)c) * 4)
  ENS(vafter, c) ENS(vlastrem, c * 4) ENS(recflags, c) ENS(recw, c * 4)
  ENS(ops, c * sizeof(dg_op)) ENS(results, c) ENS(touch, c * 12) ENS(plan, c * 24) ENS(clear, c * 4)
  ENS(grow, c * 48)
  ENS(summary, sizeof(UpdCounters) + c * 4)
#undef ENS
  if (!u.host_summary) {
    // counters, the inline vertex changes, then the publication's sequence word
    e = hipHostMalloc(&u.host_summary, sizeof(UpdCounters) + VCHANGE_INLINE * 4 + 4, hipHostMallocCoherent);
    if (e == hipSuccess) std::memset(u.host_summary, 0, sizeof(UpdCounters) + VCHANGE_INLINE * 4 + 4);
    if (e != hipSuccess) return e;
  }
  u.cap = c;
  return hipSuccess;
}

// Copies the batch counters and the first VCHANGE_INLINE vertex changes to
// coherent pinned host memory, then (system scope, last) the sequence word.
__global__ void k_upd_publish(const UpdCounters* c, const uint32_t* vchange, uint32_t* host, uint32_t seq) {
  constexpr uint32_t W = sizeof(UpdCounters) / 4;
  const uint32_t* cw = reinterpret_cast<const uint32_t*>(c);
  const uint32_t nv = min(c->n_vchange, VCHANGE_INLINE);
  for (uint32_t t = threadIdx.x; t < W + nv; t += blockDim.x) host[t] = t < W ? cw[t] : vchange[t - W];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(host + W + VCHANGE_INLINE, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Runs the pipeline once; *flags receives the batch flags.
static hipError_t run_pipeline(dg_graph* g, const dg_op* dops, uint32_t n, uint8_t* dres, hipStream_t s,
                               UpdCounters* hc) {
  UpdateScratch& u = g->us;
  // host state is read under the graph mutex; the GPU work runs without it
  Store st;
  uint32_t E, fl;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    st = g->st;
    E = g->epoch + 1;
    fl = gc_floor(g);
  }
  const uint32_t L = g->L;
  UpdCounters* c = u.summary.as<UpdCounters>();
  uint32_t* vchange = reinterpret_cast<uint32_t*>(c + 1);
  uint32_t* touch_f = u.touch.as<uint32_t>();
  uint32_t* touch_r = touch_f + 2ull * n;   // undirected inserts touch both ends
  uint32_t* plan = u.plan.as<uint32_t>();
  uint32_t* plan_ins = plan + 3ull * n;
  unsigned long long* goff = u.grow.as<unsigned long long>();   // 3n entries each
  uint32_t* glist = reinterpret_cast<uint32_t*>(goff + 3ull * n);
  uint32_t* gkept = glist + 3ull * n;
  uint32_t nb = blocks_for(n, UPD_THREADS);

  k_upd_init<<<1, 64, 0, s>>>(c, st.cursor);
  k_prep<<<nb, UPD_THREADS, 0, s>>>(dops, n, st.V, st.undirected, g->cfg.w_max, L, u.keys0.as<uint64_t>(),
                                    u.vals0.as<uint32_t>(), c);
  bool alt = radix_sort_pairs(u.keys0.as<uint64_t>(), u.vals0.as<uint32_t>(), u.keys1.as<uint64_t>(),
                              u.vals1.as<uint32_t>(), n, (int)(2 * L + 1), u.sortw.as<uint32_t>(), s);
  const uint64_t* keys = alt ? u.keys1.as<uint64_t>() : u.keys0.as<uint64_t>();
  const uint32_t* vals = alt ? u.vals1.as<uint32_t>() : u.vals0.as<uint32_t>();
  k_resolve_vertex<<<nb, UPD_THREADS, 0, s>>>(keys, vals, dops, n, L, st.alive, dres, u.vafter.as<uint8_t>(),
                                              u.vlastrem.as<uint32_t>(), u.clear.as<uint32_t>(), vchange, c);
  k_resolve_edge<<<nb, UPD_THREADS, 0, s>>>(keys, vals, dops, n, L, st, dres, u.vafter.as<uint8_t>(),
                                            u.vlastrem.as<uint32_t>(), u.recflags.as<uint8_t>(),
                                            u.recw.as<int32_t>(), touch_f, touch_r, g->insf.as<uint32_t>(),
                                            g->insr.as<uint32_t>(), c);
  k_grow_plan<<<blocks_for(3ull * n, UPD_THREADS, 4096), UPD_THREADS, 0, s>>>(
      st, touch_f, touch_r, plan, plan_ins, glist, g->insf.as<uint32_t>(), g->insr.as<uint32_t>(), fl, c);
  const uint32_t gx = blocks_for(3ull * n, 1, 512);
  k_grow_alloc<<<blocks_for(3ull * n, UPD_THREADS, 64), UPD_THREADS, 0, s>>>(st, glist, plan, goff, gkept, c);
  k_grow_init<<<dim3(gx, 8), UPD_THREADS, 0, s>>>(st, glist, plan, goff, c);
  k_grow_move<<<dim3(gx, 8), UPD_THREADS, 0, s>>>(st, touch_f, touch_r, glist, plan, goff, gkept, fl, c);
  k_grow_publish<<<blocks_for(3ull * n, UPD_THREADS, 64), UPD_THREADS, 0, s>>>(st, touch_f, touch_r, glist, plan,
                                                                             plan_ins, goff, gkept, c);
  k_clear<<<dim3(blocks_for(n, 1, 1024), 8), UPD_THREADS, 0, s>>>(st, u.clear.as<uint32_t>(), E, c);
  k_commit_edge<<<nb, UPD_THREADS, 0, s>>>(keys, n, L, st, u.recflags.as<uint8_t>(), u.recw.as<int32_t>(), E, c);
  k_commit_vertex<<<blocks_for(n, UPD_THREADS, 1024), UPD_THREADS, 0, s>>>(st, vchange, c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the device publishes the counters (and the first vertex changes) to
  // coherent pinned memory and the host polls for the sequence word; a
  // publication not seen within two seconds falls back to synchronising
  // the stream, which reports any device error
  uint32_t* hs = static_cast<uint32_t*>(u.host_summary);
  uint32_t* seqw = hs + sizeof(UpdCounters) / 4 + VCHANGE_INLINE;
  const uint32_t seq = ++u.pub_seq;
  k_upd_publish<<<1, 256, 0, s>>>(c, vchange, hs, seq);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 1; __atomic_load_n(seqw, __ATOMIC_ACQUIRE) != seq; spin++) {
    host_pause(spin);
    if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (__atomic_load_n(seqw, __ATOMIC_ACQUIRE) != seq) return hipErrorUnknown;
      break;
    }
  }
  std::memcpy(hc, u.host_summary, sizeof(UpdCounters));
  return hipSuccess;
}

static void record_vertex_changes(dg_graph* g, const uint32_t* list, uint32_t cnt, uint32_t E) {
  for (uint32_t k = 0; k < cnt; k++) {
    uint32_t x = list[k] & 0x7FFFFFFFu;
    bool now = (list[k] >> 31) != 0;
    if (g->vfirst[x] == 0) {
      g->vfirst[x] = E;
    } else {
      if (g->vhead[x] == VLOG_NONE) g->vtoggled.push_back(x);
      g->vlog.emplace_back(E, g->vhead[x]);
      g->vhead[x] = (uint32_t)(g->vlog.size() - 1);
    }
    g->n_live += now ? 1 : -1;
  }
}

dg_status apply_batch_dev(dg_graph* g, const dg_op* dops, uint64_t n, uint8_t* dres, hipStream_t s) {
  if (n == 0) return DG_OK;
  if (n > 0xFFFFFFF0ull) {
    g->err = "batch too large";
    return DG_E_INVALID_ARG;
  }
  hipError_t e = ensure_update_scratch(g, n);
  if (e != hipSuccess) {
    g->err = std::string("scratch allocation: ") + hipGetErrorString(e);
    return DG_E_OUT_OF_MEMORY;
  }
  uint8_t* res = dres ? dres : g->us.results.as<uint8_t>();
  UpdCounters hc{};
  for (int attempt = 0; attempt < 8; attempt++) {
    {
      ProfScope ps(g, KID_UPDATE, s);
      e = run_pipeline(g, dops, (uint32_t)n, res, s, &hc);
    }
    if (e != hipSuccess) {
      g->err = std::string("update pipeline: ") + hipGetErrorString(e);
      return DG_E_HIP;
    }
    if (hc.flags & F_BAD_TYPE) {
      g->err = "unknown op type in batch";
      return DG_E_INVALID_ARG;
    }
    if (hc.flags & F_BAD_VERTEX) {
      g->err = "vertex id out of range in batch";
      return DG_E_VERTEX_RANGE;
    }
    if (hc.flags & F_BAD_WEIGHT) {
      g->err = "AddEdge weight out of range in batch";
      return DG_E_WEIGHT_RANGE;
    }
    if (!(hc.flags & F_OOM)) break;
    // the growth step found the pools too small and nothing was committed:
    // enlarge them and run the batch again
    e = grow_pools(g, hc.demand_f, hc.demand_r);
    if (e != hipSuccess) {
      g->err = std::string("pool growth: ") + hipGetErrorString(e);
      return DG_E_OUT_OF_MEMORY;
    }
    if (attempt == 7) {
      g->err = "pool growth did not converge";
      return DG_E_OUT_OF_MEMORY;
    }
  }
  std::lock_guard<std::mutex> lk(g->mu);
  const uint32_t E = g->epoch + 1;
  if (hc.n_vchange <= VCHANGE_INLINE) {
    record_vertex_changes(g, reinterpret_cast<uint32_t*>(static_cast<char*>(g->us.host_summary) + sizeof(UpdCounters)),
                          hc.n_vchange, E);
  } else {
    std::vector<uint32_t> lst(hc.n_vchange);
    e = hipMemcpyAsync(lst.data(), reinterpret_cast<uint32_t*>(g->us.summary.as<UpdCounters>() + 1),
                       (size_t)hc.n_vchange * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      g->err = std::string("vertex change readback: ") + hipGetErrorString(e);
      return DG_E_HIP;
    }
    record_vertex_changes(g, lst.data(), hc.n_vchange, E);
  }
  g->epoch = E;
  g->arcs_by_epoch.push_back((uint64_t)((int64_t)g->arcs_by_epoch.back() + (int64_t)hc.arcs_delta));
  g->live_by_epoch.push_back(g->n_live);
  return DG_OK;
}

}  // namespace dg
