// Multi-source Brandes betweenness: up to MBQ sources of one BC query on
// one snapshot run as one level-synchronous search (Brandes 2001) over a
// shared frontier.
//
// Each vertex holds the group's per-source state in one record per field:
// level L[v * MBQ + s] (int32, -1 unreached), path count SG[v * MBQ + s]
// (int64) and dependency DL[v * MBQ + s] (FP64).  Forward pass at level l:
// a frontier item is a vertex with a mask of the sources that reached it at
// level l; for arc (u, w), lane s of a 16-lane group claims L[w][s] for
// level l + 1 (compare-and-swap from -1) and, where w sits at l + 1, adds
// SG[u][s] to SG[w][s] (exact int64 adds, overflow flagged).  Sources whose
// level-l+1 bit is new for w OR it into w's tagged mask for the next pass;
// the first bit enqueues w and appends it to the level's vertex list.
//
// Backward pass at level l, one wave per vertex v of the level's list, for
// each source s with L[v][s] = l:
//   DL[v][s] = sum over visible arcs v -> w with L[w][s] = l + 1 of
//              SG[v][s] / SG[w][s] * (1 + DL[w][s])
//            = SG[v][s] * (sum of CL[w][s]),  CL = (1 + DL) / SG,
// each lane summing its slots bucket after bucket (a long slab tile by
// tile) and the partial sums combining in the plain path's fixed order,
// so every dependency equals the plain path's bit for bit.  Then
// bc[v] += DL[v][s] for the group's sources in their order (v != s, v
// reached), which continues the plain path's sequence of additions.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dg_host.h"
#include "frontier.h"

namespace dg {

constexpr uint32_t MBQ = 16;
constexpr uint32_t MB_TAG_MAX = 0xFFFFu;

struct MbFwd {
  Store st;
  uint32_t e;
  int fast;
  Front fin, fout;
  int32_t* L;
  unsigned long long* SG;
  const uint32_t* nm_in;   // masks of fin's vertices (tag_in)
  uint32_t* nm_out;        // masks of the next level's vertices (tag_out)
  uint32_t* order;         // vertex lists of the levels, appended
  uint32_t order_cap;
  uint32_t tag_in, tag_out;
  int32_t next_level;
  uint32_t nq;
  QCounters* cnt_out;      // fq, n_order = level vertices appended, overflow, arcs
  QCounters* reset;
};

__device__ inline void mb_reset(QCounters* c) {
  if (blockIdx.x == 0 && threadIdx.x == 0) zero_counters(c);
}

__device__ inline bool mb_mark(uint32_t* nm, uint32_t v, uint32_t tag, uint32_t bits) {
  uint32_t old = __hip_atomic_load(&nm[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const bool same = (old >> 16) == tag;
    const uint32_t nw = same ? (old | bits) : ((tag << 16) | bits);
    if (nw == old) return false;
    const uint32_t prev = atomicCAS(&nm[v], old, nw);
    if (prev == old) return !same;
    old = prev;
  }
}

template <class T>
__device__ inline T mb_pick4(const T (&x)[4], int k) {
  return k == 0 ? x[0] : (k == 1 ? x[1] : (k == 2 ? x[2] : x[3]));
}

__device__ __forceinline__ void mb_fwd_chunk(const MbFwd& a, uint32_t c, uint32_t nitems, uint32_t nb, ItemQ& qn,
                                             U32Q& qo, LaneCounts& lc, uint32_t& ovf) {
  const uint32_t j = threadIdx.x & 15, gb = threadIdx.x & 48, grp = (threadIdx.x >> 4) & 3;
  const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
  uint32_t mk_l = 0;
  if (touches(cv)) {
    const uint32_t t = a.nm_in[cv.v];
    mk_l = (t >> 16) == a.tag_in ? (t & 0xFFFFu) : 0u;
  }
  for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
    Pairs4 s4 = load_pairs<false>(a.st.fp, cv, f0, grp, j, a.e, a.fast);
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
      const uint32_t it_k = mb_pick4(s4.item, k), d_k = mb_pick4(s4.d, k);
      const int vis_k = mb_pick4(s4.vis, k) ? 1 : 0;
      const uint32_t u = __shfl(cv.v, (int)it_k, 64);
      const uint32_t mk = __shfl(mk_l, (int)it_k, 64);
      const bool mine = j < a.nq && ((mk >> j) & 1u);
      const unsigned long long su = mine ? a.SG[(uint64_t)u * MBQ + j] : 0ull;
      uint32_t my_new = 0;
#pragma unroll 1
      for (int h = 0; h < 16; h += 8) {
        uint32_t dd[8];
        int32_t lv[8];
        bool act[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
          dd[t] = __shfl(d_k, (int)(gb + h + t), 64);
          const bool vis = __shfl(vis_k, (int)(gb + h + t), 64) != 0;
          act[t] = vis && mine;
          lv[t] = act[t] ? a.L[(uint64_t)dd[t] * MBQ + j] : 0;
          lc.arcs += act[t] ? 1 : 0;
        }
        bool found[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
          found[t] = false;
          if (act[t] && lv[t] < 0) {
            const int32_t prev = atomicCAS(&a.L[(uint64_t)dd[t] * MBQ + j], -1, a.next_level);
            found[t] = prev == -1;
            lv[t] = found[t] ? a.next_level : prev;
          }
        }
#pragma unroll
        for (int t = 0; t < 8; t++) {
          if (act[t] && lv[t] == a.next_level) {
            const unsigned long long old = atomicAdd(&a.SG[(uint64_t)dd[t] * MBQ + j], su);
            if (old + su > 0x7FFFFFFFFFFFFFFFull) ovf = 1;
          }
        }
#pragma unroll
        for (int t = 0; t < 8; t++) {
          const uint32_t bits = group16_ballot(found[t]);
          if (j == (uint32_t)(h + t)) my_new = bits;
        }
      }
      const bool first = my_new && mb_mark(a.nm_out, d_k, a.tag_out, my_new);
      const uint64_t yd = first ? a.st.fdesc[d_k] : 0;
      lc.far += bwd_is_big(yd) ? 1 : 0;   // slabs the backward splits into tiles
      room_front(qn, 64, a.fout, a.cnt_out);
      push_item(qn, first, d_k, yd);
      room_u32(qo, 64, a.order, &a.cnt_out->n_order);
      push_u32(qo, first, d_k);
    }
  }
}

__global__ __launch_bounds__(Q_THREADS) void k_mb_fwd(MbFwd a, unsigned long long nfq) {
  __shared__ Shared sh;
  mb_reset(a.reset);
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * Q_WAVES + wave, nw = gridDim.x * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  U32Q qo = u32_q(sh.ws[wave]);
  LaneCounts lc;
  uint32_t ovf = 0;
  for (uint32_t c = gw; c < nc; c += nw) mb_fwd_chunk(a, c, nitems, nb, qn, qo, lc, ovf);
  flush_u32_q(qo, a.order, &a.cnt_out->n_order);
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  if (__ballot(ovf) && lane_id() == 0) atomicOr(&a.cnt_out->overflow, OVF_SIGMA);
  lc.commit(a.cnt_out, sh);
}

// Per-lane sums of CL[w][s] = (1 + DL[w][s]) / SG[w][s] over tile
// [b0, b1) of v's slab for the sources in m (the plain path's terms and
// order, one accumulator per source).
__device__ __forceinline__ void mb_tile_lanes(const Slab& sl, uint32_t b0, uint32_t b1, uint32_t e, bool fast,
                                              uint32_t m, int32_t lvl, const int32_t* L, const double* CL,
                                              double (&acc)[MBQ]) {
  const uint32_t j = lane_id() & 15;
  for (uint32_t b = b0 + (lane_id() >> 4); b < b1; b += 4) {
    uint32_t* bp = bucket_ptr(sl, b);
    const uint32_t w = bp[j];
    if (w == EMPTY || !slot_visible(sl, bp, b, j, e, fast)) continue;
    // the 16 levels of w: one 64-byte record, four 16-byte loads
    const int4* lw = reinterpret_cast<const int4*>(&L[(uint64_t)w * MBQ]);
    int32_t lv[MBQ];
#pragma unroll
    for (int q = 0; q < (int)(MBQ / 4); q++) {
      const int4 x = lw[q];
      lv[4 * q] = x.x;
      lv[4 * q + 1] = x.y;
      lv[4 * q + 2] = x.z;
      lv[4 * q + 3] = x.w;
    }
#pragma unroll
    for (int s = 0; s < (int)MBQ; s++) {
      if (((m >> s) & 1u) && lv[s] == lvl + 1) acc[s] += CL[(uint64_t)w * MBQ + s];
    }
  }
}

// A (vertex, source)'s dependency from its path count and sum of
// coefficients, and its own coefficient.  Every operation rounds on its own
// (no fused multiply-add), as in the plain path.
__device__ inline void mb_finish(double sv, double sum, double* dl, double* cl) {
#pragma clang fp contract(off)
  const double d = sv * sum;
  *dl = d;
  *cl = (1.0 + d) / sv;
}

// The group's sources at level lvl for vertex v (wave-uniform), and their
// path counts at v.
__device__ __forceinline__ uint32_t mb_at_level(uint32_t v, int32_t lvl, uint32_t nq, const int32_t* L,
                                                const unsigned long long* SG, double (&sv)[MBQ]) {
  const uint32_t lane = lane_id(), j = lane & 15;
  const bool at = j < nq && L[(uint64_t)v * MBQ + j] == lvl;
  const uint32_t m = (uint32_t)(__ballot(at && lane < 16) & 0xFFFFull);
#pragma unroll
  for (int s = 0; s < (int)MBQ; s++) sv[s] = ((m >> s) & 1u) ? (double)SG[(uint64_t)v * MBQ + s] : 0.0;
  return m;
}

// Backward pass of level lvl over its vertex list verts[0..nv): one wave
// per vertex; slabs of more than BWD_TILE buckets are listed for the tile
// pass (k_mb_tiles, k_mb_combine).  Workgroup 0 zeroes the other parity's
// tile counts.
__global__ __launch_bounds__(Q_THREADS) void k_mb_bwd(Store st, uint32_t e, int fast, const uint32_t* verts,
                                                      uint32_t nv, int32_t lvl, uint32_t nq, const int32_t* L,
                                                      const unsigned long long* SG, double* DL, double* CL,
                                                      BwdTiles bt) {
  const uint32_t lane = lane_id();
  const uint32_t par = (uint32_t)lvl & 1u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bt.head->verts[par ^ 1] = 0;
    bt.head->tiles[par ^ 1] = 0;
  }
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6), nwaves = gridDim.x * Q_WAVES;
  for (uint32_t k = gwave; k < nv; k += nwaves) {
    const uint32_t v = verts[k];
    const uint64_t desc = st.fdesc[v];
    const Slab sl = slab_of(st.fp, desc);
    if (bwd_is_big(desc)) {
      bwd_list(bt, par, v, desc);
      continue;
    }
    double sv[MBQ], acc[MBQ];
    const uint32_t m = mb_at_level(v, lvl, nq, L, SG, sv);
#pragma unroll
    for (int s = 0; s < (int)MBQ; s++) acc[s] = 0.0;
    mb_tile_lanes(sl, 0, sl.nb, e, fast != 0, m, lvl, L, CL, acc);
#pragma unroll
    for (int s = 0; s < (int)MBQ; s++) {
      if (!((m >> s) & 1u)) continue;   // wave-uniform
      double x = acc[s];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) mb_finish(sv[s], x, &DL[(uint64_t)v * MBQ + s], &CL[(uint64_t)v * MBQ + s]);
    }
  }
}

// One wave per listed tile of level lvl: its sums into part[tile * MBQ + s].
__global__ __launch_bounds__(Q_THREADS) void k_mb_tiles(Store st, uint32_t e, int fast, int32_t lvl, uint32_t nq,
                                                        const int32_t* L, const unsigned long long* SG,
                                                        const double* CL, BwdTiles bt) {
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * Q_WAVES + (threadIdx.x >> 6), nwaves = gridDim.x * Q_WAVES;
  const uint32_t nt = min(bt.head->tiles[lvl & 1], bt.cap_tiles);
  for (uint32_t t = gwave; t < nt; t += nwaves) {
    const uint32_t i = bt.tmap[t];
    if (i >= bt.cap_verts) continue;
    const BigVert bv = bt.big[i];
    if (t < bv.base || t - bv.base >= bv.n) continue;
    const Slab sl = slab_of(st.fp, bv.desc);
    const uint32_t b0 = (t - bv.base) << BWD_TILE_LOG;
    if (b0 >= sl.nb) continue;
    double sv[MBQ], acc[MBQ];
    const uint32_t m = mb_at_level(bv.v, lvl, nq, L, SG, sv);
#pragma unroll
    for (int s = 0; s < (int)MBQ; s++) acc[s] = 0.0;
    mb_tile_lanes(sl, b0, min(sl.nb, b0 + BWD_TILE), e, fast != 0, m, lvl, L, CL, acc);
#pragma unroll
    for (int s = 0; s < (int)MBQ; s++) {
      if (!((m >> s) & 1u)) continue;   // wave-uniform
      double x = acc[s];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) bt.part[(uint64_t)t * MBQ + s] = x;
    }
  }
}

// One lane per (listed vertex, source at level lvl): the tile sums added in
// tile order.
__global__ __launch_bounds__(Q_THREADS) void k_mb_combine(int32_t lvl, uint32_t nq, const int32_t* L,
                                                          const unsigned long long* SG, double* DL, double* CL,
                                                          BwdTiles bt) {
  const uint32_t nbig = min(bt.head->verts[lvl & 1], bt.cap_verts);
  for (uint64_t x = (uint64_t)blockIdx.x * Q_THREADS + threadIdx.x; x < (uint64_t)nbig * MBQ;
       x += (uint64_t)gridDim.x * Q_THREADS) {
    const uint32_t i = (uint32_t)(x / MBQ), s = (uint32_t)(x % MBQ);
    const BigVert bv = bt.big[i];
    if (s >= nq || L[(uint64_t)bv.v * MBQ + s] != lvl) continue;
    if (bv.n == 0 || bv.base >= bt.cap_tiles || bv.n > bt.cap_tiles - bv.base) continue;
    double acc = bt.part[(uint64_t)bv.base * MBQ + s];
    for (uint32_t t = 1; t < bv.n; t++) acc += bt.part[(uint64_t)(bv.base + t) * MBQ + s];
    mb_finish((double)SG[(uint64_t)bv.v * MBQ + s], acc, &DL[(uint64_t)bv.v * MBQ + s], &CL[(uint64_t)bv.v * MBQ + s]);
  }
}

// bc[v] += DL[v][s] for the group's sources in order, where v was reached
// and is not the source.
__global__ void k_mb_accum(const int32_t* L, const double* DL, const uint32_t* src, uint32_t nq, uint64_t V,
                           double* bc) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (uint64_t)gridDim.x * blockDim.x) {
    double x = bc[v];
    for (uint32_t s = 0; s < nq; s++)
      if (L[v * MBQ + s] >= 0 && src[s] != v) x += DL[v * MBQ + s];
    bc[v] = x;
  }
}

__global__ void k_mb_init(int32_t* L, unsigned long long* SG, uint32_t* nm0, uint32_t* nm1, uint64_t V,
                          BwdHead* head) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *head = BwdHead{};
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V * MBQ; i += (uint64_t)gridDim.x * blockDim.x) {
    L[i] = -1;
    SG[i] = 0ull;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (uint64_t)gridDim.x * blockDim.x) {
    nm0[i] = 0u;
    nm1[i] = 0u;
  }
}

// Level 0: each distinct source with the mask of its group positions (the
// sources of one BC query are distinct), tag 1; the level-0 vertex list.
// One wave.
__global__ void k_mb_seed(Store st, const uint32_t* src, uint32_t n, int32_t* L, unsigned long long* SG,
                          uint32_t* nm, uint32_t* order, Front f, QCounters* cnt, QCounters* other) {
  __shared__ Shared sh;
  if (threadIdx.x == 0) {
    zero_counters(cnt);
    zero_counters(other);
  }
  __syncthreads();
  ItemQ qn = item_q(sh.ws[0], 0, WSTAGE);
  const uint32_t i = lane_id();
  uint32_t v = 0;
  uint64_t vd = 0;
  if (i < n) {
    v = src[i];
    L[(uint64_t)v * MBQ + i] = 0;
    SG[(uint64_t)v * MBQ + i] = 1ull;
    nm[v] = (1u << 16) | (1u << i);
    order[i] = v;
    vd = st.fdesc[v];
  }
  push_item(qn, i < n, v, vd);
  flush_front(qn, f, cnt);
  if (i == 0) cnt->n_order = n;
}

struct MbHost {
  QCounters c;
  uint32_t seq;
};

__global__ void k_mb_tile_flag(const BwdHead* head, QCounters* c) {
  if (threadIdx.x == 0) c->overflow = head->ovf;
}

__global__ void k_mb_publish(const QCounters* c, MbHost* h, uint32_t seq) {
  if (threadIdx.x != 0) return;
  h->c = *c;
  __threadfence_system();
  __hip_atomic_store(&h->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

static uint64_t mb_al(uint64_t x) { return (x + 255) & ~255ull; }

struct MbLayout {
  int32_t* L;
  unsigned long long* SG;
  double* DL;
  double* CL;   // (1 + DL) / SG of each finished (vertex, source)
  uint32_t *nm[2], *order;
  uint64_t order_cap;
  Item* q[2];
  uint32_t* cmap[2];
  QCounters* cnt;
  uint32_t* src;
  BwdTiles bt;
};

static uint64_t mb_layout(const Store& st, char* base, MbLayout* P) {
  const uint64_t V = st.V;
  const uint64_t items = V + 1024;
  const uint64_t chunks = st.fp.cap / CH_MIN + 2;
  // a vertex joins the list of each level where some source first reaches it
  const uint64_t order_cap = std::min<uint64_t>(MBQ * V + 1024, 0xFFFFFFFFull);
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o += mb_al(bytes);
    return base ? base + at : nullptr;
  };
  char* p;
  p = take(V * MBQ * 4); if (P) P->L = reinterpret_cast<int32_t*>(p);
  p = take(V * MBQ * 8); if (P) P->SG = reinterpret_cast<unsigned long long*>(p);
  p = take(V * MBQ * 8); if (P) P->DL = reinterpret_cast<double*>(p);
  p = take(V * MBQ * 8); if (P) P->CL = reinterpret_cast<double*>(p);
  for (int i = 0; i < 2; i++) { p = take(V * 4 + 64); if (P) P->nm[i] = reinterpret_cast<uint32_t*>(p); }
  p = take(order_cap * 4); if (P) { P->order = reinterpret_cast<uint32_t*>(p); P->order_cap = order_cap; }
  for (int i = 0; i < 2; i++) { p = take(items * sizeof(Item)); if (P) P->q[i] = reinterpret_cast<Item*>(p); }
  for (int i = 0; i < 2; i++) { p = take(chunks * 4); if (P) P->cmap[i] = reinterpret_cast<uint32_t*>(p); }
  p = take(2 * sizeof(QCounters)); if (P) P->cnt = reinterpret_cast<QCounters*>(p);
  p = take(MBQ * 4); if (P) P->src = reinterpret_cast<uint32_t*>(p);
  p = take(bwd_tiles_bytes(st.fp.cap, MBQ)); if (P) P->bt = bwd_tiles_at(p, st.fp.cap, MBQ);
  return o;
}

uint32_t ms_bc_width() { return MBQ; }

void free_mb_scratch(MbScratch& mb) {
  release(mb.area);
  if (mb.host) hipHostFree(mb.host);
  mb.host = nullptr;
}

static uint32_t mb_resident(const void* kernel) {
  int per_cu = 0, cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, Q_THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)std::max(1, per_cu * cus);
}

dg_status ms_bc_dev(dg_graph* g, const Store& st, uint32_t e, int fast, const uint32_t* srcs, uint32_t k, double* bc,
                    uint32_t chunk_buckets, MbScratch& mb, hipStream_t s, uint64_t* arcs_out) {
  auto fail = [&](dg_status code, const std::string& m) {
    g->err = "multi-source bc: " + m;
    return code;
  };
  if (k == 0) return DG_OK;
  if (k > MBQ) return fail(DG_E_INVALID_ARG, "more than 16 sources in a group");
  hipError_t he;
  if ((he = ensure(mb.area, mb_layout(st, nullptr, nullptr))) != hipSuccess)
    return fail(DG_E_OUT_OF_MEMORY, "scratch allocation");
  if (!mb.host) {
    if ((he = hipHostMalloc(&mb.host, sizeof(MbHost), hipHostMallocCoherent)) != hipSuccess) {
      mb.host = nullptr;
      return fail(DG_E_OUT_OF_MEMORY, "pinned counter block");
    }
    std::memset(mb.host, 0, sizeof(MbHost));
    mb.seq = 0;
  }
  if (!mb.fwd_grid) {
    mb.fwd_grid = mb_resident((const void*)k_mb_fwd);
    mb.bwd_grid = mb_resident((const void*)k_mb_bwd);
    mb.tiles_grid = mb_resident((const void*)k_mb_tiles);
  }
  MbLayout P;
  mb_layout(st, mb.area.as<char>(), &P);
  const uint32_t lch = 31 - __builtin_clz(std::max<uint32_t>(16, std::min<uint32_t>(64, chunk_buckets)));
  const uint32_t qcap = (uint32_t)std::min<uint64_t>(st.V + 1024, 0xFFFFFFFFu);
  const uint32_t ccap = (uint32_t)std::min<uint64_t>(st.fp.cap / CH_MIN + 2, 0xFFFFFFFFu);
  Front fr[2] = {Front{P.q[0], P.cmap[0], qcap, ccap, lch}, Front{P.q[1], P.cmap[1], qcap, ccap, lch}};
  const uint64_t V = st.V;
  k_mb_init<<<(uint32_t)std::min<uint64_t>((V * MBQ + 255) / 256, 8192), 256, 0, s>>>(P.L, P.SG, P.nm[0], P.nm[1], V, P.bt.head);
  if ((he = hipMemcpyAsync(P.src, srcs, k * 4, hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail(DG_E_HIP, std::string("upload: ") + hipGetErrorString(he));
  k_mb_seed<<<1, 64, 0, s>>>(st, P.src, k, P.L, P.SG, P.nm[0], P.order, fr[0], &P.cnt[0], &P.cnt[1]);
  MbHost* h = static_cast<MbHost*>(mb.host);
  auto read = [&](int slot, QCounters* out) -> hipError_t {
    const uint32_t seq = ++mb.seq;
    k_mb_publish<<<1, 64, 0, s>>>(&P.cnt[slot], h, seq);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t spin = 1; __atomic_load_n(&h->seq, __ATOMIC_ACQUIRE) != seq; spin++) {
      host_pause(spin);
      if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
        if ((r = hipStreamSynchronize(s)) != hipSuccess) return r;
        if (__atomic_load_n(&h->seq, __ATOMIC_ACQUIRE) != seq) return hipErrorUnknown;
        break;
      }
    }
    std::memcpy(out, &h->c, sizeof(QCounters));
    return hipSuccess;
  };
  QCounters hc;
  if ((he = read(0, &hc)) != hipSuccess) return fail(DG_E_HIP, std::string("seed: ") + hipGetErrorString(he));
  // off[l] .. off[l + 1]: the vertex list of level l in order[]
  std::vector<uint64_t> off{0, k};
  std::vector<uint32_t> nbig{1};   // listed (long-slab) vertices per level; the sources are not counted
  unsigned long long near = hc.fq;
  int slot = 0, qi = 0;
  uint32_t tag = 1;
  uint64_t arcs = 0;
  for (int32_t lvl = 0; near; lvl++) {
    yield_to_updates(g);
    if (tag >= MB_TAG_MAX) return fail(DG_E_HIP, "level count exceeds the mask tag range");
    const int nxt = slot ^ 1;
    const uint64_t used = off.back();
    MbFwd a{st,   e,          fast,          fr[qi],  fr[qi ^ 1], P.L, P.SG, P.nm[(tag - 1) & 1], P.nm[tag & 1],
            P.order + used, (uint32_t)std::min<uint64_t>(P.order_cap - used, 0xFFFFFFFFu), tag, tag + 1, lvl + 1, k,
            &P.cnt[nxt], &P.cnt[slot]};
    const uint32_t nc = fq_chunks(near, lch);
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((nc + Q_WAVES - 1) / Q_WAVES, mb.fwd_grid));
    {
      ProfScope ps(g, KID_BATCH_BC, s);
      k_mb_fwd<<<grid, Q_THREADS, 0, s>>>(a, near);
    }
    if ((he = hipGetLastError()) != hipSuccess || (he = read(nxt, &hc)) != hipSuccess)
      return fail(DG_E_HIP, std::string("forward: ") + hipGetErrorString(he));
    if (hc.overflow & OVF_QUEUE) return fail(DG_E_OUT_OF_MEMORY, "frontier queue capacity exceeded");
    if (hc.overflow & OVF_SIGMA) {
      g->err = "multi-source bc: a shortest-path count exceeded int64";
      return DG_E_OVERFLOW;
    }
    if (used + hc.n_order > P.order_cap) return fail(DG_E_OUT_OF_MEMORY, "level list capacity exceeded");
    arcs += hc.arcs;
    if (hc.n_order) {
      off.push_back(used + hc.n_order);
      nbig.push_back(hc.n_far);
    }
    near = hc.fq;
    slot = nxt;
    qi ^= 1;
    tag++;
    if (!hc.n_order) break;
  }
  // levels in decreasing order (k_mb_init zeroed the tile counts)
  ProfScope ps(g, KID_BATCH_BC, s);
  for (int32_t lvl = (int32_t)off.size() - 2; lvl >= 0; lvl--) {
    yield_to_updates(g);
    const uint64_t o0 = off[lvl], n = off[lvl + 1] - off[lvl];
    if (!n) continue;
    const uint32_t grid =
        std::max<uint32_t>(1, std::min<uint32_t>((uint32_t)((n + Q_WAVES - 1) / Q_WAVES), mb.bwd_grid));
    k_mb_bwd<<<grid, Q_THREADS, 0, s>>>(st, e, fast, P.order + o0, (uint32_t)n, lvl, k, P.L, P.SG, P.DL, P.CL, P.bt);
    // the forward's count of long slabs is exact only while no update can
    // move a slab in between
    if (nbig[lvl] || !fast) {
      k_mb_tiles<<<mb.tiles_grid, Q_THREADS, 0, s>>>(st, e, fast, lvl, k, P.L, P.SG, P.CL, P.bt);
      const uint64_t lanes = (uint64_t)std::max<uint32_t>(nbig[lvl], fast ? 0u : 4096u) * MBQ;
      k_mb_combine<<<(uint32_t)std::min<uint64_t>((lanes + Q_THREADS - 1) / Q_THREADS, 4096), Q_THREADS, 0, s>>>(
          lvl, k, P.L, P.SG, P.DL, P.CL, P.bt);
    }
  }
  k_mb_accum<<<(uint32_t)std::min<uint64_t>((V + 255) / 256, 4096), 256, 0, s>>>(P.L, P.DL, P.src, k, V, bc);
  if ((he = hipGetLastError()) != hipSuccess) return fail(DG_E_HIP, std::string("backward: ") + hipGetErrorString(he));
  // the tile lists' overflow flag (their capacity covers every level)
  k_mb_tile_flag<<<1, 64, 0, s>>>(P.bt.head, &P.cnt[0]);
  if ((he = hipGetLastError()) != hipSuccess || (he = read(0, &hc)) != hipSuccess)
    return fail(DG_E_HIP, std::string("backward: ") + hipGetErrorString(he));
  if (hc.overflow) return fail(DG_E_OUT_OF_MEMORY, "backward tile list capacity exceeded");
  if (arcs_out) *arcs_out += arcs;
  return DG_OK;
}

}  // namespace dg
