// Multi-source SSSP: up to MSQ single-source SSSP queries on one snapshot
// run as one delta-stepping search over a shared vertex frontier.
//
// Each vertex holds the MSQ = 32 queries' tentative distances in one
// 128-byte record (one cache line), D[v * MSQ + q].  A frontier item is a
// vertex with a mask of the queries for which it was improved below the
// current threshold; scanning its arcs once serves every query in the mask:
// for arc (u, w, d), lane q of a 32-lane half-wave reads D[d * MSQ + q] (one
// line for the half), and relaxes query q when u is in q's mask.  Improvements below the threshold
// OR the query's bit into d's mask for the next pass (the first bit set
// enqueues d); improvements at or above it OR the bit into d's far mask
// (the first bit set puts d on the far pile).  When the near frontier is
// empty the threshold rises by delta (or straight past the smallest far
// distance) and the pile is split: bits whose distance fell below the
// threshold move into the near masks, the rest stay.
//
// Near masks carry the pass that wrote them in their upper 32 bits
// (tag << 32 | bits) and alternate between two arrays, so a pass reads the
// masks the previous pass wrote while it writes the next ones, and no
// array ever needs clearing.  Far masks are rewritten only by the split,
// which owns each piled vertex exactly once.
//
// Relaxations are atomicMin on int32 and only lower distances, so every
// query's result is the exact shortest-path distance whatever the order;
// it equals the plain path's (and the oracle's) bit for bit.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dg_host.h"
#include "frontier.h"

namespace dg {

constexpr uint32_t MSQ = 32;
constexpr uint32_t MS_TAG_MAX = 0xFFFFFFF0u;
typedef unsigned long long u64;

struct MsPass {
  Store st;
  uint32_t e;
  int fast;
  Front fin, fout;
  int32_t* D;              // V * MSQ distances
  const u64* nm_in;        // masks of fin's vertices (tag_in)
  u64* nm_out;             // masks of fout's vertices (tag_out)
  uint32_t* fm;            // far masks
  uint32_t* pile;          // far pile entries appended by this pass
  uint32_t tag_in, tag_out;
  int32_t thr;
  uint32_t nq;             // queries in the group (lanes q >= nq idle)
  QCounters* cnt_out;      // fq of fout, n_order = pile appends, arcs = relaxations
  QCounters* reset;        // the other counter slot, cleared for the next pass
};

__device__ inline void ms_reset(QCounters* c) {
  if (blockIdx.x == 0 && threadIdx.x == 0) zero_counters(c);
}

// ORs bits into v's mask for tag (a mask of an older tag is replaced);
// returns true for the caller that set the first bit of this tag.
__device__ inline bool ms_mark(u64* nm, uint32_t v, uint32_t tag, uint32_t bits) {
  u64 old = __hip_atomic_load(&nm[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const bool same = (uint32_t)(old >> 32) == tag;
    const u64 nw = same ? (old | bits) : (((u64)tag << 32) | bits);
    if (nw == old) return false;
    const u64 prev = atomicCAS(&nm[v], old, nw);
    if (prev == old) return !same;
    old = prev;
  }
}

// 32-bit mask of the lanes of this lane's half-wave for which pred holds.
__device__ inline uint32_t half_ballot(bool pred) {
  return (uint32_t)(__ballot(pred) >> (threadIdx.x & 32));
}

// x[k] for a wave-uniform k, without indexing a register array.
template <class T>
__device__ inline T pick4(const T (&x)[4], int k) {
  return k == 0 ? x[0] : (k == 1 ? x[1] : (k == 2 ? x[2] : x[3]));
}

// One chunk of the near frontier.  load_pairs gives each 16-lane group the
// 16 slots of buckets f0 + 4 grp + k; half-wave h (lanes 32 h .. 32 h + 31)
// holds the buckets of groups 2h and 2h + 1, 32 arcs per k.  Lane q of the
// half relaxes query q over those 32 arcs, one after another (two owners:
// arcs 0..15 belong to the first bucket, 16..31 to the second), and lane s
// then publishes arc s's mask bits.
__device__ __forceinline__ void ms_relax_chunk(const MsPass& a, uint32_t c, uint32_t nitems, uint32_t nb, ItemQ& qn,
                                               U32Q& qp, LaneCounts& lc) {
  const uint32_t j = threadIdx.x & 31, hb = threadIdx.x & 32, grp = (threadIdx.x >> 4) & 3;
  const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
  uint32_t mk_l = 0;
  if (touches(cv)) {
    const u64 t = a.nm_in[cv.v];
    mk_l = (uint32_t)(t >> 32) == a.tag_in ? (uint32_t)t : 0u;
  }
  for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
    Pairs4 s4 = load_pairs<true>(a.st.fp, cv, f0, grp, threadIdx.x & 15, a.e, a.fast);
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
      const uint32_t it_k = pick4(s4.item, k), d_k = pick4(s4.d, k);
      const int32_t w_k = pick4(s4.w, k);
      const int vis_k = pick4(s4.vis, k) ? 1 : 0;
      // the two buckets' owners, their masks and this lane's query's distances
      uint32_t own[2];
      int32_t du[2];
      bool mine[2];
#pragma unroll
      for (int b = 0; b < 2; b++) {
        const int src_lane = (int)(hb + 16 * b);
        const uint32_t itb = __shfl(it_k, src_lane, 64);
        own[b] = __shfl(cv.v, (int)itb, 64);
        const uint32_t mk = __shfl(mk_l, (int)itb, 64);
        mine[b] = j < a.nq && ((mk >> j) & 1u);
        du[b] = mine[b] ? a.D[(uint64_t)own[b] * MSQ + j] : 0;
      }
      // the 32 arcs in four quarters of 8 (registers), each quarter's reads
      // and atomics issued together
      uint32_t my_near = 0, my_far = 0;
#pragma unroll 1
      for (int h = 0; h < 32; h += 8) {
        const int b = h >> 4;   // which bucket (owner) these arcs belong to
        const bool mb = b ? mine[1] : mine[0];
        const int32_t dub = b ? du[1] : du[0];
        uint32_t dd[8];
        int32_t nd[8], cur[8];
        bool act[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
          dd[t] = __shfl(d_k, (int)(hb + h + t), 64);
          const int32_t w = __shfl(w_k, (int)(hb + h + t), 64);
          const bool vis = __shfl(vis_k, (int)(hb + h + t), 64) != 0;
          act[t] = vis && mb;
          nd[t] = dub + w;
          cur[t] = act[t] ? a.D[(uint64_t)dd[t] * MSQ + j] : 0;
          lc.arcs += act[t] ? 1 : 0;          // relaxations (arc, query)
          lc.m += (j == 0 && vis) ? 1 : 0;    // arcs scanned, once for the half
        }
        // the atomicMin's result is not waited for: a tentative distance
        // that beats the read value counts as an improvement even when a
        // racing arc lowered the target further, which at worst sets a near
        // or far bit that the racing arc sets too (bits, so no duplicate
        // queue entry); distances only fall, so every result stays exact
#pragma unroll
        for (int t = 0; t < 8; t++)
          if (act[t] && nd[t] < cur[t]) atomicMin(&a.D[(uint64_t)dd[t] * MSQ + j], nd[t]);
        // lane s collects arc s's improved queries: near bits and far bits
#pragma unroll
        for (int t = 0; t < 8; t++) {
          const bool imp = act[t] && nd[t] < cur[t];
          const uint32_t nbits = half_ballot(imp && nd[t] < a.thr);
          const uint32_t fbits = half_ballot(imp && nd[t] >= a.thr);
          if (j == (uint32_t)(h + t)) {
            my_near = nbits;
            my_far = fbits;
          }
        }
      }
      const uint32_t d = d_k;
      const bool first_near = my_near && ms_mark(a.nm_out, d, a.tag_out, my_near);
      const bool first_far = my_far && atomicOr(&a.fm[d], my_far) == 0u;
      const uint64_t yd = first_near ? a.st.fdesc[d] : 0;
      room_front(qn, 64, a.fout, a.cnt_out);
      push_item(qn, first_near, d, yd);
      room_u32(qp, 64, a.pile, &a.cnt_out->n_order);
      push_u32(qp, first_far, d);
    }
  }
}

__global__ __launch_bounds__(Q_THREADS) __attribute__((amdgpu_waves_per_eu(5))) void k_ms_relax(MsPass a, unsigned long long nfq) {
  __shared__ Shared sh;
  ms_reset(a.reset);
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * Q_WAVES + wave, nw = gridDim.x * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  // the item stage and the pile stage share the wave's staging area
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  U32Q qp = u32_q(sh.ws[wave]);
  LaneCounts lc;
  for (uint32_t c = gw; c < nc; c += nw) ms_relax_chunk(a, c, nitems, nb, qn, qp, lc);
  flush_u32_q(qp, a.pile, &a.cnt_out->n_order);
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  lc.commit(a.cnt_out, sh);
}

struct MsSplit {
  Store st;
  Front fout;
  int32_t* D;
  u64* nm_out;
  uint32_t* fm;
  const uint32_t* pile_in;
  uint32_t n_in;
  uint32_t* pile_out;
  uint32_t tag_out;
  int32_t thr_old;      // the threshold of the bucket just settled
  int32_t thr;
  QCounters* cnt_out;   // fq, n_order = entries kept, far_min = least kept distance
  QCounters* reset;
};

// One lane per pile entry: the far bits whose distance now lies in
// [thr_old, thr) become the vertex's near mask, those at or above thr stay
// on the pile, and those below thr_old are dropped: such a distance was
// reached below the threshold then in force, so it went through the near
// frontier and its arcs were relaxed from it (relaxations do not clear far
// bits).
__global__ __launch_bounds__(Q_THREADS) void k_ms_split(MsSplit a) {
  __shared__ Shared sh;
  ms_reset(a.reset);
  const uint32_t wave = threadIdx.x >> 6;
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  U32Q qp = u32_q(sh.ws[wave]);
  int32_t mn = DIST_INF;
  const uint32_t stride = gridDim.x * Q_THREADS;
  for (uint32_t base = blockIdx.x * Q_THREADS + wave * 64; base < a.n_in; base += stride) {
    const uint32_t i = base + lane_id();
    uint32_t v = 0, near = 0, keep = 0;
    if (i < a.n_in) {
      v = a.pile_in[i];
      const uint32_t f = a.fm[v];
      for (uint32_t b = f; b; b &= b - 1) {
        const uint32_t q = __ffs(b) - 1;
        const int32_t dq = a.D[(uint64_t)v * MSQ + q];
        if (dq >= a.thr) {
          keep |= 1u << q;
          mn = min(mn, dq);
        } else if (dq >= a.thr_old) {
          near |= 1u << q;
        }
      }
      a.fm[v] = keep;
      if (near) a.nm_out[v] = ((u64)a.tag_out << 32) | near;
    }
    const uint64_t vd = near ? a.st.fdesc[v] : 0;
    room_front(qn, 64, a.fout, a.cnt_out);
    push_item(qn, near != 0, v, vd);
    room_u32(qp, 64, a.pile_out, &a.cnt_out->n_order);
    push_u32(qp, keep != 0, v);
  }
  flush_u32_q(qp, a.pile_out, &a.cnt_out->n_order);
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  commit_far_min(mn, a.cnt_out);
}

__global__ void k_ms_init(int32_t* D, u64* nm0, u64* nm1, uint32_t* fm, uint64_t V) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V * MSQ; i += (uint64_t)gridDim.x * blockDim.x)
    D[i] = DIST_INF;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (uint64_t)gridDim.x * blockDim.x) {
    nm0[i] = 0ull;
    nm1[i] = 0ull;
    fm[i] = 0u;
  }
}

// The seed frontier: each distinct source with the mask of its queries
// (tag 1), at distance 0 for them.  One wave.
__global__ void k_ms_seed(Store st, const uint32_t* src, const uint32_t* mask, uint32_t n, int32_t* D, u64* nm,
                          Front f, QCounters* cnt, QCounters* other) {
  __shared__ Shared sh;
  if (threadIdx.x == 0) {
    zero_counters(cnt);
    zero_counters(other);
  }
  __syncthreads();
  ItemQ qn = item_q(sh.ws[0], 0, WSTAGE);
  for (uint32_t base = 0; base < n; base += 64) {
    const uint32_t i = base + lane_id();
    uint32_t v = 0;
    uint64_t vd = 0;
    if (i < n) {
      v = src[i];
      nm[v] = (1ull << 32) | mask[i];
      for (uint32_t b = mask[i]; b; b &= b - 1) D[(uint64_t)v * MSQ + (__ffs(b) - 1)] = 0;
      vd = st.fdesc[v];
    }
    room_front(qn, 64, f, cnt);
    push_item(qn, i < n, v, vd);
  }
  flush_front(qn, f, cnt);
}

// Each query's distances into its output, -1 where unreached: a block
// reads 64 vertices' records in order (8 KiB) into LDS and writes each
// query's 64 distances as one run, so D is read once and every store is
// coalesced.
__global__ __launch_bounds__(256) void k_ms_extract(const int32_t* D, uint64_t V, int32_t* const* outs, uint32_t k) {
  __shared__ int32_t t[64][MSQ + 1];
  for (uint64_t v0 = (uint64_t)blockIdx.x * 64; v0 < V; v0 += (uint64_t)gridDim.x * 64) {
    for (uint32_t i = threadIdx.x; i < 64 * MSQ; i += 256)
      t[i / MSQ][i % MSQ] = v0 + i / MSQ < V ? D[v0 * MSQ + i] : DIST_INF;
    __syncthreads();
    const uint32_t r = threadIdx.x & 63;
    for (uint32_t q = threadIdx.x >> 6; q < k; q += 4) {
      if (v0 + r < V) {
        const int32_t x = t[r][q];
        outs[q][v0 + r] = x == DIST_INF ? -1 : x;
      }
    }
    __syncthreads();
  }
}

// One slot's counters into coherent pinned host memory, sequence number
// last.
struct MsHost {
  QCounters c;
  uint32_t seq;
};

__global__ void k_ms_publish(const QCounters* c, MsHost* h, uint32_t seq) {
  if (threadIdx.x != 0) return;
  h->c = *c;
  __threadfence_system();
  __hip_atomic_store(&h->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

static uint64_t al256(uint64_t x) { return (x + 255) & ~255ull; }

// Buffers of one group search, carved from ms.area.
struct MsLayout {
  int32_t* D;
  u64* nm[2];
  uint32_t *fm, *pile[2];
  Item* q[2];
  uint32_t* cmap[2];
  QCounters* cnt;        // two slots
  int32_t** outs;        // MSQ output pointers
  uint32_t *src, *mask;  // seed sources and masks
};

static uint64_t ms_layout(const Store& st, char* base, MsLayout* L) {
  const uint64_t V = st.V;
  const uint64_t items = V + 1024;
  const uint64_t chunks = st.fp.cap / CH_MIN + 2;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o += al256(bytes);
    return base ? base + at : nullptr;
  };
  char* p;
  p = take(V * MSQ * 4); if (L) L->D = reinterpret_cast<int32_t*>(p);
  for (int i = 0; i < 2; i++) { p = take(V * 8 + 64); if (L) L->nm[i] = reinterpret_cast<u64*>(p); }
  p = take(V * 4 + 64); if (L) L->fm = reinterpret_cast<uint32_t*>(p);
  for (int i = 0; i < 2; i++) { p = take(V * 4 + 64); if (L) L->pile[i] = reinterpret_cast<uint32_t*>(p); }
  for (int i = 0; i < 2; i++) { p = take(items * sizeof(Item)); if (L) L->q[i] = reinterpret_cast<Item*>(p); }
  for (int i = 0; i < 2; i++) { p = take(chunks * 4); if (L) L->cmap[i] = reinterpret_cast<uint32_t*>(p); }
  p = take(2 * sizeof(QCounters)); if (L) L->cnt = reinterpret_cast<QCounters*>(p);
  p = take(MSQ * sizeof(void*)); if (L) L->outs = reinterpret_cast<int32_t**>(p);
  p = take(MSQ * 4); if (L) L->src = reinterpret_cast<uint32_t*>(p);
  p = take(MSQ * 4); if (L) L->mask = reinterpret_cast<uint32_t*>(p);
  return o;
}

uint32_t ms_sssp_width() { return MSQ; }

void free_ms_scratch(MsScratch& ms) {
  release(ms.area);
  if (ms.host) hipHostFree(ms.host);
  ms.host = nullptr;
}

// Workgroups of `kernel` resident at once on the current device.
static uint32_t ms_resident(const void* kernel) {
  int per_cu = 0, cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, Q_THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)std::max(1, per_cu * cus);
}

dg_status ms_sssp_dev(dg_graph* g, const Store& st, uint32_t e, int fast, const uint32_t* srcs, uint32_t k,
                      void* const* outs, int32_t delta, uint32_t chunk_buckets, MsScratch& ms, hipStream_t s,
                      uint64_t* arcs_out) {
  auto fail = [&](dg_status code, const std::string& m) {
    g->err = "multi-source sssp: " + m;
    return code;
  };
  if (k == 0) return DG_OK;
  if (k > MSQ) return fail(DG_E_INVALID_ARG, "more than 32 queries in a group");
  hipError_t he;
  const uint64_t need = ms_layout(st, nullptr, nullptr);
  if ((he = ensure(ms.area, need)) != hipSuccess) return fail(DG_E_OUT_OF_MEMORY, "scratch allocation");
  if (!ms.host) {
    if ((he = hipHostMalloc(&ms.host, sizeof(MsHost), hipHostMallocCoherent)) != hipSuccess) {
      ms.host = nullptr;
      return fail(DG_E_OUT_OF_MEMORY, "pinned counter block");
    }
    std::memset(ms.host, 0, sizeof(MsHost));
    ms.seq = 0;
  }
  if (!ms.relax_grid) {
    ms.relax_grid = ms_resident((const void*)k_ms_relax);
    ms.split_grid = ms_resident((const void*)k_ms_split);
  }
  MsLayout L;
  ms_layout(st, ms.area.as<char>(), &L);
  const uint32_t lch = 31 - __builtin_clz(std::max<uint32_t>(16, std::min<uint32_t>(64, chunk_buckets)));
  const uint32_t qcap = (uint32_t)std::min<uint64_t>(st.V + 1024, 0xFFFFFFFFu);
  const uint32_t ccap = (uint32_t)std::min<uint64_t>(st.fp.cap / CH_MIN + 2, 0xFFFFFFFFu);
  Front fr[2] = {Front{L.q[0], L.cmap[0], qcap, ccap, lch}, Front{L.q[1], L.cmap[1], qcap, ccap, lch}};
  // seed: distinct sources with the masks of their queries
  std::vector<uint32_t> usrc, umask;
  for (uint32_t q = 0; q < k; q++) {
    auto it = std::find(usrc.begin(), usrc.end(), srcs[q]);
    if (it == usrc.end()) {
      usrc.push_back(srcs[q]);
      umask.push_back(1u << q);
    } else {
      umask[it - usrc.begin()] |= 1u << q;
    }
  }
  const uint64_t V = st.V;
  k_ms_init<<<(uint32_t)std::min<uint64_t>((V * MSQ + 255) / 256, 8192), 256, 0, s>>>(L.D, L.nm[0], L.nm[1], L.fm, V);
  if ((he = hipMemcpyAsync(L.src, usrc.data(), usrc.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (he = hipMemcpyAsync(L.mask, umask.data(), umask.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (he = hipMemcpyAsync(L.outs, outs, k * sizeof(void*), hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail(DG_E_HIP, std::string("upload: ") + hipGetErrorString(he));
  k_ms_seed<<<1, 64, 0, s>>>(st, L.src, L.mask, (uint32_t)usrc.size(), L.D, L.nm[0], fr[0], &L.cnt[0], &L.cnt[1]);
  MsHost* h = static_cast<MsHost*>(ms.host);
  auto read = [&](int slot, QCounters* out) -> hipError_t {
    const uint32_t seq = ++ms.seq;
    k_ms_publish<<<1, 64, 0, s>>>(&L.cnt[slot], h, seq);
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
  unsigned long long near = hc.fq;
  int slot = 0, qi = 0, pi = 0;
  uint32_t tag = 1, n_pile = 0;
  int32_t thr = std::max<int32_t>(1, delta);
  uint64_t arcs = 0, scanned = 0;
  for (;;) {
    if (tag >= MS_TAG_MAX) return fail(DG_E_HIP, "pass count exceeds the mask tag range");
    yield_to_updates(g);
    if (near) {
      const int nxt = slot ^ 1;
      MsPass a{st,        e,         fast,        fr[qi],  fr[qi ^ 1], L.D,           L.nm[(tag - 1) & 1],
               L.nm[tag & 1], L.fm, L.pile[pi] + n_pile, tag, tag + 1, thr, k, &L.cnt[nxt], &L.cnt[slot]};
      const uint32_t nc = fq_chunks(near, lch);
      const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((nc + Q_WAVES - 1) / Q_WAVES, ms.relax_grid));
      {
        ProfScope ps(g, KID_BATCH_SSSP, s);
        k_ms_relax<<<grid, Q_THREADS, 0, s>>>(a, near);
      }
      if ((he = hipGetLastError()) != hipSuccess || (he = read(nxt, &hc)) != hipSuccess)
        return fail(DG_E_HIP, std::string("relax: ") + hipGetErrorString(he));
      if (hc.overflow & OVF_QUEUE) return fail(DG_E_OUT_OF_MEMORY, "frontier queue capacity exceeded");
      arcs += hc.arcs;
      scanned += hc.m_next;
      near = hc.fq;
      n_pile += hc.n_order;
      slot = nxt;
      qi ^= 1;
      tag++;
      continue;
    }
    if (n_pile == 0) break;
    // raise the threshold and split the pile until something is near
    int32_t far_min = DIST_INF;
    do {
      if (tag >= MS_TAG_MAX) return fail(DG_E_HIP, "pass count exceeds the mask tag range");
      const int32_t thr_old = thr;
      thr = far_min == DIST_INF ? (int32_t)std::min<int64_t>(DIST_INF, (int64_t)thr + delta)
                                : (int32_t)std::min<int64_t>(DIST_INF, ((int64_t)far_min / delta + 1) * delta);
      const int nxt = slot ^ 1;
      // the split's near masks carry the tag the next pass reads
      MsSplit a{st,  fr[qi],  L.D, L.nm[(tag - 1) & 1], L.fm,        L.pile[pi], n_pile, L.pile[pi ^ 1],
                tag, thr_old, thr, &L.cnt[nxt],         &L.cnt[slot]};
      const uint32_t grid =
          std::max<uint32_t>(1, std::min<uint32_t>((n_pile + Q_THREADS - 1) / Q_THREADS, ms.split_grid));
      k_ms_split<<<grid, Q_THREADS, 0, s>>>(a);
      if ((he = hipGetLastError()) != hipSuccess || (he = read(nxt, &hc)) != hipSuccess)
        return fail(DG_E_HIP, std::string("split: ") + hipGetErrorString(he));
      if (hc.overflow & OVF_QUEUE) return fail(DG_E_OUT_OF_MEMORY, "frontier queue capacity exceeded");
      slot = nxt;
      pi ^= 1;
      n_pile = hc.n_order;
      near = hc.fq;
      far_min = hc.far_min;
    } while (!near && n_pile > 0);
  }
  k_ms_extract<<<(uint32_t)std::min<uint64_t>((V + 63) / 64, 8192), 256, 0, s>>>(L.D, V, L.outs, k);
  if ((he = hipGetLastError()) != hipSuccess) return fail(DG_E_HIP, std::string("extract: ") + hipGetErrorString(he));
  if (arcs_out) *arcs_out += arcs;
  prof_scans(g, KID_BATCH_SSSP_SCAN, scanned);
  return DG_OK;
}

}  // namespace dg
