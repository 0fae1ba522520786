// Multi-source BFS: up to 64 BFS queries on one snapshot as one
// level-synchronous search over a shared frontier, driven by the host one
// level at a time (a kernel boundary is the level barrier).
//
// Each vertex keeps one 16-byte record {visited mask, next-level mask} and a
// frontier mask, one bit per query.  A level's expansion (`k_mf_pass`)
// scans each frontier vertex's arcs once for all its queries: for a visible
// arc (u, v) it ORs fr[u] & ~visited[v] into v's next mask, and the first
// bit set lists v as touched and queues its slab for the next level.  The
// level's finish (`k_mf_final`) moves each touched vertex's new bits into
// its visited mask and frontier mask and records the level of each new
// query in the vertex's 64-byte level record (one line per vertex, one byte
// per query); `k_mf_extract` then writes every query's distance array in
// coalesced runs.  Query q's distance at v is the first level at which q's
// bit reaches v, which is its BFS hop distance.  Levels from MF_DIRECT on
// do not fit a byte: they go straight to the output, and the record marks
// the entry as written.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dg_host.h"
#include "frontier.h"

namespace dg {

namespace {

constexpr uint32_t MFQ = 64;
constexpr uint8_t MF_UNREACHED = 0xFF;
constexpr uint8_t MF_WRITTEN = 0xFE;   // the level went to the output directly
constexpr int32_t MF_DIRECT = 0xFE;    // levels >= this are written directly

struct MfHost {
  QCounters c;
  uint32_t seq;
};

__global__ void k_mf_init(unsigned long long* vn, unsigned long long* fr, uint4* lev, uint64_t V, QCounters* cnt) {
  const uint4 un = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (uint64_t)gridDim.x * blockDim.x) {
    reinterpret_cast<ulonglong2*>(vn)[i] = make_ulonglong2(0ull, 0ull);
    fr[i] = 0ull;
    for (int k = 0; k < 4; k++) lev[4 * i + k] = un;
  }
  if (blockIdx.x == 0 && threadIdx.x < 3) zero_counters(&cnt[threadIdx.x]);
}

// Level 0: query q's bit at its source, distance 0; one frontier item per
// distinct source (one wave).
__global__ void k_mf_seed(MsArgs a, unsigned long long* frm, const uint32_t* srcs, uint32_t k, uint8_t* lev) {
  __shared__ Shared sh;
  const uint32_t q = lane_id();
  bool first = false;
  uint32_t v = 0;
  if (q < k && q < MFQ) {
    v = srcs[q];
    const unsigned long long bit = 1ull << q;
    first = atomicOr(&a.vn[2 * (uint64_t)v], bit) == 0ull;
    atomicOr(&frm[v], bit);
    lev[(uint64_t)v * MFQ + q] = 0;
  }
  ItemQ qn = item_q(sh.ws[0], 0, WSTAGE);
  push_item(qn, first, v, first ? a.st.fdesc[v] : 0);
  flush_front(qn, a.fout, a.cnt_out);
}

// One level's expansion; workgroup 0 also zeroes the counters the host has
// already read (the current frontier's), which the next level writes.
__global__ __launch_bounds__(Q_THREADS) void k_mf_pass(MsArgs a, unsigned long long nfq, QCounters* consumed) {
  __shared__ Shared sh;
  if (blockIdx.x == 0 && threadIdx.x == 0) zero_counters(consumed);
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * Q_WAVES + wave, nw = gridDim.x * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  U32Q qt = u32_q(sh.ws[wave]);
  LaneCounts lc;
  for (uint32_t c = gw; c < nc; c += nw) msbfs_chunk(a, c, nitems, nb, qn, qt, lc);
  flush_u32_q(qt, a.touched, &a.cnt_out->n_far);
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  lc.commit(a.cnt_out, sh);
}

// One lane per touched vertex of the level: its new bits move into its
// visited mask and become its frontier mask, and each new query's level
// (lvl + 1) goes into the vertex's level record.
__global__ __launch_bounds__(Q_THREADS) void k_mf_final(MsArgs a, unsigned long long* frm, uint8_t* lev,
                                                        int32_t* const* outs, int32_t lvl, uint32_t touched_cap) {
  const uint32_t n = min(a.cnt_out->n_far, touched_cap);
  const int32_t L = lvl + 1;
  for (uint32_t i = blockIdx.x * Q_THREADS + threadIdx.x; i < n; i += gridDim.x * Q_THREADS) {
    const uint32_t v = a.touched[i];
    ulonglong2* rec = reinterpret_cast<ulonglong2*>(&a.vn[2 * (uint64_t)v]);
    ulonglong2 r = *rec;
    unsigned long long nw = r.y & ~r.x;
    r.x |= nw;
    r.y = 0ull;
    *rec = r;
    frm[v] = nw;
    while (nw) {
      const int b = __ffsll((long long)nw) - 1;
      nw &= nw - 1;
      if (L < MF_DIRECT) {
        lev[(uint64_t)v * MFQ + b] = (uint8_t)L;
      } else {
        outs[b][v] = L;
        lev[(uint64_t)v * MFQ + b] = MF_WRITTEN;
      }
    }
  }
}

// Every query's distances from the level records: a block reads 64
// vertices' records in order (4 KiB) into LDS and writes each query's 64
// distances as one coalesced run (-1 unreached; entries already written
// directly are left alone).
__global__ __launch_bounds__(256) void k_mf_extract(const uint8_t* lev, uint64_t V, int32_t* const* outs, uint32_t k) {
  __shared__ uint8_t t[64][MFQ + 4];
  for (uint64_t v0 = (uint64_t)blockIdx.x * 64; v0 < V; v0 += (uint64_t)gridDim.x * 64) {
    for (uint32_t i = threadIdx.x; i < 64 * MFQ / 4; i += 256) {
      const uint32_t r = i / (MFQ / 4), c = i % (MFQ / 4);
      const uint32_t x = v0 + r < V ? reinterpret_cast<const uint32_t*>(lev)[(v0 + r) * (MFQ / 4) + c] : 0xFFFFFFFFu;
      *reinterpret_cast<uint32_t*>(&t[r][4 * c]) = x;
    }
    __syncthreads();
    const uint32_t r = threadIdx.x & 63;
    for (uint32_t q = threadIdx.x >> 6; q < k; q += 4) {
      const uint8_t x = t[r][q];
      if (v0 + r < V && x != MF_WRITTEN) outs[q][v0 + r] = x == MF_UNREACHED ? -1 : (int32_t)x;
    }
    __syncthreads();
  }
}

__global__ void k_mf_publish(const QCounters* c, MfHost* h, uint32_t seq) {
  if (threadIdx.x != 0) return;
  h->c = *c;
  __threadfence_system();
  __hip_atomic_store(&h->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

uint64_t mf_al(uint64_t x) { return (x + 255) & ~255ull; }

struct MfLayout {
  unsigned long long *vn, *fr;
  uint8_t* lev;             // per vertex one level byte per query
  uint32_t* touched;
  uint32_t touched_cap;
  Item* q[2];
  uint32_t* cmap[2];
  uint64_t qcap, ccap;
  QCounters* cnt;
  uint32_t* srcs;
  int32_t** outs;
};

uint64_t mf_layout(const Store& st, char* base, MfLayout* P) {
  const uint64_t V = st.V;
  const uint64_t items = V + 1024;
  const uint64_t chunks = st.fp.cap / CH_MIN + 2;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o += mf_al(bytes);
    return base ? base + at : nullptr;
  };
  char* p;
  p = take(V * 16); if (P) P->vn = reinterpret_cast<unsigned long long*>(p);
  p = take(V * 8); if (P) P->fr = reinterpret_cast<unsigned long long*>(p);
  p = take(V * MFQ); if (P) P->lev = reinterpret_cast<uint8_t*>(p);
  p = take(items * 4); if (P) { P->touched = reinterpret_cast<uint32_t*>(p); P->touched_cap = (uint32_t)std::min<uint64_t>(items, 0xFFFFFFFFu); }
  for (int i = 0; i < 2; i++) { p = take(items * sizeof(Item)); if (P) P->q[i] = reinterpret_cast<Item*>(p); }
  for (int i = 0; i < 2; i++) { p = take(chunks * 4); if (P) P->cmap[i] = reinterpret_cast<uint32_t*>(p); }
  if (P) {
    P->qcap = items;
    P->ccap = chunks;
  }
  p = take(3 * sizeof(QCounters)); if (P) P->cnt = reinterpret_cast<QCounters*>(p);
  p = take(MFQ * 4); if (P) P->srcs = reinterpret_cast<uint32_t*>(p);
  p = take(MFQ * sizeof(void*)); if (P) P->outs = reinterpret_cast<int32_t**>(p);
  return o;
}

uint32_t mf_resident(const void* kernel) {
  int per_cu = 0, cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, Q_THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)std::max(1, per_cu * cus);
}

}  // namespace

uint32_t ms_bfs_width() { return MFQ; }

void free_mf_scratch(MfScratch& mf) {
  release(mf.area);
  if (mf.host) (void)hipHostFree(mf.host);
  mf.host = nullptr;
}

dg_status ms_bfs_dev(dg_graph* g, const Store& st, uint32_t e, int fast, const uint32_t* srcs, uint32_t k,
                     void* const* outs, uint32_t chunk_buckets, MfScratch& mf, hipStream_t s, uint64_t* arcs_out) {
  auto fail = [&](dg_status code, const std::string& m) {
    g->err = "multi-source bfs: " + m;
    return code;
  };
  if (k == 0) return DG_OK;
  if (k > MFQ) return fail(DG_E_INVALID_ARG, "more than 64 queries in a group");
  hipError_t he;
  if ((he = ensure(mf.area, mf_layout(st, nullptr, nullptr))) != hipSuccess)
    return fail(DG_E_OUT_OF_MEMORY, "scratch allocation");
  if (!mf.host) {
    if ((he = hipHostMalloc(&mf.host, sizeof(MfHost), hipHostMallocCoherent)) != hipSuccess) {
      mf.host = nullptr;
      return fail(DG_E_OUT_OF_MEMORY, "pinned counter block");
    }
    std::memset(mf.host, 0, sizeof(MfHost));
    mf.seq = 0;
  }
  if (!mf.pass_grid) {
    mf.pass_grid = mf_resident((const void*)k_mf_pass);
    mf.final_grid = mf_resident((const void*)k_mf_final);
  }
  MfLayout P;
  mf_layout(st, mf.area.as<char>(), &P);
  const uint32_t lch = 31 - __builtin_clz(std::max<uint32_t>(16, std::min<uint32_t>(64, chunk_buckets)));
  const uint32_t qcap = (uint32_t)std::min<uint64_t>(P.qcap, 0xFFFFFFFFu);
  const uint32_t ccap = (uint32_t)std::min<uint64_t>(P.ccap, 0xFFFFFFFFu);
  const Front fr[2] = {Front{P.q[0], P.cmap[0], qcap, ccap, lch}, Front{P.q[1], P.cmap[1], qcap, ccap, lch}};
  const uint64_t V = st.V;
  if ((he = hipMemcpyAsync(P.srcs, srcs, k * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (he = hipMemcpyAsync(P.outs, outs, k * sizeof(void*), hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail(DG_E_HIP, std::string("upload: ") + hipGetErrorString(he));
  k_mf_init<<<(uint32_t)std::min<uint64_t>((V + 255) / 256, 4096), 256, 0, s>>>(P.vn, P.fr,
                                                                               reinterpret_cast<uint4*>(P.lev), V, P.cnt);
  MsArgs a0{st, e, fast, fr[1], fr[0], P.fr, P.vn, P.touched, &P.cnt[0]};
  k_mf_seed<<<1, 64, 0, s>>>(a0, P.fr, P.srcs, k, P.lev);
  MfHost* h = static_cast<MfHost*>(mf.host);
  auto read = [&](QCounters* c, QCounters* out) -> hipError_t {
    const uint32_t seq = ++mf.seq;
    k_mf_publish<<<1, 64, 0, s>>>(c, h, seq);
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
  if ((he = read(&P.cnt[0], &hc)) != hipSuccess) return fail(DG_E_HIP, std::string("seed: ") + hipGetErrorString(he));
  unsigned long long fq = hc.fq;
  uint64_t arcs = 0;
  // level lvl: the frontier is in fr[lvl & 1] with counters cnt[lvl & 1];
  // the next one goes to fr[(lvl + 1) & 1] with counters cnt[(lvl + 1) & 1]
  for (int32_t lvl = 0; fq; lvl++) {
    yield_to_updates(g);
    const int cur = lvl & 1, nxt = cur ^ 1;
    const MsArgs a{st, e, fast, fr[cur], fr[nxt], P.fr, P.vn, P.touched, &P.cnt[nxt]};
    const uint32_t nc = fq_chunks(fq, lch);
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((nc + Q_WAVES - 1) / Q_WAVES, mf.pass_grid));
    {
      ProfScope ps(g, KID_BATCH_BFS, s);
      k_mf_pass<<<grid, Q_THREADS, 0, s>>>(a, fq, &P.cnt[cur]);
    }
    k_mf_final<<<mf.final_grid, Q_THREADS, 0, s>>>(a, P.fr, P.lev, P.outs, lvl, P.touched_cap);
    if ((he = hipGetLastError()) != hipSuccess || (he = read(&P.cnt[nxt], &hc)) != hipSuccess)
      return fail(DG_E_HIP, std::string("level: ") + hipGetErrorString(he));
    if (hc.overflow & OVF_QUEUE) return fail(DG_E_OUT_OF_MEMORY, "frontier queue capacity exceeded");
    arcs += hc.arcs;
    fq = hc.fq;
  }
  k_mf_extract<<<(uint32_t)std::min<uint64_t>((V + 63) / 64, 8192), 256, 0, s>>>(P.lev, V, P.outs, k);
  if ((he = hipGetLastError()) != hipSuccess) return fail(DG_E_HIP, std::string("extract: ") + hipGetErrorString(he));
  if (arcs_out) *arcs_out += arcs;
  return DG_OK;
}

}  // namespace dg
