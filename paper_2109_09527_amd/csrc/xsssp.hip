// Continuous multi-source SSSP (the serving loop's resident SSSP executor):
// kernels of one pass and its host driver.
//
// Each vertex holds the 32 slots' tentative distances in one 128-byte
// record, D[v * XSQ + q].  A frontier item is a vertex with the mask of
// slots for which its distance improved in the last pass.  For an arc
// (u, d, w) visible to slot q's epoch, lane q of a 32-lane half-wave
// relaxes D[d][q] with D[u][q] + w (integer atomicMin); the slots whose
// distance at d improved form d's mask for the next pass.  Masks carry the
// pass that wrote them in their upper 32 bits (tag << 32 | bits) and
// alternate between two arrays, so none is ever cleared.  Every improvement
// goes to the next pass (one bucket of unbounded width), so a slot has
// converged when a pass improves none of its distances.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "xdev.h"

namespace dg {

namespace {

constexpr uint32_t XSQ = XS_SLOTS;
constexpr uint32_t XS_SPARSE = 4;   // at most this many active slots: the one-lane-per-arc pass
typedef unsigned long long u64;

// ORs bits into v's mask for tag (a mask of an older tag is replaced);
// true for the caller that set the first bit of this tag.
__device__ inline bool xs_mark(u64* nm, uint32_t v, uint32_t tag, uint32_t bits) {
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
__device__ inline uint32_t xs_half_ballot(bool pred) { return (uint32_t)(__ballot(pred) >> (threadIdx.x & 32)); }

// x[k] for a wave-uniform k, without indexing a register array.
template <class T>
__device__ inline T xs_pick4(const T (&x)[4], int k) {
  return k == 0 ? x[0] : (k == 1 ? x[1] : (k == 2 ? x[2] : x[3]));
}

struct XsArgs {
  Store st;
  Front fin, fout;
  int32_t* D;           // V * XSQ distances
  const u64* nm_in;     // masks of fin's vertices (tag_in)
  u64* nm_out;          // masks of fout's vertices (tag_out)
  uint32_t tag_in, tag_out;
  QCounters* cnt_out;   // fq of fout, arcs = arcs scanned
  u64* progress;        // slots improved in the pass
};

// One chunk of the frontier.  load_pairs_stamps gives each 16-lane group
// the 16 slots of buckets f0 + 4 grp + k; half-wave h (lanes 32 h ..
// 32 h + 31) holds the buckets of groups 2h and 2h + 1, 32 arcs per k.
// Lane q of the half relaxes slot q over those 32 arcs (two owners: arcs
// 0..15 belong to the first bucket, 16..31 to the second), eight at a
// time, and lane s then publishes arc s's improved slots.
__device__ __forceinline__ void xs_relax_chunk(const XsArgs& a, uint32_t c, uint32_t nitems, uint32_t nb, ItemQ& qn,
                                               LaneCounts& lc, const uint32_t* ue, const u64* cm, uint32_t e_lo,
                                               uint32_t e_hi, u64 all, uint32_t& prog) {
  const uint32_t j = threadIdx.x & 31, hb = threadIdx.x & 32, grp = (threadIdx.x >> 4) & 3;
  const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
  uint32_t mk_l = 0;
  if (touches(cv)) {
    const u64 t = a.nm_in[cv.v];
    mk_l = (uint32_t)(t >> 32) == a.tag_in ? (uint32_t)t : 0u;
  }
  for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
    const PairsSt s4 = load_pairs_stamps<true>(a.st.fp, cv, f0, grp, threadIdx.x & 15);
    uint32_t vm4[4];
#pragma unroll
    for (int k = 0; k < 4; k++)
      vm4[k] = s4.d[k] != EMPTY ? (uint32_t)xb_vmask(s4.stamp[k], ue, cm, e_lo, e_hi, all) : 0u;
#pragma unroll 1
    for (int k = 0; k < 4; k++) {
      const uint32_t it_k = xs_pick4(s4.item, k), d_k = xs_pick4(s4.d, k), vm_k = xs_pick4(vm4, k);
      const int32_t w_k = xs_pick4(s4.w, k);
      uint32_t own[2];
      int32_t du[2];
      bool mine[2];
#pragma unroll
      for (int b = 0; b < 2; b++) {
        const int src_lane = (int)(hb + 16 * b);
        const uint32_t itb = __shfl(it_k, src_lane, 64);
        own[b] = __shfl(cv.v, (int)itb, 64);
        const uint32_t mk = __shfl(mk_l, (int)itb, 64);
        mine[b] = (mk >> j) & 1u;
        du[b] = mine[b] ? a.D[(uint64_t)own[b] * XSQ + j] : 0;
      }
      uint32_t my_near = 0;
#pragma unroll 1
      for (int h = 0; h < 32; h += 8) {
        const int b = h >> 4;
        const bool mb = b ? mine[1] : mine[0];
        const int32_t dub = b ? du[1] : du[0];
        uint32_t dd[8];
        int32_t nd[8], cur[8];
        bool act[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
          dd[t] = __shfl(d_k, (int)(hb + h + t), 64);
          const int32_t w = __shfl(w_k, (int)(hb + h + t), 64);
          const uint32_t vmt = __shfl(vm_k, (int)(hb + h + t), 64);
          act[t] = mb && ((vmt >> j) & 1u);
          nd[t] = dub + w;
          cur[t] = act[t] ? a.D[(uint64_t)dd[t] * XSQ + j] : 0;
          lc.arcs += (j == 0 && vmt) ? 1 : 0;   // arcs scanned, once for the half
        }
        int32_t old[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
          old[t] = DIST_INF;
          if (act[t] && nd[t] < cur[t]) old[t] = atomicMin(&a.D[(uint64_t)dd[t] * XSQ + j], nd[t]);
        }
#pragma unroll
        for (int t = 0; t < 8; t++) {
          const bool imp = act[t] && nd[t] < cur[t] && nd[t] < old[t];
          const uint32_t bits = xs_half_ballot(imp);
          if (j == (uint32_t)(h + t)) my_near = bits;
        }
      }
      prog |= my_near;
      const uint32_t d = d_k;
      const bool first = my_near && xs_mark(a.nm_out, d, a.tag_out, my_near);
      const uint64_t yd = first ? a.st.fdesc[d] : 0;
      room_front(qn, 64, a.fout, a.cnt_out);
      push_item(qn, first, d, yd);
    }
  }
}

// The same pass when few slots are active: lane l takes slot l % 16 of a
// bucket (as in the one-query relaxation) and relaxes, for each of its four
// arcs, only the slots that are both in the owner's mask and visible, one
// after another.
__device__ __forceinline__ void xs_sparse_chunk(const XsArgs& a, uint32_t c, uint32_t nitems, uint32_t nb, ItemQ& qn,
                                                LaneCounts& lc, const uint32_t* ue, const u64* cm, uint32_t e_lo,
                                                uint32_t e_hi, u64 all, uint32_t& prog) {
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
  uint32_t mk_l = 0;
  if (touches(cv)) {
    const u64 t = a.nm_in[cv.v];
    mk_l = (uint32_t)(t >> 32) == a.tag_in ? (uint32_t)t : 0u;
  }
  for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
    const PairsSt s4 = load_pairs_stamps<true>(a.st.fp, cv, f0, grp, j);
    uint32_t bits[4], u[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t mk = __shfl(mk_l, (int)s4.item[k], 64);   // all lanes take part
      u[k] = __shfl(cv.v, (int)s4.item[k], 64);
      const uint32_t vm = s4.d[k] != EMPTY ? (uint32_t)xb_vmask(s4.stamp[k], ue, cm, e_lo, e_hi, all) : 0u;
      lc.arcs += vm ? 1 : 0;
      bits[k] = mk & vm;
    }
    uint32_t imp[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      imp[k] = 0;
      for (uint32_t b = bits[k]; b; b &= b - 1) {
        const uint32_t q = __ffs(b) - 1;
        const int32_t du = a.D[(uint64_t)u[k] * XSQ + q];
        const int32_t cur = a.D[(uint64_t)s4.d[k] * XSQ + q];
        const int32_t nd = du + s4.w[k];
        if (nd < cur && nd < atomicMin(&a.D[(uint64_t)s4.d[k] * XSQ + q], nd)) imp[k] |= 1u << q;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      prog |= imp[k];
      const bool first = imp[k] && xs_mark(a.nm_out, s4.d[k], a.tag_out, imp[k]);
      const uint64_t yd = first ? a.st.fdesc[s4.d[k]] : 0;
      room_front(qn, 64, a.fout, a.cnt_out);
      push_item(qn, first, s4.d[k], yd);
    }
  }
}

template <bool SPARSE>
__global__ __launch_bounds__(Q_THREADS) void k_xs_pass(XsArgs a, unsigned long long nfq, XbEpochs ep) {
  __shared__ Shared sh;
  __shared__ uint32_t s_ue[XB_SLOTS];
  __shared__ u64 s_cm[XB_SLOTS + 1];
  for (uint32_t i = threadIdx.x; i < XB_SLOTS; i += Q_THREADS) s_ue[i] = ep.ue[i];
  for (uint32_t i = threadIdx.x; i <= XB_SLOTS; i += Q_THREADS) s_cm[i] = ep.cm[i];
  __syncthreads();
  const uint32_t ne = min(max(ep.ne, 1u), XB_SLOTS);
  const uint32_t e_lo = s_ue[0], e_hi = s_ue[ne - 1];
  const u64 all = s_cm[ne];
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * Q_WAVES + wave, nw = gridDim.x * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  LaneCounts lc;
  uint32_t prog = 0;
  for (uint32_t c = gw; c < nc; c += nw) {
    if (SPARSE) xs_sparse_chunk(a, c, nitems, nb, qn, lc, s_ue, s_cm, e_lo, e_hi, all, prog);
    else xs_relax_chunk(a, c, nitems, nb, qn, lc, s_ue, s_cm, e_lo, e_hi, all, prog);
  }
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  lc.commit(a.cnt_out, sh);
  const u64 p = wave_or_u64(prog);
  if (lane_id() == 0 && p) atomicOr(a.progress, p);
}

// New slots' sources at distance 0 join the next frontier (one wave).
__global__ void k_xs_seed(XbSeeds sd, XsArgs a) {
  __shared__ Shared sh;
  const uint32_t i = lane_id();
  bool first = false;
  uint32_t v = 0;
  if (i < sd.n && i < XSQ && sd.src[i] < a.st.V && sd.slot[i] < XSQ) {
    v = sd.src[i];
    const uint32_t bit = 1u << sd.slot[i];
    a.D[(uint64_t)v * XSQ + sd.slot[i]] = 0;
    first = xs_mark(a.nm_out, v, a.tag_out, bit);
    atomicOr(a.progress, (u64)bit);
  }
  ItemQ qn = item_q(sh.ws[0], 0, WSTAGE);
  push_item(qn, first, v, first ? a.st.fdesc[v] : 0);
  flush_front(qn, a.fout, a.cnt_out);
}

// Distances of the slots in mask reset to infinity.
__global__ void k_xs_clear(int32_t* D, uint64_t V, uint32_t mask) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V * XSQ; i += (uint64_t)gridDim.x * blockDim.x)
    if ((mask >> (i % XSQ)) & 1u) D[i] = DIST_INF;
}

// The listed slots' distances into their outputs (-1 where unreached).
struct XsOutList {
  int32_t* out[XSQ];
  uint32_t slot[XSQ];
};
// A block reads 64 vertices' records in order into LDS and writes each of
// the n listed slots' 64 distances as one run.
__global__ __launch_bounds__(256) void k_xs_extract(const int32_t* D, uint64_t V, XsOutList l, uint32_t n) {
  __shared__ int32_t t[64][XSQ + 1];
  for (uint64_t v0 = (uint64_t)blockIdx.x * 64; v0 < V; v0 += (uint64_t)gridDim.x * 64) {
    for (uint32_t i = threadIdx.x; i < 64 * XSQ; i += 256)
      t[i / XSQ][i % XSQ] = v0 + i / XSQ < V ? D[v0 * XSQ + i] : DIST_INF;
    __syncthreads();
    const uint32_t r = threadIdx.x & 63;
    for (uint32_t i = threadIdx.x >> 6; i < n; i += 4) {
      if (v0 + r < V) {
        const int32_t x = t[r][l.slot[i] % XSQ];
        l.out[i][v0 + r] = x == DIST_INF ? -1 : x;
      }
    }
    __syncthreads();
  }
}

struct XsHost {
  XbResult r;
  uint32_t seq;
};

__global__ void k_xs_publish(QCounters* out, QCounters* consumed, u64* progress, XsHost* h, uint32_t seq) {
  if (threadIdx.x != 0) return;
  XbResult r;
  r.progress = *progress;
  r.arcs = out->arcs;
  r.n_touched = 0;
  r.overflow = out->overflow;
  r.fq = out->fq;
  h->r = r;
  zero_counters(consumed);
  *progress = 0ull;
  __threadfence_system();
  __hip_atomic_store(&h->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_xs_init(int32_t* D, u64* nm0, u64* nm1, uint64_t V, QCounters* cnt, u64* prog) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V * XSQ; i += (uint64_t)gridDim.x * blockDim.x)
    D[i] = DIST_INF;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (uint64_t)gridDim.x * blockDim.x) {
    nm0[i] = 0ull;
    nm1[i] = 0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    zero_counters(&cnt[0]);
    zero_counters(&cnt[1]);
    *prog = 0ull;
  }
}

}  // namespace

struct XsState {
  DevBuf D, nm[2], q[2], cmap[2], cnt, prog;
  uint64_t qcap[2] = {0, 0}, ccap[2] = {0, 0};
  XsHost* host = nullptr;
  uint32_t seq = 0;
  int cur = 0;                  // queue (and mask array) holding the current frontier
  unsigned long long fq = 0;
  uint32_t tag = 1;             // tag of the current frontier's masks
  uint32_t lch = 6;
  uint64_t V = 0;
  uint32_t grid_pass = 0, grid_sparse = 0;
};

XsState* xs_create() { return new XsState(); }

void xs_destroy(XsState* x) {
  if (!x) return;
  release(x->D);
  for (int i = 0; i < 2; i++) {
    release(x->nm[i]);
    release(x->q[i]);
    release(x->cmap[i]);
  }
  release(x->cnt);
  release(x->prog);
  if (x->host) hipHostFree(x->host);
  delete x;
}

hipError_t xs_pass(XsState* x, dg_graph* g, const Store& st, hipStream_t s, uint32_t grid_pct, const XbEpochs& ep,
                   const XbSeeds& seeds, unsigned long long clear_mask, XbResult* res) {
  hipError_t e;
  const uint64_t V = st.V;
  if (!x->host) {
    x->V = V;
    x->lch = 31 - __builtin_clz(std::max<uint32_t>(16, std::min<uint32_t>(64, g->tune.chunk_buckets)));
    if ((e = ensure(x->D, V * XSQ * 4 + 64)) != hipSuccess || (e = ensure(x->nm[0], V * 8 + 64)) != hipSuccess ||
        (e = ensure(x->nm[1], V * 8 + 64)) != hipSuccess ||
        (e = ensure(x->cnt, 2 * sizeof(QCounters))) != hipSuccess || (e = ensure(x->prog, 64)) != hipSuccess)
      return e;
    k_xs_init<<<(uint32_t)std::min<uint64_t>((V * XSQ + 255) / 256, 8192), 256, 0, s>>>(
        x->D.as<int32_t>(), x->nm[0].as<u64>(), x->nm[1].as<u64>(), V, x->cnt.as<QCounters>(), x->prog.as<u64>());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&x->host), sizeof(XsHost), hipHostMallocCoherent)) !=
        hipSuccess) {
      x->host = nullptr;
      return e;
    }
    std::memset(x->host, 0, sizeof(XsHost));
    x->grid_pass = xb_resident((const void*)k_xs_pass<false>);
    x->grid_sparse = xb_resident((const void*)k_xs_pass<true>);
  }
  if (V != x->V) return hipErrorInvalidValue;
  const int cur = x->cur, nxt = cur ^ 1;
  const uint64_t items = V + 1024, chunks = st.fp.cap / CH_MIN + 2;
  for (int i : {nxt, cur}) {
    if (i == cur && x->q[cur].p) continue;   // the current frontier keeps its capacity
    if ((e = ensure(x->q[i], items * sizeof(Item))) != hipSuccess || (e = ensure(x->cmap[i], chunks * 4)) != hipSuccess)
      return e;
    x->qcap[i] = items;
    x->ccap[i] = chunks;
  }
  auto front = [&](int i) {
    return Front{x->q[i].as<Item>(), x->cmap[i].as<uint32_t>(), (uint32_t)std::min<uint64_t>(x->qcap[i], 0xFFFFFFFFu),
                 (uint32_t)std::min<uint64_t>(x->ccap[i], 0xFFFFFFFFu), x->lch};
  };
  QCounters* cnt = x->cnt.as<QCounters>();
  const uint32_t tag_in = x->tag, tag_out = x->tag + 1;
  XsArgs a{st,      front(cur), front(nxt), x->D.as<int32_t>(), x->nm[cur].as<u64>(), x->nm[nxt].as<u64>(),
           tag_in,  tag_out,    &cnt[nxt],  x->prog.as<u64>()};
  const uint32_t cm32 = (uint32_t)(clear_mask & 0xFFFFFFFFull);
  if (cm32)
    k_xs_clear<<<(uint32_t)std::min<uint64_t>((V * XSQ + 255) / 256, 8192), 256, 0, s>>>(a.D, V, cm32);
  if (x->fq && ep.ne) {
    // few active slots: one lane per arc instead of one per slot
    const bool sparse = __builtin_popcount((uint32_t)(ep.cm[ep.ne] & 0xFFFFFFFFull)) <= XS_SPARSE;
    const uint32_t nc = fq_chunks(x->fq, x->lch);
    const uint32_t cap = std::max<uint32_t>(
        1, (uint32_t)((uint64_t)(sparse ? x->grid_sparse : x->grid_pass) * std::min<uint32_t>(grid_pct, 100) / 100));
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((nc + Q_WAVES - 1) / Q_WAVES, cap));
    ProfScope ps(g, KID_SERVE_SSSP, s);
    if (sparse) k_xs_pass<true><<<grid, Q_THREADS, 0, s>>>(a, x->fq, ep);
    else k_xs_pass<false><<<grid, Q_THREADS, 0, s>>>(a, x->fq, ep);
  }
  if (seeds.n) k_xs_seed<<<1, 64, 0, s>>>(seeds, a);
  const uint32_t seq = ++x->seq;
  k_xs_publish<<<1, 64, 0, s>>>(&cnt[nxt], &cnt[cur], x->prog.as<u64>(), x->host, seq);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 1; __atomic_load_n(&x->host->seq, __ATOMIC_ACQUIRE) != seq; spin++) {
    host_pause(spin);
    if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (__atomic_load_n(&x->host->seq, __ATOMIC_ACQUIRE) != seq) return hipErrorUnknown;
      break;
    }
  }
  std::memcpy(res, &x->host->r, sizeof(XbResult));
  res->progress &= 0xFFFFFFFFull;
  x->cur = nxt;
  x->fq = res->fq;
  x->tag = tag_out;
  return hipSuccess;
}

hipError_t xs_extract(XsState* x, const XbOuts& outs, unsigned long long mask, hipStream_t s, hipEvent_t done) {
  XsOutList l{};
  uint32_t n = 0;
  for (uint32_t q = 0; q < XSQ; q++)
    if ((mask >> q & 1ull) && outs.out[q]) {
      l.out[n] = outs.out[q];
      l.slot[n] = q;
      n++;
    }
  if (n) k_xs_extract<<<(uint32_t)std::min<uint64_t>((x->V + 63) / 64, 8192), 256, 0, s>>>(x->D.as<int32_t>(), x->V, l, n);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && done) e = hipEventRecord(done, s);
  return e;
}

}  // namespace dg
