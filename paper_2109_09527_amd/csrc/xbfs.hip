// Continuous multi-source BFS (the serving loop's resident BFS executor):
// kernels of one pass and the host driver of a pass.  Each vertex keeps one
// 16-byte record {visited mask, next-level mask} and a frontier mask, one
// bit per slot, as in the batched multi-source BFS; what differs is that
// every slot has its own epoch, so an arc's visibility is a mask of slots
// rather than one bit, and that slots join and leave between passes.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "xdev.h"

namespace dg {

namespace {

struct XbArgs {
  Store st;
  Front fin, fout;
  unsigned long long* vn;   // {visited, next} per vertex
  unsigned long long* fr;   // frontier mask per vertex
  uint32_t* touched;        // vertices with new next-level bits (count in cnt_out->n_far)
  uint32_t touched_cap;
  QCounters* cnt_out;
};

// Expansion of the frontier items touching chunk c.
__device__ __forceinline__ void xb_chunk(const XbArgs& a, uint32_t c, uint32_t nitems, uint32_t nb, ItemQ& qn,
                                         U32Q& qt, LaneCounts& lc, const uint32_t* ue,
                                         const unsigned long long* cm, uint32_t e_lo, uint32_t e_hi,
                                         unsigned long long all) {
  const uint32_t grp = (threadIdx.x >> 4) & 3, j = threadIdx.x & 15;
  const ChunkView cv = chunk_view(a.fin, c, nitems, nb);
  const unsigned long long f_l = touches(cv) ? a.fr[cv.v] : 0ull;
  for (uint32_t f0 = cv.lo; f0 < cv.hi; f0 += 16) {
    const PairsSt s4 = load_pairs_stamps<false>(a.st.fp, cv, f0, grp, j);
    unsigned long long want[4], have[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const unsigned long long fm = __shfl(f_l, (int)s4.item[k], 64);   // all lanes take part
      want[k] = 0ull;
      have[k] = 0ull;
      if (s4.d[k] != EMPTY) {
        const unsigned long long vm = xb_vmask(s4.stamp[k], ue, cm, e_lo, e_hi, all);
        lc.arcs += vm ? 1 : 0;
        if (fm & vm) {
          // a stale copy of the next mask is a subset: at worst an atomicOr
          // that adds nothing
          const ulonglong2 r = *reinterpret_cast<const ulonglong2*>(&a.vn[2 * (uint64_t)s4.d[k]]);
          want[k] = fm & vm & ~r.x;
          have[k] = r.y;
        }
      }
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

__global__ __launch_bounds__(Q_THREADS) void k_xb_pass(XbArgs a, unsigned long long nfq, XbEpochs ep) {
  __shared__ Shared sh;
  __shared__ uint32_t s_ue[XB_SLOTS];
  __shared__ unsigned long long s_cm[XB_SLOTS + 1];
  for (uint32_t i = threadIdx.x; i < XB_SLOTS; i += Q_THREADS) s_ue[i] = ep.ue[i];
  for (uint32_t i = threadIdx.x; i <= XB_SLOTS; i += Q_THREADS) s_cm[i] = ep.cm[i];
  __syncthreads();
  const uint32_t ne = min(max(ep.ne, 1u), XB_SLOTS);
  const uint32_t e_lo = s_ue[0], e_hi = s_ue[ne - 1];
  const unsigned long long all = s_cm[ne];
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * Q_WAVES + wave, nw = gridDim.x * Q_WAVES;
  const uint32_t nitems = front_items(a.fin, nfq), nb = fq_buckets(nfq), nc = front_chunks(a.fin, nfq);
  ItemQ qn = item_q(sh.ws[wave], 0, WSTAGE);
  U32Q qt = u32_q(sh.ws[wave]);
  LaneCounts lc;
  for (uint32_t c = gw; c < nc; c += nw) xb_chunk(a, c, nitems, nb, qn, qt, lc, s_ue, s_cm, e_lo, e_hi, all);
  flush_u32_q(qt, a.touched, &a.cnt_out->n_far);
  flush_front_wg(qn, a.fout, a.cnt_out, sh);
  lc.commit(a.cnt_out, sh);
}

// New slots' sources join the pass's new vertices (one wave).  Several
// slots may share a source: the atomicOr that finds the next mask empty
// lists the vertex, once.
__global__ void k_xb_seed(XbSeeds sd, XbArgs a) {
  __shared__ Shared sh;
  const uint32_t i = lane_id();
  bool first = false;
  uint32_t v = 0;
  if (i < sd.n && i < XB_SLOTS && sd.src[i] < a.st.V && sd.slot[i] < XB_SLOTS) {
    v = sd.src[i];
    first = atomicOr(&a.vn[2 * (uint64_t)v + 1], 1ull << sd.slot[i]) == 0ull;
  }
  ItemQ qn = item_q(sh.ws[0], 0, WSTAGE);
  push_item(qn, first, v, first ? a.st.fdesc[v] : 0);
  flush_front(qn, a.fout, a.cnt_out);
  U32Q qt = u32_q(sh.ws[0]);
  push_u32(qt, first, v);
  flush_u32_q(qt, a.touched, &a.cnt_out->n_far);
}

// Visited bits of reused slots cleared (keep: the bits that stay).
__global__ void k_xb_clear(unsigned long long* vn, uint64_t V, unsigned long long keep) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (uint64_t)gridDim.x * blockDim.x)
    vn[2 * v] &= keep;
}

// The pass's new vertices: new bits move into the visited mask and become
// the vertex's frontier mask; each new slot's distance is its level.
__global__ __launch_bounds__(Q_THREADS) void k_xb_final(XbArgs a, XbOuts outs, int32_t pass,
                                                        unsigned long long* progress) {
  const uint32_t n = min(a.cnt_out->n_far, a.touched_cap);
  unsigned long long prog = 0ull;
  // every lane runs the same number of rounds, so the reduction below sees
  // the whole wave
  const uint32_t stride = gridDim.x * Q_THREADS;
  for (uint32_t base = blockIdx.x * Q_THREADS + (threadIdx.x & ~63u); base < n; base += stride) {
    const uint32_t i = base + lane_id();
    if (i >= n) continue;
    const uint32_t v = a.touched[i];
    if (v >= a.st.V) continue;
    ulonglong2* rec = reinterpret_cast<ulonglong2*>(&a.vn[2 * (uint64_t)v]);
    ulonglong2 r = *rec;
    unsigned long long nw = r.y & ~r.x;
    r.x |= nw;
    r.y = 0ull;
    *rec = r;
    a.fr[v] = nw;
    prog |= nw;
    while (nw) {
      const int b = __ffsll((long long)nw) - 1;
      nw &= nw - 1;
      int32_t* o = outs.out[b];
      if (o) o[v] = pass - outs.start[b];
    }
  }
  prog = wave_or_u64(prog);
  if (lane_id() == 0 && prog) atomicOr(progress, prog);
}

struct XbHost {
  XbResult r;
  uint32_t seq;
};

// Publishes the pass's counters, then zeroes the consumed ones (the
// current frontier's, which become the next pass's output counters) and
// the progress word.
__global__ void k_xb_publish(QCounters* out, QCounters* consumed, unsigned long long* progress, XbHost* h,
                             uint32_t seq) {
  if (threadIdx.x != 0) return;
  XbResult r;
  r.progress = *progress;
  r.arcs = out->arcs;
  r.n_touched = out->n_far;
  r.overflow = out->overflow;
  r.fq = out->fq;
  h->r = r;
  zero_counters(consumed);
  *progress = 0ull;
  __threadfence_system();
  __hip_atomic_store(&h->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_xb_zero(unsigned long long* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

}  // namespace

struct XbState {
  DevBuf vn, fr, touched, q[2], cmap[2], cnt, prog;
  uint64_t qcap[2] = {0, 0}, ccap[2] = {0, 0};
  XbHost* host = nullptr;
  uint32_t seq = 0;
  int cur = 0;                   // queue holding the current frontier
  unsigned long long fq = 0;     // the current frontier
  uint32_t lch = 6;
  uint64_t V = 0;
  uint32_t grid_pass = 0, grid_final = 0;
};

__global__ void k_xb_fill(int32_t* p, uint64_t n, int32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t fill_i32(int32_t* p, uint64_t n, int32_t v, hipStream_t s) {
  k_xb_fill<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096)), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

XbState* xb_create() { return new XbState(); }

void xb_destroy(XbState* x) {
  if (!x) return;
  release(x->vn);
  release(x->fr);
  release(x->touched);
  for (int i = 0; i < 2; i++) {
    release(x->q[i]);
    release(x->cmap[i]);
  }
  release(x->cnt);
  release(x->prog);
  if (x->host) hipHostFree(x->host);
  delete x;
}

hipError_t xb_pass(XbState* x, dg_graph* g, const Store& st, hipStream_t s, uint32_t grid_pct, int32_t pass,
                   const XbEpochs& ep, const XbOuts& outs, const XbSeeds& seeds, unsigned long long clear_mask,
                   XbResult* res) {
  hipError_t e;
  const uint64_t V = st.V;
  if (!x->host) {
    // first pass: state sized for V, all masks and counters zero
    x->V = V;
    x->lch = 31 - __builtin_clz(std::max<uint32_t>(16, std::min<uint32_t>(64, g->tune.chunk_buckets)));
    if ((e = ensure(x->vn, 2 * V * 8 + 64)) != hipSuccess || (e = ensure(x->fr, V * 8 + 64)) != hipSuccess ||
        (e = ensure(x->touched, (V + 1024) * 4)) != hipSuccess ||
        (e = ensure(x->cnt, 2 * sizeof(QCounters))) != hipSuccess || (e = ensure(x->prog, 64)) != hipSuccess)
      return e;
    k_xb_zero<<<2048, 256, 0, s>>>(x->vn.as<unsigned long long>(), 2 * V);
    k_xb_zero<<<2048, 256, 0, s>>>(x->fr.as<unsigned long long>(), V);
    k_xb_zero<<<1, 64, 0, s>>>(x->cnt.as<unsigned long long>(), 2 * sizeof(QCounters) / 8);
    k_xb_zero<<<1, 64, 0, s>>>(x->prog.as<unsigned long long>(), 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&x->host), sizeof(XbHost), hipHostMallocCoherent)) !=
        hipSuccess) {
      x->host = nullptr;
      return e;
    }
    std::memset(x->host, 0, sizeof(XbHost));
    x->grid_pass = xb_resident((const void*)k_xb_pass);
    x->grid_final = xb_resident((const void*)k_xb_final);
  }
  if (V != x->V) return hipErrorInvalidValue;
  const int cur = x->cur, nxt = cur ^ 1;
  // the next frontier's queue, sized for the pool as it is now (the current
  // one keeps the capacity it was built with)
  const uint64_t items = V + 1024, chunks = st.fp.cap / CH_MIN + 2;
  if ((e = ensure(x->q[nxt], items * sizeof(Item))) != hipSuccess ||
      (e = ensure(x->cmap[nxt], chunks * 4)) != hipSuccess)
    return e;
  x->qcap[nxt] = items;
  x->ccap[nxt] = chunks;
  if (!x->q[cur].p) {
    if ((e = ensure(x->q[cur], items * sizeof(Item))) != hipSuccess ||
        (e = ensure(x->cmap[cur], chunks * 4)) != hipSuccess)
      return e;
    x->qcap[cur] = items;
    x->ccap[cur] = chunks;
  }
  auto front = [&](int i) {
    return Front{x->q[i].as<Item>(), x->cmap[i].as<uint32_t>(), (uint32_t)std::min<uint64_t>(x->qcap[i], 0xFFFFFFFFu),
                 (uint32_t)std::min<uint64_t>(x->ccap[i], 0xFFFFFFFFu), x->lch};
  };
  QCounters* cnt = x->cnt.as<QCounters>();
  XbArgs a{st, front(cur), front(nxt), x->vn.as<unsigned long long>(), x->fr.as<unsigned long long>(),
           x->touched.as<uint32_t>(), (uint32_t)std::min<uint64_t>(V + 1024, 0xFFFFFFFFu), &cnt[nxt]};
  if (clear_mask)
    k_xb_clear<<<(uint32_t)std::min<uint64_t>((V + 255) / 256, 4096), 256, 0, s>>>(a.vn, V, ~clear_mask);
  if (x->fq && ep.ne) {
    const uint32_t nc = fq_chunks(x->fq, x->lch);
    const uint32_t cap = std::max<uint32_t>(1, (uint32_t)((uint64_t)x->grid_pass * std::min<uint32_t>(grid_pct, 100) / 100));
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((nc + Q_WAVES - 1) / Q_WAVES, cap));
    ProfScope ps(g, KID_SERVE_BFS, s);
    k_xb_pass<<<grid, Q_THREADS, 0, s>>>(a, x->fq, ep);
  }
  if (seeds.n) k_xb_seed<<<1, 64, 0, s>>>(seeds, a);
  k_xb_final<<<x->grid_final, Q_THREADS, 0, s>>>(a, outs, pass, x->prog.as<unsigned long long>());
  const uint32_t seq = ++x->seq;
  k_xb_publish<<<1, 64, 0, s>>>(&cnt[nxt], &cnt[cur], x->prog.as<unsigned long long>(), x->host, seq);
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
  x->cur = nxt;
  x->fq = res->fq;
  return hipSuccess;
}

}  // namespace dg
