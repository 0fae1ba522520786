// Maximum s-t flow of the snapshot at epoch e (the GetNF query named in the
// preamble; textbook semantics): arc weights are capacities, an undirected
// edge carrying its weight each way.  Edmonds-Karp (1972): shortest
// augmenting paths over the residual graph, until t is unreachable.
//
// The residual graph is kept implicitly over the out-arc snapshot CSR with
// capacities: arc k (u -> v) has a flow[k]; its forward residual is
// cap[k] - flow[k] and its reverse residual (v -> u) is flow[k].  The reverse
// arcs of a vertex are its in-arcs, listed by a radix sort of the arc ids by
// target.
//
// One augmentation:
//   search    level-synchronous BFS from s over compact frontier queues
//             whose entries are (vertex, piece): a vertex's out-arcs and
//             then its in-arcs, cut into pieces of NF_PIECE, so a hub's arcs
//             spread over many waves.  k_nf_level gives each entry one wave,
//             whose lanes take the forward arcs with room and the in-arcs
//             carrying flow, and claim with atomicCAS on parent[] every
//             vertex that a residual arc reaches first (the parent word
//             holds the arc id and its direction); the wave appends the
//             pieces of its claims to the next queue with one atomicAdd
//   augment   one thread walks the parents back from t, takes the smallest
//             residual and moves that much flow along the path (the walk is
//             bounded by V steps)
// The host enqueues the levels of a search in batches and reads back two
// flags per batch (t reached, frontier empty); a level launched after
// either is set returns at once, so a search of up to a batch's depth costs
// one read-back.  The flow value is exact; which maximum flow the arcs carry
// can differ between runs (any BFS tree gives a shortest path), so only the
// value is returned.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dg_host.h"

namespace dg {

constexpr uint32_t NF_THREADS = 256;
constexpr uint32_t NF_PIECE = 256;   // arcs per queue entry
constexpr uint32_t NF_NONE = 0xFFFFFFFFu;
constexpr uint32_t NF_ROOT = 0xFFFFFFFEu;

static uint32_t nf_grid(uint64_t units, uint32_t per_block, uint32_t cap = 8192) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((units + per_block - 1) / per_block, cap));
}

__global__ void k_nf_fill(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Row of every arc (binary search in the offsets) and the sort keys that
// group the arc ids by target; in-degrees counted into inoff.
__global__ void k_nf_arcs(const uint32_t* off, const uint32_t* csr, uint32_t V, uint32_t m, uint32_t* esrc,
                          uint64_t* key, uint32_t* val, uint32_t* indeg) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = V;   // last row whose offset is <= k
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (off[mid] <= k) lo = mid;
      else hi = mid;
    }
    esrc[k] = lo;
    key[k] = csr[k];
    val[k] = k;
    atomicAdd(&indeg[csr[k]], 1u);
  }
}

// Control words: [0] t reached, [1] frontier empty, [2..3] flow total,
// [4] a walk or a queue went wrong, and three queue lengths, each on a
// 128-byte line of its own, rotating by level: level L reads length L mod 3,
// appends to (L+1) mod 3 and clears (L+2) mod 3, the one level L+1 appends to.
constexpr uint32_t NF_REACHED = 0, NF_EMPTY = 1, NF_TOTAL = 2, NF_BAD = 4, NF_LINE = 32, NF_WORDS = 4 * NF_LINE;
__device__ inline uint32_t* nf_count(uint32_t* ctl, uint32_t r) { return ctl + NF_LINE * (1 + r); }

// Pieces of vertex v: its out- and in-arcs together, NF_PIECE at a time.
__device__ inline uint32_t nf_pieces(const uint32_t* off, const uint32_t* inoff, uint32_t v) {
  return (off[v + 1] - off[v] + inoff[v + 1] - inoff[v] + NF_PIECE - 1) / NF_PIECE;
}

// Start of a search: no parents, the queue of level 0 holds the pieces of s.
__global__ void k_nf_reset(uint32_t* parent, uint2* q0, uint32_t* ctl, const uint32_t* off, const uint32_t* inoff,
                           uint32_t V, uint32_t s) {
  const uint32_t np = nf_pieces(off, inoff, s);
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    parent[v] = v == s ? NF_ROOT : NF_NONE;
    if (v < np) q0[v] = make_uint2(s, v);   // np <= V: s has at most 2V arcs
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[NF_REACHED] = 0;
    ctl[NF_EMPTY] = 0;
    *nf_count(ctl, 0) = np;
    *nf_count(ctl, 1) = 0;
    *nf_count(ctl, 2) = 0;
  }
}

struct NfArgs {
  const uint32_t* off;
  const uint32_t* csr;
  const uint32_t* cap;
  const uint32_t* esrc;
  const uint32_t* inoff;
  const uint32_t* ine;    // arc ids grouped by target
  const uint32_t* flow;
  uint32_t* parent;
  uint2* q[2];            // frontier queues of (vertex, piece), qcap entries each
  uint32_t* ctl;
  uint32_t V, t, qcap;
};

// Claims y for the lane when it is still unreached; the wave then appends
// the pieces of its claims to `out` (one atomicAdd per wave) and flags t.
__device__ inline void nf_push(const NfArgs& a, bool want, uint32_t y, uint32_t word, uint2* out, uint32_t* count) {
  bool mine = false;
  if (want && __hip_atomic_load(&a.parent[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == NF_NONE)
    mine = atomicCAS(&a.parent[y], NF_NONE, word) == NF_NONE;
  if (__ballot(mine) == 0) return;
  const uint32_t lane = __lane_id();
  const uint32_t np = mine ? nf_pieces(a.off, a.inoff, y) : 0u;
  uint32_t incl = np;   // inclusive prefix sum over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t x = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += x;
  }
  const uint32_t tot = __shfl(incl, 63, 64);
  uint32_t base = 0;
  if (lane == 0 && tot) base = atomicAdd(count, tot);
  base = __shfl(base, 0, 64);
  if (mine) {
    const uint32_t at = base + incl - np;
    if (at + np <= a.qcap) {
      for (uint32_t p = 0; p < np; p++) out[at + p] = make_uint2(y, p);
    } else {
      a.ctl[NF_BAD] = 1u;
    }
    if (y == a.t) __hip_atomic_store(&a.ctl[NF_REACHED], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(NF_THREADS) void k_nf_level(NfArgs a, uint32_t L) {
  uint32_t* ctl = a.ctl;
  if (ctl[NF_REACHED] || ctl[NF_EMPTY]) return;
  const uint32_t n = *nf_count(ctl, L % 3);
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[NF_EMPTY] = 1u;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *nf_count(ctl, (L + 2) % 3) = 0;
  const uint2* in = a.q[L & 1];
  uint2* out = a.q[(L + 1) & 1];
  uint32_t* count = nf_count(ctl, (L + 1) % 3);
  const uint32_t lane = __lane_id();
  const uint32_t nw = gridDim.x * (NF_THREADS / 64);
  for (uint32_t i = blockIdx.x * (NF_THREADS / 64) + threadIdx.x / 64; i < n; i += nw) {   // wave-uniform
    if (__builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&ctl[NF_REACHED], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
      break;
    const uint2 en = in[i];
    const uint32_t x = en.x;
    const uint32_t ob = a.off[x], dout = a.off[x + 1] - ob;
    const uint32_t ib = a.inoff[x], dtot = dout + a.inoff[x + 1] - ib;
    const uint32_t j1 = min(dtot, (en.y + 1) * NF_PIECE);
    for (uint32_t j0 = en.y * NF_PIECE; j0 < j1; j0 += 64) {
      const uint32_t j = j0 + lane;
      bool want = false;
      uint32_t y = 0, word = 0;
      if (j < dout) {
        const uint32_t k = ob + j;
        if (a.cap[k] > a.flow[k]) {
          want = true;
          y = a.csr[k];
          word = k << 1;
        }
      } else if (j < j1) {
        const uint32_t k = a.ine[ib + (j - dout)];
        if (a.flow[k] > 0) {
          want = true;
          y = a.esrc[k];
          word = (k << 1) | 1u;
        }
      }
      nf_push(a, want, y, word, out, count);
    }
  }
}

// One thread: the path from t back to s, its smallest residual, and the
// flow moved along it; *total accumulates the value, *bad is set when the
// walk does not reach s within V steps.
__global__ void k_nf_augment(const uint32_t* parent, const uint32_t* csr, const uint32_t* cap, const uint32_t* esrc,
                             uint32_t* flow, uint32_t V, uint32_t s, uint32_t t, unsigned long long* total,
                             uint32_t* bad) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t x = t, b = 0xFFFFFFFFu, steps = 0;
  while (x != s && steps++ < V) {
    const uint32_t p = parent[x];
    if (p >= NF_ROOT) break;
    const uint32_t k = p >> 1;
    uint32_t r;
    if (p & 1u) {
      r = flow[k];
      x = csr[k];
    } else {
      r = cap[k] - flow[k];
      x = esrc[k];
    }
    b = min(b, r);
  }
  if (x != s || b == 0 || b == 0xFFFFFFFFu) {
    *bad = 1u;
    return;
  }
  x = t;
  steps = 0;
  while (x != s && steps++ < V) {
    const uint32_t p = parent[x];
    const uint32_t k = p >> 1;
    if (p & 1u) {
      flow[k] -= b;
      x = csr[k];
    } else {
      flow[k] += b;
      x = esrc[k];
    }
  }
  *total += b;
}

// The first eight control words to coherent pinned memory, then the
// sequence number (system scope): the host polls it instead of
// synchronising the stream after every batch of levels.
__global__ void k_nf_publish(const uint32_t* ctl, uint32_t* host, uint32_t seq) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < 8; i++) host[i] = ctl[i];
  __hip_atomic_store(&host[8], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void free_flow_scratch(FlowScratch& s) {
  release(s.off); release(s.csr); release(s.cap); release(s.esrc); release(s.keys0); release(s.keys1);
  release(s.vals0); release(s.vals1); release(s.inoff); release(s.flow); release(s.parent); release(s.queue);
  release(s.sort); release(s.scan); release(s.ctl);
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
  if (s.pub) (void)hipHostFree(s.pub);
  s.pub = nullptr;
}

dg_status maxflow_dev(dg_graph* g, uint32_t e, uint32_t src, uint32_t dst, int64_t* flow_out, hipStream_t st) {
  FlowScratch& s = g->flow;
  const uint32_t V = g->cfg.v_capacity;
  auto fail_hip = [&](hipError_t he, const char* where) {
    g->err = std::string("maxflow ") + where + ": " + hipGetErrorString(he);
    return DG_E_HIP;
  };
  *flow_out = 0;
  hipError_t he;
  if (!s.host && (he = hipHostMalloc(&s.host, 64, hipHostMallocDefault)) != hipSuccess)
    return fail_hip(he, "host buffer");
  if (!s.pub) {
    if ((he = hipHostMalloc(&s.pub, 64, hipHostMallocCoherent)) != hipSuccess) {
      s.pub = nullptr;
      return fail_hip(he, "host buffer");
    }
    std::memset(s.pub, 0, 64);
  }
  DevBuf& live = g->pr.live;
  if ((he = snapshot_live(g, e, live, st)) != hipSuccess) return fail_hip(he, "liveness");
  uint32_t m = 0;
  if ((he = snapshot_csr(g, e, g->st.fp, g->st.fdesc, live.as<uint8_t>(), s.off, s.csr, &m, st, &s.cap)) !=
      hipSuccess)
    return fail_hip(he, "snapshot");
  if (m == 0) return DG_OK;
  if (m >= 0x7FFFFFFFu) {
    g->err = "maxflow: too many arcs for 31-bit arc ids";
    return DG_E_INVALID_ARG;
  }
  // a level's entries: at most one piece per vertex plus one per NF_PIECE
  // of the arcs seen from both ends
  const uint64_t qcap = (uint64_t)V + (2ull * m) / NF_PIECE + 64;
  if (qcap > 0xFFFFFFFFull) {
    g->err = "maxflow: the frontier queues would pass 2^32 entries";
    return DG_E_INVALID_ARG;
  }
  if ((he = ensure(s.esrc, m * 4ull)) != hipSuccess || (he = ensure(s.keys0, m * 8ull)) != hipSuccess ||
      (he = ensure(s.keys1, m * 8ull)) != hipSuccess || (he = ensure(s.vals0, m * 4ull)) != hipSuccess ||
      (he = ensure(s.vals1, m * 4ull)) != hipSuccess || (he = ensure(s.inoff, (V + 1ull) * 4)) != hipSuccess ||
      (he = ensure(s.flow, m * 4ull)) != hipSuccess || (he = ensure(s.parent, V * 4ull)) != hipSuccess ||
      (he = ensure(s.queue, qcap * 16ull)) != hipSuccess || (he = ensure(s.sort, sort_scratch_words(m) * 4 + 64)) != hipSuccess ||
      (he = ensure(s.scan, scan_scratch_words(V + 1ull) * 4 + 64)) != hipSuccess ||
      (he = ensure(s.ctl, NF_WORDS * 4)) != hipSuccess)
    return fail_hip(he, "alloc");
  uint32_t* inoff = s.inoff.as<uint32_t>();
  k_nf_fill<<<nf_grid(V + 1ull, 256), 256, 0, st>>>(inoff, V + 1ull, 0u);
  k_nf_arcs<<<nf_grid(m, 256), 256, 0, st>>>(s.off.as<uint32_t>(), s.csr.as<uint32_t>(), V, m, s.esrc.as<uint32_t>(),
                                             s.keys0.as<uint64_t>(), s.vals0.as<uint32_t>(), inoff);
  exclusive_scan_u32(inoff, V + 1ull, s.scan.as<uint32_t>(), st);
  int bits = 1;
  while (bits < 32 && (1ull << bits) < V) bits++;
  const bool alt = radix_sort_pairs(s.keys0.as<uint64_t>(), s.vals0.as<uint32_t>(), s.keys1.as<uint64_t>(),
                                    s.vals1.as<uint32_t>(), m, bits, s.sort.as<uint32_t>(), st);
  const uint32_t* ine = alt ? s.vals1.as<uint32_t>() : s.vals0.as<uint32_t>();
  k_nf_fill<<<nf_grid(m, 256), 256, 0, st>>>(s.flow.as<uint32_t>(), m, 0u);
  uint32_t* ctl = s.ctl.as<uint32_t>();
  k_nf_fill<<<1, 64, 0, st>>>(ctl, NF_WORDS, 0u);
  auto* total = reinterpret_cast<unsigned long long*>(ctl + NF_TOTAL);
  uint2* q0 = s.queue.as<uint2>();
  NfArgs a{s.off.as<uint32_t>(), s.csr.as<uint32_t>(), s.cap.as<uint32_t>(), s.esrc.as<uint32_t>(), inoff, ine,
           s.flow.as<uint32_t>(), s.parent.as<uint32_t>(), {q0, q0 + qcap}, ctl, V, dst, (uint32_t)qcap};
  const uint32_t g_lv = nf_grid(qcap, NF_THREADS / 64, 1024), g_v = nf_grid(V, 256);
  uint32_t* hw = static_cast<uint32_t*>(s.host);
  // Every augmentation moves at least one unit, and the flow cannot pass the
  // capacity out of s, so the loop ends; a search has at most V + 1 levels
  // (each level but the last claims a vertex).
  uint32_t batch = 8;
  k_nf_reset<<<g_v, 256, 0, st>>>(s.parent.as<uint32_t>(), q0, ctl, s.off.as<uint32_t>(), inoff, V, src);
  for (uint32_t L = 0;;) {
    const uint32_t first = L;
    for (uint32_t j = 0; j < batch; j++, L++) {
      ProfScope ps(g, KID_MAXFLOW, st);
      k_nf_level<<<g_lv, NF_THREADS, 0, st>>>(a, L);
    }
    {
      uint32_t* pub = static_cast<uint32_t*>(s.pub);
      const uint32_t seq = ++s.seq;
      k_nf_publish<<<1, 64, 0, st>>>(ctl, pub, seq);
      if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "search");
      const auto t0 = std::chrono::steady_clock::now();
      for (uint32_t spin = 1; __atomic_load_n(&pub[8], __ATOMIC_ACQUIRE) != seq; spin++) {
        host_pause(spin);
        if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
          if ((he = hipStreamSynchronize(st)) != hipSuccess) return fail_hip(he, "search");
          if (__atomic_load_n(&pub[8], __ATOMIC_ACQUIRE) != seq) return fail_hip(hipErrorUnknown, "search");
          break;
        }
      }
      std::memcpy(hw, pub, 32);
    }
    if (hw[NF_BAD]) break;   // reported below
    if (hw[NF_REACHED]) {
      k_nf_augment<<<1, 64, 0, st>>>(s.parent.as<uint32_t>(), s.csr.as<uint32_t>(), s.cap.as<uint32_t>(),
                                     s.esrc.as<uint32_t>(), s.flow.as<uint32_t>(), V, src, dst, total, ctl + NF_BAD);
      k_nf_reset<<<g_v, 256, 0, st>>>(s.parent.as<uint32_t>(), q0, ctl, s.off.as<uint32_t>(), inoff, V, src);
      // a search that needed more than one batch doubles the batch
      if (first > 0) batch = std::min<uint32_t>(batch * 2, 64);
      L = 0;
      continue;
    }
    if (hw[NF_EMPTY]) break;
    if (L > V + 1) {
      g->err = "maxflow: a search ran past V + 1 levels";
      return DG_E_HIP;
    }
  }
  if ((he = hipMemcpyAsync(hw, ctl, 32, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return fail_hip(he, "read back");
  if (hw[NF_BAD]) {
    g->err = "maxflow: an augmenting path did not lead back to the source, or a queue overflowed";
    return DG_E_HIP;
  }
  unsigned long long tot;
  std::memcpy(&tot, hw + NF_TOTAL, 8);
  *flow_out = (int64_t)tot;
  prof_arcs(g, KID_MAXFLOW, m);
  return DG_OK;
}

}  // namespace dg
