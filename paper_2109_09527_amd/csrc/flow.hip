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
//   search    level-synchronous BFS from s: k_nf_level takes the vertices of
//             level L and claims, with atomicCAS on parent[], every vertex
//             that a residual arc reaches for the first time (the parent
//             word holds the arc id and its direction); the host reads one
//             flag and parent[t] after each level
//   augment   one thread walks the parents back from t, takes the smallest
//             residual and moves that much flow along the path (the walk is
//             bounded by V steps)
// The flow value is exact; which maximum flow the arcs carry can differ
// between runs (any BFS tree gives a shortest path), so only the value is
// returned.
#include <algorithm>
#include <cstring>

#include "dg_host.h"

namespace dg {

constexpr uint32_t NF_THREADS = 256;
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

// Start of a search: no parents, s at level 0.
__global__ void k_nf_reset(uint32_t* parent, int32_t* level, uint32_t V, uint32_t s) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    parent[v] = v == s ? NF_ROOT : NF_NONE;
    level[v] = v == s ? 0 : -1;
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
  int32_t* level;
  uint32_t* grew;
  uint32_t V;
};

__device__ inline void nf_claim(const NfArgs& a, uint32_t y, uint32_t word, int32_t L) {
  if (__hip_atomic_load(&a.parent[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != NF_NONE) return;
  if (atomicCAS(&a.parent[y], NF_NONE, word) == NF_NONE) {
    a.level[y] = L + 1;
    if (__hip_atomic_load(a.grew, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      __hip_atomic_store(a.grew, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One thread per vertex of level L: forward arcs with room, then reverse
// arcs (in-arcs carrying flow).
__global__ __launch_bounds__(NF_THREADS) void k_nf_level(NfArgs a, int32_t L) {
  for (uint32_t x = blockIdx.x * NF_THREADS + threadIdx.x; x < a.V; x += gridDim.x * NF_THREADS) {
    if (a.level[x] != L) continue;
    for (uint32_t k = a.off[x]; k < a.off[x + 1]; k++)
      if (a.cap[k] > a.flow[k]) nf_claim(a, a.csr[k], k << 1, L);
    for (uint32_t i = a.inoff[x]; i < a.inoff[x + 1]; i++) {
      const uint32_t k = a.ine[i];
      if (a.flow[k] > 0) nf_claim(a, a.esrc[k], (k << 1) | 1u, L);
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

void free_flow_scratch(FlowScratch& s) {
  release(s.off); release(s.csr); release(s.cap); release(s.esrc); release(s.keys0); release(s.keys1);
  release(s.vals0); release(s.vals1); release(s.inoff); release(s.flow); release(s.parent); release(s.level);
  release(s.sort); release(s.scan); release(s.ctl);
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
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
  if ((he = ensure(s.esrc, m * 4ull)) != hipSuccess || (he = ensure(s.keys0, m * 8ull)) != hipSuccess ||
      (he = ensure(s.keys1, m * 8ull)) != hipSuccess || (he = ensure(s.vals0, m * 4ull)) != hipSuccess ||
      (he = ensure(s.vals1, m * 4ull)) != hipSuccess || (he = ensure(s.inoff, (V + 1ull) * 4)) != hipSuccess ||
      (he = ensure(s.flow, m * 4ull)) != hipSuccess || (he = ensure(s.parent, V * 4ull)) != hipSuccess ||
      (he = ensure(s.level, V * 4ull)) != hipSuccess || (he = ensure(s.sort, sort_scratch_words(m) * 4 + 64)) != hipSuccess ||
      (he = ensure(s.scan, scan_scratch_words(V + 1ull) * 4 + 64)) != hipSuccess ||
      (he = ensure(s.ctl, 64)) != hipSuccess)
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
  uint32_t* ctl = s.ctl.as<uint32_t>();   // [0] grew, [2..3] total, [4] bad
  k_nf_fill<<<1, 64, 0, st>>>(ctl, 16, 0u);
  auto* total = reinterpret_cast<unsigned long long*>(ctl + 2);
  NfArgs a{s.off.as<uint32_t>(), s.csr.as<uint32_t>(), s.cap.as<uint32_t>(), s.esrc.as<uint32_t>(), inoff, ine,
           s.flow.as<uint32_t>(), s.parent.as<uint32_t>(), s.level.as<int32_t>(), ctl, V};
  const uint32_t g_v = nf_grid(V, NF_THREADS, 4096);
  uint32_t* hw = static_cast<uint32_t*>(s.host);
  // every augmentation moves at least one unit, and the flow cannot pass the
  // capacity out of s: the loop ends; the cap only guards against a fault
  for (uint64_t aug = 0; aug < (1ull << 32); aug++) {
    k_nf_reset<<<nf_grid(V, 256), 256, 0, st>>>(s.parent.as<uint32_t>(), s.level.as<int32_t>(), V, src);
    bool reached = false;
    for (int32_t L = 0; L <= (int32_t)V; L++) {
      k_nf_fill<<<1, 64, 0, st>>>(ctl, 1, 0u);
      {
        ProfScope ps(g, KID_MAXFLOW, st);
        k_nf_level<<<g_v, NF_THREADS, 0, st>>>(a, L);
      }
      if ((he = hipMemcpyAsync(hw, ctl, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (he = hipMemcpyAsync(hw + 1, s.parent.as<uint32_t>() + dst, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (he = hipStreamSynchronize(st)) != hipSuccess)
        return fail_hip(he, "search");
      if (hw[1] != NF_NONE) {
        reached = true;
        break;
      }
      if (!hw[0]) break;
    }
    if (!reached) break;
    k_nf_augment<<<1, 64, 0, st>>>(s.parent.as<uint32_t>(), s.csr.as<uint32_t>(), s.cap.as<uint32_t>(),
                                   s.esrc.as<uint32_t>(), s.flow.as<uint32_t>(), V, src, dst, total, ctl + 4);
  }
  if ((he = hipMemcpyAsync(hw, ctl, 32, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return fail_hip(he, "read back");
  if (hw[4]) {
    g->err = "maxflow: an augmenting path did not lead back to the source";
    return DG_E_HIP;
  }
  unsigned long long tot;
  std::memcpy(&tot, hw + 2, 8);
  *flow_out = (int64_t)tot;
  prof_arcs(g, KID_MAXFLOW, m);
  return DG_OK;
}

}  // namespace dg
