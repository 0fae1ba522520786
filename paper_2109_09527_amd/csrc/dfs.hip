// DFS collect of the snapshot at epoch e (the GetDFS query named in the
// preamble; textbook semantics): a depth-first search from s over the arcs
// visible at e, each vertex taking its out-neighbours in ascending id order.
// disc[v] is v's position in the discovery order (preorder) and parent[v]
// the vertex whose arc discovered v; both are -1 where v is not reached, and
// parent[s] is -1.
//
// A DFS in a fixed neighbour order is inherently sequential (its visit
// order is P-complete to compute), so the walk is one wave:
//   rows   the out-arc snapshot CSR, each row sorted by target with one radix
//          sort of (row, target) keys
//   walk   k_dfs_walk keeps the stack in device memory, one 16-byte frame
//          {vertex, next arc, row end} per level, the top frame in
//          registers.  At the top vertex x the 64 lanes read the next 64
//          targets of x's row and test whether each was discovered, and a
//          ballot picks the first undiscovered one, which is pushed; a row
//          with none left pops x.  The discovered set is a bitmap in LDS when
//          it fits (160 KB: 1.3 M vertices), else the disc array itself, with
//          a device-scope fence after each push.  Every step pushes or pops,
//          and a push or pop happens at most V times each, so the walk ends
//          within 2V steps (the kernel also stops and flags an error past
//          that bound).
#include <algorithm>
#include <cstring>

#include "dg_host.h"

namespace dg {

static uint32_t dfs_grid(uint64_t units, uint32_t per_block, uint32_t cap = 8192) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((units + per_block - 1) / per_block, cap));
}

__global__ void k_dfs_fill(int32_t* p, uint32_t n, int32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Sort keys (row, target): the row of arc k by binary search in the offsets.
__global__ void k_dfs_keys(const uint32_t* off, const uint32_t* csr, uint32_t V, uint32_t m, int bv, uint64_t* key,
                           uint32_t* val) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = V;   // last row whose offset is <= k
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (off[mid] <= k) lo = mid;
      else hi = mid;
    }
    key[k] = ((uint64_t)lo << bv) | csr[k];
    val[k] = k;
  }
}

struct DfsArgs {
  const uint32_t* off;
  const uint64_t* key;   // sorted (row, target) keys; the target is key & mask
  uint64_t mask;
  uint32_t s;
  uint32_t words;        // LDS bitmap words (LDS form)
  int32_t* disc;
  int32_t* parent;
  uint4* stk;            // frames {vertex, next arc, row end}, V entries
  uint32_t* ctl;         // [0] vertices reached, [1] step bound passed
  uint64_t max_steps;
};

// One wave.  Lane 0 makes every store, and the frames it stores are read
// back by lane 0 alone (broadcast with readfirstlane).  In the LDS form the
// discovered bits are the only state the other lanes read; in the global
// form they read disc, and a device-scope fence after each push makes lane
// 0's stores visible to them.
template <bool LDS>
__global__ __launch_bounds__(64) void k_dfs_walk(DfsArgs a) {
  extern __shared__ uint32_t seen[];
  const uint32_t lane = threadIdx.x;
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  if (LDS) {
    for (uint32_t i = lane; i < a.words; i += 64) seen[i] = 0u;
    __syncthreads();
  }
  uint32_t x = a.s;
  uint32_t c = a.off[x], e = a.off[x + 1];
  if (lane == 0) {
    a.disc[x] = 0;
    if (LDS) seen[x >> 5] |= 1u << (x & 31);
  }
  if (LDS) __syncthreads();
  else __threadfence();
  int32_t t = 1;
  uint32_t sp = 1;   // frames stk[0, sp - 1) are below the top, which is x
  for (uint64_t steps = 0;; steps++) {
    if (steps > a.max_steps) {
      if (lane == 0) a.ctl[1] = 1u;
      break;
    }
    // the first undiscovered target of x's row from its cursor
    uint32_t y = NONE, kf = 0;
    while (c < e) {
      const uint32_t k = c + lane;
      uint32_t tg = 0;
      bool un = false;
      if (k < e) {
        tg = (uint32_t)(a.key[k] & a.mask);
        un = LDS ? ((seen[tg >> 5] >> (tg & 31)) & 1u) == 0u : a.disc[tg] < 0;
      }
      const unsigned long long b = __ballot(un);
      if (b) {
        const uint32_t f = (uint32_t)__builtin_ctzll(b);
        kf = c + f;
        y = (uint32_t)__shfl((int)tg, (int)f, 64);
        break;
      }
      c += 64;
    }
    if (y == NONE) {   // x is finished
      if (--sp == 0) break;
      const uint4 fr = a.stk[sp - 1];
      x = __builtin_amdgcn_readfirstlane(fr.x);
      c = __builtin_amdgcn_readfirstlane(fr.y);
      e = __builtin_amdgcn_readfirstlane(fr.z);
      continue;
    }
    if (lane == 0) {
      a.stk[sp - 1] = make_uint4(x, kf + 1, e, 0u);   // x resumes after y
      a.disc[y] = t;
      a.parent[y] = (int32_t)x;
      if (LDS) seen[y >> 5] |= 1u << (y & 31);
    }
    if (LDS) __syncthreads();
    else __threadfence();
    t++;
    sp++;
    x = y;
    c = a.off[y];
    e = a.off[y + 1];
  }
  if (lane == 0) a.ctl[0] = (uint32_t)t;
}

void free_dfs_scratch(DfsScratch& s) {
  release(s.off); release(s.csr); release(s.keys0); release(s.keys1); release(s.vals0); release(s.vals1);
  release(s.par); release(s.stk); release(s.sort); release(s.ctl);
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
}

dg_status dfs_dev(dg_graph* g, uint32_t e, uint32_t src, int32_t* disc, int32_t* parent, uint32_t* n_reached,
                  hipStream_t st) {
  DfsScratch& s = g->dfs;
  const uint32_t V = g->cfg.v_capacity;
  auto fail_hip = [&](hipError_t he, const char* where) {
    g->err = std::string("dfs ") + where + ": " + hipGetErrorString(he);
    return DG_E_HIP;
  };
  hipError_t he;
  if (!s.host && (he = hipHostMalloc(&s.host, 64, hipHostMallocDefault)) != hipSuccess)
    return fail_hip(he, "host buffer");
  DevBuf& live = g->pr.live;
  if ((he = snapshot_live(g, e, live, st)) != hipSuccess) return fail_hip(he, "liveness");
  uint32_t m = 0;
  if ((he = snapshot_csr(g, e, g->st.fp, g->st.fdesc, live.as<uint8_t>(), s.off, s.csr, &m, st)) != hipSuccess)
    return fail_hip(he, "snapshot");
  const uint64_t mm = std::max<uint32_t>(m, 1);
  if ((he = ensure(s.keys0, mm * 8)) != hipSuccess || (he = ensure(s.keys1, mm * 8)) != hipSuccess ||
      (he = ensure(s.vals0, mm * 4)) != hipSuccess || (he = ensure(s.vals1, mm * 4)) != hipSuccess ||
      (he = ensure(s.stk, V * 16ull)) != hipSuccess ||
      (he = ensure(s.sort, sort_scratch_words(m) * 4 + 64)) != hipSuccess || (he = ensure(s.ctl, 64)) != hipSuccess ||
      (!parent && (he = ensure(s.par, V * 4ull)) != hipSuccess))
    return fail_hip(he, "alloc");
  int32_t* par = parent ? parent : s.par.as<int32_t>();
  k_dfs_fill<<<dfs_grid(V, 256), 256, 0, st>>>(disc, V, -1);
  k_dfs_fill<<<dfs_grid(V, 256), 256, 0, st>>>(par, V, -1);
  k_dfs_fill<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(s.ctl.p), 16, 0);
  int bv = 1;
  while (bv < 32 && (1ull << bv) < V) bv++;
  const uint64_t* keys = s.keys0.as<uint64_t>();
  if (m > 0) {
    k_dfs_keys<<<dfs_grid(m, 256), 256, 0, st>>>(s.off.as<uint32_t>(), s.csr.as<uint32_t>(), V, m, bv,
                                                 s.keys0.as<uint64_t>(), s.vals0.as<uint32_t>());
    const bool alt = radix_sort_pairs(s.keys0.as<uint64_t>(), s.vals0.as<uint32_t>(), s.keys1.as<uint64_t>(),
                                      s.vals1.as<uint32_t>(), m, 2 * bv, s.sort.as<uint32_t>(), st);
    if (alt) keys = s.keys1.as<uint64_t>();
  }
  const uint32_t words = (uint32_t)((V + 31ull) / 32);
  const DfsArgs a{s.off.as<uint32_t>(), keys, (1ull << bv) - 1, src, words, disc, par, s.stk.as<uint4>(),
                  s.ctl.as<uint32_t>(), 2ull * V + 2};
  // the LDS bitmap when the device grants one workgroup that much
  int dev = 0, max_lds = 0;
  const size_t lds = words * 4ull;
  bool use_lds = hipGetDevice(&dev) == hipSuccess &&
                 hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                 lds <= (size_t)max_lds;
  if (use_lds && lds > 65536)
    use_lds = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dfs_walk<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
  (void)hipGetLastError();   // a refused attribute only selects the global form
  {
    ProfScope ps(g, KID_DFS, st);
    if (use_lds) k_dfs_walk<true><<<1, 64, lds, st>>>(a);
    else k_dfs_walk<false><<<1, 64, 0, st>>>(a);
  }
  if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "launch");
  uint32_t* hw = static_cast<uint32_t*>(s.host);
  if ((he = hipMemcpyAsync(hw, s.ctl.p, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return fail_hip(he, "walk");
  if (hw[1]) {
    g->err = "dfs: the walk passed its step bound";
    return DG_E_HIP;
  }
  if (n_reached) *n_reached = hw[0];
  prof_arcs(g, KID_DFS, m);
  return DG_OK;
}

}  // namespace dg
