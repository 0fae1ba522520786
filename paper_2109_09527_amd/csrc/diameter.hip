// Diameter of the snapshot at epoch e (the GD query named in the preamble;
// textbook semantics): the largest hop distance d(u, v) over ordered pairs
// of vertices live at e with v reachable from u, 0 when no arc is visible.
//
// Exact, by a BFS from every live vertex, run bit-parallel: a sweep takes
// DM_W * 64 sources at once, each vertex holding DM_W 64-bit words of
// "reached" bits (one bit per source of the sweep) and as many of
// "frontier" bits.  A level ORs, for every vertex, the frontier words of
// its in-neighbours and keeps the bits it had not reached yet; the sweep
// ends when a level adds no bit, and its last level that added one is the
// largest distance from any of its sources.  OR does not depend on the
// order of updates, so the result is exact.
//
// The level pass runs over the in-arc snapshot CSR (built as for PageRank)
// cut into pieces of at most DM_PIECE arcs, one 16-lane group per piece;
// each lane reads a source's DM_W frontier words (one 32-byte load) per
// arc, and the group folds its words into the vertex with atomicOr.
#include <algorithm>
#include <cstring>
#include <vector>

#include "dg_host.h"

namespace dg {

constexpr uint32_t DM_THREADS = 256;
constexpr uint32_t DM_W = 4;         // words per vertex: 256 sources per sweep
constexpr uint32_t DM_PIECE = 256;

static uint32_t dm_grid(uint64_t units, uint32_t per_block, uint32_t cap = 8192) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((units + per_block - 1) / per_block, cap));
}

__global__ void k_dm_npieces(const uint32_t* off, uint32_t V, uint32_t* np) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v <= V; v += gridDim.x * blockDim.x)
    np[v] = v < V ? (off[v + 1] - off[v] + DM_PIECE - 1) / DM_PIECE : 0;
}

__global__ void k_dm_piece_list(const uint32_t* pfirst, uint32_t V, uint32_t* piece_v) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x)
    for (uint32_t k = pfirst[v]; k < pfirst[v + 1]; k++) piece_v[k] = v;
}

__global__ void k_dm_fill(unsigned long long* p, uint64_t n, unsigned long long x) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = x;
}

// Source k of the sweep is bit k mod 64 of word k / 64 of its vertex (the
// sources are distinct, so every word is written by one thread).
__global__ void k_dm_seed(const uint32_t* src, uint32_t ns, unsigned long long* vis, unsigned long long* fr) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < ns; k += gridDim.x * blockDim.x) {
    const uint64_t i = (uint64_t)src[k] * DM_W + k / 64;
    const unsigned long long b = 1ull << (k % 64);
    vis[i] = b;
    fr[i] = b;
  }
}

struct DmPass {
  const uint32_t* csr;
  const uint32_t* off;
  const uint32_t* pfirst;
  const uint32_t* piece_v;
  uint32_t P;
  const unsigned long long* vis;
  const unsigned long long* fr;
  unsigned long long* nx;
  uint32_t* grew;   // set when a level reached a new (vertex, source) pair
};

struct alignas(32) DmWords {
  unsigned long long w[DM_W];
};

__global__ __launch_bounds__(DM_THREADS) void k_dm_level(DmPass a) {
  const uint32_t j = threadIdx.x & 15;
  const uint32_t ng = gridDim.x * (DM_THREADS / 16);
  for (uint32_t p0 = blockIdx.x * (DM_THREADS / 16); p0 < a.P; p0 += ng) {
    const uint32_t p = p0 + (threadIdx.x >> 4);   // group-uniform
    unsigned long long acc[DM_W] = {};
    uint32_t v = 0;
    if (p < a.P) {
      v = a.piece_v[p];
      const uint32_t b = a.off[v] + (p - a.pfirst[v]) * DM_PIECE;
      const uint32_t end = min(b + DM_PIECE, a.off[v + 1]);
      for (uint32_t i = b + j; i < end; i += 16) {
        const DmWords f = reinterpret_cast<const DmWords*>(a.fr)[a.csr[i]];
#pragma unroll
        for (uint32_t w = 0; w < DM_W; w++) acc[w] |= f.w[w];
      }
    }
#pragma unroll
    for (uint32_t w = 0; w < DM_W; w++)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) acc[w] |= (unsigned long long)__shfl_xor((long long)acc[w], o, 16);
    if (p < a.P && j == 0) {
      bool any = false;
#pragma unroll
      for (uint32_t w = 0; w < DM_W; w++) {
        const unsigned long long m = acc[w] & ~a.vis[(uint64_t)v * DM_W + w];
        if (m) {
          atomicOr(&a.nx[(uint64_t)v * DM_W + w], m);
          any = true;
        }
      }
      if (any && __hip_atomic_load(a.grew, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        __hip_atomic_store(a.grew, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The level's new bits become the frontier and join the reached bits.
__global__ void k_dm_advance(unsigned long long* vis, unsigned long long* fr, unsigned long long* nx, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const unsigned long long m = nx[i];
    vis[i] |= m;
    fr[i] = m;
    nx[i] = 0;
  }
}

void free_diam_scratch(DiamScratch& s) {
  release(s.off); release(s.csr); release(s.pf); release(s.pv); release(s.vis); release(s.fr); release(s.nx);
  release(s.src); release(s.flag); release(s.scan);
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
}

dg_status diameter_dev(dg_graph* g, uint32_t e, uint32_t* diameter, hipStream_t st) {
  DiamScratch& s = g->diam;
  const uint32_t V = g->cfg.v_capacity;
  auto fail_hip = [&](hipError_t he, const char* where) {
    g->err = std::string("diameter ") + where + ": " + hipGetErrorString(he);
    return DG_E_HIP;
  };
  *diameter = 0;
  hipError_t he;
  if (!s.host && (he = hipHostMalloc(&s.host, 64, hipHostMallocDefault)) != hipSuccess)
    return fail_hip(he, "host buffer");
  // the live vertices at e, from the host's history, are the sources
  std::vector<uint32_t> srcs;
  for (uint32_t v = 0; v < V; v++)
    if (g->vfirst[v] != 0 && g->vfirst[v] <= e && (g->vhead[v] == VLOG_NONE || alive_at(g, v, e))) srcs.push_back(v);
  if (srcs.empty()) return DG_OK;
  DevBuf& live = g->pr.live;
  if ((he = snapshot_live(g, e, live, st)) != hipSuccess) return fail_hip(he, "liveness");
  const bool und = g->st.undirected != 0;
  uint32_t m = 0;
  if ((he = snapshot_csr(g, e, und ? g->st.fp : g->st.rp, und ? g->st.fdesc : g->st.rdesc, live.as<uint8_t>(), s.off,
                         s.csr, &m, st)) != hipSuccess)
    return fail_hip(he, "snapshot");
  if (m == 0) return DG_OK;
  const uint64_t P_max = (uint64_t)V + m / DM_PIECE + 1;
  const uint64_t nw = (uint64_t)V * DM_W;
  if ((he = ensure(s.pf, (V + 1ull) * 4)) != hipSuccess || (he = ensure(s.pv, P_max * 4)) != hipSuccess ||
      (he = ensure(s.scan, scan_scratch_words(V + 1ull) * 4 + 64)) != hipSuccess ||
      (he = ensure(s.vis, nw * 8)) != hipSuccess || (he = ensure(s.fr, nw * 8)) != hipSuccess ||
      (he = ensure(s.nx, nw * 8)) != hipSuccess || (he = ensure(s.src, srcs.size() * 4ull)) != hipSuccess ||
      (he = ensure(s.flag, 64)) != hipSuccess)
    return fail_hip(he, "alloc");
  k_dm_npieces<<<dm_grid(V + 1ull, 256), 256, 0, st>>>(s.off.as<uint32_t>(), V, s.pf.as<uint32_t>());
  exclusive_scan_u32(s.pf.as<uint32_t>(), V + 1ull, s.scan.as<uint32_t>(), st);
  k_dm_piece_list<<<dm_grid(V, 256), 256, 0, st>>>(s.pf.as<uint32_t>(), V, s.pv.as<uint32_t>());
  if ((he = hipMemcpyAsync(s.host, s.pf.as<uint32_t>() + V, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return fail_hip(he, "pieces");
  uint32_t P;
  std::memcpy(&P, s.host, 4);
  if (P > P_max) {
    g->err = "diameter: piece count exceeds its bound";
    return DG_E_HIP;
  }
  if ((he = hipMemcpyAsync(s.src.p, srcs.data(), srcs.size() * 4ull, hipMemcpyHostToDevice, st)) != hipSuccess)
    return fail_hip(he, "sources");
  auto* vis = s.vis.as<unsigned long long>();
  auto* fr = s.fr.as<unsigned long long>();
  auto* nx = s.nx.as<unsigned long long>();
  uint32_t* grew = s.flag.as<uint32_t>();
  const DmPass a{s.csr.as<uint32_t>(), s.off.as<uint32_t>(), s.pf.as<uint32_t>(), s.pv.as<uint32_t>(), P, vis, fr, nx,
                 grew};
  const uint32_t g_lv = dm_grid(P, DM_THREADS / 16, 16384), g_w = dm_grid(nw, 256);
  uint32_t best = 0;
  const uint32_t per = DM_W * 64;
  for (size_t s0 = 0; s0 < srcs.size(); s0 += per) {
    const uint32_t ns = (uint32_t)std::min<size_t>(per, srcs.size() - s0);
    k_dm_fill<<<g_w, 256, 0, st>>>(vis, nw, 0ull);
    k_dm_fill<<<g_w, 256, 0, st>>>(fr, nw, 0ull);
    k_dm_fill<<<g_w, 256, 0, st>>>(nx, nw, 0ull);
    k_dm_seed<<<dm_grid(ns, 256), 256, 0, st>>>(s.src.as<uint32_t>() + s0, ns, vis, fr);
    // every level reaches at least one new pair, so V levels bound a sweep
    for (uint32_t level = 0; level <= V; level++) {
      k_dm_fill<<<1, 64, 0, st>>>(reinterpret_cast<unsigned long long*>(grew), 1, 0ull);
      {
        ProfScope ps(g, KID_DIAMETER, st);
        k_dm_level<<<g_lv, DM_THREADS, 0, st>>>(a);
      }
      if ((he = hipMemcpyAsync(s.host, grew, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (he = hipStreamSynchronize(st)) != hipSuccess)
        return fail_hip(he, "level");
      uint32_t gw;
      std::memcpy(&gw, s.host, 4);
      if (!gw) break;
      best = std::max(best, level + 1);
      k_dm_advance<<<g_w, 256, 0, st>>>(vis, fr, nx, nw);
    }
    prof_arcs(g, KID_DIAMETER, m);
  }
  if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "launch");
  *diameter = best;
  return DG_OK;
}

}  // namespace dg
