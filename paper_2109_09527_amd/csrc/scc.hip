// Strongly connected components of the snapshot at epoch e (the GetSCC
// query named in the preamble; textbook semantics): comp[v] = the smallest
// id in v's component for a vertex live at e, -1 otherwise.  An undirected
// graph's components are its connected components.
//
// Colour propagation (Orzan's method, as used by the GPU SCC literature),
// in rounds over the vertices not yet assigned:
//   colour   every remaining vertex starts with its own id; passes over the
//            in-arcs lower colour[v] to the smallest colour of a remaining
//            in-neighbour until nothing changes, so colour[v] ends as the
//            smallest id that reaches v
//   roots    a vertex that kept its own id is reached by no smaller one;
//            the vertices of colour r that reach r are exactly r's
//            component, and r is its smallest member
//   collect  passes over the out-arcs mark a vertex that has a marked
//            out-neighbour of its own colour, starting from the roots,
//            until nothing changes
//   assign   marked vertices take their colour as component and leave
// The smallest remaining vertex is always a root, so every round assigns at
// least one component.  Min and "any" do not depend on the order of
// updates, so results are exact and repeatable.
//
// Both passes run over the snapshot CSRs (in-arcs and out-arcs, built as
// for PageRank) cut into pieces of at most SCC_PIECE arcs, one 16-lane
// group per piece, so a hub's arcs spread over many groups.  Each pass
// reports whether it changed anything through one flag read back by the
// host.
#include <algorithm>
#include <cstring>

#include "dg_host.h"

namespace dg {

uint64_t live_at(const dg_graph* g, uint32_t e);

constexpr uint32_t SCC_THREADS = 256;
constexpr uint32_t SCC_PIECE = 256;
constexpr uint32_t SCC_STRIPES = 64;   // words the remaining count is spread over
constexpr uint32_t SCC_NONE = 0xFFFFFFFFu;

static uint32_t scc_grid(uint64_t units, uint32_t per_block, uint32_t cap = 8192) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((units + per_block - 1) / per_block, cap));
}

__global__ void k_scc_fill(uint32_t* p, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Pieces of each vertex's CSR row (entry V stays 0 for the scan).
__global__ void k_scc_npieces(const uint32_t* off, uint32_t V, uint32_t* np) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v <= V; v += gridDim.x * blockDim.x)
    np[v] = v < V ? (off[v + 1] - off[v] + SCC_PIECE - 1) / SCC_PIECE : 0;
}

__global__ void k_scc_piece_list(const uint32_t* pfirst, uint32_t V, uint32_t* piece_v) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x)
    for (uint32_t k = pfirst[v]; k < pfirst[v + 1]; k++) piece_v[k] = v;
}

__global__ void k_scc_start(const uint8_t* live, uint32_t V, int32_t* comp, uint8_t* rem) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    comp[v] = -1;
    rem[v] = live[v];
  }
}

__global__ void k_scc_colour(const uint8_t* rem, uint32_t V, uint32_t* colour, uint8_t* mark) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    colour[v] = rem[v] ? v : SCC_NONE;
    mark[v] = 0;
  }
}

struct SccPass {
  const uint32_t* csr;
  const uint32_t* off;
  const uint32_t* pfirst;
  const uint32_t* piece_v;
  uint32_t P;
  const uint8_t* rem;
  uint32_t* colour;
  uint8_t* mark;
  uint32_t* changed;
};

__device__ inline void scc_set_changed(uint32_t* changed) {
  if (__hip_atomic_load(changed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    __hip_atomic_store(changed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One 16-lane group per piece of the in-CSR: the smallest colour among the
// remaining in-neighbours, folded into colour[v] with atomicMin.
__global__ __launch_bounds__(SCC_THREADS) void k_scc_forward(SccPass a) {
  const uint32_t j = threadIdx.x & 15;
  const uint32_t ng = gridDim.x * (SCC_THREADS / 16);
  for (uint32_t p0 = blockIdx.x * (SCC_THREADS / 16); p0 < a.P; p0 += ng) {
    const uint32_t p = p0 + (threadIdx.x >> 4);   // group-uniform
    uint32_t m = SCC_NONE, v = 0;
    if (p < a.P) {
      v = a.piece_v[p];
      if (a.rem[v]) {
        const uint32_t b = a.off[v] + (p - a.pfirst[v]) * SCC_PIECE;
        const uint32_t end = min(b + SCC_PIECE, a.off[v + 1]);
        for (uint32_t i = b + j; i < end; i += 16) {
          const uint32_t u = a.csr[i];
          if (a.rem[u]) m = min(m, __hip_atomic_load(&a.colour[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        }
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, o, 16));
    if (p < a.P && j == 0 && m != SCC_NONE && m < __hip_atomic_load(&a.colour[v], __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT)) {
      if (atomicMin(&a.colour[v], m) > m) scc_set_changed(a.changed);
    }
  }
}

__global__ void k_scc_roots(const uint8_t* rem, const uint32_t* colour, uint32_t V, uint8_t* mark) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x)
    mark[v] = rem[v] && colour[v] == v ? 1 : 0;
}

// One 16-lane group per piece of the out-CSR: an unmarked remaining vertex
// with a marked out-neighbour of its colour is marked.
__global__ __launch_bounds__(SCC_THREADS) void k_scc_collect(SccPass a) {
  const uint32_t j = threadIdx.x & 15;
  const uint32_t ng = gridDim.x * (SCC_THREADS / 16);
  for (uint32_t p0 = blockIdx.x * (SCC_THREADS / 16); p0 < a.P; p0 += ng) {
    const uint32_t p = p0 + (threadIdx.x >> 4);   // group-uniform
    bool hit = false;
    uint32_t v = 0;
    if (p < a.P) {
      v = a.piece_v[p];
      if (a.rem[v] && !__hip_atomic_load(&a.mark[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        const uint32_t c = a.colour[v];
        const uint32_t b = a.off[v] + (p - a.pfirst[v]) * SCC_PIECE;
        const uint32_t end = min(b + SCC_PIECE, a.off[v + 1]);
        for (uint32_t i = b + j; i < end && !hit; i += 16) {
          const uint32_t w = a.csr[i];
          hit = a.rem[w] && a.colour[w] == c &&
                __hip_atomic_load(&a.mark[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        }
      }
    }
    // any lane of the group
    uint32_t h = hit ? 1u : 0u;
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) h |= (uint32_t)__shfl_xor((int)h, o, 16);
    if (p < a.P && j == 0 && h) {
      __hip_atomic_store(&a.mark[v], (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      scc_set_changed(a.changed);
    }
  }
}

// Marked vertices take their colour and leave.  The vertices left and the
// roots (one per component found) are counted per workgroup into word
// blockIdx mod SCC_STRIPES of left[] and roots[].
__global__ __launch_bounds__(SCC_THREADS) void k_scc_assign(uint8_t* rem, const uint8_t* mark,
                                                            const uint32_t* colour, uint32_t V, int32_t* comp,
                                                            uint32_t* left, uint32_t* roots) {
  __shared__ uint32_t wsum[2][SCC_THREADS / 64];
  uint32_t n = 0, nr = 0;
  for (uint32_t v = blockIdx.x * SCC_THREADS + threadIdx.x; v < V; v += gridDim.x * SCC_THREADS) {
    if (!rem[v]) continue;
    if (mark[v]) {
      comp[v] = (int32_t)colour[v];
      rem[v] = 0;
      nr += colour[v] == v ? 1 : 0;
    } else {
      n++;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    n += (uint32_t)__shfl_xor((int)n, o, 64);
    nr += (uint32_t)__shfl_xor((int)nr, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    wsum[0][threadIdx.x >> 6] = n;
    wsum[1][threadIdx.x >> 6] = nr;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t t = 0;
    for (uint32_t w = 0; w < SCC_THREADS / 64; w++) t += wsum[threadIdx.x][w];
    if (t) atomicAdd(&(threadIdx.x ? roots : left)[blockIdx.x % SCC_STRIPES], t);
  }
}

void free_scc_scratch(SccScratch& s) {
  release(s.off_in); release(s.csr_in); release(s.off_out); release(s.csr_out);
  release(s.pf_in); release(s.pv_in); release(s.pf_out); release(s.pv_out);
  release(s.colour); release(s.mark); release(s.rem); release(s.flags); release(s.scan);
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
}

// Pieces of one CSR: first piece per vertex (V + 1) and the owner of each.
static hipError_t scc_pieces(SccScratch& s, const DevBuf& off, uint32_t V, uint32_t m, DevBuf& pf, DevBuf& pv,
                             uint32_t* P, hipStream_t st) {
  hipError_t he;
  const uint64_t P_max = (uint64_t)V + m / SCC_PIECE + 1;
  if ((he = ensure(pf, (V + 1ull) * 4)) != hipSuccess || (he = ensure(pv, P_max * 4)) != hipSuccess ||
      (he = ensure(s.scan, scan_scratch_words(V + 1ull) * 4 + 64)) != hipSuccess)
    return he;
  k_scc_npieces<<<scc_grid(V + 1ull, 256), 256, 0, st>>>(off.as<uint32_t>(), V, pf.as<uint32_t>());
  exclusive_scan_u32(pf.as<uint32_t>(), V + 1ull, s.scan.as<uint32_t>(), st);
  k_scc_piece_list<<<scc_grid(V, 256), 256, 0, st>>>(pf.as<uint32_t>(), V, pv.as<uint32_t>());
  if ((he = hipMemcpyAsync(s.host, pf.as<uint32_t>() + V, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return he;
  std::memcpy(P, s.host, 4);
  return *P <= P_max ? hipSuccess : hipErrorInvalidValue;
}

static hipError_t scc_read(SccScratch& s, const uint32_t* dev, uint32_t n, uint32_t* out, hipStream_t st) {
  hipError_t he;
  if ((he = hipMemcpyAsync(s.host, dev, n * 4ull, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return he;
  std::memcpy(out, s.host, n * 4ull);
  return hipSuccess;
}

dg_status scc_dev(dg_graph* g, uint32_t e, int32_t* comp, uint32_t* n_comp, uint32_t* rounds_out, hipStream_t st) {
  SccScratch& s = g->scc;
  const uint32_t V = g->cfg.v_capacity;
  auto fail_hip = [&](hipError_t he, const char* where) {
    g->err = std::string("scc ") + where + ": " + hipGetErrorString(he);
    return DG_E_HIP;
  };
  hipError_t he;
  if (!s.host && (he = hipHostMalloc(&s.host, 4096, hipHostMallocDefault)) != hipSuccess)
    return fail_hip(he, "host buffer");
  DevBuf& live = g->pr.live;
  if ((he = snapshot_live(g, e, live, st)) != hipSuccess) return fail_hip(he, "liveness");
  const bool und = g->st.undirected != 0;
  uint32_t m_in = 0, m_out = 0;
  // in-arcs: the reverse pool, or the forward one of an undirected graph,
  // whose out-arcs are then the same rows
  if ((he = snapshot_csr(g, e, und ? g->st.fp : g->st.rp, und ? g->st.fdesc : g->st.rdesc, live.as<uint8_t>(),
                         s.off_in, s.csr_in, &m_in, st)) != hipSuccess)
    return fail_hip(he, "in-arc snapshot");
  if (!und && (he = snapshot_csr(g, e, g->st.fp, g->st.fdesc, live.as<uint8_t>(), s.off_out, s.csr_out, &m_out,
                                 st)) != hipSuccess)
    return fail_hip(he, "out-arc snapshot");
  const DevBuf& off_out = und ? s.off_in : s.off_out;
  const DevBuf& csr_out = und ? s.csr_in : s.csr_out;
  if (und) m_out = m_in;
  uint32_t P_in = 0, P_out = 0;
  if ((he = scc_pieces(s, s.off_in, V, m_in, s.pf_in, s.pv_in, &P_in, st)) != hipSuccess)
    return fail_hip(he, "in pieces");
  const DevBuf& pf_out = und ? s.pf_in : s.pf_out;
  const DevBuf& pv_out = und ? s.pv_in : s.pv_out;
  if (!und && (he = scc_pieces(s, off_out, V, m_out, s.pf_out, s.pv_out, &P_out, st)) != hipSuccess)
    return fail_hip(he, "out pieces");
  if (und) P_out = P_in;
  if ((he = ensure(s.colour, V * 4ull + 64)) != hipSuccess || (he = ensure(s.mark, V + 64ull)) != hipSuccess ||
      (he = ensure(s.rem, V + 64ull)) != hipSuccess || (he = ensure(s.flags, (2 + 2 * SCC_STRIPES) * 4)) != hipSuccess)
    return fail_hip(he, "alloc");
  uint32_t* changed = s.flags.as<uint32_t>();
  uint32_t* left = changed + 2;
  uint32_t* roots = left + SCC_STRIPES;
  k_scc_fill<<<1, 64, 0, st>>>(roots, SCC_STRIPES, 0u);
  k_scc_start<<<scc_grid(V, 256), 256, 0, st>>>(live.as<uint8_t>(), V, comp, s.rem.as<uint8_t>());
  SccPass fwd{s.csr_in.as<uint32_t>(), s.off_in.as<uint32_t>(), s.pf_in.as<uint32_t>(), s.pv_in.as<uint32_t>(),
              P_in, s.rem.as<uint8_t>(), s.colour.as<uint32_t>(), s.mark.as<uint8_t>(), changed};
  SccPass bwd{csr_out.as<uint32_t>(), off_out.as<uint32_t>(), pf_out.as<uint32_t>(), pv_out.as<uint32_t>(),
              P_out, s.rem.as<uint8_t>(), s.colour.as<uint32_t>(), s.mark.as<uint8_t>(), changed};
  const uint32_t g_in = scc_grid(P_in, SCC_THREADS / 16, 16384), g_out = scc_grid(P_out, SCC_THREADS / 16, 16384);
  const uint32_t g_v = scc_grid(V, SCC_THREADS, 1024);
  uint64_t remaining = live_at(g, e);
  uint32_t rounds = 0;
  // every round assigns at least one component, so V rounds bound the loop
  while (remaining > 0 && rounds <= V) {
    rounds++;
    k_scc_colour<<<scc_grid(V, 256), 256, 0, st>>>(s.rem.as<uint8_t>(), V, s.colour.as<uint32_t>(),
                                                   s.mark.as<uint8_t>());
    for (uint32_t pass = 0;; pass++) {
      uint32_t c = 0;
      k_scc_fill<<<1, 64, 0, st>>>(changed, 1, 0u);
      {
        ProfScope ps(g, KID_SCC, st);
        k_scc_forward<<<g_in, SCC_THREADS, 0, st>>>(fwd);
      }
      if ((he = scc_read(s, changed, 1, &c, st)) != hipSuccess) return fail_hip(he, "forward");
      if (!c || pass > V) break;
    }
    k_scc_roots<<<scc_grid(V, 256), 256, 0, st>>>(s.rem.as<uint8_t>(), s.colour.as<uint32_t>(), V,
                                                  s.mark.as<uint8_t>());
    for (uint32_t pass = 0;; pass++) {
      uint32_t c = 0;
      k_scc_fill<<<1, 64, 0, st>>>(changed, 1, 0u);
      {
        ProfScope ps(g, KID_SCC, st);
        k_scc_collect<<<g_out, SCC_THREADS, 0, st>>>(bwd);
      }
      if ((he = scc_read(s, changed, 1, &c, st)) != hipSuccess) return fail_hip(he, "collect");
      if (!c || pass > V) break;
    }
    k_scc_fill<<<1, 64, 0, st>>>(left, SCC_STRIPES, 0u);
    k_scc_assign<<<g_v, SCC_THREADS, 0, st>>>(s.rem.as<uint8_t>(), s.mark.as<uint8_t>(), s.colour.as<uint32_t>(), V,
                                              comp, left, roots);
    uint32_t words[SCC_STRIPES];
    if ((he = scc_read(s, left, SCC_STRIPES, words, st)) != hipSuccess) return fail_hip(he, "assign");
    uint64_t r = 0;
    for (uint32_t k = 0; k < SCC_STRIPES; k++) r += words[k];
    if (r >= remaining) {
      g->err = "scc: a round assigned no component";
      return DG_E_HIP;
    }
    remaining = r;
  }
  prof_arcs(g, KID_SCC, (uint64_t)m_in + m_out);
  if (rounds_out) *rounds_out = rounds;
  if (n_comp) {
    uint32_t words[SCC_STRIPES];
    if ((he = scc_read(s, roots, SCC_STRIPES, words, st)) != hipSuccess) return fail_hip(he, "count");
    uint64_t c = 0;
    for (uint32_t k = 0; k < SCC_STRIPES; k++) c += words[k];
    *n_comp = (uint32_t)c;
  }
  if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "launch");
  return DG_OK;
}

}  // namespace dg
