// Snapshot PageRank on epoch e: Eq. (1) iterated synchronously, as in the
// Barrier baseline (Alg. 1).  Every live vertex starts at 1/n (n = live
// vertices at e); an iteration recomputes all of them from the previous
// values only, pr(u) = (1 - d)/n + d * sum over visible arcs (v, u) of
// pr(v)/q(v), with q(v) the visible out-degree, and the loop ends at the
// first iteration whose largest |change| is at most the threshold (the
// change is measured afresh each iteration).  A vertex without out-arcs
// passes nothing on.  FP64 throughout.
//
// The iterations run over a compact snapshot of the visible in-arcs at e
// (in-CSR, sources only), built once per call:
//   tiles   each live vertex's in-slab cut into tiles of PR_TILE buckets
//           (64 slots, one wave step), so hub slabs spread over many waves
//   count   visible slots per tile; an exclusive scan over the tiles gives
//           every tile its position in the CSR (tiles of a vertex are
//           consecutive, vertices in id order)
//   fill    each tile's visible sources, bucket by bucket, slot by slot
//   q(v)    out-degrees counted from the CSR's sources (integer atomics)
//   ranks   vertices renumbered by decreasing out-degree (stable radix sort,
//           ties by id); the CSR's rows are moved to rank order and its
//           sources mapped to ranks
// An iteration then streams 4 bytes per arc plus one random 8-byte read of
// the source's contribution, instead of re-reading buckets and stamps.  In
// rank order the most-read contributions (those of the largest
// out-degrees) share a short prefix of the array that stays in L2, and the
// per-vertex arrays are read and written in order; the ranks are mapped
// back to ids once, after the last iteration.
//
// Per iteration, two kernels:
//   k_pr_pull   one 16-lane group per piece (at most PR_PIECE consecutive
//               in-arcs of one vertex): lanes sum contrib[src] over strided
//               arcs, then a fixed shuffle tree combines them
//   k_pr_apply  one lane per vertex: its pieces' sums in piece order, the new
//               value, its change (maximum over the grid), and
//               contrib = pr/q for the next iteration
// Every summation order is fixed, so results do not vary between runs.
//
// Convergence stays on the device: iteration i's largest change goes into
// slot i of a ring (atomicMax on the bit pattern, which orders non-negative
// doubles, spread over PR_STRIPES words so that the workgroups do not queue
// on one address), and both kernels of iteration i return at once when
// iteration i - 1 stored a change within the threshold (a skipped iteration
// leaves 0 in its slot, so the skip carries on).  The host queues iterations in
// batches, reads the batch's changes back once, and sizes the next batch
// from the observed contraction.
//
// The No-Sync variant (Alg. 3) drops the barrier between iterations: one
// launch of co-resident workgroups, each owning a contiguous run of pieces
// (balanced by arcs) and the vertices whose first piece it owns.  A
// workgroup sweeps its pieces, then finishes its vertices in place, reading
// whatever contributions and piece sums the other workgroups last stored
// (coherent agent-scope loads and stores, so values cross the XCDs' L2s),
// then publishes its largest change and reads everyone's.  It sweeps again
// while the largest published change exceeds the threshold, at most
// max_iters times.  No workgroup waits for another, so every workgroup ends
// after at most max_iters sweeps whether or not all are resident.  Results
// vary from run to run within the convergence tolerance.
//
// Loop perforation (Alg. 5), in either form: a vertex whose change is
// nonzero and below freeze_below is frozen, keeps its value and is skipped
// from then on (its pieces too); 0 freezes nothing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dg_host.h"

namespace dg {

uint64_t live_at(const dg_graph* g, uint32_t e);

constexpr uint32_t PR_THREADS = 256;
constexpr uint32_t PR_TILE = 4;          // buckets per build tile (4 x 16 slots = one wave step)
constexpr uint32_t PR_PIECE = 256;       // in-arcs per pull piece (16 lanes x 16)
constexpr uint32_t PR_RING = 128;        // slots of the per-iteration change ring
constexpr uint32_t PR_STRIPES = 64;      // words of a slot (one per lane): workgroup b raises word b mod 64
constexpr uint32_t PR_APPLY_GRID = 1024; // apply workgroups at most (16 per word)
constexpr uint32_t PR_BATCH_MAX = 48;    // iterations queued per host check (<= PR_RING / 2)

__device__ inline uint32_t pr_lane() { return __lane_id(); }

__global__ void k_pr_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Tiles of each live vertex's in-slab (entry V stays 0 for the scan).  The
// descriptors are copied once, so that count and fill read the same slabs
// even if a concurrent update regrows one (an old slab keeps every version
// visible at e).
__global__ void k_pr_ntiles(const uint64_t* desc, const uint8_t* live, uint32_t V, uint64_t* dsnap,
                            uint32_t* ntiles) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u <= V; u += gridDim.x * blockDim.x) {
    uint32_t t = 0;
    if (u < V) {
      const uint64_t d = live[u] ? desc[u] : 0;
      dsnap[u] = d;
      const uint32_t nb = d ? 1u << (d & 63) : 0;
      t = (nb + PR_TILE - 1) / PR_TILE;
    }
    ntiles[u] = t;
  }
}

// tile_v[t] = owning vertex, for the tiles tfirst[u] .. tfirst[u + 1).
__global__ void k_pr_tile_list(const uint32_t* tfirst, uint32_t V, uint32_t* tile_v) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < V; u += gridDim.x * blockDim.x)
    for (uint32_t t = tfirst[u]; t < tfirst[u + 1]; t++) tile_v[t] = u;
}

// One wave step over tile t: lane l reads slot l & 15 of bucket
// tfirst-relative 4 * k + (l >> 4); returns the source or EMPTY.
__device__ inline uint32_t pr_tile_slot(const Pool& p, const uint64_t* desc, const uint32_t* tfirst,
                                        const uint32_t* tile_v, uint32_t t, uint32_t e) {
  const uint32_t lane = pr_lane();
  const uint32_t u = tile_v[t];
  const Slab s = slab_of(p, desc[u]);
  const uint32_t b = (t - tfirst[u]) * PR_TILE + (lane >> 4);
  const int j = (int)(lane & 15);
  if (b >= s.nb) return EMPTY;
  uint32_t* bp = bucket_ptr(s, b);
  const uint32_t src = bp[j];
  if (src == EMPTY || !visible(*slot_stamp(bp, j, s.words), e)) return EMPTY;
  return src;
}

__global__ __launch_bounds__(PR_THREADS) void k_pr_count(Pool p, const uint64_t* desc, const uint32_t* tfirst,
                                                         const uint32_t* tile_v, uint32_t T, uint32_t e,
                                                         uint32_t* tcount) {
  const uint32_t nw = gridDim.x * (PR_THREADS / 64);
  for (uint32_t t = blockIdx.x * (PR_THREADS / 64) + (threadIdx.x >> 6); t < T; t += nw) {
    const uint32_t src = pr_tile_slot(p, desc, tfirst, tile_v, t, e);
    const uint32_t c = (uint32_t)__popcll(__ballot(src != EMPTY));
    if (pr_lane() == 0) tcount[t] = c;
  }
}

__global__ __launch_bounds__(PR_THREADS) void k_pr_fill(Pool p, const uint64_t* desc, const uint32_t* tfirst,
                                                        const uint32_t* tile_v, uint32_t T, uint32_t e,
                                                        const uint32_t* toff, uint32_t* csr) {
  const uint32_t nw = gridDim.x * (PR_THREADS / 64);
  const uint32_t lane = pr_lane();
  for (uint32_t t = blockIdx.x * (PR_THREADS / 64) + (threadIdx.x >> 6); t < T; t += nw) {
    const uint32_t src = pr_tile_slot(p, desc, tfirst, tile_v, t, e);
    const unsigned long long m = __ballot(src != EMPTY);
    const uint32_t pos = toff[t] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (src != EMPTY && pos < toff[t + 1]) csr[pos] = src;
  }
}

// The same as k_pr_fill, with each arc's weight (forward pool) beside it.
__global__ __launch_bounds__(PR_THREADS) void k_pr_fill_w(Pool p, const uint64_t* desc, const uint32_t* tfirst,
                                                          const uint32_t* tile_v, uint32_t T, uint32_t e,
                                                          const uint32_t* toff, uint32_t* csr, uint32_t* wts) {
  const uint32_t nw = gridDim.x * (PR_THREADS / 64);
  const uint32_t lane = pr_lane();
  for (uint32_t t = blockIdx.x * (PR_THREADS / 64) + (threadIdx.x >> 6); t < T; t += nw) {
    const uint32_t u = tile_v[t];
    const Slab s = slab_of(p, desc[u]);
    const uint32_t b = (t - tfirst[u]) * PR_TILE + (lane >> 4);
    const int j = (int)(lane & 15);
    uint32_t dst = EMPTY, w = 0;
    if (b < s.nb) {
      uint32_t* bp = bucket_ptr(s, b);
      dst = bp[j];
      if (dst != EMPTY && visible(*slot_stamp(bp, j, s.words), e)) w = bp[16 + j];
      else dst = EMPTY;
    }
    const unsigned long long m = __ballot(dst != EMPTY);
    const uint32_t pos = toff[t] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (dst != EMPTY && pos < toff[t + 1]) {
      csr[pos] = dst;
      wts[pos] = w;
    }
  }
}

// CSR start of each vertex (id order).
__global__ void k_pr_offsets(const uint32_t* tfirst, const uint32_t* toff, uint32_t V, uint32_t* off) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u <= V; u += gridDim.x * blockDim.x)
    off[u] = toff[tfirst[u]];
}

__global__ void k_pr_piece_list(const uint32_t* pfirst, uint32_t V, uint32_t* piece_v) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < V; u += gridDim.x * blockDim.x)
    for (uint32_t k = pfirst[u]; k < pfirst[u + 1]; k++) piece_v[k] = u;
}

__global__ void k_pr_clear_ring(unsigned long long* ring, uint32_t first, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n * PR_STRIPES; i += blockDim.x)
    ring[((first + i / PR_STRIPES) % PR_RING) * PR_STRIPES + i % PR_STRIPES] = 0ull;
}

__global__ void k_pr_outdeg(const uint32_t* csr, uint64_t m, uint32_t* q) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
    atomicAdd(&q[csr[i]], 1u);
}

// Sort keys: decreasing out-degree, ties kept in id order by the stable sort.
__global__ void k_pr_sort_keys(const uint32_t* q, uint32_t V, uint64_t* key, uint32_t* val) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < V; u += gridDim.x * blockDim.x) {
    key[u] = 0xFFFFFFFFull - q[u];
    val[u] = u;
  }
}

// Rank-order copies of the per-vertex data; deg_r and np_r leave entry V at
// 0 for their scans (into CSR offsets and first pieces).
__global__ void k_pr_rank(const uint32_t* order, const uint32_t* q, const uint8_t* live, const uint32_t* off,
                          uint32_t V, uint32_t* rank, uint32_t* q_r, uint8_t* live_r, uint32_t* deg_r,
                          uint32_t* np_r) {
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r <= V; r += gridDim.x * blockDim.x) {
    if (r == V) {
      deg_r[V] = 0;
      np_r[V] = 0;
      continue;
    }
    const uint32_t u = order[r];
    rank[u] = r;
    q_r[r] = q[u];
    live_r[r] = live[u];
    const uint32_t d = off[u + 1] - off[u];
    deg_r[r] = d;
    np_r[r] = (d + PR_PIECE - 1) / PR_PIECE;
  }
}

// Row moves: one 16-lane group per rank-order piece copies its arcs from the
// id-order CSR, mapping sources to ranks.
__global__ __launch_bounds__(PR_THREADS) void k_pr_permute(const uint32_t* order, const uint32_t* rank,
                                                           const uint32_t* off, const uint32_t* csr,
                                                           const uint32_t* off_r, const uint32_t* pfirst,
                                                           const uint32_t* piece_v, uint32_t P, uint32_t* csr_r) {
  const uint32_t j = threadIdx.x & 15;
  const uint32_t ng = gridDim.x * (PR_THREADS / 16);
  for (uint32_t p = blockIdx.x * (PR_THREADS / 16) + (threadIdx.x >> 4); p < P; p += ng) {
    const uint32_t r = piece_v[p];
    const uint32_t k = (p - pfirst[r]) * PR_PIECE;
    const uint32_t n = min(PR_PIECE, off_r[r + 1] - off_r[r] - k);
    const uint32_t from = off[order[r]] + k, to = off_r[r] + k;
    for (uint32_t i = j; i < n; i += 16) csr_r[to + i] = rank[csr[from + i]];
  }
}

// Ranks back to ids.
__global__ void k_pr_unrank(const uint32_t* rank, const double* pr_r, uint32_t V, double* pr) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < V; u += gridDim.x * blockDim.x)
    pr[u] = pr_r[rank[u]];
}

// pr = 1/n and contrib = pr/q on live vertices, 0 elsewhere.
__global__ void k_pr_init(const uint8_t* live, const uint32_t* q, uint32_t V, double inv_n, double* pr,
                          double* contrib) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < V; u += gridDim.x * blockDim.x) {
    const double x = live[u] ? inv_n : 0.0;
    pr[u] = x;
    contrib[u] = live[u] && q[u] ? x / (double)q[u] : 0.0;
  }
}

// Wave-uniform: did iteration it - 1 stop the loop?  Every wave reads the
// slot's words (lane l the word l) and takes their maximum.
__device__ inline bool pr_skip(const unsigned long long* ring, uint32_t it, unsigned long long thr_bits) {
  if (it == 0) return false;
  unsigned long long x = __hip_atomic_load(&ring[((it - 1) % PR_RING) * PR_STRIPES + pr_lane()],
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x <= thr_bits;
}

struct PrIter {
  const uint32_t* csr;
  const uint32_t* off;
  const uint32_t* pfirst;
  const uint32_t* piece_v;
  const uint8_t* live;
  const uint32_t* q;
  double* contrib;
  double* part;
  double* pr;
  unsigned long long* ring;
  uint8_t* frozen;       // perforation: vertices no longer recomputed
  uint32_t V, P;
  double base, d, freeze_below;
  unsigned long long thr_bits;
};

__global__ __launch_bounds__(PR_THREADS) void k_pr_pull(PrIter a, uint32_t it) {
  if (pr_skip(a.ring, it, a.thr_bits)) return;
  const uint32_t j = threadIdx.x & 15;
  const uint32_t ng = gridDim.x * (PR_THREADS / 16);
  for (uint32_t p0 = blockIdx.x * (PR_THREADS / 16); p0 < a.P; p0 += ng) {
    const uint32_t p = p0 + (threadIdx.x >> 4);   // group-uniform
    double s = 0.0;
    const uint32_t u = p < a.P ? a.piece_v[p] : 0;
    // the frozen flags are read only with perforation on (uniform test)
    if (p < a.P && !(a.freeze_below > 0.0 && a.frozen[u])) {
      const uint32_t b = a.off[u] + (p - a.pfirst[u]) * PR_PIECE;
      const uint32_t end = min(b + PR_PIECE, a.off[u + 1]);
      // four arcs per lane in flight: indices first, then their contributions
      for (uint32_t i0 = b + j; i0 < end; i0 += 64) {
        uint32_t src[4];
#pragma unroll
        for (int k = 0; k < 4; k++) src[k] = i0 + 16 * k < end ? a.csr[i0 + 16 * k] : EMPTY;
        double c[4];
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = src[k] != EMPTY ? a.contrib[src[k]] : 0.0;
        s += (c[0] + c[1]) + (c[2] + c[3]);
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
    if (p < a.P && j == 0) a.part[p] = s;
  }
}

__global__ __launch_bounds__(PR_THREADS) void k_pr_apply(PrIter a, uint32_t it) {
  if (pr_skip(a.ring, it, a.thr_bits)) return;
  __shared__ double wmax[PR_THREADS / 64];
  double ch = 0.0;
  for (uint32_t u = blockIdx.x * PR_THREADS + threadIdx.x; u < a.V; u += gridDim.x * PR_THREADS) {
    if (!a.live[u] || (a.freeze_below > 0.0 && a.frozen[u])) continue;
    double s = 0.0;
    for (uint32_t k = a.pfirst[u]; k < a.pfirst[u + 1]; k++) s += a.part[k];
    const double x = a.base + a.d * s;
    const double c = fabs(a.pr[u] - x);
    ch = fmax(ch, c);
    a.pr[u] = x;
    a.contrib[u] = a.q[u] ? x / (double)a.q[u] : 0.0;
    if (c != 0.0 && c < a.freeze_below) a.frozen[u] = 1;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ch = fmax(ch, __shfl_xor(ch, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = ch;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (uint32_t w = 1; w < PR_THREADS / 64; w++) m = fmax(m, wmax[w]);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
    unsigned long long* w = &a.ring[(it % PR_RING) * PR_STRIPES + blockIdx.x % PR_STRIPES];
    // the word only grows, so a read that is not above bits is safe to skip on
    if (bits > __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(w, bits);
  }
}

// ------------------------------------------------------------- No-Sync

// Work ranges: workgroup w owns pieces [pb[w], pb[w + 1]), split evenly by
// arcs + PR_PIECE_COST per piece, and vertices [vb[w], vb[w + 1]), those
// whose first piece (pfirst, rank order) lies in its range; the last
// workgroup also takes the vertices with no piece at the end.
constexpr uint64_t PR_PIECE_COST = 32;

__device__ inline uint64_t pr_piece_weight(const uint32_t* off, const uint32_t* pfirst, const uint32_t* piece_v,
                                           uint32_t P, uint32_t m, uint32_t p) {
  if (p >= P) return (uint64_t)m + PR_PIECE_COST * P;
  const uint32_t u = piece_v[p];
  return (uint64_t)off[u] + (uint64_t)(p - pfirst[u]) * PR_PIECE + PR_PIECE_COST * p;
}

__global__ void k_pr_async_bounds(const uint32_t* off, const uint32_t* pfirst, const uint32_t* piece_v, uint32_t P,
                                  uint32_t m, uint32_t V, uint32_t G, uint32_t* pb, uint32_t* vb) {
  const uint64_t W = (uint64_t)m + PR_PIECE_COST * P;
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w <= G; w += gridDim.x * blockDim.x) {
    uint32_t p = P, u = V;
    if (w == 0) {
      p = 0;
      u = 0;
    } else if (w < G) {
      const uint64_t target = W * w / G;
      uint32_t lo = 0, hi = P;   // first p with weight >= target
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (pr_piece_weight(off, pfirst, piece_v, P, m, mid) >= target) hi = mid;
        else lo = mid + 1;
      }
      p = lo;
      uint32_t a = 0, b = V;     // first u with pfirst[u] >= p
      while (a < b) {
        const uint32_t mid = a + (b - a) / 2;
        if (pfirst[mid] >= p) b = mid;
        else a = mid + 1;
      }
      u = a;
    }
    pb[w] = p;
    vb[w] = u;
  }
}

struct PrAsync {
  const uint32_t* csr;
  const uint32_t* off;
  const uint32_t* pfirst;
  const uint32_t* piece_v;
  const uint8_t* live;
  const uint32_t* q;
  const uint32_t* pb;
  const uint32_t* vb;
  double* contrib;
  double* part;
  double* pr;
  unsigned long long* err;   // per workgroup: its last published change (bit pattern)
  uint32_t* sweeps;          // per workgroup: sweeps run
  uint8_t* frozen;
  uint32_t G, max_iters;
  double base, d, freeze_below;
  unsigned long long thr_bits;
};

__device__ inline double pr_ld(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void pr_st(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(PR_THREADS) void k_pr_nosync(PrAsync a) {
  __shared__ double wmax[PR_THREADS / 64];
  __shared__ unsigned long long umax[PR_THREADS / 64];
  __shared__ int stop;
  const uint32_t w = blockIdx.x;
  const uint32_t p0 = a.pb[w], p1 = a.pb[w + 1], r0 = a.vb[w], r1 = a.vb[w + 1];
  const uint32_t j = threadIdx.x & 15, grp = threadIdx.x >> 4;
  uint32_t sweep = 0;
  for (;;) {
    // the workgroup's pieces (16-lane groups, group-uniform loop)
    for (uint32_t p = p0 + grp; p < p1; p += PR_THREADS / 16) {
      const uint32_t u = a.piece_v[p];
      if (a.freeze_below > 0.0 && a.frozen[u]) continue;   // group-uniform
      const uint32_t b = a.off[u] + (p - a.pfirst[u]) * PR_PIECE;
      const uint32_t end = min(b + PR_PIECE, a.off[u + 1]);
      double s = 0.0;
      for (uint32_t i0 = b + j; i0 < end; i0 += 64) {
        uint32_t src[4];
#pragma unroll
        for (int k = 0; k < 4; k++) src[k] = i0 + 16 * k < end ? a.csr[i0 + 16 * k] : EMPTY;
        double c[4];
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = src[k] != EMPTY ? pr_ld(&a.contrib[src[k]]) : 0.0;
        s += (c[0] + c[1]) + (c[2] + c[3]);
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
      if (j == 0) pr_st(&a.part[p], s);
    }
    __syncthreads();
    // the workgroup's vertices, from the latest sums of their pieces
    double ch = 0.0;
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += PR_THREADS) {
      if (!a.live[r] || (a.freeze_below > 0.0 && a.frozen[r])) continue;
      double s = 0.0;
      for (uint32_t k = a.pfirst[r]; k < a.pfirst[r + 1]; k++) s += pr_ld(&a.part[k]);
      const double x = a.base + a.d * s;
      const double c = fabs(a.pr[r] - x);
      ch = fmax(ch, c);
      a.pr[r] = x;
      pr_st(&a.contrib[r], a.q[r] ? x / (double)a.q[r] : 0.0);
      if (c != 0.0 && c < a.freeze_below) a.frozen[r] = 1;
    }
    sweep++;
    // publish this workgroup's change, then take the largest published one
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ch = fmax(ch, __shfl_xor(ch, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = ch;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = wmax[0];
      for (uint32_t k = 1; k < PR_THREADS / 64; k++) m = fmax(m, wmax[k]);
      __hip_atomic_store(&a.err[w], (unsigned long long)__double_as_longlong(m), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned long long mx = 0;
    for (uint32_t t = threadIdx.x; t < a.G; t += PR_THREADS) {
      const unsigned long long x = __hip_atomic_load(&a.err[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      mx = x > mx ? x : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long y = __shfl_xor(mx, o, 64);
      mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63) == 0) umax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long m = umax[0];
      for (uint32_t k = 1; k < PR_THREADS / 64; k++) m = umax[k] > m ? umax[k] : m;
      stop = m <= a.thr_bits || sweep >= a.max_iters;
    }
    __syncthreads();
    if (stop) break;
  }
  if (threadIdx.x == 0) a.sweeps[w] = sweep;
}

static uint32_t pr_grid(uint64_t units, uint32_t per_block, uint32_t cap = 8192) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((units + per_block - 1) / per_block, cap));
}

void free_pr_scratch(PrScratch& s) {
  release(s.live); release(s.dsnap); release(s.ntiles); release(s.tile_v); release(s.tcount); release(s.off);
  release(s.pfirst); release(s.piece_v); release(s.csr); release(s.q); release(s.contrib);
  release(s.part); release(s.ring); release(s.scan); release(s.sort); release(s.key0); release(s.key1);
  release(s.val0); release(s.val1); release(s.rank); release(s.q_r); release(s.live_r); release(s.off_r);
  release(s.csr_r); release(s.pr_r); release(s.pb); release(s.vb); release(s.werr); release(s.sweeps); release(s.frozen);
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
}

static hipError_t pr_scan(PrScratch& s, uint32_t* data, uint64_t n, hipStream_t st) {
  hipError_t e = ensure(s.scan, scan_scratch_words(n) * 4 + 64);
  if (e != hipSuccess) return e;
  exclusive_scan_u32(data, n, s.scan.as<uint32_t>(), st);
  return hipGetLastError();
}

// ------------------------------------------------------ snapshot build

hipError_t snapshot_live(dg_graph* g, uint32_t e, DevBuf& live, hipStream_t st) {
  PrScratch& s = g->pr;
  const uint32_t V = g->cfg.v_capacity;
  hipError_t he;
  if (!s.host &&
      (he = hipHostMalloc(&s.host, std::max<size_t>(V, PR_RING * PR_STRIPES * 8) + 64, hipHostMallocDefault)) !=
          hipSuccess)
    return he;
  // the pinned block may still feed an earlier copy
  if ((he = hipStreamSynchronize(st)) != hipSuccess) return he;
  uint8_t* hl = static_cast<uint8_t*>(s.host);
  for (uint32_t v = 0; v < V; v++) hl[v] = g->vfirst[v] != 0 && g->vfirst[v] <= e;
  for (const uint32_t v : g->vtoggled) hl[v] = alive_at(g, v, e) ? 1 : 0;
  if ((he = ensure(live, V + 64)) != hipSuccess) return he;
  return hipMemcpyAsync(live.p, hl, V, hipMemcpyHostToDevice, st);
}

hipError_t snapshot_csr(dg_graph* g, uint32_t e, const Pool& pool, const uint64_t* desc, const uint8_t* live,
                        DevBuf& off_buf, DevBuf& csr_buf, uint32_t* m_out, hipStream_t st, DevBuf* wts) {
  PrScratch& s = g->pr;
  const uint32_t V = g->cfg.v_capacity;
  hipError_t he;
  const uint64_t T_max = pool.cap / PR_TILE + V + 1;
  if ((he = ensure(s.ntiles, (V + 1ull) * 4)) != hipSuccess || (he = ensure(s.dsnap, V * 8ull + 64)) != hipSuccess ||
      (he = ensure(s.tile_v, T_max * 4)) != hipSuccess || (he = ensure(s.tcount, (T_max + 1) * 4)) != hipSuccess ||
      (he = ensure(off_buf, (V + 1ull) * 4)) != hipSuccess)
    return he;
  uint32_t* tfirst = s.ntiles.as<uint32_t>();
  k_pr_ntiles<<<pr_grid(V + 1ull, 256), 256, 0, st>>>(desc, live, V, s.dsnap.as<uint64_t>(), tfirst);
  desc = s.dsnap.as<uint64_t>();
  if ((he = pr_scan(s, tfirst, V + 1ull, st)) != hipSuccess) return he;
  // the tile total (tfirst[V]) is needed on the host before the tile kernels
  if ((he = hipMemcpyAsync(s.host, tfirst + V, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return he;
  uint32_t T;
  std::memcpy(&T, s.host, 4);
  if (T > T_max) return hipErrorInvalidValue;
  k_pr_tile_list<<<pr_grid(V, 256), 256, 0, st>>>(tfirst, V, s.tile_v.as<uint32_t>());
  uint32_t* tc = s.tcount.as<uint32_t>();
  k_pr_fill_u32<<<1, 64, 0, st>>>(tc + T, 1, 0u);
  if (T)
    k_pr_count<<<pr_grid(T, PR_THREADS / 64), PR_THREADS, 0, st>>>(pool, desc, tfirst, s.tile_v.as<uint32_t>(), T, e,
                                                                   tc);
  if ((he = pr_scan(s, tc, T + 1ull, st)) != hipSuccess) return he;
  if ((he = hipMemcpyAsync(s.host, tc + T, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return he;
  uint32_t m;
  std::memcpy(&m, s.host, 4);
  if ((he = ensure(csr_buf, (uint64_t)m * 4 + 64)) != hipSuccess) return he;
  if (wts && (he = ensure(*wts, (uint64_t)m * 4 + 64)) != hipSuccess) return he;
  if (T && wts)
    k_pr_fill_w<<<pr_grid(T, PR_THREADS / 64), PR_THREADS, 0, st>>>(pool, desc, tfirst, s.tile_v.as<uint32_t>(), T,
                                                                    e, tc, csr_buf.as<uint32_t>(),
                                                                    wts->as<uint32_t>());
  else if (T)
    k_pr_fill<<<pr_grid(T, PR_THREADS / 64), PR_THREADS, 0, st>>>(pool, desc, tfirst, s.tile_v.as<uint32_t>(), T, e,
                                                                  tc, csr_buf.as<uint32_t>());
  k_pr_offsets<<<pr_grid(V + 1ull, 256), 256, 0, st>>>(tfirst, tc, V, off_buf.as<uint32_t>());
  *m_out = m;
  return hipGetLastError();
}

static uint32_t pr_resident(const void* kernel) {
  int per_cu = 0, cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, PR_THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)(per_cu * cus);
}

__global__ void k_pr_fill_u64(unsigned long long* p, uint32_t n, unsigned long long v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

dg_status pagerank_dev(dg_graph* g, uint32_t e, double damping, double threshold, double freeze_below,
                       uint32_t max_iters, double* pr, uint32_t* iters, double* last_change, hipStream_t st,
                       bool nosync) {
  PrScratch& s = g->pr;
  const uint32_t V = g->cfg.v_capacity;
  *iters = 0;
  *last_change = 0.0;
  auto fail_hip = [&](hipError_t he, const char* where) {
    g->err = std::string("pagerank ") + where + ": " + hipGetErrorString(he);
    return DG_E_HIP;
  };
  if (threshold == 0.0) threshold = 0.0;   // -0.0 would compare above every change
  k_pr_fill_u32<<<pr_grid(2ull * V, 256), 256, 0, st>>>(reinterpret_cast<uint32_t*>(pr), 2ull * V, 0u);
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail_hip(he, "clear");
  const uint64_t n_live = live_at(g, e);
  // the loop runs while the change exceeds the threshold, from a change of 1
  if (n_live == 0 || max_iters == 0 || !(threshold < 1.0)) return DG_OK;

  if ((he = snapshot_live(g, e, s.live, st)) != hipSuccess) return fail_hip(he, "liveness");
  // in-arcs: the reverse pool, or the forward one of an undirected graph
  const bool und = g->st.undirected != 0;
  uint32_t m = 0;
  if ((he = snapshot_csr(g, e, und ? g->st.fp : g->st.rp, und ? g->st.fdesc : g->st.rdesc, s.live.as<uint8_t>(),
                         s.off, s.csr, &m, st)) != hipSuccess)
    return fail_hip(he, "snapshot");
  if ((he = ensure(s.pfirst, (V + 1ull) * 4)) != hipSuccess || (he = ensure(s.q, V * 4ull + 64)) != hipSuccess ||
      (he = ensure(s.contrib, V * 8ull + 64)) != hipSuccess || (he = ensure(s.ring, PR_RING * PR_STRIPES * 8)) != hipSuccess)
    return fail_hip(he, "alloc");
  const uint64_t P_max = (uint64_t)V + m / PR_PIECE + 1;
  if ((he = ensure(s.piece_v, P_max * 4)) != hipSuccess || (he = ensure(s.part, P_max * 8)) != hipSuccess)
    return fail_hip(he, "alloc");
  uint32_t* off = s.off.as<uint32_t>();
  k_pr_fill_u32<<<pr_grid(V, 256), 256, 0, st>>>(s.q.as<uint32_t>(), V, 0u);
  if (m) k_pr_outdeg<<<pr_grid(m, 256), 256, 0, st>>>(s.csr.as<uint32_t>(), m, s.q.as<uint32_t>());

  // rank order: decreasing out-degree
  if ((he = ensure(s.key0, V * 8ull + 64)) != hipSuccess || (he = ensure(s.key1, V * 8ull + 64)) != hipSuccess ||
      (he = ensure(s.val0, V * 4ull + 64)) != hipSuccess || (he = ensure(s.val1, V * 4ull + 64)) != hipSuccess ||
      (he = ensure(s.sort, sort_scratch_words(V) * 4 + 64)) != hipSuccess ||
      (he = ensure(s.rank, V * 4ull + 64)) != hipSuccess || (he = ensure(s.q_r, V * 4ull + 64)) != hipSuccess ||
      (he = ensure(s.live_r, V + 64ull)) != hipSuccess || (he = ensure(s.off_r, (V + 1ull) * 4)) != hipSuccess ||
      (he = ensure(s.csr_r, (uint64_t)m * 4 + 64)) != hipSuccess || (he = ensure(s.pr_r, V * 8ull + 64)) != hipSuccess)
    return fail_hip(he, "alloc");
  k_pr_sort_keys<<<pr_grid(V, 256), 256, 0, st>>>(s.q.as<uint32_t>(), V, s.key0.as<uint64_t>(), s.val0.as<uint32_t>());
  const bool alt = radix_sort_pairs(s.key0.as<uint64_t>(), s.val0.as<uint32_t>(), s.key1.as<uint64_t>(),
                                    s.val1.as<uint32_t>(), V, 32, s.sort.as<uint32_t>(), st);
  const uint32_t* order = alt ? s.val1.as<uint32_t>() : s.val0.as<uint32_t>();
  uint32_t* pfirst = s.pfirst.as<uint32_t>();
  uint32_t* off_r = s.off_r.as<uint32_t>();
  k_pr_rank<<<pr_grid(V + 1ull, 256), 256, 0, st>>>(order, s.q.as<uint32_t>(), s.live.as<uint8_t>(), off, V,
                                                    s.rank.as<uint32_t>(), s.q_r.as<uint32_t>(),
                                                    s.live_r.as<uint8_t>(), off_r, pfirst);
  if ((he = pr_scan(s, off_r, V + 1ull, st)) != hipSuccess) return fail_hip(he, "offset scan");
  if ((he = pr_scan(s, pfirst, V + 1ull, st)) != hipSuccess) return fail_hip(he, "piece scan");
  k_pr_piece_list<<<pr_grid(V, 256), 256, 0, st>>>(pfirst, V, s.piece_v.as<uint32_t>());
  if ((he = hipMemcpyAsync(s.host, pfirst + V, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess)
    return fail_hip(he, "piece total");
  uint32_t P;
  std::memcpy(&P, s.host, 4);
  if (P > P_max) {
    g->err = "pagerank: piece count exceeds its bound";
    return DG_E_HIP;
  }
  if (P)
    k_pr_permute<<<pr_grid(P, PR_THREADS / 16, 16384), PR_THREADS, 0, st>>>(
        order, s.rank.as<uint32_t>(), off, s.csr.as<uint32_t>(), off_r, pfirst, s.piece_v.as<uint32_t>(), P,
        s.csr_r.as<uint32_t>());
  double* pr_r = s.pr_r.as<double>();
  k_pr_init<<<pr_grid(V, 256), 256, 0, st>>>(s.live_r.as<uint8_t>(), s.q_r.as<uint32_t>(), V, 1.0 / (double)n_live,
                                             pr_r, s.contrib.as<double>());
  k_pr_fill_u32<<<1, 256, 0, st>>>(reinterpret_cast<uint32_t*>(s.ring.p), PR_RING * PR_STRIPES * 2, 0u);
  if ((he = ensure(s.frozen, V + 64ull)) != hipSuccess) return fail_hip(he, "alloc");
  k_pr_fill_u32<<<pr_grid(V / 4 + 1, 256), 256, 0, st>>>(s.frozen.as<uint32_t>(), V / 4 + 1, 0u);

  PrIter a{s.csr_r.as<uint32_t>(),
           off_r,
           pfirst,
           s.piece_v.as<uint32_t>(),
           s.live_r.as<uint8_t>(),
           s.q_r.as<uint32_t>(),
           s.contrib.as<double>(),
           s.part.as<double>(),
           pr_r,
           reinterpret_cast<unsigned long long*>(s.ring.p),
           s.frozen.as<uint8_t>(),
           V,
           P,
           (1.0 - damping) / (double)n_live,
           damping,
           freeze_below,
           0};
  std::memcpy(&a.thr_bits, &threshold, 8);
  const uint32_t g_pull = pr_grid(P, PR_THREADS / 16, 16384), g_apply = pr_grid(V, PR_THREADS, PR_APPLY_GRID);
  if (nosync) {
    // co-resident workgroups, about 64 pieces each at least
    const uint32_t G = std::max<uint32_t>(1, std::min<uint32_t>(pr_resident((const void*)k_pr_nosync), (P + 63) / 64));
    if ((he = ensure(s.pb, (G + 1ull) * 4)) != hipSuccess || (he = ensure(s.vb, (G + 1ull) * 4)) != hipSuccess ||
        (he = ensure(s.werr, G * 8ull)) != hipSuccess || (he = ensure(s.sweeps, G * 4ull)) != hipSuccess)
      return fail_hip(he, "alloc");
    k_pr_async_bounds<<<pr_grid(G + 1ull, 256), 256, 0, st>>>(off_r, pfirst, s.piece_v.as<uint32_t>(), P, m, V, G,
                                                              s.pb.as<uint32_t>(), s.vb.as<uint32_t>());
    // piece sums of the starting values, so a vertex never reads an unset one
    k_pr_pull<<<g_pull, PR_THREADS, 0, st>>>(a, 0);
    // every workgroup's change starts at 1, as the loop's does
    k_pr_fill_u64<<<pr_grid(G, 256), 256, 0, st>>>(s.werr.as<unsigned long long>(), G, 0x3FF0000000000000ull);
    PrAsync x{a.csr,
              a.off,
              a.pfirst,
              a.piece_v,
              a.live,
              a.q,
              s.pb.as<uint32_t>(),
              s.vb.as<uint32_t>(),
              a.contrib,
              a.part,
              pr_r,
              s.werr.as<unsigned long long>(),
              s.sweeps.as<uint32_t>(),
              a.frozen,
              G,
              max_iters,
              a.base,
              a.d,
              a.freeze_below,
              a.thr_bits};
    {
      ProfScope ps(g, KID_PAGERANK_NOSYNC, st);
      k_pr_nosync<<<G, PR_THREADS, 0, st>>>(x);
    }
    if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "nosync launch");
    unsigned long long* hw = static_cast<unsigned long long*>(s.host);
    std::vector<unsigned long long> errs(G);
    std::vector<uint32_t> sw(G);
    if ((he = hipMemcpyAsync(hw, s.werr.p, G * 8ull, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (he = hipStreamSynchronize(st)) != hipSuccess)
      return fail_hip(he, "nosync read back");
    std::memcpy(errs.data(), hw, G * 8ull);
    if ((he = hipMemcpyAsync(hw, s.sweeps.p, G * 4ull, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (he = hipStreamSynchronize(st)) != hipSuccess)
      return fail_hip(he, "nosync read back");
    std::memcpy(sw.data(), hw, G * 4ull);
    unsigned long long mx = 0;
    uint64_t total = 0;
    for (uint32_t w = 0; w < G; w++) {
      mx = std::max(mx, errs[w]);
      *iters = std::max(*iters, sw[w]);
      total += sw[w];
    }
    std::memcpy(last_change, &mx, 8);
    // arcs examined: every workgroup's share of the arcs times its sweeps, taken as the mean
    prof_arcs(g, KID_PAGERANK_NOSYNC, (uint64_t)((double)m * (double)total / (double)G));
    k_pr_unrank<<<pr_grid(V, 256), 256, 0, st>>>(s.rank.as<uint32_t>(), pr_r, V, pr);
    if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "unrank");
    return DG_OK;
  }
  unsigned long long* ring = a.ring;
  unsigned long long* hw = static_cast<unsigned long long*>(s.host);
  double hc[PR_BATCH_MAX];
  uint32_t queued = 0, batch = 8;
  double prev_change = 0.0;
  for (;;) {
    const uint32_t b = std::min(batch, max_iters - queued);
    // clear the batch's slots (the previous batch's last slot stays readable)
    k_pr_clear_ring<<<1, 64, 0, st>>>(ring, queued % PR_RING, b);
    for (uint32_t i = queued; i < queued + b; i++) {
      ProfScope ps(g, KID_PAGERANK, st);
      k_pr_pull<<<g_pull, PR_THREADS, 0, st>>>(a, i);
      k_pr_apply<<<g_apply, PR_THREADS, 0, st>>>(a, i);
    }
    if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "launch");
    const uint32_t r0 = queued % PR_RING, n1 = std::min(b, PR_RING - r0);
    const size_t row = PR_STRIPES * 8ull;
    if ((he = hipMemcpyAsync(hw, ring + r0 * PR_STRIPES, n1 * row, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (b > n1 && (he = hipMemcpyAsync(hw + n1 * PR_STRIPES, ring, (b - n1) * row, hipMemcpyDeviceToHost, st)) !=
                       hipSuccess))
      return fail_hip(he, "read back");
    if ((he = hipStreamSynchronize(st)) != hipSuccess) return fail_hip(he, "sync");
    for (uint32_t i = 0; i < b; i++) {
      unsigned long long x = 0;
      for (uint32_t k = 0; k < PR_STRIPES; k++) x = std::max(x, hw[i * PR_STRIPES + k]);
      std::memcpy(&hc[i], &x, 8);
    }
    for (uint32_t i = 0; i < b; i++) {
      const double c = hc[i];
      if (c <= threshold) {
        *iters = queued + i + 1;
        *last_change = c;
        prof_arcs(g, KID_PAGERANK, (uint64_t)m * (i + 1));
        break;
      }
    }
    if (*iters) break;
    prof_arcs(g, KID_PAGERANK, (uint64_t)m * b);
    queued += b;
    const double last = hc[b - 1];
    if (queued >= max_iters) {
      *iters = queued;
      *last_change = last;
      break;
    }
    // iterations left at the observed contraction, plus one
    const double r = b >= 2 && hc[b - 2] > 0 ? last / hc[b - 2] : (prev_change > 0 ? last / prev_change : 0.9);
    prev_change = last;
    uint32_t want = PR_BATCH_MAX;
    if (r > 0 && r < 1 && last > threshold) {
      const double k = std::log(threshold / last) / std::log(r);
      if (k < PR_BATCH_MAX) want = (uint32_t)std::max(1.0, std::ceil(k) + 1);
    }
    batch = want;
  }
  k_pr_unrank<<<pr_grid(V, 256), 256, 0, st>>>(s.rank.as<uint32_t>(), pr_r, V, pr);
  if ((he = hipGetLastError()) != hipSuccess) return fail_hip(he, "unrank");
  return DG_OK;
}

}  // namespace dg
