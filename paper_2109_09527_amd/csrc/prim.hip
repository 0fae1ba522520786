// Device-wide primitives: exclusive scan of u32 and a stable LSD radix sort
// of (u64 key, u32 value) pairs with 8-bit digits.
//
// Radix sort, per digit pass (Satish, Harris & Garland, IPDPS 2009 layout):
//   k_rs_hist    per 2048-key tile, digit histogram -> hist[digit][tile]
//   scan         exclusive scan of hist in digit-major order -> global offsets
//                (up to 64 tiles, the scatter sums its own offsets instead)
//   k_rs_scatter per tile, stable rank of each key among equal digits of the
//                tile (wave ballots on the 8 digit bits give the lanes sharing
//                a digit; per-wave counts combine in wave order through LDS),
//                then write to offset[digit][tile] + rank.
#include "dg_host.h"

namespace dg {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[SCAN_THREADS / 64];
  uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_THREADS / 64; w++) {
    uint32_t s = wsum[w];
    if ((uint32_t)w < wave) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t* data, uint64_t n, uint32_t* partials) {
  uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++)
    if (base + i < n) s += data[base + i];
  uint32_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(uint32_t* data, uint64_t n, const uint32_t* partials) {
  uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    v[i] = base + i < n ? data[base + i] : 0;
    s += v[i];
  }
  uint32_t tot;
  uint32_t off = block_exclusive_scan(s, &tot) + (partials ? partials[blockIdx.x] : 0);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    if (base + i < n) data[base + i] = off;
    off += v[i];
  }
}

// Exclusive scan of up to SCAN_SINGLE_MAX values by one workgroup: tiles in
// order with a running carry.  For the short arrays of a batch's sort
// passes one launch costs less than the reduce / scan / down-sweep chain.
constexpr uint64_t SCAN_SINGLE_MAX = 32ull * SCAN_TILE;
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_single(uint32_t* data, uint64_t n) {
  uint32_t carry = 0;
  for (uint64_t t0 = 0; t0 < n; t0 += SCAN_TILE) {
    const uint64_t base = t0 + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
      v[i] = base + i < n ? data[base + i] : 0;
      s += v[i];
    }
    uint32_t tot;
    uint32_t off = block_exclusive_scan(s, &tot) + carry;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
      if (base + i < n) data[base + i] = off;
      off += v[i];
    }
    carry += tot;
  }
}

uint64_t scan_scratch_words(uint64_t n) {
  uint64_t w = 0;
  while (n > (uint64_t)SCAN_TILE) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    w += n;
  }
  return w + 1;
}

void exclusive_scan_u32(uint32_t* data, uint64_t n, uint32_t* scratch, hipStream_t s) {
  if (n == 0) return;
  if (n <= (uint64_t)SCAN_TILE) {
    k_scan_down<<<1, SCAN_THREADS, 0, s>>>(data, n, nullptr);
    return;
  }
  if (n <= SCAN_SINGLE_MAX) {
    k_scan_single<<<1, SCAN_THREADS, 0, s>>>(data, n);
    return;
  }
  uint64_t nblk = (n + SCAN_TILE - 1) / SCAN_TILE;
  k_scan_reduce<<<(uint32_t)nblk, SCAN_THREADS, 0, s>>>(data, n, scratch);
  exclusive_scan_u32(scratch, nblk, scratch + nblk, s);
  k_scan_down<<<(uint32_t)nblk, SCAN_THREADS, 0, s>>>(data, n, scratch);
}

// ------------------------------------------------------------ radix sort

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_WAVES = RS_THREADS / 64;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t* keys, uint32_t n, int shift,
                                                        uint32_t* hist, uint32_t ntile) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int r = 0; r < RS_ITEMS; r++) {
    uint64_t i = base + (uint64_t)r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

// Up to this many tiles, the scatter computes its tile's offsets from the
// histograms itself (a row of at most RS_FUSED_TILES counts per digit, then
// a workgroup scan of the digit totals) and the pass needs no scan launch.
constexpr uint32_t RS_FUSED_TILES = 64;

// offs: the scanned histograms, or, when `scanned` is false, the histograms
// themselves (ntile <= RS_FUSED_TILES).
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t* kin, const uint32_t* vin,
                                                           uint64_t* kout, uint32_t* vout, uint32_t n,
                                                           int shift, const uint32_t* offs, uint32_t ntile,
                                                           int scanned) {
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[RS_WAVES][256];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (scanned) {
    gbase[tid] = offs[(uint64_t)tid * ntile + blockIdx.x];
  } else {
    // digit tid: its count in the tiles before this one and in all tiles
    const uint32_t* row = offs + (uint64_t)tid * ntile;
    uint32_t before = 0, total = 0;
#pragma unroll 8
    for (uint32_t t = 0; t < ntile; t++) {
      const uint32_t h = row[t];
      before += t < blockIdx.x ? h : 0u;
      total += h;
    }
    uint32_t all;
    gbase[tid] = block_exclusive_scan(total, &all) + before;
  }
  run[tid] = 0;
  const unsigned long long lt = (1ull << lane) - 1ull;
  uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; r++) {
#pragma unroll
    for (int w = 0; w < RS_WAVES; w++) wcnt[w][tid] = 0;
    __syncthreads();
    uint64_t i = base + (uint64_t)r * RS_THREADS + tid;
    bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    uint32_t val = valid ? vin[i] : 0;
    uint32_t d = (uint32_t)(key >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      bool bit = (d >> b) & 1u;
      unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    uint32_t rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pre = run[d];
      for (uint32_t w = 0; w < wave; w++) pre += wcnt[w][d];
      uint32_t pos = gbase[d] + pre + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; w++) add += wcnt[w][tid];
    run[tid] += add;
    __syncthreads();
  }
}

uint64_t sort_scratch_words(uint32_t n) {
  uint64_t ntile = ((uint64_t)n + RS_TILE - 1) / RS_TILE;
  uint64_t h = 256 * ntile;
  return h + scan_scratch_words(h);
}

// Sorts n pairs by key bits [0, bits).  Data starts in (k0, v0); the result
// is returned in (k0, v0) if the return value is false, else in (k1, v1).
bool radix_sort_pairs(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint32_t n, int bits,
                      uint32_t* scratch, hipStream_t s) {
  if (n <= 1) return false;
  uint32_t ntile = (n + RS_TILE - 1) / RS_TILE;
  uint32_t* hist = scratch;
  uint32_t* scan_tmp = scratch + 256ull * ntile;
  bool alt = false;
  for (int shift = 0; shift < bits; shift += 8) {
    const uint64_t* ki = alt ? k1 : k0;
    const uint32_t* vi = alt ? v1 : v0;
    uint64_t* ko = alt ? k0 : k1;
    uint32_t* vo = alt ? v0 : v1;
    k_rs_hist<<<ntile, RS_THREADS, 0, s>>>(ki, n, shift, hist, ntile);
    const bool fused = ntile <= RS_FUSED_TILES;
    if (!fused) exclusive_scan_u32(hist, 256ull * ntile, scan_tmp, s);
    k_rs_scatter<<<ntile, RS_THREADS, 0, s>>>(ki, vi, ko, vo, n, shift, hist, ntile, fused ? 0 : 1);
    alt = !alt;
  }
  return alt;
}

}  // namespace dg
