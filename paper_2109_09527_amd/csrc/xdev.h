// Device helpers shared by the serving loop's executors (continuous
// multi-source BFS and SSSP): their slots carry epochs of their own, so an
// arc's visibility is the mask of slots whose epoch lies in its lifetime.
#pragma once

#include <algorithm>

#include "frontier.h"
#include "xexec.h"

namespace dg {

// Slot j of the flat positions f0 + 4 grp + k (k < 4) of a chunk, with its
// weight (WITH_W) and stamp (EMPTY and 0 past the chunk's end); item[k] is
// the lane holding the owning frontier item.  Visibility is decided per
// slot by the caller.
struct PairsSt {
  uint32_t d[4];
  int32_t w[4];
  uint64_t stamp[4];
  uint32_t item[4];
};

template <bool WITH_W>
__device__ inline PairsSt load_pairs_stamps(const Pool& p, const ChunkView& cv, uint32_t f0, uint32_t grp,
                                            uint32_t j) {
  PairsSt r;
  uint32_t* bp[4];
  // the owner of f0 is the last lane whose item starts at or before it
  const unsigned long long m0 = __ballot(cv.start <= f0);
  const uint32_t L0 = (uint32_t)__popcll(m0) - 1;
  uint32_t nxt[15];
#pragma unroll
  for (int m = 1; m < 16; m++)
    nxt[m - 1] = L0 + m < 64 ? (uint32_t)__builtin_amdgcn_readlane((int)cv.start, (int)(L0 + m)) : 0xFFFFFFFFu;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t f = f0 + grp * 4 + k;
    uint32_t own = L0;
#pragma unroll
    for (int m = 0; m < 15; m++) own += nxt[m] <= f ? 1u : 0u;
    const uint64_t desc = __shfl(cv.desc, (int)own, 64);
    const uint32_t st = __shfl(cv.start, (int)own, 64);
    r.item[k] = own;
    r.d[k] = EMPTY;
    r.w[k] = 0;
    r.stamp[k] = 0;
    bp[k] = p.base;
    if (f < cv.hi) {
      const Slab s = slab_of(p, desc);
      bp[k] = bucket_ptr(s, f - st);
      r.d[k] = bp[k][j];
      if (WITH_W) r.w[k] = (int32_t)bp[k][16 + j];
    }
  }
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (r.d[k] != EMPTY) r.stamp[k] = *slot_stamp(bp[k], j, p.words);
  return r;
}

// Number of active epochs below x (ue ascending, padded with 0xFFFFFFFF).
__device__ inline uint32_t xb_below(const uint32_t* ue, uint32_t x) {
  uint32_t pos = 0;
#pragma unroll
  for (uint32_t s = 64; s > 0; s >>= 1)
    if (pos + s <= 64 && ue[pos + s - 1] < x) pos += s;
  return pos;
}

// Slots that see an arc of lifetime [birth, death): epoch >= birth and
// epoch < death.
__device__ inline unsigned long long xb_vmask(uint64_t stamp, const uint32_t* ue, const unsigned long long* cm,
                                              uint32_t e_lo, uint32_t e_hi, unsigned long long all) {
  const uint32_t birth = (uint32_t)stamp, death = (uint32_t)(stamp >> 32);
  if (birth <= e_lo && death > e_hi) return all;
  return cm[xb_below(ue, death)] & ~cm[xb_below(ue, birth)];
}

__device__ inline unsigned long long wave_or_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x;
}

// Workgroups of `kernel` resident on the current device at once.
inline uint32_t xb_resident(const void* kernel) {
  int per_cu = 0, cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, Q_THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  return (uint32_t)std::max(1, per_cu * cus);
}

}  // namespace dg
