// Internal layout of the versioned, epoch-stamped, hash-bucketed adjacency
// store and the device helpers shared by the update and query kernels.
//
// Store (one per graph, in HBM):
//   fdesc[v] / rdesc[v]  slab descriptor of v's out-arcs / in-arcs:
//                        (first bucket index << 6) | log2(bucket count);
//                        0 = no slab (bucket 0 of each pool is never used).
//   fused[v] / rused[v]  slots of the slab in use (live + tombstoned versions)
//   fpool                forward buckets, 64 words each:
//                          [0,16)  dst      (EMPTY = 0xFFFFFFFF)
//                          [16,32) weight
//                          [32,64) stamp[16] as u64 = birth | death << 32
//   rpool                reverse buckets, 48 words each: src[16], stamp[16]
//   fsum / rsum          per-bucket summary, four u32: the largest birth of
//                        any version in the bucket, a 16-bit mask of the
//                        slots whose version has been tombstoned, the
//                        largest death among them, and a spare word.  With
//                        no concurrent writer, a scan at epoch e >= that
//                        birth reads no stamp at all when every tombstone
//                        died at or before e, and otherwise only the stamps
//                        of tombstoned slots.
//   alive[v]             liveness at the latest epoch
// A version is visible at epoch e iff birth <= e < death; death = INF for
// the current version.  A slot's bucket is hash(dst) mod buckets, with
// linear probing to the next bucket when one is full; slots of a bucket fill
// in order, so a bucket's used slots are a prefix.  Undirected graphs store
// both arcs in the forward pool and have no reverse pool.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dg {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;
constexpr uint32_t INF_EPOCH = 0xFFFFFFFFu;
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int BSLOTS = 16;
constexpr int SUM_WORDS = 4;   // bucket summary: max birth, tomb mask, max death, spare
constexpr int FWD_WORDS = 64;
constexpr int REV_WORDS = 48;
constexpr uint64_t EMPTY_STAMP = ~0ull;
constexpr int32_t DIST_INF = 0x7fffffff;

// Batch status bits, accumulated on the device during one update batch.
enum : uint32_t { F_BAD_TYPE = 1, F_BAD_VERTEX = 2, F_BAD_WEIGHT = 4, F_OOM = 8 };

struct Pool {
  uint32_t* base;       // bucket b starts at base + b * words
  uint32_t* sum;        // bucket b's summary at sum[4b .. 4b+4)
  uint64_t cap;         // buckets
  uint32_t words;       // 64 (forward) or 48 (reverse)
};

struct Store {
  uint32_t V;
  int undirected;
  uint64_t* fdesc;
  uint64_t* rdesc;
  uint32_t* fused;
  uint32_t* rused;
  Pool fp, rp;
  unsigned long long* cursor;   // [0] next free forward bucket, [1] reverse
  uint8_t* alive;
};

// Slab view of one vertex in one pool.
struct Slab {
  uint32_t* base;      // first bucket
  uint32_t* sum;       // summary of the first bucket
  uint32_t nb;         // buckets (0 = none)
  uint32_t words;
};

__host__ __device__ inline uint32_t hmix(uint32_t x) {
  // 32-bit integer finaliser ("lowbias32", C. Wellons' hash-prospector)
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__host__ __device__ inline uint64_t make_desc(uint64_t off, uint32_t lognb) { return (off << 6) | lognb; }

__device__ inline Slab slab_of(const Pool& p, uint64_t desc) {
  Slab s;
  s.words = p.words;
  if (desc == 0) {
    s.base = p.base;
    s.sum = p.sum;
    s.nb = 0;
  } else {
    s.base = p.base + (desc >> 6) * p.words;
    s.sum = p.sum + (desc >> 6) * SUM_WORDS;
    s.nb = 1u << (desc & 63);
  }
  return s;
}

__device__ inline Slab slab_at(const Pool& p, uint64_t off, uint32_t nb) {
  return Slab{p.base + off * p.words, p.sum + off * SUM_WORDS, nb, p.words};
}

__device__ inline uint32_t* bucket_ptr(const Slab& s, uint32_t b) { return s.base + (uint64_t)b * s.words; }
// dst / src word of slot j of bucket bp
__device__ inline uint32_t* slot_dst(uint32_t* bp, int j) { return bp + j; }
__device__ inline uint32_t* slot_w(uint32_t* bp, int j) { return bp + 16 + j; }
__device__ inline uint64_t* slot_stamp(uint32_t* bp, int j, uint32_t words) {
  return reinterpret_cast<uint64_t*>(bp + (words - 32)) + j;
}
__device__ inline uint32_t* slot_death(uint32_t* bp, int j, uint32_t words) {
  return bp + (words - 32) + 2 * j + 1;
}

__device__ inline bool visible(uint64_t stamp, uint32_t e) {
  uint32_t birth = (uint32_t)stamp, death = (uint32_t)(stamp >> 32);
  return birth <= e && e < death;
}

// Word loads that bypass nothing but are not cached in registers across
// other threads' writes (slabs are written concurrently in update kernels).
template <class T>
__device__ inline T ld_relaxed(const T* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// A value every lane of the wave holds equally, made visibly uniform for the
// compiler (it then lives in scalar registers, and loops and branches on it
// are uniform).
__device__ inline uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ inline int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline unsigned long long uni(unsigned long long x) {
  return (unsigned long long)uni((uint32_t)x) | ((unsigned long long)uni((uint32_t)(x >> 32)) << 32);
}
template <class T>
__device__ inline T* uni(T* p) {
  return reinterpret_cast<T*>(uni(reinterpret_cast<unsigned long long>(p)));
}
template <class T>
__device__ inline void st_relaxed(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Find the current version (death == INF) of key `x` in slab s; returns the
// slot pointer (bucket base, slot index) or nullptr.
struct SlotRef {
  uint32_t* bp;
  int j;
  uint32_t b;
};

// The 16 destination words of a bucket, read as one line (four 16-byte
// loads issued together).  Slots are claimed in order and never released
// while a slab is live, so the used slots always form a prefix of the
// bucket; a copy read while other threads claim slots can only show EMPTY
// for a slot claimed since, never a destination for an empty slot.
__device__ inline void load_dsts(const uint32_t* bp, uint32_t d[BSLOTS]) {
  const uint4* p = reinterpret_cast<const uint4*>(bp);
#pragma unroll
  for (int q = 0; q < BSLOTS / 4; q++) {
    const uint4 v = p[q];
    d[4 * q] = v.x;
    d[4 * q + 1] = v.y;
    d[4 * q + 2] = v.z;
    d[4 * q + 3] = v.w;
  }
}

// First EMPTY slot of a bucket copy (BSLOTS: none).
__device__ inline int first_empty(const uint32_t d[BSLOTS]) {
  int j0 = BSLOTS;
#pragma unroll
  for (int j = BSLOTS - 1; j >= 0; j--)
    if (d[j] == EMPTY) j0 = j;
  return j0;
}

// Every version of x already stored lies inside the prefix, so a copy that
// misses slots claimed since it was read loses none of them; the death of
// a matching slot is read fresh.
__device__ inline SlotRef find_current(const Slab& s, uint32_t x) {
  SlotRef r{nullptr, -1, 0};
  if (s.nb == 0) return r;
  uint32_t mask = s.nb - 1;
  uint32_t b = hmix(x) & mask;
  for (uint32_t probe = 0; probe < s.nb; probe++) {
    uint32_t* bp = bucket_ptr(s, b);
    uint32_t d[BSLOTS];
    load_dsts(bp, d);
    const int used = first_empty(d);
    for (int j = 0; j < used; j++) {
      if (d[j] == x && ld_relaxed(slot_death(bp, j, s.words)) == INF_EPOCH) {
        r.bp = bp;
        r.j = j;
        r.b = b;
        return r;
      }
    }
    if (used < BSLOTS) return r;
    b = (b + 1) & mask;
  }
  return r;
}

// Claim a free slot for key x whose version is born at `birth` (capacity
// is guaranteed by the growth step) and raise the bucket's largest-birth
// summary.  Readers that trust the summary never run beside a writer, so
// the two updates need no ordering between them.  Slots before the first
// EMPTY of a bucket copy are taken for good; from there each slot is tried
// with a compare-and-swap, which fails on a slot claimed since the copy.
__device__ inline SlotRef claim_slot(const Slab& s, uint32_t x, uint32_t birth) {
  SlotRef r{nullptr, -1, 0};
  uint32_t mask = s.nb - 1;
  uint32_t b = hmix(x) & mask;
  for (uint32_t probe = 0; probe < s.nb; probe++) {
    uint32_t* bp = bucket_ptr(s, b);
    uint32_t d[BSLOTS];
    load_dsts(bp, d);
    const int j0 = first_empty(d);
    if (j0 < BSLOTS) atomicMax(&s.sum[SUM_WORDS * b], birth);
    for (int j = j0; j < BSLOTS; j++) {
      if (atomicCAS(slot_dst(bp, j), EMPTY, x) == EMPTY) {
        r.bp = bp;
        r.j = j;
        r.b = b;
        return r;
      }
    }
    b = (b + 1) & mask;
  }
  return r;
}

// Record in the bucket summary that slot j now carries the finite death
// `death`.
__device__ inline void mark_tomb(const Slab& s, uint32_t b, int j, uint32_t death) {
  atomicOr(&s.sum[SUM_WORDS * b + 1], 1u << j);
  atomicMax(&s.sum[SUM_WORDS * b + 2], death);
}

// Initialise the summaries of nb fresh buckets (no version, no tombstone).
__device__ inline void clear_summaries(uint32_t* sum, uint32_t nb, uint32_t tid, uint32_t nthreads) {
  for (uint32_t t = tid; t < SUM_WORDS * nb; t += nthreads) sum[t] = 0u;
}

// Whether slot j of bucket b (holding dst d != EMPTY) is visible at e.
// `fast` is set when no writer can run concurrently with the reader: then
// the stamp is read only for a tombstoned slot or when the bucket holds a
// version born after e.
__device__ inline bool slot_visible(const Slab& s, uint32_t* bp, uint32_t b, int j, uint32_t e, bool fast) {
  if (fast) {
    const uint4 sm = *reinterpret_cast<const uint4*>(&s.sum[SUM_WORDS * b]);
    if (sm.x <= e) {
      if (!((sm.y >> j) & 1u)) return true;   // live, born at or before e
      if (sm.z <= e) return false;            // tombstoned at or before e
    }
  }
  return visible(*slot_stamp(bp, j, s.words), e);
}

// The same decision from a summary already loaded (x max birth, y tomb
// mask, z max death); `stamp` is read only when the summary cannot decide.
__device__ inline bool visible_by_summary(uint4 sm, bool fast, int j, uint32_t e, const uint64_t* stamp) {
  if (fast && sm.x <= e) {
    if (!((sm.y >> j) & 1u)) return true;
    if (sm.z <= e) return false;
  }
  return visible(*stamp, e);
}

// ------------------------------------------------------------ wave helpers

__device__ inline uint32_t lane_id() { return threadIdx.x & 63; }

// Exclusive prefix of k over the 64 lanes of the wave plus one atomicAdd on
// counter for the wave total.  Every lane of the wave must call it.
__device__ inline uint32_t wave_reserve(uint32_t* counter, uint32_t k, uint32_t* total_out = nullptr) {
  uint32_t lane = lane_id();
  uint32_t x = k;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  uint32_t total = __shfl(x, 63, 64);
  uint32_t base = 0;
  if (lane == 0 && total) base = atomicAdd(counter, total);
  base = __shfl(base, 0, 64);
  if (total_out) *total_out = total;
  return base + x - k;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// 16-bit mask of the lanes of this lane's 16-lane group for which pred holds.
__device__ inline uint32_t group16_ballot(bool pred) {
  unsigned long long m = __ballot(pred);
  return (uint32_t)((m >> (threadIdx.x & 48)) & 0xFFFFull);
}

}  // namespace dg
