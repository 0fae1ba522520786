// The serving loop's executors: continuous multi-source BFS and SSSP.
//
// BFS: up to XB_SLOTS BFS queries share one level-synchronous multi-source
// search, each bound to its own snapshot epoch.  A query is admitted at any
// pass boundary into a free slot: its source joins the next frontier, and
// its levels count from the pass it joined, so its hop distances are those
// of a search of its own.  An arc is followed for the slots whose epoch
// lies in the arc's lifetime [birth, death), so each query sees exactly its
// snapshot.  A slot whose search added no vertex in a pass is complete and
// its output is final.
//
// SSSP: up to XS_SLOTS SSSP queries share one label-correcting search (a
// frontier of vertices whose distance improved in the last pass, for a mask
// of slots; Bellman-Ford order, one bucket of unbounded width).  A query
// joins at any pass boundary with its source at distance 0; a slot whose
// distances did not change in a pass has converged to the exact
// shortest-path distances.  Relaxations are integer atomicMin, so the
// result does not depend on the order of work or on the other slots.
#pragma once

#include <string>

#include "dg_host.h"

namespace dg {

constexpr uint32_t XB_SLOTS = 64;
constexpr uint32_t XS_SLOTS = 32;

// The active slots' epochs: distinct values ascending (padded with
// 0xFFFFFFFF) and cm[i] = the slots bound to one of the i smallest, so the
// slots with epoch below x are cm[#{ue < x}].
struct XbEpochs {
  uint32_t ne;
  uint32_t ue[XB_SLOTS];
  unsigned long long cm[XB_SLOTS + 1];
};

// Per slot: its output (distance array) and the pass its source joined.
struct XbOuts {
  int32_t* out[XB_SLOTS];
  int32_t start[XB_SLOTS];
};

struct XbSeeds {
  uint32_t n;
  uint32_t slot[XB_SLOTS];
  uint32_t src[XB_SLOTS];
};

struct XbResult {
  unsigned long long progress;   // slots that reached a new vertex in the pass
  unsigned long long arcs;       // arcs followed for at least one slot
  uint32_t n_touched;
  uint32_t overflow;
  unsigned long long fq;         // the next frontier (items | buckets)
};

// p[0 .. n) = v on stream s.
hipError_t fill_i32(int32_t* p, uint64_t n, int32_t v, hipStream_t s);

struct XbState;
XbState* xb_create();
void xb_destroy(XbState* x);
// One pass on stream s: clears the visited bits of the slots in
// clear_mask, expands the frontier for the slots in `ep`, joins the seeds,
// finalises the pass's new vertices (level = pass - start of their slot)
// and waits for its counters.  grid_pct bounds the expansion's workgroups
// as a share of those resident.
hipError_t xb_pass(XbState* x, dg_graph* g, const Store& st, hipStream_t s, uint32_t grid_pct, int32_t pass,
                   const XbEpochs& ep, const XbOuts& outs, const XbSeeds& seeds, unsigned long long clear_mask,
                   XbResult* r);

struct XsState;
XsState* xs_create();
void xs_destroy(XsState* x);
// One SSSP pass on stream s: resets the distances of the slots in
// clear_mask, relaxes the frontier for the slots in `ep` (slots below
// XS_SLOTS), joins the seeds and waits for its counters; r->progress holds
// the slots whose distances changed.
hipError_t xs_pass(XsState* x, dg_graph* g, const Store& st, hipStream_t s, uint32_t grid_pct, const XbEpochs& ep,
                   const XbSeeds& seeds, unsigned long long clear_mask, XbResult* r);
// Writes the distances of the slots in mask into outs.out[slot] (-1 where
// unreached) on stream s, then records `done` on s unless it is null.
hipError_t xs_extract(XsState* x, const XbOuts& outs, unsigned long long mask, hipStream_t s, hipEvent_t done);

}  // namespace dg
