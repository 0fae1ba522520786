// Persistent multi-query executor (filled in below the plain path).
#include "dg_host.h"

namespace dg {
dg_status query_batch_dev(dg_graph* g, const dg_query*, uint32_t, dg_status*, hipStream_t) {
  g->err = "query batches are not built yet";
  return DG_E_UNIMPLEMENTED;
}
void free_batch_state(dg_graph*) {}
}  // namespace dg

extern "C" dg_status dg_query_batch(dg_graph* g, const dg_query* q, uint32_t nq, dg_status* per_query, void* stream) {
  if (!g) return DG_E_INVALID_ARG;
  return dg::query_batch_dev(g, q, nq, per_query, static_cast<hipStream_t>(stream));
}

extern "C" dg_status dg_autotune(dg_graph* g, uint32_t, dg_tuning*, void*) {
  if (!g) return DG_E_INVALID_ARG;
  g->err = "autotuner is not built yet";
  return DG_E_UNIMPLEMENTED;
}
