// Serving loop (continuous batching over the graph).
#include "dg_host.h"

extern "C" {
dg_status dg_server_start(dg_graph* g, const dg_server_config*, dg_server** out) {
  if (out) *out = nullptr;
  if (g) g->err = "serving loop is not built yet";
  return DG_E_UNIMPLEMENTED;
}
dg_status dg_server_stop(dg_server*) { return DG_E_UNIMPLEMENTED; }
dg_status dg_server_submit_update(dg_server*, const dg_op*, uint64_t, uint64_t*) { return DG_E_UNIMPLEMENTED; }
dg_status dg_server_submit_query(dg_server*, uint32_t, const uint32_t*, uint32_t, uint64_t*) { return DG_E_UNIMPLEMENTED; }
dg_status dg_server_poll(dg_server*, uint64_t, int*, dg_status*, dg_epoch*, double*) { return DG_E_UNIMPLEMENTED; }
dg_status dg_server_take(dg_server*, uint64_t, void*, uint64_t) { return DG_E_UNIMPLEMENTED; }
dg_status dg_server_drain(dg_server*) { return DG_E_UNIMPLEMENTED; }
dg_status dg_server_get_stats(dg_server*, dg_server_stats*) { return DG_E_UNIMPLEMENTED; }
}
