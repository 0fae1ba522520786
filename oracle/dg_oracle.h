/*
 * dg_oracle.h -- sequential CPU oracle for the snapshot-query dynamic graph.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no source with the HIP path.
 *
 * What it computes (plain definitions, one operation at a time):
 *   - the graph ADT operations named in the paper's preamble
 *     (PutV / RemoveV / GetV / PutE / RemoveE / GetE), applied in index
 *     order -- the linearization order of a batch;
 *   - BFS hop distances (FIFO queue), SSSP distances (binary-heap Dijkstra)
 *     and Brandes betweenness (int64 path counts, FP64 dependencies), the
 *     queries named BFS / SSSP / BC in the same preamble, on the current
 *     state;
 *   - PageRank of the current state, Eq. (1) iterated as the synchronous
 *     Barrier baseline (Alg. 1) in FP64, optionally with the loop
 *     perforation of Alg. 5;
 *   - strongly connected components (GetSCC in the preamble), by Tarjan;
 *   - the diameter (GD in the preamble), by a BFS from every vertex;
 *   - the maximum s-t flow (GetNF in the preamble), by Edmonds-Karp.
 *
 * Error codes are the integer values of the C boundary's call status.
 */
#ifndef DG_ORACLE_H
#define DG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { uint32_t type, u, v; int32_t w; } orc_op;   /* 16 bytes */

enum { ORC_ADDV = 0, ORC_REMV = 1, ORC_HASV = 2, ORC_ADDE = 3, ORC_REME = 4, ORC_HASE = 5 };
enum {
  ORC_OK = 0, ORC_E_INVALID_ARG = -1, ORC_E_OOM = -2, ORC_E_VERTEX_RANGE = -3,
  ORC_E_WEIGHT_RANGE = -4, ORC_E_SOURCE_ABSENT = -6, ORC_E_OVERFLOW = -7
};

typedef struct orc_graph orc_graph;

orc_graph* orc_create(uint32_t n_vertices, int undirected, int32_t w_max);
void       orc_destroy(orc_graph* g);
uint32_t   orc_epoch(const orc_graph* g);
/* Apply ops[0..n) in order; results[i] = 0 false / 1 true / 2 endpoint absent.
 * The whole batch is validated first; on error nothing changes. */
int        orc_apply(orc_graph* g, const orc_op* ops, uint64_t n, uint8_t* results);
int        orc_bfs(const orc_graph* g, uint32_t s, int32_t* dist);
int        orc_sssp(const orc_graph* g, uint32_t s, int32_t* dist);
int        orc_bc(const orc_graph* g, const uint32_t* S, uint32_t k, double* bc);
void       orc_counts(const orc_graph* g, uint64_t* n_live_vertices, uint64_t* n_arcs);
int        orc_alive(const orc_graph* g, uint32_t v);
/* 1 and *w set if edge key (u, v) is present, else 0. */
int        orc_edge(const orc_graph* g, uint32_t u, uint32_t v, int32_t* w);
/* Writes every stored edge key (undirected: lo < = hi); returns count.
 * Arrays must hold orc_counts' key count (n_arcs, or keys in undirected). */
uint64_t   orc_n_keys(const orc_graph* g);
uint64_t   orc_export(const orc_graph* g, uint32_t* u, uint32_t* v, int32_t* w);
/* Out-degree (visible arcs) of v. */
uint32_t   orc_out_degree(const orc_graph* g, uint32_t v);
/* PageRank (Eq. (1), Alg. 1): pr[v] for every id (0 for vertices that are not
 * live), the iterations run and the last iteration's largest change.  Stops
 * once that change is at most `threshold`, or after max_iters iterations.
 * ORC_E_INVALID_ARG for a damping factor outside [0, 1) or a negative
 * threshold. */
int        orc_pagerank(const orc_graph* g, double damping, double threshold, uint32_t max_iters, double* pr,
                        uint32_t* iters, double* last_change);
/* The same with loop perforation (Alg. 5): a live vertex whose change in an
 * iteration is nonzero and below freeze_below keeps its value and is not
 * recomputed afterwards.  freeze_below = 0 is orc_pagerank. */
/* Strongly connected components (Tarjan): comp[v] = smallest id in v's
 * component for live v, -1 otherwise. */
int        orc_scc(const orc_graph* g, int32_t* comp);
/* Diameter: largest hop distance over ordered pairs (u, v) of live vertices
 * with v reachable from u (0 without arcs); one BFS per live vertex. */
int        orc_diameter(const orc_graph* g, uint32_t* diameter);
/* Maximum s-t flow with arc weights as capacities (Edmonds-Karp). */
int        orc_maxflow(const orc_graph* g, uint32_t s, uint32_t t, int64_t* flow);
/* DFS collect: depth-first search from s taking out-neighbours in ascending
 * id order; disc[v] = preorder position, parent[v] = discovering vertex (-1
 * where not reached, and for s). */
int        orc_dfs(const orc_graph* g, uint32_t s, int32_t* disc, int32_t* parent);
int        orc_pagerank_perforated(const orc_graph* g, double damping, double threshold, double freeze_below,
                                   uint32_t max_iters, double* pr, uint32_t* iters, double* last_change);

#ifdef __cplusplus
}
#endif
#endif
