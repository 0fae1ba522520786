/*
 * dg_oracle.c -- sequential CPU oracle for the snapshot-query dynamic graph.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the package smoke check and
 * the benchmark's CPU-baseline leg.  The product path never loads it.
 *
 * The paper names the graph ADT (PutV, RemoveV, GetV, PutE, RemoveE, GetE),
 * linearizability of the shared graph object, and the snapshot queries BFS,
 * SSSP and BC only by name (preamble macro definitions); it gives no worked
 * example.  This file therefore writes out the textbook definitions:
 *
 *   ADT (one op at a time, in index order = linearization order):
 *     AddVertex(v)     alive -> 0; else make v alive and isolated -> 1
 *     RemoveVertex(v)  dead  -> 0; else delete every arc (v,*) and (*,v),
 *                      mark v dead -> 1
 *     ContainsVertex   alive(v)
 *     AddEdge(u,v,w)   u or v dead -> 2; key present -> 0 (weight kept);
 *                      else insert with weight w -> 1
 *     RemoveEdge(u,v)  u or v dead -> 2; present -> delete, 1; else 0
 *     ContainsEdge     u or v dead -> 2; present -> 1; else 0
 *   In undirected mode the key of (u,v) is {min,max} and both arcs exist.
 *
 *   BFS(s): minimum number of arcs on a path s -> v; -1 if none.
 *           FIFO queue (Moore 1959).
 *   SSSP(s): minimum total weight of a path s -> v (weights >= 1);
 *           -1 if none.  Dijkstra (1959) with a binary heap.
 *   BC(S):  Brandes (2001): per source, BFS with shortest-path counts
 *           sigma (int64, checked), then dependencies
 *           delta[v] = sum over arcs (v,w) with d[w] = d[v]+1 of
 *                      sigma[v]/sigma[w] * (1 + delta[w])
 *           in non-increasing distance order; bc[v] += delta[v] for v != s,
 *           sources taken in the caller's order.  Unweighted, no
 *           normalisation, no halving in undirected mode.
 *
 * Representation: a hash map from edge key to (weight, list positions) and
 * per-vertex out-lists (and in-lists in directed mode) with swap-removal.
 */
#include "dg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KEY_EMPTY UINT64_MAX
#define KEY_TOMB (UINT64_MAX - 1)

typedef struct { uint32_t v; int32_t w; } arc;
typedef struct { arc* a; uint32_t n, cap; } arc_list;
typedef struct { uint32_t* a; uint32_t n, cap; } id_list;
/* pa: position of the arc lo->hi in out[lo]; pb: position of lo in in[hi]
 * (directed) or of the arc hi->lo in out[hi] (undirected, lo != hi). */
typedef struct { uint64_t key; int32_t w; uint32_t pa, pb; } mslot;

struct orc_graph {
  uint32_t n;
  int undirected;
  int32_t w_max;
  uint32_t epoch;
  uint8_t* alive;
  arc_list* out;
  id_list* in;
  mslot* tab;
  uint64_t cap, used, tombs, keys;
};

/* ---------------------------------------------------------------- lists */

static int arc_push(arc_list* l, uint32_t v, int32_t w) {
  if (l->n == l->cap) {
    uint32_t nc = l->cap ? 2 * l->cap : 4;
    arc* na = (arc*)realloc(l->a, (size_t)nc * sizeof(arc));
    if (!na) return -1;
    l->a = na;
    l->cap = nc;
  }
  l->a[l->n].v = v;
  l->a[l->n].w = w;
  return (int)(l->n++);
}

static int id_push(id_list* l, uint32_t x) {
  if (l->n == l->cap) {
    uint32_t nc = l->cap ? 2 * l->cap : 4;
    uint32_t* na = (uint32_t*)realloc(l->a, (size_t)nc * sizeof(uint32_t));
    if (!na) return -1;
    l->a = na;
    l->cap = nc;
  }
  l->a[l->n] = x;
  return (int)(l->n++);
}

/* ------------------------------------------------------------------ map */

static uint64_t mix64(uint64_t x) {   /* splitmix64 finaliser */
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ULL;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebULL;
  x ^= x >> 31;
  return x;
}

static uint64_t key_of(const orc_graph* g, uint32_t u, uint32_t v) {
  if (g->undirected && u > v) { uint32_t t = u; u = v; v = t; }
  return ((uint64_t)u << 32) | v;
}

static int64_t map_find(const orc_graph* g, uint64_t key) {
  uint64_t mask = g->cap - 1, i = mix64(key) & mask;
  for (;;) {
    uint64_t k = g->tab[i].key;
    if (k == key) return (int64_t)i;
    if (k == KEY_EMPTY) return -1;
    i = (i + 1) & mask;
  }
}

static int map_rehash(orc_graph* g, uint64_t ncap) {
  mslot* old = g->tab;
  uint64_t ocap = g->cap;
  mslot* t = (mslot*)malloc((size_t)ncap * sizeof(mslot));
  if (!t) return -1;
  for (uint64_t i = 0; i < ncap; i++) t[i].key = KEY_EMPTY;
  g->tab = t;
  g->cap = ncap;
  g->used = 0;
  g->tombs = 0;
  for (uint64_t i = 0; i < ocap; i++) {
    uint64_t k = old[i].key;
    if (k == KEY_EMPTY || k == KEY_TOMB) continue;
    uint64_t j = mix64(k) & (ncap - 1);
    while (t[j].key != KEY_EMPTY) j = (j + 1) & (ncap - 1);
    t[j] = old[i];
    g->used++;
  }
  free(old);
  return 0;
}

/* Returns the slot index for a key known to be absent. */
static int64_t map_insert(orc_graph* g, uint64_t key) {
  if ((g->used + g->tombs + 1) * 10 > g->cap * 7) {
    uint64_t ncap = g->cap;
    while ((g->used + 1) * 10 > ncap * 4) ncap *= 2;
    if (map_rehash(g, ncap)) return -1;
  }
  uint64_t mask = g->cap - 1, i = mix64(key) & mask;
  while (g->tab[i].key != KEY_EMPTY && g->tab[i].key != KEY_TOMB) i = (i + 1) & mask;
  if (g->tab[i].key == KEY_TOMB) g->tombs--;
  g->tab[i].key = key;
  g->used++;
  return (int64_t)i;
}

/* ---------------------------------------------------------------- edges */

static int add_edge(orc_graph* g, uint32_t u, uint32_t v, int32_t w) {
  uint64_t key = key_of(g, u, v);
  uint32_t lo = (uint32_t)(key >> 32), hi = (uint32_t)key;
  int64_t s = map_insert(g, key);
  if (s < 0) return -1;
  g->tab[s].w = w;
  int pa = arc_push(&g->out[lo], hi, w);
  int pb = 0;
  if (!g->undirected) pb = id_push(&g->in[hi], lo);
  else if (lo != hi) pb = arc_push(&g->out[hi], lo, w);
  if (pa < 0 || pb < 0) return -1;
  g->tab[s].pa = (uint32_t)pa;
  g->tab[s].pb = (uint32_t)pb;
  g->keys++;
  return 0;
}

/* Record that the arc x -> y now sits at position p of out[x]. */
static void set_out_pos(orc_graph* g, uint32_t x, uint32_t y, uint32_t p) {
  uint64_t key = key_of(g, x, y);
  mslot* m = &g->tab[map_find(g, key)];
  if ((uint32_t)(key >> 32) == x) m->pa = p; else m->pb = p;
}

static void out_remove_at(orc_graph* g, uint32_t x, uint32_t p) {
  arc_list* l = &g->out[x];
  uint32_t last = l->n - 1;
  if (p != last) {
    l->a[p] = l->a[last];
    set_out_pos(g, x, l->a[p].v, p);
  }
  l->n--;
}

static void in_remove_at(orc_graph* g, uint32_t x, uint32_t p) {
  id_list* l = &g->in[x];
  uint32_t last = l->n - 1;
  if (p != last) {
    l->a[p] = l->a[last];
    g->tab[map_find(g, key_of(g, l->a[p], x))].pb = p;
  }
  l->n--;
}

static void remove_edge_slot(orc_graph* g, int64_t s) {
  uint64_t key = g->tab[s].key;
  uint32_t lo = (uint32_t)(key >> 32), hi = (uint32_t)key;
  uint32_t pa = g->tab[s].pa, pb = g->tab[s].pb;
  out_remove_at(g, lo, pa);
  if (!g->undirected) in_remove_at(g, hi, pb);
  else if (lo != hi) out_remove_at(g, hi, pb);
  /* the swap-removals above looked this slot up by key; erase it last */
  g->tab[s].key = KEY_TOMB;
  g->used--;
  g->tombs++;
  g->keys--;
}

static void remove_vertex_edges(orc_graph* g, uint32_t x) {
  while (g->out[x].n) {
    uint32_t y = g->out[x].a[g->out[x].n - 1].v;
    remove_edge_slot(g, map_find(g, key_of(g, x, y)));
  }
  if (!g->undirected) {
    while (g->in[x].n) {
      uint32_t y = g->in[x].a[g->in[x].n - 1];
      remove_edge_slot(g, map_find(g, key_of(g, y, x)));
    }
  }
}

/* ------------------------------------------------------------- lifetime */

orc_graph* orc_create(uint32_t n, int undirected, int32_t w_max) {
  if (n == 0 || n > 0x80000000u || w_max < 1) return NULL;
  /* SSSP distances are int32: the longest simple path must fit */
  if ((int64_t)(n - 1) * (int64_t)w_max > 0x7fffffffLL) return NULL;
  orc_graph* g = (orc_graph*)calloc(1, sizeof(orc_graph));
  if (!g) return NULL;
  g->n = n;
  g->undirected = undirected ? 1 : 0;
  g->w_max = w_max;
  g->alive = (uint8_t*)calloc(n, 1);
  g->out = (arc_list*)calloc(n, sizeof(arc_list));
  g->in = undirected ? NULL : (id_list*)calloc(n, sizeof(id_list));
  g->cap = 1024;
  g->tab = (mslot*)malloc(g->cap * sizeof(mslot));
  if (!g->alive || !g->out || (!undirected && !g->in) || !g->tab) {
    orc_destroy(g);
    return NULL;
  }
  for (uint64_t i = 0; i < g->cap; i++) g->tab[i].key = KEY_EMPTY;
  return g;
}

void orc_destroy(orc_graph* g) {
  if (!g) return;
  if (g->out)
    for (uint32_t i = 0; i < g->n; i++) free(g->out[i].a);
  if (g->in)
    for (uint32_t i = 0; i < g->n; i++) free(g->in[i].a);
  free(g->out);
  free(g->in);
  free(g->alive);
  free(g->tab);
  free(g);
}

uint32_t orc_epoch(const orc_graph* g) { return g->epoch; }

int orc_alive(const orc_graph* g, uint32_t v) { return v < g->n && g->alive[v]; }

/* ------------------------------------------------------------------ ADT */

int orc_apply(orc_graph* g, const orc_op* ops, uint64_t n, uint8_t* res) {
  /* whole-batch validation before any op takes effect */
  for (uint64_t i = 0; i < n; i++) {
    if (ops[i].type > ORC_HASE) return ORC_E_INVALID_ARG;
  }
  for (uint64_t i = 0; i < n; i++) {
    if (ops[i].u >= g->n) return ORC_E_VERTEX_RANGE;
    if (ops[i].type >= ORC_ADDE && ops[i].v >= g->n) return ORC_E_VERTEX_RANGE;
  }
  for (uint64_t i = 0; i < n; i++) {
    if (ops[i].type == ORC_ADDE && (ops[i].w < 1 || ops[i].w > g->w_max)) return ORC_E_WEIGHT_RANGE;
  }
  for (uint64_t i = 0; i < n; i++) {
    uint32_t t = ops[i].type, u = ops[i].u, v = ops[i].v;
    uint8_t r = 0;
    switch (t) {
      case ORC_ADDV:
        if (!g->alive[u]) { g->alive[u] = 1; r = 1; }
        break;
      case ORC_REMV:
        if (g->alive[u]) { remove_vertex_edges(g, u); g->alive[u] = 0; r = 1; }
        break;
      case ORC_HASV:
        r = g->alive[u];
        break;
      default: {
        if (!g->alive[u] || !g->alive[v]) { r = 2; break; }
        int64_t s = map_find(g, key_of(g, u, v));
        if (t == ORC_ADDE) {
          if (s >= 0) r = 0;
          else { if (add_edge(g, u, v, ops[i].w)) return ORC_E_OOM; r = 1; }
        } else if (t == ORC_REME) {
          if (s >= 0) { remove_edge_slot(g, s); r = 1; }
        } else {
          r = s >= 0;
        }
      }
    }
    if (res) res[i] = r;
  }
  if (n) g->epoch++;
  return ORC_OK;
}

void orc_counts(const orc_graph* g, uint64_t* nv, uint64_t* narcs) {
  uint64_t a = 0, c = 0;
  for (uint32_t i = 0; i < g->n; i++) { c += g->alive[i]; a += g->out[i].n; }
  if (nv) *nv = c;
  if (narcs) *narcs = a;
}

uint64_t orc_n_keys(const orc_graph* g) { return g->keys; }

int orc_edge(const orc_graph* g, uint32_t u, uint32_t v, int32_t* w) {
  if (u >= g->n || v >= g->n) return 0;
  int64_t s = map_find(g, key_of(g, u, v));
  if (s < 0) return 0;
  if (w) *w = g->tab[s].w;
  return 1;
}

uint64_t orc_export(const orc_graph* g, uint32_t* u, uint32_t* v, int32_t* w) {
  uint64_t k = 0;
  for (uint64_t i = 0; i < g->cap; i++) {
    uint64_t key = g->tab[i].key;
    if (key == KEY_EMPTY || key == KEY_TOMB) continue;
    u[k] = (uint32_t)(key >> 32);
    v[k] = (uint32_t)key;
    w[k] = g->tab[i].w;
    k++;
  }
  return k;
}

uint32_t orc_out_degree(const orc_graph* g, uint32_t v) { return v < g->n ? g->out[v].n : 0; }

/* -------------------------------------------------------------- queries */

static int check_source(const orc_graph* g, uint32_t s) {
  if (s >= g->n) return ORC_E_VERTEX_RANGE;
  if (!g->alive[s]) return ORC_E_SOURCE_ABSENT;
  return ORC_OK;
}

int orc_bfs(const orc_graph* g, uint32_t s, int32_t* dist) {
  int rc = check_source(g, s);
  if (rc) return rc;
  uint32_t* q = (uint32_t*)malloc((size_t)g->n * sizeof(uint32_t));
  if (!q) return ORC_E_OOM;
  for (uint32_t i = 0; i < g->n; i++) dist[i] = -1;
  uint32_t head = 0, tail = 0;
  dist[s] = 0;
  q[tail++] = s;
  while (head < tail) {
    uint32_t x = q[head++];
    const arc_list* l = &g->out[x];
    for (uint32_t j = 0; j < l->n; j++) {
      uint32_t y = l->a[j].v;
      if (dist[y] < 0) { dist[y] = dist[x] + 1; q[tail++] = y; }
    }
  }
  free(q);
  return ORC_OK;
}

typedef struct { int64_t d; uint32_t v; } hnode;

static void heap_push(hnode* h, uint64_t* n, int64_t d, uint32_t v) {
  uint64_t i = (*n)++;
  while (i > 0) {
    uint64_t p = (i - 1) / 2;
    if (h[p].d <= d) break;
    h[i] = h[p];
    i = p;
  }
  h[i].d = d;
  h[i].v = v;
}

static hnode heap_pop(hnode* h, uint64_t* n) {
  hnode top = h[0], last = h[--(*n)];
  uint64_t i = 0;
  for (;;) {
    uint64_t c = 2 * i + 1;
    if (c >= *n) break;
    if (c + 1 < *n && h[c + 1].d < h[c].d) c++;
    if (last.d <= h[c].d) break;
    h[i] = h[c];
    i = c;
  }
  if (*n) h[i] = last;
  return top;
}

int orc_sssp(const orc_graph* g, uint32_t s, int32_t* dist) {
  int rc = check_source(g, s);
  if (rc) return rc;
  uint64_t arcs = 0;
  for (uint32_t i = 0; i < g->n; i++) arcs += g->out[i].n;
  int64_t* d = (int64_t*)malloc((size_t)g->n * sizeof(int64_t));
  uint8_t* done = (uint8_t*)calloc(g->n, 1);
  hnode* h = (hnode*)malloc((size_t)(arcs + 1) * sizeof(hnode));
  if (!d || !done || !h) { free(d); free(done); free(h); return ORC_E_OOM; }
  for (uint32_t i = 0; i < g->n; i++) d[i] = INT64_MAX;
  uint64_t hn = 0;
  d[s] = 0;
  heap_push(h, &hn, 0, s);
  while (hn) {
    hnode t = heap_pop(h, &hn);
    if (done[t.v]) continue;
    done[t.v] = 1;
    const arc_list* l = &g->out[t.v];
    for (uint32_t j = 0; j < l->n; j++) {
      uint32_t y = l->a[j].v;
      int64_t nd = t.d + l->a[j].w;
      if (nd < d[y]) { d[y] = nd; heap_push(h, &hn, nd, y); }
    }
  }
  for (uint32_t i = 0; i < g->n; i++) dist[i] = d[i] == INT64_MAX ? -1 : (int32_t)d[i];
  free(d);
  free(done);
  free(h);
  return ORC_OK;
}

int orc_bc(const orc_graph* g, const uint32_t* S, uint32_t k, double* bc) {
  for (uint32_t i = 0; i < k; i++) {
    int rc = check_source(g, S[i]);
    if (rc) return rc;
    for (uint32_t j = 0; j < i; j++)
      if (S[j] == S[i]) return ORC_E_INVALID_ARG;
  }
  uint32_t n = g->n;
  int32_t* d = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* sigma = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  double* delta = (double*)malloc((size_t)n * sizeof(double));
  uint32_t* order = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  if (!d || !sigma || !delta || !order) {
    free(d); free(sigma); free(delta); free(order);
    return ORC_E_OOM;
  }
  for (uint32_t v = 0; v < n; v++) bc[v] = 0.0;
  int rc = ORC_OK;
  for (uint32_t si = 0; si < k && rc == ORC_OK; si++) {
    uint32_t s = S[si];
    for (uint32_t v = 0; v < n; v++) { d[v] = -1; sigma[v] = 0; delta[v] = 0.0; }
    /* BFS from s; order[] is the visit order (non-decreasing distance) */
    uint32_t head = 0, tail = 0;
    d[s] = 0;
    sigma[s] = 1;
    order[tail++] = s;
    while (head < tail) {
      uint32_t x = order[head++];
      const arc_list* l = &g->out[x];
      for (uint32_t j = 0; j < l->n; j++) {
        uint32_t y = l->a[j].v;
        if (d[y] < 0) { d[y] = d[x] + 1; order[tail++] = y; }
        if (d[y] == d[x] + 1) {
          if (__builtin_add_overflow(sigma[y], sigma[x], &sigma[y])) rc = ORC_E_OVERFLOW;
        }
      }
    }
    if (rc) break;
    /* dependencies in non-increasing distance order */
    for (uint32_t i = tail; i-- > 0;) {
      uint32_t x = order[i];
      const arc_list* l = &g->out[x];
      double acc = 0.0;
      for (uint32_t j = 0; j < l->n; j++) {
        uint32_t y = l->a[j].v;
        if (d[y] == d[x] + 1) acc += (double)sigma[x] / (double)sigma[y] * (1.0 + delta[y]);
      }
      delta[x] = acc;
      if (x != s) bc[x] += acc;
    }
  }
  free(d);
  free(sigma);
  free(delta);
  free(order);
  return rc;
}

/* ------------------------------------------------------------- PageRank */

/* Eq. (1): pr(u) = (1 - d)/n + d * sum over arcs (v, u) of pr(v)/q(v), with
 * n the live vertices and q(v) the out-degree of v.  Iterated as the
 * synchronous Barrier baseline (Alg. 1): every live vertex starts from 1/n in
 * the previous-iteration array; an iteration recomputes each live vertex from
 * the previous values alone, starting at (1 - d)/n and adding
 * prev(v)/q(v) * d per in-arc in turn, and records the largest
 * |prev(u) - pr(u)|; the loop continues while that change exceeds the
 * threshold.  The change is measured afresh in every iteration.  A vertex
 * with no out-arcs passes nothing on (Eq. (1) has no term for it).  In-arcs
 * of u are in[u] for a directed graph and out[u] for an undirected one,
 * whose arcs are stored in both directions. */
int orc_pagerank(const orc_graph* g, double damping, double threshold, uint32_t max_iters, double* pr,
                 uint32_t* iters, double* last_change) {
  return orc_pagerank_perforated(g, damping, threshold, 0.0, max_iters, pr, iters, last_change);
}

/* Loop perforation (Alg. 5): a vertex whose change in an iteration is
 * nonzero and below freeze_below is not recomputed in later iterations and
 * keeps its value (its change counts as 0).  freeze_below = 0 freezes
 * nothing, which is the plain iteration above. */
int orc_pagerank_perforated(const orc_graph* g, double damping, double threshold, double freeze_below,
                            uint32_t max_iters, double* pr, uint32_t* iters, double* last_change) {
  if (!(damping >= 0.0 && damping < 1.0) || !(threshold >= 0.0) || !(freeze_below >= 0.0)) return ORC_E_INVALID_ARG;
  const uint32_t n = g->n;
  uint64_t live = 0;
  for (uint32_t u = 0; u < n; u++) live += g->alive[u] ? 1 : 0;
  for (uint32_t u = 0; u < n; u++) pr[u] = 0.0;
  *iters = 0;
  *last_change = 0.0;
  if (live == 0) return ORC_OK;
  double* prev = (double*)malloc((size_t)n * sizeof(double));
  uint8_t* frozen = (uint8_t*)calloc(n ? n : 1, 1);
  if (!prev || !frozen) {
    free(prev);
    free(frozen);
    return ORC_E_OOM;
  }
  for (uint32_t u = 0; u < n; u++) prev[u] = g->alive[u] ? 1.0 / (double)live : 0.0;
  const double base = (1.0 - damping) / (double)live;
  double err = 1.0;
  uint32_t it = 0;
  while (err > threshold && it < max_iters) {
    err = 0.0;
    for (uint32_t u = 0; u < n; u++) {
      if (!g->alive[u]) continue;
      if (frozen[u]) {
        pr[u] = prev[u];
        continue;
      }
      double x = base;
      if (g->undirected) {
        const arc_list* l = &g->out[u];
        for (uint32_t j = 0; j < l->n; j++) {
          const uint32_t v = l->a[j].v;
          x = x + prev[v] / (double)g->out[v].n * damping;
        }
      } else {
        const id_list* l = &g->in[u];
        for (uint32_t j = 0; j < l->n; j++) {
          const uint32_t v = l->a[j];
          x = x + prev[v] / (double)g->out[v].n * damping;
        }
      }
      pr[u] = x;
      const double c = fabs(prev[u] - x);
      if (c > err) err = c;
      if (c != 0.0 && c < freeze_below) frozen[u] = 1;
    }
    for (uint32_t u = 0; u < n; u++) prev[u] = pr[u];
    it++;
  }
  free(prev);
  free(frozen);
  *iters = it;
  *last_change = err;
  return ORC_OK;
}

/* ------------------------------------------------------------------ SCC */

/* Strongly connected components of the current state (the GetSCC query
 * named in the preamble; textbook semantics): comp[v] = the smallest id in
 * v's component for live v, -1 for others.  Tarjan's algorithm (1972) with
 * an explicit stack; components are found in reverse topological order and
 * relabelled by their smallest member.  An undirected graph's components
 * are its connected components. */
int orc_scc(const orc_graph* g, int32_t* comp) {
  const uint32_t n = g->n;
  int64_t* index = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* low = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  uint8_t* on = (uint8_t*)calloc(n ? n : 1, 1);
  uint32_t* st = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
  uint32_t* cs_v = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
  uint32_t* cs_j = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
  if (!index || !low || !on || !st || !cs_v || !cs_j) {
    free(index); free(low); free(on); free(st); free(cs_v); free(cs_j);
    return ORC_E_OOM;
  }
  for (uint32_t v = 0; v < n; v++) {
    index[v] = -1;
    comp[v] = -1;
  }
  int64_t next = 0;
  uint32_t sp = 0;
  for (uint32_t r = 0; r < n; r++) {
    if (!g->alive[r] || index[r] >= 0) continue;
    uint32_t cp = 0;   /* call stack of (vertex, next arc) */
    cs_v[cp] = r;
    cs_j[cp] = 0;
    cp++;
    index[r] = low[r] = next++;
    st[sp++] = r;
    on[r] = 1;
    while (cp) {
      const uint32_t v = cs_v[cp - 1];
      const arc_list* l = &g->out[v];
      if (cs_j[cp - 1] < l->n) {
        const uint32_t w = l->a[cs_j[cp - 1]++].v;
        if (index[w] < 0) {
          index[w] = low[w] = next++;
          st[sp++] = w;
          on[w] = 1;
          cs_v[cp] = w;
          cs_j[cp] = 0;
          cp++;
        } else if (on[w] && index[w] < low[v]) {
          low[v] = index[w];
        }
        continue;
      }
      /* v is done: close its component if it is a root, then return */
      if (low[v] == index[v]) {
        uint32_t k = sp, m = v;
        do {
          k--;
          if (st[k] < m) m = st[k];
        } while (st[k] != v);
        for (uint32_t i = k; i < sp; i++) {
          on[st[i]] = 0;
          comp[st[i]] = (int32_t)m;
        }
        sp = k;
      }
      cp--;
      if (cp) {
        const uint32_t u = cs_v[cp - 1];
        if (low[v] < low[u]) low[u] = low[v];
      }
    }
  }
  free(index); free(low); free(on); free(st); free(cs_v); free(cs_j);
  return ORC_OK;
}

/* ------------------------------------------------------------- diameter */

/* Diameter of the current state (the GD query named in the preamble;
 * textbook semantics): the largest hop distance d(u, v) over ordered pairs
 * of live vertices with v reachable from u, 0 when no arc exists.  One FIFO
 * BFS from every live vertex. */
int orc_diameter(const orc_graph* g, uint32_t* diameter) {
  const uint32_t n = g->n;
  int32_t* dist = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  uint32_t* q = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
  if (!dist || !q) {
    free(dist);
    free(q);
    return ORC_E_OOM;
  }
  uint32_t best = 0;
  for (uint32_t s = 0; s < n; s++) {
    if (!g->alive[s]) continue;
    for (uint32_t i = 0; i < n; i++) dist[i] = -1;
    uint32_t head = 0, tail = 0;
    dist[s] = 0;
    q[tail++] = s;
    while (head < tail) {
      const uint32_t x = q[head++];
      if ((uint32_t)dist[x] > best) best = (uint32_t)dist[x];
      const arc_list* l = &g->out[x];
      for (uint32_t j = 0; j < l->n; j++) {
        const uint32_t y = l->a[j].v;
        if (dist[y] < 0) {
          dist[y] = dist[x] + 1;
          q[tail++] = y;
        }
      }
    }
  }
  free(dist);
  free(q);
  *diameter = best;
  return ORC_OK;
}

/* --------------------------------------------------------- network flow */

/* Maximum flow from s to t of the current state (the GetNF query named in
 * the preamble; textbook semantics): arc weights are capacities (an
 * undirected edge carries its weight each way).  Edmonds-Karp (1972):
 * shortest augmenting paths by BFS over the residual arcs, each arc paired
 * with a reverse of capacity 0, until t is unreachable.  ORC_E_SOURCE_ABSENT
 * when s or t is not live, ORC_E_INVALID_ARG when s == t. */
int orc_maxflow(const orc_graph* g, uint32_t s, uint32_t t, int64_t* flow) {
  if (s >= g->n || t >= g->n) return ORC_E_VERTEX_RANGE;
  if (!g->alive[s] || !g->alive[t]) return ORC_E_SOURCE_ABSENT;
  if (s == t) return ORC_E_INVALID_ARG;
  const uint32_t n = g->n;
  uint64_t m = 0;
  for (uint32_t u = 0; u < n; u++) m += g->out[u].n;
  /* residual arc 2i: arc i forward; 2i + 1: its reverse */
  uint32_t* head = (uint32_t*)malloc((size_t)(2 * m + 1) * sizeof(uint32_t));
  int64_t* cap = (int64_t*)malloc((size_t)(2 * m + 1) * sizeof(int64_t));
  uint64_t* start = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  uint64_t* adj = (uint64_t*)malloc((size_t)(2 * m + 1) * sizeof(uint64_t));
  uint64_t* fill = (uint64_t*)malloc((size_t)(n + 1) * sizeof(uint64_t));
  int64_t* par = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
  uint32_t* q = (uint32_t*)malloc((size_t)(n + 1) * sizeof(uint32_t));
  if (!head || !cap || !start || !adj || !fill || !par || !q) {
    free(head); free(cap); free(start); free(adj); free(fill); free(par); free(q);
    return ORC_E_OOM;
  }
  uint64_t i = 0;
  for (uint32_t u = 0; u < n; u++)
    for (uint32_t j = 0; j < g->out[u].n; j++, i++) {
      const uint32_t v = g->out[u].a[j].v;
      head[2 * i] = v;       /* u -> v */
      cap[2 * i] = g->out[u].a[j].w;
      head[2 * i + 1] = u;   /* v -> u */
      cap[2 * i + 1] = 0;
      start[u + 1]++;
      start[v + 1]++;
    }
  for (uint32_t u = 0; u < n; u++) start[u + 1] += start[u];
  for (uint32_t u = 0; u <= n; u++) fill[u] = start[u];
  i = 0;
  for (uint32_t u = 0; u < n; u++)
    for (uint32_t j = 0; j < g->out[u].n; j++, i++) {
      adj[fill[u]++] = 2 * i;
      adj[fill[head[2 * i]]++] = 2 * i + 1;
    }
  int64_t total = 0;
  for (;;) {
    for (uint32_t u = 0; u < n; u++) par[u] = -1;
    par[s] = -2;
    uint32_t hd = 0, tl = 0;
    q[tl++] = s;
    while (hd < tl && par[t] == -1) {
      const uint32_t x = q[hd++];
      for (uint64_t k = start[x]; k < start[x + 1]; k++) {
        const uint64_t a = adj[k];
        const uint32_t y = head[a];
        if (cap[a] > 0 && par[y] == -1) {
          par[y] = (int64_t)a;
          q[tl++] = y;
        }
      }
    }
    if (par[t] == -1) break;
    int64_t b = INT64_MAX;
    for (uint32_t y = t; y != s; y = head[par[y] ^ 1]) if (cap[par[y]] < b) b = cap[par[y]];
    for (uint32_t y = t; y != s; y = head[par[y] ^ 1]) {
      cap[par[y]] -= b;
      cap[par[y] ^ 1] += b;
    }
    total += b;
  }
  free(head); free(cap); free(start); free(adj); free(fill); free(par); free(q);
  *flow = total;
  return ORC_OK;
}

static int cmp_u32(const void* a, const void* b) {
  const uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/* DFS collect (the GetDFS query named in the preamble; textbook semantics):
 * depth-first search from s over the visible arcs, each vertex taking its
 * out-neighbours in ascending id order (recursive DFS, run here with an
 * explicit stack of vertices and a next-neighbour cursor per vertex).
 * disc[v] = v's position in the discovery order (preorder), parent[v] = the
 * vertex whose arc discovered v; both -1 where v is not reached, and
 * parent[s] = -1. */
int orc_dfs(const orc_graph* g, uint32_t s, int32_t* disc, int32_t* parent) {
  int rc = check_source(g, s);
  if (rc) return rc;
  const uint32_t n = g->n;
  uint64_t m = 0;
  for (uint32_t u = 0; u < n; u++) m += g->out[u].n;
  uint64_t* start = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  uint32_t* nb = (uint32_t*)malloc((size_t)(m + 1) * sizeof(uint32_t));
  uint64_t* cur = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  uint32_t* stk = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  if (!start || !nb || !cur || !stk) {
    free(start); free(nb); free(cur); free(stk);
    return ORC_E_OOM;
  }
  for (uint32_t u = 0; u < n; u++) {
    start[u + 1] = start[u] + g->out[u].n;
    for (uint32_t j = 0; j < g->out[u].n; j++) nb[start[u] + j] = g->out[u].a[j].v;
    qsort(nb + start[u], g->out[u].n, sizeof(uint32_t), cmp_u32);
  }
  for (uint32_t v = 0; v < n; v++) {
    disc[v] = -1;
    parent[v] = -1;
  }
  int32_t t = 0;
  uint32_t sp = 0;
  disc[s] = t++;
  cur[s] = start[s];
  stk[sp++] = s;
  while (sp > 0) {
    const uint32_t x = stk[sp - 1];
    if (cur[x] == start[x + 1]) {   /* every neighbour of x is done */
      sp--;
      continue;
    }
    const uint32_t y = nb[cur[x]++];
    if (disc[y] < 0) {
      disc[y] = t++;
      parent[y] = (int32_t)x;
      cur[y] = start[y];
      stk[sp++] = y;
    }
  }
  free(start); free(nb); free(cur); free(stk);
  return ORC_OK;
}
