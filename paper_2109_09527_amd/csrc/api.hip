// C boundary: graph lifetime, batches, single ops, snapshots, compaction,
// plain queries, statistics and tuning.  Every entry point catches its own
// failures and returns a dg_status; no exception leaves this file.
#include <algorithm>
#include <cstring>

#include <chrono>

#include "dg_host.h"

namespace dg {

static thread_local std::string g_create_err;

hipError_t ensure(DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes && b.p) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return e;
  }
  b.bytes = want;
  return hipSuccess;
}

void release(DevBuf& b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

// With p.mu held.
static hipEvent_t prof_event(Prof& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(dg_graph* g_, int kid_, hipStream_t s_) : g(g_), kid(kid_), s(s_) {
  {
    std::lock_guard<std::mutex> lk(g->prof.mu);
    if (!g->prof.on) return;
    a = prof_event(g->prof);
  }
  if (a) (void)hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
  if (!a) return;
  hipEvent_t b;
  {
    std::lock_guard<std::mutex> lk(g->prof.mu);
    b = prof_event(g->prof);
    if (!b) {
      g->prof.pool.push_back(a);
      return;
    }
  }
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g->prof.mu);
  g->prof.pending.push_back(Prof::Rec{kid, a, b});
}

void prof_arcs(dg_graph* g, int kid, uint64_t arcs) {
  std::lock_guard<std::mutex> lk(g->prof.mu);
  if (g->prof.on) g->prof.arcs[kid] += arcs;
}

void prof_scans(dg_graph* g, int kid, uint64_t arcs) {
  std::lock_guard<std::mutex> lk(g->prof.mu);
  if (!g->prof.on) return;
  g->prof.launches[kid]++;
  g->prof.arcs[kid] += arcs;
}

// With p.mu held.
static void prof_collect(Prof& p) {
  for (auto& r : p.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      p.ms[r.kid] += ms;
      p.launches[r.kid]++;
    }
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.pending.clear();
}

uint32_t gc_floor(const dg_graph* g) {
  uint32_t keep = std::max<uint32_t>(1, g->cfg.max_resident_epochs);
  uint32_t fl = g->epoch + 1 > keep ? g->epoch + 1 - keep : 0;
  if (!g->pins.empty()) fl = std::min(fl, g->pins.begin()->first);
  return fl;
}

bool alive_at(const dg_graph* g, uint32_t v, uint32_t e) {
  uint32_t t0 = g->vfirst[v];
  if (t0 == 0 || t0 > e) return false;
  uint32_t toggles = 1;
  for (uint32_t i = g->vhead[v]; i != VLOG_NONE; i = g->vlog[i].second)
    if (g->vlog[i].first <= e) toggles++;
  return toggles & 1;
}

uint64_t arcs_at(const dg_graph* g, uint32_t e) { return e < g->arcs_by_epoch.size() ? g->arcs_by_epoch[e] : 0; }
uint64_t live_at(const dg_graph* g, uint32_t e) { return e < g->live_by_epoch.size() ? g->live_by_epoch[e] : 0; }

static hipError_t realloc_pool(DevBuf& buf, DevBuf& sbuf, Pool& p, uint64_t new_cap, uint64_t used_buckets) {
  void* np = nullptr;
  void* ns = nullptr;
  hipError_t e = hipMalloc(&np, new_cap * p.words * 4ull);
  if (e != hipSuccess) return e;
  if ((e = hipMalloc(&ns, new_cap * SUM_WORDS * 4ull)) != hipSuccess) {
    hipFree(np);
    return e;
  }
  if (used_buckets) {
    e = hipMemcpy(np, p.base, used_buckets * p.words * 4ull, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(ns, p.sum, used_buckets * SUM_WORDS * 4ull, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      hipFree(np);
      hipFree(ns);
      return e;
    }
  }
  hipFree(buf.p);
  hipFree(sbuf.p);
  buf.p = np;
  buf.bytes = new_cap * p.words * 4ull;
  sbuf.p = ns;
  sbuf.bytes = new_cap * SUM_WORDS * 4ull;
  p.base = static_cast<uint32_t*>(np);
  p.sum = static_cast<uint32_t*>(ns);
  p.cap = new_cap;
  return hipSuccess;
}

// Enlarge the bucket pools so that `need` more buckets fit.  Every queued
// kernel on every stream finishes first: offsets stay valid (the contents
// are copied to the same offsets), only the base addresses change.
void pool_read_begin(dg_graph* g, std::unique_lock<std::mutex>& lk) {
  g->pool_cv.wait(lk, [g] { return g->pool_writers == 0; });
  g->pool_readers++;
}

void yield_to_updates(dg_graph* g) {
  const auto t0 = std::chrono::steady_clock::now();
  while (g->update_running.load() && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(4))
    std::this_thread::sleep_for(std::chrono::microseconds(20));
}

void pool_read_end(dg_graph* g) {
  std::lock_guard<std::mutex> lk(g->mu);
  g->pool_readers--;
  g->pool_cv.notify_all();
}

// Holds off new pool readers and waits for running ones, with g->mu held in
// lk; the destructor lets readers in again.
struct PoolWrite {
  dg_graph* g;
  PoolWrite(dg_graph* g_, std::unique_lock<std::mutex>& lk) : g(g_) {
    g->pool_writers++;
    g->pool_cv.wait(lk, [this] { return g->pool_readers == 0; });
  }
  ~PoolWrite() {
    g->pool_writers--;
    g->pool_cv.notify_all();
  }
};

hipError_t grow_pools(dg_graph* g, uint64_t need_f, uint64_t need_r) {
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_lock<std::mutex> lk(g->mu);
  PoolWrite pw(g, lk);
  struct Clock {
    dg_graph* g;
    std::chrono::steady_clock::time_point t0;
    ~Clock() {
      std::lock_guard<std::mutex> lk(g->prof.mu);
      if (!g->prof.on) return;
      g->prof.launches[KID_POOL_GROW]++;
      g->prof.ms[KID_POOL_GROW] +=
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
  } clock{g, t0};
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  unsigned long long cur[2];
  e = hipMemcpy(cur, g->st.cursor, sizeof(cur), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  if (cur[0] + need_f > g->st.fp.cap) {
    uint64_t nc = std::max<uint64_t>(2 * g->st.fp.cap, cur[0] + 2 * need_f + 1024);
    if ((e = realloc_pool(g->fpool, g->fsum, g->st.fp, nc, cur[0])) != hipSuccess) return e;
  }
  if (!g->st.undirected && cur[1] + need_r > g->st.rp.cap) {
    uint64_t nc = std::max<uint64_t>(2 * g->st.rp.cap, cur[1] + 2 * need_r + 1024);
    if ((e = realloc_pool(g->rpool, g->rsum, g->st.rp, nc, cur[1])) != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------ compaction
// Rebuild every slab into a fresh pool: keep the versions visible to some
// queryable epoch (death > floor), size each slab for <= 50% load, lay the
// slabs out in vertex order (offsets from an exclusive scan).

__global__ __launch_bounds__(256) void k_compact_plan(Pool p, const uint64_t* desc, uint32_t V, uint32_t floor_e,
                                                      uint32_t* nbk, uint32_t* kept_out) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t gwave = blockIdx.x * 4 + (threadIdx.x >> 6), nwaves = gridDim.x * 4;
  for (uint32_t v = gwave; v < V; v += nwaves) {
    Slab s = slab_of(p, desc[v]);
    uint32_t kept = 0;
    for (uint32_t t = lane; t < s.nb * BSLOTS; t += 64) {
      uint32_t* bp = bucket_ptr(s, t / BSLOTS);
      uint32_t j = t % BSLOTS;
      if (*slot_dst(bp, j) != EMPTY && *slot_death(bp, j, s.words) > floor_e) kept++;
    }
    kept = wave_sum_u32(kept);
    if (lane == 0) {
      uint32_t nb = 0;
      if (kept) {
        nb = 1;
        while (8ull * nb < kept) nb <<= 1;
      }
      nbk[v] = nb;
      kept_out[v] = kept;
    }
  }
}

__global__ __launch_bounds__(256) void k_compact_exec(Pool op, Pool np, uint64_t* desc, uint32_t* used, uint32_t V,
                                                      uint32_t floor_e, const uint32_t* nbk, const uint32_t* offs,
                                                      const uint32_t* kept) {
  for (uint32_t v = blockIdx.x; v < V; v += gridDim.x) {
    uint32_t nb = nbk[v];
    Slab os = slab_of(op, desc[v]);
    __syncthreads();
    if (nb == 0) {
      if (threadIdx.x == 0) {
        desc[v] = 0;
        used[v] = 0;
      }
      continue;
    }
    uint64_t off = 1ull + offs[v];   // bucket 0 stays unused
    Slab ns = slab_at(np, off, nb);
    for (uint64_t t = threadIdx.x; t < (uint64_t)nb * np.words; t += 256) ns.base[t] = 0xFFFFFFFFu;
    clear_summaries(ns.sum, nb, threadIdx.x, 256);
    __threadfence();
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < os.nb * BSLOTS; t += 256) {
      uint32_t* bp = bucket_ptr(os, t / BSLOTS);
      uint32_t j = t % BSLOTS;
      uint32_t d = *slot_dst(bp, j);
      if (d == EMPTY) continue;
      uint64_t stamp = *slot_stamp(bp, j, os.words);
      if ((uint32_t)(stamp >> 32) <= floor_e) continue;
      SlotRef r = claim_slot(ns, d, (uint32_t)stamp);
      if (np.words == FWD_WORDS) *slot_w(r.bp, r.j) = *slot_w(bp, j);
      *slot_stamp(r.bp, r.j, ns.words) = stamp;
      if ((uint32_t)(stamp >> 32) != INF_EPOCH) mark_tomb(ns, r.b, r.j, (uint32_t)(stamp >> 32));
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t lg = 0;
      while ((1u << lg) < nb) lg++;
      desc[v] = make_desc(off, lg);
      used[v] = kept[v];
    }
  }
}

static dg_status compact_pool(dg_graph* g, bool fwd, hipStream_t s) {
  const uint32_t V = g->cfg.v_capacity;
  Pool& p = fwd ? g->st.fp : g->st.rp;
  DevBuf& buf = fwd ? g->fpool : g->rpool;
  uint64_t* desc = fwd ? g->st.fdesc : g->st.rdesc;
  uint32_t* used = fwd ? g->st.fused : g->st.rused;
  DevBuf nbk, kept, scr;
  hipError_t e;
  if ((e = ensure(nbk, (V + 1) * 4ull)) != hipSuccess) return DG_E_OUT_OF_MEMORY;
  if ((e = ensure(kept, (V + 1) * 4ull)) != hipSuccess) return DG_E_OUT_OF_MEMORY;
  if ((e = ensure(scr, scan_scratch_words(V + 1) * 4 + 64)) != hipSuccess) return DG_E_OUT_OF_MEMORY;
  uint32_t fl = gc_floor(g);
  k_compact_plan<<<std::min<uint32_t>((V + 3) / 4, 8192), 256, 0, s>>>(p, desc, V, fl, nbk.as<uint32_t>(),
                                                                        kept.as<uint32_t>());
  hipMemsetAsync(nbk.as<uint32_t>() + V, 0, 4, s);
  DevBuf offs;
  if ((e = ensure(offs, (V + 1) * 4ull)) != hipSuccess) return DG_E_OUT_OF_MEMORY;
  hipMemcpyAsync(offs.p, nbk.p, (V + 1) * 4ull, hipMemcpyDeviceToDevice, s);
  exclusive_scan_u32(offs.as<uint32_t>(), V + 1, scr.as<uint32_t>(), s);
  uint32_t total = 0;
  hipMemcpyAsync(&total, offs.as<uint32_t>() + V, 4, hipMemcpyDeviceToHost, s);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) {
    g->err = std::string("compaction: ") + hipGetErrorString(e);
    return DG_E_HIP;
  }
  uint64_t need = 1ull + total;
  uint64_t ncap = std::max<uint64_t>(need * 2 + 1024, std::min<uint64_t>(p.cap, need * 4 + 1024));
  void* np = nullptr;
  void* nsum = nullptr;
  if ((e = hipMalloc(&np, ncap * p.words * 4ull)) != hipSuccess) {
    g->err = "compaction: out of device memory";
    return DG_E_OUT_OF_MEMORY;
  }
  if ((e = hipMalloc(&nsum, ncap * SUM_WORDS * 4ull)) != hipSuccess) {
    hipFree(np);
    g->err = "compaction: out of device memory";
    return DG_E_OUT_OF_MEMORY;
  }
  Pool npool{static_cast<uint32_t*>(np), static_cast<uint32_t*>(nsum), ncap, p.words};
  k_compact_exec<<<std::min<uint32_t>(V, 16384), 256, 0, s>>>(p, npool, desc, used, V, fl, nbk.as<uint32_t>(),
                                                             offs.as<uint32_t>(), kept.as<uint32_t>());
  unsigned long long cur = need;
  hipMemcpyAsync(g->st.cursor + (fwd ? 0 : 1), &cur, 8, hipMemcpyHostToDevice, s);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) {
    hipFree(np);
    hipFree(nsum);
    g->err = std::string("compaction: ") + hipGetErrorString(e);
    return DG_E_HIP;
  }
  DevBuf& sbuf = fwd ? g->fsum : g->rsum;
  hipFree(buf.p);
  hipFree(sbuf.p);
  buf.p = np;
  buf.bytes = ncap * p.words * 4ull;
  sbuf.p = nsum;
  sbuf.bytes = ncap * SUM_WORDS * 4ull;
  p = npool;
  release(nbk);
  release(kept);
  release(scr);
  release(offs);
  return DG_OK;
}

}  // namespace dg

using namespace dg;

// ------------------------------------------------------------------ ABI

static dg_status fail(dg_graph* g, dg_status st, const std::string& msg) {
  if (g) g->err = msg;
  else g_create_err = msg;
  return st;
}

extern "C" {

const char* dg_last_error(const dg_graph* g) { return g ? g->err.c_str() : g_create_err.c_str(); }

dg_epoch dg_latest_epoch(const dg_graph* g) {
  if (!g) return 0;
  std::lock_guard<std::mutex> lk(const_cast<dg_graph*>(g)->mu);
  return g->epoch;
}

dg_status dg_create(const dg_config* cfg, dg_graph** out) {
  if (!cfg || !out) return fail(nullptr, DG_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (cfg->v_capacity == 0 || cfg->v_capacity > 0x80000000u) return fail(nullptr, DG_E_INVALID_ARG, "v_capacity");
  if (cfg->w_max < 1) return fail(nullptr, DG_E_INVALID_ARG, "w_max");
  if ((int64_t)(cfg->v_capacity - 1) * (int64_t)cfg->w_max > 0x7fffffffLL)
    return fail(nullptr, DG_E_INVALID_ARG, "(v_capacity - 1) * w_max exceeds int32 distances");
  dg_graph* g = new (std::nothrow) dg_graph();
  if (!g) return fail(nullptr, DG_E_OUT_OF_MEMORY, "host allocation");
  g->cfg = *cfg;
  if (g->cfg.max_resident_epochs == 0) g->cfg.max_resident_epochs = 8;
  hipGetDevice(&g->device);
  const uint32_t V = cfg->v_capacity;
  uint32_t L = 1;
  while (L < 31 && (1ull << L) < V) L++;
  g->L = L;
  const bool und = (cfg->flags & DG_UNDIRECTED) != 0;
  uint64_t arcs = std::max<uint64_t>(cfg->edge_capacity, 1024);
  // initial pools: one bucket per vertex plus the arcs at ~50% load, x1.5
  uint64_t fcap = (uint64_t)(1.5 * (double)(V + arcs / 8)) + 1024;
  uint64_t rcap = und ? 1 : fcap;
  if (cfg->mem_budget) {
    uint64_t per = (uint64_t)FWD_WORDS * 4 + (und ? 0 : REV_WORDS * 4);
    uint64_t fixed = (uint64_t)V * (8 + 8 + 4 + 4 + 1 + 8);
    if (cfg->mem_budget > fixed) fcap = std::min<uint64_t>(fcap, (cfg->mem_budget - fixed) / per);
    rcap = und ? 1 : fcap;
  }
  hipError_t e = hipSuccess;
  auto E = [&](DevBuf& b, size_t bytes) {
    if (e == hipSuccess) e = ensure(b, bytes);
  };
  E(g->fdesc, V * 8ull);
  E(g->rdesc, V * 8ull);
  E(g->fused, V * 4ull);
  E(g->rused, V * 4ull);
  E(g->alive, V);
  E(g->insf, V * 4ull);
  E(g->insr, V * 4ull);
  E(g->cursor, 16);
  E(g->fpool, fcap * FWD_WORDS * 4ull);
  E(g->rpool, rcap * REV_WORDS * 4ull);
  E(g->fsum, fcap * SUM_WORDS * 4ull);
  E(g->rsum, rcap * SUM_WORDS * 4ull);
  if (e == hipSuccess) {
    hipMemset(g->fdesc.p, 0, V * 8ull);
    hipMemset(g->rdesc.p, 0, V * 8ull);
    hipMemset(g->fused.p, 0, V * 4ull);
    hipMemset(g->rused.p, 0, V * 4ull);
    hipMemset(g->alive.p, 0, V);
    hipMemset(g->insf.p, 0, V * 4ull);
    hipMemset(g->insr.p, 0, V * 4ull);
    unsigned long long cur[2] = {1, 1};
    hipMemcpy(g->cursor.p, cur, 16, hipMemcpyHostToDevice);
    e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    std::string msg = std::string("device allocation: ") + hipGetErrorString(e);
    dg_destroy(g);
    return fail(nullptr, DG_E_OUT_OF_MEMORY, msg);
  }
  Store& st = g->st;
  st.V = V;
  st.undirected = und ? 1 : 0;
  st.fdesc = g->fdesc.as<uint64_t>();
  st.rdesc = g->rdesc.as<uint64_t>();
  st.fused = g->fused.as<uint32_t>();
  st.rused = g->rused.as<uint32_t>();
  st.fp = Pool{g->fpool.as<uint32_t>(), g->fsum.as<uint32_t>(), fcap, (uint32_t)FWD_WORDS};
  st.rp = Pool{g->rpool.as<uint32_t>(), g->rsum.as<uint32_t>(), rcap, (uint32_t)REV_WORDS};
  st.cursor = g->cursor.as<unsigned long long>();
  st.alive = g->alive.as<uint8_t>();
  g->vfirst.assign(V, 0);
  g->vhead.assign(V, VLOG_NONE);
  // set-up that later calls must not repeat: the event updates wait on, and
  // the address of this device's fixed area for the allocation-free calls
  if ((e = hipEventCreateWithFlags(&g->last_query, hipEventDisableTiming)) != hipSuccess ||
      (e = noalloc_setup(g->device)) != hipSuccess) {
    std::string msg = std::string("set-up: ") + hipGetErrorString(e);
    dg_destroy(g);
    return fail(nullptr, DG_E_HIP, msg);
  }
  *out = g;
  return DG_OK;
}

dg_status dg_destroy(dg_graph* g) {
  if (!g) return DG_E_INVALID_ARG;
  hipDeviceSynchronize();
  for (DevBuf* b : {&g->fdesc, &g->rdesc, &g->fused, &g->rused, &g->fpool, &g->rpool, &g->fsum, &g->rsum,
                    &g->cursor, &g->alive, &g->insf, &g->insr})
    release(*b);
  UpdateScratch& u = g->us;
  for (DevBuf* b : {&u.keys0, &u.keys1, &u.vals0, &u.vals1, &u.sortw, &u.vafter, &u.vlastrem, &u.recflags,
                    &u.recw, &u.ops, &u.results, &u.touch, &u.plan, &u.clear, &u.summary})
    release(*b);
  if (u.host_summary) hipHostFree(u.host_summary);
  free_query_scratch(g->qs);
  free_pr_scratch(g->pr);
  free_scc_scratch(g->scc);
  free_diam_scratch(g->diam);
  free_flow_scratch(g->flow);
  free_dfs_scratch(g->dfs);
  free_batch_state(g);
  for (auto& r : g->prof.pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (hipEvent_t e : g->prof.pool) hipEventDestroy(e);
  if (g->last_query) hipEventDestroy(g->last_query);
  delete g;
  return DG_OK;
}

dg_status dg_apply_batch(dg_graph* g, const dg_op* ops, uint64_t n, uint8_t* results, dg_epoch* new_epoch,
                         void* stream) {
  if (!g) return DG_E_INVALID_ARG;
  if (n && !ops) return fail(g, DG_E_INVALID_ARG, "ops is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    if (n == 0) {
      if (new_epoch) *new_epoch = dg_latest_epoch(g);
      return DG_OK;
    }
    std::lock_guard<std::mutex> lk(g->upd_mu);
    hipError_t e = hipSuccess;
    const dg_op* dops = ops;
    if (!is_device_ptr(ops)) {
      // size all of the batch scratch first: growing it later would replace
      // the staging buffer under the copy
      if ((e = ensure_update_scratch(g, n)) != hipSuccess) return fail(g, DG_E_OUT_OF_MEMORY, "ops staging");
      if ((e = hipMemcpyAsync(g->us.ops.p, ops, n * sizeof(dg_op), hipMemcpyHostToDevice, s)) != hipSuccess)
        return fail(g, DG_E_HIP, std::string("ops copy: ") + hipGetErrorString(e));
      dops = g->us.ops.as<dg_op>();
    }
    bool dev_res = results && is_device_ptr(results);
    // plain queries scan buckets without per-slot stamps when no writer
    // runs beside them: let queued query work finish before the batch
    if (g->last_query && (e = hipStreamWaitEvent(s, g->last_query, 0)) != hipSuccess)
      return fail(g, DG_E_HIP, std::string("stream wait: ") + hipGetErrorString(e));
    dg_status st = apply_batch_dev(g, dops, n, dev_res ? results : nullptr, s);
    if (st != DG_OK) return st;
    if (results && !dev_res) {
      if ((e = hipMemcpyAsync(results, g->us.results.p, n, hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(g, DG_E_HIP, std::string("results copy: ") + hipGetErrorString(e));
    }
    if (new_epoch) *new_epoch = dg_latest_epoch(g);
    return DG_OK;
  } catch (const std::bad_alloc&) {
    return fail(g, DG_E_OUT_OF_MEMORY, "host allocation");
  } catch (...) {
    return fail(g, DG_E_HIP, "unexpected failure in dg_apply_batch");
  }
}

static dg_status single(dg_graph* g, uint32_t type, uint32_t u, uint32_t v, int32_t w, uint8_t* res, dg_epoch* ep) {
  dg_op op{type, u, v, w};
  uint8_t r = 0;
  dg_status st = dg_apply_batch(g, &op, 1, &r, ep, nullptr);
  if (st == DG_OK && res) *res = r;
  return st;
}

dg_status dg_add_vertex(dg_graph* g, uint32_t v, uint8_t* res, dg_epoch* ep) {
  return single(g, DG_ADD_VERTEX, v, 0, 0, res, ep);
}
dg_status dg_remove_vertex(dg_graph* g, uint32_t v, uint8_t* res, dg_epoch* ep) {
  return single(g, DG_REMOVE_VERTEX, v, 0, 0, res, ep);
}
dg_status dg_contains_vertex(dg_graph* g, uint32_t v, uint8_t* res, dg_epoch* ep) {
  return single(g, DG_CONTAINS_VERTEX, v, 0, 0, res, ep);
}
dg_status dg_add_edge(dg_graph* g, uint32_t u, uint32_t v, int32_t w, uint8_t* res, dg_epoch* ep) {
  return single(g, DG_ADD_EDGE, u, v, w, res, ep);
}
dg_status dg_remove_edge(dg_graph* g, uint32_t u, uint32_t v, uint8_t* res, dg_epoch* ep) {
  return single(g, DG_REMOVE_EDGE, u, v, 0, res, ep);
}
dg_status dg_contains_edge(dg_graph* g, uint32_t u, uint32_t v, uint8_t* res, dg_epoch* ep) {
  return single(g, DG_CONTAINS_EDGE, u, v, 0, res, ep);
}

static dg_status resolve_epoch(dg_graph* g, dg_epoch want, uint32_t* e) {
  uint32_t ep = want == DG_EPOCH_LATEST ? g->epoch : want;
  if (ep > g->epoch) return fail(g, DG_E_EPOCH_RETIRED, "epoch not yet published");
  if (ep < gc_floor(g)) return fail(g, DG_E_EPOCH_RETIRED, "epoch below the retained window");
  *e = ep;
  return DG_OK;
}

dg_status dg_snapshot_acquire(dg_graph* g, dg_epoch want, dg_epoch* pinned) {
  if (!g) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  g->pins[e]++;
  if (pinned) *pinned = e;
  return DG_OK;
}

dg_status dg_snapshot_release(dg_graph* g, dg_epoch e) {
  if (!g) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g->mu);
  auto it = g->pins.find(e);
  if (it == g->pins.end()) return fail(g, DG_E_INVALID_ARG, "epoch is not pinned");
  if (--it->second == 0) g->pins.erase(it);
  return DG_OK;
}

dg_status dg_compact(dg_graph* g, void* stream) {
  if (!g) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lku(g->upd_mu);
  std::unique_lock<std::mutex> lk(g->mu);
  // running multi-pass searches hold slab descriptors between passes
  struct Waiting {
    dg_graph* g;
    ~Waiting() {
      g->compact_waiting--;
      g->pool_cv.notify_all();
    }
  } waiting{g};
  g->compact_waiting++;
  g->pool_cv.wait(lk, [g] { return g->search_holds == 0; });
  PoolWrite pw(g, lk);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipDeviceSynchronize() != hipSuccess) return fail(g, DG_E_HIP, "compaction: device sync");
  dg_status st = compact_pool(g, true, s);
  if (st == DG_OK && !g->st.undirected) st = compact_pool(g, false, s);
  return st;
}

static dg_status note_query(dg_graph* g, dg_status st, void* stream) {
  if (st != DG_OK) return st;
  if (hipEventRecord(g->last_query, static_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(g, DG_E_HIP, "event record");
  return DG_OK;
}

static dg_status check_source(dg_graph* g, uint32_t e, uint32_t src) {
  if (src >= g->cfg.v_capacity) return fail(g, DG_E_VERTEX_RANGE, "source id out of range");
  if (!alive_at(g, src, e)) return fail(g, DG_E_SOURCE_ABSENT, "source is not live at the epoch");
  return DG_OK;
}

dg_status dg_bfs(dg_graph* g, dg_epoch want, uint32_t src, int32_t* dist, void* stream) {
  if (!g || !dist) return DG_E_INVALID_ARG;
  if (!is_device_ptr(dist)) return fail(g, DG_E_INVALID_ARG, "dist must be device memory");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st == DG_OK) st = check_source(g, e, src);
  if (st != DG_OK) return st;
  return note_query(g, bfs_dev(g, e, src, dist, static_cast<hipStream_t>(stream), g->qs), stream);
}

dg_status dg_bfs_noalloc(dg_graph* g, dg_epoch want, uint32_t src, int32_t* dist, void* stream) {
  if (!g || !dist) return DG_E_INVALID_ARG;
  if (!is_device_ptr(dist)) return fail(g, DG_E_INVALID_ARG, "dist must be device memory");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st == DG_OK) st = check_source(g, e, src);
  if (st != DG_OK) return st;
  const uint64_t need = bfs_fixed_layout(g, nullptr, nullptr);
  if (need > DG_NOALLOC_SCRATCH_BYTES)
    return fail(g, DG_E_OUT_OF_MEMORY,
                "dg_bfs_noalloc: this graph's search needs " + std::to_string(need) +
                    " bytes of scratch; the fixed area holds " + std::to_string(DG_NOALLOC_SCRATCH_BYTES));
  char* area = static_cast<char*>(noalloc_area(g->device));
  if (!area) return fail(g, DG_E_HIP, "dg_bfs_noalloc: fixed area not set up on this device");
  QueryScratch q;
  bfs_fixed_layout(g, area, &q);
  return note_query(g, bfs_dev(g, e, src, dist, static_cast<hipStream_t>(stream), q), stream);
}

dg_status dg_sssp(dg_graph* g, dg_epoch want, uint32_t src, int32_t* dist, void* stream) {
  if (!g || !dist) return DG_E_INVALID_ARG;
  if (!is_device_ptr(dist)) return fail(g, DG_E_INVALID_ARG, "dist must be device memory");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st == DG_OK) st = check_source(g, e, src);
  if (st != DG_OK) return st;
  return note_query(g, sssp_dev(g, e, src, dist, static_cast<hipStream_t>(stream), g->qs), stream);
}

dg_status dg_bc(dg_graph* g, dg_epoch want, const uint32_t* srcs, uint32_t k, double* bc, void* stream) {
  if (!g || !bc || (k && !srcs)) return DG_E_INVALID_ARG;
  if (!is_device_ptr(bc)) return fail(g, DG_E_INVALID_ARG, "bc must be device memory");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  std::vector<uint32_t> S(srcs, srcs + k);
  for (uint32_t i = 0; i < k; i++)
    if ((st = check_source(g, e, S[i])) != DG_OK) return st;
  std::vector<uint32_t> sorted = S;
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(g, DG_E_INVALID_ARG, "repeated BC source");
  return note_query(g, bc_dev(g, e, S.data(), k, bc, static_cast<hipStream_t>(stream), g->qs), stream);
}

static dg_status pagerank_call(dg_graph* g, dg_epoch want, const dg_pagerank_opts& o, double* pr,
                               uint32_t* iterations, double* last_change, void* stream) {
  if (!g || !pr) return DG_E_INVALID_ARG;
  if (!is_device_ptr(pr)) return fail(g, DG_E_INVALID_ARG, "pr must be device memory");
  if (!(o.damping >= 0.0 && o.damping < 1.0)) return fail(g, DG_E_INVALID_ARG, "damping must lie in [0, 1)");
  if (!(o.threshold >= 0.0)) return fail(g, DG_E_INVALID_ARG, "threshold must be non-negative");
  if (!(o.freeze_below >= 0.0)) return fail(g, DG_E_INVALID_ARG, "freeze_below must be non-negative");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  uint32_t it = 0;
  double ch = 0.0;
  st = pagerank_dev(g, e, o.damping, o.threshold, o.freeze_below, o.max_iters, pr, &it, &ch,
                    static_cast<hipStream_t>(stream), o.nosync != 0);
  if (iterations) *iterations = it;
  if (last_change) *last_change = ch;
  return note_query(g, st, stream);
}

dg_status dg_pagerank(dg_graph* g, dg_epoch want, double damping, double threshold, uint32_t max_iters, double* pr,
                      uint32_t* iterations, double* last_change, void* stream) {
  const dg_pagerank_opts o{damping, threshold, 0.0, max_iters, 0};
  return pagerank_call(g, want, o, pr, iterations, last_change, stream);
}

dg_status dg_pagerank_nosync(dg_graph* g, dg_epoch want, double damping, double threshold, uint32_t max_iters,
                             double* pr, uint32_t* sweeps, double* last_change, void* stream) {
  const dg_pagerank_opts o{damping, threshold, 0.0, max_iters, 1};
  return pagerank_call(g, want, o, pr, sweeps, last_change, stream);
}

dg_status dg_pagerank_ex(dg_graph* g, dg_epoch want, const dg_pagerank_opts* opts, double* pr, uint32_t* iterations,
                         double* last_change, void* stream) {
  if (!opts) return DG_E_INVALID_ARG;
  return pagerank_call(g, want, *opts, pr, iterations, last_change, stream);
}

dg_status dg_scc(dg_graph* g, dg_epoch want, int32_t* comp, uint32_t* n_components, void* stream) {
  if (!g || !comp) return DG_E_INVALID_ARG;
  if (!is_device_ptr(comp)) return fail(g, DG_E_INVALID_ARG, "comp must be device memory");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  return note_query(g, scc_dev(g, e, comp, n_components, nullptr, static_cast<hipStream_t>(stream)), stream);
}

dg_status dg_diameter(dg_graph* g, dg_epoch want, uint32_t* diameter, void* stream) {
  if (!g || !diameter) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  return note_query(g, diameter_dev(g, e, diameter, static_cast<hipStream_t>(stream)), stream);
}

dg_status dg_maxflow(dg_graph* g, dg_epoch want, uint32_t s, uint32_t t, int64_t* flow, void* stream) {
  if (!g || !flow) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  if ((st = check_source(g, e, s)) != DG_OK || (st = check_source(g, e, t)) != DG_OK) return st;
  if (s == t) return fail(g, DG_E_INVALID_ARG, "maxflow: source and sink are the same vertex");
  return note_query(g, maxflow_dev(g, e, s, t, flow, static_cast<hipStream_t>(stream)), stream);
}

dg_status dg_dfs(dg_graph* g, dg_epoch want, uint32_t s, int32_t* disc, int32_t* parent, uint32_t* n_reached,
                 void* stream) {
  if (!g || !disc) return DG_E_INVALID_ARG;
  if (!is_device_ptr(disc) || (parent && !is_device_ptr(parent)))
    return fail(g, DG_E_INVALID_ARG, "disc and parent must be device memory");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  if ((st = check_source(g, e, s)) != DG_OK) return st;
  return note_query(g, dfs_dev(g, e, s, disc, parent, n_reached, static_cast<hipStream_t>(stream)), stream);
}

dg_status dg_stats(dg_graph* g, dg_epoch want, uint64_t* n_vertices, uint64_t* n_arcs, void* stream) {
  if (!g) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  if (n_vertices) *n_vertices = live_at(g, e);
  if (n_arcs) return stats_dev(g, e, n_arcs, nullptr, static_cast<hipStream_t>(stream));
  return DG_OK;
}

dg_status dg_out_degrees(dg_graph* g, dg_epoch want, uint32_t* deg, void* stream) {
  if (!g || !deg) return DG_E_INVALID_ARG;
  if (!is_device_ptr(deg)) return fail(g, DG_E_INVALID_ARG, "deg must be device memory");
  std::lock_guard<std::mutex> lk(g->mu);
  uint32_t e;
  dg_status st = resolve_epoch(g, want, &e);
  if (st != DG_OK) return st;
  return stats_dev(g, e, nullptr, deg, static_cast<hipStream_t>(stream));
}

dg_status dg_profile_enable(dg_graph* g, int on) {
  if (!g) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g->mu);
  std::lock_guard<std::mutex> lp(g->prof.mu);
  g->prof.on = on != 0;
  // events for a few thousand timed launches, so that timing them creates
  // no event inside the region being timed
  constexpr size_t PROF_POOL = 4096;
  while (g->prof.on && g->prof.pool.size() + g->prof.pending.size() * 2 < PROF_POOL) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) break;
    g->prof.pool.push_back(e);
  }
  return DG_OK;
}

dg_status dg_profile_read(dg_graph* g, dg_kernel_stat* out, uint32_t cap, uint32_t* n_out, int reset) {
  static const char* names[KID_COUNT] = {"update_batch", "bfs_top_down", "bfs_bottom_up", "sssp_relax",
                                         "sssp_split",   "bc_forward",   "bc_backward",   "batch_bfs",
                                         "batch_sssp",   "batch_bc",     "pagerank",     "pagerank_nosync", "scc",
                                         "diameter",     "maxflow",      "dfs",          "pool_growth",  "batch_sssp_scan",
                                         "serve_bfs",    "serve_sssp"};
  if (!g) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g->mu);
  std::lock_guard<std::mutex> lp(g->prof.mu);
  prof_collect(g->prof);
  uint32_t n = 0;
  for (int k = 0; k < KID_COUNT && n < cap; k++) {
    if (!out) break;
    out[n].name = names[k];
    out[n].launches = g->prof.launches[k];
    out[n].total_ms = g->prof.ms[k];
    out[n].arcs = g->prof.arcs[k];
    n++;
  }
  if (n_out) *n_out = out ? n : KID_COUNT;
  if (reset) {
    std::fill(std::begin(g->prof.launches), std::end(g->prof.launches), 0ull);
    std::fill(std::begin(g->prof.ms), std::end(g->prof.ms), 0.0);
    std::fill(std::begin(g->prof.arcs), std::end(g->prof.arcs), 0ull);
  }
  return DG_OK;
}

dg_status dg_get_tuning(const dg_graph* g, dg_tuning* t) {
  if (!g || !t) return DG_E_INVALID_ARG;
  t->chunk_buckets = g->tune.chunk_buckets;
  t->sssp_delta = g->tune.sssp_delta;
  t->alpha = g->tune.alpha;
  t->beta = g->tune.beta;
  t->batch_groups = g->tune.batch_groups;
  t->batch_delta = g->tune.batch_delta;
  t->batch_gang = g->tune.batch_gang;
  return DG_OK;
}

dg_status dg_set_tuning(dg_graph* g, const dg_tuning* t) {
  if (!g || !t) return DG_E_INVALID_ARG;
  const uint32_t C = t->chunk_buckets;
  if (C != 16 && C != 32 && C != 64) return fail(g, DG_E_INVALID_ARG, "chunk_buckets must be 16, 32 or 64");
  if (t->sssp_delta == 0 || t->alpha == 0 || t->beta == 0 || t->batch_delta == 0)
    return fail(g, DG_E_INVALID_ARG, "tuning values must be positive");
  if (t->batch_gang > 128) return fail(g, DG_E_INVALID_ARG, "batch_gang must be at most 128");
  std::lock_guard<std::mutex> lk(g->mu);
  g->tune.chunk_buckets = C;
  g->tune.sssp_delta = t->sssp_delta;
  g->tune.alpha = t->alpha;
  g->tune.beta = t->beta;
  g->tune.batch_groups = t->batch_groups;
  g->tune.batch_delta = t->batch_delta;
  g->tune.batch_gang = t->batch_gang;
  return DG_OK;
}

}  // extern "C"
