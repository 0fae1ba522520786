// Serving loop: continuous batching of update batches and snapshot queries
// over one graph.
//
//   update thread  applies update requests in arrival order on its own
//                  stream; each publishes the next epoch.
//   query lanes    (query_lanes threads, each with a stream and an engine
//                  instance of its own) each take, whenever it is free, the
//                  waiting queries at the head of the queue in arrival order
//                  while their output memory fits the budget and the
//                  in-flight cap allows (up to max_batch at once), bind them
//                  to the latest published epoch (their linearization point)
//                  and run them in one persistent engine launch.  A query
//                  arriving while a lane is busy is taken by the next lane to
//                  come free, so the launches of different lanes overlap on
//                  the device with each other and with the update stream.
// While a server runs, scans read per-slot stamps (no summary fast path),
// since update kernels may write slabs under running queries, and the
// engine launches share part of the device's resident-workgroup capacity
// (the rest stays free for the update kernels).  Latency = completion -
// submission, host clock.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "dg_host.h"

namespace {

using clk = std::chrono::steady_clock;

struct Req {
  uint64_t ticket = 0;
  int kind = -1;                 // -1 update, else DG_Q_*
  std::vector<dg_op> ops;
  std::vector<uint32_t> srcs;
  double t_arrive = 0, t_done = 0;
  dg_status status = DG_OK;
  uint32_t epoch = 0;
  bool done = false;
  std::vector<uint8_t> results;  // update: per-op result bytes
  std::vector<char> out;         // query: host copy of the output
  uint64_t reserve = 0;
};

double pct(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::max(1.0, std::ceil(p / 100.0 * (double)v.size()));
  return v[std::min(k, v.size()) - 1];
}

}  // namespace

struct dg_server {
  dg_graph* g = nullptr;
  dg_server_config cfg{};
  std::mutex m;
  std::condition_variable cv, cv_done;
  std::deque<Req*> uq, qq;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next = 1;
  bool stop = false;
  uint64_t mem_used = 0;
  uint32_t busy = 0;             // requests taken by a worker, not yet finished
  uint32_t q_running = 0;        // queries taken by a lane, not yet finished
  std::thread tu;
  std::vector<std::thread> tq;   // one per query lane
  hipStream_t su = nullptr;
  std::vector<hipStream_t> sq;   // one per query lane
  clk::time_point t0;
  std::vector<double> lat_all, lat_q, lat_u;
  uint64_t ops_applied = 0, arcs = 0, n_upd = 0, n_qry = 0;
  double t_first = -1, t_last = 0;
  // the log: finished requests in completion order (sorted into
  // linearization order when read), with their ops (if kept) and sources
  struct LogRec {
    dg_log_record r;
    int cls;   // 0: an update that published r.epoch; 1: a query or a rejected update
  };
  std::vector<LogRec> log;
  std::vector<dg_op> log_ops;
  std::vector<uint32_t> log_srcs;

  double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }

  uint64_t out_bytes(const Req* r) const {
    uint64_t V = g->cfg.v_capacity;
    return r->kind == DG_Q_BC ? V * 8 : V * 4;
  }

  void finish(Req* r, dg_status st, uint32_t ep) {
    std::lock_guard<std::mutex> lk(m);
    r->status = st;
    r->epoch = ep;
    r->t_done = now();
    r->done = true;
    double lat = (r->t_done - r->t_arrive) * 1e3;
    lat_all.push_back(lat);
    (r->kind < 0 ? lat_u : lat_q).push_back(lat);
    if (r->kind < 0) {
      n_upd++;
      if (st == DG_OK) ops_applied += r->ops.size();
    } else {
      n_qry++;
    }
    LogRec lr{};
    lr.r.ticket = r->ticket;
    lr.r.kind = r->kind;
    lr.r.status = st;
    lr.r.epoch = ep;
    lr.r.t_arrive_ms = r->t_arrive * 1e3;
    lr.r.t_done_ms = r->t_done * 1e3;
    lr.cls = (r->kind < 0 && st == DG_OK) ? 0 : 1;
    if (r->kind < 0) {
      lr.r.n = (uint32_t)r->ops.size();
      lr.r.off = UINT64_MAX;
      if (cfg.log_ops) {
        lr.r.off = log_ops.size();
        log_ops.insert(log_ops.end(), r->ops.begin(), r->ops.end());
      }
    } else {
      lr.r.n = (uint32_t)r->srcs.size();
      lr.r.off = log_srcs.size();
      log_srcs.insert(log_srcs.end(), r->srcs.begin(), r->srcs.end());
    }
    log.push_back(lr);
    t_last = std::max(t_last, r->t_done);
    mem_used -= r->reserve;
    r->reserve = 0;
    busy--;
    if (r->kind >= 0) q_running--;
    cv_done.notify_all();
    cv.notify_all();
  }

  void update_loop() {
    for (;;) {
      Req* r;
      {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return stop || !uq.empty(); });
        if (uq.empty()) return;
        r = uq.front();
        uq.pop_front();
        busy++;
      }
      r->results.assign(r->ops.size(), 0);
      dg_epoch ep = 0;
      dg_status st = dg_apply_batch(g, r->ops.data(), r->ops.size(), r->results.data(), &ep, su);
      // a rejected batch publishes nothing: it stands at the epoch that is
      // latest (only this thread publishes, so that is still the one it saw)
      if (st != DG_OK) ep = dg_latest_epoch(g);
      finish(r, st, ep);
    }
  }

  void query_loop(uint32_t lane) {
    std::vector<Req*> batch;
    std::vector<dg::DevBuf> outs;
    hipStream_t sq_ = sq[lane];
    for (;;) {
      batch.clear();
      {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] {
          if (stop && qq.empty()) return true;
          return !qq.empty() && q_running < cfg.max_inflight && mem_used + out_bytes(qq.front()) <= cfg.mem_budget;
        });
        if (qq.empty()) {
          for (auto& o : outs) dg::release(o);
          return;
        }
        while (!qq.empty() && batch.size() < cfg.max_batch && q_running < cfg.max_inflight) {
          Req* r = qq.front();
          uint64_t need = out_bytes(r);
          if (mem_used + need > cfg.mem_budget) break;   // arrival order: the head waits
          mem_used += need;
          r->reserve = need;
          batch.push_back(r);
          qq.pop_front();
          busy++;
          q_running++;
        }
      }
      // linearization point: the latest published epoch, pinned until done
      dg_epoch e_bind = 0;
      const bool pinned = dg_snapshot_acquire(g, DG_EPOCH_LATEST, &e_bind) == DG_OK;
      const size_t n = batch.size();
      if (outs.size() < n) outs.resize(n);
      std::vector<dg_query> qs(n);
      bool alloc_ok = true;
      for (size_t i = 0; i < n; i++) {
        Req* r = batch[i];
        if (dg::ensure(outs[i], out_bytes(r)) != hipSuccess) alloc_ok = false;
        qs[i] = dg_query{(uint32_t)r->kind, r->kind == DG_Q_BC ? 0u : (r->srcs.empty() ? 0u : r->srcs[0]), e_bind,
                         r->kind == DG_Q_BC ? (uint32_t)r->srcs.size() : 0u,
                         r->kind == DG_Q_BC ? r->srcs.data() : nullptr, outs[i].p};
      }
      // BFS and SSSP first, BC after, on the same epoch: the short queries
      // of a round finish without waiting for its BC sources
      std::vector<size_t> order;
      for (int heavy = 0; heavy < 2; heavy++)
        for (size_t i = 0; i < n; i++)
          if ((batch[i]->kind == DG_Q_BC) == (heavy == 1)) order.push_back(i);
      size_t o0 = 0;
      while (o0 < n) {
        const bool heavy = batch[order[o0]]->kind == DG_Q_BC;
        size_t o1 = o0;
        while (o1 < n && (batch[order[o1]]->kind == DG_Q_BC) == heavy) o1++;
        std::vector<dg_query> part;
        for (size_t t = o0; t < o1; t++) part.push_back(qs[order[t]]);
        std::vector<dg_status> pst(part.size(), DG_OK);
        const uint64_t arcs0 = g->engine_arcs.load();
        dg_status call = alloc_ok ? dg::query_batch_dev(g, part.data(), (uint32_t)part.size(), pst.data(), sq_, 1 + lane)
                                  : DG_E_OUT_OF_MEMORY;
        {
          std::lock_guard<std::mutex> lk(m);
          arcs += g->engine_arcs.load() - arcs0;
        }
        for (size_t t = o0; t < o1; t++) {
          const size_t i = order[t];
          Req* r = batch[i];
          dg_status s = call != DG_OK ? call : pst[t - o0];
          if (s == DG_OK) {
            r->out.resize(out_bytes(r));
            if (hipMemcpyAsync(r->out.data(), outs[i].p, r->out.size(), hipMemcpyDeviceToHost, sq_) != hipSuccess ||
                hipStreamSynchronize(sq_) != hipSuccess)
              s = DG_E_HIP;
          }
          finish(r, s, e_bind);
        }
        o0 = o1;
      }
      if (pinned) dg_snapshot_release(g, e_bind);
    }
  }
};

extern "C" {

dg_status dg_server_start(dg_graph* g, const dg_server_config* cfg, dg_server** out) {
  if (!g || !cfg || !out) return DG_E_INVALID_ARG;
  *out = nullptr;
  auto* s = new (std::nothrow) dg_server();
  if (!s) return DG_E_OUT_OF_MEMORY;
  s->g = g;
  s->cfg = *cfg;
  if (!s->cfg.mem_budget) s->cfg.mem_budget = 8ull << 30;
  if (!s->cfg.max_batch) s->cfg.max_batch = 64;
  if (!s->cfg.max_inflight) s->cfg.max_inflight = 1024;
  if (!s->cfg.query_lanes) s->cfg.query_lanes = 1;
  if (s->cfg.query_lanes > 4) {
    delete s;
    g->err = "query_lanes must be at most 4";
    return DG_E_INVALID_ARG;
  }
  bool ok = hipStreamCreateWithFlags(&s->su, hipStreamNonBlocking) == hipSuccess;
  for (uint32_t i = 0; ok && i < s->cfg.query_lanes; i++) {
    hipStream_t x = nullptr;
    ok = hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess;
    if (ok) s->sq.push_back(x);
  }
  if (!ok) {
    if (s->su) hipStreamDestroy(s->su);
    for (hipStream_t x : s->sq) hipStreamDestroy(x);
    delete s;
    g->err = "server stream creation";
    return DG_E_HIP;
  }
  {
    std::lock_guard<std::mutex> lk(g->mu);
    g->concurrent_writers++;
    // three quarters of the resident workgroups, split over the lanes
    g->engine_share_pct = std::max<uint32_t>(1, 75 / s->cfg.query_lanes);
  }
  s->t0 = clk::now();
  s->tu = std::thread([s] { s->update_loop(); });
  for (uint32_t i = 0; i < s->cfg.query_lanes; i++) s->tq.emplace_back([s, i] { s->query_loop(i); });
  *out = s;
  return DG_OK;
}

dg_status dg_server_stop(dg_server* s) {
  if (!s) return DG_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
  }
  s->cv.notify_all();
  s->tu.join();
  for (auto& t : s->tq) t.join();
  hipStreamSynchronize(s->su);
  hipStreamDestroy(s->su);
  for (hipStream_t x : s->sq) {
    hipStreamSynchronize(x);
    hipStreamDestroy(x);
  }
  {
    std::lock_guard<std::mutex> lk(s->g->mu);
    s->g->concurrent_writers--;
    if (!s->g->concurrent_writers) s->g->engine_share_pct = 100;
  }
  delete s;
  return DG_OK;
}

static dg_status submit(dg_server* s, std::unique_ptr<Req> r, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(s->m);
  if (s->stop) return DG_E_BUSY;
  r->ticket = s->next++;
  r->t_arrive = s->now();
  if (s->t_first < 0) s->t_first = r->t_arrive;
  Req* raw = r.get();
  s->reqs[raw->ticket] = std::move(r);
  (raw->kind < 0 ? s->uq : s->qq).push_back(raw);
  if (ticket) *ticket = raw->ticket;
  s->cv.notify_all();
  return DG_OK;
}

dg_status dg_server_submit_update(dg_server* s, const dg_op* ops, uint64_t n, uint64_t* ticket) {
  if (!s || (n && !ops)) return DG_E_INVALID_ARG;
  auto r = std::make_unique<Req>();
  r->kind = -1;
  r->ops.assign(ops, ops + n);
  return submit(s, std::move(r), ticket);
}

dg_status dg_server_submit_query(dg_server* s, uint32_t kind, const uint32_t* srcs, uint32_t k, uint64_t* ticket) {
  if (!s || kind > DG_Q_BC || (k && !srcs) || (kind != DG_Q_BC && k != 1)) return DG_E_INVALID_ARG;
  uint64_t need = kind == DG_Q_BC ? 8ull * s->g->cfg.v_capacity : 4ull * s->g->cfg.v_capacity;
  if (need > s->cfg.mem_budget) return DG_E_BUSY;   // could never be admitted
  auto r = std::make_unique<Req>();
  r->kind = (int)kind;
  r->srcs.assign(srcs, srcs + k);
  return submit(s, std::move(r), ticket);
}

dg_status dg_server_poll(dg_server* s, uint64_t ticket, int* done, dg_status* status, dg_epoch* epoch,
                         double* latency_ms) {
  if (!s) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return DG_E_INVALID_ARG;
  Req* r = it->second.get();
  if (done) *done = r->done ? 1 : 0;
  if (r->done) {
    if (status) *status = r->status;
    if (epoch) *epoch = r->epoch;
    if (latency_ms) *latency_ms = (r->t_done - r->t_arrive) * 1e3;
  }
  return DG_OK;
}

dg_status dg_server_take(dg_server* s, uint64_t ticket, void* host_out, uint64_t bytes) {
  if (!s) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || !it->second->done) return DG_E_INVALID_ARG;
  Req* r = it->second.get();
  const void* src = r->kind < 0 ? (const void*)r->results.data() : (const void*)r->out.data();
  uint64_t have = r->kind < 0 ? r->results.size() : r->out.size();
  if (host_out && bytes) std::memcpy(host_out, src, std::min(bytes, have));
  s->reqs.erase(it);
  return DG_OK;
}

dg_status dg_server_log(dg_server* s, dg_log_record* recs, uint64_t rec_cap, uint64_t* n_recs, dg_op* ops,
                        uint64_t ops_cap, uint64_t* n_ops, uint32_t* srcs, uint64_t srcs_cap, uint64_t* n_srcs) {
  if (!s) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  if (recs && rec_cap) {
    std::vector<const dg_server::LogRec*> order;
    order.reserve(s->log.size());
    for (const auto& x : s->log) order.push_back(&x);
    std::sort(order.begin(), order.end(), [](const dg_server::LogRec* a, const dg_server::LogRec* b) {
      if (a->r.epoch != b->r.epoch) return a->r.epoch < b->r.epoch;
      if (a->cls != b->cls) return a->cls < b->cls;
      return a->r.ticket < b->r.ticket;
    });
    for (uint64_t i = 0; i < order.size() && i < rec_cap; i++) recs[i] = order[i]->r;
  }
  if (ops && ops_cap) std::memcpy(ops, s->log_ops.data(), std::min<uint64_t>(ops_cap, s->log_ops.size()) * sizeof(dg_op));
  if (srcs && srcs_cap)
    std::memcpy(srcs, s->log_srcs.data(), std::min<uint64_t>(srcs_cap, s->log_srcs.size()) * sizeof(uint32_t));
  if (n_recs) *n_recs = s->log.size();
  if (n_ops) *n_ops = s->log_ops.size();
  if (n_srcs) *n_srcs = s->log_srcs.size();
  return DG_OK;
}

dg_status dg_server_drain(dg_server* s) {
  if (!s) return DG_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->m);
  s->cv_done.wait(lk, [&] { return s->uq.empty() && s->qq.empty() && s->busy == 0; });
  return DG_OK;
}

dg_status dg_server_get_stats(dg_server* s, dg_server_stats* st) {
  if (!s || !st) return DG_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  st->completed = s->n_upd + s->n_qry;
  st->updates = s->n_upd;
  st->queries = s->n_qry;
  st->ops_applied = s->ops_applied;
  st->p50_ms = pct(s->lat_all, 50);
  st->p99_ms = pct(s->lat_all, 99);
  st->p50_query_ms = pct(s->lat_q, 50);
  st->p99_query_ms = pct(s->lat_q, 99);
  st->p50_update_ms = pct(s->lat_u, 50);
  st->p99_update_ms = pct(s->lat_u, 99);
  st->wall_s = s->t_first < 0 ? 0.0 : s->t_last - s->t_first;
  st->edges_traversed = s->arcs;
  return DG_OK;
}

}  // extern "C"
