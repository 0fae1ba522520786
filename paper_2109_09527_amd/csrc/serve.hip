// Serving loop: continuous batching of update batches and snapshot queries
// over one graph.
//
//   update thread  applies update requests in arrival order on its own
//                  stream; each publishes the next epoch.
//   executors      one for BFS (64 slots) and one for SSSP (32 slots), each
//                  a multi-source search that runs pass after pass on its
//                  own stream while any slot is active; before every pass,
//                  waiting queries of its kind take the free slots, each
//                  bound to the latest published epoch at that moment (its
//                  linearization point), and join the running search.  A
//                  finished slot's output is copied to the host by a copy
//                  thread, after which the slot is reused.
//   query lanes    (query_lanes threads, each with a stream and an engine
//                  instance of its own) each take, whenever it is free, the
//                  waiting BC queries at the head of the queue in arrival
//                  order while their output memory fits the budget and the
//                  in-flight cap allows (up to max_batch at once), bind them
//                  to the latest published epoch and run them in one engine
//                  call.  A query arriving while a lane is busy is taken by
//                  the next lane to come free, so the launches of the lanes,
//                  the executors and the update stream overlap on the
//                  device.  (With bfs_rounds or sssp_rounds set, queries of
//                  that kind go to the lanes too.)
// While a server runs, scans read per-slot stamps (no summary fast path),
// since update kernels may write slabs under running queries, and the
// engine launches share part of the device's resident-workgroup capacity
// (the rest stays free for the update kernels).  Latency = completion -
// submission, host clock.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "dg_host.h"
#include "xexec.h"

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
  // the continuous executors (BFS and SSSP): waiting queries, slots whose
  // output is being copied, and each one's thread, stream and event
  struct ExecQ {
    int kind;
    uint32_t nslots;
    std::deque<Req*> q;
    unsigned long long draining = 0;
    hipStream_t s = nullptr;
    // SSSP: per slot, its output extracted up to here (one event per slot, so
    // no event is recorded again while the copy thread may wait on it)
    std::vector<hipEvent_t> ready;
    std::thread t;
    uint64_t joined_running = 0;      // admitted while others of the search were running
  };
  ExecQ xb{DG_Q_BFS, dg::XB_SLOTS}, xs{DG_Q_SSSP, dg::XS_SLOTS};
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
  // a thread that copies finished executor outputs to the host, so that
  // the executors' passes keep running
  std::thread tc;
  hipStream_t sc = nullptr;
  struct Done {
    Req* r;
    ExecQ* x;
    uint32_t slot;
    const void* dev;
    uint32_t epoch;
    hipEvent_t ready;   // the output is final once this event completes (null: already)
  };
  std::deque<Done> copies;
  std::condition_variable cv_copy;
  bool copy_stop = false;
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
      g->update_running.store(1);
      dg_status st = dg_apply_batch(g, r->ops.data(), r->ops.size(), r->results.data(), &ep, su);
      g->update_running.store(0);
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

  // ---- continuous executors (BFS, SSSP)
  //
  // One multi-source search of up to 64 (BFS) or 32 (SSSP) slots runs pass
  // after pass while any slot is active.  Before each pass, waiting queries
  // of the executor's kind take free slots (arrival order, within the memory
  // budget and the in-flight cap), each bound to the latest published epoch
  // at that moment; their sources join the pass.  A slot that made no
  // progress in a pass is finished: its output goes to the copy thread, and
  // its slot is reused once the copy is done (its state is reset when the
  // next query takes it).
  struct XSlot {
    Req* r = nullptr;
    uint32_t epoch = 0;
    bool pinned = false;
    dg::DevBuf out;
    int32_t start = 0;
  };

  void exec_loop(ExecQ& X) {
    const bool bfs = X.kind == DG_Q_BFS;
    dg::XbState* xbs = bfs ? dg::xb_create() : nullptr;
    dg::XsState* xss = bfs ? nullptr : dg::xs_create();
    const unsigned long long all_slots = X.nslots >= 64 ? ~0ull : ((1ull << X.nslots) - 1);
    std::vector<XSlot> slot(X.nslots);
    unsigned long long active = 0, dirty = 0;
    int32_t pass = 0;
    const uint64_t V = g->cfg.v_capacity;
    const uint32_t share = std::max<uint32_t>(1, g->engine_share_pct);
    bool held = false;   // this search's hold (compaction waits while it is held)
    auto hold = [&](bool on) {
      std::unique_lock<std::mutex> lk(g->mu);
      if (on) {
        g->pool_cv.wait(lk, [&] { return g->compact_waiting.load() == 0; });
        g->search_holds++;
      } else {
        g->search_holds--;
        g->pool_cv.notify_all();
      }
      held = on;
    };
    auto free_slots = [&] { return all_slots & ~(active | X.draining); };
    for (;;) {
      std::vector<uint32_t> joined;
      if (!active) {
        if (held) hold(false);
        pass = 0;   // BFS levels count from each slot's start, so the pass number may restart
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] {
          return (stop && X.q.empty() && !X.draining) ||
                 (!X.q.empty() && free_slots() != 0 && q_running < cfg.max_inflight &&
                  mem_used + out_bytes(X.q.front()) <= cfg.mem_budget);
        });
        if (X.q.empty() && stop && !X.draining) break;
      }
      if (!held) hold(true);
      {
        std::unique_lock<std::mutex> lk(m);
        // no admission while a compaction waits: the search drains first
        auto admissible = [&] {
          return !X.q.empty() && free_slots() != 0 && q_running < cfg.max_inflight &&
                 mem_used + out_bytes(X.q.front()) <= cfg.mem_budget && g->compact_waiting.load() == 0;
        };
        const bool others = active != 0;
        while (admissible()) {
          Req* r = X.q.front();
          const uint64_t need = out_bytes(r);
          X.q.pop_front();
          mem_used += need;
          r->reserve = need;
          busy++;
          q_running++;
          const uint32_t b = (uint32_t)__builtin_ctzll(free_slots());
          slot[b].r = r;
          active |= 1ull << b;
          joined.push_back(b);
          if (others) X.joined_running++;
        }
      }
      dg::XbSeeds seeds{};
      unsigned long long clear = 0;
      for (uint32_t b : joined) {
        XSlot& sl = slot[b];
        dg_epoch e = 0;
        sl.pinned = dg_snapshot_acquire(g, DG_EPOCH_LATEST, &e) == DG_OK;
        sl.epoch = e;
        const uint32_t src = sl.r->srcs[0];
        dg_status st = DG_OK;
        if (src >= V) {
          st = DG_E_VERTEX_RANGE;
        } else {
          std::lock_guard<std::mutex> lk(g->mu);
          if (!dg::alive_at(g, src, e)) st = DG_E_SOURCE_ABSENT;
        }
        if (st == DG_OK && dg::ensure(sl.out, V * 4) != hipSuccess) st = DG_E_OUT_OF_MEMORY;
        // a BFS writes levels as it goes; an SSSP output is written whole at the end
        if (st == DG_OK && bfs && dg::fill_i32(sl.out.as<int32_t>(), V, -1, X.s) != hipSuccess) st = DG_E_HIP;
        if (st != DG_OK) {
          if (sl.pinned) dg_snapshot_release(g, e);
          sl.pinned = false;
          active &= ~(1ull << b);
          Req* r = sl.r;
          sl.r = nullptr;
          finish(r, st, e);
          continue;
        }
        sl.start = pass;
        seeds.slot[seeds.n] = b;
        seeds.src[seeds.n] = src;
        seeds.n++;
        if (dirty >> b & 1ull) clear |= 1ull << b;
      }
      dirty &= ~clear;
      if (!active) continue;
      // the active slots' epochs, ascending, with their cumulative masks
      dg::XbEpochs ep{};
      dg::XbOuts outs{};
      {
        std::vector<std::pair<uint32_t, uint32_t>> es;
        for (uint32_t b = 0; b < X.nslots; b++)
          if (active >> b & 1ull) {
            es.push_back({slot[b].epoch, b});
            outs.out[b] = slot[b].out.as<int32_t>();
            outs.start[b] = slot[b].start;
          }
        std::sort(es.begin(), es.end());
        unsigned long long cum = 0;
        for (size_t i = 0; i < es.size(); i++) {
          if (i == 0 || es[i].first != es[i - 1].first) {
            ep.cm[ep.ne] = cum;
            ep.ue[ep.ne++] = es[i].first;
          }
          cum |= 1ull << es[i].second;
        }
        ep.cm[ep.ne] = cum;
        for (uint32_t i = ep.ne; i < dg::XB_SLOTS; i++) {
          ep.ue[i] = 0xFFFFFFFFu;
          ep.cm[i + 1] = cum;
        }
      }
      // updates go first: wait (up to a few ms) for a running batch
      dg::yield_to_updates(g);
      dg::Store st;
      {
        std::unique_lock<std::mutex> lk(g->mu);
        dg::pool_read_begin(g, lk);
        st = g->st;
      }
      dg::XbResult res{};
      hipError_t he = bfs ? dg::xb_pass(xbs, g, st, X.s, share, pass, ep, outs, seeds, clear, &res)
                          : dg::xs_pass(xss, g, st, X.s, share, ep, seeds, clear, &res);
      dg::pool_read_end(g);
      pass++;
      const unsigned long long done = he == hipSuccess && !res.overflow ? active & ~res.progress : 0ull;
      if (done && !bfs) {
        he = dg::xs_extract(xss, outs, done, X.s, nullptr);
        for (uint32_t b = 0; he == hipSuccess && b < X.nslots; b++)
          if (done >> b & 1ull) he = hipEventRecord(X.ready[b], X.s);
      }
      if (he != hipSuccess || res.overflow) {
        // the search state is lost: fail its queries and start afresh
        for (uint32_t b = 0; b < X.nslots; b++)
          if (active >> b & 1ull) {
            if (slot[b].pinned) dg_snapshot_release(g, slot[b].epoch);
            slot[b].pinned = false;
            Req* r = slot[b].r;
            slot[b].r = nullptr;
            finish(r, he != hipSuccess ? DG_E_HIP : DG_E_OUT_OF_MEMORY, slot[b].epoch);
          }
        active = 0;
        dirty = 0;
        (void)hipStreamSynchronize(X.s);
        if (bfs) {
          dg::xb_destroy(xbs);
          xbs = dg::xb_create();
        } else {
          dg::xs_destroy(xss);
          xss = dg::xs_create();
        }
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(m);
        arcs += res.arcs;
      }
      if (done) {
        std::lock_guard<std::mutex> lk(m);
        for (uint32_t b = 0; b < X.nslots; b++)
          if (done >> b & 1ull) {
            if (slot[b].pinned) dg_snapshot_release(g, slot[b].epoch);
            slot[b].pinned = false;
            copies.push_back(Done{slot[b].r, &X, b, slot[b].out.p, slot[b].epoch, bfs ? nullptr : X.ready[b]});
            slot[b].r = nullptr;
          }
        active &= ~done;
        dirty |= done;
        X.draining |= done;
        cv_copy.notify_all();
      }
    }
    if (held) hold(false);
    for (auto& sl : slot) dg::release(sl.out);
    if (xbs) dg::xb_destroy(xbs);
    if (xss) dg::xs_destroy(xss);
  }

  // Copies finished executor outputs to the host, then frees their slots.
  // Each output goes by DMA into pinned staging, then into the request.
  void copy_loop() {
    const uint64_t bytes = g->cfg.v_capacity * 4;
    void* stage = nullptr;
    if (hipHostMalloc(&stage, bytes, hipHostMallocDefault) != hipSuccess) stage = nullptr;
    for (;;) {
      Done d;
      {
        std::unique_lock<std::mutex> lk(m);
        cv_copy.wait(lk, [&] { return copy_stop || !copies.empty(); });
        if (copies.empty()) {
          if (stage) hipHostFree(stage);
          return;
        }
        d = copies.front();
        copies.pop_front();
      }
      dg_status st = DG_OK;
      d.r->out.resize(bytes);
      void* dst = stage ? stage : (void*)d.r->out.data();
      if ((d.ready && hipStreamWaitEvent(sc, d.ready, 0) != hipSuccess) ||
          hipMemcpyAsync(dst, d.dev, bytes, hipMemcpyDeviceToHost, sc) != hipSuccess ||
          hipStreamSynchronize(sc) != hipSuccess)
        st = DG_E_HIP;
      else if (stage)
        std::memcpy(d.r->out.data(), stage, bytes);
      finish(d.r, st, d.epoch);
      {
        std::lock_guard<std::mutex> lk(m);
        d.x->draining &= ~(1ull << d.slot);
      }
      cv.notify_all();
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
  bool ok = hipStreamCreateWithFlags(&s->su, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&s->sc, hipStreamNonBlocking) == hipSuccess;
  for (dg_server::ExecQ* x : {&s->xb, &s->xs}) {
    const bool on = x->kind == DG_Q_BFS ? !s->cfg.bfs_rounds : !s->cfg.sssp_rounds;
    if (ok && on) ok = hipStreamCreateWithFlags(&x->s, hipStreamNonBlocking) == hipSuccess;
    if (ok && on && x->kind == DG_Q_SSSP) {
      x->ready.assign(x->nslots, nullptr);
      for (hipEvent_t& ev : x->ready)
        if (ok) ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    }
  }
  for (uint32_t i = 0; ok && i < s->cfg.query_lanes; i++) {
    hipStream_t x = nullptr;
    ok = hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess;
    if (ok) s->sq.push_back(x);
  }
  if (!ok) {
    if (s->su) hipStreamDestroy(s->su);
    if (s->sc) hipStreamDestroy(s->sc);
    for (dg_server::ExecQ* x : {&s->xb, &s->xs}) {
      if (x->s) hipStreamDestroy(x->s);
      for (hipEvent_t ev : x->ready)
        if (ev) hipEventDestroy(ev);
    }
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
  for (dg_server::ExecQ* x : {&s->xb, &s->xs})
    if (x->s) x->t = std::thread([s, x] { s->exec_loop(*x); });
  if (s->xb.s || s->xs.s) s->tc = std::thread([s] { s->copy_loop(); });
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
  for (dg_server::ExecQ* x : {&s->xb, &s->xs})
    if (x->t.joinable()) x->t.join();
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->copy_stop = true;
  }
  s->cv_copy.notify_all();
  if (s->tc.joinable()) s->tc.join();
  hipStreamSynchronize(s->sc);
  hipStreamDestroy(s->sc);
  for (dg_server::ExecQ* x : {&s->xb, &s->xs}) {
    if (x->s) {
      hipStreamSynchronize(x->s);
      hipStreamDestroy(x->s);
    }
    for (hipEvent_t ev : x->ready)
      if (ev) hipEventDestroy(ev);
  }
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
  if (raw->kind < 0) s->uq.push_back(raw);
  else if (raw->kind == DG_Q_BFS && s->xb.s) s->xb.q.push_back(raw);
  else if (raw->kind == DG_Q_SSSP && s->xs.s) s->xs.q.push_back(raw);
  else s->qq.push_back(raw);
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
  s->cv_done.wait(lk, [&] { return s->uq.empty() && s->qq.empty() && s->xb.q.empty() && s->xs.q.empty() && s->busy == 0; });
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
  st->joined_running = s->xb.joined_running + s->xs.joined_running;
  return DG_OK;
}

}  // extern "C"
