"""Serving measurement: open-loop Poisson arrivals into the dg serving loop.

Workload: R-MAT scale 22 (4,194,304 vertices, 67.1M sampled directed edges,
int32 weights uniform in [1, 255]) bulk-loaded, then requests at `rate` per
second for `duration` seconds: 30% update batches of log-uniform [1k, 256k]
edge ops (half AddEdge, half RemoveEdge), 70% queries split 40/40/20 between
BFS, SSSP and BC with 16 sources.  Requests are generated before the clock
starts and submitted at their arrival times; the run then drains.

Prints one JSON line per offered rate: offered and achieved request rates,
p50/p99 latency (all, queries, updates; arrival to completion), updates/s,
arcs examined by the queries per second, and whether the offered load was
sustained.  Several rates (--rate 2000,100,25) run one after another on the
same loaded graph, each with its own request stream and server.

Usage: python -m paper_2109_09527_amd.serve_bench [--scale 22] [--rate 2000] [--duration 2] [--lanes 1]
"""
from __future__ import annotations

import argparse
import gc
import json
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--rate", default="2000", help="offered requests/s; a comma-separated list runs each")
    ap.add_argument("--duration", type=float, default=2.0)
    ap.add_argument("--mem-gb", type=float, default=24.0)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--lanes", default="1", help="query lanes (engine launches in flight); a comma-separated list runs each")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rounds", action="store_true",
                    help="BFS and SSSP queries in the lanes' rounds instead of the continuous executors")
    args = ap.parse_args()
    # the drivers are short-lived and make few reference cycles: no collector
    # pause of this interpreter lands inside a timed region
    gc.collect()
    gc.disable()

    import torch
    from paper_2109_09527_amd import dg, synth

    torch.cuda.set_device(0)
    t0 = time.time()
    gr = synth.rmat_graph(args.scale, 16, 255, seed=args.seed)
    g = dg.Graph(gr.n, w_max=255, max_resident_epochs=16, edge_capacity=2 * gr.m)
    g.apply(dg.ops_to_device(synth.load_ops(gr)))
    torch.cuda.synchronize()
    print(f"[serve] loaded V={gr.n} m={gr.m} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    for lanes in (int(x) for x in str(args.lanes).split(",")):
        for k, rate in enumerate(float(x) for x in str(args.rate).split(",")):
            run_rate(args, g, gr, rate, args.seed + k, lanes)


def run_rate(args, g, gr, rate, seed, lanes):
    import torch
    from paper_2109_09527_amd import dg, synth
    reqs = synth.serving_requests(gr, rate=rate, duration=args.duration, seed=seed)
    print(f"[serve] rate {rate:g}/s, {lanes} lanes: {len(reqs)} requests", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    srv = dg.Server(g, mem_budget=int(args.mem_gb * (1 << 30)), max_inflight=1024, max_batch=args.max_batch,
                    query_lanes=lanes, bfs_rounds=args.rounds, sssp_rounds=args.rounds)
    tickets = []
    start = time.perf_counter()
    for r in reqs:
        delay = r.t - (time.perf_counter() - start)
        if delay > 0:
            time.sleep(delay)
        if r.kind == "update":
            tickets.append(("update", srv.submit_update(r.ops), len(r.ops)))
        elif r.kind == "bc":
            tickets.append(("bc", srv.submit_query(dg.Q_BC, r.srcs), 0))
        else:
            tickets.append((r.kind, srv.submit_query(dg.Q_BFS if r.kind == "bfs" else dg.Q_SSSP, [r.src]), 0))
    t_submit = time.perf_counter() - start
    print(f"[serve] submitted {len(tickets)} in {t_submit:.2f}s", file=sys.stderr, flush=True)
    srv.drain()
    t_all = time.perf_counter() - start
    st = srv.stats()
    by_kind = {}
    fails = 0
    for kind, t, _ in tickets:
        done, status, ep, lat = srv.poll(t)
        fails += status != 0
        by_kind.setdefault(kind, []).append(lat)
        srv.take(t, np.zeros(0, np.uint8))
    srv.stop()

    def p(xs, q):
        xs = sorted(xs)
        return round(xs[max(1, int(np.ceil(q / 100 * len(xs)))) - 1], 3) if xs else None

    achieved = len(tickets) / st["wall_s"] if st["wall_s"] else None
    out = {
        "workload": f"R-MAT scale {args.scale} serving: Poisson {rate:g}/s for {args.duration:g}s, 30% updates "
                    "(log-uniform 1k-256k edge ops), 70% queries (BFS 40%, SSSP 40%, BC-16 20%)",
        "query_lanes": lanes, "max_batch": args.max_batch,
        "bfs_sssp": "lanes' rounds" if args.rounds else "continuous executors",
        "joined_running": st["joined_running"],
        "requests": len(tickets), "offered_rps": rate, "achieved_rps": round(achieved, 1) if achieved else None,
        "sustained": bool(achieved and achieved >= 0.95 * rate),
        "wall_s": round(st["wall_s"], 3), "drain_s": round(t_all - t_submit, 3),
        "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
        "query_p50_ms": round(st["p50_query_ms"], 3), "query_p99_ms": round(st["p99_query_ms"], 3),
        "update_p50_ms": round(st["p50_update_ms"], 3), "update_p99_ms": round(st["p99_update_ms"], 3),
        "per_kind_p50_ms": {k: p(v, 50) for k, v in by_kind.items()},
        "per_kind_p99_ms": {k: p(v, 99) for k, v in by_kind.items()},
        "updates_per_s": round(st["ops_applied"] / st["wall_s"], 1) if st["wall_s"] else None,
        "query_arcs_per_s": round(st["edges_traversed"] / st["wall_s"], 1) if st["wall_s"] else None,
        "failed": fails,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
