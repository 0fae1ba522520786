"""Benchmark of the snapshot-query dynamic graph on one MI355X.

Workload (one "step" = one pass of the hot path over one batch):
  R-MAT scale 20 (1,048,576 vertices, 16.8M sampled directed edges with
  a=0.57 b=0.19 c=0.19 d=0.05, repeated keys and self-loops dropped), int32
  weights uniform in [1, 255], bulk-loaded before timing.  Each step applies
  one update batch of 65,536 edge ops (half AddEdge with fresh R-MAT
  endpoints, half RemoveEdge of generated edges) plus 656 vertex ops (half
  AddVertex, half RemoveVertex), shuffled, publishing one epoch; then one
  snapshot BFS and one delta-stepping SSSP from sources drawn among vertices
  with an initial out-arc, on that epoch.

Reported value: snapshot-query GTEPS of the whole job = sum over the
queries of the edges in the traversed component (visible out-degree summed
over reached vertices) / wall time of all timed steps (updates included).
Also: updates/s, query-only GTEPS, p50/p99 latencies, the dominant
kernel's achieved bandwidth against the HBM roofline (HIP events inside
the library, on the stream the kernels run on), and the CPU oracle timed on
a sample of the same steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per visible arc examined, by kernel family:
#   sssp_relax    dst 4 + weight 4 + stamp 8 + dist 4 (atomicMin target)
#   bfs_top_down  dst 4 + stamp 8 + dist 4
#   bfs_bottom_up src 4 + stamp 8 (frontier bit test stays in L2)
BYTES_PER_ARC = {"sssp_relax": 20, "bfs_top_down": 16, "bfs_bottom_up": 12}
METRIC = "snapshot-query GTEPS + updates/s; p50/p99 query latency, batched vs plain"
# HBM bytes per launch measured with rocprofv3 counters, valid only while the
# kernel's sources are unchanged (their digest is stored beside the figure).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sssp_relax_rmat20_traffic.txt")


def measured_traffic(kernel):
    """Per-launch HBM bytes of `kernel` from the committed counter summary,
    or None when there is none or the kernel's sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = next(json.loads(line[5:]) for line in f if line.startswith("json:"))
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("kernel") != kernel or "sources" not in rec:
        return None
    from paper_2109_09527_amd.rocprof_summary import sources_digest
    try:
        if sources_digest([os.path.join(ROOT, p) for p in rec["sources"]]) != rec.get("sources_sha256"):
            return None
    except OSError:
        return None
    return rec["bytes_per_dispatch"]


def pct(xs, p):
    """Nearest-rank percentile."""
    xs = sorted(xs)
    if not xs:
        return None
    k = max(1, int(np.ceil(p / 100.0 * len(xs))))
    return xs[k - 1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle sample size in steps (0 = skip)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (a reference kernel for "
                         "calibrating HBM byte counters)")
    ap.add_argument("--tuning-file", default=None,
                    help="JSON tuning: loaded (and the autotuner skipped) if the file exists, else written "
                         "after autotuning, so a profiled run can replay the tuned configuration")
    ap.add_argument("--batch-queries", type=int, default=128,
                    help="queries of the batched-vs-plain comparison (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the store and its queries run on a single GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2109_09527_amd import dg, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    K, W = args.steps, args.warmup
    n_batches = K + W
    t0 = time.time()
    wl = synth.update_batches(scale=args.scale, n_batches=n_batches, seed=0)
    gr = wl.graph
    print(f"[bench] workload generated in {time.time() - t0:.1f}s: V={gr.n} m={gr.m}", file=sys.stderr, flush=True)

    g = dg.Graph(gr.n, w_max=255, max_resident_epochs=n_batches + 4, edge_capacity=2 * gr.m)
    load = synth.load_ops(gr)
    t0 = time.time()
    dload = dg.ops_to_device(load)
    dres = torch.empty(len(load), dtype=torch.uint8, device="cuda")
    g.apply(dload, dres)
    torch.cuda.synchronize()
    print(f"[bench] bulk load of {len(load)} ops in {time.time() - t0:.2f}s", file=sys.stderr, flush=True)
    del dload, dres

    dbatches = [dg.ops_to_device(b) for b in wl.batches]
    dresults = [torch.empty(len(b), dtype=torch.uint8, device="cuda") for b in wl.batches]
    dist_b = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for _ in range(n_batches)]
    dist_s = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for _ in range(n_batches)]
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    marks = []
    epochs = []

    def step(i):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record()
        _, ep = g.apply(dbatches[i], dresults[i])
        e1.record()
        g.bfs(int(wl.bfs_src[i]), ep, dist_b[i])
        e2.record()
        g.sssp(int(wl.sssp_src[i]), ep, dist_s[i])
        e3.record()
        return ep, (e0, e1, e2, e3)

    if args.tuning_file and os.path.exists(args.tuning_file):
        with open(args.tuning_file) as f:
            g.set_tuning(**json.load(f))
    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    fixed_tuning = bool(args.tuning_file and os.path.exists(args.tuning_file))
    if fixed_tuning:
        tuning = g.get_tuning()
    else:
        tuning = g.autotune(seed=0) if not args.no_autotune else g.get_tuning()
        if args.tuning_file:
            with open(args.tuning_file, "w") as f:
                json.dump(tuning, f)
    print(f"[bench] tuning {tuning}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if not args.no_profile:
        g.profile(True)
        g.profile_read(reset=True)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()   # no collector pause of this interpreter inside a timed region
    t_start = time.perf_counter()
    for i in range(W, W + K):
        ep, m = step(i)
        epochs.append(ep)
        marks.append(m)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    gc.enable()
    prof = g.profile_read(reset=True) if not args.no_profile else {}
    g.profile(False)

    upd_ms = [a.elapsed_time(b) for a, b, _, _ in marks]
    bfs_ms = [b.elapsed_time(c) for _, b, c, _ in marks]
    sssp_ms = [c.elapsed_time(d) for _, _, c, d in marks]

    # TEPS numerators: visible out-degree summed over reached vertices
    m_bfs, m_sssp = [], []
    for j, i in enumerate(range(W, W + K)):
        deg = g.out_degrees(epochs[j]).to(torch.int64)
        m_bfs.append(int(deg[dist_b[i] >= 0].sum().item()))
        m_sssp.append(int(deg[dist_s[i] >= 0].sum().item()))
    m_total = sum(m_bfs) + sum(m_sssp)
    n_ops = sum(len(wl.batches[i]) for i in range(W, W + K))
    value = m_total / t_total / 1e9
    q_time = (sum(bfs_ms) + sum(sssp_ms)) / 1e3

    roof = None
    if prof:
        cands = [(v["total_ms"], k) for k, v in prof.items() if k in BYTES_PER_ARC]
        if cands:
            _, kname = max(cands)
            kp = prof[kname]
            avg_ms = kp["total_ms"] / kp["launches"]
            bytes_per_launch = kp["arcs"] * BYTES_PER_ARC[kname] / kp["launches"]
            achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
            traffic = measured_traffic("k_" + kname)
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                    "avg_launch_us": round(avg_ms * 1e3, 2), "launches": kp["launches"],
                    "bytes_per_launch": int(bytes_per_launch)}

    batched = None
    if args.batch_queries > 0:
        batched = batched_vs_plain(g, wl, epochs, args.batch_queries)

    cpu = None
    if args.cpu_steps > 0:
        cpu = cpu_baseline(wl, W, min(args.cpu_steps, K), m_bfs, m_sssp, dist_b, dist_s)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(t_total / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"R-MAT scale {args.scale} dynamic graph: per step one batch of 65,536 edge add/remove "
                        f"(50/50) + 656 vertex add/remove, then one snapshot BFS and one delta-stepping SSSP",
            "vertices": gr.n, "loaded_edges": gr.m, "weights": "int32 U[1,255]",
            "ops_per_batch": len(wl.batches[0]), "parallelism": "single GPU", "tuning": tuning,
        },
        "updates_per_s": round(n_ops / (sum(upd_ms) / 1e3), 1),
        "query_gteps": round(m_total / q_time / 1e9, 4),
        "latency_ms": {
            "update_p50": round(pct(upd_ms, 50), 3), "update_p99": round(pct(upd_ms, 99), 3),
            "bfs_p50": round(pct(bfs_ms, 50), 3), "bfs_p99": round(pct(bfs_ms, 99), 3),
            "sssp_p50": round(pct(sssp_ms, 50), 3), "sssp_p99": round(pct(sssp_ms, 99), 3),
        },
        "kernels": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3), "arcs": v["arcs"]}
                    for k, v in prof.items()},
        "roofline": roof,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.copy_mib > 0:
        n = args.copy_mib << 18   # int32 elements
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copied {args.copy_mib} MiB device to device", file=sys.stderr, flush=True)


def kernel_roof(prof, name, bytes_per_arc):
    kp = prof.get(name)
    if not kp or not kp["launches"] or kp["total_ms"] <= 0:
        return None
    achieved = kp["arcs"] * bytes_per_arc / (kp["total_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": name,
            "avg_launch_us": round(kp["total_ms"] / kp["launches"] * 1e3, 2), "launches": kp["launches"],
            "bytes_per_launch": int(kp["arcs"] * bytes_per_arc / kp["launches"])}


def batched_vs_plain(g, wl, epochs, nq):
    """nq BFS/SSSP queries (alternating) over the last 8 retained epochs:
    one dg_query_batch launch versus one plain call per query.  Outputs of
    the two forms are compared element by element."""
    import torch
    from paper_2109_09527_amd import dg
    n = g.n
    eps = epochs[-8:]
    srcs = np.concatenate([wl.bfs_src, wl.sssp_src])
    qs = [(dg.Q_BFS if i % 2 == 0 else dg.Q_SSSP, eps[i % len(eps)], int(srcs[(i * 7) % len(srcs)]))
          for i in range(nq)]
    plain = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in qs]
    batch = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in qs]
    # warm-up of both forms; the engine's warm-up runs the whole batch, so
    # its scratch (sized by the batch) is allocated before the clock starts
    g.query_batch([(k, e, s, o) for (k, e, s), o in zip(qs, batch)])
    for (k, e, s), o in zip(qs[:2], plain[:2]):
        (g.bfs if k == dg.Q_BFS else g.sssp)(s, e, o)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    lat = []
    t0 = time.perf_counter()
    for (k, e, s), o in zip(qs, plain):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        (g.bfs if k == dg.Q_BFS else g.sssp)(s, e, o)
        b.record()
        lat.append((a, b))
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain_ms = [a.elapsed_time(b) for a, b in lat]
    g.profile(True)
    g.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.query_batch([(k, e, s, o) for (k, e, s), o in zip(qs, batch)])
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    gc.enable()
    prof = g.profile_read(reset=True)
    g.profile(False)
    same = all(x == 0 for x in st) and all(torch.equal(a, b) for a, b in zip(plain, batch))
    degs = {e: g.out_degrees(e).to(torch.int64) for e in set(eps)}
    m = sum(int(degs[e][o >= 0].sum().item()) for (k, e, s), o in zip(qs, batch))
    roof = {k: kernel_roof(prof, f"batch_{k}", BYTES_PER_ARC["sssp_relax" if k == "sssp" else "bfs_top_down"])
            for k in ("bfs", "sssp")}
    return {"queries": nq, "epochs": len(set(eps)), "plain_s": round(t_plain, 4), "batched_s": round(t_batch, 4),
            "plain_gteps": round(m / t_plain / 1e9, 4), "batched_gteps": round(m / t_batch / 1e9, 4),
            "speedup": round(t_plain / t_batch, 2),
            "plain_latency_ms": {"p50": round(pct(plain_ms, 50), 3), "p99": round(pct(plain_ms, 99), 3)},
            "batched_latency_ms": {"p50": round(t_batch * 1e3, 3), "p99": round(t_batch * 1e3, 3)},
            "outputs_equal": same,
            "kernels": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3), "arcs": v["arcs"]}
                        for k, v in prof.items()},
            "roofline": roof}


def cpu_baseline(wl, W, S, m_bfs, m_sssp, dist_b, dist_s):
    """The sequential oracle on the host: load and the W warm-up batches
    untimed, then S steps (batch + BFS + SSSP) timed with the same metric.
    Its outputs are also compared with the GPU's for those steps."""
    from oracle import Oracle
    gr = wl.graph
    o = Oracle(gr.n, w_max=255)
    t0 = time.time()
    o.apply(synth_load(gr))
    for i in range(W):
        o.apply(wl.batches[i])
    print(f"[bench] oracle setup {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    same = True
    t = 0.0
    for j in range(S):
        i = W + j
        t1 = time.perf_counter()
        o.apply(wl.batches[i])
        _, db = o.bfs(int(wl.bfs_src[i]))
        _, ds = o.sssp(int(wl.sssp_src[i]))
        t += time.perf_counter() - t1
        same &= bool(np.array_equal(db, dist_b[i].cpu().numpy()) and np.array_equal(ds, dist_s[i].cpu().numpy()))
    m = sum(m_bfs[:S]) + sum(m_sssp[:S])
    return {"value": round(m / t / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{S} steps (batch + BFS + SSSP) of the same workload after the bulk load and warm-up "
                      f"batches; single-threaded C on {platform.processor() or platform.machine()}",
            "seconds": round(t, 2), "matches_gpu": same}


def synth_load(gr):
    from paper_2109_09527_amd import synth
    return synth.load_ops(gr)


if __name__ == "__main__":
    main()
