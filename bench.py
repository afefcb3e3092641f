#!/usr/bin/env python3
"""Benchmark: top-k weighted triangle queries on one MI355X.

One step = one pass of the whole hot path over the resident edge list of the workload:
  1. graph_load from device-resident src/dst/w (validation + degree-oriented CSR build);
  2. exact top-k queries (topk_triangles) at each p of the workload;
  3. weighted edge sampling queries (sample_heavy_triangles) at the same p's (workloads with a
     sampling budget);
  4. graph_free.
`value` is queries per second over the timed steps (all queries of a step / step time).

Default workload ("large"): Chung-Lu n=100M, ~2B edges, gamma 2.0, Zipf(s=1.5) weights on
[1, 1e6], seed 0; top-1000 at p = 1 and p = +inf, the CSR built cold in every step (queries
on the resident CSR are reported beside it).  "medium" (n=1M, ~20M edges, 50 planted heavy
4-cliques, four p, sampling 1e7 draws), "small", "batch" and "serve" are the other workloads.

The JSON line also carries:
  roofline       : the enumeration pass (k_enum: filter + intersect kernels of one band),
                   algorithmic bytes per pass / its mean duration measured with HIP events on
                   the graph's stream; bytes per unit: 6 per streamed entry (its weight and the
                   amortised row-maximum gathers), 20 per candidate entry (two row extents and
                   its weight), 8 per intersected adjacency entry, 8 per triangle found;
                   `traffic` is the counter-measured HBM bytes per pass from profiles/;
  build_roofline : the cold CSR build, 20 bytes per edge (12 read, 8 written) / its duration;
  cpu_baseline   : the CPU oracle (plain enumeration + per-thread heaps) timed on this host's
                   cores; on the 2B-edge graph time-boxed on the whole graph, with a
                   vertex-sample extrapolation and a one-thread time beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "top-k triangle queries/sec + intersected edges/sec (HBM GB/s %); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of the enumeration pass, per unit: a streaming pass reads each entry's
# weight (4 B) plus the row maxima it is compared with, gathered once per row and amortised
# over the row (<= 2 B per entry: 8-12 GB for a 2B-entry pass); a candidate reads its two row
# extents and its weight (20 B); an intersected adjacency entry its head and weight (8 B); a
# triangle found the two other weights (8 B)
B_STREAM = 6
B_CAND = 20
B_INTER = 8
B_EMIT = 8
B_BUILD = 20    # cold CSR build, per edge: 12 B read (src, dst, w) + 8 B written (col, wgt)

WORKLOADS = {
    "medium": dict(gen="medium", k=1000, ps=(-math.inf, 1.0, 2.0, math.inf), budget=10_000_000,
                   desc="chung-lu n=1M m~20M gamma2.1 zipf(1.8)[1,1e6] +50 planted K4 x1000 seed0; "
                        "top-1000 exact + edge sampling 1e7 draws at p in {-inf,1,2,+inf}"),
    "small": dict(gen="small", k=100, ps=(1.0,), budget=100_000,
                  desc="chung-lu n=2000 m~20k gamma2.5 zipf(2)[1,1e6] seed0; top-100 exact + edge sampling 1e5 at p=1"),
    "large": dict(gen="large", k=1000, ps=(1.0, math.inf), budget=0, cpu_timebox=60.0,
                  desc="chung-lu n=100M m~2B gamma2.0 zipf(1.5)[1,1e6] seed0; top-1000 exact at p in {1,+inf}, "
                       "cold (CSR built in the step) and warm"),
}


def recorded_traffic(workload):
    """HBM bytes per enumeration pass from the counter runs summarised in profiles/, or None if
    they were taken on another workload or the enumeration sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_enum_{workload}_traffic.md")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
    except OSError:
        return None
    h = hashlib.sha256()
    for f in ("enum.h", "query.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_1910_00692_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("workload") != workload or fields.get("sources_sha256_16") != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_pass"])


def single_breakdown(reqs, ms, res):
    """Where the single-query path spends its time: per p and for subset requests, the count,
    the mean wall time and the mean device time of the passes and the selection."""
    groups = {}
    fields = ("passes", "edges_streamed", "candidate_edges", "intersected_entries", "restarts", "bound_order")
    for r, t, x in zip(reqs, ms, res):
        key = "subset" if r["subset"] is not None else f"p={r['p']}"
        st = x["stats"]
        g = groups.setdefault(key, {"n": 0, "ms": 0.0, "device_ms": 0.0, **{f: 0.0 for f in fields}})
        g["n"] += 1
        g["ms"] += t
        g["device_ms"] += st["enum_kernel_ms"] + st["select_ms"]
        for f in fields:
            g[f] += st[f]
    return {k: {"n": g["n"], "mean_ms": g["ms"] / g["n"], "mean_device_ms": g["device_ms"] / g["n"],
                **{"mean_" + f: g[f] / g["n"] for f in fields}} for k, g in sorted(groups.items())}


def run_methods(args):
    """The paper's other methods on the 1M-vertex workload (top-1000 at p = 1): edge sampling
    (Alg. 3), wedge and path sampling (Algs. 4, 5) at growing budgets, static heavy-light (Alg. 1)
    at growing heavy fractions, each timed on the GPU with the fraction of the exact top-k it
    returns; DHL and Auto-HL (Alg. 2) on the host; and the clique extension (Sec. 4.5) on a
    30K-vertex graph with planted 5-cliques, sampled against its exact top cliques."""
    import torch
    import graphgen
    import paper_1910_00692_amd as tt
    from paper_1910_00692_amd import dhl

    torch.cuda.init()
    k, p = 1000, 1.0
    g = graphgen.medium()
    G = tt.Graph(g.n, g.src, g.dst, g.w)

    def timed(fn, reps=3):
        fn()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        return (time.perf_counter() - t) * 1e3 / reps, r

    def tri_set(r):
        return set(zip(r["i"].tolist(), r["j"].tolist(), r["l"].tolist()))

    ms_exact, exact = timed(lambda: G.topk(k, p))
    ref = tri_set(exact)

    def acc(r):
        return len(tri_set(r) & ref) / len(ref)

    out = {"metric": "paper's methods: time and fraction of the exact top-k found", "unit": "ms", "n_gpus": 1,
           "data": "synthetic", "higher_is_better": False,
           "config": {"workload": "chung-lu n=1M m~20M gamma2.1 zipf(1.8) +50 planted K4 x1000 seed0; top-1000 at p=1",
                      "n": g.n, "m": g.m, "k": k, "p": p},
           "exact_gpu_ms": ms_exact, "edge_sampling": [], "wedge_sampling": [], "path_sampling": [], "shl": []}
    for budget in (100_000, 1_000_000, 10_000_000):
        ms, r = timed(lambda: G.sample(k, p, budget, seed=5))
        out["edge_sampling"].append({"budget": budget, "ms": ms, "accuracy": acc(r)})
        for scheme in ("wedge", "path"):
            ms, r = timed(lambda: G.sample_by(scheme, k, p, budget, seed=5))
            out[scheme + "_sampling"].append({"budget": budget, "ms": ms, "accuracy": acc(r),
                                              "distinct_triangles": r["distinct"]})
        print(f"[bench] samplers at budget {budget} done", file=sys.stderr, flush=True)
    wsorted = np.sort(g.w)[::-1]
    for f in (0.001, 0.01, 0.1, 0.5):
        tau = int(wsorted[max(int(f * len(wsorted)) - 1, 0)]) - 1
        ms, r = timed(lambda: G.shl(k, p, tau))
        out["shl"].append({"heavy_fraction": f, "tau": tau, "heavy_edges": r["heavy_edges"], "ms": ms,
                           "accuracy": acc(r)})
    G.close()
    nthreads = min(16, os.cpu_count() or 1)
    out["dhl_cpu"] = {}
    for name, alpha in (("dhl_alpha_1.25", 1.25), ("auto_hl", 0.0)):
        t = time.perf_counter()
        r = dhl.topk(g.n, g.src, g.dst, g.w, k, p, alpha, threads=nthreads)
        out["dhl_cpu"][name] = {"ms": (time.perf_counter() - t) * 1e3, "threads": nthreads,
                                "equals_gpu_exact": bool(np.array_equal(r["i"], exact["i"]) and
                                                         np.array_equal(r["j"], exact["j"]) and
                                                         np.array_equal(r["l"], exact["l"]) and
                                                         np.array_equal(r["score"], exact["score"]))}
    print("[bench] dhl done", file=sys.stderr, flush=True)
    h = graphgen.chung_lu(5000, 60000, 2.5, 1.8, seed=51, plant=6, plant_size=5, plant_mult=1000)
    H = tt.Graph(h.n, h.src, h.dst, h.w)
    out["cliques"] = {"graph": "chung-lu n=5K m~60K gamma2.5 zipf(1.8) +6 planted K5 x1000 seed51",
                      "size": 5, "k": 20, "p": p, "runs": []}
    try:
        ms, ex = timed(lambda: H.cliques(5, 20, p, all_edges=True))
        cref = set(map(tuple, ex["v"].tolist()))
        out["cliques"]["exact_ms"] = ms
        for budget in (1_000, 10_000, 100_000):
            ms, r = timed(lambda: H.cliques(5, 20, p, budget=budget, seed=9))
            got = set(map(tuple, r["v"].tolist()))
            out["cliques"]["runs"].append({"budget": budget, "ms": ms,
                                           "accuracy": len(got & cref) / max(len(cref), 1)})
    except tt.TopKError as e:  # more common neighbours than the clique kernel holds
        out["cliques"]["error"] = str(e)
    H.close()
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Served workload: a resident n=10M, ~200M-edge graph and a Poisson request stream (mean
    2,000 req/s; k log-uniform in [10, 1e4]; p from {-inf, -1, 0, 1, 2, +inf}; 20% restricted
    to triangles touching 1,000 random vertices), submitted at its arrival times to the
    continuous-batching server; compared with the same requests run one at a time."""
    import threading
    # two hardware queues per server slot, so the slots' streams share no queue with each other or
    # with the runtime's own copies (HIP reads this when the runtime starts, i.e. before torch
    # touches the GPU; the default is 4)
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues or min(32, max(4, 2 * args.slots)))
    import torch
    import graphgen
    import paper_1910_00692_amd as tt

    t = time.time()
    g = graphgen.serve_graph(n=args.serve_n, m=args.serve_m)
    print(f"[bench] serve graph n={g.n} m={g.m} ({time.time() - t:.1f}s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    s_d = torch.from_numpy(g.src.view(np.int32)).to(dev)
    d_d = torch.from_numpy(g.dst.view(np.int32)).to(dev)
    w_d = torch.from_numpy(g.w.view(np.int32)).to(dev)
    t = time.perf_counter()
    G = tt.Graph(g.n, s_d, d_d, w_d, stream=torch.cuda.current_stream(dev))
    build_ms = (time.perf_counter() - t) * 1e3
    del s_d, d_d, w_d
    reqs = graphgen.query_stream(args.requests, g.n, seed=1)
    print(f"[bench] built in {build_ms:.0f} ms; {len(reqs)} requests", file=sys.stderr, flush=True)
    # plain single-query path, one request after the other (service time only)
    for r in reqs[:8]:
        G.topk(r["k"], r["p"], subset=r["subset"])
    single = []
    single_res = []
    t0 = time.perf_counter()
    for r in reqs:
        a = time.perf_counter()
        single_res.append(G.topk(r["k"], r["p"], subset=r["subset"], with_stats=True))
        single.append((time.perf_counter() - a) * 1e3)
    single_s = time.perf_counter() - t0
    print(f"[bench] single-query path: {len(reqs) / single_s:.1f} req/s", file=sys.stderr, flush=True)
    S = tt.Server(G, slots=args.slots, scratch_budget=args.budget_gb << 30)
    for r in reqs[:8]:
        S.wait(S.submit(r["k"], r["p"], r["subset"]))
    tickets = [None] * len(reqs)
    lat = [None] * len(reqs)
    done_t = [None] * len(reqs)
    served_res = [None] * len(reqs)
    ready = threading.Semaphore(0)

    def waiter():
        for i in range(len(reqs)):
            ready.acquire()
            res = S.wait(tickets[i])
            lat[i] = res["stats"]["total_ms"]
            done_t[i] = time.perf_counter()
            served_res[i] = res

    th = threading.Thread(target=waiter)
    th.start()
    start = time.perf_counter()
    for i, r in enumerate(reqs):
        now = time.perf_counter() - start
        if r["t"] > now:
            time.sleep(r["t"] - now)
        tickets[i] = S.submit(r["k"], r["p"], r["subset"])
        ready.release()
    th.join()
    span = max(done_t) - start
    # every served result must be the single-query result of the same request (same scores in
    # the same order; the triangles themselves where no tie sits at the k-th score)
    mismatched = 0
    for a, b in zip(single_res, served_res):
        same = a["n_out"] == b["n_out"] and np.array_equal(a["score"], b["score"])
        if same:
            untied = a["score"] != a["score"][-1] if a["n_out"] else np.zeros(0, bool)
            for f in ("i", "j", "l"):
                same = same and np.array_equal(a[f][untied], b[f][untied])
        mismatched += not same
    info = S.info()
    S.close()
    G.close()
    out = {
        "metric": METRIC, "value": len(reqs) / span, "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": span * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "served: chung-lu n=10M m~200M gamma2.1 zipf(1.8); Poisson 2000 req/s, k log-uniform "
                               "[10,1e4], p in {-inf,-1,0,1,2,+inf}, 20% subset(1000) queries",
                   "n": g.n, "m": g.m, "requests": len(reqs), "slots": args.slots, "budget_gb": args.budget_gb,
                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat)},
        "single_query_path": {"queries_per_s": len(reqs) / single_s, "p50_ms": pct(single, 50),
                              "p99_ms": pct(single, 99)},
        "offered_rate": len(reqs) / max(reqs[-1]["t"], 1e-9), "server": info, "build_ms": build_ms,
        "gpu_matches_single": mismatched == 0, "mismatched_requests": mismatched,
        "single_by_kind": single_breakdown(reqs, single, single_res),
    }
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Batched workload: 4,096 independent Chung-Lu graphs (n log-uniform in [50, 20000], mean
    degree uniform in [4, 40], gamma 2.5, Zipf(2) weights), top-10 of every graph at p = 1, all
    graphs answered by one replay of the captured launch sequence (autotuned on first use).
    `value` = graphs answered per second; the same graphs queried one at a time through the
    single-graph path are reported beside it."""
    import torch
    import graphgen
    import paper_1910_00692_amd as tt

    t = time.time()
    gs = graphgen.batch(count=args.batch_count)
    total_m = sum(g.m for g in gs)
    print(f"[bench] batch of {len(gs)} graphs, m={total_m} ({time.time() - t:.1f}s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    ns = np.array([g.n for g in gs], np.uint32)
    ms = np.array([g.m for g in gs], np.uint64)
    cat = [np.concatenate([getattr(g, x) for g in gs]) for x in ("src", "dst", "w")]
    src, dst, w = (torch.from_numpy(c.view(np.int32)).to(dev) for c in cat)
    torch.cuda.synchronize()
    t = time.perf_counter()
    B = tt.Batch(ns=ns, ms=ms, src=src, dst=dst, w=w, stream=torch.cuda.current_stream(dev))
    load_ms = (time.perf_counter() - t) * 1e3
    k, p = 10, 1.0
    first = B.topk(k, p, with_stats=True)  # autotunes and captures
    tune = first["stats"]
    print(f"[bench] loaded in {load_ms:.0f} ms; tuned config {tune['config']} in {tune['tune_ms']:.0f} ms",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        B.topk(k, p)
    torch.cuda.synchronize()
    lat, dev_ms, agg = [], [], {"stream": 0, "cand": 0, "inter": 0, "emit": 0}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = B.topk(k, p, with_stats=True)
        st = r["stats"]
        lat.append(st["total_ms"])
        dev_ms.append(st["launch_ms"])
        agg["stream"] += st["edges_streamed"]; agg["cand"] += st["candidate_edges"]
        agg["inter"] += st["intersected_entries"]; agg["emit"] += st["triangles_emitted"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    same = all(np.array_equal(first[x], r[x]) for x in ("i", "j", "l", "score", "n_out"))
    alg = (B_STREAM * agg["stream"] + B_CAND * agg["cand"] + B_INTER * agg["inter"] + B_EMIT * agg["emit"])
    mean_dev = float(np.mean(dev_ms))
    achieved = alg / args.steps / (mean_dev * 1e-3) / 1e9
    # the single-graph path on the same graphs: each graph resident, one query after the other
    Gs = [tt.Graph(g.n, g.src, g.dst, g.w) for g in gs[: args.single_count]]
    for G in Gs[:16]:
        G.topk(k, p)
    t1 = time.perf_counter()
    for G in Gs:
        G.topk(k, p)
    single_s = time.perf_counter() - t1
    for G in Gs:
        G.close()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        sample = gs[: args.cpu_sample]
        tc = time.perf_counter()
        for g in sample:
            oracle.topk(g.n, g.src, g.dst, g.w, k, p, nthreads=nthreads)
        cpu_s = time.perf_counter() - tc
        cpu = {"value": len(sample) / cpu_s, "unit": "graphs/s", "cores": nthreads, "kind": "oracle",
               "sample": f"top-{k} at p=1 of the first {len(sample)} graphs of the batch, one after the other, "
                         f"{cpu_s:.2f}s"}
    B.close()
    out = {
        "metric": METRIC, "value": len(gs) * args.steps / elapsed, "unit": "graphs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"batched: {len(gs)} chung-lu graphs, n log-uniform [50,2e4], mean degree U[4,40], "
                               "gamma2.5 zipf(2)[1,1e6]; top-10 per graph at p=1, one captured launch sequence",
                   "graphs": len(gs), "m": total_m, "k": k, "p": "1", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "batched sequence (plan, scan, filter, intersect per pass; select)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": alg / args.steps, "mean_launch_ms": mean_dev},
        "cpu_baseline": cpu,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "autotune": {"config": tune["config"], "growth": tune["growth"], "filter_blocks": tune["filter_blocks"],
                     "intersect_blocks": tune["intersect_blocks"], "passes": tune["passes"], "restart_rounds": tune["restart_rounds"], "merge_max": tune["merge_max"],
                     "tune_ms": tune["tune_ms"]},
        "restarts": first["stats"]["restarts"], "replays_identical": bool(same), "load_ms": load_ms,
        "single_query_path": {"graphs": len(Gs), "graphs_per_s": len(Gs) / single_s},
    }
    print(json.dumps(out), flush=True)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q)) if xs else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS) + ["serve", "batch", "methods"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sampling", action="store_true", help="exact queries only")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the resident-graph queries after the timed steps (counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device 3 times (a kernel of known traffic for counter runs)")
    ap.add_argument("--requests", type=int, default=2000, help="served workload: number of requests")
    ap.add_argument("--slots", type=int, default=4, help="served workload: server slots")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="served workload: hardware queues of the process (default: two per slot, 4 to 32)")
    ap.add_argument("--budget-gb", type=int, default=16, help="served workload: scratch budget (GiB)")
    ap.add_argument("--serve-n", type=int, default=10_000_000)
    ap.add_argument("--serve-m", type=int, default=200_000_000)
    ap.add_argument("--batch-count", type=int, default=4096, help="batched workload: number of graphs")
    ap.add_argument("--single-count", type=int, default=1024,
                    help="batched workload: graphs also run through the single-graph path")
    ap.add_argument("--cpu-sample", type=int, default=512, help="batched workload: graphs timed on the oracle")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on one GPU; there is no multi-GPU path to measure "
              "(the replicated-graph sharding it would use is described with the design notes).",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "methods":
        return run_methods(args)

    import graphgen

    W = WORKLOADS[args.workload]
    t = time.time()
    g = getattr(graphgen, W["gen"])()
    gen_s = time.time() - t
    print(f"[bench] workload {args.workload}: n={g.n} m={g.m} (generated in {gen_s:.1f}s)", file=sys.stderr, flush=True)
    k, ps, budget = W["k"], W["ps"], W["budget"]
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cpu = None
    if not args.no_cpu_baseline and W.get("cpu_timebox"):
        # before anything touches the GPU (the time-boxed run starts a child process)
        cpu = cpu_baseline_timeboxed(g, W["gen"], k, W["cpu_timebox"], nthreads)

    import torch
    import paper_1910_00692_amd as tt

    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    dev = torch.device("cuda:0")
    s_d = torch.from_numpy(g.src.view(np.int32)).to(dev)
    d_d = torch.from_numpy(g.dst.view(np.int32)).to(dev)
    w_d = torch.from_numpy(g.w.view(np.int32)).to(dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()

    do_es = budget > 0 and not args.no_sampling
    lat = {"build": [], "exact": [], "sample": []}
    agg = {"stream": 0, "cand": 0, "inter": 0, "emit": 0, "kernel_ms": 0.0, "launches": 0, "queries": 0}
    first_results = {}
    build_ev = []

    def step(record: bool, idx: int):
        t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        G = tt.Graph(g.n, s_d, d_d, w_d, stream=stream)
        e1.record(stream)
        t1 = time.perf_counter()
        nq = 0
        for p in ps:
            r = G.topk(k, p, with_stats=True)
            nq += 1
            if idx == 0 and not record:
                first_results[("exact", p)] = r
            if record:
                st = r["stats"]
                lat["exact"].append(st["total_ms"])
                agg["stream"] += st["edges_streamed"]; agg["cand"] += st["candidate_edges"]
                agg["inter"] += st["intersected_entries"]; agg["emit"] += st["triangles_emitted"]
                agg["kernel_ms"] += st["enum_kernel_ms"]; agg["launches"] += st["passes"]
        if do_es:
            for p in ps:
                r = G.sample(k, p, budget, seed=1234 + idx, with_stats=True)
                nq += 1
                if record:
                    st = r["stats"]
                    lat["sample"].append(st["total_ms"])
                    agg["stream"] += st["edges_streamed"]; agg["cand"] += st["candidate_edges"]
                    agg["inter"] += st["intersected_entries"]; agg["emit"] += st["triangles_emitted"]
                    agg["kernel_ms"] += st["enum_kernel_ms"]; agg["launches"] += st["passes"]
        G.close()
        if record:
            lat["build"].append((t1 - t0) * 1e3)
            build_ev.append((e0, e1))
            agg["queries"] += nq
        return nq

    for i in range(args.warmup):
        step(False, i)
        print(f"[bench] warmup step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nq_total = 0
    for i in range(args.steps):
        nq_total += step(True, i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)

    value = nq_total / elapsed
    alg_bytes = (B_STREAM * agg["stream"] + B_CAND * agg["cand"] + B_INTER * agg["inter"] + B_EMIT * agg["emit"])
    launches = max(agg["launches"], 1)
    mean_launch_ms = agg["kernel_ms"] / launches
    achieved = (alg_bytes / launches) / (mean_launch_ms * 1e-3) / 1e9 if mean_launch_ms > 0 else None
    traffic = recorded_traffic(args.workload)
    roofline = {"bound": "hbm", "kernel": "k_enum (k_filter + k_intersect + k_intersect_heavy of one band)",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "traffic_over_algorithmic": (traffic / (alg_bytes / launches)) if traffic and alg_bytes else None,
                "bytes_per_launch": alg_bytes / launches, "mean_launch_ms": mean_launch_ms, "launches": launches,
                "units_per_launch": {x: agg[x] / launches for x in ("stream", "cand", "inter", "emit")}}
    build_ms = float(np.median([a.elapsed_time(b) for a, b in build_ev])) if build_ev else None
    build_roofline = None
    if build_ms:
        bach = B_BUILD * g.m / (build_ms * 1e-3) / 1e9
        build_roofline = {"bound": "hbm", "kernel": "CSR build (graph_load: every build kernel)", "achieved": bach,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": bach / HBM_PEAK_GBS,
                          "bytes_per_launch": B_BUILD * g.m, "mean_launch_ms": build_ms}

    warm = {}
    if args.workload == "large" and not args.no_warm:
        # queries on a resident CSR (the steps above build it cold every time): the second query
        # of each p, then the steady state once repeated queries of p have built its bound order
        def brief(r):
            st = r["stats"]
            return {"ms": st["total_ms"], "kernel_ms": st["enum_kernel_ms"], "streamed": st["edges_streamed"],
                    "passes": st["passes"], "heavy_candidates": st["heavy_candidates"],
                    "heavy_overflow": st["heavy_overflow"], "bound_order": st["bound_order"]}
        G = tt.Graph(g.n, s_d, d_d, w_d, stream=stream)
        for p in ps:
            G.topk(k, p)
            second = brief(G.topk(k, p, with_stats=True))
            steady, n_q = None, 2
            while n_q < 12:
                r = G.topk(k, p, with_stats=True)
                n_q += 1
                if r["stats"]["bound_order"]:
                    steady = brief(G.topk(k, p, with_stats=True))  # the order already built
                    break
            warm[str(p)] = {"second_query": second, "with_bound_order": steady, "queries_until_order": n_q}
        G.close()

    if not args.no_cpu_baseline and not W.get("cpu_timebox"):
        import oracle
        print(f"[bench] cpu baseline: oracle top-{k} at p=1 on {nthreads} threads, {g.m} edges", file=sys.stderr,
              flush=True)
        tc = time.perf_counter()
        want = oracle.topk(g.n, g.src, g.dst, g.w, k, 1.0, nthreads=nthreads)
        cpu_s = time.perf_counter() - tc
        got = first_results.get(("exact", 1.0))
        checked = None
        if got is not None:
            checked = bool(np.array_equal(got["i"], want["i"]) and np.array_equal(got["j"], want["j"])
                           and np.array_equal(got["l"], want["l"]) and np.array_equal(got["score"], want["score"]))
        cpu = {"value": 1.0 / cpu_s, "unit": "queries/s", "cores": nthreads, "kind": "oracle",
               "sample": f"one exact top-{k} query at p=1 on the full workload graph ({want['total']} triangles "
                         f"enumerated), {cpu_s:.2f}s", "gpu_matches_oracle": checked, "cpu_model": cpu_model(),
               "paper_method": dhl_times(g.n, g.src, g.dst, g.w, k, want, nthreads)}

    out = {
        "metric": METRIC, "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": W["desc"], "n": g.n, "m": g.m, "k": k, "p": [str(p) for p in ps],
                   "sample_budget": budget if do_es else 0, "queries_per_step": nq_total // max(args.steps, 1),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "build_roofline": build_roofline,
        "cpu_baseline": cpu,
        "intersected_edges_per_s": agg["inter"] / elapsed,
        "latency_ms": {kk: {"p50": pct(v, 50), "p99": pct(v, 99), "n": len(v)} for kk, v in lat.items()},
        "warm_exact_queries_per_s": (1e3 / np.mean(lat["exact"])) if lat["exact"] else None,
    }
    if warm:
        out["warm_resident_csr"] = warm
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def dhl_times(n, src, dst, w, k, want, nthreads):
    """The paper's exact method on the CPU (Alg. 2 with alpha_p = 1.25, and Auto-HL) on the same
    input as an oracle run `want`: seconds per query and whether the answer is the oracle's."""
    from paper_1910_00692_amd import dhl
    out = {}
    for name, alpha in (("dhl_alpha_1.25", 1.25), ("auto_hl", 0.0)):
        t = time.perf_counter()
        r = dhl.topk(n, src, dst, w, k, 1.0, alpha, threads=nthreads)
        el = time.perf_counter() - t
        same = all(np.array_equal(r[x], want[x]) for x in ("i", "j", "l", "score"))
        out[name] = {"s": el, "sort_build_s": r["stats"]["build_ms"] / 1e3, "loop_s": r["stats"]["loop_ms"] / 1e3,
                     "enumerated": r["stats"]["enumerated"], "matches_oracle": bool(same)}
    return out


def _oracle_child(conn, gen, k, nthreads):
    """Generates the workload graph again (a fresh process: the oracle's OpenMP runtime must not
    be inherited through fork) and runs the oracle on it; reports readiness, then the time."""
    sys.path.insert(0, ROOT)
    import graphgen
    import oracle
    g = getattr(graphgen, gen)()
    conn.send("ready")
    t = time.perf_counter()
    r = oracle.topk(g.n, g.src, g.dst, g.w, k, 1.0, nthreads=nthreads)
    conn.send((time.perf_counter() - t, r["total"]))
    conn.close()


def cpu_baseline_timeboxed(g, gen, k, budget_s, nthreads):
    """The oracle on the whole graph, top-k at p = 1, in a child process stopped after budget_s
    (the value is then an upper bound, as the paper reports a run that did not finish); beside it
    the oracle on vertex samples (every vertex kept with probability f, the graph's IDs being a
    random permutation: the vertices with ID < f n) at f = 0.1 and 0.15, extrapolated to f = 1
    by the triangles it enumerates (it lists every triangle: the samples hold T(1) f^3 of them, so
    T(1) is estimated from each sample, and the time per triangle is the larger sample's), and
    the f = 0.1 sample on one thread."""
    import multiprocessing as mp
    import oracle
    ctx = mp.get_context("spawn")
    parent, child = ctx.Pipe(duplex=False)
    print(f"[bench] cpu baseline: oracle on the whole graph, {nthreads} threads, time box {budget_s:.0f}s",
          file=sys.stderr, flush=True)
    proc = ctx.Process(target=_oracle_child, args=(child, gen, k, nthreads))
    proc.start()
    child.close()
    whole = None
    if parent.poll(600) and parent.recv() == "ready" and parent.poll(budget_s):
        whole = parent.recv()
    proc.kill()
    proc.join()

    def induced(f):
        lim = np.uint32(int(f * g.n))
        parts = []
        for lo in range(0, g.m, 1 << 27):
            s, d = g.src[lo:lo + (1 << 27)], g.dst[lo:lo + (1 << 27)]
            parts.append(np.nonzero((s < lim) & (d < lim))[0] + lo)
        sel = np.concatenate(parts)
        return g.src[sel], g.dst[sel], g.w[sel]

    samples = {}
    dhl_on_sample = None
    for f in (0.1, 0.15):
        s, d, w = induced(f)
        t = time.perf_counter()
        r = oracle.topk(g.n, s, d, w, k, 1.0, nthreads=nthreads)
        samples[f] = (time.perf_counter() - t, len(s), r["total"])
        print(f"[bench] cpu sample f={f}: {len(s)} edges, {r['total']} triangles, {samples[f][0]:.2f}s",
              file=sys.stderr, flush=True)
        if f == 0.15:
            dhl_on_sample = dhl_times(g.n, s, d, w, k, r, nthreads)
            dhl_on_sample.update({"f": f, "oracle_s": samples[f][0]})
    s, d, w = induced(0.1)
    t = time.perf_counter()
    oracle.topk(g.n, s, d, w, k, 1.0, nthreads=1)
    one_thread = time.perf_counter() - t
    (f1, (t1, m1, T1)), (f2, (t2, m2, T2)) = sorted(samples.items())
    T_est = 0.5 * (T1 / f1 ** 3 + T2 / f2 ** 3)  # the two estimates agree within a few percent
    ns_per_triangle = t2 / max(T2, 1) * 1e9
    extrap = T_est * ns_per_triangle * 1e-9
    if whole:
        value, desc = 1.0 / whole[0], f"one exact top-{k} query at p=1 on the whole graph ({whole[1]} triangles), " \
                                      f"{whole[0]:.1f}s"
    else:
        value = 1.0 / budget_s
        desc = (f"one exact top-{k} query at p=1 on the whole graph, time-boxed: not finished in {budget_s:.0f}s, so "
                f"the value is an upper bound; extrapolated from vertex samples: {extrap:.0f}s per query")
    return {"value": value, "unit": "queries/s", "cores": nthreads, "kind": "oracle", "sample": desc,
            "finished": bool(whole), "time_box_s": budget_s, "cpu_model": cpu_model(),
            "vertex_samples": [{"f": f, "edges": m_, "triangles": T_, "s": t_}
                               for f, (t_, m_, T_) in sorted(samples.items())],
            "extrapolated_s_per_query": extrap, "extrapolated_queries_per_s": 1.0 / extrap,
            "triangles_estimate": T_est, "triangles_estimates_per_sample": [T1 / f1 ** 3, T2 / f2 ** 3],
            "ns_per_triangle": ns_per_triangle,
            "paper_method_on_sample": dhl_on_sample,
            "one_thread": {"f": 0.1, "s": one_thread, "threads_speedup": one_thread / samples[0.1][0]}}


if __name__ == "__main__":
    main()
