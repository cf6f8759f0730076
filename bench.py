#!/usr/bin/env python3
"""Throughput of the HIP subgraph matcher on one MI355X.

Workload (default, ``--workload large``): R-MAT data graph, 2^21 vertices,
edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), unlabelled.  One step lists
every triangle embedding into HBM (5.7 x 10^9 rows, handed chunk by chunk to
a device-side consumer), counts the triangles once per subgraph, and counts
the 4-clique, 5-cycle and house+tail embeddings on fixed root slices.

``--workload powerlaw`` enumerates the 20 power-law queries (R-MAT 2^17, 16
Zipf labels); ``batch`` compares batched and per-launch queries/s; ``serving``
reports p50/p99 latency under Poisson arrivals.

Prints one JSON line: embeddings/s over the timed steps, the expansion
kernel's roofline (algorithmic bytes over its HIP-event time, and the HBM
bytes rocprofv3 measured for the same command when a record of them matches
the current sources), and the CPU oracle timed on a bounded sample of the
same workload.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources whose change invalidates a stored traffic record: the kernels and
# every host file that chooses launch shapes, chunks or what is launched.
TRAFFIC_SOURCES = ["paper_2003_01527_amd/csrc/" + f for f in
                   ("kernels.hip", "match.cpp", "batch.cpp", "plan.cpp", "capi.cpp", "gsm_internal.h")] + ["bench.py"]


def sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_record_path(workload):
    return os.path.join(ROOT, "profiles", "k_expand_%s_traffic.json" % workload)


VERTEX_ORDER = {False: "graph stored renumbered by ascending degree (GSM_GRAPH_DEGREE_ORDER); results in "
                       "the generator's ids",
                True: "graph stored in the generator's numbering"}


def measured_traffic(workload, vertex_order):
    """HBM bytes per expansion launch from the committed rocprofv3 counter
    record of this workload, or None when any source it depends on changed
    since it was taken."""
    try:
        rec = json.load(open(traffic_record_path(workload)))
        sha = sources_sha1()
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha1") != sha or rec.get("vertex_order") != vertex_order:
        return None
    return rec["traffic_bytes_per_launch"]


def write_traffic_record(workload, vertex_order, fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes):
    """Builds the traffic record from four rocprofv3 --pmc runs (csv output):
    FETCH_SIZE and WRITE_SIZE of the bench command (k_expand dispatches), and
    of a plain device copy of copy_bytes bytes (the calibration: what each
    counter reads per byte actually moved)."""
    import csv
    import glob

    def per_kernel(d, counter, match):
        tot, n = 0.0, 0
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter and match in r.get("Kernel_Name", ""):
                    tot += float(r["Counter_Value"])
                    n += 1
        return tot, n

    f_kib, nf = per_kernel(fetch_dir, "FETCH_SIZE", "k_expand")
    w_kib, nw = per_kernel(write_dir, "WRITE_SIZE", "k_expand")
    cf_kib, _ = per_kernel(cfetch_dir, "FETCH_SIZE", "copyBuffer")
    cw_kib, _ = per_kernel(cwrite_dir, "WRITE_SIZE", "copyBuffer")
    fscale = copy_bytes / (cf_kib * 1024.0)
    wscale = copy_bytes / (cw_kib * 1024.0)
    fetch = f_kib * 1024.0 * fscale
    write = w_kib * 1024.0 * wscale
    launches = max(nf, 1)
    rec = {"kernel": "k_expand", "workload": workload, "vertex_order": vertex_order, "sources_sha1": sources_sha1(),
           "launches": launches, "fetch_bytes": round(fetch), "write_bytes": round(write),
           "traffic_bytes_per_launch": round((fetch + write) / launches),
           "fetch_scale": fscale, "write_scale": wscale, "dispatch_records": [nf, nw]}
    with open(traffic_record_path(workload), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


def host_cores():
    """Threads the CPU baseline uses (the host CPUs this process may run on,
    at most 16, the CPU share of one GPU on the measurement boxes) and the
    host's own count."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return min(16, avail), os.cpu_count() or 1


def oracle_queries_per_s(graph, queries, mod=64, budget_s=20.0):
    """CPU baseline for the query-throughput workloads: the oracle, count
    only, on all host threads it may use, over the queries in arrival order,
    each on the root slice of residue k % mod of query vertex 0 (a 1/mod share
    of its work), until budget_s seconds are spent; queries/s = slices done /
    mod / seconds."""
    import oracle
    cores, nproc = host_cores()
    t = time.perf_counter()
    done = 0
    for k, qr in enumerate(queries):
        oracle.match(graph, qr, rows=False, threads=cores, root=(0, mod, k % mod))
        done += 1
        if time.perf_counter() - t > budget_s:
            break
    dt = time.perf_counter() - t
    return {"value": round(done / mod / dt, 2), "unit": "queries/s", "cores": cores, "host_nproc": nproc,
            "kind": "oracle",
            "sample": "the first %d queries in arrival order, each on the root slice splitmix64(f(0)) %% %d == k %% %d "
                      "(1/%d of its embeddings), count only, %.1f s; value = slices / %d / s"
                      % (done, mod, mod, mod, dt, mod)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--mode", choices=["enumerate", "count"], default="enumerate")
    ap.add_argument("--queries", type=int, default=20)
    ap.add_argument("--cpu-slice", type=int, default=16,
                    help="oracle sample: root slice 1/N of every query")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--items", type=int, default=0)
    ap.add_argument("--workload", choices=["large", "powerlaw", "batch", "serving"], default="large",
                    help="large: embeddings/s on the 2^21-vertex graph (default); powerlaw: embeddings/s "
                         "on the 20 labelled queries; batch: batched vs per-launch queries/s; "
                         "serving: p50/p99 latency and queries/s under Poisson arrivals")
    ap.add_argument("--arrivals", type=int, default=10000, help="serving: number of requests")
    ap.add_argument("--workers", type=int, default=4, help="serving: worker streams")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (JSON)")
    ap.add_argument("--batch-cap-log2", type=int, default=32,
                    help="batch: reject queries whose spanning-tree bound exceeds 2^N (20 = light mix)")
    ap.add_argument("--vertex-order", choices=["auto", "degree", "caller"], default="auto",
                    help="store the data graph renumbered by ascending degree (GSM_GRAPH_DEGREE_ORDER) or in "
                         "the generator's numbering; auto: the generator's for the power-law listing (its "
                         "2^17-vertex graph is cache-resident and translating 8 x 10^10 listed ids back costs "
                         "more than locality gains), by degree for the others")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (calibrates "
                         "the HBM byte counters of rocprofv3) and exit")
    ap.add_argument("--write-traffic-record", nargs=4, metavar=("FETCH", "WRITE", "CFETCH", "CWRITE"),
                    help="rocprofv3 --pmc output folders of FETCH_SIZE and WRITE_SIZE for this workload "
                         "and for a --copy-gib 1 run: store the traffic record and exit")
    args = ap.parse_args()
    if args.vertex_order == "auto":
        args.vertex_order = "caller" if args.workload == "powerlaw" else "degree"
    args.caller_ids = args.vertex_order == "caller"

    if args.write_traffic_record:
        return write_traffic_record(args.workload, args.vertex_order, *args.write_traffic_record, copy_bytes=1 << 30)

    if args.copy_gib > 0:
        import torch
        nbytes = int(args.copy_gib * (1 << 30))
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes}), flush=True)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU: the matcher runs on a single device "
              "(root-slice sharding across GPUs is a design note, not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "large":
        return bench_large(args)
    return bench_powerlaw(args)


def bench_powerlaw(args):
    import torch

    from paper_2003_01527_amd import gsm
    from paper_2003_01527_amd import workloads as W

    t = time.time()
    w = W.powerlaw()
    queries = w.queries[:args.queries]
    log("workload %s: n=%d nnz=%d, %d queries (%.1fs)" % (w.graph.name, w.graph.n, w.graph.nnz,
                                                        len(queries), time.time() - t))
    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    G = gsm.Graph.from_workload(w.graph, degree_order=not args.caller_ids)
    Qs = [gsm.Query.from_workload(q) for q in queries]
    budget = int(args.budget_gb * (1 << 30))

    def sink(ptr, nrows, q):  # device-side consumer: the rows are left in HBM
        return False

    def one_step(profile=False):
        counts, bytes_, ms_exp, launches, stats = [], 0, 0.0, 0, []
        for Q in Qs:
            if args.mode == "enumerate":
                c, _, st = gsm.match(G, Q, emit_device=sink, budget=budget, stream=stream.cuda_stream,
                                     profile=profile, wg_size=args.wg, tile_items=args.items)
            else:
                c, _, st = gsm.match(G, Q, budget=budget, stream=stream.cuda_stream, profile=profile,
                                     wg_size=args.wg, tile_items=args.items)
            counts.append(c)
            bytes_ += st["alg_bytes"]
            ms_exp += st["ms_expand"]
            launches += st["expand_launches"]
            stats.append(st)
        return counts, bytes_, ms_exp, launches, stats

    for i in range(args.warmup):
        t = time.time()
        counts, _, _, _, _ = one_step()
        log("warmup %d: %.3fs, embeddings %d" % (i, time.time() - t, sum(counts)))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_emb, tot_bytes, tot_ms, tot_launch = 0, 0, 0.0, 0
    for i in range(args.steps):
        counts, b, ms, nl, stats = one_step(profile=True)
        tot_emb += sum(counts)
        tot_bytes += b
        tot_ms += ms
        tot_launch += nl
        log("step %d done: embeddings %d" % (i, sum(counts)))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    value = tot_emb / elapsed
    achieved = (tot_bytes / 1e9) / (tot_ms / 1e3) if tot_ms > 0 else 0.0
    traffic = (measured_traffic("powerlaw", args.vertex_order) if args.mode == "enumerate" and not (args.wg or args.items)
               else None)
    roofline = {
        "kernel": "k_expand (expand-verify-compact)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_unit": "HBM bytes per k_expand launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "alg_bytes_per_launch": tot_bytes // max(tot_launch, 1),
        "alg_bytes_per_step": tot_bytes // max(args.steps, 1),
        "kernel_ms_per_step": round(tot_ms / max(args.steps, 1), 3),
        "launches_per_step": tot_launch // max(args.steps, 1),
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores, nproc = host_cores()
        mod = args.cpu_slice
        t = time.perf_counter()
        emb = 0
        for qr in queries:
            c, _ = oracle.match(w.graph, qr, rows=False, threads=cores, root=(0, mod, 0))
            emb += c
        dt = time.perf_counter() - t
        cpu = {"value": round(emb / dt, 1), "unit": "embeddings/s", "cores": cores, "kind": "oracle",
               "host_nproc": nproc,
               "sample": "all %d queries restricted to the root slice splitmix64(f(query vertex 0)) %% %d == 0 "
                         "(%d embeddings, %.1f s, count only)" % (len(queries), mod, emb, dt)}
        log("cpu baseline: %s" % cpu)

    out = {
        "metric": "embeddings/s",
        "value": round(value, 1),
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / max(args.steps, 1), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "powerlaw R-MAT 2^17 ef8 (0.57,0.19,0.19), 16 Zipf(1.0) labels; "
                        "%d random-walk induced queries, 5-6 vertices, 5-9 edges; %s"
                        % (len(queries), "full enumeration into HBM" if args.mode == "enumerate"
                           else "count only"),
            "vertex_order": VERTEX_ORDER[args.caller_ids],
            "graph_vertices": w.graph.n,
            "graph_csr_entries": w.graph.nnz,
            "queries": len(queries),
            "embeddings_per_step": tot_emb // max(args.steps, 1),
            "memory_budget_gb": args.budget_gb,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# Large unlabelled workload: every triangle embedding listed into HBM, the
# triangles counted once per subgraph (unique mode), and the 4-clique, 5-cycle
# and house+tail counted on deterministic root slices (their full counts take
# minutes to hours even on the GPU).  (label, shape, root slice, list, unique)
LARGE_STEP = [("K3", "K3", None, True, False), ("K3 unique", "K3", None, False, True),
              ("K4", "K4", (0, 512, 1), False, False), ("C5", "C5", (0, 1 << 17, 1), False, False),
              ("house_tail", "house_tail", (0, 1 << 20, 1), False, False)]


def bench_large(args):
    import torch

    from paper_2003_01527_amd import gsm
    from paper_2003_01527_amd import workloads as W

    t = time.time()
    g = W.large_graph()
    log("workload %s: n=%d nnz=%d (%.1fs)" % (g.name, g.n, g.nnz, time.time() - t))
    torch.cuda.init()
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    G = gsm.Graph.from_workload(g, degree_order=not args.caller_ids)
    budget = int(args.budget_gb * (1 << 30))
    Qs = [(name, gsm.Query.from_workload(W.shape(shape)), root, emit, uniq)
          for name, shape, root, emit, uniq in LARGE_STEP]

    unique_of = {name: uniq for name, _, _, _, uniq in LARGE_STEP}

    def sink(ptr, nrows, q):
        return False

    def one_step(profile=False):
        out = []
        for name, Q, root, emit, uniq in Qs:
            kw = dict(budget=budget, stream=stream.cuda_stream, profile=profile, wg_size=args.wg,
                      tile_items=args.items, unique=uniq)
            if root is not None:
                kw["root"] = root
            if emit:
                kw["emit_device"] = sink
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            c, _, st = gsm.match(G, Q, **kw)
            torch.cuda.synchronize()
            out.append((name, c, time.perf_counter() - t1, st))
            log("  %s: %d embeddings, %.3fs" % (name, c, out[-1][2]))
        return out

    for i in range(args.warmup):
        t = time.time()
        one_step()
        log("warmup %d: %.3fs" % (i, time.time() - t))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = {}
    tot_emb, tot_bytes, tot_ms, tot_launch = 0, 0, 0.0, 0
    for i in range(args.steps):
        for name, c, dt, st in one_step(profile=True):
            tot_emb += 0 if unique_of[name] else c  # subgraph counts are not embeddings
            tot_bytes += st["alg_bytes"]
            tot_ms += st["ms_expand"]
            tot_launch += st["expand_launches"]
            e = per.setdefault(name, {"embeddings": c, "s": 0.0})
            e["s"] += dt
        log("step %d done" % i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for name, shape, root, emit, uniq in LARGE_STEP:
        e = per[name]
        e["s"] = round(e["s"] / args.steps, 4)
        e["embeddings_per_s"] = round(e["embeddings"] / e["s"], 1) if e["s"] > 0 else None
        e["root_slice"] = list(root) if root else None
        e["listed"] = emit
        e["unique"] = uniq
    achieved = (tot_bytes / 1e9) / (tot_ms / 1e3) if tot_ms > 0 else 0.0
    launches = max(tot_launch, 1)
    traffic = measured_traffic("large", args.vertex_order) if not (args.wg or args.items) else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores, nproc = host_cores()
        t = time.perf_counter()
        c, _ = oracle.match(g, W.shape("K3"), rows=False, threads=cores, root=(0, 64, 0))
        dt = time.perf_counter() - t
        cpu = {"value": round(c / dt, 1), "unit": "embeddings/s", "cores": cores, "kind": "oracle",
               "host_nproc": nproc,
               "sample": "triangle embeddings with splitmix64(f(vertex 0)) %% 64 == 0 (%d, %.1f s, count only)"
                         % (c, dt)}
        log("cpu baseline: %s" % cpu)
    print(json.dumps({
        "metric": "embeddings/s",
        "value": round(tot_emb / elapsed, 1),
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / max(args.steps, 1), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "large unlabelled R-MAT 2^21 ef16 (0.57,0.19,0.19): every triangle embedding listed "
                        "into HBM, triangles counted once per subgraph (not in value), 4-clique on the root slice "
                        "splitmix64(f(0)) %% 512 == 1, 5-cycle on %% 2^17 == 1, house+tail on %% 2^20 == 1, "
                        "counted",
            "vertex_order": VERTEX_ORDER[args.caller_ids],
            "graph_vertices": g.n,
            "graph_csr_entries": g.nnz,
            "per_query": per,
            "memory_budget_gb": args.budget_gb,
        },
        "roofline": {
            "kernel": "k_expand (expand-verify-compact)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per k_expand launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_frac": (round(traffic * launches / (tot_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic and tot_ms > 0 else None),
            "alg_bytes_per_launch": tot_bytes // launches,
            "alg_bytes_per_step": tot_bytes // max(args.steps, 1),
            "kernel_ms_per_step": round(tot_ms / max(args.steps, 1), 3),
            "avg_launch_us": round(1e3 * tot_ms / launches, 1),
            "launches_per_step": tot_launch // max(args.steps, 1),
        },
        "cpu_baseline": cpu,
    }), flush=True)


def bench_batch(args):
    """512 random-walk queries (3-8 vertices, edge density 0.3-1.0) on the 2^17
    power-law graph, counted in batched launches vs one gsm_match per query."""
    import numpy as np
    import torch

    from paper_2003_01527_amd import gsm
    from paper_2003_01527_amd import workloads as W

    from paper_2003_01527_amd import autotune

    w = W.batch(cap=float(2 ** args.batch_cap_log2))
    torch.cuda.init()
    G = gsm.Graph.from_workload(w.graph, degree_order=not args.caller_ids)
    Qs = [gsm.Query.from_workload(q) for q in w.queries]
    budget = int(args.budget_gb * (1 << 30))
    stream = torch.cuda.current_stream().cuda_stream
    best = autotune.tune_batch(G, Qs, w.queries, budget, cache_path=args.tune_cache, log=log)
    log("autotuned: %s" % best)
    kw = dict(budget=best.get("budget", budget), stream=stream, wg_size=best["wg_size"],
              tile_items=best["tile_items"], stage_bytes=best.get("stage_bytes", 0))

    def per_launch():
        return np.array([gsm.match(G, Q, **kw)[0] for Q in Qs], dtype=np.uint64)

    def batched():
        return gsm.match_batch(G, Qs, batch_heavy_pairs=best["batch_heavy_pairs"], **kw)

    ref = per_launch()
    got = batched()
    assert np.array_equal(ref, got), "batched counts differ from per-query counts"
    res = {}
    for name, fn in (("per_launch", per_launch), ("batched", batched)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t) / args.steps
        log("%s: %.1f ms per pass of %d queries" % (name, res[name] * 1e3, len(Qs)))
    qps_b = len(Qs) / res["batched"]
    qps_p = len(Qs) / res["per_launch"]
    out = {
        "metric": "queries/s (batched)",
        "value": round(qps_b, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["batched"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "batch: R-MAT 2^17 ef8, 16 Zipf labels; %d random-walk queries, 3-8 vertices, "
                               "edge density 0.3-1.0, spanning-tree bound <= 2^%d; count only"
                               % (len(Qs), args.batch_cap_log2),
                   "vertex_order": VERTEX_ORDER[args.caller_ids],
                   "embeddings_per_step": int(ref.sum())},
        "per_launch_queries_per_s": round(qps_p, 1),
        "autotuned": best,
        "batched_over_per_launch": round(qps_b / qps_p, 3),
        "cpu_baseline": None if args.no_cpu_baseline else oracle_queries_per_s(w.graph, w.queries),
    }
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Open-loop Poisson arrivals of random-walk queries (3-8 vertices) on a
    resident 2^20-vertex R-MAT graph with 32 Zipf labels; the serving engine
    admits by frontier-memory estimate and batches what is waiting."""
    import numpy as np
    import torch

    from paper_2003_01527_amd import gsm
    from paper_2003_01527_amd import workloads as W

    t = time.time()
    w = W.serving(nq=args.arrivals)
    log("serving workload: n=%d nnz=%d, %d arrivals from %d distinct queries (%.1fs)"
        % (w.graph.n, w.graph.nnz, len(w.queries), len({id(q) for q in w.queries}), time.time() - t))
    torch.cuda.init()
    G = gsm.Graph.from_workload(w.graph, degree_order=not args.caller_ids)
    pool = {}
    Qs = []
    for qr in w.queries:
        if id(qr) not in pool:
            pool[id(qr)] = gsm.Query.from_workload(qr)
        Qs.append(pool[id(qr)])
    # alone, for the equality check on a sample
    sample = list(range(0, len(Qs), max(1, len(Qs) // 200)))
    alone = {k: gsm.match(G, Qs[k])[0] for k in sample}

    def run(rate):
        srv = gsm.Server(G, workers=args.workers, arena_bytes=int(args.budget_gb * (1 << 30)), max_batch=64)
        gaps = None if rate is None else w.arrivals * (1000.0 / rate)  # arrivals are for rate 1000/s
        t0 = time.perf_counter()
        tickets = []
        for k, Q in enumerate(Qs):
            if gaps is not None:
                d = t0 + gaps[k] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
            tickets.append(srv.submit(Q))
        res = [srv.wait(tk) for tk in tickets]
        srv.close()
        for k in sample:
            assert res[k]["count"] == alone[k], "served result differs from the query alone"
        lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) / 1e6 for r in res])
        span = (max(r["t_done_ns"] for r in res) - min(r["t_submit_ns"] for r in res)) / 1e9
        return {"queries_per_s": round(len(res) / span, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_batch": round(float(np.mean([r["batch_size"] for r in res])), 2),
                "arrivals": len(res), "rate_per_s": None if rate is None else round(rate, 1)}

    cpu = None if args.no_cpu_baseline else oracle_queries_per_s(w.graph, w.queries)
    log("cpu baseline: %s" % cpu)
    sat = run(None)
    log("saturation (all submitted at once): %s" % sat)
    r08 = run(0.8 * sat["queries_per_s"])
    log("Poisson at 0.8 x saturation: %s" % r08)
    r05 = run(0.5 * sat["queries_per_s"])
    log("Poisson at 0.5 x saturation: %s" % r05)
    out = {
        "metric": "p50/p99 query latency (ms) and queries/s under Poisson arrivals",
        "value": r08["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "serving: R-MAT 2^20 ef12, 32 Zipf labels; %d Poisson arrivals of random-walk "
                               "queries (3-8 vertices), count only; %d workers" % (len(Qs), args.workers),
                   "vertex_order": VERTEX_ORDER[args.caller_ids]},
        "latency_at_0.8x_saturation": r08,
        "latency_at_0.5x_saturation": r05,
        "saturation": sat,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
