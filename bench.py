"""Benchmark: exact subgraph-matching throughput on one MI355X.

One step = every query of the workload counted once (root candidates, initial
pool, persistent depth-first search: the whole hot path), inputs resident in
HBM.  Prints ONE JSON line on stdout; progress goes to stderr.

Workload (default): R-MAT scale 20, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05),
16 Zipf(1.0) labels, 100 random-walk queries of 8 vertices (50 dense, 50 sparse),
each counted exactly with a cap of 1e8 embeddings.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
KERNEL_SRCS = [os.path.join(ROOT, "paper_2604_10601_amd", "csrc", f)
               for f in ("kernels.hip", "gm_internal.h", "engine.cpp", "graph_build.hip")]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    """Hash of the sources that decide what the search kernel reads (kernels, layouts, graph upload)."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def traffic_file_for(workload: str) -> str:
    """Committed counter summary of the search kernel on a workload."""
    short = {"rmat24_ef16_zipf8_q12-32": "rmat24_q12-32", "rmat20_ef16_zipf16_q8": "rmat20_q8"}.get(workload, workload)
    return os.path.join(ROOT, "profiles", f"search_kernel_{short}_traffic.txt")


def read_traffic(path: str) -> dict | None:
    """HBM traffic per launch from a committed counter summary, if it matches this kernel source."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha") != kernel_sha():
        return None
    try:
        return {"bytes_per_launch": float(kv["traffic_bytes_per_launch"])}
    except (KeyError, ValueError):
        return None


def make_workload(name: str, num_queries: int, stride: int = 1):
    from paper_2604_10601_amd import workloads as wl
    if name == "medium":
        w = wl.medium_rmat20()
    elif name == "small":
        w = wl.small_er()
    elif name == "large":
        t = time.time()
        g = wl.rmat24_graph()
        log(f"R-MAT scale 24 graph generated in {time.time() - t:.1f} s; extracting queries")
        w = wl.large_rmat24(g=g)
    elif name in ("batch", "serve"):
        w = wl.batch_rmat20()
    else:
        raise SystemExit(f"unknown workload {name}")
    w.queries = w.queries[::max(1, stride)]
    if num_queries > 0:
        w.queries = w.queries[:num_queries]
    return w


def cpu_baseline(w, phis, budget_s: float, cap: int, per_query_s: float, gpu_results) -> dict:
    """The oracle, as it is, on the host cores, over a bounded sample of the same
    queries; its counts are compared with the GPU's for every query both decided."""
    import oracle
    total = 0
    secs = 0.0
    used = 0
    threads = 0
    capped = 0
    compared = 0
    mismatched = []
    for i, (q, phi) in enumerate(zip(w.queries, phis)):
        if secs >= budget_s:
            break
        r = oracle.count(w.graph, q, order=phi, cap=cap, time_limit_s=per_query_s)
        total += r.count
        secs += r.seconds
        used += 1
        threads = r.threads
        capped += r.outcome == oracle.CAPPED
        g = gpu_results[i]
        if r.outcome != oracle.TIMEOUT and g.outcome != 2:
            compared += 1
            if (r.count, r.outcome) != (g.count, g.outcome):
                mismatched.append(i)
    rate = total / secs if secs > 0 else 0.0
    return {"value": rate, "unit": "embeddings/s", "cores": threads, "kind": "oracle",
            "sample": (f"first {used} of the {len(w.queries)} queries in workload order, each with the "
                       f"workload's cap ({cap}) and at most {per_query_s} s ({capped} reached the cap); "
                       f"stopped after {secs:.1f} s of oracle time"),
            "counts_compared": compared, "same_counts": not mismatched, "mismatched_queries": mismatched}


def copy_probe(nbytes: int) -> None:
    """One device-to-device copy of nbytes (a plain copy kernel of known size, used to
    calibrate the FETCH_SIZE / WRITE_SIZE counters)."""
    hip = ctypes.CDLL("libamdhip64.so")
    src, dst = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(src), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(ctypes.byref(dst), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMemset(src, 1, ctypes.c_size_t(nbytes)) == 0
    assert hip.hipDeviceSynchronize() == 0
    assert hip.hipMemcpy(dst, src, ctypes.c_size_t(nbytes), 3) == 0   # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(src)
    hip.hipFree(dst)


def _csvs(root: str, suffix: str):
    import glob
    return sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True))


def kernel_key(name: str) -> str:
    """Short name of a dispatched kernel: search kernels by mode, copies, others by function name."""
    import re
    m = re.search(r"search_kernel<(\d+), (true|false), (true|false), (true|false), (\d+)>", name)
    if m:
        return {"0": "search", "1": "enumerate", "2": "expand"}[m.group(1)] + (
            "<slim" if m.group(2) == "true" else "<full") + (",sb" if m.group(3) == "true" else "") + (
            ",cg" if m.group(4) == "true" else "") + (",5w>" if m.group(5) == "5" else ">")
    if "copyBuffer" in name:
        return "copy"
    base = name[:-1].rsplit("(", 1)[0] if name.endswith(")") else name
    return base.replace("gm::(anonymous namespace)::", "").replace("void ", "")


def summarize_stats(root: str) -> str:
    """Kernel table from a rocprofv3 --kernel-trace --stats run (csv output)."""
    import csv
    lines = []
    for path in _csvs(root, "kernel_stats.csv"):
        for row in csv.DictReader(open(path)):
            lines.append(f"{kernel_key(row.get('Name', '')):<34} calls={row.get('Calls'):>5} "
                         f"total_ms={float(row.get('TotalDurationNs', 0)) / 1e6:10.3f} "
                         f"avg_ms={float(row.get('AverageNs', 0)) / 1e6:9.4f} "
                         f"min_ms={float(row.get('MinNs', 0)) / 1e6:9.4f} "
                         f"max_ms={float(row.get('MaxNs', 0)) / 1e6:9.4f} pct={float(row.get('Percentage', 0)):6.2f}")
    return "\n".join(lines)


def pmc_per_kernel(root: str, counter: str) -> dict:
    """Mean counter value per dispatch for each kernel key; for the calibration copy, the largest dispatch."""
    import csv
    acc = {}
    for path in _csvs(root, "counter_collection.csv"):
        for row in csv.DictReader(open(path)):
            if row.get("Counter_Name") != counter:
                continue
            acc.setdefault(kernel_key(row.get("Kernel_Name", "")), []).append(float(row["Counter_Value"]))
    out = {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}
    if "copy" in acc:
        out["copy"] = (max(acc["copy"]), 1)
    return out


def merge_means(parts) -> tuple:
    """(mean, count) pairs -> the mean over all of them and the total count."""
    n = sum(c for _, c in parts)
    return (sum(m * c for m, c in parts) / n if n else 0.0), n


def summarize_trace(root: str, skip: int, take: int) -> str:
    """Durations of the search kernel's dispatches from a rocprofv3 --kernel-trace run,
    in dispatch order: all of them, and the window [skip, skip + take) -- the timed
    steps of a bench run when skip = warmup x queries and take = steps x queries."""
    import csv
    rows = []
    for path in _csvs(root, "kernel_trace.csv"):
        for row in csv.DictReader(open(path)):
            k = kernel_key(row.get("Kernel_Name", ""))
            if k.startswith("search<"):
                rows.append((int(row["Dispatch_Id"]), k,
                             (float(row["End_Timestamp"]) - float(row["Start_Timestamp"])) / 1e6))
    rows.sort()
    win = rows[skip:skip + take]
    lines = [f"search dispatches: {len(rows)}"]
    for name, part in (("all", rows), (f"window [{skip}, {skip + take})", win)):
        if not part:
            continue
        ms = [d for _, _, d in part]
        by = {}
        for _, k, d in part:
            by.setdefault(k, []).append(d)
        lines.append(f"{name}: dispatches={len(ms)} avg_ms={sum(ms) / len(ms):.4f} total_ms={sum(ms):.3f} " +
                     " ".join(f"{k}: n={len(v)} avg_ms={sum(v) / len(v):.4f}" for k, v in sorted(by.items())))
    return "\n".join(lines)


def summarize_pmc(root: str) -> str:
    """Counters of a rocprofv3 --pmc run, summed over the search kernel's dispatches,
    with the ratios used to read them: the fraction of wave-cycles spent waiting,
    and instructions per wave."""
    import csv
    sums, dispatches, keys = {}, {}, set()
    for path in _csvs(root, "counter_collection.csv"):
        for row in csv.DictReader(open(path)):
            k = kernel_key(row.get("Kernel_Name", ""))
            if not k.startswith("search<"):
                continue
            keys.add(k)  # every build of the search kernel the run dispatched
            name = row["Counter_Name"]
            sums[name] = sums.get(name, 0.0) + float(row["Counter_Value"])
            dispatches.setdefault(name, set()).add(row.get("Dispatch_Id", row.get("Correlation_Id", "")))
    lines = [f"kernel: {'+'.join(sorted(keys)) or None}", f"kernel_sha: {kernel_sha()}"]
    for name in sorted(sums):
        lines.append(f"{name}: {sums[name]:.0f}  (dispatches {len(dispatches[name])})")
    if sums.get("SQ_WAVE_CYCLES"):
        if "SQ_WAIT_ANY" in sums:
            lines.append(f"wait_any_fraction: {sums['SQ_WAIT_ANY'] / sums['SQ_WAVE_CYCLES']:.4f}")
        if "SQ_WAIT_INST_ANY" in sums:
            lines.append(f"wait_inst_fraction: {sums['SQ_WAIT_INST_ANY'] / sums['SQ_WAVE_CYCLES']:.4f}")
    if sums.get("SQ_WAVES"):
        for name in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS"):
            if name in sums:
                lines.append(f"{name.lower()}_per_wave: {sums[name] / sums['SQ_WAVES']:.0f}")
    return "\n".join(lines)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--train-queries", type=int, default=3126,
                    help="learned: training queries (4 candidate orders x 4 splits each, half on each graph)")
    ap.add_argument("--eval-queries", type=int, default=1000, help="learned: held-out queries")
    ap.add_argument("--eval-scale", type=int, default=24, choices=[20, 22, 24], help="learned: held-out graph")
    ap.add_argument("--train-cap", type=int, default=10_000_000,
                    help="learned: cap of the training runs (a tenth of the evaluation's: past launch overhead, "
                         "and 50,000 runs fit in minutes)")
    ap.add_argument("--train-limit", type=float, default=0.05, help="learned: time limit of the training runs (s)")
    ap.add_argument("--plan-table", type=int, default=0, metavar="N",
                    help="learned: also time every (order, split) plan of every N-th held-out query once "
                         "(0 = off), for the best plan per query and the model's pick measured side by side")
    ap.add_argument("--plan-table-limit", type=float, default=0.5,
                    help="learned: time limit of each plan-table run (s); a plan cut off counts at the limit")
    ap.add_argument("--eval-cap", type=int, default=100_000_000, help="learned: cap of the evaluation runs")
    ap.add_argument("--eval-limit", type=float, default=2.0, help="learned: time limit of the evaluation runs (s)")
    ap.add_argument("--margin", type=float, default=0.5,
                    help="learned: predicted log2 gain a plan needs over the heuristic one to be proposed")
    ap.add_argument("--probe-cap", type=int, default=10_000_000,
                    help="learned: matches each plan counts when measured runtime judges a proposal (0 = no judge)")
    ap.add_argument("--probe-limit", type=float, default=0.2, help="learned: time limit of each judging run (s)")
    ap.add_argument("--workload", default="large",
                    choices=["medium", "small", "large", "batch", "serve", "learned", "cg", "dense"],
                    help="batch = 10,000 mixed-size queries in shared launches (autotuned); "
                         "serve = the same queries as a Poisson request stream through the server; "
                         "cg = large queries searched on G and on the candidate graph G'; "
                         "dense = small dense queries on a dense graph under each LDS-staging ratio")
    ap.add_argument("--cg-per-size", type=int, default=20, help="cg: queries of each size (16, 24, 32)")
    ap.add_argument("--dense-vertices", type=int, default=8192,
                    help="dense: vertices of the G(n, M) graph (average degree 192)")
    ap.add_argument("--cg-graph", default="rmat", choices=["rmat", "er"],
                    help="cg: R-MAT scale 20 (hubs) or G(n, M) with 2^20 vertices and average degree 16")
    ap.add_argument("--load", type=float, default=0.7,
                    help="serve: offered rate as a fraction of the measured batched throughput")
    ap.add_argument("--slots", type=int, default=0, help="serve: concurrent launches (0 = default)")
    ap.add_argument("--max-batch", type=int, default=0, help="serve: requests per launch (0 = default)")
    ap.add_argument("--no-tune", action="store_true", help="batch workload: keep the default launch settings")
    ap.add_argument("--alone-sample", type=int, default=10,
                    help="batch workload: time every N-th query alone as the one-at-a-time reference")
    ap.add_argument("--queries", type=int, default=0, help="use only the first N queries (0 = all)")
    ap.add_argument("--query-stride", type=int, default=1, help="use every S-th query")
    ap.add_argument("--time-limit", type=float, default=-1.0, help="override the workload's per-query limit")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="oracle time budget for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side-medium", action="store_true",
                    help="large workload: skip the side measurement of the 8-vertex scale-20 workload")
    ap.add_argument("--merge-ratio", type=int, default=0,
                    help="LDS-staged intersection: stage a list when its length <= ratio x the candidates "
                         "testing it (0 = default, -1 = never)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the extra gm_count_batch pass over the same queries (profiling runs)")
    ap.add_argument("--tau", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--disable-stealing", action="store_true")
    ap.add_argument("--stack-layout", type=int, default=0, help="0 auto, 1 full, 2 slim")
    ap.add_argument("--steal-threshold", type=int, default=0)
    ap.add_argument("--hub-cut", type=int, default=0, help="first-phase tasks per root (0 = default 1)")
    ap.add_argument("--no-hub-bitmaps", action="store_true", help="bisect hub lists instead of reading bitmaps")
    ap.add_argument("--hub-mib", type=int, default=0, help="device memory for hub bitmaps in MiB (0 = default)")
    ap.add_argument("--roots-per-item", type=int, default=0,
                    help="first-vertex candidates per first-phase work item, 1..64 (0 = automatic)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB device-to-device (counter calibration)")
    ap.add_argument("--summarize-stats", metavar="DIR", help="print the kernel table of a rocprofv3 --stats run")
    ap.add_argument("--summarize-pmc", metavar="DIR", help="print the search kernel's counters of a rocprofv3 --pmc run")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print the search kernel's dispatch durations of a rocprofv3 --kernel-trace run")
    ap.add_argument("--trace-skip", type=int, default=0, help="summarize-trace: dispatches before the window")
    ap.add_argument("--trace-take", type=int, default=0, help="summarize-trace: dispatches in the window")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print HBM traffic per search launch from two rocprofv3 --pmc runs")
    ap.add_argument("--copy-bytes", type=int, default=0, help="size of the calibration copy in those runs")
    args = ap.parse_args()

    if args.summarize_stats:
        print(summarize_stats(args.summarize_stats))
        return 0
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc))
        return 0
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.trace_skip, args.trace_take))
        return 0
    if args.summarize_traffic:
        fetch = pmc_per_kernel(args.summarize_traffic[0], "FETCH_SIZE")
        write = pmc_per_kernel(args.summarize_traffic[1], "WRITE_SIZE")
        # every build of the search kernel the run dispatched (register budgets differ by
        # query size), weighted by its dispatches, as the bench averages all its launches
        key = "+".join(sorted(k for k in fetch if k.startswith("search<")))
        f_search, n_f = merge_means([fetch[k] for k in fetch if k.startswith("search<")])
        w_search, n_w = merge_means([write[k] for k in write if k.startswith("search<")])
        f_copy = fetch["copy"][0]
        w_copy = write["copy"][0]
        kf = args.copy_bytes / (f_copy * 1024.0)
        kw = args.copy_bytes / (w_copy * 1024.0)
        traffic = f_search * 1024.0 * kf + w_search * 1024.0 * kw
        print(f"kernel: {key}")
        print(f"kernel_sha: {kernel_sha()}")
        print(f"search_fetch_kib_per_dispatch: {f_search:.1f}  (dispatches {n_f})")
        print(f"search_write_kib_per_dispatch: {w_search:.1f}  (dispatches {n_w})")
        print(f"copy_fetch_kib: {f_copy:.1f}  copy_write_kib: {w_copy:.1f}  copy_bytes: {args.copy_bytes}")
        print(f"fetch_scale: {kf:.4f}")
        print(f"write_scale: {kw:.4f}")
        print(f"traffic_bytes_per_launch: {traffic:.0f}")
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported: the engine "
              "searches each query on a single GPU (multi-GPU sharding is a design, not built)", file=sys.stderr)
        return 2

    import paper_2604_10601_amd as gm

    if args.workload == "batch":
        return bench_batch(args, gm)
    if args.workload == "serve":
        return bench_serve(args, gm)
    if args.workload == "learned":
        return bench_learned(args, gm)
    if args.workload == "cg":
        return bench_cg(args, gm)
    if args.workload == "dense":
        return bench_dense(args, gm)

    t = time.time()
    w = make_workload(args.workload, args.queries, args.query_stride)
    if args.time_limit >= 0:
        w.time_limit_s = args.time_limit
    log(f"workload {w.name}: n={w.graph.n} |E|={w.graph.num_edges} queries={len(w.queries)} "
        f"({time.time() - t:.1f} s to generate)")
    opts = dict(tau=args.tau, waves_per_cu=args.waves_per_cu, disable_stealing=args.disable_stealing,
                steal_threshold=args.steal_threshold, stack_layout=args.stack_layout, pool_hub_cut=args.hub_cut,
                disable_hub_bitmaps=args.no_hub_bitmaps, hub_bitmap_mib=args.hub_mib,
                pool_roots_per_item=args.roots_per_item, merge_ratio=args.merge_ratio)
    e = gm.Engine(device=0, **opts)
    t = time.time()
    e.load(w.graph)
    qids = [e.add(q) for q in w.queries]
    phis = [e.get_order(qid) for qid in qids]
    cap = w.cap
    limit = w.time_limit_s
    log(f"graph and queries loaded in {time.time() - t:.1f} s")

    for i in range(args.warmup):
        res = plain_pass(e, qids, cap, limit)
        log(f"warmup {i}: {pass_line(res)}")
    t0 = time.perf_counter()
    steps = []
    for i in range(args.steps):
        steps.append(plain_pass(e, qids, cap, limit))
    t1 = time.perf_counter()
    wall = t1 - t0
    for i, res in enumerate(steps):  # progress is written after the timed region
        log(f"step {i}: {pass_line(res)}")

    flat = [r for s_ in steps for r in s_]
    solved = [r for r in flat if r.outcome != gm.GM_TIMEOUT]
    embeddings = sum(r.count for r in flat)
    tasks = sum(r.tasks for r in flat)
    lat = np.array([r.search_ms for r in flat])
    outcomes = {"done": sum(r.outcome == gm.GM_DONE for r in steps[-1]),
                "capped": sum(r.outcome == gm.GM_CAPPED for r in steps[-1]),
                "timeout": sum(r.outcome == gm.GM_TIMEOUT for r in steps[-1])}

    out = {
        "metric": "embeddings/s",
        "value": embeddings / wall,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1000.0 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "graph_vertices": w.graph.n, "graph_edges": w.graph.num_edges,
                   "queries": len(w.queries), "query_sizes": sorted({q.k for q in w.queries}),
                   "cap": cap, "time_limit_s": limit, "order": "RI heuristic",
                   "initial_pool": (f"breadth-first to tau={args.tau}" if args.tau > 0 else
                                    "first-vertex candidates" if args.tau < 0 else "two-phase pool"),
                   "work_stealing": not args.disable_stealing},
        # the paper's task count: sum of |C^L| over task groups (Sec. 4.1)
        "intersected_edges_per_s": tasks / wall,
        # candidates actually read (label slices of C^L)
        "scanned_candidates_per_s": sum(r.scanned for r in flat) / wall,
        "metric_notes": {"intersected_edges_per_s": "the paper's task count: sum of |C^L| over task groups "
                                                    "(Sec. 4.1), not list entries read",
                         "scanned_candidates_per_s": "candidate ids the kernel actually read (the label "
                                                     "slice of C^L that can match)"},
        "query_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "mean": float(lat.mean())},
        "outcomes_per_step": outcomes,
        "solved_queries": len(solved) // max(1, args.steps),
        "idle_rate": 1.0 - sum(r.lanes_active for r in flat) / max(1, sum(r.lanes_issued for r in flat)),
        "steals_per_step": sum(r.steals for r in flat) // max(1, args.steps),
        # membership tests (list bounds read) and the list entries they examined
        "membership": {"lookups_per_step": sum(r.kernel_lookups for r in flat) // max(1, args.steps),
                       "probes_per_lookup": sum(r.kernel_probes for r in flat) /
                       max(1, sum(r.kernel_lookups for r in flat))},
        "roofline": roofline(flat, traffic_file_for(w.name)),
    }
    if not args.no_batched:
        # the same queries in shared persistent launches (gm_count_batch), one call
        e.count_batch(qids, cap=cap, time_limit_s=limit)
        t0 = time.perf_counter()
        bres, binfo = e.count_batch(qids, cap=cap, time_limit_s=limit)
        bwall = time.perf_counter() - t0
        out["batched"] = {"value": binfo.count / bwall, "unit": "embeddings/s", "ms": bwall * 1000.0,
                          "kernel_ms": binfo.kernel_ms, "launches": binfo.launches,
                          "same_counts": all((a.count, a.outcome) == (b.count, b.outcome)
                                             for a, b in zip(steps[-1], bres)
                                             if a.outcome != gm.GM_TIMEOUT and b.outcome != gm.GM_TIMEOUT)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, phis, args.cpu_seconds, cap, 10.0, steps[-1])
    e.close()
    if args.workload == "large" and not args.no_side_medium:
        out["medium"] = side_medium(gm, opts)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib << 20)
    print(json.dumps(out), flush=True)
    return 0


def plain_pass(e, qids, cap, limit):
    """One step of the plain method: every query counted alone (gm_count), in order."""
    return [e.count(qid, cap=cap, time_limit_s=limit) for qid in qids]


def pass_line(res) -> str:
    import paper_2604_10601_amd as gm
    return (f"{sum(r.count for r in res)} embeddings, {sum(r.search_ms for r in res):.1f} ms search time, "
            f"outcomes done/capped/timeout = {sum(r.outcome == gm.GM_DONE for r in res)}/"
            f"{sum(r.outcome == gm.GM_CAPPED for r in res)}/{sum(r.outcome == gm.GM_TIMEOUT for r in res)}, "
            f"slowest query {max(r.search_ms for r in res):.1f} ms")


def roofline(flat, traffic_file: str) -> dict:
    """HBM roofline of the search kernel over the timed launches: bytes it
    requested (counted by the kernel where each load or store is issued) over its
    device time (HIP events on the engine's stream)."""
    kernel_s = sum(r.kernel_ms for r in flat) / 1000.0
    launches = sum(1 for r in flat if r.kernel_ms > 0)
    issued = sum(r.kernel_bytes for r in flat)
    late = sum(r.kernel_bytes_late for r in flat)
    achieved = issued / kernel_s / 1e9 if kernel_s > 0 else 0.0
    traffic = read_traffic(traffic_file)
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "kernel": "search_kernel (persistent depth-first search)",
        "launches": launches,
        "avg_launch_ms": kernel_s * 1000.0 / max(1, launches),
        "issued_bytes_per_launch": issued / max(1, launches),
        # upper bound on the bytes spent after a query reached its cap (or time limit)
        "late_bytes_per_launch_max": late / max(1, launches),
        "frac_excluding_late": (issued - late) / kernel_s / 1e9 / HBM_PEAK_GBS if kernel_s > 0 else 0.0,
        "traffic_fraction_of_peak": (traffic["bytes_per_launch"] * launches / kernel_s / 1e9 / HBM_PEAK_GBS
                                     if traffic and kernel_s > 0 else None),
    }


def side_medium(gm, opts) -> dict:
    """The 8-vertex workload on the scale-20 graph (100 queries, cap 1e8), three
    passes after one warm-up: a side figure next to the headline."""
    w = make_workload("medium", 0)
    e = gm.Engine(device=0, **opts)
    e.load(w.graph)
    qids = [e.add(q) for q in w.queries]
    plain_pass(e, qids, w.cap, w.time_limit_s)
    t0 = time.perf_counter()
    passes = [plain_pass(e, qids, w.cap, w.time_limit_s) for _ in range(3)]
    wall = time.perf_counter() - t0
    e.close()
    flat = [r for p_ in passes for r in p_]
    lat = np.array([r.search_ms for r in flat])
    rf = roofline(flat, traffic_file_for(w.name))
    return {"workload": w.name, "value": sum(r.count for r in flat) / wall, "unit": "embeddings/s",
            "ms_per_pass": wall * 1000.0 / 3, "query_latency_ms": {"p50": float(np.percentile(lat, 50)),
                                                                   "p99": float(np.percentile(lat, 99))},
            "outcomes_per_pass": {"done": sum(r.outcome == gm.GM_DONE for r in passes[-1]),
                                  "capped": sum(r.outcome == gm.GM_CAPPED for r in passes[-1])},
            "roofline_frac": rf["frac"], "avg_launch_ms": rf["avg_launch_ms"],
            "issued_bytes_per_launch": rf["issued_bytes_per_launch"]}


def bench_batch(args, gm) -> int:
    """Many uneven queries in shared persistent launches (gm_count_batch), after the
    autotuner picked the launch settings on a sample; the reference is the same
    engine counting a sample of the queries one at a time."""
    t = time.time()
    w = make_workload("batch", args.queries, args.query_stride)
    if args.time_limit >= 0:
        w.time_limit_s = args.time_limit
    log(f"workload {w.name}: n={w.graph.n} |E|={w.graph.num_edges} queries={len(w.queries)} "
        f"({time.time() - t:.1f} s to generate)")
    e = gm.Engine(device=0, waves_per_cu=args.waves_per_cu, disable_stealing=args.disable_stealing,
                  steal_threshold=args.steal_threshold, stack_layout=args.stack_layout)
    e.load(w.graph)
    qids = [e.add(q) for q in w.queries]
    cap, limit = w.cap, w.time_limit_s
    tuning = None
    if not args.no_tune:
        sample = qids[::20]
        t = time.time()
        tuning = e.tune_batch(sample, cap=cap, time_limit_s=limit).as_dict()
        log(f"autotuner on {len(sample)} queries ({time.time() - t:.1f} s): {tuning}")
    for i in range(args.warmup):
        e.count_batch(qids, cap=cap, time_limit_s=limit)
    infos, results = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        res, info = e.count_batch(qids, cap=cap, time_limit_s=limit)
        infos.append(info)
        results.append(res)
        log(f"step {i}: {info.count} embeddings in {info.total_ms:.1f} ms ({info.launches} launches)")
    wall = time.perf_counter() - t0
    last = results[-1]
    # one query at a time on a sample, the plain reference
    sample = list(range(0, len(qids), max(1, args.alone_sample)))
    t0 = time.perf_counter()
    alone = [e.count(qids[i], cap=cap, time_limit_s=limit) for i in sample]
    alone_wall = time.perf_counter() - t0
    same = all((a.count, a.outcome) == (last[i].count, last[i].outcome)
               for i, a in zip(sample, alone) if a.outcome != gm.GM_TIMEOUT and last[i].outcome != gm.GM_TIMEOUT)
    embeddings = sum(i.count for i in infos)
    kernel_s = sum(i.kernel_ms for i in infos) / 1000.0
    launches = sum(i.launches for i in infos)
    issued = sum(i.bytes for i in infos)
    achieved = issued / kernel_s / 1e9 if kernel_s > 0 else 0.0
    alone_lat = np.array([a.search_ms for a in alone])
    out = {
        "metric": "embeddings/s",
        "value": embeddings / wall,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1000.0 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "graph_vertices": w.graph.n, "graph_edges": w.graph.num_edges,
                   "queries": len(w.queries), "query_sizes": [min(q.k for q in w.queries),
                                                              max(q.k for q in w.queries)],
                   "cap": cap, "time_limit_s": limit, "order": "RI heuristic", "launch": "gm_count_batch"},
        "queries_per_s": len(qids) * args.steps / wall,
        "outcomes_per_step": {"done": sum(r.outcome == gm.GM_DONE for r in last),
                              "capped": sum(r.outcome == gm.GM_CAPPED for r in last),
                              "timeout": sum(r.outcome == gm.GM_TIMEOUT for r in last)},
        "tuning": tuning,
        "one_at_a_time": {"sample": f"every {max(1, args.alone_sample)}-th query ({len(sample)} queries)",
                          "queries_per_s": len(sample) / alone_wall,
                          "embeddings_per_s": sum(a.count for a in alone) / alone_wall,
                          "latency_ms": {"p50": float(np.percentile(alone_lat, 50)),
                                         "p99": float(np.percentile(alone_lat, 99))},
                          "same_counts_as_batched": same},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "search_kernel (persistent depth-first search, shared by the batch)",
                     "launches": launches, "avg_launch_ms": kernel_s * 1000.0 / max(1, launches),
                     "issued_bytes_per_launch": issued / max(1, launches),
                     "late_bytes_per_launch_max": sum(i.bytes_late for i in infos) / max(1, launches)},
    }
    e.close()
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args, gm) -> int:
    """Continuous batching: the batched workload's queries as a Poisson request
    stream at a fixed rate (a fraction of the measured batched throughput)
    through gm_serve_*, with per-request latency.  Reference: the same arrivals
    served one query at a time by gm_count in a FIFO queue, replayed with every
    query's measured gm_count time."""
    t = time.time()
    w = make_workload("serve", args.queries, args.query_stride)
    if args.time_limit >= 0:
        w.time_limit_s = args.time_limit
    log(f"workload {w.name}: n={w.graph.n} |E|={w.graph.num_edges} queries={len(w.queries)} "
        f"({time.time() - t:.1f} s to generate)")
    e = gm.Engine(device=0)
    e.load(w.graph)
    qids = [e.add(q) for q in w.queries]
    cap, limit = w.cap, w.time_limit_s
    tuning = None if args.no_tune else e.tune_batch(qids[::20], cap=cap, time_limit_s=limit).as_dict()
    e.count_batch(qids, cap=cap, time_limit_s=limit)
    t0 = time.perf_counter()
    bres, _ = e.count_batch(qids, cap=cap, time_limit_s=limit)
    batch_qps = len(qids) / (time.perf_counter() - t0)
    rate = args.load * batch_qps
    log(f"batched throughput {batch_qps:.0f} queries/s; offered load {rate:.0f} requests/s; tuning {tuning}")
    # one query at a time: every query's gm_count time (the service time of a FIFO server)
    t0 = time.perf_counter()
    alone = [e.count(q, cap=cap, time_limit_s=limit) for q in qids]
    alone_wall = time.perf_counter() - t0
    service = np.array([a.search_ms for a in alone]) / 1000.0
    rng = np.random.default_rng(4242)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(qids)))
    fifo_done = np.empty_like(arrivals)
    free_at = 0.0
    for i, (a, sv) in enumerate(zip(arrivals, service)):
        free_at = max(a, free_at) + sv
        fifo_done[i] = free_at
    fifo_lat = (fifo_done - arrivals) * 1000.0
    # the stream through the server
    srv = e.serve(slots=args.slots, max_batch=args.max_batch)
    results = {}
    tickets = {}
    start = time.perf_counter()
    for i, qid in enumerate(qids):
        while time.perf_counter() - start < arrivals[i]:
            for r in srv.poll():
                results[r.ticket] = r
        tickets[srv.submit(qid, cap=cap, time_limit_s=limit)] = i
    while len(results) < len(tickets):
        for r in srv.poll(wait_s=0.01):
            results[r.ticket] = r
    wall = time.perf_counter() - start
    srv.close()
    lat = np.array([r.latency_ms for r in results.values()])
    served = [None] * len(qids)
    for tk, i in tickets.items():
        served[i] = results[tk].result
    same = all((a.count, a.outcome) == (b.count, b.outcome) for a, b in zip(alone, served)
               if a.outcome != gm.GM_TIMEOUT and b.outcome != gm.GM_TIMEOUT)
    embeddings = sum(r.count for r in served)
    slots_used = sorted({r.slot for r in results.values()})
    out = {
        "metric": "embeddings/s",
        "value": embeddings / wall,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": wall * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "graph_vertices": w.graph.n, "graph_edges": w.graph.num_edges,
                   "queries": len(qids), "cap": cap, "time_limit_s": limit, "order": "RI heuristic",
                   "launch": "gm_serve (continuous batching)", "arrivals": "Poisson, seed 4242",
                   "offered_requests_per_s": rate, "load_vs_batched": args.load},
        "serving": {"requests_per_s": len(qids) / wall,
                    "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                   "mean": float(lat.mean())},
                    "slots_used": slots_used, "same_counts_as_alone": same},
        "one_at_a_time": {"requests_per_s_capacity": len(qids) / alone_wall,
                          "fifo_latency_ms": {"p50": float(np.percentile(fifo_lat, 50)),
                                              "p99": float(np.percentile(fifo_lat, 99))},
                          "note": "same arrivals replayed through a one-query FIFO with each query's gm_count time"},
        "batched_queries_per_s": batch_qps,
        "tuning": tuning,
    }
    e.close()
    print(json.dumps(out), flush=True)
    return 0


def bench_learned(args, gm) -> int:
    """Learned plan (matching order and task split): (query, order, split) search
    times measured by the engine on R-MAT scale-20 and scale-22 graphs train the
    cost model; held-out queries on the scale-24 graph then run with the
    heuristic plan (RI order, default split) and with the plan the model picks,
    one query at a time (gm_count) and all together in batched launches
    (gm_count_batch, where the order matters and the split does not).  Counts
    must not change; total time, p50 and p99 are compared."""
    from paper_2604_10601_amd import workloads as wl
    train_cap, train_limit, cap, limit = args.train_cap, args.train_limit, args.eval_cap, args.eval_limit
    n_orders, splits = 4, (1, 4, 16, 64)
    xs, ys, starts = [], [], []
    half = max(1, args.train_queries // 2)
    for scale, seed in ((20, 60), (22, 61)):
        t = time.time()
        g = wl.rmat20_graph() if scale == 20 else wl.rmat22_graph()
        qs = wl.walk_queries(g, wl.order_sizes(half, seed), seed)
        log(f"training graph scale {scale}: |E|={g.num_edges}, {len(qs)} queries ({time.time() - t:.1f} s)")
        with gm.Engine(device=0) as e:
            e.load(g)
            t = time.time()
            for i, q in enumerate(qs):
                qid = e.add(q)
                starts.append(len(ys))
                for o in e.candidate_orders(qid, max_orders=n_orders, seed=i):
                    e.set_order(qid, o)
                    for sp in splits:
                        e.set_split(qid, sp)
                        r = e.count(qid, cap=train_cap, time_limit_s=train_limit)
                        xs.append(e.order_features(qid))
                        ys.append(np.log2(max(r.search_ms, 1e-3)))
                e.free_query(qid)
                if (i + 1) % 250 == 0:
                    log(f"  scale {scale}: {i + 1} queries, {len(ys)} samples ({time.time() - t:.0f} s)")
        del g
    x = np.stack(xs).astype(np.float32)
    y_abs = np.asarray(ys, dtype=np.float32)
    # the model only ranks plans of one query, so it learns each plan's time
    # relative to the mean over that query's plans (log2 units)
    y = y_abs.copy()
    for a, b in zip(starts, starts[1:] + [len(ys)]):
        y[a:b] -= y_abs[a:b].mean()
    rng = np.random.default_rng(7)
    perm = rng.permutation(len(y))
    n_val = max(1, len(y) // 10)
    val, tr = perm[:n_val], perm[n_val:]
    model = gm.Model(gm.ORDER_FEATURES, 128, seed=1)
    t = time.time()
    loss = model.train(x[tr], y[tr], epochs=40, batch=256, lr=1e-3, seed=3)
    pv = model.predict(x[val])
    val_mse = float(np.mean((pv - y[val]) ** 2))
    log(f"model: {len(tr)} training samples, last-epoch mse {loss:.3f}, held-out mse {val_mse:.3f} "
        f"(target variance {float(np.var(y)):.3f}), {time.time() - t:.1f} s")
    # held-out queries on the evaluation graph
    t = time.time()
    g = {20: wl.rmat20_graph, 22: wl.rmat22_graph, 24: wl.rmat24_graph}[args.eval_scale]()
    qs = wl.walk_queries(g, wl.order_sizes(args.eval_queries, 62), 62)
    log(f"evaluation graph scale {args.eval_scale}: |E|={g.num_edges}, {len(qs)} queries ({time.time() - t:.1f} s)")
    plain, learned, other_order, other_split, same = [], [], 0, 0, True
    with gm.Engine(device=0) as e:
        e.load(g)
        qids = [e.add(q) for q in qs]
        heuristic = {}
        mine = {}
        probe_ms = np.zeros(len(qids))
        for i, qid in enumerate(qids):
            if i % 100 == 0:
                log(f"  choosing plans: {i} queries ({time.time() - t:.0f} s)")
            heuristic[qid] = (e.get_order(qid), e.get_split(qid))
            co, cs, _, probe_ms[i] = e.choose_plan(model, qid, splits=splits, max_orders=n_orders, seed=i,
                                                   margin=args.margin, probe_cap=args.probe_cap,
                                                   probe_limit_s=args.probe_limit)
            mine[qid] = (e.get_order(qid), e.get_split(qid))
            other_order += not np.array_equal(mine[qid][0], heuristic[qid][0])
            other_split += mine[qid][1] != heuristic[qid][1]

        def use(qid, plan):
            e.set_order(qid, plan[0])
            e.set_split(qid, plan[1])

        # one query at a time; alternate which plan runs first (neither gains from warm caches)
        for i, qid in enumerate(qids):
            runs = {}
            for which in (("h", "l") if i % 2 == 0 else ("l", "h")):
                use(qid, heuristic[qid] if which == "h" else mine[qid])
                runs[which] = e.count(qid, cap=cap, time_limit_s=limit)
            a, b = runs["h"], runs["l"]
            if a.outcome != gm.GM_TIMEOUT and b.outcome != gm.GM_TIMEOUT:
                same &= (a.count, a.outcome) == (b.count, b.outcome)
            plain.append(a)
            learned.append(b)
            if (i + 1) % 250 == 0:
                log(f"  evaluated {i + 1} queries one at a time ({time.time() - t:.0f} s)")
        # batched launches: every query in one gm_count_batch call per plan, twice each, alternating
        batched = {"h": [], "l": []}
        for rep in range(2):
            for which in (("h", "l") if rep == 0 else ("l", "h")):
                for qid in qids:
                    use(qid, heuristic[qid] if which == "h" else mine[qid])
                t0 = time.perf_counter()
                res, info = e.count_batch(qids, cap=cap, time_limit_s=limit)
                batched[which].append((time.perf_counter() - t0, info, res))
                log(f"  batched launch, {'heuristic' if which == 'h' else 'learned'} plans: "
                    f"{batched[which][-1][0]:.1f} s")
        table = None
        if args.plan_table > 0:
            # every plan of a sample of the queries once: what the best choice per query would save
            tot = {"heuristic": 0.0, "model": 0.0, "best": 0.0}
            pick_rank = []
            sample = list(enumerate(qids))[::args.plan_table]
            for n_done, (i, qid) in enumerate(sample):
                times = []
                for o in e.candidate_orders(qid, max_orders=n_orders, seed=i):
                    for sp in splits:
                        e.set_order(qid, o)
                        e.set_split(qid, sp)
                        r = e.count(qid, cap=cap, time_limit_s=args.plan_table_limit)
                        times.append((r.search_ms, np.array_equal(o, heuristic[qid][0]) and sp == heuristic[qid][1],
                                      np.array_equal(o, mine[qid][0]) and sp == mine[qid][1]))
                ts = np.array([x[0] for x in times])
                tot["heuristic"] += float(ts[[x[1] for x in times]].min())
                tot["model"] += float(ts[[x[2] for x in times]].min())
                tot["best"] += float(ts.min())
                pick_rank.append(int((ts < ts[[x[2] for x in times]].min()).sum()))
                if (n_done + 1) % 10 == 0:
                    log(f"  timed every plan of {n_done + 1} queries ({time.time() - t:.0f} s)")
            # the pick of the last evaluation, for the queries sampled
            table = {"queries": len(sample), "total_ms": tot, "plans_per_query": len(times),
                     "model_pick_rank_mean": float(np.mean(pick_rank)),
                     "time_limit_s": args.plan_table_limit,
                     "note": "every plan of every sampled query timed once, one query at a time, with the "
                             "time limit above; rank 0 = the fastest plan"}
        bh, bl = batched["h"][-1][2], batched["l"][-1][2]
        same_batched = all((a.count, a.outcome) == (b.count, b.outcome) for a, b in zip(bh, bl)
                           if a.outcome != gm.GM_TIMEOUT and b.outcome != gm.GM_TIMEOUT)
        same_batched &= all((a.count, a.outcome) == (b.count, b.outcome) for a, b in zip(bh, plain)
                            if a.outcome != gm.GM_TIMEOUT and b.outcome != gm.GM_TIMEOUT)
    model.close()
    lp = np.array([r.search_ms for r in plain])
    ll = np.array([r.search_ms for r in learned]) + probe_ms   # the judge's probes are the learned plan's cost

    def batch_summary(which):
        walls = [w for w, _, _ in batched[which]]
        res = batched[which][-1][2]
        qms = np.array([r.query_ms for r in res])
        return {"wall_ms": 1000.0 * float(min(walls)), "kernel_ms": float(min(i.kernel_ms for _, i, _ in batched[which])),
                "query_p50_ms": float(np.percentile(qms, 50)), "query_p99_ms": float(np.percentile(qms, 99)),
                "timeouts": int(sum(r.outcome == gm.GM_TIMEOUT for r in res))}

    out = {
        "metric": "query-set time (ms), learned vs heuristic plan",
        "value": float(ll.sum()),
        "unit": "ms",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": float(ll.sum()),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 search, bf16/fp32 model",
        "data": "synthetic",
        "config": {"workload": f"learned plan: train R-MAT 20+22, evaluate R-MAT {args.eval_scale}",
                   "train_queries": 2 * half, "orders_per_query": n_orders, "splits": list(splits),
                   "samples": int(len(y)), "train_cap": train_cap, "train_time_limit_s": train_limit,
                   "eval_queries": len(qs), "cap": cap, "time_limit_s": limit, "margin_log2": args.margin,
                   "target": "log2 search ms minus the query's mean over its plans",
                   "judge": {"probe_cap": args.probe_cap, "probe_time_limit_s": args.probe_limit}},
        "heuristic": {"total_ms": float(lp.sum()), "p50_ms": float(np.percentile(lp, 50)),
                      "p99_ms": float(np.percentile(lp, 99)),
                      "timeouts": int(sum(r.outcome == gm.GM_TIMEOUT for r in plain))},
        "learned": {"total_ms": float(ll.sum()), "p50_ms": float(np.percentile(ll, 50)),
                    "p99_ms": float(np.percentile(ll, 99)),
                    "timeouts": int(sum(r.outcome == gm.GM_TIMEOUT for r in learned)),
                    "probe_ms_included": float(probe_ms.sum()),
                    "queries_probed": int((probe_ms > 0).sum()),
                    "queries_with_another_order": int(other_order), "queries_with_another_split": int(other_split)},
        "batched": {"heuristic": batch_summary("h"), "learned": batch_summary("l"), "same_counts": bool(same_batched)},
        "model": {"train_mse": loss, "heldout_mse": val_mse, "target_variance": float(np.var(y))},
        "plan_table": table,
        "same_counts": bool(same),
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_dense(args, gm) -> int:
    """LDS-staged intersection where it applies: G(n, M) with 8,192 vertices (or
    --dense-vertices), average degree 192 (no vertex reaches the hub degree) and one
    label, so every list is a
    whole neighbour list of about 192 entries and a parent's candidates fill runs of
    64 lanes; dense queries of 4 and 5 vertices.  Every query is counted alone under
    merge ratios never, 1, 2, 4 and 8; counts must agree, total time is compared."""
    from paper_2604_10601_amd import workloads as wl
    n, deg = args.dense_vertices, 192
    rp, col = wl.erdos_renyi(n, n * deg // 2, seed=7301)
    g = wl.Graph(rp, col, np.zeros(n, dtype=np.int32))
    shapes = {"triangle": [(0, 1), (1, 2), (2, 0)],
              "4-cycle": [(0, 1), (1, 2), (2, 3), (3, 0)],
              "diamond": [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)],
              "4-clique": [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
              "5-cycle with chord": [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 2)]}
    queries = []
    for name, edges in shapes.items():
        k = 1 + max(max(e) for e in edges)
        pairs = np.asarray([sorted(e) for e in edges], dtype=np.int32)
        queries.append((name, wl.Query(k, pairs, np.zeros(k, dtype=np.int32))))
    cap, limit = 10**10, 20.0
    runs = {}
    for ratio in (-1, 1, 2, 4, 8):
        with gm.Engine(device=0, merge_ratio=ratio) as e:
            e.load(g)
            qids = [e.add(q) for _, q in queries]
            e.count(qids[0], cap=cap, time_limit_s=limit)  # warm-up
            res = [e.count(qid, cap=cap, time_limit_s=limit) for qid in qids]
        runs[ratio] = res
        log(f"merge ratio {ratio}: {sum(r.search_ms for r in res):.1f} ms")
    base = runs[-1]
    same = all((a.count, a.outcome) == (b.count, b.outcome) for r in runs.values() for a, b in zip(base, r))
    per = {str(ratio): {"total_ms": float(sum(r.search_ms for r in res)),
                        "per_query_ms": {name: float(r.search_ms) for (name, _), r in zip(queries, res)},
                        "probes_per_lookup": float(sum(r.kernel_probes for r in res) /
                                                   max(1, sum(r.kernel_lookups for r in res)))}
           for ratio, res in runs.items()}
    best = min(runs, key=lambda x: per[str(x)]["total_ms"])
    out = {
        "metric": "embeddings/s",
        "value": sum(r.count for r in runs[best]) / (per[str(best)]["total_ms"] / 1000.0),
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": per[str(best)]["total_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"er{n}_d192_1label_dense4-5", "graph_vertices": n, "graph_edges": g.num_edges,
                   "queries": [name for name, _ in queries], "cap": cap, "time_limit_s": limit},
        "by_merge_ratio": per,
        "counts": {name: int(r.count) for (name, _), r in zip(queries, base)},
        "outcomes": {name: int(r.outcome) for (name, _), r in zip(queries, base)},
        "best_ratio": best,
        "speedup_best_vs_never": per["-1"]["total_ms"] / per[str(best)]["total_ms"],
        "same_counts": bool(same),
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_cg(args, gm) -> int:
    """Candidate graph: the same large queries searched on G and on G' (built per
    query on the device, its build inside each query's time).  Counts of queries
    that finish in both modes must agree; total time and p50/p99 are compared."""
    from paper_2604_10601_amd import workloads as wl
    t = time.time()
    w = wl.cg_rmat20(per_size=args.cg_per_size) if args.cg_graph == "rmat" else wl.cg_er20(per_size=args.cg_per_size)
    if args.time_limit >= 0:
        w.time_limit_s = args.time_limit
    log(f"workload {w.name}: n={w.graph.n} |E|={w.graph.num_edges} queries={len(w.queries)} "
        f"({time.time() - t:.1f} s to generate)")
    runs = {}
    for mode in ("plain", "candidate_graph"):
        with gm.Engine(device=0, candidate_graph=(mode == "candidate_graph"),
                       pool_roots_per_item=args.roots_per_item) as e:
            e.load(w.graph)
            qids = [e.add(q) for q in w.queries]
            e.count(qids[0], cap=w.cap, time_limit_s=w.time_limit_s)  # warm-up
            res = []
            t = time.time()
            for i, qid in enumerate(qids):
                res.append(e.count(qid, cap=w.cap, time_limit_s=w.time_limit_s))
                if (i + 1) % 10 == 0:
                    log(f"  {mode}: {i + 1} queries ({time.time() - t:.1f} s)")
            runs[mode] = res
    plain, cg = runs["plain"], runs["candidate_graph"]
    both_done = [(a, b) for a, b in zip(plain, cg) if a.outcome != gm.GM_TIMEOUT and b.outcome != gm.GM_TIMEOUT]
    same = all((a.count, a.outcome) == (b.count, b.outcome) for a, b in both_done)

    def summary(rs):
        ms = np.array([r.search_ms for r in rs])
        cnt = sum(r.count for r in rs)
        return {"total_ms": float(ms.sum()), "p50_ms": float(np.percentile(ms, 50)),
                "p99_ms": float(np.percentile(ms, 99)), "embeddings": int(cnt),
                "embeddings_per_s": float(cnt / (ms.sum() / 1e3)) if ms.sum() > 0 else 0.0,
                "outcomes": {"done": sum(r.outcome == gm.GM_DONE for r in rs),
                             "capped": sum(r.outcome == gm.GM_CAPPED for r in rs),
                             "timeout": sum(r.outcome == gm.GM_TIMEOUT for r in rs)}}

    sp, sc = summary(plain), summary(cg)
    sc["build_ms_total"] = float(sum(r.candidate_ms for r in cg))
    sc["search_ms_without_build"] = sc["total_ms"] - sc["build_ms_total"]
    sc["filter_sweeps_mean"] = float(np.mean([r.candidate_rounds for r in cg]))
    sc["list_entries_mean"] = float(np.mean([r.candidate_edges for r in cg]))
    sc["roots_mean"] = float(np.mean([r.pool_rows for r in cg]))
    sp["roots_mean"] = float(np.mean([r.pool_rows for r in plain]))
    out = {
        "metric": "embeddings/s",
        "value": sc["embeddings_per_s"],
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": sc["total_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "graph_vertices": int(w.graph.n), "graph_edges": int(w.graph.num_edges),
                   "queries": len(w.queries), "query_sizes": sorted({int(q.k) for q in w.queries}),
                   "cap": w.cap, "time_limit_s": w.time_limit_s, "order": "RI heuristic"},
        "plain": sp,
        "candidate_graph": sc,
        "speedup_total_time": sp["total_ms"] / sc["total_ms"] if sc["total_ms"] > 0 else None,
        "compared_queries": len(both_done),
        "same_counts": bool(same),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
