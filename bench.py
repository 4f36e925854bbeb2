"""Benchmark: batch fully dynamic exact 4-graphlet counting on one MI355X.

Workload: R-MAT scale 22, edge factor 16 (n = 4,194,304, m = 67,108,864 after
dedupe and loop removal, a=0.57 b=0.19 c=0.19, seeded id permutation),
resident on the GPU; a stream of update batches with sizes log-uniform in
[10, 1e5], half deletions of uniform existing edges, half insertions from the
same R-MAT generator.  One step = one batch through the whole path (ingest,
merge, region of change, fused two-version count, combine, purge), timed from
the host call to the counts on the host (result download included).  The
timed batches are resident in HBM before the timed region and go through the
device-array entry point.

Checks: the counts of the initial graph and after the last batch are compared
with the oracle's static recount stored in tests/golden (written by
tests/golden/make_scale.py from the oracle alone), and with a static recount
on the GPU.  The graph is then taken back to its state before the timed
batches (one net batch) and the same timed batches run again through the
host-array entry point: the PCIe-inclusive rate, never ``value``, and the
counts must come out the same.

Also in the same line (skipped with --no-served / --no-batched): the served
form (continuous batching into multi-version passes, Poisson arrivals at
0.5x, 0.9x and 1.5x the plain path's saturation rate) and the batched form
(256 graphs in one pooled pass against one call per graph).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form plain|batched|served]

Prints one JSON line.  The oracle (test infrastructure) is used only by the
cpu_baseline leg.
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

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = max(0, min(len(xs) - 1, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


def read_kv(path):
    kv = {}
    if os.path.exists(path):
        for line in open(path):
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def measured_traffic(kernel_file, summary):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None once the kernel source differs from the one the counters saw."""
    import hashlib
    kv = read_kv(os.path.join(ROOT, "profiles", summary))
    src = os.path.join(ROOT, "paper_2308_14493_amd", "csrc", kernel_file)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if kv.get("source_sha256_prefix") != sha or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "cpu_model": model}


def golden_counts(w, steps):
    """Oracle counts stored for this stream (step j = after j batches), keyed
    by the digest of the graph and its first j batches; {} if none match."""
    from graphgen import workloads as wl
    path = os.path.join(ROOT, "tests", "golden", "scale_rmat_s22_bench.json")
    if not os.path.exists(path):
        return {}
    g = json.load(open(path))
    have = dict(zip(g.get("prefix_sha256", []), g["counts"]))
    out = {}
    for j in steps:
        c = have.get(wl.prefix_digest(w, j))
        if c is not None:
            out[j] = c
    return out


def cpu_baseline(n, s, d, mean_batch, stride, scale, ef):
    """The oracle's static recount (the per-batch work of the
    recount-from-scratch baseline) of the benchmark graph, timed on a
    bounded sample: the adjacency build in full, the per-vertex loops over
    every stride-th vertex (ids are randomly permuted, so a uniform sample),
    scaled by the stride.  Also reports the full recount of the same graph
    measured on this kind of host, when a profile of it is committed."""
    from oracle import native
    native.build()
    t_build, t_loops = native.sample_seconds(n, s, d, stride, 0)
    est = t_build + stride * t_loops
    hi = host_info()
    out = {"value": mean_batch / est, "unit": "updates/s", "cores": native.threads(), "kind": "oracle",
           "sample": "oracle static recount of the benchmark graph, R-MAT scale %d ef %d (m=%d): adjacency build "
                     "%.1fs in full, per-vertex loops over 1 vertex in %d %.1fs, scaled: %.0fs per recount on %d "
                     "threads (%s); updates/s = mean batch size %.0f / recount time" % (
                         scale, ef, s.size, t_build, stride, t_loops, est, native.threads(), hi["cpu_model"],
                         mean_batch),
           "recount_s_estimated": est, "host": hi}
    kv = read_kv(os.path.join(ROOT, "profiles", "cpu_oracle_rmat_s22.md"))
    if "full_recount_s" in kv and scale == 22 and ef == 16:
        out["full_recount_s_measured"] = float(kv["full_recount_s"])
        out["full_recount_threads"] = int(kv.get("threads", "0"))
        out["full_recount_cpu_model"] = kv.get("cpu_model", "")
        out["single_thread_recount_s_rmat_s18_ef8"] = float(kv.get("single_thread_s18_ef8_s", "nan"))
    return out


# ------------------------------------------------------------------ forms
def run_batched(args):
    """Many independent R-MAT graphs (n log-uniform in [1e3, 2e5], edge factor
    in {4, 8, 16}), one update batch per graph per round (log-uniform in
    [100, 1e4], 50/50, the same size every round): one pooled pass per round
    for all graphs, replayed from a captured HIP graph, against the same pool
    launching kernel by kernel and against one call per graph.  Every form
    first applies the same warm-up rounds (the autotuner's ten trial passes --
    hub-window and tier thresholds -- then the capture); the timed rounds
    follow."""
    from graphgen import rmat_graph, rmat_batches
    import paper_2308_14493_amd as pkg
    import torch
    rng = np.random.default_rng(4)
    t0 = time.time()
    warm, rounds = 11, args.rounds
    work = []
    for i in range(args.graphs):
        n = int(round(10 ** rng.uniform(3, math.log10(2e5))))
        ef = int(rng.choice([4, 8, 16]))
        size = int(round(10 ** rng.uniform(2, 4)))
        scale = max(1, math.ceil(math.log2(n)))
        gs = int(rng.integers(0, 2**31 - 1))
        n, s, d, samp = rmat_graph(scale, ef, gs, n=n)
        work.append((n, s, d, rmat_batches(n, s, d, samp, [size] * (warm + rounds), gs + 1)))
    m_tot = sum(w[1].size for w in work)
    log("batched: generated %d graphs (sum m = %d) in %.1fs" % (len(work), m_tot, time.time() - t0))
    pkg.load()
    torch.cuda.init()
    offered = [sum(w[3][warm + r][0].size + w[3][warm + r][2].size for w in work) for r in range(rounds)]

    def pooled(graphs):
        pool = pkg.Graph.pool([w[0] for w in work], [w[1] for w in work], [w[2] for w in work],
                              radius=args.radius, graphs=graphs)
        for r in range(warm):
            pool.apply_batches([w[3][r] for w in work])
        times, res = [], []
        for r in range(rounds):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            res.append(pool.apply_batches([w[3][warm + r] for w in work]))
            times.append(time.perf_counter() - t1)
        rep = pool.graph_replays()
        pool.close()
        return times, res, rep

    t_graph, r_graph, rep = pooled(1)
    log("batched: pooled pass, replayed graph: %s ms (captures %d, graph launches %d)" %
        (["%.2f" % (t * 1e3) for t in t_graph], rep[0], rep[1]))
    t_direct, r_direct, _ = pooled(0)
    log("batched: pooled pass, kernel by kernel: %s ms" % ["%.2f" % (t * 1e3) for t in t_direct])
    # graph by graph, kernel by kernel, every timed round
    seq, t_seq = [[] for _ in range(rounds)], [0.0] * rounds
    for n, s, d, bs in work:
        g = pkg.Graph(n, s, d, radius=args.radius, graphs=0)
        for r in range(warm):
            g.apply_batch(*bs[r])
        for r in range(rounds):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            seq[r].append(g.apply_batch(*bs[warm + r]))
            t_seq[r] += time.perf_counter() - t1
        g.close()
    log("batched: graph by graph: %s ms" % ["%.2f" % (t * 1e3) for t in t_seq])
    same = seq == r_graph and r_graph == r_direct
    tg = float(np.mean(t_graph))
    return {"graphs": len(work), "sum_m": m_tot, "rounds": rounds, "warmup_rounds": warm,
            "updates_per_s": float(np.mean(offered)) / tg, "ms_per_round": tg * 1e3,
            "direct_pool_ms": float(np.mean(t_direct)) * 1e3,
            "sequential_updates_per_s": float(np.sum(offered)) / float(np.sum(t_seq)),
            "sequential_ms_per_round": float(np.mean(t_seq)) * 1e3,
            "speedup_vs_sequential": float(np.mean(t_seq)) / tg,
            "graph_captures": rep[0], "graph_launches": rep[1], "results_equal": bool(same)}


def run_served(args, n, s, d, sampler):
    """Serving: the graph resident in a server; one fixed sequence of batches
    (sizes log-uniform in [min, max], 50/50) is offered as a Poisson stream
    at 0.5x, 0.9x and 1.5x the saturation rate of the plain path (1 / mean
    service time, measured on the same sequence through the server one
    request at a time).  Between rates one net batch takes the graph back to
    where the sequence started, so every rate sees the same sequence on the
    same graph and every result must equal the one-at-a-time result.
    Latency = submit -> counts on the host."""
    import threading
    from graphgen import BatchStream, log_uniform_sizes, poisson_arrivals
    from graphgen.workloads import net_batch
    import paper_2308_14493_amd as pkg
    import torch
    t0 = time.time()
    sizes = log_uniform_sizes(args.requests, args.min_batch, args.max_batch, args.seed + 5)
    stream = BatchStream.from_edges(n, s, d, args.seed + 6, ins_sampler=sampler)
    keys0 = stream.keys.copy()
    batches = [stream.next_batch(sz // 2, sz - sz // 2) for sz in sizes]
    restore = net_batch(stream.keys, keys0)
    offered = sum(b[0].size + b[2].size for b in batches)
    log("served: generated %d batches in %.1fs" % (len(batches), time.time() - t0))
    pkg.load()
    torch.cuda.init()
    srv = pkg.Server()
    gid = srv.add_graph(n, s, d, radius=args.radius)
    base = srv.counts(gid)

    def closed_loop(seq):
        return [srv.wait(srv.submit(gid, *b)) for b in seq]

    closed_loop(batches[:1] + [(batches[0][2], batches[0][3], batches[0][0], batches[0][1])])  # warm-up
    t1 = time.perf_counter()
    plain = closed_loop(batches)
    t_plain = time.perf_counter() - t1
    final = srv.counts(gid)
    closed_loop([restore])
    assert srv.counts(gid) == base
    service = t_plain / len(batches)
    runs = {}
    for f in (0.5, 0.9, 1.5):
        arr = poisson_arrivals(f / service, len(batches), args.seed + int(f * 10))
        tickets = [None] * len(batches)
        start = time.perf_counter()

        def feeder():
            for i, b in enumerate(batches):
                dt = start + arr[i] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(gid, *b)

        th = threading.Thread(target=feeder)
        th.start()
        lat, same, passes = [], True, []
        for i in range(len(batches)):
            while tickets[i] is None:
                time.sleep(0.0005)
            c, st, l, q = srv.wait(tickets[i])
            lat.append(l)
            passes.append(st["pass_batches"])
            same &= [int(x) for x in c] == [int(x) for x in plain[i][0]]
        end = time.perf_counter()
        th.join()
        assert srv.counts(gid) == final
        runs["%.1fx" % f] = {"offered_rate_batches_per_s": f / service, "updates_per_s": offered / (end - start),
                             "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                             "mean_batches_per_pass": float(np.mean(passes)),
                             "results_equal_to_plain": bool(same)}
        log("served: rate %.1fx: %s" % (f, runs["%.1fx" % f]))
        closed_loop([restore])
        assert srv.counts(gid) == base
    srv.close()
    lat_plain = [p[2] for p in plain]
    best = max(r["updates_per_s"] for r in runs.values())
    return {"requests": len(batches), "plain_closed_loop_updates_per_s": offered / t_plain,
            "plain_service_ms": service * 1e3,
            "plain_p50_ms": percentile(lat_plain, 50), "plain_p99_ms": percentile(lat_plain, 99),
            "best_served_updates_per_s": best, "served_vs_plain": best / (offered / t_plain),
            "results_equal_to_plain": all(r["results_equal_to_plain"] for r in runs.values()), "rates": runs}


def run_protocol(args):
    """The paper's experimental protocol (Sec. 6) on stand-ins of its four
    graphs (Table 1 sizes): the edges in a seeded order, the graph built from
    all but the last ones, then insert-only batches of 10 and of 100 (Alg. 1)
    and fully dynamic batches of 100 with the p = 0.7 labelling (Alg. 2),
    each stream on a fresh copy of that graph.  Reported per stream: the
    cumulative time after every batch (Figs. 2-4), and the baseline that
    recounts the whole graph after every batch (the oracle's static recount,
    timed once per graph on the whole edge list -- every stream ends within
    20,000 edges of it -- times the batch count)."""
    from graphgen import protocol
    import paper_2308_14493_amd as pkg
    import torch
    from oracle import native
    pkg.load()
    torch.cuda.init()
    # one call on a tiny graph first: the library load and the start of its
    # thread pool are not part of any graph's recount time
    native.static_counts(4, np.array([0, 1, 2], np.int32), np.array([1, 2, 3], np.int32))
    out = {}
    for name in args.protocol_graphs.split(","):
        t0 = time.time()
        n, s, d = protocol.table1_standin(name, 11)
        s, d = protocol.edge_order(s, d, 12)
        K = args.protocol_batches
        res = {"n": n, "m": int(s.size)}
        streams = {
            "insert_10": (s.size - 10 * K, lambda m0: protocol.incremental_batches(s, d, 10, start=m0, count=K)),
            "insert_100": (s.size - 100 * K, lambda m0: protocol.incremental_batches(s, d, 100, start=m0, count=K)),
            "dynamic_100": (s.size - int(100 * K / 0.7 * 1.1), lambda m0: protocol.fully_dynamic_batches(
                s[m0:], d[m0:], 100, 0.7, 13, count=K, lag=1000)),
        }
        log("protocol %s: n=%d m=%d drawn in %.1fs" % (name, n, s.size, time.time() - t0))
        t1 = time.perf_counter()
        native.static_counts(n, s, d)
        rec = time.perf_counter() - t1
        res["baseline_recount_s"] = rec
        log("protocol %s: oracle recount of the whole graph %.1fs" % (name, rec))
        for key, (m0, make) in streams.items():
            batches = make(m0)
            g = pkg.Graph(n, s[:m0], d[:m0], radius=args.radius, delta=args.delta)
            cum, tot = [], 0.0
            lat = []
            for b in batches:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                g.apply_batch(*b)
                dt = time.perf_counter() - t1
                tot += dt
                lat.append(dt * 1e3)
                cum.append(tot)
            g.close()
            step = max(1, len(cum) // 10)
            res[key] = {"m_start": int(m0), "batches": len(batches), "gpu_total_s": tot,
                        "gpu_p50_ms": percentile(lat, 50), "gpu_p99_ms": percentile(lat, 99),
                        "baseline_total_s": rec * len(batches),
                        "speedup_vs_baseline": rec * len(batches) / max(tot, 1e-9),
                        "cumulative_s": {str(i + 1): round(cum[i], 4) for i in range(step - 1, len(cum), step)}}
            log("protocol %s %s: %d batches, GPU %.3fs (p50 %.2f ms), baseline %.1fs per batch" % (
                name, key, len(batches), tot, res[key]["gpu_p50_ms"], rec))
        out[name] = res
    return out


def form_line(args, metric, value, ms, extra):
    out = {"metric": metric, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic"}
    out.update(extra)
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ plain
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--ef", type=int, default=16)
    ap.add_argument("--seed", type=int, default=22)
    ap.add_argument("--min-batch", type=float, default=10)
    ap.add_argument("--max-batch", type=float, default=1e5)
    ap.add_argument("--radius", type=int, default=2)
    ap.add_argument("--delta", type=int, default=0,
                    help="edge-local passes: 1 always, -1 never, 0 the faster kind per batch-size decade (default)")
    ap.add_argument("--cpu-stride", type=int, default=16, help="cpu_baseline: every stride-th vertex is timed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recount-check", action="store_true")
    ap.add_argument("--no-host-rerun", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--protocol-graphs", default="WikiVote,WikiTalk,Pokec,LiveJournal")
    ap.add_argument("--protocol-batches", type=int, default=200)
    ap.add_argument("--form", choices=["plain", "batched", "served", "protocol"], default="plain",
                    help="plain (default; the served and batched forms ride along as extra keys), or one of the "
                         "other forms alone")
    ap.add_argument("--graphs", type=int, default=256)
    ap.add_argument("--requests", type=int, default=64, help="served form: batches per offered rate")
    ap.add_argument("--rounds", type=int, default=3, help="batched form: timed rounds")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB copied device-to-device once before the batches (a plain copy kernel of known size, "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: runs on one GPU; --gpus %d is not supported "
              "(sharding a graph over several GPUs is not implemented)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    from graphgen import workloads as wl
    import paper_2308_14493_amd as pkg

    if args.form == "protocol":
        pr = run_protocol(args)
        tot = sum(v[k]["batches"] * (100 if k.endswith("100") else 10) for v in pr.values()
                  for k in ("insert_10", "insert_100", "dynamic_100"))
        secs = sum(v[k]["gpu_total_s"] for v in pr.values() for k in ("insert_10", "insert_100", "dynamic_100"))
        return form_line(args, "updates/sec, the paper's protocol (Sec. 6) on Table 1 stand-ins", tot / secs,
                         secs * 1e3 / max(1, args.protocol_batches), {
                             "config": {"workload": "stand-ins of %s; insert-only batches of 10 and 100, fully "
                                                    "dynamic batches of 100 (p = 0.7), %d batches each"
                                                    % (args.protocol_graphs, args.protocol_batches),
                                        "form": "protocol"}, "protocol": pr})
    if args.form == "batched":
        b = run_batched(args)
        return form_line(args, "updates/sec, %d-graph pool, one batch per graph" % b["graphs"], b["updates_per_s"],
                         b["ms_per_round"], {"config": {"workload": "%d R-MAT graphs, n log-uniform [1e3, 2e5], ef "
                                                        "{4,8,16}, one batch per graph per round log-uniform "
                                                        "[100, 1e4], 50/50" % b["graphs"], "form": "batched"},
                                             "batched": b})

    t0 = time.time()
    total = args.warmup + args.steps
    w, sizes, stream = wl.rmat_s22_bench_stream(total, 0, args.min_batch, args.max_batch, args.scale, args.ef,
                                                args.seed, snapshot_at=args.warmup)
    n, s, d = w.n, w.src, w.dst
    log("generated R-MAT scale %d ef %d: n=%d m=%d and %d batches in %.1fs (sizes %s)" % (
        args.scale, args.ef, n, s.size, total, time.time() - t0, sizes))
    if args.form == "served":
        sv = run_served(args, n, s, d, stream.ins_sampler)
        return form_line(args, "updates/sec + p50/p99 batch latency, served, exact 4-graphlet counts, R-MAT s%d"
                         % args.scale, sv["best_served_updates_per_s"], sv["plain_service_ms"],
                         {"config": {"workload": "R-MAT scale %d ef %d, %d batches log-uniform [%g, %g], Poisson "
                                                 "arrivals at 0.5/0.9/1.5x plain saturation" % (
                                                     args.scale, args.ef, sv["requests"], args.min_batch,
                                                     args.max_batch), "form": "served"}, "served": sv})
    gold = golden_counts(w, [0, total])

    pkg.load()
    import torch  # device plumbing only
    torch.cuda.init()
    if args.calibrate_copy:
        src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calibrate_copy)
        del src, dst
    t0 = time.time()
    g = pkg.Graph(n, s, d, radius=args.radius, delta=args.delta)
    torch.cuda.synchronize()
    c0 = g.counts()
    log("graph resident on the GPU in %.2fs; counts %s" % (time.time() - t0, c0))
    checks = {}
    if 0 in gold:
        checks["initial"] = c0 == gold[0]

    # batches resident in HBM before the timed region (device-array entry point)
    batches = w.batches
    dev_batches = [[torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32)).cuda() for x in b] for b in batches]
    torch.cuda.synchronize()
    lat, offered, stats = [], 0, []
    for i, (b, db) in enumerate(zip(batches, dev_batches)):
        if i == args.warmup:
            torch.cuda.synchronize()
            tstart = time.perf_counter()
        t1 = time.perf_counter()
        _, st = g.apply_batch_dev(*db, stats=True)
        t2 = time.perf_counter()
        if i >= args.warmup:
            lat.append((t2 - t1) * 1e3)
            offered += b[0].size + b[2].size
            stats.append(st)
        log("step %d: batch %d updates, %.2f ms (tri %.2f edge %.2f c4 %.2f/%.2f/%.2f prep %.2f fin %.2f) dmin %d "
            "tiers %d/%d/%d whole %d delta %d region_e=%d c4_tail=%d/%d hubs=%d windows=%d searches=%d tri_e=%d" % (
                i, b[0].size + b[2].size, (t2 - t1) * 1e3, st["ms_tri"], st["ms_edge"], st["ms_c4_small"],
                st["ms_c4_mid"], st["ms_c4_large"], st["ms_prepare"], st["ms_finish"], st["c4_dense_min"],
                st["tri_small_max"], st["c4_small_max"], st["c4_mid_max"],
                st["whole_graph"], st["delta"], st["region_entries"], st["c4_tail_wedges"], st["wedges"],
                st["tier_c4_large"], st["c4_windows"], st["c4_searches"], st["tri_entries"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tstart
    value = offered / elapsed
    c_end = g.counts()
    if total in gold:
        checks["after_last_batch"] = c_end == gold[total]
    log("oracle check: %s" % checks)
    recount_ok = None
    if not args.no_recount_check:
        recount_ok = g.recount() == c_end
        log("maintained counts == GPU static recount: %s" % recount_ok)

    # the same timed batches again as host arrays (upload over PCIe included),
    # from the same graph: one net batch takes it back first
    host_rate, host_same = None, None
    if not args.no_host_rerun and args.steps > 0:
        back = wl.net_batch(stream.keys, stream.snapshot)
        g.apply_batch(*back)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for b in batches[args.warmup:]:
            g.apply_batch(*b)
        host_rate = offered / (time.perf_counter() - t1)
        host_same = g.counts() == c_end
        log("host-array (PCIe-inclusive) rate over the same %d batches: %.1f updates/s, counts equal: %s" %
            (args.steps, host_rate, host_same))

    # rooflines: the large 4-cycle tier (the dominant kernel, one launch per
    # batch) and the triangle tiers; algorithmic bytes = 4 B per adjacency
    # entry the method reads (counted by the kernels)
    # per launch: over the passes that ran the kernel (region passes; an
    # edge-local pass runs none of them)
    ran = [st for st in stats if not st["delta"]]
    nl = max(1, len(ran))
    phases = ["ms_tri", "ms_edge", "ms_c4_small", "ms_c4_mid", "ms_c4_large"]
    tot = {p: sum(st[p] for st in ran) for p in phases}
    dom = max(tot, key=tot.get)

    def roof(kernel, bytes_, ms, traffic):
        if not ran or ms <= 0:  # no timed pass ran the kernel: nothing to report
            return {"kernel": kernel, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": None, "traffic": traffic, "bytes_per_launch": None, "avg_launch_ms": None,
                    "launches": 0, "traffic_frac": None}
        ach = bytes_ / (ms / 1e3) / 1e9
        return {"kernel": kernel, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": traffic, "bytes_per_launch": bytes_ / nl,
                "avg_launch_ms": ms / nl, "launches": len(ran),
                "traffic_frac": round(traffic / (ms / nl / 1e3) / 1e9 / HBM_PEAK_GBS, 5) if traffic else None}

    # the compulsory bytes of a region pass: the region's rows read once
    # (4 B per entry, 16 B per vertex for its offset, length and degrees)
    comp = None
    if ran:
        cb = [4.0 * st["region_entries"] + 16.0 * st["region_vertices"] for st in ran]
        cms = [st["ms_total"] for st in ran]
        comp = {"bytes_per_region_pass": sum(cb) / len(cb), "GBps": sum(cb) / (sum(cms) / 1e3) / 1e9,
                "unit": "GB/s", "over": "wall time of the region passes"}
    s22 = args.scale == 22 and args.ef == 16
    roof_c4 = roof("k_c4_large", sum(4.0 * st["c4_entries_large"] for st in ran), tot["ms_c4_large"],
                   measured_traffic("count.hip", "pmc_k_c4_large_rmat_s22.md") if s22 else None)
    roof_c4.update({"dominant_phase": dom, "phase_ms_avg_region_passes": {p: round(tot[p] / nl, 3) for p in phases},
                    "edge_local_passes": len(stats) - len(ran)})
    roof_tri = roof("k_tri_small + k_tri_large tiers", sum(4.0 * st["tri_entries"] for st in ran), tot["ms_tri"],
                    measured_traffic("count.hip", "pmc_tri_tiers_rmat_s22.md") if s22 else None)
    # speed knobs as the autotuner left them: those of the last timed region
    # pass, and which kind of pass each timed batch ran
    last_region = [st for st in stats if not st["delta"]]
    tuned = None
    if last_region:
        lr = last_region[-1]
        tuned = {"c4_dense_min": lr["c4_dense_min"], "tri_small_max": lr["tri_small_max"],
                 "c4_small_max": lr["c4_small_max"], "c4_mid_max": lr["c4_mid_max"],
                 "timed_passes": {"edge_local": len(stats) - len(last_region),
                                  "whole_graph": sum(1 for st in last_region if st["whole_graph"]),
                                  "region": sum(1 for st in last_region if not st["whole_graph"])}}
    g.close()
    del dev_batches

    cpu = None
    if not args.no_cpu_baseline:
        mean_batch = float(np.mean([x[0].size + x[2].size for x in batches[args.warmup:]]))
        cpu = cpu_baseline(n, s, d, mean_batch, args.cpu_stride, args.scale, args.ef)
        log("cpu baseline: %s" % cpu["sample"])
    served = None if args.no_served else run_served(args, n, s, d, stream.ins_sampler)
    batched = None if args.no_batched else run_batched(args)

    out = {
        "metric": "updates/sec + p50/p99 batch latency, exact 4-graphlet counts, R-MAT s22",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / max(1, args.steps), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "R-MAT scale %d edge factor %d (n=%d, m=%d), batches log-uniform in [%g, %g], "
                               "50/50 insert/delete, plain per-batch path, radius %d, edge-local passes %s"
                               % (args.scale, args.ef, n, s.size, args.min_batch, args.max_batch, args.radius,
                                  {0: "auto", 1: "always", -1: "never"}[args.delta]),
                   "form": "plain"},
        "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
        "oracle_check": {"golden": "tests/golden/scale_rmat_s22_bench.json", "after_batches": sorted(gold),
                         "equal": checks, "all_equal": bool(checks) and all(checks.values())},
        "recount_check": recount_ok,
        "host_array_updates_per_s": host_rate, "host_array_counts_equal": host_same,
        "effective_updates_per_s": sum(st["eff_ins"] + st["eff_del"] for st in stats) / elapsed,
        "roofline": roof_c4, "roofline_tri": roof_tri, "compulsory_bandwidth": comp,
        "tuned": tuned,
        "cpu_baseline": cpu,
        "served": served, "batched": batched,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
