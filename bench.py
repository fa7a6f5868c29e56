#!/usr/bin/env python3
"""Throughput of LocalContraction connected components on one MI355X.

A step is one full solve -- every round until no edge is left, then the label of every
vertex -- of the headline workload, with its edge list already resident in HBM.  Each step
draws fresh priorities (seed base + step index).  The value is input edges per second.

Headline workload (default, --workload rmat26): R-MAT scale 26, edge factor 16 (2^26 ids,
2^30 packed records), quadrants (0.57, 0.19, 0.19, 0.05) with +-10% noise per level, ids
permuted -- the largest single-GPU configuration of the hot path.  The G(2^24, 2^27) graph
plus 10,000 paths of 1,000 vertices and the small G(65,536, 262,144) graph are timed after it
as secondary figures.

Printed (stdout, one JSON line): the metric; the roofline of the dominant step of the hot
path (its algorithmic bytes by the byte model below over the measured time of the kernels
that carry it out, against 8 TB/s); the CPU oracle timed on a bounded sample of the same
workload with a single-thread union-find beside it; the secondary workloads; the same
workload under TreeContraction, the one-hop label, the union-find finish and MergeToLarge;
the batched and the serving legs.  Diagnostics go to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_REPS = 5             # timed repetitions of the 1 GiB calibration copy

# The steps of a round (rows a2-a7 of the hot path) and the kernel families that carry out
# each.  The tiled round 0's partition belongs to the implementation (it moves no algorithmic
# byte); rounds inside a captured tail or the persistent launch are timed together ("tail").
FAMILY_STEP = {
    "round_begin": "a2_one_hop", "min1_round0": "a2_one_hop", "min1": "a2_one_hop", "min1_tiled": "a2_one_hop",
    "min2_round0": "a3_two_hop", "min2": "a3_two_hop", "min2_tiled": "a3_two_hop", "parent": "a3_two_hop",
    "label_ranks": "a4_relabel", "relabel_round0": "a4_relabel", "relabel": "a4_relabel",
    "relabel_tiled": "a4_relabel",
    "sort_hist": "a5_dedup", "sort_scan": "a5_dedup", "sort_scatter": "a5_dedup", "unique": "a5_dedup",
    "hash_dedup": "a5_dedup", "bucket_sort": "a5_dedup",
    "node_scan": "a6_nodes", "nodes": "a6_nodes", "map": "a6_nodes", "round_end": "a6_nodes",
    "compose": "a7_labels", "flatten": "a7_labels",
    "part_a_hist": "partition", "part_a_scatter": "partition", "part_b_hist": "partition",
    "part_b_scatter": "partition", "part_scan": "partition", "part_rows_hist": "partition",
    "part_rows_scatter": "partition",
    "tail_graph": "tail", "fused_rounds": "tail", "uf_finish": "finish", "merge_large": "merge_large",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_bytes(stats, n0, in_graph=None):
    """Algorithmic bytes of each step of the hot path over one solve (the byte model:
    what the method must move once, int32 names and 8-byte records).  Per round r, with N the
    nodes addressed (n0 in round 0), M the records read, S the survivors of the relabel
    (repeats counted) and M' the distinct edges out:
        a2 one-hop minimum   8 M + 4 N          records; m1 written
        a3 two-hop minimum   8 M + 8 N          records; m1 read, l (the parent) written
        a4 relabel           8 M + 4 N + 8 S    records; parents read; survivors written
        a5 duplicate drop    8 S + 8 M'         survivors read once, distinct edges written,
                                                however many passes the implementation makes
        a6 next nodes, map   4 N                the round's map written
        a7 labels            4 N (+ 4 n0)       the map read; the labels written once
    Total 24 M + 16 S + 8 M' + 24 N per round, plus 4 n0.  Random-access amplification, extra
    sort passes and the tiled round 0's partition are the implementation's overhead.  Rounds
    that ran inside a captured tail or the persistent launch (in_graph[i] nonzero) count under
    "tail"."""
    out = {}

    def add(k, v):
        out[k] = out.get(k, 0) + v

    for i, (r, n_active, m_in, s, m_out, _fin) in enumerate(stats):
        N = n0 if r == 0 else n_active
        M = m_in
        parts = {"a2_one_hop": 8 * M + 4 * N, "a3_two_hop": 8 * M + 8 * N, "a4_relabel": 8 * M + 4 * N + 8 * s,
                 "a5_dedup": 8 * s + 8 * m_out, "a6_nodes": 4 * N, "a7_labels": 4 * N}
        tail = bool(in_graph[i]) if in_graph is not None else False
        for k, v in parts.items():
            add("tail" if tail else k, v)
    add("a7_labels", 4 * n0)
    return out


def job_alg_bytes(stats, n0):
    """The whole solve's algorithmic bytes: the sum of step_bytes."""
    return sum(step_bytes(stats, n0).values())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown CPU"


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1

def bench_variants(args, lc, n0, m0, src, dst, layout, stream, base_seed):
    """The same workload, seeds and residency under the other label rules and with the
    union-find finish (cc_run as a user calls it, no per-kernel events).  Each variant's
    CC_CANONICAL labels are compared with LocalContraction's (same partition)."""
    import torch

    dev = src.device
    out = {}

    def canonical(flags, finish):
        with lc.Solver(n0, src, dst, seed=base_seed, flags=flags | lc.CC_CANONICAL, stream=stream, layout=layout,
                       finish_edges=finish) as s:
            s.run()
            lab = s.labels()
            torch.cuda.synchronize()
            return lab

    want = canonical(0, 0)
    for name, flags, finish in (("tree", lc.CC_TREE, 0), ("one_hop", lc.CC_ONE_HOP, 0),
                                ("uf_finish", 0, args.finish_edges), ("merge_to_large", lc.CC_MERGE_TO_LARGE, 0)):
        with lc.Solver(n0, src, dst, seed=base_seed, flags=flags, stream=stream, layout=layout,
                       finish_edges=finish) as s:
            labels = torch.empty(n0, dtype=torch.int32, device=dev)
            s.reset(base_seed + 999)
            s.run()                                  # warm-up
            torch.cuda.synchronize()
            rounds, finished = [], []
            t0 = time.perf_counter()
            for i in range(args.variant_steps):
                s.reset(base_seed + i)
                rounds.append(s.run())
                finished.append(s.finished)
                s.labels(labels)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        same = bool(torch.equal(canonical(flags, finish), want))
        ent = {"ms_per_step": dt * 1e3 / args.variant_steps, "value": m0 * args.variant_steps / dt,
               "unit": "edges/s", "rounds": rounds, "canonical_labels_identical": same}
        if finish:
            ent["finish_edges"] = finish
            ent["finished"] = finished
        out[name] = ent
        log("variant %s: %.2f ms/step, rounds %s, canonical labels identical: %s"
            % (name, ent["ms_per_step"], rounds, same))
    return out


def cpu_baseline(workload, rmat_scale, er_shrink):
    """The oracle (single-threaded C, as it stands) on a bounded sample of the headline
    workload -- the same generator recipe at a smaller size -- and a textbook single-thread
    union-find (the partition only, the paper's choice for a graph that fits one machine,
    Section 6) on the same sample."""
    import graphgen
    import oracle
    if workload.startswith("rmat"):
        g = graphgen.workload_rmat(scale=rmat_scale)
        what = ("R-MAT scale %d, edge factor 16, same recipe as the headline graph (n=%d, m=%d records)"
                % (rmat_scale, g.n, g.m))
    elif workload == "small":
        g = graphgen.workload_small()
        what = "the same graph (n=%d, m=%d records)" % (g.n, g.m)
    else:
        g = graphgen.workload_er_paths(shrink=er_shrink)
        what = ("the same G(n,m)+paths mix scaled by 1/%d (n=%d, m=%d records)" % (er_shrink, g.n, g.m))
    t0 = time.perf_counter()
    res = oracle.run(g.n, g.src, g.dst, seed=graphgen.CONFIG_SEED_BASE + 1)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.components_min_id(g.n, g.src, g.dst)
    dt_uf = time.perf_counter() - t0
    host = "%s, 1 of %d cores" % (cpu_model(), host_cores())
    return {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "%s: %d rounds in %.1f s on %s" % (what, res.rounds, dt, host),
            "host": host, "seconds": round(dt, 2),
            "union_find": {"value": g.m / dt_uf, "unit": "edges/s", "cores": 1, "seconds": round(dt_uf, 2),
                           "kind": "textbook union-find, partition only"}}


def bench_batch(args, log_prefix="batch"):
    """4,096 independent graphs (half G(n,m) with average degree U[1.5,16], half R-MAT with
    edge factor 8, vertex counts log-uniform in [2^8, 2^18]) solved as one batch, against
    the same graphs solved one after another with the plain API on the same GPU."""
    import numpy as np
    import torch

    import graphgen
    import paper_1807_10727_amd as lc
    from paper_1807_10727_amd import autotune

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    b = graphgen.batch_mix(count=args.batch_graphs, log2_max=args.batch_log2_max)
    log("%s: generated %d graphs, n=%d, m=%d in %.1fs" % (log_prefix, b.count, int(b.voff[-1]), int(b.eoff[-1]),
                                                          time.perf_counter() - t0))
    src = torch.from_numpy(b.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(b.dst.view(np.int32)).to(dev)
    bt = lc.Batch(b.voff, b.eoff, b.seeds, src, dst)
    t0 = time.perf_counter()
    rejected = []
    cfg, _, tried = autotune.tune(bt, repeats=1, cache=args.tune_cache, log=log if args.verbose_tune else None,
                                  rejected=rejected)
    log("%s: autotune picked %s (%d candidates timed, %.1fs)" % (log_prefix, cfg, tried, time.perf_counter() - t0))
    n_small, union_m = bt.split()
    lab, rounds = bt.run()                      # warm (captures the graph if needed)
    torch.cuda.synchronize()
    ts = []
    for _ in range(args.batch_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.run(with_rounds=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_batch = sorted(ts)[len(ts) // 2]
    batch_labels = bt.labels_buf[:bt.n_total].clone()
    bt.close()
    del bt
    torch.cuda.empty_cache()

    # sequential plain solves: one context per graph on its own (aligned) copy of its records
    seq_labels = torch.empty(max(int(b.voff[-1]), 1), dtype=torch.int32, device=dev)
    solvers = []
    for j in range(b.count):
        a, e = int(b.eoff[j]), int(b.eoff[j + 1])
        sj = src[a:e].clone() if e > a else torch.zeros(1, dtype=torch.int32, device=dev)[:0]
        dj = dst[a:e].clone() if e > a else torch.zeros(1, dtype=torch.int32, device=dev)[:0]
        solvers.append(lc.Solver(int(b.n[j]), sj, dj, seed=int(b.seeds[j])))
    for j in range(min(64, b.count)):
        solvers[j].run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, sv in enumerate(solvers):
        sv.reset(int(b.seeds[j]))
        sv.run()
        if sv.n:
            sv.labels(seq_labels[int(b.voff[j]):int(b.voff[j + 1])])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for sv in solvers:
        sv.close()
    same = bool(torch.equal(seq_labels[:int(b.voff[-1])], batch_labels))
    log("%s: batch %.1f ms, sequential %.1f ms, labels identical: %s" % (log_prefix, t_batch * 1e3, t_seq * 1e3, same))
    if not same:
        raise RuntimeError("batched labels differ from the sequential solves")
    del solvers, seq_labels, batch_labels, src, dst
    torch.cuda.empty_cache()
    return {"graphs": b.count, "records": int(b.eoff[-1]), "vertices": int(b.voff[-1]),
            "graphs_per_s": b.count / t_batch, "ms": t_batch * 1e3,
            "sequential_graphs_per_s": b.count / t_seq, "sequential_ms": t_seq * 1e3,
            "speedup_vs_sequential": t_seq / t_batch, "labels_identical_to_sequential": same,
            "lds_path_graphs": n_small, "union_records": union_m, "max_rounds": int(rounds.max()),
            "config": cfg,
            "tuner_rejected": [{"knob": k, "value": v, "reason": why} for k, v, why in rejected]}


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


def bench_serve(args):
    """Continuous batching under load.  A pool of graphs (vertex counts log-uniform in
    [2^10, 2^24], half G(n,m) with average degree U[4,16], half R-MAT with edge factor 16) is
    made resident in HBM; the trace is serve_warmup + serve_requests requests with Poisson
    arrivals, each a pool graph drawn at random with a priority seed of its own, so that a
    trace of thousands of requests needs only the pool's memory.  The server (HBM budget,
    slots) replays it at several loads; the same trace served FIFO by sequential plain solves
    (each request's measured service time) is the baseline.  Latency percentiles and graphs/s
    cover the requests after the warm-up ones; every request's labels must equal its solo
    solve."""
    import numpy as np
    import torch

    import graphgen
    import paper_1807_10727_amd as lc

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    pool_spec = graphgen.request_trace(graphgen.CONFIG_SEED_BASE + 4, args.serve_pool, rate=1.0,
                                       log2_min=10, log2_max=args.serve_log2_max)
    pool = []
    for r in pool_spec:
        g = r.graph()
        pool.append((g.n, torch.from_numpy(g.src.view(np.int32)).to(dev), torch.from_numpy(g.dst.view(np.int32)).to(dev)))
        del g
    total = args.serve_warmup + args.serve_requests
    base_arr, which, seeds = graphgen.request_mix(graphgen.CONFIG_SEED_BASE + 5, total, len(pool))
    reqs = [pool[k] + (seeds[i],) for i, k in enumerate(which)]
    pool_m = sum(int(x[1].shape[0]) for x in pool)
    total_m = sum(int(pool[k][1].shape[0]) for k in which)
    torch.cuda.synchronize()
    log("serve: pool of %d graphs (%d records) generated and uploaded in %.1fs; trace of %d + %d requests"
        % (len(pool), pool_m, time.perf_counter() - t0, args.serve_warmup, args.serve_requests))

    # sequential plain solves in trace order, back to back: service times and reference labels
    ref = []
    service = []
    for (n, s, d, sd) in reqs[:min(4, len(reqs))]:          # warm the kernels
        lc.solve(n, s, d, seed=sd)
    for (n, s, d, sd) in reqs:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lab, _, _ = lc.solve(n, s, d, seed=sd)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t1)
        ref.append(lab)
    cap = len(reqs) / sum(service)
    log("serve: sequential capacity %.1f requests/s (service p50 %.2f ms, max %.2f ms)"
        % (cap, 1e3 * _pct(service, 50), 1e3 * max(service)))
    W = args.serve_warmup

    def fifo(arrivals):
        fin, lat, done = 0.0, [], []
        for a, sv in zip(arrivals, service):
            fin = max(fin, a) + sv
            lat.append(fin - a)
            done.append(fin)
        return lat[W:], done[-1] - arrivals[W] if len(arrivals) > W else 0.0

    loads = []
    identical = True
    srv = lc.Server(args.serve_budget_gib << 30, n_slots=args.serve_slots, small_variant=args.serve_small_variant,
                    max_small_per_launch=256, cohort_max=args.serve_cohort_max,
                    cohort_max_vertices=1 << args.serve_cohort_log2_vertices)
    try:
        for rho in args.serve_loads:
            lam = rho * cap
            arr = [a / lam for a in base_arr]
            seq_lat, seq_span = fifo(arr)
            labs = {}
            t_start = srv.info()["now"]
            for i, (n, s, d, sd) in enumerate(reqs):
                while srv.info()["now"] - t_start < arr[i] - arr[0]:
                    time.sleep(0.0002)
                rid, lab = srv.submit(n, s, d, sd)
                labs[rid] = (i, lab)
            res = srv.drain()
            if len(res) != len(reqs) or any(x["status"] != 0 for x in res):
                raise RuntimeError("serving run lost or failed requests")
            timed = [x for x in res if labs[x["id"]][0] >= W]
            lat = [x["t_done"] - x["t_submit"] for x in timed]
            span = max(x["t_done"] for x in timed) - min(x["t_submit"] for x in timed) if timed else 0.0
            for x in res:
                i, lab = labs[x["id"]]
                identical &= bool(torch.equal(lab, ref[i]))
            del labs
            loads.append({"load": rho, "lambda_req_per_s": lam,
                          "p50_ms": 1e3 * _pct(lat, 50), "p99_ms": 1e3 * _pct(lat, 99),
                          "graphs_per_s": len(timed) / span if span > 0 else None,
                          "sequential_p50_ms": 1e3 * _pct(seq_lat, 50), "sequential_p99_ms": 1e3 * _pct(seq_lat, 99),
                          "sequential_graphs_per_s": len(seq_lat) / seq_span if seq_span > 0 else None,
                          "small_path": sum(1 for x in timed if x["small_path"]),
                          "in_cohorts": sum(1 for x in timed if x["cohort"] > 1)})
            log("serve: load %.1f  p50 %.2f ms  p99 %.2f ms  %s graphs/s | sequential p50 %.2f ms  p99 %.2f ms  %s graphs/s"
                % (rho, loads[-1]["p50_ms"], loads[-1]["p99_ms"], loads[-1]["graphs_per_s"],
                   loads[-1]["sequential_p50_ms"], loads[-1]["sequential_p99_ms"], loads[-1]["sequential_graphs_per_s"]))
        peak = srv.info()["peak_bytes"]
    finally:
        srv.close()
    del reqs, ref, pool
    torch.cuda.empty_cache()
    if not identical:
        raise RuntimeError("served labels differ from the solo solves")
    return {"requests": args.serve_requests, "warmup_requests": W, "pool_graphs": args.serve_pool,
            "cohort_max": args.serve_cohort_max, "cohort_max_vertices": 1 << args.serve_cohort_log2_vertices,
            "pool_records": pool_m, "trace_records": total_m, "budget_gib": args.serve_budget_gib,
            "slots": args.serve_slots, "sequential_capacity_req_per_s": cap, "loads": loads,
            "labels_identical_to_solo": identical, "peak_arena_gib": peak / 2**30}


WORKLOADS = ("rmat26", "er_paths", "small", "rmat24")


def make_workload(name):
    """(graph, description) of a named workload (seeded generators, no method arithmetic)."""
    import graphgen
    if name == "er_paths":
        return graphgen.workload_er_paths(), "G(n=2^24, m=2^27) + 10,000 paths x 1,000 vertices, int32 ids"
    if name == "small":
        return graphgen.workload_small(), "G(n=65,536, m=262,144), int32 ids"
    scale = 26 if name == "rmat26" else 24
    return (graphgen.workload_rmat(scale=scale),
            "R-MAT scale %d, edge factor 16, (0.57,0.19,0.19,0.05) +-10%%, permuted ids, packed u64 records" % scale)


def upload(name, g, dev):
    import numpy as np
    import torch
    import paper_1807_10727_amd as lc
    if name.startswith("rmat"):
        keys = graphgen_pack(g)
        return torch.from_numpy(keys).to(dev), None, lc.CC_EDGES_PACKED_U64
    return (torch.from_numpy(g.src.view(np.int32)).to(dev), torch.from_numpy(g.dst.view(np.int32)).to(dev),
            lc.CC_EDGES_SOA_I32)


def graphgen_pack(g):
    import numpy as np
    import graphgen
    return graphgen.pack(g.src, g.dst).view(np.int64)


def bench_secondary(name, steps, warmup):
    """A secondary workload: `steps` full solves (a reused context, as a user runs them),
    input edges per second and the job's algorithmic bytes over the step time."""
    import torch
    import graphgen
    import paper_1807_10727_amd as lc
    dev = torch.device("cuda:0")
    g, wname = make_workload(name)
    src, dst, layout = upload(name, g, dev)
    n0, m0 = g.n, int(src.shape[0])
    del g
    stream = torch.cuda.current_stream(dev)
    base = graphgen.CONFIG_SEED_BASE + 1
    labels = torch.empty(n0, dtype=torch.int32, device=dev)
    with lc.Solver(n0, src, dst, seed=base, stream=stream, layout=layout) as s:
        for i in range(warmup):
            s.reset(base + 1000 + i)
            s.run()
            s.labels(labels)
        torch.cuda.synchronize()
        stats, rounds = [], []
        t0 = time.perf_counter()
        for i in range(steps):
            s.reset(base + i)
            rounds.append(s.run())
            s.labels(labels)
            stats.append(s.stats(rounds[-1]))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    job = sum(job_alg_bytes(st, n0) for st in stats)
    out = {"workload": wname, "n_vertices": n0, "n_records": m0, "steps": steps,
           "ms_per_step": dt * 1e3 / steps, "value": m0 * steps / dt, "unit": "edges/s", "rounds": rounds[0],
           "job_alg_frac": round(job / dt / 1e9 / HBM_PEAK_GBS, 4)}
    log("secondary %s: %.3f ms/step, %.3g edges/s, rounds %s" % (name, out["ms_per_step"], out["value"], rounds))
    del src, dst, labels
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat26", choices=WORKLOADS)
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--eager", action="store_true", help="run every round eagerly (no captured tails)")
    ap.add_argument("--round0", default="auto", choices=["auto", "direct", "tiled", "rows"],
                    help="how round 0 reads the input records (auto: the library's choice by size, then the "
                         "tuner's; rows: tiled, with the one-pass row partition)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-rmat-scale", type=int, default=21,
                    help="R-MAT scale of the oracle's sample of an R-MAT headline (same recipe)")
    ap.add_argument("--cpu-shrink", type=int, default=8, help="divisor of the G(n,m)+paths sample")
    ap.add_argument("--secondary", default="er_paths,small",
                    help="comma-separated secondary workloads timed after the headline ('' for none)")
    ap.add_argument("--secondary-steps", type=int, default=10)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-mode leg")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched-mode leg")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-log2-max", type=int, default=18)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--tune-cache", default=None, help="autotune cache file (default: none, tune every run)")
    ap.add_argument("--no-tune", action="store_true", help="keep the solver's default knobs (no autotuning)")
    ap.add_argument("--tune-knobs", default="", help="comma-separated knobs to tune (default: all of them)")
    ap.add_argument("--set", default="", metavar="KNOB=V,...",
                    help="solver knobs (include/cc.h, cc_tuning) set as given; the tuner leaves them alone")
    ap.add_argument("--verbose-tune", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000, help="timed requests of the serving trace")
    ap.add_argument("--serve-warmup", type=int, default=200, help="untimed requests before them")
    ap.add_argument("--serve-pool", type=int, default=128, help="distinct graphs the trace draws from")
    ap.add_argument("--serve-cohort-max", type=int, default=16,
                    help="large requests the server may start together as one union (0: none)")
    ap.add_argument("--serve-cohort-log2-vertices", type=int, default=20,
                    help="largest request (log2 vertices) that may join a cohort")
    ap.add_argument("--serve-log2-max", type=int, default=24)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-small-variant", type=int, default=3)
    ap.add_argument("--serve-budget-gib", type=int, default=128)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.8, 1.2])
    ap.add_argument("--no-variants", action="store_true",
                    help="skip TreeContraction, the one-hop label, the union-find finish and MergeToLarge")
    ap.add_argument("--variant-steps", type=int, default=5)
    ap.add_argument("--finish-edges", type=int, default=1 << 22)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen
    import paper_1807_10727_amd as lc

    if args.batch_only:
        print(json.dumps({"batched": bench_batch(args)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": bench_serve(args)}), flush=True)
        return

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    g, wname = make_workload(args.workload)
    log("generated %s: n=%d m=%d in %.1fs" % (wname, g.n, g.m, time.perf_counter() - t0))
    src, dst, layout = upload(args.workload, g, dev)
    n0, m0 = g.n, int(src.shape[0])
    del g
    torch.cuda.synchronize()

    # the streaming bandwidth this GPU reaches: a plain 1 GiB device copy timed with events
    # (read + write), reported beside the 8 TB/s peak
    cal_a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cal_b = torch.empty_like(cal_a)
    cal_b.copy_(cal_a)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(COPY_REPS):
        cal_b.copy_(cal_a)
    ev[1].record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * cal_a.numel() * COPY_REPS / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
    log("plain 1 GiB device copy: %.1f GB/s (read + write)" % copy_gbs)
    del cal_a, cal_b

    flags = 0 if args.no_profile else lc.CC_PROFILE
    if args.eager:
        flags |= lc.CC_EAGER
    round0_flag = {"auto": 0, "direct": lc.CC_ROUND0_DIRECT, "tiled": lc.CC_ROUND0_TILED,
                   "rows": lc.CC_ROUND0_TILED}[args.round0]
    flags |= round0_flag
    stream = torch.cuda.current_stream(dev)
    base_seed = graphgen.CONFIG_SEED_BASE + 1

    # The solver's knobs (form of round 0, workgroups per CU, round 0's key sets) are tuned on
    # this graph first, without per-kernel events; every candidate must give the same labels.
    fixed = {}
    tuner_rejected = []   # candidates the tuner could not use (a failed solve, other labels)
    for item in filter(None, args.set.split(",")):
        k, _, v = item.partition("=")
        if k not in lc.TUNING_KNOBS or not v.lstrip("-").isdigit():
            raise SystemExit("--set takes knob=integer pairs of %s" % ",".join(lc.TUNING_KNOBS))
        fixed[k] = int(v)
    tuning = None
    if not args.no_tune:
        from paper_1807_10727_amd import autotune
        space = dict(autotune.SOLVER_SPACE)
        if args.tune_knobs:
            keep = args.tune_knobs.split(",")
            unknown = [k for k in keep if k not in space]
            if unknown:
                raise SystemExit("unknown tuning knobs: %s" % ",".join(unknown))
            space = {k: v for k, v in space.items() if k in keep}
        space = {k: v for k, v in space.items() if k not in fixed}   # knobs set as given stay
        if args.round0 != "auto":
            space.pop("round0", None)     # the form asked for stays
        t0 = time.perf_counter()
        with lc.Solver(n0, src, dst, seed=base_seed, flags=round0_flag, stream=stream, layout=layout) as ts:
            if args.round0 == "rows" or fixed:
                ts.set_tuning(**dict({"round0": 3} if args.round0 == "rows" else {}, **fixed))
            tuning, t_best, tried = autotune.tune_solver(ts, seed=base_seed + 500, repeats=1, cache=args.tune_cache,
                                                         rejected=tuner_rejected,
                                                         log=log if args.verbose_tune else None, space=space)
        torch.cuda.empty_cache()
        log("solver autotune picked %s (%d candidates timed, best %.3f ms, %.1fs)"
            % (tuning, tried, t_best * 1e3, time.perf_counter() - t0))

    labels = torch.empty(n0, dtype=torch.int32, device=dev)
    solver = lc.Solver(n0, src, dst, seed=base_seed, flags=flags, stream=stream, layout=layout)
    if tuning:
        solver.set_tuning(**tuning)
    elif args.round0 == "rows" or fixed:
        tuning = dict({"round0": 3} if args.round0 == "rows" else {}, **fixed)
        solver.set_tuning(**tuning)
    log("workspace %.2f GiB" % (solver.ws_bytes / 2**30))

    def step(i):
        solver.reset(base_seed + i)
        r = solver.run()
        solver.labels(labels)
        return r

    def collect(acc_ms, acc_n):
        for k, (ms, n) in solver.kernel_times().items():   # per solve (reset clears them)
            acc_ms[k] = acc_ms.get(k, 0.0) + ms
            acc_n[k] = acc_n.get(k, 0) + n

    def steps_of(acc, fams):
        out = {}
        for k, v in acc.items():
            st = FAMILY_STEP.get(k, k)
            if fams is None or k in fams:
                out[st] = out.get(st, 0) + v
        return out

    # Warm-up: every kernel family is timed with events; the step of the hot path whose kernels
    # take the most time is the dominant one.  The timed steps then put events around that
    # step's families only (events around every launch slow the stream down), and the last
    # warm-up step runs with that setting (it also captures the tails the timed steps replay).
    # Events sit only on eagerly launched rounds, and the bytes of rounds inside captured
    # tails are counted under "tail", so time and bytes cover the same launches.
    warm_ms, warm_n, warm_bytes = {}, {}, {}
    n_warm = max(args.warmup - 1, 0) if not args.no_profile else args.warmup
    for i in range(n_warm):
        r = step(1000 + i)
        for k, v in step_bytes(solver.stats(r), n0, solver.rounds_in_graph(r)).items():
            warm_bytes[k] = warm_bytes.get(k, 0) + v
        collect(warm_ms, warm_n)
    torch.cuda.synchronize()
    dom_step, dom_fams = None, None
    step_rooflines = None
    if not args.no_profile and warm_ms:
        per_step = steps_of(warm_ms, None)
        step_rooflines = {}
        log("warm-up: step            ms/solve   GB/s (algorithmic)")
        for k in sorted(per_step, key=lambda x: -per_step[x]):
            gbs = warm_bytes.get(k, 0) / (per_step[k] * 1e-3) / 1e9 if per_step[k] > 0 else 0.0
            log("  %-18s %8.3f %10.1f" % (k, per_step[k] / n_warm, gbs))
            # every step of the hot path, timed with events around all of its kernels
            step_rooflines[k] = {"ms_per_solve": round(per_step[k] / n_warm, 4),
                                 "bytes_per_solve": int(warm_bytes[k] / n_warm) if k in warm_bytes else None,
                                 "achieved_gbs": round(gbs, 1) if k in warm_bytes else None,
                                 "frac": round(gbs / HBM_PEAK_GBS, 4) if k in warm_bytes else None}
        log("warm-up: kernel family       ms/solve  launches/solve")
        for k in sorted(warm_ms, key=lambda x: -warm_ms[x]):
            if warm_n[k]:
                log("  %-18s %8.3f %10.1f" % (k, warm_ms[k] / n_warm, warm_n[k] / n_warm))
        log("warm-up: sum of kernel time per solve %.3f ms" % (sum(warm_ms.values()) / n_warm))
        timed = {k: v for k, v in per_step.items() if k in warm_bytes and k not in ("tail",)}
        dom_step = max(timed, key=lambda k: timed[k])
        dom_fams = sorted(k for k, v in warm_n.items() if v and FAMILY_STEP.get(k) == dom_step)
        solver.profile_families(dom_fams)
        step(2000)
        torch.cuda.synchronize()
    solver.reset(base_seed)            # clears the per-kernel timers too
    all_stats, in_graph, rounds = [], [], []
    fam_ms, fam_n = {}, {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step(i)
        rounds.append(r)
        all_stats.append(solver.stats(r))
        in_graph.append(solver.rounds_in_graph(r))
        collect(fam_ms, fam_n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = m0 * args.steps / dt
    log("rounds per step: %s" % rounds)
    for st, ig in zip(all_stats[0], in_graph[0]):
        log("  round %d: n_active=%d m_in=%d survive=%d m_out=%d finalised=%d" % st + (" (tail)" if ig else ""))

    job_bytes = sum(job_alg_bytes(st, n0) for st in all_stats)
    roofline = None
    if dom_step is not None:
        b = {}
        for st, ig in zip(all_stats, in_graph):
            for k, v in step_bytes(st, n0, ig).items():
                b[k] = b.get(k, 0) + v
        ms = sum(fam_ms.get(k, 0.0) for k in dom_fams)
        launches = sum(fam_n.get(k, 0) for k in dom_fams)
        achieved = b[dom_step] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        top = max(dom_fams, key=lambda k: fam_ms.get(k, 0.0))
        roofline = {"bound": "hbm", "kernel": dom_step, "families": dom_fams, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None, "bytes_per_solve": int(b[dom_step] / args.steps),
                    "ms_per_solve": round(ms / args.steps, 4), "launches_per_solve": launches / args.steps,
                    "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2),
                    "largest_family": top, "largest_family_ms_per_solve": round(fam_ms.get(top, 0.0) / args.steps, 4),
                    "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
        log("timed steps: %s (%s) %.3f ms/solve over %.1f launches/solve, %.1f GB/s algorithmic"
            % (dom_step, ",".join(dom_fams), ms / args.steps, launches / args.steps, achieved))
    job_gbs = job_bytes / dt / 1e9
    log("job algorithmic bytes per step %.2f GB -> %.1f GB/s (%.1f%% of 8 TB/s)"
        % (job_bytes / args.steps / 1e9, job_gbs, 100 * job_gbs / HBM_PEAK_GBS))

    solver.close()
    del solver, labels
    torch.cuda.empty_cache()
    variants = None
    if not args.no_variants:
        try:
            variants = bench_variants(args, lc, n0, m0, src, dst, layout, stream, base_seed)
        except Exception as e:  # the main figure stands on its own
            log("variants leg failed: %r" % (e,))
            variants = {"error": repr(e)}
    del src, dst
    torch.cuda.empty_cache()

    secondary = {}
    for name in [x for x in args.secondary.split(",") if x and x != args.workload]:
        try:
            secondary[name] = bench_secondary(name, args.secondary_steps if name != "small" else 5 * args.secondary_steps,
                                              2)
        except Exception as e:  # the main figure stands on its own
            log("secondary %s failed: %r" % (name, e))
            secondary[name] = {"error": repr(e)}

    batched = None
    if not args.no_batch:
        try:
            batched = bench_batch(args)
        except Exception as e:  # the main figure stands on its own
            log("batched leg failed: %r" % (e,))
            batched = {"error": repr(e)}

    serving = None
    if not args.no_serve:
        try:
            serving = bench_serve(args)
        except Exception as e:  # the main figure stands on its own
            log("serving leg failed: %r" % (e,))
            serving = {"error": repr(e)}

    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(args.workload, args.cpu_rmat_scale, args.cpu_shrink)
            log("cpu baseline: %s" % cpu["sample"])
        except Exception as e:  # the GPU figure stands on its own
            log("cpu baseline failed: %r" % (e,))

    out = {
        "metric": "input edges/sec to full CC labels (1 GPU)",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": wname, "n_vertices": n0, "n_records": m0, "rounds": rounds[0],
                   "round0": args.round0, "tuning": tuning, "parallelism": "single GPU"},
        "tuner_rejected": [{"knob": k, "value": v, "reason": why} for k, v, why in tuner_rejected],
        "roofline": roofline,
        "step_rooflines": step_rooflines,
        "job_alg_frac": round(job_gbs / HBM_PEAK_GBS, 4),
        "job_alg_frac_of_copy": round(job_gbs / copy_gbs, 4),
        "cpu_baseline": cpu,
        "secondary": secondary,
        "variants": variants,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
