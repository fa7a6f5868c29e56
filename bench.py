#!/usr/bin/env python3
"""Throughput of LocalContraction connected components on one MI355X.

A step is one full solve -- every round until no edge is left, then the label of every
vertex -- of the G(n, m) graph with n = 2^24, m = 2^27 (int32 ids, endpoints uniform,
duplicates and self-loops kept) plus 10,000 disjoint random paths of 1,000 vertices,
with the edge list already resident in HBM.  Each step draws fresh priorities (seed
base + step index).  The value is input edges per second.

Printed (stdout, one JSON line): the metric, the roofline of the dominant kernel family
(algorithmic bytes per launch over its HIP-event launch time, against 8 TB/s), the CPU
oracle timed on a bounded sample of the same mix, the same workload under TreeContraction,
the one-hop label and the union-find finish, the batched and the serving legs.
Diagnostics go to stderr.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
COPY_REPS = 5             # timed repetitions of the 1 GiB calibration copy
# kernel symbol (as rocprofv3 prints it) of each timed family of the int32 input path
FAMILY_SYMBOL = {
    "min1_round0": "lc::k_min1<lc::ReadSoa32<4>, true, false>",
    "min2_round0": "lc::k_min2<lc::ReadSoa32<4> >",
    "relabel_round0": "lc::k_relabel<lc::ReadSoa32<4> >",
    "min1": "lc::k_min1_seeded",
    "min2": "lc::k_min2<lc::ReadInternal>",
    "relabel": "lc::k_relabel<lc::ReadInternal>",
    "sort_hist": "lc::k_sort_hist",
    "sort_scatter": "lc::k_sort_scatter",
    "compose": "lc::k_compose<false, false>",
    "part_a_hist": "lc::k_part_a_hist<lc::ReadSoa32<4> >",
    "part_a_scatter": "lc::k_part_a_scatter<lc::ReadSoa32<4> >",
    "part_b_hist": "lc::k_part_b_hist",
    "part_b_scatter": "lc::k_part_b_scatter",
    "min1_tiled": "lc::k_tiled_min<1>",
    "min2_tiled": "lc::k_tiled_min<2>",
    "relabel_tiled": "lc::k_tiled_relabel",
}


def tail_free(family):
    """Whether a kernel family never runs inside a captured tail.  A tail holds rounds >= 1 of
    at most 2^22 records, which drop repeats by hashing: no radix pass and no unique, and
    round 0's families run once."""
    return (family in ("sort_hist", "sort_scan", "sort_scatter", "unique") or family.endswith("_round0")
            or family.startswith("part_") or family.endswith("_tiled"))


# rounds >= 1 with at most this many keys drop repeated edges by hashing (the library's
# kHashMaxRecords; the bench graph's key buffers always hold the table)
HASH_MAX_RECORDS = 1 << 22


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ceil_log2(n):
    b = 0
    while (1 << b) < n:
        b += 1
    return b


def family_bytes(stats, n0, tiled=False, loops=0, sorted_keys=None):
    """Algorithmic bytes each kernel family must move, summed over the rounds of a solve.

    Per round r: N = nodes addressed (n0 in round 0), M = records read, S = survivors,
    K = keys the relabel wrote and the sort processed (S less the repeats the relabel
    workgroups dropped), M' = distinct edges out, P = radix passes over the keys: they carry
    2 ceil(log2 L) bits in digits of at most 8 bits, L = the round's labels = the next round's
    nodes plus the labels the round finalised.  Rounds >= 1 with at most HASH_MAX_RECORDS
    keys drop repeats through a hashed key set instead of sorting.
    Random-access amplification (cache-line reads for 4-byte gathers and atomics) is
    implementation overhead and deliberately not counted.  With the tiled round 0,
    T = 2 (M - loops) directed records are written once, re-read by the row pass and read
    by each row kernel."""
    fam = {}

    def add(k, v):
        fam[k] = fam.get(k, 0) + v

    for i, (r, n_active, m_in, s, m_out, fin) in enumerate(stats):
        N = n0 if r == 0 else n_active
        M = m_in
        K = sorted_keys[i]
        L = fin + (stats[i + 1][1] if i + 1 < len(stats) else 0)
        P = (2 * ceil_log2(max(L, 2)) + 7) // 8
        sfx = "_round0" if r == 0 else ""
        add("round_begin", 10 * N)                 # m1, lv (4 B) and two flag bytes per node
        add("label_ranks", 8 * N + 3 * N // 8)     # parents in, their label ranks out, label map scanned
        if r == 0 and tiled:
            T = 2 * (M - loops)
            add("part_a_hist", 8 * M)              # records in
            add("part_a_scatter", 8 * M + 8 * T)   # records in, directed records out
            add("part_b_hist", 8 * T)
            add("part_b_scatter", 16 * T)
            add("min1_tiled", 8 * T + 4 * N)       # directed records in, m1 out
            add("min2_tiled", 8 * T + 8 * N)       # directed records in, m1 in once, parent out
            add("relabel_tiled", 8 * T + 4 * N + 8 * K)   # directed records, parents once, keys out
        else:
            add("min1" + sfx, 8 * M + 4 * N)           # records in, m1 out once
            add("min2" + sfx, 8 * M + 8 * N)           # records in, m1 in once, lv out once
            add("parent", 8 * N)                       # lv in, parent out
            add("relabel" + sfx, 8 * M + 4 * N + 8 * K)   # records in, parents in once, keys out
        if r >= 1 and K <= HASH_MAX_RECORDS:
            # keys in, each distinct key stored in the key set and read back by the count and
            # the write, renamed unique keys out
            add("hash_dedup", 8 * K + 32 * m_out)
        else:
            add("sort_hist", 8 * K * P)                # keys in per pass
            add("sort_scatter", 16 * K * P)            # keys in and out per pass
            add("unique", 16 * K + 8 * m_out)          # sorted keys read twice, renamed unique keys out
        add("node_scan", 2 * N)                    # flags of the labels (at most N) in twice, node map out
        add("nodes", 9 * N)
        add("map", 9 * N)
    fam["compose"] = fam.get("compose", 0) + 8 * n0
    return fam


def job_alg_bytes(stats, n0):
    """The job's algorithmic bytes: three streaming reads of the records, the survivors
    written and read once, the unique edges written, 24 bytes of node state per node and
    round, and the labels.  Survivors as the method defines them (m_survive), whatever
    share of them the implementation drops before writing."""
    b = 4 * n0
    for (r, n_active, m_in, s, m_out, _fin) in stats:
        N = n0 if r == 0 else n_active
        b += 24 * m_in + 16 * s + 8 * m_out + 24 * N
    return b


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


def cpu_baseline(shrink):
    import graphgen
    import oracle
    g = graphgen.workload_er_paths(shrink=shrink)
    t0 = time.perf_counter()
    res = oracle.run(g.n, g.src, g.dst, seed=graphgen.CONFIG_SEED_BASE)
    dt = time.perf_counter() - t0
    return {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "same G(n,m)+paths mix scaled by 1/%d: n=%d, m=%d records, %d rounds, %.1f s single-threaded"
                      % (shrink, g.n, g.m, res.rounds, dt)}


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
    cfg, _, tried = autotune.tune(bt, repeats=1, cache=args.tune_cache, log=log if args.verbose_tune else None)
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
            "config": cfg}


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


def bench_serve(args):
    """Poisson arrivals of requests with vertex counts log-uniform in [2^10, 2^24] (half
    G(n,m) with average degree U[4,16], half R-MAT with edge factor 16), inputs resident in
    HBM, served by the continuous-batching server under an HBM budget, against the same
    trace served FIFO by sequential plain solves (their measured service times)."""
    import numpy as np
    import torch

    import graphgen
    import paper_1807_10727_amd as lc

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    trace = graphgen.request_trace(graphgen.CONFIG_SEED_BASE + 4, args.serve_requests, rate=1.0,
                                   log2_min=10, log2_max=args.serve_log2_max)
    reqs = []
    for r in trace:
        g = r.graph()
        reqs.append((r, g.n, torch.from_numpy(g.src.view(np.int32)).to(dev),
                     torch.from_numpy(g.dst.view(np.int32)).to(dev)))
        del g
    total_m = sum(int(x[2].shape[0]) for x in reqs)
    torch.cuda.synchronize()
    log("serve: %d requests, %d records, generated and uploaded in %.1fs" % (len(reqs), total_m, time.perf_counter() - t0))

    # sequential plain solves, back to back: service times and reference labels
    ref = []
    service = []
    for (r, n, s, d) in reqs[:min(4, len(reqs))]:          # warm the kernels
        lc.solve(n, s, d, seed=r.seed)
    for (r, n, s, d) in reqs:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lab, _, _ = lc.solve(n, s, d, seed=r.seed)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t1)
        ref.append(lab)
    cap = len(reqs) / sum(service)
    log("serve: sequential capacity %.1f requests/s (service p50 %.2f ms, max %.2f ms)"
        % (cap, 1e3 * _pct(service, 50), 1e3 * max(service)))

    def fifo(arrivals):
        fin, lat = 0.0, []
        for a, sv in zip(arrivals, service):
            fin = max(fin, a) + sv
            lat.append(fin - a)
        return lat, fin - arrivals[0]

    base_arr = [r.arrival for (r, _, _, _) in reqs]
    loads = []
    identical = True
    srv = lc.Server(args.serve_budget_gib << 30, n_slots=args.serve_slots, small_variant=1,
                    max_small_per_launch=256)
    try:
        for rho in args.serve_loads:
            lam = rho * cap
            arr = [a / lam for a in base_arr]
            seq_lat, seq_span = fifo(arr)
            labs = {}
            t_start = srv.info()["now"]
            for i, (r, n, s, d) in enumerate(reqs):
                while srv.info()["now"] - t_start < arr[i] - arr[0]:
                    time.sleep(0.0002)
                rid, lab = srv.submit(n, s, d, r.seed)
                labs[rid] = (i, lab)
            res = srv.drain()
            if len(res) != len(reqs) or any(x["status"] != 0 for x in res):
                raise RuntimeError("serving run lost or failed requests")
            lat = [x["t_done"] - x["t_submit"] for x in res]
            span = max(x["t_done"] for x in res) - min(x["t_submit"] for x in res)
            for x in res:
                i, lab = labs[x["id"]]
                identical &= bool(torch.equal(lab, ref[i]))
            loads.append({"load": rho, "lambda_req_per_s": lam,
                          "p50_ms": 1e3 * _pct(lat, 50), "p99_ms": 1e3 * _pct(lat, 99),
                          "graphs_per_s": len(res) / span,
                          "sequential_p50_ms": 1e3 * _pct(seq_lat, 50), "sequential_p99_ms": 1e3 * _pct(seq_lat, 99),
                          "sequential_graphs_per_s": len(res) / seq_span,
                          "small_path": sum(1 for x in res if x["small_path"])})
            log("serve: load %.1f  p50 %.2f ms  p99 %.2f ms  %.1f graphs/s | sequential p50 %.2f ms  p99 %.2f ms  %.1f graphs/s"
                % (rho, loads[-1]["p50_ms"], loads[-1]["p99_ms"], loads[-1]["graphs_per_s"],
                   loads[-1]["sequential_p50_ms"], loads[-1]["sequential_p99_ms"], loads[-1]["sequential_graphs_per_s"]))
        peak = srv.info()["peak_bytes"]
    finally:
        srv.close()
    del reqs, ref
    torch.cuda.empty_cache()
    if not identical:
        raise RuntimeError("served labels differ from the solo solves")
    return {"requests": len(base_arr), "records": total_m, "budget_gib": args.serve_budget_gib,
            "slots": args.serve_slots, "sequential_capacity_req_per_s": cap, "loads": loads,
            "labels_identical_to_solo": identical, "peak_arena_gib": peak / 2**30}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="er_paths", choices=["er_paths", "small", "rmat26", "rmat24"])
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--eager", action="store_true",
                    help="run every round eagerly even without per-kernel timing (as the timed run does)")
    ap.add_argument("--round0", default="auto", choices=["auto", "direct", "tiled"],
                    help="how round 0 reads the input records (auto: the library's choice by size)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-shrink", type=int, default=8)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-mode leg")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched-mode leg")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-log2-max", type=int, default=18)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--tune-cache", default=None, help="autotune cache file (default: none, tune every run)")
    ap.add_argument("--verbose-tune", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=128)
    ap.add_argument("--serve-log2-max", type=int, default=24)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=int, default=128)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.8, 1.2])
    ap.add_argument("--no-variants", action="store_true",
                    help="skip TreeContraction, the one-hop label and the union-find finish")
    ap.add_argument("--variant-steps", type=int, default=5)
    ap.add_argument("--finish-edges", type=int, default=1 << 22)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    if args.workload == "er_paths":
        g = graphgen.workload_er_paths()
        wname = "G(n=2^24, m=2^27) + 10,000 paths x 1,000 vertices, int32 ids"
    elif args.workload == "small":
        g = graphgen.workload_small()
        wname = "G(n=65,536, m=262,144), int32 ids"
    else:
        scale = 26 if args.workload == "rmat26" else 24
        g = graphgen.workload_rmat(scale=scale)
        wname = "R-MAT scale %d, edge factor 16, (0.57,0.19,0.19,0.05) +-10%%, permuted ids" % scale
    log("generated %s: n=%d m=%d in %.1fs" % (wname, g.n, g.m, time.perf_counter() - t0))

    if args.workload.startswith("rmat"):
        keys = graphgen.pack(g.src, g.dst).view(np.int64)
        src = torch.from_numpy(keys).to(dev)
        dst = None
        layout = lc.CC_EDGES_PACKED_U64
    else:
        src = torch.from_numpy(g.src.view(np.int32)).to(dev)
        dst = torch.from_numpy(g.dst.view(np.int32)).to(dev)
        layout = lc.CC_EDGES_SOA_I32
    loops = int(np.count_nonzero(g.src == g.dst))
    del g.src, g.dst
    n0, m0 = g.n, int(src.shape[0])
    torch.cuda.synchronize()

    # calibration copy for the HBM traffic counters: one plain 1 GiB device-to-device copy
    cal_a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cal_b = torch.empty_like(cal_a)
    cal_b.copy_(cal_a)
    torch.cuda.synchronize()
    # the same copy timed with events: the streaming bandwidth this GPU reaches (read + write),
    # the second denominator beside the 8 TB/s peak
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(COPY_REPS):
        cal_b.copy_(cal_a)
    ev[1].record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * cal_a.numel() * COPY_REPS / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
    log("plain 1 GiB device copy: %.1f GB/s (read + write)" % copy_gbs)
    del cal_a, cal_b

    # Per-kernel events sit only on eagerly launched rounds (a captured tail carries none).
    # Later rounds replay captured tails, unless the dominant family also runs in such rounds:
    # then the solver is made again with every round eager (CC_EAGER), so that each of its
    # launches carries its events on the stream.
    flags = 0 if args.no_profile else lc.CC_PROFILE
    if args.eager:
        flags |= lc.CC_EAGER
    flags |= {"auto": 0, "direct": lc.CC_ROUND0_DIRECT, "tiled": lc.CC_ROUND0_TILED}[args.round0]
    stream = torch.cuda.current_stream(dev)
    base_seed = graphgen.CONFIG_SEED_BASE + 1
    labels = torch.empty(n0, dtype=torch.int32, device=dev)
    solver = lc.Solver(n0, src, dst, seed=base_seed, flags=flags, stream=stream, layout=layout)
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

    def fam_bytes_of(stats_list, keys_list, launches):
        out = {}
        for st, ks in zip(stats_list, keys_list):
            for k, v in family_bytes(st, n0, tiled=launches.get("min1_tiled", 0) > 0, loops=loops,
                                     sorted_keys=ks).items():
                out[k] = out.get(k, 0) + v
        return out

    def log_families(title, acc_ms, acc_n, acc_bytes, steps):
        log("%s: kernel family       ms/step  launches/step  GB/s(alg)" % title)
        for k in sorted(acc_ms, key=lambda x: -acc_ms[x]):
            if acc_n[k] == 0:
                continue
            gbs = acc_bytes.get(k, 0) / (acc_ms[k] * 1e-3) / 1e9 if acc_ms[k] > 0 else 0.0
            log("  %-16s %8.3f %10.1f %10.1f" % (k, acc_ms[k] / steps, acc_n[k] / steps, gbs))

    # Warm-up steps time every kernel family; the dominant one (largest kernel time) is then
    # the only family timed during the measured steps, so that the events of the others do
    # not slow the stream down.  One more warm-up step runs with that setting (it captures
    # the tails of rounds the measured steps replay).
    warm_ms, warm_n, warm_stats, warm_keys = {}, {}, [], []
    for i in range(max(args.warmup - 1, 0) if not args.no_profile else args.warmup):
        r = step(1000 + i)
        warm_stats.append(solver.stats(r))
        warm_keys.append(solver.sorted_keys(r))
        collect(warm_ms, warm_n)
    torch.cuda.synchronize()
    dom = None
    if not args.no_profile and warm_ms:
        warm_bytes = fam_bytes_of(warm_stats, warm_keys, warm_n)
        steps_w = len(warm_stats)
        log_families("warm-up", warm_ms, warm_n, warm_bytes, steps_w)
        log("warm-up: sum of kernel time per step %.3f ms" % (sum(warm_ms.values()) / steps_w))
        dom = max((k for k in warm_ms if k in warm_bytes and warm_n[k] > 0), key=lambda k: warm_ms[k])
        if not tail_free(dom) and not flags & lc.CC_EAGER:
            log("dominant family %s also runs in captured tails: every round eager" % dom)
            flags |= lc.CC_EAGER
            solver.close()
            solver = lc.Solver(n0, src, dst, seed=base_seed, flags=flags, stream=stream, layout=layout)
        solver.profile_families([dom])
        step(2000)
        torch.cuda.synchronize()
    solver.reset(base_seed)            # clears the per-kernel timers too
    all_stats = []
    all_keys = []
    rounds = []
    fam_ms = {}
    fam_n = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step(i)
        rounds.append(r)
        all_stats.append(solver.stats(r))
        all_keys.append(solver.sorted_keys(r))
        collect(fam_ms, fam_n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = m0 * args.steps / dt
    log("rounds per step: %s" % rounds)
    for st, k in zip(all_stats[0], all_keys[0]):
        log("  round %d: n_active=%d m_in=%d survive=%d m_out=%d finalised=%d" % st + " sorted=%d" % k)

    # algorithmic bytes per family over the timed steps
    fam_bytes = fam_bytes_of(all_stats, all_keys, fam_n if dom is None else warm_n)
    job_bytes = sum(job_alg_bytes(st, n0) for st in all_stats)

    roofline = None
    if not args.no_profile and fam_ms:
        if dom is None:
            log_families("timed", fam_ms, fam_n, fam_bytes, args.steps)
            dom = max((k for k in fam_ms if k in fam_bytes and fam_n[k] > 0), key=lambda k: fam_ms[k])
        avg_launch_s = fam_ms[dom] * 1e-3 / fam_n[dom]
        bytes_per_launch = fam_bytes[dom] / fam_n[dom]
        achieved = bytes_per_launch / avg_launch_s / 1e9
        traffic = None
        if dom in FAMILY_SYMBOL and args.workload == "er_paths":
            from paper_1807_10727_amd import profiling
            traffic = profiling.load_traffic(TRAFFIC_FILE, FAMILY_SYMBOL[dom])
        roofline = {"bound": "hbm", "kernel": dom, "symbol": FAMILY_SYMBOL.get(dom), "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else int(traffic),
                    "bytes_per_launch": int(bytes_per_launch), "avg_launch_us": round(avg_launch_s * 1e6, 2),
                    "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
        log("timed steps: %s %.3f ms/step over %d launches/step, %.1f GB/s algorithmic"
            % (dom, fam_ms[dom] / args.steps, fam_n[dom] / args.steps, achieved))

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
            cpu = cpu_baseline(args.cpu_shrink if args.workload == "er_paths" else 8)
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
                   "round0": args.round0, "parallelism": "single GPU"},
        "roofline": roofline,
        "job_alg_frac": round(job_gbs / HBM_PEAK_GBS, 4),
        "job_alg_frac_of_copy": round(job_gbs / copy_gbs, 4),
        "cpu_baseline": cpu,
        "variants": variants,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
