"""Full-size checks, in the launch configuration bench.py times (default flags: the tiled
round 0 where the size allows it, the caller's stream, per-kernel timing on).

Beside the full replays below, each test checks what can be computed one by one or what
holds at any size (the only checks for R-MAT scale 26, too large to replay):
  * round-0 parents of sampled vertices, straight from the definition (the vertex of least
    priority in the closed two-hop neighbourhood, Section 3), in 64-bit (priority, id) keys
    computed with the test-side priority restatement that test_oracle pins to the oracle;
  * round-0 statistics that have a closed form (active nodes, records read);
  * the final labels against textbook union-find: every label is an id of its vertex's
    component and there are exactly as many distinct labels as components;
  * the tiled and the direct round 0 give identical statistics and labels.
The bench graph itself is small enough for the oracle to replay in full (about 1.5 to 2
minutes a run on one core): its labels, round count and per-round statistics are compared
bit for bit, for LocalContraction in the timed configuration and for the other label rules
and the union-find finish as the bench's variant leg runs them.  The four oracle runs start
in threads (the oracle's calls release the interpreter lock) when the module's first test
starts, so they overlap the GPU work.
The batched and serving workloads are checked graph by graph on a seeded sample against the
oracle (labels and round counts, bit for bit)."""
import hashlib
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import graphgen
import oracle
from lcref import spec_priority

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
BENCH_SEED = graphgen.CONFIG_SEED_BASE + 1     # the seed of bench.py's first timed step
RMAT26_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat26_seed_c0ffee01.json")


@pytest.fixture(scope="module")
def lc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10727_amd as lc
    return lc


# How bench.py runs each rule on the bench graph: (oracle variant, solver flags, finish edges).
FULL_RUNS = {
    "local": ("local", "timed", 0),          # CC_PROFILE, the timed steps' flags, on a reused context
    "tree": ("tree", "tree", 0),
    "one_hop": ("one_hop", "one_hop", 0),
    "uf_finish": ("local", 0, 1 << 22),
    "merge_to_large": ("merge_to_large", "merge_to_large", 0),   # default alpha, max(2, ceil(ln n))
}


@pytest.fixture(scope="module")
def er_full():
    """The bench graph and the oracle's runs of it, started in background threads."""
    g = graphgen.workload_er_paths()
    oracle.run(2, np.array([0], np.uint32), np.array([1], np.uint32))   # load the library once
    pool = ThreadPoolExecutor(max_workers=len(FULL_RUNS))
    # LocalContraction's run also keeps round 0's parents (for the round-0 edge set)
    futs = {k: pool.submit(oracle.run, g.n, g.src, g.dst, seed=BENCH_SEED, variant=v, finish_edges=f,
                           record_parents=k == "local", parents_cap=1)
            for k, (v, _, f) in FULL_RUNS.items()}
    yield g, futs
    pool.shutdown(wait=True)


def sampled_round0_parents(src, dst, seed, sample):
    """Round-0 parent of each sampled vertex by the definition; -1 without a loop-free record."""
    keep = src != dst
    a, b = src[keep], dst[keep]

    def key(x):
        x = np.asarray(x, dtype=np.uint32)
        return (spec_priority(seed, 0, x).astype(np.uint64) << np.uint64(32)) | x.astype(np.uint64)

    S = np.unique(np.asarray(sample, dtype=np.uint32))
    ma, mb = np.isin(a, S), np.isin(b, S)
    pv = np.concatenate([a[ma], b[mb]])          # (sampled vertex, neighbour) pairs
    pu = np.concatenate([b[ma], a[mb]])
    U = np.unique(np.concatenate([S, pu]))
    # one-hop minimum over the closed neighbourhood of every u in U
    m1 = key(U)
    has = np.zeros(U.size, dtype=bool)
    for x, y in ((a, b), (b, a)):
        sel = np.isin(x, U)
        idx = np.searchsorted(U, x[sel])
        np.minimum.at(m1, idx, key(y[sel]))
        has[idx] = True
    # two-hop minimum of the sampled vertices
    si = np.searchsorted(U, S)
    lv = m1[si].copy()
    np.minimum.at(lv, np.searchsorted(S, pv), m1[np.searchsorted(U, pu)])
    par = (lv & np.uint64(0xFFFFFFFF)).astype(np.int64)
    par[~has[si]] = -1
    return S, par


def check_partition(labels, comp_min):
    labels = labels.astype(np.int64)
    assert labels.min() >= 0 and labels.max() < comp_min.size
    np.testing.assert_array_equal(comp_min[labels], comp_min)        # label lies in the component
    assert np.unique(labels).size == np.unique(comp_min).size        # one label per component


def solve_full(lc, n, src_t, dst_t, layout, flags, seed):
    out = {}
    stream = torch.cuda.current_stream()
    with lc.Solver(n, src_t, dst_t, seed=seed, flags=flags | lc.CC_PROFILE, stream=stream, layout=layout) as s:
        st, stats0 = s.contract_round()
        assert st == lc.CC_OK
        par, k = s.parents()
        out["par0"] = par.cpu().numpy().astype(np.int64)
        rounds = s.run()
        out["stats"] = s.stats(rounds)
        out["labels"] = s.labels().cpu().numpy()
        out["times"] = s.kernel_times()
    return out


def run_full_graph(lc, g, layout, seed, sample_size):
    n = g.n
    if layout == "packed":
        keys = graphgen.pack(g.src, g.dst).view(np.int64)
        src_t, dst_t, lay = torch.from_numpy(keys).to(DEV), None, lc.CC_EDGES_PACKED_U64
        del keys
    else:
        src_t = torch.from_numpy(g.src.view(np.int32)).to(DEV)
        dst_t = torch.from_numpy(g.dst.view(np.int32)).to(DEV)
        lay = lc.CC_EDGES_SOA_I32
    torch.cuda.synchronize()
    tiled = solve_full(lc, n, src_t, dst_t, lay, 0, seed)
    assert tiled["times"]["min1_tiled"][1] == 1          # the default chose the tiled round 0
    direct = solve_full(lc, n, src_t, dst_t, lay, lc.CC_ROUND0_DIRECT, seed)
    assert direct["times"]["min1_round0"][1] == 1
    del src_t, dst_t
    torch.cuda.empty_cache()
    assert tiled["stats"] == direct["stats"]
    np.testing.assert_array_equal(tiled["labels"], direct["labels"])
    np.testing.assert_array_equal(tiled["par0"], direct["par0"])

    # round 0 statistics with a closed form
    keep = g.src != g.dst
    active = np.unique(np.concatenate([g.src[keep], g.dst[keep]])).size
    r0 = tiled["stats"][0]
    assert r0[0] == 0 and r0[1] == active and r0[2] == g.m

    # sampled round-0 parents from the definition
    rng = np.random.default_rng(seed & 0xFFFF)
    sample = rng.choice(n, size=sample_size, replace=False)
    S, want = sampled_round0_parents(g.src, g.dst, seed, sample)
    np.testing.assert_array_equal(tiled["par0"][S], want)

    # labels against union-find
    check_partition(tiled["labels"], oracle.components_min_id(n, g.src, g.dst).astype(np.int64))
    return tiled


@pytest.mark.timeout(900)
def test_er_paths_full_size(lc, er_full):
    """G(2^24, 2^27) + 10,000 paths of 1,000 vertices (26,777,216 ids, 144,207,728 records)."""
    g, _ = er_full
    out = run_full_graph(lc, g, "soa32", BENCH_SEED, 2000)
    assert len(out["stats"]) >= 5           # a 1,000-vertex path needs >= log5(1000) phases (Section 7)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("rule", list(FULL_RUNS))
def test_er_paths_full_size_vs_oracle(lc, er_full, rule):
    """The bench graph at the bench's first seed, bit for bit against the oracle: labels,
    round count, per-round statistics, and whether the union-find finish ran."""
    g, futs = er_full
    _, how, finish = FULL_RUNS[rule]
    flags = {"timed": lc.CC_PROFILE, "tree": lc.CC_TREE, "one_hop": lc.CC_ONE_HOP,
             "merge_to_large": lc.CC_MERGE_TO_LARGE}.get(how, how)
    src_t = torch.from_numpy(g.src.view(np.int32)).to(DEV)
    dst_t = torch.from_numpy(g.dst.view(np.int32)).to(DEV)
    with lc.Solver(g.n, src_t, dst_t, seed=BENCH_SEED, flags=flags, stream=torch.cuda.current_stream(),
                   finish_edges=finish) as s:
        if how == "timed":
            # as in the bench's timed steps: a context that has solved before, so the rounds
            # of at most 2^22 records replay a captured tail
            s.reset(BENCH_SEED + 1000)
            s.run()
            s.reset(BENCH_SEED)
        rounds = s.run()
        if how == "timed":
            assert any(s.rounds_in_graph(rounds))
        stats = s.stats(rounds)
        keys = s.sorted_keys(rounds)
        finished = s.finished
        labels = s.labels().cpu().numpy()
    del src_t, dst_t
    torch.cuda.empty_cache()
    # Round 1 reads more records than the host lets a round hash, so the device chooses once
    # the relabel has counted its keys: LocalContraction's 121 M records leave ~1.5 M keys
    # (hashed), the one-hop rule keeps 108 M distinct edges (sorted).  Both choices are then
    # checked bit for bit below.
    if rule != "merge_to_large":
        assert stats[1][2] > 1 << 22
    if rule == "local":
        assert keys[1] <= 1 << 22
    if rule == "one_hop":
        assert keys[1] > 1 << 22
    want = futs[rule].result()
    assert rounds == want.rounds
    assert finished == want.finished == (finish > 0)
    assert [tuple(x) for x in stats] == [tuple(x) for x in want.stats]
    np.testing.assert_array_equal(labels.astype(np.uint32), want.labels)


@pytest.mark.timeout(900)
def test_er_paths_round0_edges(lc, er_full):
    """The edge set round 0 leaves on the bench graph (121.8 M distinct edges out of 144 M
    records), in the timed configuration, equals the input contracted through the oracle's
    round-0 parents, edge for edge."""
    from lcref import contract_edges
    g, _ = er_full
    src_t = torch.from_numpy(g.src.view(np.int32)).to(DEV)
    dst_t = torch.from_numpy(g.dst.view(np.int32)).to(DEV)
    with lc.Solver(g.n, src_t, dst_t, seed=BENCH_SEED, flags=lc.CC_PROFILE | lc.CC_EAGER,
                   stream=torch.cuda.current_stream()) as s:
        st, stats = s.contract_round()
        assert st == lc.CC_OK
        got = s.edges()
        got = np.sort(got.cpu().numpy().view(np.uint64))
    del src_t, dst_t
    torch.cuda.empty_cache()
    g, futs = er_full
    want = contract_edges(g.src, g.dst, futs["local"].result().parents[0])
    assert want.size == stats[4] == got.size
    np.testing.assert_array_equal(got, want)


TUNED = [{"round0_sort": 2}, {"round0": 3}, {"round0": 3, "round0_sort": 2, "round0_key_sets": 0},
         {"round0": 1, "round0_sort": 2}, {"row_pairs": 8, "relabel_pairs": 4, "row_generation": -1, "scatter_waves": 4},
         {"radix_form": 2, "tail": 3}, {"round0": 1, "radix_form": 2, "tail": 2}]


@pytest.mark.timeout(900)
def test_er_paths_tuned_vs_oracle(lc, er_full):
    """The bench graph under the knobs the tuner may pick (the sampled-bucket sort of round 0's
    129 M keys, the one-pass row partition, the direct round 0, other row-pass and scatter
    builds, the one-sweep radix passes, the small rounds in one persistent launch): rounds,
    statistics and labels bit for bit against the oracle."""
    g, futs = er_full
    src_t = torch.from_numpy(g.src.view(np.int32)).to(DEV)
    dst_t = torch.from_numpy(g.dst.view(np.int32)).to(DEV)
    want = futs["local"].result()
    with lc.Solver(g.n, src_t, dst_t, seed=BENCH_SEED, stream=torch.cuda.current_stream()) as s:
        for knobs in TUNED:
            print("knobs", knobs, flush=True)
            s.set_tuning(**knobs)
            rounds = s.run()
            assert rounds == want.rounds, knobs
            assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats], knobs
            np.testing.assert_array_equal(s.labels().cpu().numpy().view(np.uint32), want.labels, err_msg=str(knobs))
    del src_t, dst_t
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def rmat26():
    return graphgen.workload_rmat()


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_rmat26_full_size(lc, rmat26):
    """R-MAT scale 26, edge factor 16 (1,073,741,824 packed records, 2^26 ids): the checks
    that hold at any size (sampled round-0 parents from the definition, closed-form round-0
    statistics, partition against union-find, tiled = direct)."""
    run_full_graph(lc, rmat26, "packed", graphgen.CONFIG_SEED_BASE + 2, 500)


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_rmat26_bit_exact_vs_oracle(lc, rmat26):
    """R-MAT scale 26 at the bench's first seed against the oracle's stored results
    (tests/golden/rmat26_seed_c0ffee01.json, written by make_rmat26_golden.py from the oracle
    alone): in the timed configuration (tiled round 0, CC_PROFILE, a context that has solved
    before) the round count, every round's statistics and the SHA-256 of the raw labels; the
    same under the knobs the tuner may pick; with
    every round recorded, round 0 direct and tiled, the SHA-256 of every round's parents by
    name; and the canonical labels."""
    with open(RMAT26_GOLDEN) as f:
        gold = json.load(f)
    assert gold["seed"] == BENCH_SEED and gold["n_records"] == rmat26.m
    keys = torch.from_numpy(graphgen.pack(rmat26.src, rmat26.dst).view(np.int64)).to(DEV)
    n = rmat26.n
    stream = torch.cuda.current_stream()
    want_stats = [tuple(x) for x in gold["stats"]]
    with lc.Solver(n, keys, None, seed=BENCH_SEED, flags=lc.CC_PROFILE, stream=stream) as s:
        s.reset(BENCH_SEED + 1000)
        s.run()
        s.reset(BENCH_SEED)
        rounds = s.run()
        assert s.kernel_times()["min1_tiled"][1] == 1
        assert rounds == gold["rounds"]
        assert [tuple(x) for x in s.stats(rounds)] == want_stats
        assert _sha(s.labels().cpu().numpy().view(np.uint32)) == gold["labels_sha256"]
    torch.cuda.empty_cache()
    with lc.Solver(n, keys, None, seed=BENCH_SEED, stream=stream) as s:   # the knobs the tuner may pick
        for knobs in TUNED:
            print("knobs", knobs, flush=True)
            s.set_tuning(**knobs)
            rounds = s.run()
            assert rounds == gold["rounds"], knobs
            assert [tuple(x) for x in s.stats(rounds)] == want_stats, knobs
            assert _sha(s.labels().cpu().numpy().view(np.uint32)) == gold["labels_sha256"], knobs
    torch.cuda.empty_cache()
    for flags in (lc.CC_ROUND0_DIRECT, lc.CC_ROUND0_TILED | lc.CC_CANONICAL):
        with lc.Solver(n, keys, None, seed=BENCH_SEED, flags=flags | lc.CC_RECORD_ROUNDS, stream=stream) as s:
            rounds = s.run()
            assert rounds == gold["rounds"]
            assert [tuple(x) for x in s.stats(rounds)] == want_stats
            for r in range(rounds):
                par, k = s.parents(r)
                assert _sha(par.cpu().numpy()) == gold["parents_sha256"][r], "round %d, flags %d" % (r, flags)
                assert k == want_stats[r][1]
            lab = s.labels().cpu().numpy().view(np.uint32)
            key = "canonical_labels_sha256" if flags & lc.CC_CANONICAL else "labels_sha256"
            assert _sha(lab) == gold[key]
        torch.cuda.empty_cache()
    del keys
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_batch_4096_sampled(lc):
    """The 4,096-graph batch of the batched benchmark, default configuration: 96 graphs
    drawn at random are each checked against the oracle's labels and round count."""
    b = graphgen.batch_mix()
    src = torch.from_numpy(b.src.view(np.int32)).to(DEV)
    dst = torch.from_numpy(b.dst.view(np.int32)).to(DEV)
    with lc.Batch(b.voff, b.eoff, b.seeds, src, dst) as bt:
        lab, rounds = bt.run()
        lab = lab.cpu().numpy()
    pick = np.random.default_rng(7).choice(b.count, size=96, replace=False)
    for j in pick:
        g = b.graph(int(j))
        want = oracle.run(g.n, g.src, g.dst, seed=int(b.seeds[j]))
        a = int(b.voff[j])
        np.testing.assert_array_equal(lab[a:a + g.n].astype(np.uint32), want.labels, err_msg="graph %d" % j)
        assert rounds[j] == want.rounds, "graph %d" % j


@pytest.mark.timeout(900)
def test_serving_trace_sampled(lc):
    """The first 24 requests of the serving benchmark's trace (log-uniform sizes up to
    2^24 vertices, 620 M records in all), submitted at once: each result equals its solo
    solve and the oracle's labels and round count (the oracle runs in threads, started
    first, so that it overlaps the GPU work)."""
    trace = graphgen.request_trace(graphgen.CONFIG_SEED_BASE + 4, 24, rate=1.0)
    graphs = [r.graph() for r in trace]
    oracle.run(2, np.array([0], np.uint32), np.array([1], np.uint32))   # load the library once
    pool = ThreadPoolExecutor(max_workers=8)
    order = sorted(range(len(graphs)), key=lambda i: -graphs[i].m)      # largest first
    futs = {i: pool.submit(oracle.run, graphs[i].n, graphs[i].src, graphs[i].dst, seed=trace[i].seed)
            for i in order}
    dev = [(torch.from_numpy(g.src.view(np.int32)).to(DEV), torch.from_numpy(g.dst.view(np.int32)).to(DEV))
           for g in graphs]
    torch.cuda.synchronize()
    with lc.Server(96 << 30, n_slots=8, small_variant=1, max_small_per_launch=256) as srv:
        labs = {}
        for i, (g, r) in enumerate(zip(graphs, trace)):
            rid, lab = srv.submit(g.n, dev[i][0], dev[i][1], r.seed)
            labs[rid] = (i, lab)
        results = srv.drain()
    assert len(results) == len(trace)
    for res in results:
        assert res["status"] == 0
        i, lab = labs[res["id"]]
        g, r = graphs[i], trace[i]
        got = lab.cpu().numpy()
        solo, rounds, _ = lc.solve(g.n, dev[i][0], dev[i][1], seed=r.seed)
        np.testing.assert_array_equal(got, solo.cpu().numpy(), err_msg="request %d" % i)
        assert res["rounds"] == rounds
        want = futs[i].result()
        np.testing.assert_array_equal(got.astype(np.uint32), want.labels, err_msg="request %d" % i)
        assert res["rounds"] == want.rounds
    pool.shutdown(wait=True)
