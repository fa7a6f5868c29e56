"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact on integers: per-round parents by name, per-round statistics, round count and
final labels, on seeded synthetic graphs that span several sort tiles with ragged tails,
all input layouts, and the degenerate cases of the method.
"""
import numpy as np
import pytest

import graphgen
import oracle
from lcref import all_graph_adjacency, brute_all, contract_edges, graph_records, spec_priority, split_keys

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10727_amd as lc
    return lc


DEV = "cuda:0"
# round 0 reads the input directly, or through the tiled layout (flag values of include/cc.h)
MODES = {"direct": 1 << 2, "tiled": 1 << 3}


def to_device(g, layout="soa32", offset=0):
    """Edge tensors of graph `g` in the given layout; `offset` > 0 misaligns the pointers."""
    if layout == "soa32":
        s = torch.from_numpy(np.concatenate([np.zeros(offset, np.uint32), g.src]).view(np.int32)).to(DEV)
        d = torch.from_numpy(np.concatenate([np.zeros(offset, np.uint32), g.dst]).view(np.int32)).to(DEV)
        return s[offset:], d[offset:], None
    if layout == "soa64":
        s = torch.from_numpy(np.concatenate([np.zeros(offset, np.int64), g.src.astype(np.int64)])).to(DEV)
        d = torch.from_numpy(np.concatenate([np.zeros(offset, np.int64), g.dst.astype(np.int64)])).to(DEV)
        return s[offset:], d[offset:], None
    k = graphgen.pack(g.src, g.dst).view(np.int64)
    k = torch.from_numpy(np.concatenate([np.zeros(offset, np.int64), k])).to(DEV)
    return k[offset:], None, 2


def gpu_solve(lc, g, seed, layout="soa32", per_round=True, flags=0, max_rounds=0, offset=0, tuning=None):
    s_t, d_t, lay = to_device(g, layout, offset)
    out = {"parents": [], "stats": []}
    with lc.Solver(g.n, s_t, d_t, seed=seed, flags=flags, max_rounds=max_rounds, layout=lay) as s:
        if tuning:
            s.set_tuning(**tuning)
        if per_round:
            while max_rounds == 0 or len(out["stats"]) < max_rounds:
                st, stats = s.contract_round()
                if st == lc.CC_DONE:
                    break
                out["stats"].append(stats)
                par, k = s.parents()
                out["parents"].append(par.cpu().numpy().view(np.uint32).copy())
                assert k == stats[1]
                out.setdefault("edges", []).append(np.sort(s.edges().cpu().numpy().view(np.uint64)))
            # finish via cc_run (no rounds left, or stops at max_rounds)
            out["rounds"] = s.run()
        else:
            out["rounds"] = s.run()
            out["stats"] = s.stats(out["rounds"])
        lab = s.labels()
        torch.cuda.synchronize()
        out["labels"] = lab.cpu().numpy()
    return out


def check(lc, g, seed, **kw):
    max_rounds = kw.get("max_rounds", 0)
    want = oracle.run(g.n, g.src, g.dst, seed=seed, record_parents=True, max_rounds=max_rounds)
    got = gpu_solve(lc, g, seed, **kw)
    assert got["rounds"] == want.rounds
    assert [tuple(x) for x in got["stats"]] == [tuple(x) for x in want.stats]
    if kw.get("per_round", True):
        assert len(got["parents"]) == want.rounds
        for r in range(want.rounds):
            np.testing.assert_array_equal(got["parents"][r], want.parents[r], err_msg="round %d" % r)
        # the graph each round left: the contraction of the previous one through the oracle's
        # parents (the input records for round 0)
        a, b = g.src, g.dst
        for r in range(len(got.get("edges", []))):
            want_e = contract_edges(a, b, want.parents[r])
            np.testing.assert_array_equal(got["edges"][r], want_e, err_msg="edges after round %d" % r)
            assert want_e.size == want.stats[r][4]
            a, b = split_keys(want_e)
    lab = got["labels"]
    np.testing.assert_array_equal(lab.astype(np.int64), want.labels.astype(np.int64))
    return want


# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("n,m,seed", [(100, 300, 1), (1000, 4097, 2), (5000, 20001, 3), (3000, 2000, 4),
                                      (20000, 61441, 5)])
def test_gnm_parity(lc, n, m, seed, mode):
    g = graphgen.Graph(n, *graphgen.gnm(seed * 7919, n, m))
    check(lc, g, seed, flags=MODES[mode])


@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
@pytest.mark.parametrize("n,m,seed", [(5000, 20001, 3), ((1 << 20) + 3, (1 << 22) + 1, 6)])
def test_bucket_sort_parity(lc, n, m, seed, mode):
    """Round 0's keys ordered by the sampled buckets (two levels of splitters, each final
    bucket sorted in LDS) instead of the radix passes, round by round against the oracle; the
    larger graph fills the 65,536 final buckets with ~60 keys each."""
    g = graphgen.Graph(n, *graphgen.gnm(seed * 7919, n, m))
    tuning = {"round0_sort": 2, "round0": 3 if mode == "rows" else 0}
    check(lc, g, seed, flags=MODES["direct" if mode == "direct" else "tiled"], tuning=tuning)


@pytest.mark.parametrize("n,m,seed", [((1 << 20) + 3, (1 << 22) + 1, 6), ((1 << 22) + 7777, 1 << 23, 7)])
def test_tiled_full_blocks_parity(lc, n, m, seed):
    """Sizes where the tiled round 0 is the default: 256 row blocks of 2^12 ids, then
    row blocks of 2^15 ids (the whole LDS) with 2^15-id column blocks, ragged last blocks."""
    g = graphgen.Graph(n, *graphgen.gnm(seed * 104729, n, m))
    check(lc, g, seed)


def test_tiled_largest_id_space(lc):
    """The largest id space the tiled round 0 takes (2^26 ids: 2048 row blocks of 2^15 ids,
    the most the row digit holds), sparse records over all of it, against the oracle round
    by round."""
    n = 1 << 26
    g = graphgen.Graph(n, *graphgen.gnm(0x7171, n, 1 << 21))
    check(lc, g, 13, flags=MODES["tiled"])


def test_small_workload_parity(lc):
    """G(n, m) with n = 65,536 and m = 262,144, every round and the labels bit-exact."""
    g = graphgen.workload_small()
    w = check(lc, g, seed=0xC0FFEE00)
    assert w.rounds >= 2


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("scale,ef", [(10, 8), (13, 16)])
def test_rmat_parity(lc, scale, ef, mode):
    g = graphgen.Graph(1 << scale, *graphgen.rmat(scale * 31, scale, ef << scale))
    check(lc, g, seed=scale, flags=MODES[mode])


@pytest.mark.parametrize("mode", sorted(MODES))
def test_paths_parity_many_rounds(lc, mode):
    g = graphgen.er_with_paths(17, 1 << 11, 1 << 12, 30, 700)
    w = check(lc, g, seed=99, flags=MODES[mode])
    assert w.rounds >= 5


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("layout", ["soa32", "soa64", "packed"])
@pytest.mark.parametrize("offset", [0, 1])
def test_layouts_and_alignment(lc, layout, offset, mode):
    g = graphgen.Graph(3001, *graphgen.gnm(44, 3001, 9003))
    check(lc, g, seed=5, layout=layout, offset=offset, per_round=False, flags=MODES[mode])


@pytest.mark.parametrize("mode", sorted(MODES))
def test_union_of_all_graphs_on_five_vertices(lc, mode):
    adj = all_graph_adjacency(5)
    src, dst, eoff = graph_records(adj)
    G = adj.shape[0]
    gid = np.repeat(np.arange(G), np.diff(eoff))
    g = graphgen.Graph(5 * G, (src + 5 * gid).astype(np.uint32), (dst + 5 * gid).astype(np.uint32))
    check(lc, g, seed=12345, flags=MODES[mode])


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("case", ["empty", "no_edges", "loops_only", "single_edge", "duplicates", "isolated",
                                  "one_vertex"])
def test_degenerate_cases(lc, case, mode):
    if case == "empty":
        g = graphgen.Graph(0, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    elif case == "no_edges":
        g = graphgen.Graph(17, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    elif case == "loops_only":
        g = graphgen.Graph(9, np.array([3, 3, 8], np.uint32), np.array([3, 3, 8], np.uint32))
    elif case == "single_edge":
        g = graphgen.Graph(2, np.array([1], np.uint32), np.array([0], np.uint32))
    elif case == "duplicates":
        g = graphgen.Graph(6, np.array([0, 1, 1, 0, 2, 4, 5, 4], np.uint32), np.array([1, 0, 0, 1, 2, 5, 4, 5], np.uint32))
    elif case == "isolated":
        g = graphgen.Graph(1000, np.array([10, 500], np.uint32), np.array([999, 10], np.uint32))
    else:
        g = graphgen.Graph(1, np.zeros(3, np.uint32), np.zeros(3, np.uint32))
    check(lc, g, seed=3, flags=MODES[mode])


@pytest.mark.parametrize("mode", sorted(MODES))
def test_max_rounds_partial_labels(lc, mode):
    g = graphgen.er_with_paths(5, 0, 0, 20, 400)
    for k in (1, 2, 3):
        check(lc, g, seed=8, max_rounds=k, flags=MODES[mode])
        # cc_run alone, the rounds after round 0 in the persistent launch, stopping at k
        check(lc, g, seed=8, max_rounds=k, flags=MODES[mode], per_round=False, tuning={"tail": 2})


def test_canonical_labels(lc):
    g = graphgen.workload_small(seed=77)
    s_t, d_t, _ = to_device(g)
    lab, rounds, _ = lc.solve(g.n, s_t, d_t, seed=4, flags=lc.CC_CANONICAL)
    np.testing.assert_array_equal(lab.cpu().numpy().astype(np.uint32), oracle.components_min_id(g.n, g.src, g.dst))


@pytest.mark.parametrize("mode", sorted(MODES))
def test_invalid_ids_rejected(lc, mode):
    g = graphgen.Graph(100, np.array([1, 2, 100], np.uint32), np.array([2, 3, 4], np.uint32))
    s_t, d_t, _ = to_device(g)
    with lc.Solver(g.n, s_t, d_t, seed=1, flags=MODES[mode]) as s:
        with pytest.raises(lc.CCError) as e:
            s.run()
        assert e.value.status == -2
    neg = torch.tensor([-1, 2], dtype=torch.int32, device=DEV)
    ok = torch.tensor([2, 3], dtype=torch.int32, device=DEV)
    with lc.Solver(10, neg, ok, seed=1, flags=MODES[mode]) as s:
        with pytest.raises(lc.CCError):
            s.run()


def test_reset_repeat_and_reseed(lc):
    g = graphgen.Graph(4000, *graphgen.gnm(2, 4000, 12000))
    s_t, d_t, _ = to_device(g)
    with lc.Solver(g.n, s_t, d_t, seed=1) as s:
        s.run()
        a = s.labels().cpu().numpy().copy()
        s.reset(1)
        s.run()
        b = s.labels().cpu().numpy().copy()
        s.reset(2)
        r2 = s.run()
        c = s.labels().cpu().numpy().copy()
    np.testing.assert_array_equal(a, b)
    want = oracle.run(g.n, g.src, g.dst, seed=2)
    assert r2 == want.rounds
    np.testing.assert_array_equal(c.astype(np.uint32), want.labels)


def test_edge_order_does_not_matter(lc):
    g = graphgen.Graph(5000, *graphgen.gnm(9, 5000, 15000))
    perm = np.random.default_rng(0).permutation(g.m)
    h = graphgen.Graph(g.n, g.dst[perm].copy(), g.src[perm].copy())
    a = gpu_solve(lc, g, 3, per_round=False)
    b = gpu_solve(lc, h, 3, per_round=False)
    np.testing.assert_array_equal(a["labels"], b["labels"])
    assert a["stats"] == b["stats"]


def test_profile_times_kernels(lc):
    g = graphgen.workload_small()
    s_t, d_t, _ = to_device(g)
    with lc.Solver(g.n, s_t, d_t, seed=1, flags=lc.CC_PROFILE | lc.CC_EAGER) as s:
        r = s.run()
        t = s.kernel_times()
    assert t["min1_round0"][1] == 1 and t["min1"][1] == r - 1 and t["min1_tiled"][1] == 0
    assert t["min1_round0"][0] > 0 and t["sort_scatter"][0] > 0
    with lc.Solver(g.n, s_t, d_t, seed=1, flags=lc.CC_PROFILE | lc.CC_ROUND0_TILED | lc.CC_EAGER) as s:
        r2 = s.run()
        t = s.kernel_times()
    assert r2 == r
    assert t["min1_round0"][1] == 0 and t["min1_tiled"][1] == 1 and t["relabel_tiled"][1] == 1
    assert t["part_a_hist"][1] == 1 and t["part_b_scatter"][1] == 1 and t["min1"][1] == r - 1
    with lc.Solver(g.n, s_t, d_t, seed=1, flags=lc.CC_PROFILE) as s:
        s.profile_families(["sort_scatter"])
        s.run()
        t = s.kernel_times()
    assert t["sort_scatter"][1] > 0 and t["sort_scatter"][0] > 0
    assert all(n == 0 for k, (_, n) in t.items() if k != "sort_scatter")


def test_tuning_knobs_keep_results(lc):
    """Every cc_tuning setting gives the oracle's rounds, counts and labels: the three round-0
    forms (direct, tiled with the two-pass partition, tiled with the one-pass row partition),
    grid sizes and round 0's key sets, on a power-law graph of many partition tiles with a
    ragged last tile."""
    g = graphgen.Graph(1 << 16, *graphgen.rmat(0x7077, 16, (12 << 16) + 4093))
    want = oracle.run(g.n, g.src, g.dst, seed=11)
    s_t, d_t, _ = to_device(g)
    with lc.Solver(g.n, s_t, d_t, seed=11, flags=MODES["tiled"] | lc.CC_PROFILE) as s:
        for r0 in (1, 2, 3):
            for bpc in (1, 8, 16):
                for ks in (1, 0):
                    s.set_tuning(round0=r0, blocks_per_cu=bpc, round0_key_sets=ks)
                    assert {k: s.tuning[k] for k in ("round0", "blocks_per_cu", "round0_key_sets")} == \
                        {"round0": r0, "blocks_per_cu": bpc, "round0_key_sets": ks}
                    r = s.run()
                    assert r == want.rounds, (r0, bpc, ks)
                    assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats], (r0, bpc, ks)
                    assert np.array_equal(s.labels().cpu().numpy().view(np.uint32), want.labels), (r0, bpc, ks)
                    t = s.kernel_times()   # this solve's launches (a reset clears them)
                    ran = {f for f in ("min1_round0", "part_a_hist", "part_b_scatter", "part_rows_hist",
                                       "part_rows_scatter") if t[f][1]}
                    assert ran == [set(), {"min1_round0"}, {"part_a_hist", "part_b_scatter"},
                                   {"part_rows_hist", "part_rows_scatter"}][r0], (r0, ran)


@pytest.mark.parametrize("r0", [2, 3])
def test_kernel_knobs_keep_results(lc, r0):
    """The kernel builds and launch shapes the tuner may pick (radix scatter waves, record
    pairs in flight in the tiled row passes, rows launched together, round 0's sampled-bucket
    sort) give the oracle's rounds, statistics and labels, on a power-law graph of many rows
    and partition tiles."""
    g = graphgen.Graph(1 << 17, *graphgen.rmat(0x7078, 17, (12 << 17) + 1021))
    want = oracle.run(g.n, g.src, g.dst, seed=13)
    s_t, d_t, _ = to_device(g)
    with lc.Solver(g.n, s_t, d_t, seed=13, flags=MODES["tiled"]) as s:
        for knob, values in (("scatter_waves", (2, 3, 4)), ("row_pairs", (2, 4, 8)), ("relabel_pairs", (1, 2, 4)),
                             ("row_generation", (1, 2, 8, -1)), ("round0_sort", (1, 2)), ("radix_form", (1, 2))):
            for v in values:
                s.set_tuning(round0=r0, **{knob: v})
                assert s.tuning[knob] == v and s.tuning["round0"] == r0
                r = s.run()
                assert r == want.rounds, (knob, v)
                assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats], (knob, v)
                assert np.array_equal(s.labels().cpu().numpy().view(np.uint32), want.labels), (knob, v)


# --- heavy repeats and a hub ------------------------------------------------------------

def dup_path(nv, reps, seed):
    """A path on nv ids whose every edge is repeated reps times, in shuffled order."""
    a = np.repeat(np.arange(nv - 1, dtype=np.uint32), reps)
    perm = np.random.default_rng(seed).permutation(a.size)
    return graphgen.Graph(nv, a[perm].copy(), (a[perm] + 1).astype(np.uint32))


def sun(k, seed):
    """A centre joined to k paths of six edges; the centre and the first two vertices of
    every path take the low ids, so after round 0 the merged centre is the smaller
    endpoint of most edges of the next graph (a hub with about k distinct neighbours)."""
    c = 0
    a = 1 + np.arange(k, dtype=np.uint32)
    b = 1 + k + np.arange(k, dtype=np.uint32)
    rest = [1 + 2 * k + j * k + np.arange(k, dtype=np.uint32) for j in range(4)]
    chain = [np.full(k, c, np.uint32), a, b] + rest
    src = np.concatenate(chain[:-1])
    dst = np.concatenate(chain[1:])
    perm = np.random.default_rng(seed).permutation(src.size)
    return graphgen.Graph(1 + 6 * k, src[perm].copy(), dst[perm].copy())


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("case", ["dup_path_12", "dup_path_300", "sun_40000"])
def test_heavy_repeats_and_hub(lc, case, mode):
    """Survivors with 9,000 repeats of every key (12 and 300 ids), and a hub whose edges to
    ~40,000 distinct neighbours all share their smaller endpoint: the duplicate drop keeps
    exactly one copy; bit-exact with the oracle."""
    seed = 21
    if case == "dup_path_12":
        g = dup_path(12, 9000, 1)
    elif case == "dup_path_300":
        g = dup_path(300, 9000, 2)
    else:
        g = sun(40000, 3)
    w = check(lc, g, seed, flags=MODES[mode])
    assert w.stats[0][3] > 2 * w.stats[0][4] or case == "sun_40000"   # many repeats dropped


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("seed", [2, 5])
def test_relabel_drops_workgroup_repeats(lc, mode, seed):
    """G(2^15, 2^18), seeds whose round 1 maps 3,100-4,600 survivors onto five or fewer
    parent pairs.  The relabel workgroups drop the repeats they recognise themselves before
    the sort: the keys sorted lie between the distinct edges out and the survivors, far fewer
    than the survivors in round 1, and rounds, statistics and labels stay bit-exact with the
    oracle."""
    g = graphgen.Graph(1 << 15, *graphgen.gnm(31, 1 << 15, 1 << 18))
    s_t, d_t, _ = to_device(g)
    with lc.Solver(g.n, s_t, d_t, seed=seed, flags=MODES[mode] | lc.CC_EAGER) as s:
        r = s.run()
        st = [tuple(x) for x in s.stats(r)]
        ks = s.sorted_keys(r)
        lab = s.labels().cpu().numpy()
    want = oracle.run(g.n, g.src, g.dst, seed=seed)
    assert r == want.rounds and st == [tuple(x) for x in want.stats]
    np.testing.assert_array_equal(lab.astype(np.uint32), want.labels)
    for x, k in zip(st, ks):
        assert x[4] <= k <= x[3]
    assert st[1][3] > 1000 and ks[1] * 10 < st[1][3]


def test_captured_tail_matches_eager_and_oracle(lc):
    """On a reused context cc_run replays a captured graph of rounds once the remaining graph
    is small: the same statistics and labels as eager rounds and as the oracle, for
    consecutive solves with different seeds on one context, on a graph of many rounds."""
    g = graphgen.er_with_paths(17, 1 << 11, 1 << 12, 30, 700)
    s_t, d_t, _ = to_device(g)
    with lc.Solver(g.n, s_t, d_t, seed=1) as tail, lc.Solver(g.n, s_t, d_t, seed=1, flags=lc.CC_EAGER) as eager:
        first = True
        for seed in (11, 12, 13, 11):
            tail.reset(seed)
            eager.reset(seed)
            rt, re_ = tail.run(), eager.run()
            want = oracle.run(g.n, g.src, g.dst, seed=seed)
            assert rt == re_ == want.rounds
            assert [tuple(x) for x in tail.stats(rt)] == [tuple(x) for x in want.stats]
            assert tail.stats(rt) == eager.stats(re_)
            flags = tail.rounds_in_graph(rt)
            if first:   # a fresh context solves eagerly; reuse brings the captured tail
                assert not any(flags)
            else:
                assert not flags[0] and any(flags)
            first = False
            assert not any(eager.rounds_in_graph(re_))
            lt, le = tail.labels(), eager.labels()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(lt.cpu().numpy(), le.cpu().numpy())
            np.testing.assert_array_equal(lt.cpu().numpy().astype(np.uint32), want.labels)
        with pytest.raises(lc.CCError) as e:
            tail.parents()
        assert e.value.status == -5     # CC_E_STATE: the last round ran inside the graph
        with pytest.raises(lc.CCError) as e:
            tail.edges()
        assert e.value.status == -5
        assert eager.edges().numel() == 0   # an eager solve that ran to the end left no edge


@pytest.mark.parametrize("mode", sorted(MODES))
def test_one_sweep_radix_parity(lc, mode):
    """cc_tuning.radix_form = 2 (one count pass for every digit, then per digit a scatter whose
    tile offsets come from decoupled look-back across the workgroups running at once): round
    by round and the labels, on a uniform graph of 2^20 ids whose rounds 0 and 1 sort (round 1
    also with the hashed drop enqueued, the device choosing), and on an R-MAT graph."""
    for g, seed in ((graphgen.Graph(1 << 20, *graphgen.gnm(0x5EE9, 1 << 20, 3 << 20)), 7),
                    (graphgen.Graph(1 << 18, *graphgen.rmat(0x5EEA, 18, 16 << 18)), 8)):
        check(lc, g, seed, flags=MODES[mode], tuning={"radix_form": 2})


@pytest.mark.parametrize("tail", [2, 3, 4])
@pytest.mark.parametrize("rule", ["local", "one_hop", "tree"])
def test_persistent_rounds_match_oracle(lc, tail, rule):
    """cc_tuning.tail >= 2: the rounds after round 0 run in one cooperative launch with
    grid-wide barriers between their steps.  The oracle's rounds, statistics and labels, on a
    fresh and a reused context with several seeds, on a graph whose round 1 has more than 2^18
    nodes (the label and node maps' multi-phase form) and whose later rounds have fewer (the
    one-workgroup form); those rounds report in_graph = 2 and are timed as "fused_rounds"."""
    g = graphgen.er_with_paths(0xB16, 1 << 12, 1 << 13, 1000, 1000)
    s_t, d_t, _ = to_device(g)
    flags = {"local": 0, "one_hop": lc.CC_ONE_HOP, "tree": lc.CC_TREE}[rule]
    with lc.Solver(g.n, s_t, d_t, seed=1, flags=flags | lc.CC_PROFILE) as s:
        s.set_tuning(tail=tail)
        assert s.tuning["tail"] == tail
        for seed in (21, 22, 21):
            s.reset(seed)
            r = s.run()
            want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=rule)
            assert rule == "tree" or want.stats[1][1] > 1 << 18
            assert r == want.rounds
            assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats]
            ig = [lc.cc_get_round_stats(s.ctx, k, True)[-1] for k in range(r)]
            first = ig.index(2)   # before it: round 0, and rounds too large for the hashed drop
            assert ig == [0] * first + [2] * (r - first), ig
            if rule == "local":
                assert first == 1   # round 1, of more than 2^18 nodes, inside the launch
            # one launch, or more where the per-round maps fill their arena (the launch stops,
            # the host folds the maps and launches again: one-hop, seed 22)
            assert s.kernel_times()["fused_rounds"][1] >= 1
            lab = s.labels()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(lab.cpu().numpy().view(np.uint32), want.labels)


# --- the largest vertex ids ---------------------------------------------------------------

@pytest.mark.parametrize("variant", ["local", "tree", "one_hop"])
@pytest.mark.parametrize("layout", ["soa32", "packed"])
def test_largest_vertex_ids(lc, layout, variant):
    """n_vertices = 2^31 - 1, the most the boundary takes (include/cc.h), with edges among
    eight ids at both ends of the range.  Their per-round parents and statistics, the round
    count and their labels come from the brute force over their names (priorities depend on
    names only, Section 3); every other id has no edge and keeps its own id (checked on the
    device, in chunks)."""
    n = (1 << 31) - 1
    names = np.array([0, 1, n - 8, n - 5, n - 4, n - 3, n - 2, n - 1], np.uint32)
    local = [(0, 7), (7, 6), (6, 4), (1, 2), (2, 3), (3, 1)]
    adj = np.zeros((1, names.size), np.uint8)
    for i, j in local:
        adj[0, i] |= np.uint8(1 << j)
        adj[0, j] |= np.uint8(1 << i)
    seed = 0x5EED
    lab_b, rounds_b, par_b, stats_b = brute_all(adj, lambda r: spec_priority(seed, r, names), max_rounds=8,
                                                variant=variant)
    g = graphgen.Graph(n, names[[i for i, _ in local]], names[[j for _, j in local]])
    s_t, d_t, lay = to_device(g, layout)
    nm = torch.from_numpy(names.astype(np.int64)).to(DEV)
    flags = {"local": 0, "tree": lc.CC_TREE, "one_hop": lc.CC_ONE_HOP}[variant]
    with lc.Solver(n, s_t, d_t, seed=seed, layout=lay, flags=flags) as s:
        r = 0
        while True:
            st, stats = s.contract_round()
            if st == lc.CC_DONE:
                break
            par, k = s.parents()
            got = par[nm].cpu().numpy().astype(np.int64)
            del par
            pb = par_b[r, 0].astype(np.int64)
            want = np.where(pb == 255, -1, names[np.minimum(pb, names.size - 1)].astype(np.int64))
            np.testing.assert_array_equal(got, want, err_msg="round %d" % r)
            assert tuple(stats[1:]) == tuple(int(x) for x in stats_b[r, 0])
            assert k == stats[1]
            r += 1
        assert r == rounds_b[0]
        assert s.run() == r
        lab = s.labels()
        np.testing.assert_array_equal(lab[nm].cpu().numpy().astype(np.int64), names[lab_b[0]].astype(np.int64))
        moved = []
        chunk = 1 << 28
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            ids = torch.arange(a, b, device=DEV, dtype=lab.dtype)
            moved += (torch.nonzero(lab[a:b] != ids).flatten() + a).cpu().tolist()
            del ids
        assert set(moved) <= set(int(x) for x in names)
        del lab
    del s_t, d_t
    torch.cuda.empty_cache()
