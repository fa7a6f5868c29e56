"""Parity of the other label rules and of the union-find finish (HIP path through the C ABI)
with the CPU oracle.

TreeContraction (CC_TREE) and the one-hop label (CC_ONE_HOP): per-round parents by name,
per-round statistics, round counts and labels bit for bit.  The union-find finish
(cc_set_finish): the rounds before the switch and the labels after it (every remaining
component named by its smallest name) bit for bit.
"""
import numpy as np
import pytest

import graphgen
import oracle
from lcref import contract_edges, split_keys

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def lc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10727_amd as lc
    return lc


def dev(g):
    return (torch.from_numpy(g.src.view(np.int32)).to(DEV), torch.from_numpy(g.dst.view(np.int32)).to(DEV))


def dup_path(nv, reps, seed):
    a = np.repeat(np.arange(nv - 1, dtype=np.uint32), reps)
    perm = np.random.default_rng(seed).permutation(a.size)
    return graphgen.Graph(nv, a[perm].copy(), (a[perm] + 1).astype(np.uint32))


GRAPHS = {
    "gnm_small": lambda: graphgen.Graph(1000, *graphgen.gnm(11, 1000, 4097)),
    "gnm_mid": lambda: graphgen.Graph(20000, *graphgen.gnm(12, 20000, 61441)),
    "sparse": lambda: graphgen.Graph(30000, *graphgen.gnm(13, 30000, 12000)),
    "rmat": lambda: graphgen.Graph(1 << 14, *graphgen.rmat(14, 14, 8 << 14)),
    "paths": lambda: graphgen.er_with_paths(15, 1 << 11, 1 << 12, 30, 300),
    "dup_path": lambda: dup_path(300, 500, 16),
    "workload_small": graphgen.workload_small,
}

VARIANT_FLAGS = {"tree": 1 << 5, "one_hop": 1 << 6}


MODES = {"direct": 1 << 2, "tiled": 1 << 3}


def per_round(lc, g, seed, flags):
    s_t, d_t = dev(g)
    out = {"parents": [], "stats": []}
    with lc.Solver(g.n, s_t, d_t, seed=seed, flags=flags) as s:
        while True:
            st, stats = s.contract_round()
            if st == lc.CC_DONE:
                break
            out["stats"].append(tuple(stats))
            par, k = s.parents()
            out["parents"].append(par.cpu().numpy().view(np.uint32).copy())
            assert k == stats[1]
            out.setdefault("edges", []).append(np.sort(s.edges().cpu().numpy().view(np.uint64)))
        out["rounds"] = s.run()
        out["labels"] = s.labels().cpu().numpy()
    return out


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("variant", sorted(VARIANT_FLAGS))
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_variant_parity(lc, variant, name, mode):
    g = GRAPHS[name]()
    seed = 0xA11CE + len(name)
    want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=variant, record_parents=True)
    got = per_round(lc, g, seed, VARIANT_FLAGS[variant] | MODES[mode])
    assert got["rounds"] == want.rounds
    assert got["stats"] == [tuple(x) for x in want.stats]
    for r in range(want.rounds):
        np.testing.assert_array_equal(got["parents"][r], want.parents[r], err_msg="round %d" % r)
    np.testing.assert_array_equal(got["labels"].astype(np.uint32), want.labels)
    a, b = g.src, g.dst          # each round's graph: the contraction through the oracle's parents
    for r in range(want.rounds):
        want_e = contract_edges(a, b, want.parents[r])
        np.testing.assert_array_equal(got["edges"][r], want_e, err_msg="edges after round %d" % r)
        a, b = split_keys(want_e)


@pytest.mark.parametrize("variant", sorted(VARIANT_FLAGS))
def test_variant_cc_run_and_reuse(lc, variant):
    """cc_run (captured tails on a reused context) equals the oracle for several seeds."""
    g = graphgen.er_with_paths(17, 1 << 11, 1 << 12, 30, 700)
    s_t, d_t = dev(g)
    with lc.Solver(g.n, s_t, d_t, seed=1, flags=VARIANT_FLAGS[variant]) as s:
        for seed in (3, 4, 3):
            s.reset(seed)
            r = s.run()
            want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=variant)
            assert r == want.rounds
            assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats]
            np.testing.assert_array_equal(s.labels().cpu().numpy().astype(np.uint32), want.labels)


def test_tree_halves_the_nodes(lc):
    """Every TreeContraction class has at least two nodes: each round at least halves them."""
    g = graphgen.workload_small()
    _, rounds, st = lc.solve(g.n, *dev(g), seed=9, flags=VARIANT_FLAGS["tree"])
    for r in range(1, rounds):
        assert 2 * st[r][1] <= st[r - 1][1]


def test_variant_flags_exclusive(lc):
    g = GRAPHS["gnm_small"]()
    s_t, d_t = dev(g)
    with pytest.raises(lc.CCError) as e:
        lc.Solver(g.n, s_t, d_t, flags=VARIANT_FLAGS["tree"] | VARIANT_FLAGS["one_hop"])
    assert e.value.status == -1


@pytest.mark.parametrize("variant", sorted(VARIANT_FLAGS))
def test_variant_tiled_default_sizes(lc, variant):
    """G(2^20 + 3, 2^22 + 1): the default picks the tiled round 0 for the other rules too."""
    g = graphgen.Graph((1 << 20) + 3, *graphgen.gnm(61, (1 << 20) + 3, (1 << 22) + 1))
    s_t, d_t = dev(g)
    want = oracle.run(g.n, g.src, g.dst, seed=8, variant=variant)
    with lc.Solver(g.n, s_t, d_t, seed=8, flags=VARIANT_FLAGS[variant] | lc.CC_PROFILE) as s:
        r = s.run()
        assert s.kernel_times()["min1_tiled"][1] == 1
        assert r == want.rounds
        assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().cpu().numpy().astype(np.uint32), want.labels)


@pytest.mark.parametrize("variant", ["local", "tree"])
@pytest.mark.parametrize("name,finish", [("paths", 3000), ("paths", 1), ("workload_small", 50000),
                                         ("rmat", 10 ** 9), ("dup_path", 100)])
def test_finish_parity(lc, name, finish, variant):
    g = GRAPHS[name]()
    seed = 77
    flags = VARIANT_FLAGS.get(variant, 0)
    want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=variant, finish_edges=finish)
    s_t, d_t = dev(g)
    with lc.Solver(g.n, s_t, d_t, seed=seed, flags=flags | lc.CC_EAGER, finish_edges=finish) as s:
        r = s.run()
        assert r == want.rounds
        assert s.finished == want.finished
        assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().cpu().numpy().astype(np.uint32), want.labels)
        if want.finished:
            for query in (s.parents, s.edges):
                with pytest.raises(lc.CCError) as e:
                    query()
                assert e.value.status == -5
        # the same context without the finish: the plain labels again
        s.set_finish(0)
        s.reset(seed)
        r2 = s.run()
        plain = oracle.run(g.n, g.src, g.dst, seed=seed, variant=variant)
        assert r2 == plain.rounds and not s.finished
        np.testing.assert_array_equal(s.labels().cpu().numpy().astype(np.uint32), plain.labels)


@pytest.mark.parametrize("finish", [1, 300, 3000])
def test_finish_after_persistent_rounds(lc, finish):
    """The union-find finish after rounds run in the persistent launch (cc_tuning.tail): the
    launch stops once the graph has at most `finish` records, and the finish ends the solve
    with the oracle's rounds, statistics and labels."""
    g = graphgen.er_with_paths(0x7A11, 20000, 50000, 40, 400)
    want = oracle.run(g.n, g.src, g.dst, seed=10, finish_edges=finish)
    s_t, d_t = dev(g)
    with lc.Solver(g.n, s_t, d_t, seed=10, finish_edges=finish) as s:
        s.set_tuning(tail=3)
        r = s.run()
        assert r == want.rounds and s.finished == want.finished
        assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().cpu().numpy().astype(np.uint32), want.labels)


def test_finish_canonical_labels_unchanged(lc):
    """With CC_CANONICAL the finish changes nothing: the smallest id of every component."""
    g = graphgen.er_with_paths(19, 1 << 12, 1 << 13, 40, 500)
    s_t, d_t = dev(g)
    want = oracle.components_min_id(g.n, g.src, g.dst)
    for finish in (0, 1, 5000):
        with lc.Solver(g.n, s_t, d_t, seed=5, flags=lc.CC_CANONICAL, finish_edges=finish) as s:
            s.run()
            np.testing.assert_array_equal(s.labels().cpu().numpy().astype(np.uint32), want)


def test_hashed_rounds_launch_structure(lc):
    """G(2^13, 2^17) plus 30 paths of 300 vertices (six rounds): every round after the first
    holds at most half the input's records, so the host sends each to the hashed key set.  The radix kernels then run only in round 0
    (one launch per 8-bit digit of its 2 ceil(log2 n)-bit keys), each later round launches the
    five hashing kernels (clear, insert, count, the tile-count scan, write), and the result
    equals the oracle's."""
    g = graphgen.er_with_paths(15, 1 << 13, 1 << 17, 30, 300)
    s_t, d_t = dev(g)
    with lc.Solver(g.n, s_t, d_t, seed=5, flags=lc.CC_PROFILE | lc.CC_EAGER) as s:
        r = s.run()
        stats = s.stats(r)
        times = s.kernel_times()
        labels = s.labels().cpu().numpy().astype(np.uint32)
    assert r >= 3
    assert all(2 * st[2] + 1 <= g.m for st in stats[1:])
    kb = int(np.ceil(np.log2(g.n)))
    passes = (2 * kb + 7) // 8
    assert times["sort_scatter"][1] == passes and times["sort_hist"][1] == passes
    assert times["unique"][1] == 3                      # round 0's count, scan and write
    assert times["hash_dedup"][1] == 5 * (r - 1)
    want = oracle.run(g.n, g.src, g.dst, seed=5)
    assert r == want.rounds
    assert [tuple(x) for x in stats] == [tuple(x) for x in want.stats]
    np.testing.assert_array_equal(labels, want.labels)


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("alphas", [[2], [3, 6, 12], [1 << 30]])
@pytest.mark.parametrize("name", ["gnm_mid", "rmat", "paths", "workload_small"])
def test_merge_to_large_parity(lc, name, alphas, mode):
    """MergeToLarge (Section 5): every round -- the LocalContraction steps and the steps after
    them -- against the oracle: parents by name, statistics, edges left, labels."""
    g = GRAPHS[name]()
    seed = 0x3E7 + len(name)
    want = oracle.run(g.n, g.src, g.dst, seed=seed, variant="merge_to_large", alphas=alphas, record_parents=True)
    s_t, d_t = dev(g)
    with lc.Solver(g.n, s_t, d_t, seed=seed, flags=lc.CC_MERGE_TO_LARGE | MODES[mode]) as s:
        s.set_merge_to_large(alphas)
        a, b = g.src, g.dst
        r = 0
        while True:
            st, stats = s.contract_round()
            if st == lc.CC_DONE:
                break
            assert tuple(stats) == tuple(want.stats[r])
            par, _ = s.parents()
            np.testing.assert_array_equal(par.cpu().numpy().view(np.uint32), want.parents[r], err_msg="round %d" % r)
            got_e = np.sort(s.edges().cpu().numpy().view(np.uint64))
            want_e = contract_edges(a, b, want.parents[r])
            np.testing.assert_array_equal(got_e, want_e, err_msg="edges after round %d" % r)
            a, b = split_keys(want_e)
            r += 1
        assert s.run() == want.rounds == r
        np.testing.assert_array_equal(s.labels().cpu().numpy().view(np.uint32), want.labels)
        # cc_run alone, the rounds after round 0 in the persistent launch
        s.set_tuning(tail=2)
        s.set_merge_to_large(alphas)
        assert s.run() == want.rounds
        assert [tuple(x) for x in s.stats(want.rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().cpu().numpy().view(np.uint32), want.labels)
