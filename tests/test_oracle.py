"""Pins of the CPU oracle against what the paper and mathematics fix (no GPU needed).

Each test checks the oracle against something other than itself: published hash values,
the definition by brute force, hand-worked fixtures, textbook/library component routines,
or an invariant or bound stated in the paper.
"""
import glob
import math
import os
from itertools import permutations

import numpy as np
import pytest

import graphgen
import oracle
from lcref import (all_graph_adjacency, brute_all, canon, contract_edges, graph_records, merge_to_large_reference,
                   scipy_components, simple_edges,
                   spec_priority, spec_priority_inverse, two_hop_parents, union_find)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------------------------------
# priority specification
# ---------------------------------------------------------------------------------------

def test_hash_published_values():
    # SplitMix64 (Steele, Lea, Flood 2014): the first outputs of the generator seeded with 0.
    assert oracle.sm64(0) == 0xE220A8397B1DCDAF
    # MurmurHash3_x86_32 of the empty input reduces to fmix32(seed): seed 1 -> 0x514E28B7,
    # seed 0xFFFFFFFF -> 0x81F16F39 (published verification values).
    assert oracle.fmix32(1) == 0x514E28B7
    assert oracle.fmix32(0xFFFFFFFF) == 0x81F16F39
    assert oracle.fmix32(0) == 0


def test_priority_matches_independent_spec():
    rng = np.random.default_rng(1)
    names = rng.integers(0, 1 << 32, size=200, dtype=np.uint64).astype(np.uint32)
    for seed in (0, 1, 0xC0FFEE00, (1 << 64) - 1):
        for r in (0, 1, 7, 31):
            want = spec_priority(seed, r, names)
            got = np.array([oracle.priority(seed, r, int(x)) for x in names], np.uint32)
            np.testing.assert_array_equal(got, want)


def test_priority_is_a_bijection():
    # Structure: xor with a constant, xor-shift-right and multiplication by an odd constant
    # are each invertible on 32-bit words, so their composition is a bijection.  Checked
    # here by an explicit inverse on 2^24 inputs and exact distinctness on a 2^24 block.
    for seed, r in ((0, 0), (12345, 3)):
        x = np.arange(1 << 24, dtype=np.uint32) * np.uint32(251) + np.uint32(seed & 0xFFFF)
        p = spec_priority(seed, r, x)
        np.testing.assert_array_equal(spec_priority_inverse(seed, r, p), x)
        assert np.unique(p).shape[0] == x.shape[0]


# ---------------------------------------------------------------------------------------
# brute force from the definition on every labelled graph with up to 7 vertices
# ---------------------------------------------------------------------------------------

def _oracle_all(adj, seed):
    src, dst, eoff = graph_records(adj)
    G, n = adj.shape
    voff = np.arange(G + 1, dtype=np.int64) * n
    seeds = np.full(G, seed, np.uint64)
    cap = 8
    labels, rounds, par = oracle.run_batch(voff, eoff, src, dst, seeds, record_parents=True, parents_cap=cap)
    return labels.reshape(G, n), rounds, par.reshape(G, cap, n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_oracle_equals_bruteforce_all_graphs(n):
    adj = all_graph_adjacency(n)
    for seed in (0, 0xC0FFEE00, 977):
        lab_o, rounds_o, par_o = _oracle_all(adj, seed)
        lab_b, rounds_b, par_b, _ = brute_all(adj, lambda r: spec_priority(seed, r, np.arange(n)), max_rounds=8)
        np.testing.assert_array_equal(rounds_o, rounds_b)
        np.testing.assert_array_equal(lab_o, lab_b.astype(np.uint32))
        for r in range(int(rounds_b.max(initial=0))):
            want = np.where(par_b[r] == 255, np.uint32(oracle.NOT_A_NODE), par_b[r].astype(np.uint32))
            live = rounds_b > r
            np.testing.assert_array_equal(par_o[live, r, :], want[live])


def test_oracle_stats_equal_bruteforce():
    n = 6
    adj = all_graph_adjacency(n)
    rng = np.random.default_rng(5)
    pick = rng.choice(adj.shape[0], size=400, replace=False)
    seed = 31337
    _, rounds_b, _, stats_b = brute_all(adj[pick], lambda r: spec_priority(seed, r, np.arange(n)), max_rounds=8)
    src, dst, eoff = graph_records(adj[pick])
    for j in range(pick.shape[0]):
        a, b = eoff[j], eoff[j + 1]
        res = oracle.run(n, src[a:b], dst[a:b], seed)
        assert res.rounds == rounds_b[j]
        for r, st in enumerate(res.stats):
            assert st[0] == r
            assert list(st[1:]) == list(stats_b[r, j])


@pytest.mark.parametrize("n", [3, 4, 5])
def test_oracle_all_orderings(n):
    """Every graph on n vertices under every ordering of its vertices (explicit priorities)."""
    adj = all_graph_adjacency(n)
    src, dst, eoff = graph_records(adj)
    G = adj.shape[0]
    for perm in permutations(range(n)):
        prio = np.array(perm, np.int64)
        lab_b, rounds_b, par_b, stats_b = brute_all(adj, lambda r: prio, max_rounds=8)
        for g in range(G):
            a, b = eoff[g], eoff[g + 1]
            res = oracle.run(n, src[a:b], dst[a:b], explicit_prio=prio.astype(np.uint32), record_parents=True)
            assert res.rounds == rounds_b[g]
            np.testing.assert_array_equal(res.labels, lab_b[g].astype(np.uint32))
            for r in range(res.rounds):
                want = np.where(par_b[r, g] == 255, np.uint32(oracle.NOT_A_NODE), par_b[r, g].astype(np.uint32))
                np.testing.assert_array_equal(res.parents[r], want)


# ---------------------------------------------------------------------------------------
# hand-worked fixtures
# ---------------------------------------------------------------------------------------

def load_fixture(path):
    fx = {"parents": {}, "stats": {}}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key == "n":
                fx["n"] = int(vals[0])
            elif key == "edges":
                fx["edges"] = [tuple(int(t) for t in v.split("-")) for v in vals]
            elif key == "prio":
                fx["prio"] = [int(v) for v in vals]
            elif key.startswith("parents"):
                fx["parents"][int(key[7:])] = [None if v == "-" else int(v) for v in vals]
            elif key == "labels":
                fx["labels"] = [int(v) for v in vals]
            elif key == "rounds":
                fx["rounds"] = int(vals[0])
            elif key.startswith("stats"):
                fx["stats"][int(key[5:])] = [int(v) for v in vals]
    return fx


FIXTURES = sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))


@pytest.mark.parametrize("path", FIXTURES, ids=[os.path.basename(p) for p in FIXTURES])
def test_oracle_hand_worked(path):
    fx = load_fixture(path)
    src = [a for a, _ in fx["edges"]]
    dst = [b for _, b in fx["edges"]]
    res = oracle.run(fx["n"], src, dst, explicit_prio=np.array(fx["prio"], np.uint32), record_parents=True)
    assert res.rounds == fx["rounds"]
    assert res.labels.tolist() == fx["labels"]
    for r, want in fx["parents"].items():
        got = [None if v == oracle.NOT_A_NODE else int(v) for v in res.parents[r]]
        assert got == want, (r, got, want)
    for r, want in fx["stats"].items():
        assert list(res.stats[r][1:]) == want


# ---------------------------------------------------------------------------------------
# closed forms and special cases
# ---------------------------------------------------------------------------------------

def test_edgeless_graph():
    res = oracle.run(10, [3, 7], [3, 7], seed=4)   # loops only
    assert res.rounds == 0
    assert res.labels.tolist() == list(range(10))
    res = oracle.run(0, [], [], seed=4)
    assert res.rounds == 0


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 13, 64, 101])
def test_path_identity_order_closed_form(k):
    """Under rho(name) = name a path 0-1-...-(k-1) loses two nodes per phase: the two-hop
    minimum of vertex i is max(0, i-2), so the classes are {0,1,2},{3},{4},... and the next
    graph is again an increasing path; hence ceil((k-1)/2) phases."""
    src = list(range(k - 1))
    dst = list(range(1, k))
    res = oracle.run(k, src, dst, explicit_prio=np.arange(k, dtype=np.uint32), record_parents=True)
    assert res.rounds == math.ceil((k - 1) / 2)
    if k >= 2:
        assert res.parents[0].tolist() == [max(0, i - 2) for i in range(k)]
    assert res.labels.tolist() == [0] * k


@pytest.mark.parametrize("shape", ["star", "clique"])
def test_diameter_two_one_phase(shape):
    n = 40
    if shape == "star":
        src, dst = [7] * (n - 1), [v for v in range(n) if v != 7]
    else:
        src, dst = zip(*[(a, b) for a in range(n) for b in range(a + 1, n)])
    for seed in range(5):
        res = oracle.run(n, src, dst, seed=seed)
        assert res.rounds == 1
        assert len(set(res.labels.tolist())) == 1


def test_path_lower_bound():
    """A phase merges only vertices at distance <= 4, so a path shrinks at most 5 times per
    phase and needs at least ceil(log_5 L) phases (Section 7, first theorem)."""
    for L in (26, 126, 1000, 3125):
        src, dst = np.arange(L - 1), np.arange(1, L)
        for seed in range(4):
            res = oracle.run(L, src, dst, seed=seed)
            assert res.rounds >= math.ceil(math.log(L, 5) - 1e-9)
            assert res.stats[0][1] == L
            for before, after in zip(res.stats, res.stats[1:]):
                assert after[1] * 5 >= before[1]       # a path never shrinks by more than 5x


def test_disjoint_union_is_union_of_results():
    """Components never interact (priorities are only compared within a component), so a
    graph made of two copies run with the same priority per name gives each copy's result."""
    g = graphgen.workload_small(seed=99)
    n = 2000
    keep = (g.src < n) & (g.dst < n)
    s, d = g.src[keep], g.dst[keep]
    prio = spec_priority(5, 0, np.arange(2 * n))
    both = oracle.run(2 * n, np.concatenate([s, s + n]), np.concatenate([d, d + n]), explicit_prio=prio)
    a = oracle.run(n, s, d, explicit_prio=prio[:n])
    b = oracle.run(n, s + 0, d + 0, explicit_prio=prio[n:])
    np.testing.assert_array_equal(both.labels[:n], a.labels)
    np.testing.assert_array_equal(both.labels[n:], b.labels + n)


# ---------------------------------------------------------------------------------------
# partition against textbook and library routines, and per-phase invariants
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["gnm", "rmat", "paths", "sparse"])
def test_partition_matches_union_find_and_scipy(kind):
    if kind == "gnm":
        g = graphgen.workload_small()
    elif kind == "rmat":
        g = graphgen.Graph(1 << 14, *graphgen.rmat(7, 14, 8 << 14))
    elif kind == "paths":
        g = graphgen.er_with_paths(11, 1 << 12, 1 << 12, 50, 200)
    else:
        g = graphgen.Graph(1 << 15, *graphgen.gnm(3, 1 << 15, 1 << 14))   # below the threshold
    res = oracle.run(g.n, g.src, g.dst, seed=42)
    want = canon(union_find(g.n, g.src, g.dst))
    np.testing.assert_array_equal(canon(res.labels), want)
    np.testing.assert_array_equal(canon(scipy_components(g.n, g.src, g.dst)), want)
    # labels are vertices of the vertex's own component
    np.testing.assert_array_equal(want[res.labels.astype(np.int64)], want)


@pytest.mark.parametrize("kind", ["gnm", "rmat", "paths", "sparse", "isolated_ends", "loops_repeats",
                                  "no_edges", "one_vertex", "chain_merge"])
def test_components_min_id_equals_library_components(kind):
    """The oracle's union-find (`components_min_id`) against scipy's connected_components
    (a library routine) and the textbook union-find of lcref: every vertex gets the
    smallest id of its component.  Covers ids 0 and n-1 in singleton components, records
    with loops and repeats, an edgeless graph, n = 1, and a merge order in which the root
    union by size keeps is not the component's smallest id."""
    if kind == "gnm":
        g = graphgen.workload_small()
    elif kind == "rmat":
        g = graphgen.Graph(1 << 14, *graphgen.rmat(7, 14, 8 << 14))
    elif kind == "paths":
        g = graphgen.er_with_paths(11, 1 << 12, 1 << 12, 50, 200)
    elif kind == "sparse":
        g = graphgen.Graph(1 << 15, *graphgen.gnm(3, 1 << 15, 1 << 14))
    elif kind == "isolated_ends":
        # ids 0 and n-1 appear in no record; the rest form a few components
        n = 1000
        s, d = graphgen.gnm(5, n - 2, 600)
        g = graphgen.Graph(n, s + np.uint32(1), d + np.uint32(1))
    elif kind == "loops_repeats":
        s, d = graphgen.gnm(9, 300, 500)
        s = np.concatenate([s, s, np.arange(300, dtype=np.uint32)])
        d = np.concatenate([d, d, np.arange(300, dtype=np.uint32)])
        g = graphgen.Graph(300, s, d)
    elif kind == "no_edges":
        g = graphgen.Graph(17, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    elif kind == "one_vertex":
        g = graphgen.Graph(1, np.zeros(1, np.uint32), np.zeros(1, np.uint32))
    else:
        # a large tree on high ids is built first, then a small one containing id 2 joins it:
        # union by size keeps the large tree's root, which is not the component's minimum
        hi = np.arange(50, 99, dtype=np.uint32)
        s = np.concatenate([hi, np.array([2, 3], np.uint32)])
        d = np.concatenate([hi + np.uint32(1), np.array([3, 60], np.uint32)])
        g = graphgen.Graph(120, s, d)
    got = oracle.components_min_id(g.n, g.src, g.dst).astype(np.int64)
    want = canon(scipy_components(g.n, g.src, g.dst)) if g.n else np.zeros(0, np.int64)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(got, canon(union_find(g.n, g.src, g.dst)))
    # every value is the smallest member of its class, and classes are closed under records
    assert np.all(got <= np.arange(g.n))
    assert np.all(got[got] == got)
    np.testing.assert_array_equal(got[g.src.astype(np.int64)], got[g.dst.astype(np.int64)])


@pytest.mark.parametrize("variant", ["local", "one_hop"])
def test_recorded_minima_follow_the_definition(variant):
    """The oracle's per-round minima (record_minima): m1[x] = min of rho over the closed
    N(x), l[x] = min of rho over N(N(x)) (Section 3; N(x) contains x, Section 2), recomputed
    here with numpy on each round's graph (the input's simple edges, then each previous
    graph contracted through the oracle's own parents), and l[x] = rho(parent(x))."""
    g = graphgen.er_with_paths(21, 3000, 6000, 20, 40)
    seed = 77
    res = oracle.run(g.n, g.src, g.dst, seed=seed, variant=variant, record_parents=True, record_minima=True)
    assert res.rounds >= 3
    lo, hi = simple_edges(g.src, g.dst)
    a, b = lo.astype(np.int64), hi.astype(np.int64)
    for r in range(res.rounds):
        rho = spec_priority(seed, r, np.arange(g.n)).astype(np.int64)
        nodes = np.unique(np.concatenate([a, b]))
        m1 = np.full(g.n, 0xFFFFFFFF, np.int64)
        m1[nodes] = rho[nodes]
        np.minimum.at(m1, a, rho[b])
        np.minimum.at(m1, b, rho[a])
        l2 = m1.copy()
        if variant == "local":
            np.minimum.at(l2, a, m1[b])
            np.minimum.at(l2, b, m1[a])
        np.testing.assert_array_equal(res.m1[r].astype(np.int64), m1, err_msg="round %d" % r)
        np.testing.assert_array_equal(res.l[r].astype(np.int64), l2, err_msg="round %d" % r)
        par = res.parents[r].astype(np.int64)
        np.testing.assert_array_equal(rho[par[nodes]], l2[nodes])
        k = contract_edges(a, b, np.where(par >= 0xFFFFFFFF, np.arange(g.n), par))
        a, b = (k >> np.uint64(32)).astype(np.int64), (k & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert a.size == 0


def test_components_min_id_rejects_out_of_range_ids():
    with pytest.raises(ValueError):
        oracle.components_min_id(4, np.array([0, 4], np.uint32), np.array([1, 2], np.uint32))


def test_per_phase_definition_and_invariants():
    """Replays the phases independently: each recorded parent must be the argmin of the
    priority over the closed two-hop ball (sparse (A+I)^2), rho(p(x)) <= rho(x) (proof of the
    O(log n) lemma, Section 4), and components are preserved."""
    g = graphgen.er_with_paths(21, 1 << 12, 3 << 11, 20, 100)
    seed = 77
    res = oracle.run(g.n, g.src, g.dst, seed=seed, record_parents=True)
    lo, hi = simple_edges(g.src, g.dst)
    n_comp0 = np.unique(canon(scipy_components(g.n, g.src, g.dst))[np.unique(np.concatenate([lo, hi]))]).shape[0]
    finalised = 0
    for r in range(res.rounds):
        prio = spec_priority(seed, r, np.arange(g.n))
        nodes, want = two_hop_parents(g.n, lo, hi, prio)
        par = res.parents[r]
        np.testing.assert_array_equal(par[nodes].astype(np.int64), want[nodes])
        assert np.all(prio[par[nodes]] <= prio[nodes])
        assert np.count_nonzero(par != oracle.NOT_A_NODE) == nodes.shape[0] == res.stats[r][1]
        # next graph
        plo, phi = par[lo].astype(np.int64), par[hi].astype(np.int64)
        lo, hi = simple_edges(plo, phi)
        assert res.stats[r][4] == lo.shape[0]
        finalised += res.stats[r][5]
        if lo.shape[0]:
            nxt = np.unique(np.concatenate([lo, hi]))
            comp = canon(scipy_components(g.n, lo, hi))[nxt]
            n_now = np.unique(comp).shape[0]
        else:
            n_now = 0
        assert n_now + finalised == n_comp0
    assert lo.shape[0] == 0


def test_expected_labels_at_most_three_quarters():
    """E[#labels] <= 3n/4 for graphs without isolated vertices (Section 4, O(log n) lemma)."""
    n = 600
    src, dst = np.arange(0, n, 2), np.arange(1, n, 2)       # a perfect matching
    ps, pd = np.arange(n - 1), np.arange(1, n)              # a path
    for s, d in ((src, dst), (ps, pd)):
        counts = []
        for seed in range(100):
            res = oracle.run(n, s, d, seed=seed, max_rounds=1, record_parents=True)
            counts.append(np.unique(res.parents[0]).shape[0])
        assert np.mean(counts) <= 0.75 * n


def test_max_rounds_stops_early():
    g = graphgen.er_with_paths(3, 0, 0, 4, 300)
    full = oracle.run(g.n, g.src, g.dst, seed=9)
    part = oracle.run(g.n, g.src, g.dst, seed=9, max_rounds=2)
    assert full.rounds > 2 and part.rounds == 2
    assert full.stats[:2] == part.stats


def test_rejects_out_of_range_ids():
    with pytest.raises(ValueError):
        oracle.run(3, [0, 5], [1, 2])


# ---------------------------------------------------------------------------------------
# TreeContraction, the one-hop label, the union-find finish
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["tree", "one_hop"])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_variant_equals_bruteforce(variant, n):
    """Labels, parents, rounds and statistics of every graph on up to 5 vertices (a sample
    of 600 on 6) under two seeds equal the brute force from the definition: for
    TreeContraction the walk to the terminal 2-cycle of v -> f(v), an independent route to
    the weakly connected components that the oracle forms by union-find."""
    adj = all_graph_adjacency(n)
    pick = np.arange(adj.shape[0])
    if n == 6:
        pick = np.random.default_rng(n).choice(adj.shape[0], size=600, replace=False)
    adj = adj[pick]
    src, dst, eoff = graph_records(adj)
    for seed in (1, 0xBEEF):
        lab_b, rounds_b, par_b, stats_b = brute_all(adj, lambda r: spec_priority(seed, r, np.arange(n)),
                                                    max_rounds=12, variant=variant)
        for g in range(adj.shape[0]):
            a, b = eoff[g], eoff[g + 1]
            res = oracle.run(n, src[a:b], dst[a:b], seed=seed, variant=variant, record_parents=True)
            assert res.rounds == rounds_b[g]
            np.testing.assert_array_equal(res.labels, lab_b[g].astype(np.uint32))
            for r in range(res.rounds):
                want = np.where(par_b[r, g] == 255, np.uint32(oracle.NOT_A_NODE), par_b[r, g].astype(np.uint32))
                np.testing.assert_array_equal(res.parents[r], want)
                assert list(res.stats[r][1:]) == list(stats_b[r, g])


@pytest.mark.parametrize("variant", ["tree", "one_hop"])
@pytest.mark.parametrize("kind", ["gnm", "rmat", "paths"])
def test_variant_partition(variant, kind):
    if kind == "gnm":
        g = graphgen.workload_small()
    elif kind == "rmat":
        g = graphgen.Graph(1 << 13, *graphgen.rmat(7, 13, 8 << 13))
    else:
        g = graphgen.er_with_paths(11, 1 << 11, 1 << 11, 30, 150)
    res = oracle.run(g.n, g.src, g.dst, seed=42, variant=variant)
    want = canon(scipy_components(g.n, g.src, g.dst))
    np.testing.assert_array_equal(canon(res.labels), want)
    np.testing.assert_array_equal(want[res.labels.astype(np.int64)], want)


def test_tree_classes_are_connected_and_never_single():
    """TreeContraction merges along edges v -> f(v): every class of a phase has at least two
    nodes (each node points to a neighbour), induces a connected subgraph, and contains its
    label; so a phase at least halves the nodes and the contracted graph is a minor."""
    g = graphgen.er_with_paths(5, 1 << 11, 3 << 10, 20, 60)
    res = oracle.run(g.n, g.src, g.dst, seed=8, variant="tree", record_parents=True)
    lo, hi = simple_edges(g.src, g.dst)
    assert res.rounds >= 2
    for r in range(res.rounds):
        par = res.parents[r].astype(np.int64)
        nodes = np.nonzero(res.parents[r] != oracle.NOT_A_NODE)[0]
        cls, size = np.unique(par[nodes], return_counts=True)
        assert size.min() >= 2
        assert np.all(par[cls] == cls)                       # the label is in its own class
        assert cls.shape[0] * 2 <= nodes.shape[0]
        # connected inside each class: edges between members of one class join them all
        same = par[lo] == par[hi]
        comp = scipy_components(g.n, lo[same], hi[same])
        for c in cls[:200]:
            members = nodes[par[nodes] == c]
            assert np.unique(comp[members]).shape[0] == 1
        lo, hi = simple_edges(par[lo], par[hi])


@pytest.mark.parametrize("finish", [1, 50, 2000, 10 ** 9])
def test_finish_is_smallest_remaining_name(finish):
    """Union-find finish (Section 6): the phases before the switch are those of the plain run;
    after it every vertex is labelled with the smallest name its component still has, i.e.
    the minimum, over the component's vertices, of their labels after those phases."""
    g = graphgen.er_with_paths(13, 1 << 11, 1 << 12, 10, 120)
    plain = oracle.run(g.n, g.src, g.dst, seed=4)
    res = oracle.run(g.n, g.src, g.dst, seed=4, finish_edges=finish)
    k = res.rounds
    assert res.stats == plain.stats[:k]
    assert res.finished == (k < plain.rounds)
    if res.finished:
        assert plain.stats[k - 1][4] <= finish < min([plain.stats[j][4] for j in range(k - 1)], default=2 ** 62)
    part = oracle.run(g.n, g.src, g.dst, seed=4, max_rounds=k)
    comp = canon(scipy_components(g.n, g.src, g.dst))
    want = np.full(g.n, np.iinfo(np.int64).max, np.int64)
    np.minimum.at(want, comp, part.labels.astype(np.int64))
    np.testing.assert_array_equal(res.labels.astype(np.int64), want[comp])


@pytest.mark.parametrize("variant", ["local", "tree", "one_hop"])
def test_edge_counts_follow_the_contraction(variant):
    """Each round's distinct edges out (m_out) and the next round's records (m_in) equal the
    size of the previous edge set contracted through the oracle's own parents: the distinct
    loop-free parent pairs (proof of the contraction-step lemma, Section 3)."""
    from lcref import contract_edges, split_keys
    for g, seed in ((graphgen.Graph(3000, *graphgen.gnm(31, 3000, 9001)), 4),
                    (graphgen.er_with_paths(32, 1 << 10, 1 << 11, 20, 50), 5),
                    (graphgen.Graph(1 << 12, *graphgen.rmat(33, 12, 8 << 12)), 6)):
        want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=variant, record_parents=True)
        a, b = g.src, g.dst
        for r in range(want.rounds):
            e = contract_edges(a, b, want.parents[r])
            assert e.size == want.stats[r][4]
            if r + 1 < want.rounds:
                assert want.stats[r + 1][2] == e.size
            a, b = split_keys(e)
        assert a.size == 0


# ---------------------------------------------------------------------------------------
# MergeToLarge (Section 5)
# ---------------------------------------------------------------------------------------

def _mtl_check(n, src, dst, seed, alphas, table=None):
    if table is None:
        prio_of = lambda r, v: oracle.priority(seed, r, v)   # noqa: E731 (pinned separately above)
    else:
        prio_of = lambda r, v: int(table[v])                   # noqa: E731
    lab, rounds, pars, stats = merge_to_large_reference(n, src, dst, prio_of, alphas)
    res = oracle.run(n, src, dst, seed=seed, variant="merge_to_large", alphas=alphas, record_parents=True,
                     explicit_prio=table)
    assert res.rounds == rounds
    assert [tuple(x) for x in res.stats] == stats
    for r in range(rounds):
        want = np.full(n, oracle.NOT_A_NODE, np.uint32)
        for v, p in pars[r].items():
            want[v] = p
        np.testing.assert_array_equal(res.parents[r], want, err_msg="round %d" % r)
    np.testing.assert_array_equal(res.labels.astype(np.int64), lab)
    return res


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_merge_to_large_equals_restatement_all_graphs(n):
    """Every labelled graph on n vertices, two seeds, alpha in {1, 2, 3}: the oracle's
    MergeToLarge run equals the step-by-step restatement round by round."""
    adj = all_graph_adjacency(n)
    src, dst, eoff = graph_records(adj)
    for g in range(adj.shape[0]):
        a, b = eoff[g], eoff[g + 1]
        for seed in (1, 2):
            for alpha in (1, 2, 3):
                _mtl_check(n, src[a:b], dst[a:b], seed, [alpha])


@pytest.mark.parametrize("kind", ["gnm", "paths", "dense"])
def test_merge_to_large_equals_restatement_random(kind):
    if kind == "gnm":
        g = graphgen.Graph(300, *graphgen.gnm(4, 300, 500))
    elif kind == "paths":
        g = graphgen.er_with_paths(6, 100, 150, 4, 40)
    else:
        g = graphgen.Graph(120, *graphgen.gnm(8, 120, 1500))
    for alphas in ([2], [3, 6, 12], [1]):
        res = _mtl_check(g.n, g.src, g.dst, 31, alphas)
        np.testing.assert_array_equal(canon(res.labels), canon(scipy_components(g.n, g.src, g.dst)))
    tab = np.random.default_rng(5).permutation(g.n).astype(np.uint32)
    _mtl_check(g.n, g.src, g.dst, 0, [2], table=tab)


def test_merge_to_large_without_large_nodes_is_local_contraction():
    """With alpha larger than any class no node is large: every MergeToLarge step keeps each
    node (no survivor lost, same edges), and under one explicit ordering the LocalContraction
    steps are exactly the plain run's phases."""
    g = graphgen.er_with_paths(12, 2000, 3000, 10, 200)
    tab = np.random.default_rng(2).permutation(g.n).astype(np.uint32)
    plain = oracle.run(g.n, g.src, g.dst, explicit_prio=tab, record_parents=True)
    res = oracle.run(g.n, g.src, g.dst, explicit_prio=tab, variant="merge_to_large", alphas=[g.n + 1],
                     record_parents=True)
    assert res.rounds == 2 * plain.rounds - 1
    np.testing.assert_array_equal(res.labels, plain.labels)
    for i in range(plain.rounds):
        np.testing.assert_array_equal(res.parents[2 * i], plain.parents[i])
        assert res.stats[2 * i][1:] == plain.stats[i][1:]
        if 2 * i + 1 < res.rounds:
            st = res.stats[2 * i + 1]
            assert st[2] == st[3] == st[4] and st[5] == 0
            nodes = res.parents[2 * i + 1] != oracle.NOT_A_NODE
            np.testing.assert_array_equal(res.parents[2 * i + 1][nodes], np.nonzero(nodes)[0])


def test_merge_to_large_shrinks_dense_random_graphs():
    """Section 5, lemma on G(n, alpha_n / n) with alpha_n >= 4 ln n: one phase of
    LocalContraction with the MergeToLarge step (parameter alpha_n / 4) leaves at most
    n / alpha_n nodes (with high probability; checked over several seeds)."""
    n = 1 << 14
    alpha_n = int(math.ceil(4 * math.log(n)))
    m = n * alpha_n // 2
    for seed in range(4):
        g = graphgen.Graph(n, *graphgen.gnm(100 + seed, n, m))
        res = oracle.run(n, g.src, g.dst, seed=seed, variant="merge_to_large", alphas=[alpha_n // 4], max_rounds=2)
        st = res.stats[1]
        nodes_after = len(np.unique(res.labels))
        assert nodes_after <= n / alpha_n, (seed, nodes_after, st)
