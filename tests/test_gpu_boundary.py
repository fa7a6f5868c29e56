"""The test and inspection half of the boundary, through the C ABI, against the oracle:
explicit priorities (every ordering of every graph on at most 6 vertices), the parents of
every round (CC_RECORD_ROUNDS), the one-hop and two-hop minima of a round, and round
checkpoints (save, a failure forced from the host, load, resume)."""
from itertools import permutations

import numpy as np
import pytest

import graphgen
import oracle
from lcref import all_graph_adjacency, graph_records

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
DIRECT, TILED = 1 << 2, 1 << 3


@pytest.fixture(scope="module")
def lc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10727_amd as lc
    return lc


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


def all_orderings_union(max_n):
    """Every labelled graph on n <= max_n vertices, each under every ordering of its vertices,
    as one disjoint union: copy (n, ordering k, graph j) takes ids base .. base + n - 1, and
    the priority of id base + v is base + perm_k[v].  The table is then a permutation of all
    ids that orders every copy by its own ordering (only priorities inside a component are
    compared, Section 3)."""
    srcs, dsts, tabs = [], [], []
    off = 0
    for n in range(1, max_n + 1):
        adj = all_graph_adjacency(n)
        G = adj.shape[0]
        src, dst, eoff = graph_records(adj)
        gid = np.repeat(np.arange(G, dtype=np.uint32), np.diff(eoff).astype(np.int64))
        perms = np.array(list(permutations(range(n))), dtype=np.uint32)   # [P, n]
        P = perms.shape[0]
        blk = np.arange(P, dtype=np.uint32)[:, None] * np.uint32(G)       # copy index of (k, 0)
        base_rec = (blk + gid[None, :]) * np.uint32(n) + np.uint32(off)   # [P, records]
        srcs.append((base_rec + src[None, :]).ravel())
        dsts.append((base_rec + dst[None, :]).ravel())
        base_v = (np.arange(P * G, dtype=np.uint32) * np.uint32(n) + np.uint32(off)).reshape(P, G, 1)
        tabs.append((base_v + perms[:, None, :]).ravel())
        off += P * G * n
    return off, np.concatenate(srcs), np.concatenate(dsts), np.concatenate(tabs)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("max_n", [5, 6])
def test_every_ordering_of_every_small_graph(lc, max_n):
    """Per-round parents (by name), statistics, round count and labels under explicit
    priorities, for every ordering of every labelled graph with at most max_n vertices
    (max_n = 6: 23.6 M graphs, 142 M ids, 177 M records), bit for bit against the oracle
    given the same table."""
    n, src, dst, tab = all_orderings_union(max_n)
    assert np.array_equal(np.sort(tab), np.arange(n, dtype=np.uint32))
    print("union of n=%d ids, %d records" % (n, src.size), flush=True)
    s_t, d_t, t_t = dev32(src), dev32(dst), dev32(tab)
    with lc.Solver(n, s_t, d_t, seed=5, flags=lc.CC_EXPLICIT_PRIO | lc.CC_RECORD_ROUNDS) as s:
        s.set_priorities(0, t_t)
        rounds = s.run()
        stats = s.stats(rounds)
        parents = [s.parents(r)[0].cpu().numpy().view(np.uint32) for r in range(rounds)]
        labels = s.labels().cpu().numpy().view(np.uint32)
    del s_t, d_t, t_t
    torch.cuda.empty_cache()
    want = oracle.run(n, src, dst, explicit_prio=tab, record_parents=True, parents_cap=8)
    assert rounds == want.rounds
    assert [tuple(x) for x in stats] == [tuple(x) for x in want.stats]
    for r in range(rounds):
        np.testing.assert_array_equal(parents[r], want.parents[r], err_msg="round %d" % r)
    np.testing.assert_array_equal(labels, want.labels)


def test_explicit_identity_order_on_a_path(lc):
    """rho(name) = name on the path 0 - 1 - ... - (k-1): every phase merges the first three
    nodes and keeps the rest, so the solve takes ceil((k-1)/2) phases (derived from the
    two-hop rule, Section 3); the labels are all 0."""
    k = 101
    src = np.arange(k - 1, dtype=np.uint32)
    dst = src + np.uint32(1)
    with lc.Solver(k, dev32(src), dev32(dst), flags=lc.CC_EXPLICIT_PRIO) as s:
        s.set_priorities(0, dev32(np.arange(k)))
        rounds = s.run()
        labels = s.labels().cpu().numpy()
    assert rounds == (k - 1 + 1) // 2
    assert np.all(labels == 0)


def test_explicit_tables_per_round(lc):
    """A different ordering in every round (rounds past the last table keep it), against the
    oracle's multi-row explicit priorities; a round before any table would use the hash."""
    g = graphgen.er_with_paths(0xE1, 3000, 5000, 30, 60)
    rng = np.random.default_rng(11)
    rows = np.stack([rng.permutation(g.n).astype(np.uint32) for _ in range(4)])
    want = oracle.run(g.n, g.src, g.dst, explicit_prio=rows, record_parents=True)
    assert want.rounds > 4
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), flags=lc.CC_EXPLICIT_PRIO | lc.CC_RECORD_ROUNDS) as s:
        tabs = [dev32(r) for r in rows]
        for r in (2, 0, 3, 1):
            s.set_priorities(r, tabs[r])
        rounds = s.run()
        assert rounds == want.rounds
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        for r in range(rounds):
            np.testing.assert_array_equal(s.parents(r)[0].cpu().numpy().view(np.uint32), want.parents[r])
        np.testing.assert_array_equal(s.labels().cpu().numpy().view(np.uint32), want.labels)


def test_explicit_table_must_be_a_permutation(lc):
    g = graphgen.Graph(500, *graphgen.gnm(3, 500, 900))
    bad = np.arange(500, dtype=np.uint32)
    bad[7] = 3                    # two names with priority 3, none with 7
    big = np.arange(500, dtype=np.uint32)
    big[0] = 500                  # a priority outside [0, n)
    for table in (bad, big):
        with lc.Solver(g.n, dev32(g.src), dev32(g.dst), flags=lc.CC_EXPLICIT_PRIO) as s:
            s.set_priorities(0, dev32(table))
            with pytest.raises(lc.CCError) as e:
                s.run()
            assert e.value.status == -2   # CC_E_INPUT


@pytest.mark.parametrize("mode", ["direct", "tiled"])
@pytest.mark.parametrize("rule", ["local", "tree", "one_hop"])
def test_recorded_parents_of_every_round(lc, mode, rule):
    """CC_RECORD_ROUNDS: the parents of every round of a finished solve, by name, equal the
    oracle's; the node count is the round's n_active."""
    g = graphgen.er_with_paths(0xBEEF, 40000, 90001, 40, 300)
    flags = {"direct": DIRECT, "tiled": TILED}[mode] | {"local": 0, "tree": lc.CC_TREE, "one_hop": lc.CC_ONE_HOP}[rule]
    want = oracle.run(g.n, g.src, g.dst, seed=9, variant=rule, record_parents=True)
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), seed=9, flags=flags | lc.CC_RECORD_ROUNDS) as s:
        rounds = s.run()
        assert rounds == want.rounds
        stats = s.stats(rounds)
        for r in range(rounds):
            par, k = s.parents(r)
            np.testing.assert_array_equal(par.cpu().numpy().view(np.uint32), want.parents[r], err_msg="round %d" % r)
            assert k == stats[r][1] == want.stats[r][1]
        with pytest.raises(lc.CCError):
            s.parents(rounds + 1)
    # without the flag only the most recent round is kept
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), seed=9, flags=flags | lc.CC_EAGER) as s:
        s.contract_round()
        s.contract_round()
        np.testing.assert_array_equal(s.parents(1)[0].cpu().numpy().view(np.uint32), want.parents[1])
        with pytest.raises(lc.CCError) as e:
            s.parents(0)
        assert e.value.status == -5   # CC_E_STATE


@pytest.mark.parametrize("mode", ["direct", "tiled"])
def test_round_minima(lc, mode):
    """cc_debug_round_arrays after each round: the one-hop minimum m1 and the two-hop minimum
    l of every node equal the oracle's (after the tiled round 0, l is the priority of the
    parent, which equals the two-hop minimum by definition)."""
    g = graphgen.er_with_paths(0xA11, 1 << 20, (1 << 21) + 5, 100, 200)
    want = oracle.run(g.n, g.src, g.dst, seed=4, record_minima=True, minima_cap=32)
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), seed=4, flags={"direct": DIRECT, "tiled": TILED}[mode]) as s:
        r = 0
        while True:
            st, _ = s.contract_round()
            if st == lc.CC_DONE:
                break
            m1, l2 = s.minima()
            np.testing.assert_array_equal(m1.cpu().numpy().view(np.uint32), want.m1[r], err_msg="m1 round %d" % r)
            np.testing.assert_array_equal(l2.cpu().numpy().view(np.uint32), want.l[r], err_msg="l round %d" % r)
            r += 1
        assert r == want.rounds


def test_explicit_minima(lc):
    """The minima under an explicit table are values of that table."""
    g = graphgen.Graph(2000, *graphgen.gnm(8, 2000, 3000))
    tab = np.random.default_rng(8).permutation(g.n).astype(np.uint32)
    want = oracle.run(g.n, g.src, g.dst, explicit_prio=tab, record_minima=True)
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), flags=lc.CC_EXPLICIT_PRIO) as s:
        s.set_priorities(0, dev32(tab))
        s.contract_round()
        m1, l2 = s.minima()
    np.testing.assert_array_equal(m1.cpu().numpy().view(np.uint32), want.m1[0])
    np.testing.assert_array_equal(l2.cpu().numpy().view(np.uint32), want.l[0])


@pytest.mark.parametrize("k", [0, 1, 2, 4, 99])
def test_checkpoint_resume_equals_uninterrupted(lc, k):
    """Save after k rounds (k = 99: after the solve), load into a fresh context of the same
    graph (round 0 tiled in the first, direct in the second), continue: rounds, statistics and
    labels equal the oracle's uninterrupted solve."""
    g = graphgen.er_with_paths(0xC4, 1 << 20, 1 << 22, 200, 300)
    want = oracle.run(g.n, g.src, g.dst, seed=21)
    assert want.rounds > 4
    s_t, d_t = dev32(g.src), dev32(g.dst)
    with lc.Solver(g.n, s_t, d_t, seed=21, flags=TILED, max_rounds=k) as a:
        if k:
            a.run()
        blob = a.save_state()
    with lc.Solver(g.n, s_t, d_t, seed=1234, flags=DIRECT) as b:
        b.load_state(blob)
        rounds = b.run()
        assert rounds == want.rounds
        assert [tuple(x) for x in b.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(b.labels().cpu().numpy().view(np.uint32), want.labels)


def test_checkpoint_after_a_forced_failure(lc):
    """A failure forced from the host after round 2 (a priority table that is not a
    permutation makes round 3 fail with CC_E_INPUT), then the checkpoint taken after round 2
    is loaded into the same context, the good table is set again, and the solve ends as the
    uninterrupted one does."""
    g = graphgen.er_with_paths(0xF00, 20000, 40000, 50, 400)
    tab = np.random.default_rng(3).permutation(g.n).astype(np.uint32)
    want = oracle.run(g.n, g.src, g.dst, explicit_prio=tab)
    assert want.rounds > 4
    bad = tab.copy()
    bad[:2] = bad[0]
    good_t, bad_t = dev32(tab), dev32(bad)
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), flags=lc.CC_EXPLICIT_PRIO) as s:
        s.set_priorities(0, good_t)
        for _ in range(3):
            s.contract_round()
        blob = s.save_state()
        s.set_priorities(3, bad_t)
        with pytest.raises(lc.CCError) as e:
            s.contract_round()
        assert e.value.status == -2
        with pytest.raises(lc.CCError):      # the context stays failed
            s.run()
        s.load_state(blob)
        s.set_priorities(3, good_t)
        rounds = s.run()
        assert rounds == want.rounds
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().cpu().numpy().view(np.uint32), want.labels)


def test_checkpoint_rejects_another_graph(lc):
    g = graphgen.Graph(3000, *graphgen.gnm(1, 3000, 6000))
    h = graphgen.Graph(3001, *graphgen.gnm(1, 3000, 6000))
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), seed=2) as a:
        a.contract_round()
        blob = a.save_state()
    with lc.Solver(h.n, dev32(h.src), dev32(h.dst), seed=2) as b:
        with pytest.raises(lc.CCError) as e:
            b.load_state(blob)
        assert e.value.status == -1
        with pytest.raises(lc.CCError) as e:
            b.load_state(b"not a checkpoint" * 8)
        assert e.value.status == -1
    with lc.Solver(g.n, dev32(g.src), dev32(g.dst), seed=2, flags=lc.CC_TREE) as c:
        with pytest.raises(lc.CCError) as e:     # another label rule
            c.load_state(blob)
        assert e.value.status == -1
