"""The HIP library's own sources, built for the host against an emulation of the HIP
execution model (tests/hipemu), against the oracle -- no GPU needed.

This checks the kernels' and the engine's logic bit for bit (indexing, bounds, LDS, wave
ballots and shuffles, barriers, the host round engine, captured graphs, the batch and the
server), including the boundary calls for explicit priorities, recorded rounds, round minima
and checkpoints.  It does not replace the GPU parity tests (tests/test_gpu_*.py): the
hardware's timing and memory model are not emulated."""
from itertools import permutations

import ctypes

import numpy as np
import pytest

import graphgen
import oracle
from lcref import all_graph_adjacency, contract_edges, graph_records, split_keys

hipemu = pytest.importorskip("hipemu")

DIRECT, TILED = 1 << 2, 1 << 3
RULES = {"local": 0, "tree": 1 << 5, "one_hop": 1 << 6}


@pytest.fixture(scope="module")
def cc():
    try:
        return hipemu.binding()
    except Exception as e:   # no host compiler: nothing to emulate with
        pytest.skip("emulated build unavailable: %r" % (e,))


def dev(a, dt=np.int32):
    return hipemu.device(a, dt)


def inputs(g, layout):
    if layout == "soa32":
        return dev(g.src), dev(g.dst)
    if layout == "soa64":
        return dev(g.src, np.int64), dev(g.dst, np.int64)
    return dev(graphgen.pack(g.src, g.dst), np.uint64), None


def check_solve(cc, g, seed, flags=0, layout="soa32", rule="local", per_round=True, round0=0, tuning=None):
    want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=rule, record_parents=True)
    s_, d_ = inputs(g, layout)
    with hipemu.Solver(g.n, s_, d_, seed=seed, flags=flags | RULES[rule] | cc.CC_EAGER) as s:
        if round0 or tuning:
            s.set_tuning(round0=round0, **(tuning or {}))
        a, b = g.src, g.dst
        r = 0
        while per_round:
            st, stats = s.contract_round()
            if st == cc.CC_DONE:
                break
            assert stats == tuple(want.stats[r])
            par, k = s.parents()
            np.testing.assert_array_equal(par.view(np.uint32), want.parents[r], err_msg="round %d" % r)
            e = np.sort(s.edges())
            want_e = contract_edges(a, b, want.parents[r])
            np.testing.assert_array_equal(e, want_e, err_msg="edges after round %d" % r)
            a, b = split_keys(want_e)
            r += 1
        rounds = s.run()
        assert rounds == want.rounds
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
    return want


@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
@pytest.mark.parametrize("layout", ["soa32", "soa64", "packed"])
def test_emulated_solve_matches_oracle(cc, mode, layout):
    """Round by round (parents, edges, counts) and the final labels; "rows" is the tiled round
    0 fed by the one-pass row partition."""
    g = graphgen.Graph(6000, *graphgen.gnm(0x5151, 6000, 20011))
    check_solve(cc, g, 3, flags={"direct": DIRECT, "tiled": TILED, "rows": TILED}[mode], layout=layout,
                round0=3 if mode == "rows" else 0)


@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
@pytest.mark.parametrize("rule", ["local", "one_hop"])
def test_emulated_one_sweep_radix(cc, mode, rule):
    """cc_tuning.radix_form = 2: one count pass for every digit, then per digit a scatter whose
    tile offsets come from decoupled look-back.  Round by round (parents, edges, counts) and
    the labels, on a graph whose rounds 0 and 1 sort (round 1 with the sort and the hashed
    drop both enqueued, the device choosing)."""
    g = graphgen.Graph(60000, *graphgen.gnm(0x5EE9, 60000, 200000))
    check_solve(cc, g, 7, flags={"direct": DIRECT, "tiled": TILED, "rows": TILED}[mode], rule=rule,
                round0=3 if mode == "rows" else 0, tuning={"radix_form": 2})


@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
@pytest.mark.parametrize("rule", ["tree", "one_hop"])
def test_emulated_rules_match_oracle(cc, mode, rule):
    g = graphgen.er_with_paths(0x77, 3000, 7000, 10, 50)
    check_solve(cc, g, 4, flags={"direct": DIRECT, "tiled": TILED, "rows": TILED}[mode], rule=rule,
                round0=3 if mode == "rows" else 0)


def test_emulated_degenerate_inputs(cc):
    """Loops and repeats only, an edgeless graph, out-of-range ids."""
    g = graphgen.Graph(50, np.arange(50, dtype=np.uint32), np.arange(50, dtype=np.uint32))
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=1) as s:
        assert s.run() == 0
        np.testing.assert_array_equal(s.labels(), np.arange(50))
    g = graphgen.Graph(40, np.array([3, 3, 3, 9], np.uint32), np.array([9, 9, 9, 3], np.uint32))
    check_solve(cc, g, 2)
    with hipemu.Solver(10, dev(np.array([1, 12])), dev(np.array([2, 3])), seed=1) as s:
        with pytest.raises(cc.CCError) as e:
            s.run()
        assert e.value.status == cc.CC_E_INPUT


def test_emulated_captured_tails(cc):
    """A reused context replays captured tails for the small rounds (one readback each);
    rounds, statistics and labels are unchanged."""
    g = graphgen.er_with_paths(0x7A11, 20000, 50000, 40, 400)
    want = oracle.run(g.n, g.src, g.dst, seed=10)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=99) as s:
        s.run()
        s.reset(10)
        rounds = s.run()
        assert any(cc.cc_get_round_stats(s.ctx, r, True)[-1] for r in range(rounds))
        assert rounds == want.rounds
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


def in_graph(cc, s, rounds):
    return [cc.cc_get_round_stats(s.ctx, r, True)[-1] for r in range(rounds)]


@pytest.mark.parametrize("tail", [2, 3, 4])
@pytest.mark.parametrize("rule", ["local", "one_hop", "tree"])
def test_emulated_persistent_rounds(cc, tail, rule):
    """cc_tuning.tail >= 2: the rounds after round 0 small enough for the hashed duplicate drop
    run inside one cooperative launch, whose
    workgroups the emulation runs on host threads of their own, meeting at real grid-wide
    barriers.  Rounds, statistics and labels are the oracle's on a fresh and on a reused
    context; those rounds report in_graph = 2, and their parents are not available."""
    g = graphgen.er_with_paths(0x7A11, 20000, 50000, 40, 400)
    want = oracle.run(g.n, g.src, g.dst, seed=10, variant=rule)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=10, flags=RULES[rule]) as s:
        s.set_tuning(tail=tail)
        assert s.tuning["tail"] == tail
        for _ in range(2):
            rounds = s.run()
            assert rounds == want.rounds
            # round 0, and a round too large for the hashed duplicate drop, run on their own
            ig = in_graph(cc, s, rounds)
            first = ig.index(2)
            assert first >= 1 and ig == [0] * first + [2] * (rounds - first)
            assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
            np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
            with pytest.raises(cc.CCError) as e:
                s.parents()
            assert e.value.status == cc.CC_E_STATE
            s.reset(10)
        # back to the default: launch sequences per round (captured tails on this reused context)
        s.set_tuning(tail=1)
        rounds = s.run()
        assert 2 not in in_graph(cc, s, rounds)
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=10, flags=RULES[rule] | cc.CC_EAGER) as s:
        s.set_tuning(tail=tail)
        rounds = s.run()
        assert in_graph(cc, s, rounds) == [0] * rounds
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


@pytest.mark.parametrize("alphas", [[3], [2, 5, 4]])
@pytest.mark.parametrize("tail", [2, 3])
def test_emulated_persistent_merge_to_large(cc, alphas, tail):
    """MergeToLarge inside the persistent launch: LocalContraction steps (with the class sizes
    and alpha-th priorities after each) alternating with MergeToLarge steps (two candidate
    passes), each phase with its own alpha: rounds, statistics and labels are the oracle's."""
    g = graphgen.er_with_paths(0x7A11, 20000, 50000, 40, 400)
    want = oracle.run(g.n, g.src, g.dst, seed=5, variant="merge_to_large", alphas=alphas)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=5, flags=(1 << 9) | cc.CC_PROFILE) as s:
        s.set_tuning(tail=tail)
        s.set_merge_to_large(alphas)
        rounds = s.run()
        assert rounds == want.rounds
        assert 2 in in_graph(cc, s, rounds) and cc.cc_kernel_times(s.ctx)["fused_rounds"][1] >= 1
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


@pytest.mark.parametrize("max_rounds", [3, 5])
def test_emulated_persistent_rounds_stop_at_max_rounds(cc, max_rounds):
    """cc_options.max_rounds inside the persistent launch: the solve stops after exactly that
    many rounds, with the oracle's statistics and partial labels."""
    g = graphgen.er_with_paths(0x7A11, 20000, 50000, 40, 400)
    want = oracle.run(g.n, g.src, g.dst, seed=10, max_rounds=max_rounds)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=10, max_rounds=max_rounds) as s:
        s.set_tuning(tail=2)
        rounds = s.run()
        assert rounds == want.rounds == max_rounds
        assert in_graph(cc, s, rounds)[-1] == 2
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


@pytest.mark.parametrize("finish", [300, 1000])
def test_emulated_persistent_rounds_then_union_find(cc, finish):
    """The union-find finish after rounds in the persistent launch: the launch stops once the
    graph has at most `finish` records, and the finish ends the solve as the oracle's does."""
    g = graphgen.er_with_paths(0x7A11, 20000, 50000, 40, 400)
    want = oracle.run(g.n, g.src, g.dst, seed=10, finish_edges=finish)
    assert want.finished
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=10, finish_edges=finish) as s:
        s.set_tuning(tail=3)
        rounds = s.run()
        assert rounds == want.rounds and 2 in in_graph(cc, s, rounds)
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


@pytest.mark.parametrize("rule,seed,launches", [("local", 3, 1), ("one_hop", 22, 2), ("tree", 3, 1)])
def test_emulated_persistent_rounds_large(cc, rule, seed, launches):
    """About a million path vertices.  LocalContraction: round 1 has more than 2^18 nodes, so
    the label and node maps take the count, scan and write phases with grid-wide barriers
    between them instead of one workgroup.  One-hop rule at this seed: the rounds' nodes add up
    to more than the per-round map arena holds, so the launch stops before the round that
    would overflow it, the host folds the maps, and a second launch finishes the solve.
    TreeContraction: its pointer-jumping passes inside the launch, over 250,000 nodes."""
    g = graphgen.er_with_paths(0xB16, 1 << 12, 1 << 13, 1000, 1000)
    want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=rule)
    assert rule == "tree" or want.stats[1][1] > 1 << 18
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=seed, flags=RULES[rule] | cc.CC_PROFILE) as s:
        s.set_tuning(tail=2)
        rounds = s.run()
        assert rounds == want.rounds
        ig = in_graph(cc, s, rounds)
        assert ig[0] == 0 and ig[-1] == 2 and (rule != "local" or ig[1:] == [2] * (rounds - 1))
        assert cc.cc_kernel_times(s.ctx)["fused_rounds"][1] == launches
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


def test_emulated_kernel_counts(cc):
    """Kernels executed per solve (run and labels) on a graph of many rounds: the persistent
    launch of the small rounds and the one-sweep radix passes each execute fewer kernels than
    the default launch sequences, and both together fewer than half as many, with the same
    labels."""
    lib = ctypes.CDLL(cc.LIB_PATH)
    lib.hipemu_launches.restype = ctypes.c_longlong
    g = graphgen.er_with_paths(0xD15, 1 << 14, 1 << 17, 40, 500)
    want = oracle.run(g.n, g.src, g.dst, seed=3)
    assert want.rounds >= 6
    counts = {}
    for name, kn in (("default", {}), ("tail", {"tail": 2}), ("sweep", {"radix_form": 2}),
                     ("both", {"tail": 2, "radix_form": 2})):
        with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=3, flags=DIRECT) as s:
            s.set_tuning(**kn)
            k0 = lib.hipemu_launches()
            assert s.run() == want.rounds
            lab = s.labels()
            counts[name] = lib.hipemu_launches() - k0
            np.testing.assert_array_equal(lab.astype(np.uint32), want.labels)
    assert counts["tail"] < counts["default"] and counts["sweep"] < counts["default"]
    assert 2 * counts["both"] < counts["default"], counts


FALLBACK_CHECK = r"""
import sys
sys.path[:0] = [%r, %r]
import numpy as np, graphgen, oracle, hipemu
cc = hipemu.binding()
g = graphgen.er_with_paths(0x7A11, 20000, 50000, 40, 400)
want = oracle.run(g.n, g.src, g.dst, seed=10)
with hipemu.Solver(g.n, hipemu.device(g.src, np.int32), hipemu.device(g.dst, np.int32), seed=10,
                   flags=cc.CC_PROFILE) as s:
    s.set_tuning(tail=4)
    r = s.run()
    ok = r == want.rounds and [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats] and \
        np.array_equal(s.labels().astype(np.uint32), want.labels)
    launches = cc.cc_kernel_times(s.ctx)["fused_rounds"][1]
    print("OK", ok, launches, [cc.cc_get_round_stats(s.ctx, k, True)[-1] for k in range(r)])
"""


def test_emulated_persistent_rounds_fall_back(cc):
    """A device that cannot keep even one workgroup of the persistent kernel resident per
    compute unit refuses the cooperative launch; the context then runs the rounds one launch
    sequence each, with the same results."""
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, HIPEMU_RESIDENT_PER_CU="0")
    proc = subprocess.run([sys.executable, "-c", FALLBACK_CHECK % (os.path.dirname(here), here)], env=env,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600)
    assert proc.returncode == 0, proc.stderr[-2000:]
    assert "OK True 0 [0, 0, 0" in proc.stdout and "2" not in proc.stdout.split("OK True 0")[1], proc.stdout


def test_emulated_union_find_finish_and_canonical(cc):
    g = graphgen.er_with_paths(0xF1, 5000, 9000, 20, 100)
    want = oracle.run(g.n, g.src, g.dst, seed=5, finish_edges=300)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=5, finish_edges=300) as s:
        rounds = s.run()
        assert rounds == want.rounds and want.finished
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
    comp = oracle.components_min_id(g.n, g.src, g.dst)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=5, flags=cc.CC_CANONICAL) as s:
        s.run()
        np.testing.assert_array_equal(s.labels().astype(np.uint32), comp)


# ---- explicit priorities ---------------------------------------------------------------------

def all_orderings_union(max_n):
    """Every labelled graph on n <= max_n vertices under every ordering of its vertices, as
    one disjoint union with a priority table that orders each copy by its own ordering."""
    srcs, dsts, tabs = [], [], []
    off = 0
    for n in range(1, max_n + 1):
        adj = all_graph_adjacency(n)
        G = adj.shape[0]
        src, dst, eoff = graph_records(adj)
        gid = np.repeat(np.arange(G, dtype=np.uint32), np.diff(eoff).astype(np.int64))
        perms = np.array(list(permutations(range(n))), dtype=np.uint32)
        P = perms.shape[0]
        base_rec = (np.arange(P, dtype=np.uint32)[:, None] * np.uint32(G) + gid[None, :]) * np.uint32(n) + np.uint32(off)
        srcs.append((base_rec + src[None, :]).ravel())
        dsts.append((base_rec + dst[None, :]).ravel())
        base_v = (np.arange(P * G, dtype=np.uint32) * np.uint32(n) + np.uint32(off)).reshape(P, G, 1)
        tabs.append((base_v + perms[:, None, :]).ravel())
        off += P * G * n
    return off, np.concatenate(srcs), np.concatenate(dsts), np.concatenate(tabs)


def test_emulated_every_ordering_of_every_graph_up_to_5(cc):
    n, src, dst, tab = all_orderings_union(5)
    assert np.array_equal(np.sort(tab), np.arange(n, dtype=np.uint32))
    want = oracle.run(n, src, dst, explicit_prio=tab, record_parents=True)
    with hipemu.Solver(n, dev(src), dev(dst), flags=cc.CC_EXPLICIT_PRIO | cc.CC_RECORD_ROUNDS) as s:
        s.set_priorities(0, tab)
        rounds = s.run()
        assert rounds == want.rounds
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        for r in range(rounds):
            np.testing.assert_array_equal(s.parents(r)[0].view(np.uint32), want.parents[r], err_msg="round %d" % r)
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


def test_emulated_identity_order_on_a_path(cc):
    k = 61
    src = np.arange(k - 1, dtype=np.uint32)
    with hipemu.Solver(k, dev(src), dev(src + 1), flags=cc.CC_EXPLICIT_PRIO) as s:
        s.set_priorities(0, np.arange(k))
        assert s.run() == (k - 1 + 1) // 2
        assert np.all(s.labels() == 0)


def test_emulated_tables_per_round(cc):
    g = graphgen.er_with_paths(0xE1, 3000, 5000, 30, 60)
    rng = np.random.default_rng(11)
    rows = np.stack([rng.permutation(g.n).astype(np.uint32) for _ in range(4)])
    want = oracle.run(g.n, g.src, g.dst, explicit_prio=rows, record_parents=True)
    assert want.rounds > 4
    for rule_flags in (0, RULES["tree"], RULES["one_hop"]):
        if rule_flags:
            want = oracle.run(g.n, g.src, g.dst, explicit_prio=rows, record_parents=True,
                              variant="tree" if rule_flags == RULES["tree"] else "one_hop")
        with hipemu.Solver(g.n, dev(g.src), dev(g.dst),
                           flags=cc.CC_EXPLICIT_PRIO | cc.CC_RECORD_ROUNDS | rule_flags) as s:
            for r in (2, 0, 3, 1):
                s.set_priorities(r, rows[r])
            rounds = s.run()
            assert rounds == want.rounds
            assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
            for r in range(rounds):
                np.testing.assert_array_equal(s.parents(r)[0].view(np.uint32), want.parents[r])
            np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


def test_emulated_table_must_be_a_permutation(cc):
    g = graphgen.Graph(500, *graphgen.gnm(3, 500, 900))
    bad = np.arange(500, dtype=np.uint32)
    bad[7] = 3
    big = np.arange(500, dtype=np.uint32)
    big[0] = 500
    for table in (bad, big):
        with hipemu.Solver(g.n, dev(g.src), dev(g.dst), flags=cc.CC_EXPLICIT_PRIO) as s:
            s.set_priorities(0, table)
            with pytest.raises(cc.CCError) as e:
                s.run()
            assert e.value.status == cc.CC_E_INPUT


def test_emulated_hash_before_the_first_table(cc):
    """Rounds before the first table use the seeded hash: a table from round 1 on leaves
    round 0 as in a hashed solve."""
    g = graphgen.er_with_paths(0xE2, 2000, 4000, 10, 80)
    plain = oracle.run(g.n, g.src, g.dst, seed=8, record_parents=True)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=8, flags=cc.CC_EXPLICIT_PRIO) as s:
        s.set_priorities(1, np.arange(g.n))
        s.contract_round()
        np.testing.assert_array_equal(s.parents()[0].view(np.uint32), plain.parents[0])


# ---- recorded rounds, minima, checkpoints ------------------------------------------------------

@pytest.mark.parametrize("mode", ["direct", "tiled"])
@pytest.mark.parametrize("rule", ["local", "tree", "one_hop"])
def test_emulated_recorded_parents(cc, mode, rule):
    g = graphgen.er_with_paths(0xBEEF, 4000, 9001, 10, 120)
    want = oracle.run(g.n, g.src, g.dst, seed=9, variant=rule, record_parents=True)
    flags = {"direct": DIRECT, "tiled": TILED}[mode] | RULES[rule] | cc.CC_RECORD_ROUNDS
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=9, flags=flags) as s:
        rounds = s.run()
        assert rounds == want.rounds
        stats = s.stats(rounds)
        for r in range(rounds):
            par, k = s.parents(r)
            np.testing.assert_array_equal(par.view(np.uint32), want.parents[r], err_msg="round %d" % r)
            assert k == stats[r][1]
        with pytest.raises(cc.CCError):
            s.parents(rounds + 1)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=9, flags=flags & ~cc.CC_RECORD_ROUNDS) as s:
        s.contract_round()
        s.contract_round()
        np.testing.assert_array_equal(s.parents(1)[0].view(np.uint32), want.parents[1])
        with pytest.raises(cc.CCError) as e:
            s.parents(0)
        assert e.value.status == cc.CC_E_STATE


@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
def test_emulated_round_minima(cc, mode):
    g = graphgen.er_with_paths(0xA11, 6000, 15000, 10, 200)
    want = oracle.run(g.n, g.src, g.dst, seed=4, record_minima=True, minima_cap=64)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=4, flags={"direct": DIRECT, "tiled": TILED,
                                                                    "rows": TILED}[mode]) as s:
        if mode == "rows":
            s.set_tuning(round0=3, round0_sort=2)
        r = 0
        while s.contract_round()[0] != cc.CC_DONE:
            m1, l2 = s.minima()
            np.testing.assert_array_equal(m1, want.m1[r], err_msg="m1 round %d" % r)
            np.testing.assert_array_equal(l2, want.l[r], err_msg="l round %d" % r)
            r += 1
        assert r == want.rounds


def test_emulated_explicit_minima(cc):
    g = graphgen.Graph(2000, *graphgen.gnm(8, 2000, 3000))
    tab = np.random.default_rng(8).permutation(g.n).astype(np.uint32)
    want = oracle.run(g.n, g.src, g.dst, explicit_prio=tab, record_minima=True)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), flags=cc.CC_EXPLICIT_PRIO) as s:
        s.set_priorities(0, tab)
        s.contract_round()
        m1, l2 = s.minima()
    np.testing.assert_array_equal(m1, want.m1[0])
    np.testing.assert_array_equal(l2, want.l[0])


@pytest.mark.parametrize("k", [0, 1, 2, 4, 99])
def test_emulated_checkpoint_resume(cc, k):
    g = graphgen.er_with_paths(0xC4, 6000, 14000, 20, 300)
    want = oracle.run(g.n, g.src, g.dst, seed=21)
    assert want.rounds > 4
    s_, d_ = dev(g.src), dev(g.dst)
    with hipemu.Solver(g.n, s_, d_, seed=21, flags=TILED, max_rounds=k) as a:
        if k:
            a.run()
        blob = a.save_state()
    for tail in (1, 3):   # the resumed solve in launch sequences, or in the persistent launch
        with hipemu.Solver(g.n, s_, d_, seed=1234, flags=DIRECT) as b:
            b.set_tuning(tail=tail)
            b.load_state(blob)
            rounds = b.run()
            assert rounds == want.rounds
            assert [tuple(x) for x in b.stats(rounds)] == [tuple(x) for x in want.stats]
            np.testing.assert_array_equal(b.labels().astype(np.uint32), want.labels)
            assert (2 in in_graph(cc, b, rounds)) == (tail == 3 and rounds > max(k, 1))


def test_emulated_checkpoint_after_a_forced_failure(cc):
    g = graphgen.er_with_paths(0xF00, 5000, 10000, 20, 300)
    tab = np.random.default_rng(3).permutation(g.n).astype(np.uint32)
    want = oracle.run(g.n, g.src, g.dst, explicit_prio=tab)
    assert want.rounds > 4
    bad = tab.copy()
    bad[:2] = bad[0]
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), flags=cc.CC_EXPLICIT_PRIO) as s:
        s.set_priorities(0, tab)
        for _ in range(3):
            s.contract_round()
        blob = s.save_state()
        s.set_priorities(3, bad)
        with pytest.raises(cc.CCError) as e:
            s.contract_round()
        assert e.value.status == cc.CC_E_INPUT
        with pytest.raises(cc.CCError):
            s.run()
        s.load_state(blob)
        s.set_priorities(3, tab)
        rounds = s.run()
        assert rounds == want.rounds
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


def test_emulated_checkpoint_rejects_another_graph(cc):
    g = graphgen.Graph(3000, *graphgen.gnm(1, 3000, 6000))
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=2) as a:
        a.contract_round()
        blob = a.save_state()
    with hipemu.Solver(g.n + 1, dev(g.src), dev(g.dst), seed=2) as b:
        for data in (blob, b"not a checkpoint" * 8, blob[:100]):
            with pytest.raises(cc.CCError) as e:
                b.load_state(data)
            assert e.value.status == cc.CC_E_ARG
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=2, flags=cc.CC_TREE) as c:
        with pytest.raises(cc.CCError) as e:
            c.load_state(blob)
        assert e.value.status == cc.CC_E_ARG
    # a device state that disagrees with the header, or would index past the map arena, is
    # refused before anything reaches the device (header: 120 bytes, n_stats at byte 60, n_cur
    # at byte 72; state fields n_cur at byte 0, map_off at byte 32, e_sel at byte 64)
    n_stats = int(np.frombuffer(blob, np.int32, 1, 60)[0])
    st0 = 120 + n_stats * ctypes.sizeof(cc.cc_round_stats)
    assert n_stats == 1
    assert int(np.frombuffer(blob, np.uint64, 1, st0)[0]) == int(np.frombuffer(blob, np.int64, 1, 72)[0]) > 0
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=2) as d:
        d.load_state(blob)                       # the blob as written loads
        for at, value in ((st0 + 32, 1 << 40), (st0 + 64, 7)):
            bad = bytearray(blob)
            bad[at:at + 8] = int(value).to_bytes(8, "little")
            with pytest.raises(cc.CCError) as e:
                d.load_state(bytes(bad))
            assert e.value.status == cc.CC_E_ARG


# ---- batch and serving -----------------------------------------------------------------------

@pytest.mark.parametrize("variant", [0, 1, 3])
@pytest.mark.parametrize("fill", [0x00, 0xFF])
@pytest.mark.parametrize("radix_form", [1, 2])
def test_emulated_batch(cc, variant, fill, radix_form):
    """The batch (LDS solver and union path, captured and replayed; the union's radix passes in
    either form) on a workspace that starts with arbitrary bytes: each graph's labels and
    rounds are the oracle's."""
    b = graphgen.batch_mix(seed=31, count=24, log2_min=4, log2_max=11)
    want_lab, want_rounds, _ = oracle.run_batch(b.voff, b.eoff, b.src, b.dst, b.seeds)
    with hipemu.Batch(b.voff, b.eoff, b.seeds, b.src, b.dst, ws_fill=fill, small_variant=variant,
                      radix_form=radix_form) as bt:
        assert bt.config["radix_form"] == radix_form
        n_small, _ = bt.split()
        assert (n_small > 0) == (variant > 0)
        for _ in range(2):
            lab, rounds = bt.run()
            np.testing.assert_array_equal(rounds, want_rounds)
            np.testing.assert_array_equal(lab.astype(np.uint32), want_lab)


def test_emulated_contexts_end_without_a_device_wide_wait(cc):
    """Destroying a context while others run must not wait for the whole device: its pinned
    host mirror of the round state goes back to a pool instead of being freed."""
    syncs = cc._lib.hipemu_device_syncs
    syncs.restype = ctypes.c_longlong
    g = graphgen.Graph(500, *graphgen.gnm(0x51, 500, 1500))
    want = oracle.run(g.n, g.src, g.dst, seed=5)
    before = syncs()
    for _ in range(6):
        with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=5) as s:
            assert s.run() == want.rounds
            np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
    assert syncs() == before


def test_emulated_server(cc):
    """Requests of both paths (fused LDS launch and per-slot rounds) in one server: every
    result is the oracle's.  While it serves, the server makes no call that synchronises the
    whole device (such as freeing pinned host memory when a request completes), which would
    stall every other request in flight."""
    import time
    syncs = cc._lib.hipemu_device_syncs
    syncs.restype = ctypes.c_longlong
    trace = graphgen.request_trace(0x5E7, 10, rate=1.0, log2_min=5, log2_max=13)
    graphs = [r.graph() for r in trace]
    arena = hipemu._aligned(1 << 28, None)
    srv = cc.cc_server_create(arena.ctypes.data, arena.size, n_slots=3, small_variant=1,
                              max_small_per_launch=4)
    keep, out = {}, {}
    syncs0 = syncs()
    try:
        for i, (g, r) in enumerate(zip(graphs, trace)):
            s_, d_ = dev(g.src), dev(g.dst)
            lab = np.full(max(g.n, 1), -7, np.int32)
            rid = cc.cc_server_submit(srv, g.n, g.m, cc.CC_EDGES_SOA_I32, s_.ctypes.data, d_.ctypes.data, r.seed,
                                      lab.ctypes.data)
            keep[rid] = (i, s_, d_, lab)
        t_end = time.time() + 300
        while len(out) < len(graphs) and time.time() < t_end:
            for res in cc.cc_server_wait(srv, 0.5):
                out[res["id"]] = res
        served_syncs = syncs() - syncs0
    finally:
        cc.cc_server_destroy(srv)
    assert len(out) == len(graphs)
    assert served_syncs == 0
    small = 0
    for rid, res in out.items():
        i, _, _, lab = keep[rid]
        g = graphs[i]
        want = oracle.run(g.n, g.src, g.dst, seed=trace[i].seed)
        assert res["status"] == 0 and res["rounds"] == want.rounds
        np.testing.assert_array_equal(lab[:g.n].astype(np.uint32), want.labels, err_msg="request %d" % i)
        small += res["small_path"]
    assert 0 < small < len(graphs)


def test_emulated_server_cohorts(cc):
    """Large requests started together as cohorts (one disjoint union, one launch sequence a
    round for all of them): every request's labels and round count are the oracle's; a
    request with an id out of range fails alone, its cohort's others are unaffected; no
    device-wide wait while serving."""
    import time
    syncs = cc._lib.hipemu_device_syncs
    syncs.restype = ctypes.c_longlong
    rng = np.random.default_rng(5)
    graphs = []
    for i in range(11):
        n = int(rng.integers(600, 4000))
        g = graphgen.Graph(n, *graphgen.gnm(700 + i, n, int(rng.integers(n // 2, 3 * n))))
        graphs.append(g)
    bad = 6   # this request names a vertex out of range
    graphs[bad] = graphgen.Graph(graphs[bad].n, graphs[bad].src.copy(), graphs[bad].dst.copy())
    graphs[bad].dst[3] = graphs[bad].n + 5
    arena = hipemu._aligned(1 << 28, None)
    srv = cc.cc_server_create(arena.ctypes.data, arena.size, n_slots=2, small_variant=1, max_small_per_launch=4,
                              cohort_max=4, cohort_max_vertices=1 << 12)
    keep, out = {}, {}
    syncs0 = syncs()
    try:
        cc.cc_server_pause(srv, True)   # the whole burst waits, then starts as cohorts
        for i, g in enumerate(graphs):
            s_, d_ = dev(g.src), dev(g.dst)
            lab = np.full(g.n, -7, np.int32)
            rid = cc.cc_server_submit(srv, g.n, g.m, cc.CC_EDGES_SOA_I32, s_.ctypes.data, d_.ctypes.data, 40 + i,
                                      lab.ctypes.data)
            keep[rid] = (i, s_, d_, lab)
        cc.cc_server_pause(srv, False)
        t_end = time.time() + 300
        while len(out) < len(graphs) and time.time() < t_end:
            for res in cc.cc_server_wait(srv, 0.5):
                out[res["id"]] = res
        served_syncs = syncs() - syncs0
    finally:
        cc.cc_server_destroy(srv)
    assert len(out) == len(graphs)
    assert served_syncs == 0
    cohorts = 0
    for rid, res in out.items():
        i, _, _, lab = keep[rid]
        if i == bad:
            assert res["status"] == cc.CC_E_INPUT and res["cohort"] == 4
            continue
        g = graphs[i]
        want = oracle.run(g.n, g.src, g.dst, seed=40 + i)
        assert res["status"] == 0 and res["rounds"] == want.rounds, (i, res)
        np.testing.assert_array_equal(lab.astype(np.uint32), want.labels, err_msg="request %d" % i)
        cohorts += res["cohort"] > 1
    assert cohorts == 10   # every request ran fused: 4 + 4 (with the bad one) + 3


def test_emulated_server_pause(cc):
    """While paused the server admits nothing (submissions wait, info reports them pending);
    destroying a paused server with waiting requests ends them and returns."""
    import time
    g = graphgen.Graph(3000, *graphgen.gnm(9, 3000, 9000))
    s_, d_ = dev(g.src), dev(g.dst)
    labs = [np.full(g.n, -7, np.int32) for _ in range(3)]
    arena = hipemu._aligned(1 << 26, None)
    srv = cc.cc_server_create(arena.ctypes.data, arena.size, n_slots=2, small_variant=1, cohort_max=4)
    try:
        cc.cc_server_pause(srv, True)
        for i, lab in enumerate(labs):
            cc.cc_server_submit(srv, g.n, g.m, cc.CC_EDGES_SOA_I32, s_.ctypes.data, d_.ctypes.data, 3, lab.ctypes.data)
        time.sleep(0.2)
        info = cc.cc_server_info(srv)
        assert info["pending"] == 3 and info["active"] == 0
        assert cc.cc_server_poll(srv) == []
        assert all((lab == -7).all() for lab in labs)
    finally:
        cc.cc_server_destroy(srv)   # paused, with waiting requests: must return


# ---- MergeToLarge ----------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
@pytest.mark.parametrize("alphas", [[1], [2], [3, 5, 9], [10 ** 6]])
def test_emulated_merge_to_large(cc, mode, alphas):
    """Every round (LocalContraction steps and MergeToLarge steps) against the oracle: parents
    by name, statistics, the edges each round leaves, labels."""
    g = graphgen.er_with_paths(0x3E7, 5000, 16000, 20, 150)
    want = oracle.run(g.n, g.src, g.dst, seed=12, variant="merge_to_large", alphas=alphas, record_parents=True,
                      parents_cap=64)
    flags = {"direct": DIRECT, "tiled": TILED, "rows": TILED}[mode] | cc.CC_MERGE_TO_LARGE | cc.CC_RECORD_ROUNDS
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=12, flags=flags) as s:
        if mode == "rows":
            s.set_tuning(round0=3)
        s.set_merge_to_large(alphas)
        a, b = g.src, g.dst
        r = 0
        while s.contract_round()[0] != cc.CC_DONE:
            e = np.sort(s.edges())
            want_e = contract_edges(a, b, want.parents[r])
            np.testing.assert_array_equal(e, want_e, err_msg="edges after round %d" % r)
            a, b = split_keys(want_e)
            r += 1
        rounds = s.run()
        assert rounds == want.rounds == r
        assert [tuple(x) for x in s.stats(rounds)] == [tuple(x) for x in want.stats]
        for q in range(rounds):
            np.testing.assert_array_equal(s.parents(q)[0].view(np.uint32), want.parents[q], err_msg="round %d" % q)
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


def test_emulated_merge_to_large_default_alpha_and_explicit(cc):
    g = graphgen.Graph(3000, *graphgen.gnm(0x3E8, 3000, 12000))
    want = oracle.run(g.n, g.src, g.dst, seed=2, variant="merge_to_large")      # default alpha
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=2, flags=cc.CC_MERGE_TO_LARGE) as s:
        assert s.run() == want.rounds
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
    tab = np.random.default_rng(4).permutation(g.n).astype(np.uint32)
    want = oracle.run(g.n, g.src, g.dst, explicit_prio=tab, variant="merge_to_large", alphas=[4])
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), flags=cc.CC_MERGE_TO_LARGE | cc.CC_EXPLICIT_PRIO) as s:
        s.set_merge_to_large([4])
        s.set_priorities(0, tab)
        assert s.run() == want.rounds
        assert [tuple(x) for x in s.stats(want.rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_emulated_merge_to_large_checkpoint(cc, k):
    """A checkpoint after a LocalContraction step carries the classes' sizes and priorities
    that the following MergeToLarge step reads."""
    g = graphgen.er_with_paths(0x3E9, 4000, 12000, 20, 150)
    want = oracle.run(g.n, g.src, g.dst, seed=6, variant="merge_to_large", alphas=[3])
    assert want.rounds > k
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=6, flags=cc.CC_MERGE_TO_LARGE, max_rounds=k) as a:
        a.set_merge_to_large([3])
        a.run()
        blob = a.save_state()
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=6, flags=cc.CC_MERGE_TO_LARGE) as b:
        b.set_merge_to_large([3])
        b.load_state(blob)
        assert b.run() == want.rounds
        assert [tuple(x) for x in b.stats(want.rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(b.labels().astype(np.uint32), want.labels)


def test_emulated_merge_to_large_arguments(cc):
    g = graphgen.Graph(100, *graphgen.gnm(1, 100, 200))
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst)) as s:
        with pytest.raises(cc.CCError) as e:
            s.set_merge_to_large([3])
        assert e.value.status == cc.CC_E_STATE
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), flags=cc.CC_MERGE_TO_LARGE) as s:
        for bad in ([0], [3, -1]):
            with pytest.raises(cc.CCError) as e:
                s.set_merge_to_large(bad)
            assert e.value.status == cc.CC_E_ARG
    for rule in (cc.CC_TREE, cc.CC_ONE_HOP):
        with pytest.raises(cc.CCError) as e:
            hipemu.Solver(g.n, dev(g.src), dev(g.dst), flags=cc.CC_MERGE_TO_LARGE | rule)
        assert e.value.status == cc.CC_E_ARG


# ---- order independence ------------------------------------------------------------------------

ORDER_CHECK = r"""
import sys
sys.path[:0] = [%r, %r]
import numpy as np, graphgen, oracle, hipemu
cc = hipemu.binding()
fails = []
rmat = graphgen.Graph(1 << 14, *graphgen.rmat(3, 14, 16 << 14))
cases = [("rmat", rmat, cc.CC_ROUND0_TILED, 0, {}),
         ("rmat rows buckets", rmat, cc.CC_ROUND0_TILED, 0, {"round0": 3, "round0_sort": 2}),
         ("paths", graphgen.er_with_paths(9, 3000, 6000, 20, 200), cc.CC_ROUND0_DIRECT, 0, {}),
         ("paths persistent", graphgen.er_with_paths(9, 3000, 6000, 20, 200), cc.CC_ROUND0_DIRECT, 0, {"tail": 3}),
         ("rmat one sweep", rmat, cc.CC_ROUND0_TILED, 0, {"radix_form": 2}),
         ("gnm one sweep", graphgen.Graph(30000, *graphgen.gnm(8, 30000, 100000)), cc.CC_ROUND0_DIRECT, 0,
          {"radix_form": 2}),
         ("mtl", graphgen.er_with_paths(10, 3000, 9000, 20, 100), cc.CC_ROUND0_TILED, cc.CC_MERGE_TO_LARGE, {})]
for name, g, flags, extra, knobs in cases:
    want = oracle.run(g.n, g.src, g.dst, seed=5, variant="merge_to_large" if extra else "local", alphas=[3] if extra else None)
    with hipemu.Solver(g.n, hipemu.device(g.src, np.int32), hipemu.device(g.dst, np.int32), seed=5,
                       flags=flags | extra) as s:
        if knobs:
            s.set_tuning(**knobs)
        if extra:
            s.set_merge_to_large([3])
        r = s.run()
        ok = r == want.rounds and [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats] and \
            np.array_equal(s.labels().astype(np.uint32), want.labels)
    if not ok:
        fails.append(name)
b = graphgen.batch_mix(seed=41, count=16, log2_min=4, log2_max=11)
lab_w, rounds_w, _ = oracle.run_batch(b.voff, b.eoff, b.src, b.dst, b.seeds)
with hipemu.Batch(b.voff, b.eoff, b.seeds, b.src, b.dst, small_variant=1) as bt:
    lab, rounds = bt.run()
    if not (np.array_equal(rounds, rounds_w) and np.array_equal(lab.astype(np.uint32), lab_w)):
        fails.append("batch")
print("FAILS", fails)
"""


@pytest.mark.parametrize("order", ["reverse", "12345", "777", "forward/items reversed", "4242/threads"])
def test_emulated_results_do_not_depend_on_workgroup_order(cc, order):
    """The same solves with the workgroups of every launch run in reverse or shuffled order:
    atomics, cursors and the relabel's key sets then see other interleavings, and the results
    must not change.  "items reversed" keeps the workgroups in order but runs the work-items of
    each one last to first between synchronisation points, which would expose waves sharing
    LDS or global words without a barrier between them.  "threads" runs the workgroups of
    every launch on four host threads at once, so that workgroups really race on global
    memory."""
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    code = ORDER_CHECK % (os.path.dirname(here), here)
    env = dict(os.environ, HIPEMU_BLOCK_ORDER=order.split("/")[0])
    if order.endswith("items reversed"):
        env["HIPEMU_ITEM_ORDER"] = "reverse"
    if order.endswith("threads"):
        env["HIPEMU_THREADS"] = "4"
    proc = subprocess.run([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                          text=True, timeout=600)
    assert proc.returncode == 0, proc.stderr[-2000:]
    assert "FAILS []" in proc.stdout, proc.stdout


@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
def test_emulated_round0_key_sets(cc, mode):
    """Round 0 on a power-law graph: the relabel workgroups' key sets drop most repeated keys
    before the sort (m_sorted well below m_survive), and everything the method defines is
    unchanged; on a uniform random graph the sets switch themselves off early.  "rows": the
    tiled round 0 with the one-pass row partition."""
    flags = {"direct": DIRECT, "tiled": TILED, "rows": TILED}[mode]

    def solver(h, seed):
        s = hipemu.Solver(h.n, dev(h.src), dev(h.dst), seed=seed, flags=flags)
        if mode == "rows":
            s.set_tuning(round0=3)
        return s

    g = graphgen.Graph(1 << 15, *graphgen.rmat(21, 15, 16 << 15))
    want = oracle.run(g.n, g.src, g.dst, seed=17)
    with solver(g, 17) as s:
        assert s.run() == want.rounds
        assert [tuple(x) for x in s.stats(want.rounds)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
    with solver(g, 17) as s:
        s.contract_round()
        assert cc.cc_get_round_sorted(s.ctx, 0) * 4 < want.stats[0][3]
    u = graphgen.Graph(1 << 15, *graphgen.gnm(22, 1 << 15, 1 << 17))
    want = oracle.run(u.n, u.src, u.dst, seed=17)
    with solver(u, 17) as s:
        s.contract_round()
        assert cc.cc_get_round_sorted(s.ctx, 0) > 0.9 * want.stats[0][3]


# ---- tuning knobs ------------------------------------------------------------------------------

def test_emulated_tuning_knobs_keep_results(cc):
    """Every cc_tuning setting (round-0 form, workgroups per CU, round 0's key sets) gives the
    oracle's results; impossible settings are refused."""
    g = graphgen.Graph(1 << 15, *graphgen.rmat(4, 15, 8 << 15))
    want = oracle.run(g.n, g.src, g.dst, seed=3)
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=3, flags=TILED) as s:
        for r0 in (1, 2, 3):
            for bpc in (1, 4, 16):
                for ks in (1, 0):
                    s.set_tuning(round0=r0, blocks_per_cu=bpc, round0_key_sets=ks)
                    assert {k: s.tuning[k] for k in ("round0", "blocks_per_cu", "round0_key_sets")} == \
                        {"round0": r0, "blocks_per_cu": bpc, "round0_key_sets": ks}
                    r = s.run()
                    assert r == want.rounds
                    assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats]
                    np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)
        with pytest.raises(cc.CCError) as e:
            s.set_tuning(blocks_per_cu=65)
        assert e.value.status == cc.CC_E_ARG
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=3, flags=DIRECT) as s:   # workspace sized for direct
        with pytest.raises(cc.CCError) as e:
            s.set_tuning(round0=2)
        assert e.value.status == cc.CC_E_NOMEM
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), flags=cc.CC_EXPLICIT_PRIO) as s:
        with pytest.raises(cc.CCError) as e:
            s.set_tuning(round0=2)
        assert e.value.status == cc.CC_E_ARG


@pytest.mark.parametrize("mode", ["direct", "tiled", "rows"])
@pytest.mark.parametrize("layout", ["soa32", "packed"])
def test_emulated_bucket_sort_matches_oracle(cc, mode, layout):
    """Round 0's keys ordered by the sampled buckets instead of the radix passes: parents,
    edges, statistics and labels of every round equal the oracle's."""
    g = graphgen.Graph(6000, *graphgen.gnm(0x5152, 6000, 24011))
    check_solve(cc, g, 3, flags={"direct": DIRECT, "tiled": TILED, "rows": TILED}[mode], layout=layout,
                round0=3 if mode == "rows" else 0, tuning={"round0_sort": 2})


@pytest.mark.parametrize("key_sets", [1, 0])
def test_emulated_bucket_sort_heavy_keys(cc, key_sets):
    """A power-law graph whose round-0 keys repeat many times (most of all with the relabel's
    key sets off): heavy keys get buckets of their own; the results stay the oracle's."""
    g = graphgen.Graph(1 << 14, *graphgen.rmat(31, 14, 20 << 14))
    for flags in (TILED, DIRECT):
        check_solve(cc, g, 8, flags=flags, per_round=False,
                    tuning={"round0_sort": 2, "round0_key_sets": key_sets})
    star = graphgen.Graph(3000, np.zeros(40000, np.uint32), (np.arange(40000) % 2999 + 1).astype(np.uint32))
    check_solve(cc, star, 2, flags=TILED, tuning={"round0_sort": 2, "round0_key_sets": key_sets})


KERNEL_KNOBS = [("scatter_waves", (2, 4)), ("row_pairs", (2, 8)), ("relabel_pairs", (1, 4)),
                ("row_generation", (2, 8, -1))]


@pytest.mark.parametrize("r0", [2, 3])
def test_emulated_kernel_knobs_keep_results(cc, r0):
    """The kernel builds and launch shapes the tuner may pick (radix scatter waves, record
    pairs in flight in the tiled row passes, rows launched together) give the oracle's rounds,
    statistics and labels, round by round; 0 means the default and is reported resolved; values
    outside the built set are refused."""
    g = graphgen.Graph(1 << 15, *graphgen.rmat(9, 15, (8 << 15) + 777))
    for knob, values in KERNEL_KNOBS:
        for v in values:
            check_solve(cc, g, 6, flags=TILED, round0=r0, per_round=(knob == "row_pairs"), tuning={knob: v})
    with hipemu.Solver(g.n, dev(g.src), dev(g.dst), seed=3, flags=TILED) as s:
        s.set_tuning()
        t = s.tuning
        assert (t["scatter_waves"], t["row_pairs"], t["relabel_pairs"], t["row_generation"], t["round0_sort"]) == \
            (3, 4, 2, 1, 1)
        for knob, bad in (("scatter_waves", 5), ("row_pairs", 3), ("relabel_pairs", 8), ("row_generation", 9),
                          ("row_generation", -2), ("round0_sort", 3)):
            with pytest.raises(cc.CCError) as e:
                s.set_tuning(**{knob: bad})
            assert e.value.status == cc.CC_E_ARG
