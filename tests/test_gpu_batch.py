"""Batched mode: every graph of a batch, solved on the LDS path or the union path, in a
captured graph or eagerly, gets exactly the oracle's labels and round count for its own
seed (its solo result)."""
import numpy as np
import pytest

import graphgen
import oracle
from lcref import all_graph_adjacency, graph_records

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def lc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10727_amd as lc
    return lc


def make_batch(count, seed, log2_min=5, log2_max=13, **kw):
    return graphgen.batch_mix(seed=seed, count=count, log2_min=log2_min, log2_max=log2_max, **kw)


def check_batch(lc, b, labels, rounds):
    want_lab, want_rounds, _ = oracle.run_batch(b.voff, b.eoff, b.src, b.dst, b.seeds)
    np.testing.assert_array_equal(rounds, want_rounds)
    np.testing.assert_array_equal(labels.cpu().numpy().astype(np.uint32), want_lab)


def dev_arrays(b):
    return (torch.from_numpy(b.src.view(np.int32)).to(DEV), torch.from_numpy(b.dst.view(np.int32)).to(DEV))


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("use_graph", [1, 0])
@pytest.mark.parametrize("radix_form", [1, 2])
def test_batch_matches_oracle(lc, variant, use_graph, radix_form):
    b = make_batch(96, seed=11)
    s, d = dev_arrays(b)
    with lc.Batch(b.voff, b.eoff, b.seeds, s, d, small_variant=variant, use_graph=use_graph,
                  radix_form=radix_form) as bt:
        n_small, um = bt.split()
        if variant == 0:
            assert n_small == 0 and um == b.eoff[-1]
        else:
            assert n_small > 0
        lab, rounds = bt.run()
        check_batch(lc, b, lab, rounds)
        lab2, rounds2 = bt.run()     # replay of the captured graph
        check_batch(lc, b, lab2, rounds2)


@pytest.mark.parametrize("fill", [0x00, 0xA5, 0xFF])
def test_batch_ignores_workspace_contents(lc, fill):
    """The workspace arrives with arbitrary bytes (a torch.empty tensor): whatever it holds,
    including a round state full of ones, every run of the batch (the captured graph and its
    replays, union and LDS paths) gives the oracle's labels and round counts."""
    b = make_batch(64, seed=23)
    s, d = dev_arrays(b)
    with lc.Batch(b.voff, b.eoff, b.seeds, s, d, ws_fill=fill, small_variant=1) as bt:
        for _ in range(3):
            lab, rounds = bt.run()
            check_batch(lc, b, lab, rounds)


def test_batch_more_rounds_than_captured(lc):
    b = make_batch(40, seed=5, log2_min=8, log2_max=12, deg_lo=1.5, deg_hi=2.0)
    s, d = dev_arrays(b)
    with lc.Batch(b.voff, b.eoff, b.seeds, s, d, small_variant=0, rounds_per_graph=2) as bt:
        lab, rounds = bt.run()
        assert rounds.max() > 2
        check_batch(lc, b, lab, rounds)


@pytest.mark.parametrize("threads,blocks", [(256, 1), (512, 4)])
def test_batch_small_solver_shapes(lc, threads, blocks):
    b = make_batch(64, seed=3, log2_min=4, log2_max=10)
    s, d = dev_arrays(b)
    with lc.Batch(b.voff, b.eoff, b.seeds, s, d, small_variant=3, small_threads=threads,
                  small_blocks_per_cu=blocks) as bt:
        assert bt.split()[1] == 0          # everything on the LDS path
        lab, rounds = bt.run()
        check_batch(lc, b, lab, rounds)


def test_batch_of_all_graphs_on_five_vertices(lc):
    adj = all_graph_adjacency(5)
    src, dst, eoff = graph_records(adj)
    G = adj.shape[0]
    voff = np.arange(G + 1, dtype=np.int64) * 5
    seeds = np.array([graphgen.sm64(77 ^ g) for g in range(G)], dtype=np.uint64)
    b = graphgen.Batch(np.full(G, 5), np.diff(eoff), voff, eoff, seeds, src, dst)
    s, d = dev_arrays(b)
    for variant in (0, 1):
        with lc.Batch(voff, eoff, seeds, s, d, small_variant=variant) as bt:
            lab, rounds = bt.run()
            check_batch(lc, b, lab, rounds)


def test_batch_of_all_graphs_on_seven_vertices(lc):
    """Every labelled graph on 7 vertices (2^21 graphs, 22 M records) as one batch, on the
    union path and on the LDS path, each with its own seed: labels and round counts equal
    the oracle's graph by graph (the oracle itself equals the brute force on these graphs)."""
    adj = all_graph_adjacency(7)
    src, dst, eoff = graph_records(adj)
    G = adj.shape[0]
    voff = np.arange(G + 1, dtype=np.int64) * 7
    seeds = np.array([graphgen.sm64(91 ^ g) for g in range(G)], dtype=np.uint64)
    b = graphgen.Batch(np.full(G, 7), np.diff(eoff), voff, eoff, seeds, src, dst)
    s, d = dev_arrays(b)
    for variant in (0, 1):
        with lc.Batch(voff, eoff, seeds, s, d, small_variant=variant) as bt:
            assert bt.split()[0] == (G if variant else 0)
            lab, rounds = bt.run()
            check_batch(lc, b, lab, rounds)


def test_batch_degenerate_members(lc):
    specs = [("gnm", 0, 0, 1), ("gnm", 7, 0, 2), ("gnm", 1, 3, 3), ("gnm", 3000, 9000, 4), ("gnm", 2, 1, 5),
             ("rmat", 1 << 12, 8 << 12, 6)]
    b = graphgen.make_batch(specs)
    s, d = dev_arrays(b)
    for variant in (0, 2):
        with lc.Batch(b.voff, b.eoff, b.seeds, s, d, small_variant=variant) as bt:
            lab, rounds = bt.run()
            check_batch(lc, b, lab, rounds)


def test_batch_equals_solo_solves(lc):
    b = make_batch(12, seed=21, log2_min=9, log2_max=13)
    s, d = dev_arrays(b)
    with lc.Batch(b.voff, b.eoff, b.seeds, s, d) as bt:
        lab, rounds = bt.run()
        lab = lab.cpu().numpy()
    for j in range(b.count):
        g = b.graph(j)
        st = torch.from_numpy(g.src.view(np.int32)).to(DEV)
        dt = torch.from_numpy(g.dst.view(np.int32)).to(DEV)
        solo, r, _ = lc.solve(g.n, st, dt, seed=int(b.seeds[j]))
        np.testing.assert_array_equal(lab[b.voff[j]:b.voff[j + 1]], solo.cpu().numpy())
        assert r == rounds[j]


def test_batch_rejects_bad_ids(lc):
    specs = [("gnm", 100, 300, 1), ("gnm", 50, 100, 2)]
    b = graphgen.make_batch(specs)
    b.dst[310] = 50          # graph 1 has only 50 vertices
    s, d = dev_arrays(b)
    for variant in (0, 1):
        with lc.Batch(b.voff, b.eoff, b.seeds, s, d, small_variant=variant) as bt:
            with pytest.raises(lc.CCError) as e:
                bt.run()
            assert e.value.status == -2


def test_autotune_candidates_agree(lc):
    """Every candidate the autotuner times gives bit-identical labels (it raises otherwise),
    and the configuration it picks matches the oracle graph by graph."""
    from paper_1807_10727_amd import autotune
    b = make_batch(300, 0xA070, log2_min=4, log2_max=12)
    s, d = dev_arrays(b)
    with lc.Batch(b.voff, b.eoff, b.seeds, s, d) as bt:
        cfg, _, tried = autotune.tune(bt, repeats=1, cache=None)
        assert tried > 1
        assert bt.config == cfg or all(bt.config[k] == v for k, v in cfg.items())
        lab, rounds = bt.run()
        check_batch(lc, b, lab, rounds)
