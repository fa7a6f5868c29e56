"""Randomised parity of the emulated device code with the oracle (CPU only).

Hypothesis draws the graph (size, density, a power-law or uniform mix, repeated records,
loops, isolated ids), the seed, the input layout, the label rule (with MergeToLarge's
parameters) and the solver's knobs (round-0
form, key sets, the order of round 0's keys, kernel builds, grid size, the persistent launch of
the small rounds, the one-sweep radix passes); every draw must give
the oracle's round count, statistics and labels.  The draws are derandomised, so a failure
is reproducible, and sized so that the whole test takes about a minute.
"""
import numpy as np
import pytest

import graphgen
import oracle

hypothesis = pytest.importorskip("hypothesis")
hipemu = pytest.importorskip("hipemu")
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402

from test_emu_parity import DIRECT, RULES, TILED, inputs  # noqa: E402

MTL = 1 << 9   # CC_MERGE_TO_LARGE (include/cc.h)


@st.composite
def graphs(draw):
    n = draw(st.integers(1, 3000))
    m = draw(st.integers(0, 4 * n + 50))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    kind = draw(st.sampled_from(["gnm", "rmat", "paths"]))
    if m == 0:
        src = dst = np.zeros(0, np.uint32)
    elif kind == "gnm":
        src, dst = graphgen.gnm(seed, n, m)
    elif kind == "rmat":
        scale = max(1, int(np.ceil(np.log2(n))))
        src, dst = graphgen.rmat(seed, scale, m)
        src, dst = src % np.uint32(n), dst % np.uint32(n)
    else:
        g = graphgen.er_with_paths(seed, n, m // 2, max(1, n // 50), min(50, n))
        return g
    # repeats and loops on top
    extra = draw(st.integers(0, 20))
    if extra and src.size:
        pick = np.arange(extra) % src.size
        src = np.concatenate([src, src[pick], dst[pick[:extra // 2]]]).astype(np.uint32)
        dst = np.concatenate([dst, dst[pick], dst[pick[:extra // 2]]]).astype(np.uint32)
    return graphgen.Graph(n, src, dst)


KNOBS = st.fixed_dictionaries({
    "round0": st.sampled_from([1, 2, 3]),
    "round0_key_sets": st.sampled_from([0, 1]),
    "round0_sort": st.sampled_from([1, 2]),
    "scatter_waves": st.sampled_from([2, 3, 4]),
    "row_pairs": st.sampled_from([2, 4, 8]),
    "relabel_pairs": st.sampled_from([1, 2, 4]),
    "row_generation": st.sampled_from([-1, 1, 2]),
    "blocks_per_cu": st.sampled_from([1, 8]),
    "tail": st.sampled_from([1, 2, 4]),
    "radix_form": st.sampled_from([1, 2]),
})


@settings(max_examples=100, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(g=graphs(), seed=st.integers(0, 2 ** 64 - 1), layout=st.sampled_from(["soa32", "soa64", "packed"]),
       rule=st.sampled_from(["local", "local", "tree", "one_hop", "merge_to_large"]), knobs=KNOBS,
       alphas=st.lists(st.integers(1, 6), min_size=1, max_size=3))
def test_random_solves_match_the_oracle(g, seed, layout, rule, knobs, alphas):
    mtl = rule == "merge_to_large"
    want = oracle.run(g.n, g.src, g.dst, seed=seed, variant=rule, alphas=alphas if mtl else None)
    s_, d_ = inputs(g, layout)
    # every knob setting needs the tiled workspace; the context sizes for it with CC_ROUND0_TILED
    flags = (TILED if g.n > 0 else DIRECT) | (MTL if mtl else RULES[rule])
    with hipemu.Solver(g.n, s_, d_, seed=seed, flags=flags) as s:
        if g.n > 0:
            s.set_tuning(**knobs)
        if mtl:
            s.set_merge_to_large(alphas)
        r = s.run()
        assert r == want.rounds
        assert [tuple(x) for x in s.stats(r)] == [tuple(x) for x in want.stats]
        np.testing.assert_array_equal(s.labels().astype(np.uint32), want.labels)


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(seed=st.integers(0, 2 ** 32 - 1), count=st.integers(1, 24), log2_max=st.integers(2, 12),
       small_variant=st.sampled_from([0, 1, 2, 3]), small_threads=st.sampled_from([256, 512]),
       use_graph=st.sampled_from([0, 1]), blocks_per_cu=st.sampled_from([1, 8]), fill=st.sampled_from([0x00, 0xA5]),
       radix_form=st.sampled_from([1, 2]))
def test_random_batches_match_the_oracle(seed, count, log2_max, small_variant, small_threads, use_graph,
                                         blocks_per_cu, fill, radix_form):
    """Random batches (sizes, the LDS solver's limits and workgroup size, captured or eager
    rounds, grid size, workspace contents, the form of the union's radix passes): every graph's
    labels and rounds are the oracle's, run twice on the same batch."""
    b = graphgen.batch_mix(seed=seed, count=count, log2_min=1, log2_max=log2_max)
    want_lab, want_rounds, _ = oracle.run_batch(b.voff, b.eoff, b.src, b.dst, b.seeds)
    with hipemu.Batch(b.voff, b.eoff, b.seeds, b.src, b.dst, ws_fill=fill, small_variant=small_variant,
                      small_threads=small_threads, use_graph=use_graph, blocks_per_cu=blocks_per_cu,
                      radix_form=radix_form) as bt:
        for _ in range(2):
            lab, rounds = bt.run()
            np.testing.assert_array_equal(rounds, want_rounds)
            np.testing.assert_array_equal(lab.astype(np.uint32), want_lab)
