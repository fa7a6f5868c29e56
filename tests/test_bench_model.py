"""The byte model bench.py divides by kernel time (host logic, no GPU), against values worked
out by hand from its definition: per round, with N the nodes addressed (n0 in round 0), M the
records read, S the survivors, M' the distinct edges out,
    a2 = 8M + 4N, a3 = 8M + 8N, a4 = 8M + 4N + 8S, a5 = 8S + 8M', a6 = 4N, a7 = 4N,
plus 4 n0 for the labels; the duplicate drop counts its survivors and edges once, however many
passes run, and the tiled round 0's partition moves no algorithmic byte."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402

# (round, n_active, m_in, m_survive, m_out, n_finalised)
TOY = [(0, 5, 10, 6, 3, 1), (1, 4, 3, 2, 1, 0)]


def test_steps_of_a_toy_solve():
    # worked by hand for n0 = 8: round 0 has N = 8, M = 10, S = 6, M' = 3; round 1 has
    # N = 4, M = 3, S = 2, M' = 1
    b = bench.step_bytes(TOY, 8)
    assert b == {"a2_one_hop": 112 + 40, "a3_two_hop": 144 + 56, "a4_relabel": 160 + 56,
                 "a5_dedup": 72 + 24, "a6_nodes": 32 + 16, "a7_labels": 32 + 16 + 32}
    assert bench.job_alg_bytes(TOY, 8) == 792


def test_rounds_inside_a_captured_tail():
    b = bench.step_bytes(TOY, 8, in_graph=[0, 1])
    assert b["tail"] == 40 + 56 + 56 + 24 + 16 + 16
    assert b["a5_dedup"] == 72 and b["a7_labels"] == 32 + 32


def test_round0_dedup_of_the_full_size_graphs():
    # G(2^24, 2^27) + paths at the bench seed: 129,152,105 survivors, 121,755,054 edges out
    er = (0, 26777215, 144207728, 129152105, 121755054, 0)
    assert bench.step_bytes([er], 26777216)["a5_dedup"] == 2_007_257_272
    # R-MAT scale 26 at the bench seed (tests/golden/rmat26_seed_c0ffee01.json, round 0)
    rm = (0, 32233922, 1073741824, 846500557, 1883670, 11443)
    b = bench.step_bytes([rm], 1 << 26)
    assert b["a5_dedup"] == 6_787_073_816
    assert b["a2_one_hop"] == 8_858_370_048           # 8 * 2^30 + 4 * 2^26
    assert b["a4_relabel"] == 15_630_374_504          # 8 * 2^30 + 4 * 2^26 + 8 * 846,500,557


def test_partition_and_tails_are_not_steps_of_the_method():
    assert bench.FAMILY_STEP["part_b_scatter"] == bench.FAMILY_STEP["part_rows_scatter"] == "partition"
    from paper_1807_10727_amd import _cc
    assert set(_cc.cc_kernel_family_names()) <= set(bench.FAMILY_STEP)   # every kernel is placed
    assert bench.FAMILY_STEP["sort_scatter"] == bench.FAMILY_STEP["hash_dedup"] == "a5_dedup"
    assert "partition" not in bench.step_bytes(TOY, 8)
