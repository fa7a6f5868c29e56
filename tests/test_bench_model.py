"""The byte model bench.py divides by kernel time (host logic, no GPU).

The statistics below are one solve of the bench graph as the library reported them
(cc_round_stats: round, n_active, m_in, m_survive, m_out, n_finalised; m_sorted), with the
radix passes each round would run as the library counted them on the device.  bench.py must
derive the same passes from the statistics alone: keys carry 2 ceil(log2 L) bits, L = the
round's labels = the next round's nodes plus the labels finalised."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402

STATS = [(0, 26777215, 144207728, 129152105, 121755054, 0), (1, 3773340, 121755054, 57677051, 1106428, 0),
         (2, 1114120, 1106428, 363522, 363514, 0), (3, 373515, 363514, 116857, 116857, 1),
         (4, 126857, 116857, 34695, 34695, 0), (5, 44695, 34695, 6659, 6659, 4092),
         (6, 12567, 6659, 22, 22, 5886), (7, 44, 22, 0, 0, 22)]
SORTED = [129152105, 1473052, 363514, 116857, 34695, 6659, 22, 0]
DEVICE_PASSES = [6, 6, 5, 5, 4, 4, 4, 2]


def test_radix_passes_follow_the_labels():
    fb = bench.family_bytes(STATS, 26777216, tiled=True, loops=0, sorted_keys=SORTED)
    # round 0 sorts; rounds 1.. (at most 2^22 keys each, round 1 from 121 M records) hash
    sorted_rounds = [i for i, st in enumerate(STATS) if st[0] == 0 or SORTED[i] > bench.HASH_MAX_RECORDS]
    assert sorted_rounds == [0]
    assert fb["sort_scatter"] == sum(16 * SORTED[i] * DEVICE_PASSES[i] for i in sorted_rounds)
    assert fb["sort_hist"] == sum(8 * SORTED[i] * DEVICE_PASSES[i] for i in sorted_rounds)
    assert fb["hash_dedup"] == sum(8 * SORTED[i] + 32 * STATS[i][4] for i in range(1, len(STATS)))


def test_round0_tiled_families():
    fb = bench.family_bytes(STATS[:1] + STATS[1:2], 26777216, tiled=True, loops=0, sorted_keys=SORTED[:2])
    T = 2 * STATS[0][2]
    assert fb["part_b_scatter"] == 16 * T
    assert fb["min2_tiled"] == 8 * T + 8 * 26777216
    assert fb["unique"] == 16 * SORTED[0] + 8 * STATS[0][4]
    assert fb["hash_dedup"] == 8 * SORTED[1] + 32 * STATS[1][4]


def test_families_outside_captured_tails():
    # a captured tail holds rounds >= 1 of at most 2^22 records: they hash, so the radix and
    # unique families and round 0's never run there; the per-round families do
    for fam in ("sort_scatter", "sort_hist", "sort_scan", "unique", "min2_tiled", "part_b_scatter",
                "relabel_round0"):
        assert bench.tail_free(fam)
    for fam in ("min1", "min2", "relabel", "hash_dedup", "round_begin", "map", "nodes"):
        assert not bench.tail_free(fam)
