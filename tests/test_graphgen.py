"""Seeded input generators: determinism, shapes and value ranges."""
import numpy as np

import graphgen


def test_gnm_deterministic_and_in_range():
    a = graphgen.gnm(5, 1000, 5000)
    b = graphgen.gnm(5, 1000, 5000)
    c = graphgen.gnm(6, 1000, 5000)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])
    assert a[0].max() < 1000 and a[1].max() < 1000
    # uniform endpoints: every id is hit about 10 times
    counts = np.bincount(np.concatenate(a), minlength=1000)
    assert counts.min() > 0 and abs(counts.mean() - 10) < 1e-9


def test_paths_are_disjoint_paths():
    s, d = graphgen.paths(3, 7, 50, id_base=100)
    assert s.shape[0] == 7 * 49
    ids = np.concatenate([s, d])
    assert ids.min() >= 100 and ids.max() < 100 + 350
    deg = np.bincount(ids - 100, minlength=350)
    assert np.count_nonzero(deg == 1) == 14 and np.count_nonzero(deg == 2) == 350 - 14


def test_rmat_shape_and_skew():
    s, d = graphgen.rmat(9, 12, 8 << 12)
    assert s.max() < 4096 and d.max() < 4096
    deg = np.bincount(np.concatenate([s, d]), minlength=4096)
    assert deg.max() > 20 * deg.mean()           # power-law hubs
    assert np.count_nonzero(deg == 0) > 0        # and many untouched ids


def test_workloads_sizes():
    g = graphgen.workload_small()
    assert g.n == 65536 and g.m == 262144
    g = graphgen.workload_er_paths(shrink=64)
    assert g.n == (1 << 24) // 64 + (10000 // 64) * 1000
    assert g.m == (1 << 27) // 64 + (10000 // 64) * 999


def test_batch_mix_layout():
    specs = graphgen.batch_specs(1, 16, log2_min=6, log2_max=10)
    b = graphgen.make_batch(specs)
    assert b.count == 16 and b.eoff[-1] == b.src.shape[0]
    for j in range(16):
        g = b.graph(j)
        assert g.m == 0 or g.src.max() < g.n
    assert b.n[1::2].tolist() == [s[1] for s in specs[1::2]]


def test_request_trace_poisson():
    tr = graphgen.request_trace(4, 2000, rate=100.0, log2_min=6, log2_max=12)
    t = np.array([r.arrival for r in tr])
    gaps = np.diff(t)
    assert np.all(gaps > 0) and abs(gaps.mean() - 0.01) < 0.001
