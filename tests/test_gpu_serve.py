"""Serving: every request's labels equal the oracle's (its solo result) whether it runs
alone or in a mix of overlapping requests, under memory pressure, with cancellations and
with bad input in a neighbouring request."""
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def lc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10727_amd as lc
    return lc


def request_graphs(count, seed, log2_min=6, log2_max=15):
    tr = graphgen.request_trace(seed, count, rate=1000.0, log2_min=log2_min, log2_max=log2_max, deg_lo=2.0,
                                deg_hi=8.0, rmat_ef=8)
    out = []
    for r in tr:
        g = r.graph()
        out.append((g, r.seed, torch.from_numpy(g.src.view(np.int32)).to(DEV),
                    torch.from_numpy(g.dst.view(np.int32)).to(DEV)))
    return out


def expect(g, seed):
    return oracle.run(g.n, g.src, g.dst, seed=seed)


def test_mix_equals_alone_and_oracle(lc):
    reqs = request_graphs(40, seed=1)
    torch.cuda.synchronize()
    with lc.Server(1 << 30, n_slots=4, small_variant=1, max_small_per_launch=16) as srv:
        # alone: one request at a time
        alone = []
        for g, sd, s, d in reqs:
            rid, lab = srv.submit(g.n, s, d, sd)
            res = []
            while not res:
                res = srv.wait(5.0)
            assert res[0]["id"] == rid and res[0]["status"] == 0
            alone.append((lab.cpu().numpy().copy(), res[0]["rounds"]))
        # mix: all submitted with small gaps, overlapping on the device
        labs = {}
        for i, (g, sd, s, d) in enumerate(reqs):
            rid, lab = srv.submit(g.n, s, d, sd)
            labs[rid] = (i, lab)
            if i % 7 == 0:
                time.sleep(0.002)
        results = srv.drain()
        info = srv.info()
    assert len(results) == len(reqs)
    assert any(r["small_path"] for r in results) and not all(r["small_path"] for r in results)
    for r in results:
        assert r["status"] == 0
        i, lab = labs[r["id"]]
        g, sd, _, _ = reqs[i]
        got = lab.cpu().numpy()
        want = expect(g, sd)
        np.testing.assert_array_equal(got.astype(np.uint32), want.labels)
        assert r["rounds"] == want.rounds
        np.testing.assert_array_equal(got, alone[i][0])
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    assert info["pending"] == 0 and info["active"] == 0


def test_tiny_budget_defers_and_completes(lc):
    reqs = request_graphs(12, seed=2, log2_min=12, log2_max=15)
    torch.cuda.synchronize()
    budget = 8 << 20
    with lc.Server(budget, n_slots=8, small_variant=0) as srv:
        labs = {}
        for i, (g, sd, s, d) in enumerate(reqs):
            rid, lab = srv.submit(g.n, s, d, sd)
            labs[rid] = (i, lab)
        results = srv.drain()
        info = srv.info()
    assert len(results) == len(reqs) and info["peak_bytes"] <= budget
    for r in results:
        assert r["status"] == 0
        i, lab = labs[r["id"]]
        g, sd, _, _ = reqs[i]
        np.testing.assert_array_equal(lab.cpu().numpy().astype(np.uint32), expect(g, sd).labels)


def test_over_budget_request_refused(lc):
    g = graphgen.Graph(1 << 16, *graphgen.gnm(3, 1 << 16, 1 << 18))
    s = torch.from_numpy(g.src.view(np.int32)).to(DEV)
    d = torch.from_numpy(g.dst.view(np.int32)).to(DEV)
    with lc.Server(1 << 20, n_slots=2, small_variant=0) as srv:
        with pytest.raises(lc.CCError) as e:
            srv.submit(g.n, s, d, 1)
        assert e.value.status == -6


def test_cancel_and_bad_input_leave_others_intact(lc):
    reqs = request_graphs(16, seed=3)
    bad = graphgen.Graph(50, np.array([1, 2, 60], np.uint32), np.array([3, 4, 5], np.uint32))
    bad_big = graphgen.Graph(5000, *graphgen.gnm(4, 5000, 20000))
    bad_big.dst[123] = 7000
    torch.cuda.synchronize()
    with lc.Server(1 << 30, n_slots=2, small_variant=1) as srv:
        labs = {}
        for i, (g, sd, s, d) in enumerate(reqs):
            rid, lab = srv.submit(g.n, s, d, sd)
            labs[rid] = (i, lab)
        bad_ids = set()
        for bg in (bad, bad_big):
            rid, _ = srv.submit(bg.n, torch.from_numpy(bg.src.view(np.int32)).to(DEV),
                                torch.from_numpy(bg.dst.view(np.int32)).to(DEV), 9)
            bad_ids.add(rid)
        # cancel the last two regular requests if they are still waiting
        cancelled = set()
        for rid in list(labs)[-2:]:
            try:
                srv.cancel(rid)
                cancelled.add(rid)
            except lc.CCError:
                pass   # already completed
        results = srv.drain()
    assert len(results) == len(reqs) + 2
    for r in results:
        if r["id"] in bad_ids:
            assert r["status"] == -2
            continue
        if r["id"] in cancelled and r["status"] != 0:
            assert r["status"] == -5
            continue
        assert r["status"] == 0
        i, lab = labs[r["id"]]
        g, sd, _, _ = reqs[i]
        np.testing.assert_array_equal(lab.cpu().numpy().astype(np.uint32), expect(g, sd).labels)


def test_degenerate_requests(lc):
    cases = [graphgen.Graph(0, np.zeros(0, np.uint32), np.zeros(0, np.uint32)),
             graphgen.Graph(9, np.zeros(0, np.uint32), np.zeros(0, np.uint32)),
             graphgen.Graph(4, np.array([1, 1], np.uint32), np.array([1, 1], np.uint32)),
             graphgen.Graph(3000, np.array([5], np.uint32), np.array([2999], np.uint32))]
    with lc.Server(1 << 28, n_slots=2, small_variant=1) as srv:
        labs = {}
        for i, g in enumerate(cases):
            s = torch.from_numpy(g.src.view(np.int32)).to(DEV)
            d = torch.from_numpy(g.dst.view(np.int32)).to(DEV)
            rid, lab = srv.submit(g.n, s, d, 5)
            labs[rid] = (i, lab)
        results = srv.drain()
    assert len(results) == len(cases)
    for r in results:
        assert r["status"] == 0
        i, lab = labs[r["id"]]
        g = cases[i]
        want = expect(g, 5)
        np.testing.assert_array_equal(lab.cpu().numpy().astype(np.uint32), want.labels)
        assert r["rounds"] == want.rounds


@pytest.mark.parametrize("cohort_max", [4, 64])
def test_cohorts_equal_oracle(lc, cohort_max):
    """Large requests fused into cohorts (one disjoint union, one launch sequence a round for
    all of them): every request's labels and rounds are the oracle's, a request with an id
    out of range fails alone, and a cancelled one ends cancelled."""
    reqs = request_graphs(48, seed=7, log2_min=9, log2_max=16)
    bad_g = graphgen.Graph(3000, *graphgen.gnm(77, 3000, 9000))
    bad_dst = bad_g.dst.astype(np.int64)
    bad_dst[11] = 3000 + 9
    bad = (bad_g, 123, torch.from_numpy(bad_g.src.view(np.int32)).to(DEV),
           torch.from_numpy(bad_dst.astype(np.int32)).to(DEV))
    reqs.insert(20, bad)
    torch.cuda.synchronize()
    with lc.Server(2 << 30, n_slots=2, small_variant=1, max_small_per_launch=16, cohort_max=cohort_max,
                   cohort_max_vertices=1 << 16) as srv:
        srv.pause()   # the whole burst waits, then starts as cohorts
        labs = {}
        for i, (g, sd, s, d) in enumerate(reqs):
            rid, lab = srv.submit(g.n, s, d, sd)
            labs[rid] = (i, lab)
        cancel_id = max(labs)
        try:
            srv.cancel(cancel_id)
        except lc.CCError:
            pass   # already completed
        srv.pause(False)
        res = srv.drain()
    assert len(res) == len(reqs)
    fused = 0
    for x in res:
        i, lab = labs[x["id"]]
        if i == 20:
            assert x["status"] == -2   # CC_E_INPUT
            continue
        if x["id"] == cancel_id and x["status"] != 0:
            assert x["status"] == -5   # CC_E_STATE
            continue
        g, sd = reqs[i][0], reqs[i][1]
        want = expect(g, sd)
        assert x["status"] == 0 and x["rounds"] == want.rounds, (i, x)
        np.testing.assert_array_equal(lab.cpu().numpy().view(np.uint32), want.labels)
        fused += x["cohort"] > 1
    assert fused > 0
