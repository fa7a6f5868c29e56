"""The autotuners' walks (host logic, no GPU): coordinate descent over the knobs, the row-pass
knobs skipped for a direct round 0, and candidates that fail or change the labels never
picked -- recorded when the caller asks, raised otherwise; for single solves and batches."""
import sys
import types

import numpy as np
import pytest

from paper_1807_10727_amd import autotune


class FakeSolver:
    """Stands in for paper_1807_10727_amd.Solver: the time of a solve is a function of the
    knobs, so the walk's choice is known in advance."""
    n, m = 1000, 5000

    def __init__(self, cost, fail=(), wrong=()):
        self.t = {"round0": 1, "tail": 1, "radix_form": 1, "row_pairs": 4}
        self.cost, self.fail, self.wrong = cost, fail, wrong
        self.clock = 0.0

    @property
    def tuning(self):
        return dict(self.t)

    def set_tuning(self, **kw):
        self.t.update(kw)

    def reset(self, seed):
        pass

    def run(self):
        if tuple(self.t.items()) in self.fail or any(self.t.get(k) == v for k, v in self.fail):
            raise RuntimeError("the device refused it")
        self.clock += self.cost(self.t)
        return 3

    def labels(self):
        bad = any(self.t.get(k) == v for k, v in self.wrong)
        return types.SimpleNamespace(cpu=lambda: types.SimpleNamespace(numpy=lambda: np.array([9 if bad else 5])))


@pytest.fixture()
def clocked(monkeypatch):
    """A torch stand-in (synchronize only) and a clock driven by the fake solver."""
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    monkeypatch.setattr(autotune, "device_key", lambda: "fake")
    state = {"solver": None}
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: state["solver"].clock if state["solver"] else 0.0)
    return state


SPACE = {"round0": [1, 2], "tail": [1, 2, 3], "radix_form": [1, 2], "row_pairs": [4, 8]}


def test_walk_picks_the_fastest_setting(clocked):
    s = FakeSolver(lambda t: 10.0 - 3 * (t["tail"] == 2) - 2 * (t["radix_form"] == 2) - (t["round0"] == 2))
    clocked["solver"] = s
    cfg, best, tried = autotune.tune_solver(s, cache=None, space=SPACE)
    assert cfg["tail"] == 2 and cfg["radix_form"] == 2 and cfg["round0"] == 2 and best == 4.0
    assert s.tuning == cfg


def test_direct_round0_skips_the_row_knobs(clocked):
    s = FakeSolver(lambda t: 5.0 - (t["row_pairs"] == 8))
    clocked["solver"] = s
    cfg, _, tried = autotune.tune_solver(s, cache=None, space={"row_pairs": [4, 8]})
    assert cfg["row_pairs"] == 4 and tried == 1


def test_failed_and_wrong_candidates_are_never_picked(clocked):
    # tail 3 would be fastest but its solve fails; radix_form 2 is fast but gives other labels
    s = FakeSolver(lambda t: 10.0 - 5 * (t["tail"] == 3) - 4 * (t["radix_form"] == 2) - (t["tail"] == 2),
                   fail=[("tail", 3)], wrong=[("radix_form", 2)])
    clocked["solver"] = s
    rejected = []
    cfg, best, _ = autotune.tune_solver(s, cache=None, space=SPACE, rejected=rejected)
    assert cfg["tail"] == 2 and cfg["radix_form"] == 1 and best == 9.0
    assert [(k, v) for k, v, _ in rejected] == [("tail", 3), ("radix_form", 2)]
    assert "failed" in rejected[0][2] and "labels" in rejected[1][2]
    # without a list to record them in, the walk stops at the first such candidate
    s2 = FakeSolver(lambda t: 1.0, wrong=[("radix_form", 2)])
    clocked["solver"] = s2
    with pytest.raises(RuntimeError):
        autotune.tune_solver(s2, cache=None, space={"radix_form": [1, 2]})


class FakeBatch:
    """Stands in for paper_1807_10727_amd.Batch: run() advances the clock by the cost of the
    configuration; one setting fails, another gives other labels."""

    def __init__(self, cost, fail=(), wrong=()):
        self.c = {"small_variant": 2, "blocks_per_cu": 8, "radix_form": 1, "use_graph": 1}
        self.cost, self.fail, self.wrong = cost, fail, wrong
        self.clock = 0.0
        self.n_total = 4

    @property
    def config(self):
        return dict(self.c)

    def configure(self, **kw):
        self.c.update(kw)

    def run(self, with_rounds=True):
        if any(self.c.get(k) == v for k, v in self.fail):
            raise RuntimeError("the device refused it")
        self.clock += self.cost(self.c)
        bad = any(self.c.get(k) == v for k, v in self.wrong)
        return types.SimpleNamespace(cpu=lambda: types.SimpleNamespace(numpy=lambda: np.array([9 if bad else 5]))), None


def test_batch_walk_skips_failed_and_wrong_candidates(clocked, monkeypatch):
    monkeypatch.setattr(autotune, "size_class", lambda b: "fake")
    bt = FakeBatch(lambda c: 10.0 - 5 * (c["small_variant"] == 3) - 3 * (c["radix_form"] == 2) - (c["blocks_per_cu"] == 16),
                   fail=[("small_variant", 3)], wrong=[("radix_form", 2)])
    clocked["solver"] = bt
    rejected = []
    cfg, best, _ = autotune.tune(bt, repeats=1, cache=None, rejected=rejected,
                                 space={"small_variant": [2, 3], "blocks_per_cu": [8, 16], "radix_form": [1, 2]})
    assert cfg["small_variant"] == 2 and cfg["blocks_per_cu"] == 16 and cfg["radix_form"] == 1 and best == 9.0
    assert [(k, v) for k, v, _ in rejected] == [("small_variant", 3), ("radix_form", 2)]
