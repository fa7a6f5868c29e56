"""Autotuners for the batched and the single-graph solves.

The knobs of ``cc_batch_config`` (grid size of the streaming kernels, the LDS solver's
size limits, workgroup size and persistence) and of ``cc_tuning`` (the form of round 0,
workgroups per compute unit, round 0's key sets, the radix scatter build, the record pairs
and launch generations of the tiled row passes, how round 0 sorts its keys) change only
speed: every candidate must
give bit-identical labels, and the tuner checks that.  Candidates are timed on the batch or
the graph itself, coordinate by coordinate, and the winner is cached as JSON under a key made
of the device (architecture, CU count) and the size class (log2 of the counts).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

DEFAULT_CACHE = os.environ.get("LC_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "lc_mi355x", "tune.json"))

SEARCH_SPACE = {
    "small_variant": [0, 1, 2, 3],
    "small_threads": [256, 512],
    "small_blocks_per_cu": [1, 2, 4],
    "blocks_per_cu": [4, 8, 16],
    "radix_form": [1, 2],              # the union's radix passes: count, scan and scatter a digit; one sweep
}


def device_key():
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "gpu").split(":")[0]
    return "%s:%dcu" % (arch, p.multi_processor_count)


def size_class(batch) -> str:
    m = int(batch.eoff[-1])
    return "G2^%d:M2^%d" % (max(0, round(math.log2(max(batch.G, 1)))), max(0, round(math.log2(max(m, 1)))))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_run(batch, repeats):
    import torch
    best = float("inf")
    digest = None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lab, _ = batch.run(with_rounds=False)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        if digest is None:
            digest = hashlib.sha1(lab.cpu().numpy().tobytes()).hexdigest()
    return best, digest


def tune(batch, repeats: int = 2, cache: str | None = DEFAULT_CACHE, log=None, space=None, rejected=None):
    """Pick the fastest configuration for `batch` (a paper_1807_10727_amd.Batch), apply it
    and return (config dict, seconds of the best run, number of candidates timed).  Every
    candidate must give the labels of the first one; a candidate that fails or does not is
    treated as in tune_solver (recorded in `rejected` when given, raised otherwise)."""
    key = "%s|%s" % (device_key(), size_class(batch))
    if cache:
        hit = _load(cache).get(key)
        if hit:
            batch.configure(**hit["config"])
            return hit["config"], hit["seconds"], 0
    space = space or SEARCH_SPACE
    cfg = dict(batch.config)
    cfg["use_graph"] = 1
    batch.configure(**cfg)
    best_t, ref = _time_run(batch, repeats)
    tried = 1
    for knob, values in space.items():
        for v in values:
            if v == cfg[knob]:
                continue
            cand = dict(cfg, **{knob: v})
            try:
                batch.configure(**cand)
            except Exception:          # e.g. an LDS variant larger than the device allows
                continue
            try:
                t, digest = _time_run(batch, repeats)
            except Exception as e:     # e.g. CCError from the library
                if rejected is None:
                    raise
                rejected.append((knob, v, "run failed: %s" % (e,)))
                continue
            tried += 1
            if digest != ref:
                if rejected is None:
                    raise RuntimeError("autotune candidate %r changed the labels" % (cand,))
                rejected.append((knob, v, "labels differ from the first candidate's"))
                continue
            if log:
                log("  tune %-22s %s -> %.2f ms" % (knob, v, t * 1e3))
            if t < best_t:
                best_t, cfg = t, cand
        batch.configure(**cfg)
    if cache:
        data = _load(cache)
        data[key] = {"config": cfg, "seconds": best_t}
        _store(cache, data)
    return cfg, best_t, tried


# ---- single-graph solve ------------------------------------------------------------------

SOLVER_SPACE = {
    "round0": [1, 2, 3],               # direct, tiled, tiled with the one-pass row partition
                                       # (the tiled forms where the context can take them)
    "blocks_per_cu": [4, 8, 16],
    "round0_key_sets": [1, 0],
    "scatter_waves": [3, 2, 4],
    "row_pairs": [4, 2, 8],            # the tiled forms only (no effect on a direct round 0)
    "relabel_pairs": [2, 1, 4],
    "row_generation": [1, 2, -1],
    "round0_sort": [1, 2],             # LSD radix passes, sampled buckets
    "tail": [1, 2, 3],                 # small rounds: launch sequences, one persistent launch
                                       # (1 or 2 workgroups per compute unit)
    "radix_form": [1, 2],              # radix passes: count, scan and scatter a digit; one sweep
}


ROW_KNOBS = ("row_pairs", "relabel_pairs", "row_generation")


def solver_size_class(solver) -> str:
    return "n2^%d:m2^%d" % (max(0, round(math.log2(max(solver.n, 1)))), max(0, round(math.log2(max(solver.m, 1)))))


def _time_solver(solver, seed, repeats):
    import torch
    best = float("inf")
    digest = None
    for i in range(repeats + 1):       # the first run warms the candidate (and its kernels)
        solver.reset(seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.run()
        lab = solver.labels()
        torch.cuda.synchronize()
        if i:
            best = min(best, time.perf_counter() - t0)
        if digest is None:
            digest = hashlib.sha1(lab.cpu().numpy().tobytes()).hexdigest()
    return best, digest


def tune_solver(solver, seed: int = 0, repeats: int = 1, cache: str | None = DEFAULT_CACHE, log=None, space=None,
                rejected=None):
    """Pick the fastest ``cc_tuning`` for `solver` (a paper_1807_10727_amd.Solver whose
    workspace was sized for its default form), apply it and return (tuning dict, seconds of
    the best solve, number of candidates timed).  Each candidate solves the graph with `seed`
    and must give the labels of the first one.  A candidate whose solve fails or gives other
    labels is never picked: with a list passed as `rejected` it is recorded there (knob,
    value, reason) and the walk goes on; without one its labels raise RuntimeError."""
    key = "solver|%s|%s" % (device_key(), solver_size_class(solver))
    if cache:
        hit = _load(cache).get(key)
        if hit:
            solver.set_tuning(**hit["config"])
            return hit["config"], hit["seconds"], 0
    space = space or SOLVER_SPACE
    cfg = dict(solver.tuning)
    solver.set_tuning(**cfg)
    best_t, ref = _time_solver(solver, seed, repeats)
    tried = 1
    for knob, values in space.items():
        if knob in ROW_KNOBS and cfg["round0"] == 1:
            continue                   # a direct round 0 has no row passes
        for v in values:
            if v == cfg[knob]:
                continue
            cand = dict(cfg, **{knob: v})
            try:
                solver.set_tuning(**cand)
            except Exception:          # e.g. a tiled round 0 the context cannot take
                continue
            try:
                t, digest = _time_solver(solver, seed, repeats)
            except Exception as e:     # e.g. CCError from the library
                if rejected is None:
                    raise
                rejected.append((knob, v, "solve failed: %s" % (e,)))
                continue
            tried += 1
            if digest != ref:
                if rejected is None:
                    raise RuntimeError("autotune candidate %r changed the labels" % (cand,))
                rejected.append((knob, v, "labels differ from the first candidate's"))
                continue
            if log:
                log("  tune %-16s %s -> %.3f ms" % (knob, v, t * 1e3))
            if t < best_t:
                best_t, cfg = t, cand
        solver.set_tuning(**cfg)
    if cache:
        data = _load(cache)
        data[key] = {"config": cfg, "seconds": best_t}
        _store(cache, data)
    return cfg, best_t, tried
