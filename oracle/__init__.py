"""CPU oracle for LocalContraction -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never loads it and it never loads the GPU library.

``lc_oracle.c`` holds the plain, step-by-step algorithm (Section 3, paragraph
"LocalContraction"; closed neighbourhoods from Section 2; the contraction step from the
proof of the lemma in Section 3; isolated nodes are final as in Section 6).  This module
only compiles it and marshals arrays.

Parity status of its functions (what pins each one; the tests hold the pins):
  * ``priority``     -- pinned to the published definitions of SplitMix64 and MurmurHash3's
                        finaliser (known output values) and to an independent numpy version.
  * ``run`` parents  -- pinned by brute force from the definition (closed two-hop reachability
                        then argmin) on every labelled graph with up to 7 vertices, by all
                        orderings of small graphs, and by hand-worked fixtures.
  * ``run`` labels   -- pinned as a partition to scipy's connected_components and to a
                        textbook union-find; raw label values under the hash are pinned only
                        by the frozen priority specification (the paper fixes no values).
  * ``run`` stats    -- pinned by recount from the brute force on small graphs and by the
                        paper's invariants (component count preserved, path lower bound).
  * ``run(variant="tree")`` -- TreeContraction (Section 3): pinned by a brute force that walks
                        v, f(v), f(f(v)), ... to the terminal 2-cycle (Lemma "cycle") on every
                        labelled graph with up to 6 vertices, by the lemma's invariants (every
                        merged class has at least two nodes, classes are connected, two
                        nodes share a class iff their terminal cycles agree), and by partition.
  * ``run(variant="one_hop")`` -- closed one-hop labels: pinned by the same brute force with
                        one hop, and by partition.
  * ``run(finish_edges=T)`` -- union-find finish (Section 6): pinned by the per-round results
                        being those of the plain run up to the switch, and by labels equal to
                        the smallest name of each remaining component (recomputed with scipy).
  * ``run(variant="merge_to_large")`` -- MergeToLarge (Section 5): pinned by an independent
                        step-by-step Python restatement (sets and dictionaries) on every
                        graph with up to 5 vertices and on random graphs, by the step's own
                        invariants (each node within distance 2 of a large node joins the
                        class of the best one; the others keep theirs), by the reduction to
                        LocalContraction when no node can be large, and by partition.
  * ``components_min_id`` -- textbook union-find (smallest id of each component): pinned to
                        scipy's connected_components and to an independent Python union-find on
                        random, power-law, path, edgeless and one-vertex graphs, with isolated
                        ids at both ends, loops, repeats, and a merge order whose kept root is
                        not the component's smallest id.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lc_oracle.c")
_LIB = os.path.join(_HERE, "liblcoracle.so")
_lib = None

NOT_A_NODE = 0xFFFFFFFF


class RoundStats(ctypes.Structure):
    _fields_ = [("round", ctypes.c_int32), ("pad_", ctypes.c_int32), ("n_active", ctypes.c_int64),
                ("m_in", ctypes.c_int64), ("m_survive", ctypes.c_int64), ("m_out", ctypes.c_int64),
                ("n_finalised", ctypes.c_int64)]

    def as_tuple(self):
        return (self.round, self.n_active, self.m_in, self.m_survive, self.m_out, self.n_finalised)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.lco_sm64.restype = ctypes.c_uint64
        lib.lco_sm64.argtypes = [ctypes.c_uint64]
        lib.lco_fmix32.restype = ctypes.c_uint32
        lib.lco_fmix32.argtypes = [ctypes.c_uint32]
        lib.lco_priority.restype = ctypes.c_uint32
        lib.lco_priority.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32]
        lib.lco_run.restype = ctypes.c_int32
        lib.lco_run.argtypes = [ctypes.c_int64, ctypes.c_int64, u32p, u32p, ctypes.c_uint64, u32p, ctypes.c_int32,
                                ctypes.c_int32, u32p, ctypes.POINTER(RoundStats), ctypes.c_int32, u32p,
                                ctypes.c_int32]
        lib.lco_run_variant.restype = ctypes.c_int32
        lib.lco_run_variant.argtypes = lib.lco_run.argtypes + [ctypes.c_int32, ctypes.c_int64,
                                                               ctypes.POINTER(ctypes.c_int32)]
        lib.lco_run_full.restype = ctypes.c_int32
        lib.lco_run_full.argtypes = lib.lco_run_variant.argtypes + [u32p, u32p, ctypes.c_int32, i64p, ctypes.c_int32]
        lib.lco_run_batch.restype = ctypes.c_int32
        lib.lco_run_batch.argtypes = [ctypes.c_int64, i64p, i64p, u32p, u32p, ctypes.POINTER(ctypes.c_uint64), u32p,
                                      ctypes.POINTER(ctypes.c_int32), u32p, ctypes.c_int32]
        lib.lco_components_min_id.restype = ctypes.c_int32
        lib.lco_components_min_id.argtypes = [ctypes.c_int64, ctypes.c_int64, u32p, u32p, u32p]
        _lib = lib
    return _lib


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


def sm64(x: int) -> int:
    return int(_load().lco_sm64(x & 0xFFFFFFFFFFFFFFFF))


def fmix32(x: int) -> int:
    return int(_load().lco_fmix32(x & 0xFFFFFFFF))


def priority(seed: int, rnd: int, name: int) -> int:
    return int(_load().lco_priority(seed & 0xFFFFFFFFFFFFFFFF, rnd, name & 0xFFFFFFFF))


VARIANTS = {"local": 0, "tree": 1, "one_hop": 2, "merge_to_large": 3}


@dataclass
class Result:
    labels: np.ndarray                 # uint32 [n0]
    rounds: int
    stats: list = field(default_factory=list)   # tuples (round, n_active, m_in, m_survive, m_out, n_finalised)
    parents: np.ndarray | None = None  # uint32 [min(rounds, cap), n0], NOT_A_NODE off V_r
    finished: bool = False             # the union-find finish ran
    m1: np.ndarray | None = None       # uint32 [min(rounds, cap), n0] one-hop minima, 0xFFFFFFFF off V_r
    l: np.ndarray | None = None        # uint32 [min(rounds, cap), n0] two-hop minima


def run(n: int, src, dst, seed: int = 0, explicit_prio=None, max_rounds: int = 0,
        record_parents: bool = False, parents_cap: int = 64, stats_cap: int = 256, variant: str = "local",
        finish_edges: int = 0, record_minima: bool = False, minima_cap: int = 16, alphas=None) -> Result:
    """Run the oracle.  `explicit_prio` is an optional [rows, n] table of priorities (phase r
    uses row min(r, rows-1)).  `variant`: "local" (LocalContraction), "tree"
    (TreeContraction), "one_hop" or "merge_to_large" (LocalContraction phases, each followed
    by a MergeToLarge step with parameter alphas[min(i, len - 1)] in phase i; default: one
    alpha, default_alpha(n)); `finish_edges` > 0 finishes with union-find once a phase
    leaves at most that many edges."""
    lib = _load()
    src = _u32(src)
    dst = _u32(dst)
    m = int(src.shape[0])
    labels = np.empty(max(n, 1), dtype=np.uint32)
    stats = (RoundStats * stats_cap)()
    par = np.empty((parents_cap, max(n, 1)), dtype=np.uint32) if record_parents else None
    ep = None
    rows = 0
    if explicit_prio is not None:
        ep = np.ascontiguousarray(np.atleast_2d(explicit_prio), dtype=np.uint32)
        assert ep.shape[1] == n
        rows = ep.shape[0]
    fin = ctypes.c_int32(0)
    m1 = np.empty((minima_cap, max(n, 1)), dtype=np.uint32) if record_minima else None
    l2 = np.empty((minima_cap, max(n, 1)), dtype=np.uint32) if record_minima else None
    al = None
    if variant == "merge_to_large":
        al = np.ascontiguousarray([default_alpha(n)] if alphas is None else alphas, dtype=np.int64)
    r = lib.lco_run_full(n, m, _ptr(src, ctypes.c_uint32), _ptr(dst, ctypes.c_uint32), seed & 0xFFFFFFFFFFFFFFFF,
                         _ptr(ep, ctypes.c_uint32), rows, max_rounds, _ptr(labels, ctypes.c_uint32), stats,
                         stats_cap, _ptr(par, ctypes.c_uint32), parents_cap if record_parents else 0,
                         VARIANTS[variant], int(finish_edges), ctypes.byref(fin), _ptr(m1, ctypes.c_uint32),
                         _ptr(l2, ctypes.c_uint32), minima_cap if record_minima else 0, _ptr(al, ctypes.c_int64),
                         0 if al is None else int(al.shape[0]))
    if r < 0:
        raise ValueError("oracle rejected the input (ids out of range or out of memory)")
    res = Result(labels[:n], int(r), [stats[i].as_tuple() for i in range(min(r, stats_cap))],
                 finished=bool(fin.value))
    if record_parents:
        res.parents = par[:min(r, parents_cap), :n]
    if record_minima:
        res.m1 = m1[:min(r, minima_cap), :n]
        res.l = l2[:min(r, minima_cap), :n]
    return res


def default_alpha(n: int) -> int:
    """MergeToLarge parameter used when none is given: max(2, ceil(ln n))."""
    import math
    return max(2, int(math.ceil(math.log(max(n, 2)))))


def run_batch(voff, eoff, src, dst, seeds, record_parents: bool = False, parents_cap: int = 8):
    """Run every graph of a packed arena independently.  Returns (labels, rounds, parents)."""
    lib = _load()
    voff = np.ascontiguousarray(voff, dtype=np.int64)
    eoff = np.ascontiguousarray(eoff, dtype=np.int64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    src = _u32(src)
    dst = _u32(dst)
    G = int(voff.shape[0] - 1)
    labels = np.empty(max(int(voff[-1]), 1), dtype=np.uint32)
    rounds = np.empty(max(G, 1), dtype=np.int32)
    par = np.empty(max(int(voff[-1]) * parents_cap, 1), dtype=np.uint32) if record_parents else None
    st = lib.lco_run_batch(G, _ptr(voff, ctypes.c_int64), _ptr(eoff, ctypes.c_int64), _ptr(src, ctypes.c_uint32),
                           _ptr(dst, ctypes.c_uint32), _ptr(seeds, ctypes.c_uint64), _ptr(labels, ctypes.c_uint32),
                           _ptr(rounds, ctypes.c_int32), _ptr(par, ctypes.c_uint32),
                           parents_cap if record_parents else 0)
    if st != 0:
        raise ValueError("oracle rejected a graph of the batch")
    return labels[:int(voff[-1])], rounds[:G], par


def components_min_id(n: int, src, dst) -> np.ndarray:
    """Smallest vertex id of each vertex's connected component (textbook union-find)."""
    src = _u32(src)
    dst = _u32(dst)
    out = np.empty(max(n, 1), dtype=np.uint32)
    if _load().lco_components_min_id(n, int(src.shape[0]), _ptr(src, ctypes.c_uint32), _ptr(dst, ctypes.c_uint32),
                                     _ptr(out, ctypes.c_uint32)) != 0:
        raise ValueError("ids out of range or out of memory")
    return out[:n]
