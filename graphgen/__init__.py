"""Seeded synthetic graph generators (harness input shared by the oracle and the GPU path).

Nothing in this module computes any part of the connected-components method; it only
draws edge lists.  The heavy loops live in ``gen.c`` (compiled by :func:`build`), the
Python side composes them into the workloads used by the tests and the benchmark:

* ``gnm``        Erdos-Renyi G(n, m) records, duplicates and self-loops kept.
* ``paths``      disjoint random paths on fresh ids.
* ``rmat``       R-MAT with per-level probability noise and a seeded id permutation.
* ``er_with_paths``  G(n, m) followed by appended disjoint paths.
* ``batch_mix``  many independent graphs (half G(n, m), half R-MAT) packed in one arena.
* ``request_trace``  Poisson arrivals of graphs with log-uniform sizes.

All randomness is counter based (see ``gen.c``), so every workload is a pure function of
its seed.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# Seeds of the named workloads: workload i uses CONFIG_SEED_BASE + i.
CONFIG_SEED_BASE = 0xC0FFEE00

ST_BATCH = 10
ST_TRACE = 11
ST_MIX = 12


def build(force: bool = True) -> str:
    """Compile gen.c into libgraphgen.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.gg_sm64.restype = ctypes.c_uint64
        lib.gg_sm64.argtypes = [ctypes.c_uint64]
        lib.gg_gnm.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, u32p, u32p]
        lib.gg_paths.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, u32p, u32p]
        lib.gg_rmat.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64] + [ctypes.c_double] * 5 + [
            ctypes.c_int32, ctypes.c_uint32, u32p, u32p]
        lib.gg_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, u64p]
        lib.gg_pack.argtypes = [ctypes.c_int64, u32p, u32p, u64p]
        lib.gg_permutation.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, u32p]
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def sm64(x: int) -> int:
    return int(_load().gg_sm64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def draws(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_draws(seed, stream, start, count, _p64(out))
    return out


def gnm(seed: int, n: int, m: int, id_base: int = 0):
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    _load().gg_gnm(seed, n, m, id_base, _p32(src), _p32(dst))
    return src, dst


def paths(seed: int, count: int, length: int, id_base: int = 0):
    per = max(length - 1, 0)
    src = np.empty(count * per, dtype=np.uint32)
    dst = np.empty(count * per, dtype=np.uint32)
    _load().gg_paths(seed, count, length, id_base, _p32(src), _p32(dst))
    return src, dst


def rmat(seed: int, scale: int, m: int, probs=(0.57, 0.19, 0.19, 0.05), noise: float = 0.1,
         permute: bool = True, id_base: int = 0):
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    a, b, c, d = probs
    _load().gg_rmat(seed, scale, m, a, b, c, d, noise, int(permute), id_base, _p32(src), _p32(dst))
    return src, dst


def permutation(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _load().gg_permutation(seed, stream, n, _p32(out))
    return out


def pack(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """u64 records with the first endpoint in the high 32 bits."""
    out = np.empty(src.shape[0], dtype=np.uint64)
    _load().gg_pack(src.shape[0], _p32(np.ascontiguousarray(src)), _p32(np.ascontiguousarray(dst)), _p64(out))
    return out


@dataclass
class Graph:
    n: int
    src: np.ndarray  # uint32 [m]
    dst: np.ndarray  # uint32 [m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def er_with_paths(seed: int, n: int, m: int, n_paths: int, path_len: int, name: str = "") -> Graph:
    """G(n, m) records, then `n_paths` disjoint random paths on ids [n, n + n_paths*path_len)."""
    s1, d1 = gnm(seed, n, m)
    if n_paths:
        s2, d2 = paths(seed, n_paths, path_len, id_base=n)
        s1 = np.concatenate([s1, s2])
        d1 = np.concatenate([d1, d2])
    return Graph(n + n_paths * path_len, s1, d1, name)


def workload_small(seed: int = CONFIG_SEED_BASE + 0) -> Graph:
    """G(n, m), n = 65,536, m = 262,144 (average degree 8), int32 ids."""
    s, d = gnm(seed, 1 << 16, 1 << 18)
    return Graph(1 << 16, s, d, "gnm_n65536_m262144")


def workload_er_paths(seed: int = CONFIG_SEED_BASE + 1, shrink: int = 1) -> Graph:
    """G(n, m) with n = 2^24, m = 2^27, plus 10,000 disjoint paths of 1,000 vertices.

    `shrink` divides n, m and the path count (for bounded samples of the same mix)."""
    return er_with_paths(seed, (1 << 24) // shrink, (1 << 27) // shrink, 10_000 // shrink, 1000,
                         name="gnm_n2^24_m2^27_paths10000x1000" + ("" if shrink == 1 else "_div%d" % shrink))


def workload_rmat(seed: int = CONFIG_SEED_BASE + 2, scale: int = 26, edge_factor: int = 16) -> Graph:
    """R-MAT scale 26, edge factor 16, quadrants (0.57, 0.19, 0.19, 0.05), +-10% noise per level."""
    s, d = rmat(seed, scale, edge_factor << scale)
    return Graph(1 << scale, s, d, "rmat_s%d_ef%d" % (scale, edge_factor))


@dataclass
class Batch:
    """Independent graphs packed in one arena with local ids per graph."""
    n: np.ndarray        # int64 [G] vertex counts
    m: np.ndarray        # int64 [G] record counts
    voff: np.ndarray     # int64 [G+1]
    eoff: np.ndarray     # int64 [G+1]
    seeds: np.ndarray    # uint64 [G] per-graph priority seeds
    src: np.ndarray      # uint32 [sum m] local ids
    dst: np.ndarray      # uint32 [sum m]

    @property
    def count(self) -> int:
        return int(self.n.shape[0])

    def graph(self, j: int) -> Graph:
        a, b = int(self.eoff[j]), int(self.eoff[j + 1])
        return Graph(int(self.n[j]), self.src[a:b], self.dst[a:b], "batch[%d]" % j)


def _unit(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def batch_specs(seed: int, count: int, log2_min: int = 8, log2_max: int = 18,
                deg_lo: float = 1.5, deg_hi: float = 16.0, rmat_ef: int = 8):
    """Per-graph (kind, n, m, seed) of the batched mix: even graphs G(n, m) with n
    log-uniform in [2^log2_min, 2^log2_max] and average degree uniform in [deg_lo, deg_hi],
    odd graphs R-MAT with scale uniform in {log2_min..log2_max} and the given edge factor."""
    r = draws(seed, ST_BATCH, 3 * count)
    specs = []
    for j in range(count):
        gseed = sm64(seed ^ j)
        if j % 2 == 0:
            u = float(_unit(r[3 * j:3 * j + 1])[0])
            n = int(math.floor(2.0 ** (log2_min + (log2_max - log2_min) * u)))
            d = deg_lo + (deg_hi - deg_lo) * float(_unit(r[3 * j + 1:3 * j + 2])[0])
            specs.append(("gnm", n, int(math.floor(d * n / 2)), gseed))
        else:
            scale = log2_min + int((int(r[3 * j + 2]) >> 32) * (log2_max - log2_min + 1) >> 32)
            specs.append(("rmat", 1 << scale, rmat_ef << scale, gseed))
    return specs


def make_batch(specs) -> Batch:
    G = len(specs)
    n = np.array([s[1] for s in specs], dtype=np.int64)
    m = np.array([s[2] for s in specs], dtype=np.int64)
    voff = np.zeros(G + 1, dtype=np.int64)
    eoff = np.zeros(G + 1, dtype=np.int64)
    np.cumsum(n, out=voff[1:])
    np.cumsum(m, out=eoff[1:])
    src = np.empty(int(eoff[-1]), dtype=np.uint32)
    dst = np.empty(int(eoff[-1]), dtype=np.uint32)
    seeds = np.array([s[3] for s in specs], dtype=np.uint64)
    for j, (kind, nj, mj, gs) in enumerate(specs):
        a, b = int(eoff[j]), int(eoff[j + 1])
        if kind == "gnm":
            s, d = gnm(gs, nj, mj)
        else:
            s, d = rmat(gs, int(nj).bit_length() - 1, mj)
        src[a:b] = s
        dst[a:b] = d
    return Batch(n, m, voff, eoff, seeds, src, dst)


def batch_mix(seed: int = CONFIG_SEED_BASE + 3, count: int = 4096, **kw) -> Batch:
    return make_batch(batch_specs(seed, count, **kw))


@dataclass
class Request:
    arrival: float   # seconds from trace start
    kind: str
    n: int
    m: int
    seed: int        # graph seed (also its priority seed)

    def graph(self) -> Graph:
        if self.kind == "gnm":
            s, d = gnm(self.seed, self.n, self.m)
        else:
            s, d = rmat(self.seed, int(self.n).bit_length() - 1, self.m)
        return Graph(self.n, s, d, "req")


def request_trace(seed: int, count: int, rate: float, log2_min: int = 10, log2_max: int = 24,
                  deg_lo: float = 4.0, deg_hi: float = 16.0, rmat_ef: int = 16):
    """Poisson arrivals at `rate` per second.  Sizes log-uniform in [2^log2_min, 2^log2_max];
    half G(n, m) with average degree uniform in [deg_lo, deg_hi], half R-MAT with scale
    ceil(log2 n) and the given edge factor."""
    r = draws(seed, ST_TRACE, 4 * count)
    u = _unit(r)
    t = 0.0
    out = []
    for j in range(count):
        t += -math.log(1.0 - float(u[4 * j])) / rate
        n = int(math.floor(2.0 ** (log2_min + (log2_max - log2_min) * float(u[4 * j + 1]))))
        gseed = sm64(seed ^ (j + 0x5EED))
        if float(u[4 * j + 2]) < 0.5:
            d = deg_lo + (deg_hi - deg_lo) * float(u[4 * j + 3])
            out.append(Request(t, "gnm", n, int(math.floor(d * n / 2)), gseed))
        else:
            scale = max(1, int(math.ceil(math.log2(n))))
            out.append(Request(t, "rmat", 1 << scale, rmat_ef << scale, gseed))
    return out


def request_mix(seed: int, count: int, pool: int, rate: float = 1.0):
    """A long request trace over a pool of `pool` graphs: Poisson arrivals at `rate` per
    second, each request a uniformly drawn pool graph with a priority seed of its own.
    Returns (arrivals, pool indices, priority seeds) as lists."""
    u = _unit(draws(seed, ST_MIX, 2 * count))
    t, arr, idx, seeds = 0.0, [], [], []
    for j in range(count):
        t += -math.log(1.0 - float(u[2 * j])) / rate
        arr.append(t)
        idx.append(min(pool - 1, int(float(u[2 * j + 1]) * pool)))
        seeds.append(sm64(seed ^ (j + 0x7A11)))
    return arr, idx, seeds
