"""A CPU build of the HIP library for tests -- TEST INFRASTRUCTURE ONLY.

The library's sources (paper_1807_10727_amd/csrc, unchanged) are compiled as host C++
against ``include/hip/hip_runtime.h`` here, which emulates the HIP execution model (fibers
for work-items, 64-lane waves with ballots and shuffles, LDS, barriers, atomics, streams and
captured graphs) on the host.  Tests drive that build through the same ctypes binding
(``_cc.py``, copied next to it) with numpy arrays as device memory, and compare it with the
oracle.  It checks the kernels' logic -- indexing, bounds, synchronisation, the host engine
-- without a GPU; it says nothing about timing or about the hardware's memory model.

The product package never loads this build: it lives under tests/hipemu/_build and is
imported here under another module name.
"""
from __future__ import annotations

import ctypes
import importlib.util
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
# HIPEMU_ASAN=1: the bounds-checking build -- AddressSanitizer, with a guard gap after every
# workspace buffer (LC_WS_GUARD), so that any access outside an allocation or past a carved
# buffer's end stops the process with a report, and a tiny sample and LDS capacity for the
# sampled-bucket sort's second level and final buckets (its global-memory path then runs too).  The process must preload
# asan_runtime().
ASAN = os.environ.get("HIPEMU_ASAN") == "1"
BUILD = os.path.join(HERE, "_build_asan" if ASAN else "_build")
CSRC = os.path.join(ROOT, "paper_1807_10727_amd", "csrc")
LIB = os.path.join(BUILD, "libcc.so")
CXX = os.environ.get("HIPEMU_CXX", "/opt/rocm/llvm/bin/clang++")
WS_FILL = 0xA5   # the workspace starts with these bytes, as a torch.empty tensor holds anything

_cc = None


def _sources():
    spec = importlib.util.spec_from_file_location("lc_hip_build_for_emu", os.path.join(ROOT, "paper_1807_10727_amd",
                                                                                         "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return [os.path.join(CSRC, s) for s in mod.SOURCES] + [os.path.join(HERE, "runtime.cpp")]


def _deps():
    out = []
    for d in (CSRC, os.path.join(HERE, "include", "hip"), os.path.join(ROOT, "include")):
        out += [os.path.join(d, f) for f in os.listdir(d)]
    return out + [os.path.join(HERE, "runtime.cpp"), os.path.join(ROOT, "paper_1807_10727_amd", "_cc.py")]


def build(force: bool = False) -> str:
    """Compile the emulated library (parallel, one object per source) unless it is newer than
    every source it depends on."""
    os.makedirs(BUILD, exist_ok=True)
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(p) <= t for p in _deps()):
            return LIB
    flags = ["-std=c++17", "-O2", "-fPIC", "-pthread", "-Wno-unknown-attributes", "-Wno-ignored-attributes",
             "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    link = []
    if ASAN:
        # the sampled-bucket sort cuts its second level from 4 sampled keys and holds at most
        # 16 keys of a final bucket in LDS here, so that its in-place global sort of larger
        # buckets runs in every test that uses that sort
        flags += ["-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-DLC_WS_GUARD=256",
                  "-DLC_BUCKET_CAP=16", "-DLC_BUCKET_SAMPLE2=4"]
        link = ["-fsanitize=address", "-shared-libasan"]

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        lang = ["-x", "c++"] if src.endswith(".hip") else []
        subprocess.run([CXX] + lang + flags + ["-c", src, "-o", obj], check=True, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, _sources()))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([CXX, "-shared", "-pthread"] + link + ["-o", tmp] + objs, check=True)
    os.replace(tmp, LIB)
    shutil.copyfile(os.path.join(ROOT, "paper_1807_10727_amd", "_cc.py"), os.path.join(BUILD, "_cc.py"))
    return LIB


def asan_runtime() -> str:
    """The AddressSanitizer runtime that a process loading the HIPEMU_ASAN build preloads."""
    out = subprocess.run([CXX, "-print-file-name=libclang_rt.asan-x86_64.so"], stdout=subprocess.PIPE, text=True,
                         check=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        raise RuntimeError("no AddressSanitizer runtime next to " + CXX)
    return out


def asan_env(env=None) -> dict:
    """Environment of a child process that runs the bounds-checking build."""
    env = dict(os.environ if env is None else env)
    env["HIPEMU_ASAN"] = "1"
    env["LD_PRELOAD"] = asan_runtime()
    # fibers switch stacks by hand: no fake stacks; leaks are not what is checked
    env["ASAN_OPTIONS"] = "detect_leaks=0:detect_stack_use_after_return=0:halt_on_error=1"
    return env


def binding():
    """The ctypes binding (_cc.py) bound to the emulated library."""
    global _cc
    if _cc is None:
        build()
        spec = importlib.util.spec_from_file_location("hipemu_cc", os.path.join(BUILD, "_cc.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        assert os.path.dirname(mod.LIB_PATH) == BUILD
        _cc = mod
    return _cc


def _aligned(nbytes: int, fill: int | None = WS_FILL):
    raw = np.empty(nbytes + 256, np.uint8)
    off = (-raw.ctypes.data) % 256
    buf = raw[off:off + nbytes]
    if fill is not None:
        buf.fill(fill)
    return buf


def device(a, dtype=None):
    """A host array standing in for device memory (contiguous, copied)."""
    return np.ascontiguousarray(a, dtype=dtype).copy()


class Solver:
    """One graph's solve on the emulated library, the counterpart of the package's Solver
    with numpy arrays in place of device tensors."""

    def __init__(self, n, src, dst=None, seed=0, flags=0, max_rounds=0, layout=None, finish_edges=0,
                 ws_fill=WS_FILL):
        cc = binding()
        self.cc = cc
        self.n = int(n)
        if layout is None:
            if dst is None:
                layout = cc.CC_EDGES_PACKED_U64
            elif src.dtype in (np.int64, np.uint64):
                layout = cc.CC_EDGES_SOA_I64
            else:
                layout = cc.CC_EDGES_SOA_I32
        self.layout = layout
        self._src, self._dst = src, dst
        self.m = int(src.shape[0])
        self.ctx = cc.cc_create(self.n, self.m, layout, src.ctypes.data if self.m else 0,
                                dst.ctypes.data if dst is not None and self.m else 0, seed=seed,
                                max_rounds=max_rounds, flags=flags)
        self.ws_bytes = cc.cc_workspace_size(self.ctx)
        self.ws = _aligned(self.ws_bytes, ws_fill)
        cc.cc_set_workspace(self.ctx, self.ws.ctypes.data, self.ws_bytes)
        if finish_edges:
            cc.cc_set_finish(self.ctx, finish_edges)
        self._tables = {}

    def run(self):
        return self.cc.cc_run(self.ctx)

    def contract_round(self):
        return self.cc.cc_contract_round(self.ctx)

    def reset(self, seed):
        self.cc.cc_reset(self.ctx, seed)

    def labels(self):
        out = np.empty(max(self.n, 1), np.int64 if self.layout == self.cc.CC_EDGES_SOA_I64 else np.int32)
        self.cc.cc_labels(self.ctx, out.ctypes.data)
        return out[:self.n]

    def parents(self, r=-1):
        out = np.empty(max(self.n, 1), np.int32)
        k = self.cc.cc_round_parents(self.ctx, r, out.ctypes.data)
        return out[:self.n], k

    def minima(self):
        m1 = np.empty(max(self.n, 1), np.uint32)
        l2 = np.empty(max(self.n, 1), np.uint32)
        self.cc.cc_debug_round_arrays(self.ctx, m1.ctypes.data, l2.ctypes.data)
        return m1[:self.n], l2[:self.n]

    def edges(self):
        m = self.cc.cc_round_edges(self.ctx, 0, 0)
        out = np.empty(max(m, 1), np.uint64)
        k = self.cc.cc_round_edges(self.ctx, out.ctypes.data, out.size)
        return out[:k]

    def set_priorities(self, r, table):
        t = device(table, np.uint32)
        self._tables[int(r)] = t
        self.cc.cc_set_explicit_priorities(self.ctx, r, t.ctypes.data)

    def set_tuning(self, **kw):
        self.cc.cc_set_tuning(self.ctx, **kw)

    @property
    def tuning(self):
        return self.cc.cc_get_tuning(self.ctx)

    def set_merge_to_large(self, alphas):
        self.cc.cc_set_merge_to_large(self.ctx, alphas)

    def stats(self, rounds):
        return [self.cc.cc_get_round_stats(self.ctx, r) for r in range(rounds)]

    def save_state(self):
        return self.cc.cc_save_state(self.ctx)

    def load_state(self, blob):
        self.cc.cc_load_state(self.ctx, blob)

    def close(self):
        if self.ctx:
            self.cc.cc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """The batched solve on the emulated library (int32 local ids per graph)."""

    def __init__(self, voff, eoff, seeds, src, dst, ws_fill=WS_FILL, **config):
        cc = binding()
        self.cc = cc
        self.voff = np.ascontiguousarray(voff, np.int64)
        self.eoff = np.ascontiguousarray(eoff, np.int64)
        self.G = int(self.voff.shape[0] - 1)
        self.n_total = int(self.voff[-1])
        self._src, self._dst = device(src, np.int32), device(dst, np.int32)
        self.b = cc.cc_batch_create(self.voff, self.eoff, seeds, self._src.ctypes.data, self._dst.ctypes.data)
        self.ws_bytes = cc.cc_batch_workspace_size(self.b)
        self.ws = _aligned(self.ws_bytes, ws_fill)
        cc.cc_batch_set_workspace(self.b, self.ws.ctypes.data, self.ws_bytes)
        if config:
            cc.cc_batch_set_config(self.b, **config)
        self.labels = np.empty(max(self.n_total, 1), np.int32)

    def run(self):
        rounds = np.zeros(max(self.G, 1), np.int32)
        self.cc.cc_batch_run(self.b, self.labels.ctypes.data, rounds)
        return self.labels[:self.n_total].copy(), rounds[:self.G].copy()

    def split(self):
        return self.cc.cc_batch_split(self.b)

    @property
    def config(self):
        return self.cc.cc_batch_get_config(self.b)

    def close(self):
        if self.b:
            self.cc.cc_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
